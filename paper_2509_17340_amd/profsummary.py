"""Summarise a rocprofv3 kernel-trace database by kernel and launch shape.

    python -m paper_2509_17340_amd.profsummary <results.db> [--title TEXT] [--cmd TEXT]
    python -m paper_2509_17340_amd.profsummary --fetch F.db --write W.db \
        --copy-fetch CF.db --copy-write CW.db [--copy-mib 512]

Prints a Markdown table (calls, grid, workgroup, VGPRs, average / min / max
duration in microseconds) with one row per (kernel, grid size), so that launches
of the same kernel with different shapes (for example the Stage-I and Stage-II
distance passes) are reported separately.
"""
import argparse
import re
import sqlite3
import statistics


def summarise(db):
    con = sqlite3.connect(db)
    cur = con.cursor()
    rows = cur.execute(
        "select name, grid_x, workgroup_x, vgpr_count, accum_vgpr_count, lds_size, duration "
        "from kernels").fetchall()
    groups = {}
    for name, gx, wx, vg, ag, lds, dur in rows:
        groups.setdefault((name, gx, wx, vg, ag, lds), []).append(dur / 1000.0)
    out = []
    for (name, gx, wx, vg, ag, lds), d in groups.items():
        out.append(dict(name=name, grid=gx, wg=wx, vgpr=vg, agpr=ag, lds=lds, calls=len(d),
                        avg_us=statistics.fmean(d), min_us=min(d), max_us=max(d), total_us=sum(d)))
    out.sort(key=lambda r: -r["total_us"])
    return out


def pmc(db, counter):
    """{(kernel, grid): (mean value, calls)} of one counter from a --pmc database."""
    con = sqlite3.connect(db)
    rows = con.cursor().execute(
        "select kernel_name, grid_size, value from counters_collection where counter_name = ?",
        (counter,)).fetchall()
    groups = {}
    for name, grid, v in rows:
        groups.setdefault((short(name), grid), []).append(v)
    return {k: (statistics.fmean(v), len(v)) for k, v in groups.items()}


def copy_factor(db, counter, mib):
    """Counter KiB per true KiB for the calibration copy of `mib` MiB."""
    vals = [v for (name, grid), (v, n) in pmc(db, counter).items() if "copyBuffer" in name
            and v > 0.25 * mib * 1024]
    return max(vals) / (mib * 1024.0) if vals else float("nan")


def short(name):
    m = re.search(r"(\w+)\(", name)
    return m.group(1) if m else name


def main_pmc(a):
    fetch, write = pmc(a.fetch, "FETCH_SIZE"), pmc(a.write, "WRITE_SIZE")
    ff = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_mib)
    fw = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_mib)
    print(f"# {a.title}\n")
    for c in a.cmd:
        print(f"Command: `{c}`\n")
    print(f"Calibration: a plain {a.copy_mib} MiB device copy reads FETCH_SIZE = {ff:.4f} x and "
          f"WRITE_SIZE = {fw:.4f} x its true KiB; the byte columns divide by these factors.\n")
    print("| kernel | grid (threads) | calls | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB |")
    print("|---|---|---|---|---|---|---|")
    keys = sorted(set(fetch) | set(write), key=lambda k: -fetch.get(k, (0, 0))[0])
    for k in keys:
        f, n = fetch.get(k, (float("nan"), 0))
        w, _ = write.get(k, (float("nan"), 0))
        print(f"| {k[0]} | {k[1]} | {n} | {f:.1f} | {w:.1f} | {f * 1024 / ff / 1e6:.3f} | "
              f"{w * 1024 / fw / 1e6:.3f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--title", default="rocprofv3 kernel trace")
    ap.add_argument("--cmd", default=[], action="append")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=512)
    a = ap.parse_args()
    if a.fetch:
        return main_pmc(a)
    a.cmd = [c for c in a.cmd if c]
    rows = summarise(a.db)
    total = sum(r["total_us"] for r in rows)
    print(f"# {a.title}\n")
    for c in a.cmd:
        print(f"Command: `{c}`\n")
    print("| kernel | calls | grid (threads) | wg | VGPR | AGPR | LDS B | avg us | min us | max us | % time |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {short(r['name'])} | {r['calls']} | {r['grid']} | {r['wg']} | {r['vgpr']} | "
              f"{r['agpr']} | {r['lds']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | "
              f"{r['max_us']:.2f} | {100 * r['total_us'] / total:.1f} |")


if __name__ == "__main__":
    main()
