"""Summarise a rocprofv3 kernel-trace database by kernel and launch shape.

    python -m paper_2509_17340_amd.profsummary <results.db> [--title TEXT] [--cmd TEXT]

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


def short(name):
    m = re.search(r"(\w+)\(", name)
    return m.group(1) if m else name


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--title", default="rocprofv3 kernel trace")
    ap.add_argument("--cmd", default="")
    a = ap.parse_args()
    rows = summarise(a.db)
    total = sum(r["total_us"] for r in rows)
    print(f"# {a.title}\n")
    if a.cmd:
        print(f"Command: `{a.cmd}`\n")
    print("| kernel | calls | grid (threads) | wg | VGPR | AGPR | LDS B | avg us | min us | max us | % time |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {short(r['name'])} | {r['calls']} | {r['grid']} | {r['wg']} | {r['vgpr']} | "
              f"{r['agpr']} | {r['lds']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | "
              f"{r['max_us']:.2f} | {100 * r['total_us'] / total:.1f} |")


if __name__ == "__main__":
    main()
