"""Benchmark: AERO-MPPI planning steps on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--poses P] [--batched B]
                    [--no-cpu-baseline] [--lean]

Headline workload (the largest single-GPU configuration): the closed loop through
a dense incline corridor at 7 m/s.  Every planning step is one replayed pose with
its own 1,000,000-point LiDAR cloud (8 sweeps of 1024 x 128 beams, 40 m, 2 cm
noise), M = 16 instances (8 x 2 anchors), K = 8192 samples, N = 60 steps,
dt = 0.04 s: partition -> anchors -> guides -> Stage I (noise, RK4, cost with the
nearest distance to the raw cloud, update) -> Stage II (explicit rollouts,
argmin) -> one adjoint refinement of the selected plan -> warm start of the next
pose.  W untimed poses settle the autotuner; then K consecutive poses (warm start
carried from pose to pose, clouds resident in device memory before the timed
region, each moved into the planner's cloud buffer inside it) are timed, and the
flight continues to P poses for the plan-step distribution.

Named legs on the same GPU: the one-step ensemble on a 50k forest cloud (captured
as a HIP graph), the 64-problem uneven batch (batched call vs 64 plain calls), the
adjoint (backward vs forward), the paper's operating point (P_f collision set,
K = 128 and 256), and the FP64 oracle timed on the host's cores.  Prints one JSON
line.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPPI rollout-steps/s + plan-step ms; batched/adjoint vs plain, same GPU, ≤1e-4"
FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
F16_PEAK_TFLOPS = 2500.0      # MI355X published FP16 dense matrix peak
HBM_PEAK_GBS = 8000.0         # MI355X published HBM3E bandwidth
FLOP_PER_PAIR = 8             # 3 sub + 3 mul + 2 add per (position, point) pair

# Pass-A variants: kernel, roofline bound and the published peak of the unit it runs
# on, the FLOP it executes per pair, and the positions of one query block.
PASS_A = {
    0: dict(kernel="k_pass_a_valu", bound="alu", peak=FP32_PEAK_TFLOPS, qpb=2048,
            unit_note="FP32 vector (VALU) peak", executed_flop_per_pair=6),
    1: dict(kernel="k_pass_a_f16s<4>", bound="mfma", peak=F16_PEAK_TFLOPS, qpb=512,
            unit_note="FP16 dense MFMA peak (split hi/lo operands, FP32 accumulation)",
            executed_flop_per_pair=32),
    2: dict(kernel="k_pass_a_f16s<8>", bound="mfma", peak=F16_PEAK_TFLOPS, qpb=1024,
            unit_note="FP16 dense MFMA peak (split hi/lo operands, FP32 accumulation)",
            executed_flop_per_pair=32),
}
# Pair-rate ceiling of the split-FP16 pass: the K = 16 MFMA (32 FLOP per pair at the
# FP16 dense peak) and the running minimum (one v_min3_f32 per two pairs on 16 lanes
# x 4 SIMDs x 256 CUs at 2.4 GHz) both allow about 7.8e13 pairs/s.
F16S_PAIR_CEILING = min(F16_PEAK_TFLOPS * 1e12 / 32, 16 * 4 * 256 * 2.4e9 * 2)


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def pool_size():
    """Worker processes for host work: the CPUs this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_pool(workers, initializer=None, initargs=()):
    """A process pool of single-threaded workers (spawned, so that they inherit no
    device state)."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    return ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                               initializer=initializer, initargs=initargs)


def measured_traffic(kernel, path):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter summary (its
    indented `key = value` blocks, one per kernel), or None when the summary or the
    kernel's block is missing, or the kernel's source file changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", path)
    if not os.path.exists(path):
        return None
    blocks, kv = [], {}
    for line in open(path):
        if "=" in line and line.startswith("    "):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
        elif kv:
            blocks.append(kv)
            kv = {}
    if kv:
        blocks.append(kv)
    for kv in blocks:
        if kv.get("kernel") != kernel or "kernel_source" not in kv:
            continue
        src = os.path.join(ROOT, kv["kernel_source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        return int(kv["traffic_bytes_per_launch"]) if sha == kv.get("kernel_source_sha256") else None
    return None


def steps_per_plan_of(M, K, N):
    """Rollout steps of one planning step: Stage I (M K N) and Stage II (M N)."""
    return M * K * N + M * N


def pcts(ms):
    s = sorted(ms)
    return s[len(s) // 2], s[min(len(s) - 1, int(0.99 * len(s)))]


# ----------------------------------------------------------------------------
# oracle on the host cores
# ----------------------------------------------------------------------------
_W = {}


def _oracle_init(prob, coef):
    _W["prob"], _W["coef"] = prob, coef


def _oracle_stage1(task):
    """Stage I of instance m for the samples ks, with the oracle's own Philox stream."""
    import numpy as np

    from oracle import mppi as OM
    from oracle import philox as OPh
    m, ks = task
    prob, coef = _W["prob"], _W["coef"]
    prm, N = prob["params"], prob["N"]
    t0 = time.perf_counter()
    k = np.asarray(ks)[:, None]
    t = np.arange(N)[None, :]
    w = OPh.philox4x32_10((k, t, np.full_like(k + t, m), np.full_like(k + t, prm["iter_base"])),
                          OPh.philox_key(prm["seed"], prob["problem_id"]))
    n0, n1 = OPh.box_muller(w[0], w[1])
    n2, n3 = OPh.box_muller(w[2], w[3])
    normals = np.stack([n0, n1, n2, n3], -1)[None]
    sub = dict(prob, M=1, K=len(ks), u_nom=prob["u_nom"][m:m + 1])
    st = OM.mppi_step(sub, coef[m:m + 1], normals=normals)
    return time.perf_counter() - t0, st["S1"][0]


def _oracle_stage2(m):
    import numpy as np

    from oracle import mppi as OM
    prob = _W["prob"]
    t0 = time.perf_counter()
    sel = OM.select_best(prob, np.asarray(prob["u_nom"][m:m + 1], np.float32))
    return time.perf_counter() - t0, float(sel["S2"][0])


def cpu_baseline(prob, samples_per_instance, workers):
    """The FP64 oracle as it is, on a bounded sample of one planning step, over a pool
    of single-threaded worker processes: partition + guides in the parent, Stage I of
    `samples_per_instance` evenly spaced samples of every instance and Stage II of every
    instance on the pool; Stage I extrapolated to all K samples."""
    import numpy as np

    from oracle import guides as OG
    from oracle import partition as OP

    part = prob["partition"]
    M, K, N = prob["M"], prob["K"], prob["N"]
    t0 = time.perf_counter()
    pa = OP.partition_anchors(prob["cloud"], prob["goal_dir"], part["n_az_c"], part["n_el_c"],
                              part["f_a"], part["f_e"], part["r_max"], part["ell"],
                              prob["M_h"], prob["M_v"])
    T = np.float32(N * np.float32(prob["params"]["dt"]))
    coef = OG.build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3), pa["anchors"], T)
    t1 = time.perf_counter()
    sub = np.linspace(0, K - 1, samples_per_instance).round().astype(int)
    chunks = [(m, sub[i:i + 2]) for m in range(M) for i in range(0, len(sub), 2)]
    with host_pool(workers, _oracle_init, (prob, coef)) as ex:
        # every worker up (and holding the cloud) before the clock starts
        list(ex.map(_worker_pid, range(4 * workers)))
        t2 = time.perf_counter()
        r1 = list(ex.map(_oracle_stage1, chunks))
        t3 = time.perf_counter()
        r2 = list(ex.map(_oracle_stage2, range(M)))
        t4 = time.perf_counter()
    stage1 = (t3 - t2) * (K / len(sub))
    full = (t1 - t0) + stage1 + (t4 - t3)
    cpu_s = sum(r[0] for r in r1) + sum(r[0] for r in r2)
    return {
        "value": steps_per_plan_of(M, K, N) / full, "unit": "rollout-steps/s",
        "cores": workers, "kind": "oracle",
        "sample": (f"FP64 NumPy oracle over {workers} single-threaded worker processes: "
                   f"partition + guides ({t1 - t0:.1f} s, one process) and Stage II of all "
                   f"{M} instances ({t4 - t3:.1f} s) in full; Stage I (Philox noise, RK4, "
                   f"brute-force nearest over all {len(prob['cloud'])} points, cost) on "
                   f"{len(sub)} of {K} samples per instance ({t3 - t2:.1f} s wall, "
                   f"{sum(r[0] for r in r1):.0f} s CPU), extrapolated to all samples: "
                   f"{full:.0f} s per planning step; the refinement and warm start are "
                   f"not included"),
        "measured_wall_s": t4 - t2 + (t1 - t0), "measured_cpu_s": cpu_s,
        "host_cpus": os.cpu_count(),
    }


def _worker_pid(_):
    time.sleep(0.05)
    return os.getpid()


def _loop_fixture(s):
    from fixtures import make_loop_step
    return make_loop_step(s)


# ----------------------------------------------------------------------------
# legs
# ----------------------------------------------------------------------------
def kernel_ms(kt, n):
    return {k: v[0] / n for k, v in kt.items() if v[1]}


def distance_rooflines(kt, steps, stats, brute_pairs, variant, label):
    """Rooflines of the two distance passes from the library's live event timers and the
    work counted by aero_read_distance_stats, summed over the same `steps` planning
    steps: algorithmic FLOP = 8 per (position, point) pair a pass evaluates (pass A:
    the cull step's items x block positions x sub-tile points; pass B: the pairs of its
    hit words), with the brute-force-equivalent rate beside pass A's."""
    out = {}
    va = PASS_A[variant]
    ms_a, n_a = kt["min_dist"]
    if n_a:
        t = ms_a * 1e-3
        rate = stats["pairs_a_eval"] / t
        prod_rate = stats["pairs_a_products"] / t
        achieved = FLOP_PER_PAIR * rate / 1e12
        a = {"bound": va["bound"], "kernel": f"{va['kernel']} ({label}, first pass; autotuned "
                                             f"variant {variant})",
             "kernel_name": va["kernel"],
             "achieved": achieved, "peak": va["peak"], "unit": "TFLOP/s",
             "peak_is": va["unit_note"], "frac": achieved / va["peak"],
             "flop_counted": "8 per (position, point) pair evaluated: per cull item, each "
                             "wave's existing positions x the points of the 32-point groups "
                             "it takes (groups beyond reach of the wave's positions skipped)",
             "pairs_per_launch": stats["pairs_a_eval"] / n_a, "avg_launch_ms": ms_a / n_a,
             "pairs_per_s": rate,
             "listed_pairs_per_launch": stats["pairs_a"] / n_a,
             "executed_pairs_per_launch": stats["pairs_a_products"] / n_a,
             "executed_tflops": va["executed_flop_per_pair"] * prod_rate / 1e12,
             "executed_frac": va["executed_flop_per_pair"] * prod_rate / 1e12 / va["peak"],
             "executed_is": "the matrix-core products' pairs (32 points x 32 positions, "
                            "padding included) at 32 FLOP per pair" if va["bound"] == "mfma"
                            else "the evaluated pairs at the FLOP the kernel executes per pair",
             "brute_force_pairs_per_launch": brute_pairs / n_a,
             "brute_force_equivalent_tflops": FLOP_PER_PAIR * brute_pairs / t / 1e12}
        if va["bound"] == "mfma":
            a["pair_ceiling_per_s"] = F16S_PAIR_CEILING
            a["frac_of_pair_ceiling"] = prod_rate / F16S_PAIR_CEILING
        out["pass_a"] = a
    ms_b, n_b = kt["min_dist_exact"]
    if n_b:
        t = ms_b * 1e-3
        rate = stats["pairs_b_eval"] / t
        achieved = FLOP_PER_PAIR * rate / 1e12
        out["pass_b"] = {
            "bound": "alu", "kernel": f"k_pass_b ({label}, exact pass over the hit pairs)",
            "kernel_name": "k_pass_b<false>",
            "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "peak_is": "FP32 vector (VALU) peak", "frac": achieved / FP32_PEAK_TFLOPS,
            "flop_counted": "8 per (position, point) pair pass B evaluates (3 sub, 3 mul, "
                            "2 add): each listed query against the 32-point groups of its "
                            "hit sub-tiles that lie within its cap",
            "pairs_per_launch": stats["pairs_b_eval"] / n_b, "avg_launch_ms": ms_b / n_b,
            "pairs_per_s": rate,
            "listed_pairs_per_launch": stats["pairs_b"] / n_b,
            "issue_ceiling_tflops": FP32_PEAK_TFLOPS * FLOP_PER_PAIR / 14,
            "issue_ceiling_note": "per pair 3 v_sub + v_mul + 2 v_fma at full rate and half "
                                  "a v_min3 at half rate: 7 issue slots for 8 FLOP, against "
                                  "14 FLOP for 7 FMAs",
            "items": stats["items_b"], "items_taken_whole": stats["items_whole"]}
    return out


def dominant(rl, kt):
    """The roofline of the slower distance pass."""
    if "pass_b" in rl and (kt["min_dist_exact"][0] > kt["min_dist"][0] or "pass_a" not in rl):
        return dict(rl["pass_b"])
    return dict(rl["pass_a"])


def sum_stats(a, b):
    return {k: a.get(k, 0) + b[k] for k in b}


def bench_loop(poses, warmup, steps, n_total):
    """The closed loop: W warm-up poses, then K timed consecutive poses from a hover
    start (warm start carried), then on to n_total poses for the distribution."""
    import torch

    import paper_2509_17340_amd as aero
    from paper_2509_17340_amd.planner import LoopRunner

    lr = LoopRunner(poses[0])
    ps = lr.ps
    clouds = [torch.from_numpy(p["cloud"]).to("cuda") for p in poses]
    torch.cuda.synchronize()

    timing = [False]

    def step(i):
        lr.load_device(clouds[i], poses[i])
        aero.timing_enable(timing[0])            # the planning step's kernels only
        lr.plan()
        aero.timing_enable(False)
        lr.refine()

    for i in range(warmup):
        step(i % len(poses))
    torch.cuda.synchronize()
    ps.reset()                                   # hover start for the timed flight
    timing[0] = True
    aero.timing_read(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_total + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        step(i)
        ev[i + 1].record()
    torch.cuda.synchronize()
    kt = aero.timing_read(reset=True)
    timing[0] = False
    total_ms = ev[0].elapsed_time(ev[steps])
    for i in range(steps, n_total):              # the flight goes on (not in `value`)
        step(i)
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(n_total)]
    # the timed poses again from the same start (every result is reproducible bit for
    # bit), reading the distance passes' work after each: not timed
    ps.reset()
    stats = {}
    for i in range(steps):
        lr.load_device(clouds[i], poses[i])
        ps.front_end()
        ps.stage1()
        torch.cuda.synchronize()       # read before Stage II reuses the workspace
        stats = sum_stats(stats, aero.distance_stats([ps.problem], ps.ws))
        ps.stage2()
        lr.refine()
    return dict(total_ms=total_ms, per=per, kt=kt, stats=stats, M=ps.M, K=ps.K, N=ps.N,
                P=ps.n_points, variant=aero.pass_a_variant([ps.problem]))


def bench_ensemble(prob, steps, warmup):
    """The one-step ensemble on the 50k forest cloud: eager (timed kernels) and as a
    replayed HIP graph."""
    import torch

    import paper_2509_17340_amd as aero
    from paper_2509_17340_amd.planner import GraphStep, PlanStep

    ps = PlanStep(prob)
    for _ in range(warmup):
        ps.reset()
        ps.run()
    torch.cuda.synchronize()
    aero.timing_enable(True)
    aero.timing_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ps.reset()
        ps.run()
    e1.record()
    torch.cuda.synchronize()
    kt = aero.timing_read(reset=True)
    aero.timing_enable(False)
    eager = e0.elapsed_time(e1) / steps
    ps.reset()
    ps.front_end()
    ps.stage1()
    torch.cuda.synchronize()           # read before Stage II reuses the workspace
    st = aero.distance_stats([ps.problem], ps.ws)
    stats = {k: v * steps for k, v in st.items()}
    g = GraphStep(ps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        g.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    gms = ev[0].elapsed_time(ev[-1]) / steps
    p50, p99 = pcts([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    M, K, N, P = ps.M, ps.K, ps.N, ps.n_points
    variant = aero.pass_a_variant([ps.problem])
    rl = distance_rooflines(kt, steps, stats, M * K * N * P * steps, variant,
                            "Stage I nearest distance")
    return {
        "ms_per_step": gms, "eager_ms_per_step": eager, "p50_ms": p50, "p99_ms": p99,
        "rollout_steps_per_s": steps_per_plan_of(M, K, N) / (gms * 1e-3),
        "launch_mode": "hip_graph",
        "roofline": dominant(rl, kt), "distance_passes": rl, "distance_work_per_step": st,
        "kernels_ms_per_step": kernel_ms(kt, steps),
        "workload": f"ensemble-forest-50k: one planning step (partition 32x8 coarse x 4x4, "
                    f"M={M}, K={K}, N={N}, dt=0.05, {P}-point LiDAR cloud, Stage I + Stage II)",
    }


def bench_adjoint(prob, iters=20):
    """Forward vs backward on the same GPU.  The forward is one Stage-I call that also
    stores the nearest point of every rollout position; the backward is
    aero_mppi_step_backward_indexed from those indices (no distance pass).  The
    self-contained aero_mppi_step_backward (its own distance passes) is timed too."""
    import torch

    import paper_2509_17340_amd as aero
    from paper_2509_17340_amd.planner import PlanStep

    ps = PlanStep(prob)
    ps.front_end()
    M, K, N = prob["M"], prob["K"], prob["N"]
    nidx = torch.empty((M, N, K), dtype=torch.int32, device="cuda")
    u_work = ps.u_nom.clone()
    fwd = aero.Problem(ps.cloud, M, K, N, prob["x0"], prob["p_goal"], u_work, coef=ps.coef,
                       v_goal=prob["v_goal"], q_goal=prob["q_goal"], S1=ps.S1, nearest_idx=nidx)
    bwd = aero.Problem(ps.cloud, M, K, N, prob["x0"], prob["p_goal"], ps.u_nom, coef=ps.coef,
                       v_goal=prob["v_goal"], q_goal=prob["q_goal"], nearest_idx=nidx)
    plain = aero.Problem(ps.cloud, M, K, N, prob["x0"], prob["p_goal"], ps.u_nom, coef=ps.coef,
                         v_goal=prob["v_goal"], q_goal=prob["q_goal"])
    ws = torch.empty(max(aero.workspace_size(aero.CALL_BACKWARD, [bwd]),
                         aero.workspace_size(aero.CALL_BACKWARD, [plain]),
                         aero.workspace_size(aero.CALL_MPPI_STEP, [fwd])), dtype=torch.uint8,
                     device="cuda")
    gu = torch.empty((M, N, 4), dtype=torch.float32, device="cuda")
    gw = torch.empty(5, dtype=torch.float32, device="cuda")
    res = {}
    legs = {
        "forward": lambda: (u_work.copy_(ps.u_nom), aero.mppi_step(prob["params"], [fwd], ws)),
        "backward": lambda: aero.mppi_step_backward_indexed(prob["params"], bwd, None, gu, gw, ws),
        "backward_self_contained": lambda: aero.mppi_step_backward(prob["params"], plain, None, gu,
                                                                   gw, ws),
    }
    for name in ("forward", "backward", "backward_self_contained"):
        once = legs[name]
        for _ in range(7):              # past the autotuner's per-shape timing trials
            once()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            once()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = e0.elapsed_time(e1) / iters
    res["backward_over_forward"] = res["backward_ms"] / res["forward_ms"]
    res["self_contained_backward_over_forward"] = res["backward_self_contained_ms"] / res["forward_ms"]
    res["workload"] = (f"gradient of sum S1 w.r.t. u_nom [{M}][{N}][4] and the 5 weights at the "
                       f"ensemble-forest-50k step (checkpoints every 8 steps); the forward "
                       f"stores nearest indices, the backward reads them")
    return res


def bench_paper_point(K, steps=200):
    """The paper's operating point (M=15, N=25, 120x60 partition, 200k-point cloud,
    P_f collision set), replayed from a HIP graph: planning rate on one GPU."""
    import torch

    from fixtures import make_paper_point_problem
    from paper_2509_17340_amd.planner import GraphStep, PlanStep

    prob = make_paper_point_problem(K=K)
    ps = PlanStep(prob)
    g = GraphStep(ps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        g.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    p50, p99 = pcts([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    ms = ev[0].elapsed_time(ev[-1]) / steps
    M, N = prob["M"], prob["N"]
    tensors = [ps.cloud, ps.tables, ps.fine_key, ps.fine_idx, ps.coarse_best, ps.anchor_cell,
               ps.anchor_fine, ps.anchors, ps.pf, ps.coef, ps.u_init, ps.u_nom, ps.S1, ps.S2,
               ps.best, ps.ws]
    mem = sum(t.numel() * t.element_size() for t in tensors)
    return {"ms_per_step": ms, "p50_ms": p50, "p99_ms": p99, "plans_per_s": 1e3 / ms,
            "rollout_steps_per_s": steps_per_plan_of(M, K, N) / (ms * 1e-3),
            "device_bytes": mem,
            "workload": f"M={M} (5x3), K={K}, N={N}, dt=0.05, 200k-point cloud within 10 m, "
                        "120x60 fine / 20x10 coarse partition, collision set P_f"}


def bench_batched(n_steps):
    """64 uneven problems: 64 plain per-problem calls vs one batched call."""
    import numpy as np
    import torch

    import paper_2509_17340_amd as aero
    from fixtures import make_batched_problems
    from paper_2509_17340_amd.planner import BatchPlan

    t0 = time.perf_counter()
    probs = make_batched_problems()
    log(f"batched fixtures: {time.perf_counter() - t0:.1f} s")
    bp = BatchPlan(probs)
    res = {}
    outs = {}
    for mode in ("plain", "batched"):
        run = bp.run_plain if mode == "plain" else bp.run_batched
        for _ in range(7):              # past the autotuner's per-shape timing trials
            bp.reset()
            run()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps + 1)]
        ev[0].record()
        for i in range(n_steps):
            bp.reset()
            run()
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[-1]) / n_steps
        p50, p99 = pcts([ev[i].elapsed_time(ev[i + 1]) for i in range(n_steps)])
        res[mode] = {"ms_per_step": ms, "p50_ms": p50, "p99_ms": p99,
                     "rollout_steps_per_s": bp.rollout_steps / (ms * 1e-3)}
        aero.timing_enable(True)
        aero.timing_read(reset=True)
        bp.reset()
        run()
        res[mode]["kernels_ms"] = kernel_ms(aero.timing_read(reset=True), 1)
        aero.timing_enable(False)
        outs[mode] = [(s.u_nom.cpu().numpy().copy(), s.S1.cpu().numpy().copy()) for s in bp.steps]
        outs[mode].append((bp.S2.cpu().numpy().copy(), bp.best.cpu().numpy().copy()))
        log(f"batched workload {mode}: {ms:.2f} ms/step")
    # the batched step captured as one HIP graph and replayed
    g = bp.graph()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps + 1)]
    ev[0].record()
    for i in range(n_steps):
        g.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / n_steps
    p50, p99 = pcts([ev[i].elapsed_time(ev[i + 1]) for i in range(n_steps)])
    graph_out = [(s.u_nom.cpu().numpy().copy(), s.S1.cpu().numpy().copy()) for s in bp.steps]
    res["batched_graph"] = {
        "ms_per_step": ms, "p50_ms": p50, "p99_ms": p99,
        "rollout_steps_per_s": bp.rollout_steps / (ms * 1e-3),
        "equals_eager_batched_bitwise": bool(
            all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
                for a, b in zip(outs["batched"][:-1], graph_out))
            and np.array_equal(bp.S2.cpu().numpy(), outs["batched"][-1][0]))}
    log(f"batched workload graph: {ms:.2f} ms/step")
    same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
               for a, b in zip(outs["plain"][:-1], outs["batched"][:-1]))
    plain_S2 = np.concatenate([s.S2.cpu().numpy() for s in bp.steps])
    same = same and np.array_equal(plain_S2, outs["batched"][-1][0])
    res.update(problems=len(probs), rollout_steps=bp.rollout_steps, pairs_brute_force=bp.pairs,
               speedup=res["plain"]["ms_per_step"] / res["batched"]["ms_per_step"],
               speedup_graph=res["plain"]["ms_per_step"] / res["batched_graph"]["ms_per_step"],
               batched_equals_plain_bitwise=bool(same), steps=n_steps,
               workload="64 uneven problems: forest / verticals+wall / incline scenes, "
                        "P ~ LogNormal(ln 5e4, 0.5) in [1e4, 2e5], M ~ U{4..16}, "
                        "K ~ U{512..4096}, N ~ U{30, 40, 60}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed closed-loop poses")
    ap.add_argument("--warmup", type=int, default=7, help="untimed closed-loop poses")
    ap.add_argument("--poses", type=int, default=200,
                    help="length of the flight for the plan-step distribution")
    ap.add_argument("--batched", type=int, default=3,
                    help="steps of the 64-problem batch, plain and batched (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lean", action="store_true",
                    help="headline only (no named legs, no CPU baseline)")
    ap.add_argument("--only", choices=("ensemble", "batched", "adjoint", "paper"),
                    help="run one named leg alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    K_steps, W = max(1, args.steps), max(0, args.warmup)
    n_total = max(args.poses, K_steps)
    workers = pool_size()
    if args.only:
        from fixtures import make_ensemble_problem
        leg = {"ensemble": lambda: bench_ensemble(make_ensemble_problem(), K_steps, W),
               "batched": lambda: bench_batched(max(1, args.batched)),
               "adjoint": lambda: bench_adjoint(make_ensemble_problem()),
               "paper": lambda: {"K128": bench_paper_point(128), "K256": bench_paper_point(256)}}
        print(json.dumps({"leg": args.only, **leg[args.only]()}))
        return

    # fixtures on the host pool, before anything touches the GPU
    t0 = time.perf_counter()
    with host_pool(workers) as ex:
        poses = list(ex.map(_loop_fixture, range(n_total)))
    log(f"{n_total} closed-loop poses generated in {time.perf_counter() - t0:.1f} s "
        f"on {workers} workers")

    import torch

    import paper_2509_17340_amd as aero
    from fixtures import make_ensemble_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    loop = bench_loop(poses, W, K_steps, n_total)
    M, K, N, P = loop["M"], loop["K"], loop["N"], loop["P"]
    ms = loop["total_ms"] / K_steps
    p50, p99 = pcts(loop["per"][:K_steps])
    a50, a99 = pcts(loop["per"])
    log(f"closed loop: {ms:.3f} ms per pose over {K_steps} timed poses; p50/p99 over "
        f"{n_total}: {a50:.2f} / {a99:.2f} ms")
    kt = loop["kt"]
    variant = loop["variant"]
    rl = distance_rooflines(kt, K_steps, loop["stats"], M * K * N * P * K_steps, variant,
                            "Stage I nearest distance")
    out = {
        "metric": METRIC,
        "value": steps_per_plan_of(M, K, N) / (ms * 1e-3),
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": K_steps,
        "warmup": W,
        "ms_per_step": ms,
        "plan_step_ms_p50": p50,
        "plan_step_ms_p99": p99,
        "launch_mode": "eager (per-pose host inputs change every step)",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "rollout and costs in f64; distances in f32 (exact pass), first "
                        "distance pass on split-f16 operands with f32 accumulation when "
                        "that variant is tuned in",
        "data": "synthetic",
        "config": {"workload": f"closed-loop-incline-1M: consecutive planning steps of a "
                               f"7 m/s flight through an incline corridor (M={M}, K={K}, "
                               f"N={N}, dt=0.04, {P}-point LiDAR cloud per pose, partition "
                               f"32x8 coarse x 4x4, Stage I + Stage II + one adjoint "
                               f"refinement + warm start)",
                   "M": M, "K": K, "N": N, "points": P, "collision_set": "raw cloud",
                   "rollout_steps_per_plan": steps_per_plan_of(M, K, N)},
        "roofline": dominant(rl, kt),
        "distance_passes": rl,
        "distance_work_per_step": {k: v / K_steps for k, v in loop["stats"].items()},
        "kernels_ms_per_step": kernel_ms(kt, K_steps),
        "kernels_note": "event-timed kernels of the planning step (partition .. Stage II); "
                        "the refinement and warm start run untimed after them",
        "closed_loop_flight": {"poses": n_total, "p50_ms": a50, "p99_ms": a99,
                               "max_ms": max(loop["per"]), "min_ms": min(loop["per"]),
                               "mean_ms": sum(loop["per"]) / n_total,
                               "note": "poses 0..P-1 of one flight, warm start carried; the "
                                       "first K are the timed region of `value`"},
    }
    out["roofline"]["traffic"] = measured_traffic(out["roofline"].get("kernel_name"),
                                                  "traffic_closed_loop_incline_1m.md")
    if not args.lean:
        prob2 = make_ensemble_problem()
        out["ensemble_forest_50k"] = bench_ensemble(prob2, 100, 20)
        log(f"ensemble: {out['ensemble_forest_50k']['ms_per_step']:.3f} ms/step (graph)")
        out["adjoint"] = bench_adjoint(prob2)
        out["paper_operating_point"] = {
            "K128": bench_paper_point(128), "K256": bench_paper_point(256),
            "paper_context": "500 Hz on GeForce RTX 4080 SUPER at K=128-256, N=25; "
                             "<600 MB at N=25, K=256 (Sec. V-B-1)"}
        if args.batched:
            out["batched_uneven_64"] = bench_batched(args.batched)
        if not args.no_cpu_baseline:
            log("cpu baseline: the oracle on a bounded sample of pose 0")
            out["cpu_baseline"] = cpu_baseline(poses[0], 24, workers)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
