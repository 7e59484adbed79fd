"""Benchmark: one AERO-MPPI planning step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the anchor-guided ensemble step on a synthetic forest LiDAR cloud of
50,000 points (partition 32 x 8 coarse cells refined 4 x 4, M = 8 instances,
K = 1024 samples, N = 40 steps, dt = 0.05 s), followed by Stage II.  A step is
partition -> anchors -> guides -> Stage I (noise, RK4, cost with brute-force
nearest distance, update) -> Stage II (explicit rollouts, argmin), all with
inputs resident in device memory.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPPI rollout-steps/s + plan-step ms; batched/adjoint vs plain, same GPU, ≤1e-4"
FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
FLOP_PER_PAIR = 8             # 3 sub + 3 mul + 2 add per (position, point) pair

# Pass-A variants: kernel, roofline bound and the published peak of the unit it runs
# on, the FLOP it executes per pair, and the source file holding it.
PASS_A = {
    0: dict(kernel="k_min_dist_approx", bound="alu", peak=FP32_PEAK_TFLOPS,
            unit_note="FP32 vector (VALU) peak", executed_flop_per_pair=6,
            source="paper_2509_17340_amd/csrc/distance.hip"),
    1: dict(kernel="k_min_dist_approx_mfma", bound="mfma", peak=157.3,
            unit_note="FP32 dense MFMA peak", executed_flop_per_pair=8,
            source="paper_2509_17340_amd/csrc/distance_mfma.hip"),
    2: dict(kernel="k_min_dist_approx_f16s", bound="mfma", peak=2500.0,
            unit_note="FP16 dense MFMA peak (split hi/lo operands, FP32 accumulation)",
            executed_flop_per_pair=32,
            source="paper_2509_17340_amd/csrc/distance_mfma.hip"),
}
# Pair-rate ceiling of the split-FP16 pass: the K = 16 MFMA (32 FLOP per pair at the
# FP16 dense peak) and the running minimum (one v_min3_f32 per two pairs on 16 lanes
# x 4 SIMDs x 256 CUs at 2.4 GHz) both allow about 7.8e13 pairs/s.
F16S_PAIR_CEILING = min(2500e12 / 32, 16 * 4 * 256 * 2.4e9 * 2)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_ensemble_forest_50k.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and line.startswith("    "):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or "kernel_source" not in kv:
        return None
    src = os.path.join(ROOT, kv["kernel_source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return int(kv["traffic_bytes_per_launch"]) if sha == kv.get("kernel_source_sha256") else None


def steps_per_plan_of(prob):
    return prob["M"] * prob["K"] * prob["N"] + prob["M"] * prob["N"]


def cpu_baseline(prob, samples_per_instance=32):
    """The oracle as it is, on a bounded sample of the same planning step."""
    import numpy as np

    from oracle import guides as OG
    from oracle import mppi as OM
    from oracle import partition as OP
    from oracle import philox as OPh

    part = prob["partition"]
    M, K, N = prob["M"], prob["K"], prob["N"]
    prm = prob["params"]
    t0 = time.perf_counter()
    pa = OP.partition_anchors(prob["cloud"], prob["goal_dir"], part["n_az_c"], part["n_el_c"],
                              part["f_a"], part["f_e"], part["r_max"], part["ell"],
                              prob["M_h"], prob["M_v"])
    T = np.float32(N * np.float32(prm["dt"]))
    coef = OG.build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3), pa["anchors"], T)
    t1 = time.perf_counter()
    normals = OPh.normals(prm["seed"], prob["problem_id"], M, K, N, prm["iter_base"])
    sub = np.arange(0, K, K // samples_per_instance)[:samples_per_instance]
    p2 = dict(prob)
    p2["K"] = len(sub)
    t2 = time.perf_counter()
    st = OM.mppi_step(p2, coef, normals=normals[:, sub])
    t3 = time.perf_counter()
    OM.select_best(prob, st["u_new"])
    t4 = time.perf_counter()
    full = (t1 - t0) + (t3 - t2) * (K / len(sub)) + (t4 - t3)
    steps = M * K * N + M * N
    return {
        "value": steps / full, "unit": "rollout-steps/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 NumPy oracle, single thread: partition+guides and Stage II in full, "
                   f"Stage I on {len(sub)} of {K} samples per instance (brute-force nearest "
                   f"over all {len(prob['cloud'])} points), extrapolated to the full step "
                   f"({full:.1f} s/step; measured {t4 - t0:.1f} s)"),
        "host_cpus": os.cpu_count(),
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
        for _ in range(3):
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
    res["workload"] = (f"gradient of sum S1 w.r.t. u_nom [{M}][{N}][4] and the 5 weights, "
                       f"same inputs as the headline step (checkpoints every 8 steps); the forward "
                       f"stores nearest indices, the backward reads them")
    return res


def bench_paper_point(steps=200):
    """The paper's operating point (M=15, K=128, N=25, 120x60 partition, 200k-point
    cloud, P_f collision set), replayed from a HIP graph: planning rate on one GPU."""
    import torch

    from fixtures import make_paper_point_problem
    from paper_2509_17340_amd.planner import GraphStep, PlanStep

    prob = make_paper_point_problem()
    ps = PlanStep(prob)
    g = GraphStep(ps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        g.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    ms = ev[0].elapsed_time(ev[-1]) / steps
    M, K, N = prob["M"], prob["K"], prob["N"]
    tensors = [ps.cloud, ps.tables, ps.fine_key, ps.fine_idx, ps.coarse_best, ps.anchor_cell,
               ps.anchor_fine, ps.anchors, ps.pf, ps.coef, ps.u_init, ps.u_nom, ps.S1, ps.S2,
               ps.best, ps.ws]
    mem = sum(t.numel() * t.element_size() for t in tensors)
    return {"ms_per_step": ms, "p50_ms": per[steps // 2], "p99_ms": per[int(0.99 * steps)],
            "plans_per_s": 1e3 / ms, "rollout_steps_per_s": (M * K * N + M * N) / (ms * 1e-3),
            "device_bytes": mem,
            "workload": f"M={M} (5x3), K={K}, N={N}, dt=0.05, 200k-point cloud within 10 m, "
                        "120x60 fine / 20x10 coarse partition, collision set P_f",
            "paper_context": "500 Hz on GeForce RTX 4080 SUPER at K=128-256, N=25; "
                             "<600 MB at N=25, K=256 (Sec. V-B-1)"}


def bench_loop(n_steps, stride=40):
    """Closed loop over replayed poses of the incline flight (7 m/s): M=16, K=8192,
    N=60, dt=0.04, 1,000,000-point cloud per step, plus one adjoint refinement of
    the selected plan and the warm start.  Cloud upload excluded from the timing."""
    import torch

    from fixtures import make_loop_step
    from paper_2509_17340_amd.planner import LoopRunner

    poses = [i * stride for i in range(n_steps)]
    t0 = time.perf_counter()
    probs = [make_loop_step(s) for s in poses]
    print(f"# loop fixtures: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    lr = LoopRunner(probs[0])
    for _ in range(3):                  # warm-up: the autotuner's timing trials
        lr.load(probs[0])
        lr.step()
    torch.cuda.synchronize()
    times = []
    for p in probs:
        lr.load(p)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lr.step()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        print(f"# loop pose {len(times)}: {times[-1]:.1f} ms", file=sys.stderr, flush=True)
    ps = lr.ps
    steps = ps.M * ps.K * ps.N + ps.M * ps.N
    srt = sorted(times)
    return {"poses": poses, "ms": times, "p50_ms": srt[len(srt) // 2], "p99_ms": srt[-1],
            "rollout_steps_per_s": steps / (sum(times) / len(times) * 1e-3),
            "pairs_per_step": ps.M * ps.K * ps.N * int(ps.cloud.shape[0]),
            "workload": "incline corridor, 7 m/s replayed poses, M=16 (8x2), K=8192, N=60, "
                        "dt=0.04, 1e6-point cloud, + adjoint refinement of the selected plan "
                        "(4 step candidates) and warm start; p99 over the timed poses"}


def bench_batched(n_steps):
    """64 uneven problems: 64 plain per-problem calls vs one batched call."""
    import numpy as np
    import torch

    from fixtures import make_batched_problems
    from paper_2509_17340_amd.planner import BatchPlan

    t0 = time.perf_counter()
    probs = make_batched_problems()
    print(f"# batched fixtures: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    bp = BatchPlan(probs)
    res = {}
    outs = {}
    for mode in ("plain", "batched"):
        run = bp.run_plain if mode == "plain" else bp.run_batched
        for _ in range(4):              # past the autotuner's per-shape timing trials
            bp.reset()
            run()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(n_steps):
            bp.reset()
            run()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / n_steps
        res[mode] = {"ms_per_step": ms, "rollout_steps_per_s": bp.rollout_steps / (ms * 1e-3)}
        outs[mode] = [(s.u_nom.cpu().numpy().copy(), s.S1.cpu().numpy().copy()) for s in bp.steps]
        print(f"# batched workload {mode}: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
               for a, b in zip(outs["plain"], outs["batched"]))
    res.update(problems=len(probs), rollout_steps=bp.rollout_steps, pairs=bp.pairs,
               speedup=res["plain"]["ms_per_step"] / res["batched"]["ms_per_step"],
               batched_equals_plain_bitwise=bool(same), steps=n_steps,
               workload="64 uneven problems: forest / verticals+wall / incline scenes, "
                        "P ~ LogNormal(ln 5e4, 0.5) in [1e4, 2e5], M ~ U{4..16}, "
                        "K ~ U{512..4096}, N ~ U{30, 40, 60}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--loop", type=int, default=5,
                    help="closed-loop leg: number of replayed poses (0 = skip)")
    ap.add_argument("--lean", action="store_true",
                    help="headline step only (no graph, adjoint, paper-point or CPU legs)")
    ap.add_argument("--batched", type=int, default=0,
                    help="also time the 64-problem uneven batch (plain vs batched), N steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_17340_amd as aero
    from fixtures import make_ensemble_problem
    from paper_2509_17340_amd.planner import PlanStep

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = make_ensemble_problem()
    M, K, N, P = prob["M"], prob["K"], prob["N"], len(prob["cloud"])
    ps = PlanStep(prob)
    print(f"# workload M={M} K={K} N={N} P={P}; warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ps.reset()
        ps.run()
    torch.cuda.synchronize()

    aero.timing_enable(True)
    aero.timing_read(reset=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for i in range(args.steps):
        ps.reset()
        ps.run()
        evs[i + 1].record()
    torch.cuda.synchronize()
    ms = evs[0].elapsed_time(evs[-1]) / args.steps
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    kt = aero.timing_read(reset=True)
    aero.timing_enable(False)
    print(f"# timed {args.steps} eager steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    if args.lean:
        print(json.dumps({"metric": METRIC, "value": steps_per_plan_of(prob) / (ms * 1e-3),
                          "ms_per_step": ms, "kernels_ms_per_step":
                          {k: v[0] / args.steps for k, v in kt.items()}}))
        return
    # the same step captured once as a HIP graph and replayed
    from paper_2509_17340_amd.planner import GraphStep
    g = GraphStep(ps)
    gev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    gev[0].record()
    for i in range(args.steps):
        g.replay()
        gev[i + 1].record()
    torch.cuda.synchronize()
    gms = gev[0].elapsed_time(gev[-1]) / args.steps
    g_steps = sorted(gev[i].elapsed_time(gev[i + 1]) for i in range(args.steps))
    print(f"# timed {args.steps} graph replays: {gms:.3f} ms/step", file=sys.stderr, flush=True)

    steps_per_plan = M * K * N + M * N
    md_ms, md_n = kt["min_dist"]
    md_avg = md_ms / max(md_n, 1)
    pairs = (M * K * N) * P
    flop = FLOP_PER_PAIR * pairs
    achieved = flop / (md_avg * 1e-3) / 1e12
    variant = aero.pass_a_variant([ps.problem])
    va = PASS_A.get(variant, PASS_A[0])
    pairs_per_s = pairs / (md_avg * 1e-3)
    dist_ms = (kt["min_dist"][0] + kt["flag"][0] + kt["min_dist_exact"][0]) / args.steps
    best_ms = min(ms, gms)
    out = {
        "metric": METRIC,
        "value": steps_per_plan / (best_ms * 1e-3),
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best_ms,
        "launch_mode": "hip_graph" if gms <= ms else "eager",
        "eager_ms_per_step": ms,
        "graph_ms_per_step": gms,
        "plan_step_ms_p50": (g_steps if gms <= ms else per_step)[args.steps // 2],
        "plan_step_ms_p99": (g_steps if gms <= ms else per_step)[
            min(args.steps - 1, int(0.99 * args.steps))],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "rollout and costs in f64; distances in f32 (exact pass), pass A on "
                        "split-f16 operands with f32 accumulation when that variant is tuned in",
        "data": "synthetic",
        "config": {"workload": f"ensemble-forest-{P // 1000}k: one planning step "
                               f"(partition 32x8 coarse x 4x4, M={M}, K={K}, N={N}, dt=0.05, "
                               f"{P}-point LiDAR cloud, Stage I + Stage II)",
                   "M": M, "K": K, "N": N, "points": P, "collision_set": "raw cloud"},
        "roofline": {"bound": va["bound"],
                     "kernel": va["kernel"] + " (Stage I nearest distance, pass A over every "
                               "rollout position; autotuned variant %d)" % variant,
                     "achieved": achieved, "peak": va["peak"], "unit": "TFLOP/s",
                     "peak_is": va["unit_note"],
                     "frac": achieved / va["peak"], "traffic": measured_traffic(va["kernel"]),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "flop_per_launch": flop, "flop_counted": "8 per (position, point) pair",
                     "avg_launch_ms": md_avg, "pairs_per_s": pairs_per_s,
                     "executed_tflops": va["executed_flop_per_pair"] * pairs_per_s / 1e12,
                     "executed_frac": va["executed_flop_per_pair"] * pairs_per_s / 1e12 / va["peak"],
                     "distance_all_passes_ms": dist_ms,
                     "distance_all_passes_tflops": flop / (dist_ms * 1e-3) / 1e12},
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
    }
    # the cost kernel's algorithmic FLOP rate against the FP32 vector peak (the scale
    # on which the plain VALU form of the pass is judged), whichever variant runs
    out["roofline"]["algorithmic_frac_of_fp32_valu_peak"] = achieved / FP32_PEAK_TFLOPS
    if variant == 2:
        out["roofline"]["pair_ceiling_per_s"] = F16S_PAIR_CEILING
        out["roofline"]["frac_of_pair_ceiling"] = pairs_per_s / F16S_PAIR_CEILING
    out["adjoint"] = bench_adjoint(prob)
    out["paper_operating_point"] = bench_paper_point()
    if args.batched:
        out["batched"] = bench_batched(args.batched)
    if args.loop:
        out["closed_loop"] = bench_loop(args.loop)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle on a bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
