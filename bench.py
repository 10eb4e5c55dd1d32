"""Benchmark: WNNC normal orientation of a 500k-point cloud on one MI355X.

One step = the whole hot path on one synthetic cloud already resident in
device memory: normalization, octree build, 40 iterations of Alg. 3 (each a
gradient step with A, A^T, A and a WNNC update with G, with the moment pass
before every operator), and the unit-normal output.

Prints one JSON line.  ``value`` is pair interactions per second over the
whole step (every near and far pair evaluation of every operator call,
counted in a separate counting run with identical decisions), ``ms_per_step``
the 40-iteration wall time.  ``roofline`` is for the traversal kernel with
the largest total time, timed with HIP events on the library's stream during
the timed steps.  ``cpu_baseline`` times the FP64 oracle treecode on a sample
of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WNNC 40-iter time & Gpair-interactions/s at N=500k; warm-start vs plain speedup"
FLOPS_PER_PAIR = {0: 18, 1: 18, 2: 31}  # A, A^T, G (FMA = 2, rsqrt = 1)
KIND = {0: "A", 1: "AT", 2: "G"}
PEAK_FP32_TFLOPS = 157.3


def load_profile(name: str, grid=None):
    """A committed rocprofv3 summary (profiles/NAME.json), if it was taken on
    the current traversal sources (and, given `grid`, on dispatches of that
    many threads: the same workload and launch configuration)."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    from paper_2405_16634_amd.profiling import traversal_digest
    if d.get("source_sha") != traversal_digest():
        return None
    if grid is not None and d.get("grid_threads") != grid:
        return None
    return d


def moments_counters(st_all, calls_per_run):
    """HBM bytes of the moment pass per call (committed counter summary of
    the benchmark cloud's chunk and straddler passes) over this run's
    average moment-pass time per call."""
    path = os.path.join(ROOT, "profiles", "traffic_moments_torusknot500k.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    n_calls = sum(int(calls_per_run[k]) for k in range(3))
    per_call_ms = st_all["moments_ms"] / max(n_calls, 1)
    b = tr["bytes_per_call"]
    return {"bytes_per_call": b, "ms_per_call": round(per_call_ms, 4),
            "gb_per_s": round(b / (per_call_ms * 1e-3) / 1e9, 1),
            "frac_of_8TBps": round(b / (per_call_ms * 1e-3) / 8e12, 4)}


def cpu_baseline(cloud, w: float, c: float):
    """The FP64 oracle treecode on the same cloud for one WNNC iteration's
    four operator calls (A, A^T, A, G over all points; a run has 159), from
    the ground-truth-normal state.  Reports pair interactions per second."""
    import oracle
    x, _, sc = oracle.normalize(cloud.points)
    x = x.astype(np.float64)
    mu = cloud.normals.astype(np.float64) * (cloud.area * sc * sc / cloud.n)
    mu[~np.isfinite(mu).all(axis=1)] = 0.0
    t0 = time.perf_counter()
    T = oracle.Tree(x)
    t1 = time.perf_counter()
    p = 0
    s, _, k = T.apply("A", mu, w, c, with_stats=True)
    p += int(k.sum())
    r, _, k = T.apply("AT", 0.5 - s, w, c, with_stats=True)
    p += int(k.sum())
    _, _, k = T.apply("A", r, w, c, with_stats=True)
    p += int(k.sum())
    _, _, k = T.apply("G", mu, w, c, with_stats=True)
    p += int(k.sum())
    t2 = time.perf_counter()
    return {
        "value": round(p / (t2 - t1) / 1e9, 4),
        "unit": "Gpair-interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle treecode (C, OpenMP): one iteration's 4 operator calls (A, A^T, A, G; "
                   f"159 per 40-iteration run) over all {cloud.n} points of the torus-knot cloud, "
                   f"{p} pairs in {t2 - t1:.2f} s; oracle tree build {t1 - t0:.2f} s not included"),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_plan():
    """The FP64 oracle timed as the measurement plan states it, on the host
    cores: the treecode run (Alg. 3, 40 iterations of Alg. 4 operators) on
    the 50k noisy ellipsoid union (widths 0.02 -> 0.08, the 0.25 % noise
    setting of Sec. 5.2.5), T_pre (operator set-up: normalization and the
    octree) and T_main (the iterations) separately, median of 3 on all
    cores and one run on one thread; the exact direct sums for the 40
    iterations on the 2k sphere and for one operator call on the 50k cloud.
    Pair counts give the CPU rates beside the device's."""
    import oracle
    import synth
    from statistics import median
    out = {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "kind": "oracle"}
    all_threads = oracle.num_threads()
    c2 = synth.ellipsoid_union(50000, 2)

    def tree_run(threads):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        x, _, _ = oracle.normalize(c2.points)
        t1 = time.perf_counter()
        tm, pc = {}, [0]
        oracle.orient(x, iters=40, w1=0.02, w2=0.08, backend="tree", pair_count=pc, timing=tm)
        return (t1 - t0) + tm["pre"], tm["main"], pc[0]

    runs = [tree_run(all_threads) for _ in range(3)]
    pre = median(r[0] for r in runs)
    main = median(r[1] for r in runs)
    pairs = runs[0][2]
    one = tree_run(1)
    oracle.set_threads(all_threads)
    out["treecode_ellipsoids50k_40iter"] = {
        "threads": all_threads, "t_pre_s": round(pre, 4), "t_main_s": round(main, 3),
        "t_main_runs_s": [round(r[1], 3) for r in runs], "pairs": pairs,
        "gpairs_per_s": round(pairs / main / 1e9, 4),
        "one_thread": {"t_pre_s": round(one[0], 4), "t_main_s": round(one[1], 3),
                       "gpairs_per_s": round(one[2] / one[1] / 1e9, 4)}}
    c1 = synth.fibonacci_sphere(2000, 0)
    x1, _, _ = oracle.normalize(c1.points)
    t0 = time.perf_counter()
    oracle.orient(x1, iters=40, w1=0.002, w2=0.016, backend="direct")
    t1 = time.perf_counter()
    n1 = c1.n
    out["direct_sphere2k_40iter"] = {
        "threads": all_threads, "t_s": round(t1 - t0, 4), "pairs": 159 * n1 * n1,
        "gpairs_per_s": round(159 * n1 * n1 / (t1 - t0) / 1e9, 4)}
    x2, _, sc = oracle.normalize(c2.points)
    mu = c2.normals.astype(np.float64) * (c2.area * sc * sc / c2.n)
    t0 = time.perf_counter()
    oracle.direct("A", x2, mu, 0.02)
    t1 = time.perf_counter()
    out["direct_ellipsoids50k_one_A"] = {
        "threads": all_threads, "t_s": round(t1 - t0, 3), "pairs": c2.n * c2.n,
        "gpairs_per_s": round(c2.n * c2.n / (t1 - t0) / 1e9, 4)}
    return out


def _dirs(a, b, mask):
    """Flip rate and AE_pcd (Sec. 5.1.4) of directions a against b over mask
    (rows where both are nonzero and finite)."""
    from paper_2405_16634_amd.metrics import ae_pcd, flip_rate
    return flip_rate(a, b, mask), ae_pcd(a, b, mask)


def _timed(stream, fn):
    """Device time (ms, HIP events on `stream`) of fn() and its result."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    r = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), r


def warm_start_section(ctx, w, mu_plain, stream, iters, w1, w2, gt, mu0_random):
    """Warm-started orientation on the same cloud and tree against the plain
    run (mu_plain, 40 iterations from mu = 0), with the trained network in the
    package data.  Equal accuracy: on the surface points (outliers have no
    normal), a result disagrees with the plain one on at most 0.1 % of the
    points and orients at least as many correctly (P_co against the
    generator's normals gt, within 0.1 %).  Beside it: the same short
    schedule from mu = 0 without the network (what the network adds), the
    warm start continued until at most 0.1 % of the points change sign per
    update (or the count stops falling), and the plain method from
    random initial vectors scaled by the mean area (mu0_random)."""
    import torch
    from paper_2405_16634_amd import warmstart as ws
    if not os.path.exists(ws.DEFAULT_WEIGHTS):
        return None
    params = ws.load_params(ws.DEFAULT_WEIGHTS)
    out = torch.empty_like(mu_plain)
    w.wnnc_warm_orient(ctx.handle, params, out)  # warm-up
    t_plain, _ = _timed(stream, lambda: w.wnnc_orient(ctx.handle, mu_plain, None, iters, w1, w2))
    t_warm, rep = _timed(stream, lambda: w.wnnc_warm_orient(ctx.handle, params, out))
    warm_iters = 6  # the warm schedule's length (wnnc_warm_opts default)
    ctrl = torch.empty_like(mu_plain)
    t_ctrl, _ = _timed(stream, lambda: w.wnnc_orient(ctx.handle, ctrl, None, warm_iters, w1, w2))
    conv = torch.empty_like(mu_plain)
    t_conv, rep_c = _timed(stream, lambda: w.wnnc_warm_orient(ctx.handle, params, conv,
                                                              max_iters=iters, stop_frac=1e-3))
    rnd = torch.empty_like(mu_plain)
    m0 = torch.from_numpy(mu0_random).to(mu_plain.device)
    t_rnd, _ = _timed(stream, lambda: w.wnnc_orient(ctx.handle, rnd, m0, iters, w1, w2))
    torch.cuda.synchronize()
    pred = torch.empty_like(mu_plain)
    feat = torch.empty(mu_plain.shape[0], 48, device=mu_plain.device, dtype=torch.float32)
    w.wnnc_knn_features(ctx.handle, feat, None)
    w.wnnc_mlp_forward(ctx.handle, params, feat, pred)
    a = mu_plain.cpu().numpy().astype(np.float64)
    b = out.cpu().numpy().astype(np.float64)
    pr = pred.cpu().numpy().astype(np.float64)
    surf = np.isfinite(gt).all(axis=1)
    every = np.ones(len(a), bool)
    flip_s, _ = _dirs(b, a, surf)
    flip_all, _ = _dirs(b, a, every)
    pco_plain = 1.0 - _dirs(a, gt, surf)[0]
    pco_warm = 1.0 - _dirs(b, gt, surf)[0]
    pred_flip, pred_ae = _dirs(pr, a, surf)

    def judged(m, ms, extra=None):
        r = m.cpu().numpy().astype(np.float64)
        f_s = _dirs(r, a, surf)[0]
        pc = 1.0 - _dirs(r, gt, surf)[0]
        d = {"ms": round(ms, 3), "flip_vs_plain_surface": round(f_s, 6),
             "flip_vs_plain_all_points": round(_dirs(r, a, every)[0], 6), "P_co": round(pc, 6),
             "equal_accuracy": bool(f_s <= 1e-3 and pc >= pco_plain - 1e-3)}
        d.update(extra or {})
        return d

    return {"plain_ms": round(t_plain, 3), "warm_ms": round(t_warm, 3),
            "speedup": round(t_plain / t_warm, 3), "plain_iterations": iters,
            "warm_iterations": rep["iterations"], "fallback": rep["fallback"],
            "self_check_max_disagree": round(rep["max_disagree"], 6),
            "self_check_max_pred_disagree": round(rep["max_pred_disagree"], 6),
            "flip_vs_plain_surface": round(flip_s, 6), "flip_vs_plain_all_points": round(flip_all, 6),
            "P_co_plain": round(pco_plain, 6), "P_co_warm": round(pco_warm, 6),
            "prediction_vs_plain": {"flip": round(pred_flip, 5), "AE_pcd": round(pred_ae, 5)},
            "equal_accuracy": bool(flip_s <= 1e-3 and pco_warm >= pco_plain - 1e-3),
            "control_same_schedule_no_network": judged(ctrl, t_ctrl, {"iterations": warm_iters}),
            "until_convergence": judged(conv, t_conv, {"iterations": rep_c["iterations"],
                                                       "fallback": rep_c["fallback"],
                                                       "max_iters": iters}),
            "random_init_plain": judged(rnd, t_rnd, {"iterations": iters,
                                                     "speedup_of_warm": round(t_rnd / t_warm, 3)})}


def far_field_section(ctx, w, step, mu, stream, steps, normals):
    """The same step with the order-2 far field and the cutoff-safe
    acceptance (the precision-control extension): time per step, per-kind
    traversal launch times, and agreement with the generator's normals."""
    import torch
    ctx.set_far_field(2, True)
    step()
    ctx.set_flags(w.FLAG_TIME_KERNELS)
    ctx.reset_stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    st = ctx.stats()
    ctx.set_flags(0)
    ctx.set_far_field(0, False)
    ms = e0.elapsed_time(e1) / steps
    m = mu.cpu().numpy()
    ok = np.isfinite(normals).all(axis=1)
    pco = float(((m[ok] * normals[ok]).sum(1) > 0).mean())
    return {"order": 2, "wsafe": True, "ms_per_step": round(ms, 3),
            "traverse_avg_ms": {KIND[k]: round(st["traverse_ms"][k] / max(st["calls"][k], 1), 4)
                                for k in range(3)},
            "moments_ms_per_step": round(st["moments_ms"] / steps, 3),
            "P_co": round(pco, 5)}


def leaf_cap_section(w, P, stream, iters, w1, w2, c, depth, steps, normals, K=8):
    """The same step on a tree whose leaves hold up to K points (an
    extension: the paper splits down to single points); the targets that do
    not accept such a leaf sum its points directly."""
    import torch
    ctx = w.Context(0, stream)
    Pn = torch.empty_like(P)
    mu = torch.empty_like(P)
    nrm = torch.empty_like(P)

    def step():
        cs = w.wnnc_normalize(ctx.handle, P, Pn)
        w.wnnc_build(ctx.handle, Pn, c, depth, K)
        w.wnnc_orient(ctx.handle, mu, None, iters, w1, w2)
        w.wnnc_normals(ctx.handle, mu, cs[1], nrm)

    w.wnnc_normalize(ctx.handle, P, Pn)
    w.wnnc_build(ctx.handle, Pn, c, depth, K)
    ctx.autotune(w1)
    ctx.set_flags(w.FLAG_COUNT_PAIRS)
    ctx.reset_stats()
    step()
    torch.cuda.synchronize()
    pairs = int(sum(ctx.stats()["pairs"][:3]))
    ctx.set_flags(0)
    step()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    m = nrm.cpu().numpy()
    ok = np.isfinite(normals).all(axis=1)
    pco = float(((m[ok] * normals[ok]).sum(1) > 0).mean())
    ctx.close()
    return {"leaf_cap": K, "ms_per_step": round(ms, 3), "pairs_per_step": pairs,
            "gpairs_per_s": round(pairs / (ms * 1e-3) / 1e9, 3), "P_co": round(pco, 5)}


def union50k_section(w, stream, iters, c, depth, steps):
    """The 50k-point noisy ellipsoid union (6 members, 0.25 % noise, seed 2;
    widths 0.02 -> 0.08 for that noise): the whole step (normalize, build,
    40 iterations, output) after the autotuner, the median of `steps`
    timed steps, with the build and the iterations split as in the main
    line; accuracy against the generator's normals."""
    import torch
    import synth
    from paper_2405_16634_amd.metrics import p_co
    cloud = synth.ellipsoid_union(50000, 2)
    w1, w2 = 0.02, 0.08
    P = torch.from_numpy(cloud.points).to("cuda:0")
    ctx = w.Context(0, stream)
    Pn = torch.empty_like(P)
    mu = torch.empty_like(P)
    nrm = torch.empty_like(P)
    w.wnnc_normalize(ctx.handle, P, Pn)
    w.wnnc_build(ctx.handle, Pn, c, depth)
    ctx.autotune(w1)
    ctx.set_flags(w.FLAG_COUNT_PAIRS)
    ctx.reset_stats()
    w.wnnc_orient(ctx.handle, mu, None, iters, w1, w2)
    torch.cuda.synchronize()
    pairs = int(sum(ctx.stats()["pairs"][:3]))
    ctx.set_flags(0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    pre, main = [], []
    for rep in range(steps + 1):
        ev[0].record(stream)
        cs = w.wnnc_normalize(ctx.handle, P, Pn)
        w.wnnc_build(ctx.handle, Pn, c, depth)
        ev[1].record(stream)
        w.wnnc_orient(ctx.handle, mu, None, iters, w1, w2)
        w.wnnc_normals(ctx.handle, mu, cs[1], nrm)
        ev[2].record(stream)
        torch.cuda.synchronize()
        if rep > 0:  # the first is a warm-up
            pre.append(ev[0].elapsed_time(ev[1]))
            main.append(ev[1].elapsed_time(ev[2]))
    tot = [a + b for a, b in zip(pre, main)]
    k = int(np.argsort(tot)[len(tot) // 2])
    pco = p_co(nrm.cpu().numpy(), cloud.normals)
    ctx.close()
    return {"workload": "ellipsoids50k", "n_points": cloud.n, "iters": iters, "w1": w1, "w2": w2,
            "ms_per_step": round(tot[k], 3), "t_pre_ms": round(pre[k], 3),
            "t_main_ms": round(main[k], 3), "pairs_per_step": pairs,
            "gpairs_per_s": round(pairs / (tot[k] * 1e-3) / 1e9, 3), "P_co": round(pco, 5),
            "timing": f"median of {steps} steps after one warm-up (HIP events)"}


def batched_section(w, stream, iters, w1, w2, c, depth):
    """The 64-cloud workload (sizes log-uniform in [5k, 200k], seed 1): one
    forest with one launch per operator and per-cloud step lengths, against
    the same clouds run one by one (normalize, build, 40 iterations each),
    wall time on the same GPU; equal accuracy as the flip rate between the
    two results."""
    import torch
    import synth
    sizes = synth.batched_sizes(64, 1)
    clouds = synth.batched_clouds(64, 1, sizes)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P = torch.from_numpy(np.concatenate([cl.points for cl in clouds])).to("cuda:0")
    ctx = w.Context(0, stream)
    Pn = torch.empty_like(P)
    mu_b = torch.empty_like(P)

    def batched():
        w.wnnc_normalize_batched(ctx.handle, P, Pn, off)
        w.wnnc_build_batched(ctx.handle, Pn, off, c, depth)
        w.wnnc_orient(ctx.handle, mu_b, None, iters, w1, w2)

    batched()
    ctx.autotune(w1)
    batched()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    batched()
    e1.record(stream)
    torch.cuda.synchronize()
    t_batched = e0.elapsed_time(e1)
    one = w.Context(0, stream)
    parts = [P[off[k]:off[k + 1]] for k in range(64)]
    outs = [torch.empty_like(p_) for p_ in parts]
    norms = [torch.empty_like(p_) for p_ in parts]

    def one_by_one():
        for p_, q_, o_ in zip(parts, norms, outs):
            w.wnnc_normalize(one.handle, p_, q_)
            w.wnnc_build(one.handle, q_, c, depth)
            w.wnnc_orient(one.handle, o_, None, iters, w1, w2)

    one_by_one()
    torch.cuda.synchronize()
    e0.record(stream)
    one_by_one()
    e1.record(stream)
    torch.cuda.synchronize()
    t_single = e0.elapsed_time(e1)
    a = mu_b.cpu().numpy()
    b = torch.cat(outs).cpu().numpy()
    flip = float(((a * b).sum(1) <= 0).mean())
    po = ctx.stats()["prefetch_ops"]
    tile = {"targets_per_lane": ctx.tile(), "prefetch": bool(ctx.prefetch()),
            "split_visits": ctx.split(),
            "prefetch_by_op": {KIND[k]: bool((po >> k) & 1) for k in range(3)}}
    ctx.close()
    one.close()
    return {"clouds": 64, "points": int(off[-1]), "tile": tile, "batched_ms": round(t_batched, 2),
            "one_by_one_ms": round(t_single, 2), "speedup": round(t_single / t_batched, 3),
            "flip_batched_vs_one_by_one": flip, "equal_accuracy": bool(flip <= 1e-3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=500000)
    ap.add_argument("--iters", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--core-only", action="store_true",
                    help="only the timed steps and their figures (no warm-start, far-field, "
                         "leaf-capacity or batched sections): for profiling runs")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="only time the CPU oracle as the measurement plan states it "
                         "(about two minutes) and print that JSON")
    ap.add_argument("--split", type=int, default=None,
                    help="walk split (node visits per part) used after the autotuner instead "
                         "of its choice: for profiling runs of one launch configuration")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(multi-GPU sharding is a design note only).", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.cpu_plan:
        print(json.dumps(cpu_plan()), flush=True)
        return

    import torch
    import paper_2405_16634_amd as w
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w1, w2, c, depth = 0.002, 0.016, 2.0, 15
    cloud = synth.torus_knot(args.n, 3)
    P = torch.from_numpy(cloud.points).to(dev)
    stream = torch.cuda.current_stream()
    ctx = w.Context(0, stream)
    Pn = torch.empty_like(P)
    mu = torch.empty_like(P)
    nrm = torch.empty_like(P)

    def step():
        cs = w.wnnc_normalize(ctx.handle, P, Pn)
        w.wnnc_build(ctx.handle, Pn, c, depth)
        w.wnnc_orient(ctx.handle, mu, None, args.iters, w1, w2)
        w.wnnc_normals(ctx.handle, mu, cs[1], nrm)

    # tile shape, prefetch and split size: the autotuner times each on this
    # tree; later builds keep the choice
    cs0 = w.wnnc_normalize(ctx.handle, P, Pn)
    w.wnnc_build(ctx.handle, Pn, c, depth)
    tile_ms = ctx.autotune(w1)
    if args.split is not None:
        ctx.set_split(args.split)

    # pair counts: one run with the counting kernels (same decisions)
    ctx.set_flags(w.FLAG_COUNT_PAIRS)
    ctx.reset_stats()
    step()
    torch.cuda.synchronize()
    cst = ctx.stats()
    pairs = cst["pairs"]
    calls_per_run = cst["calls"]
    total_pairs = int(sum(pairs))

    ctx.set_flags(0)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed steps; each traversal launch carries HIP events (on the library's
    # stream), the other launches none
    ctx.set_flags(w.FLAG_TIME_TRAVERSAL)
    ctx.reset_stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_host1 = time.perf_counter()
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    st = ctx.stats()
    ctx.set_flags(0)
    # the moment and combining passes: one more step with every launch timed
    ctx.set_flags(w.FLAG_TIME_KERNELS)
    ctx.reset_stats()
    step()
    torch.cuda.synchronize()
    st_all = ctx.stats()
    # and once more with the split walks' combining passes as launches of
    # their own (the moment passes alone, as the traffic counters took them)
    ctx.set_flags(w.FLAG_TIME_KERNELS | w.FLAG_SEPARATE_COMBINE)
    ctx.reset_stats()
    step()
    torch.cuda.synchronize()
    st_sep = ctx.stats()
    ctx.set_flags(0)

    # build time and the main loop, separately (one more untimed-kernel step)
    torch.cuda.synchronize()
    e_a = torch.cuda.Event(enable_timing=True)
    e_b = torch.cuda.Event(enable_timing=True)
    e_c = torch.cuda.Event(enable_timing=True)
    e_a.record(stream)
    cs = w.wnnc_normalize(ctx.handle, P, Pn)
    w.wnnc_build(ctx.handle, Pn, c, depth)
    e_b.record(stream)
    w.wnnc_orient(ctx.handle, mu, None, args.iters, w1, w2)
    w.wnnc_normals(ctx.handle, mu, cs[1], nrm)
    e_c.record(stream)
    torch.cuda.synchronize()
    t_pre = e_a.elapsed_time(e_b)
    t_main = e_b.elapsed_time(e_c)

    # dominant traversal kernel
    per_kind = {}
    for k in range(3):
        calls = st["calls"][k]
        if calls == 0:
            continue
        avg_ms = st["traverse_ms"][k] / calls
        pairs_per_launch = pairs[k] / max(calls_per_run[k], 1)
        flop = pairs_per_launch * FLOPS_PER_PAIR[k]
        per_kind[KIND[k]] = dict(total_ms=st["traverse_ms"][k] / args.steps, launches=calls // args.steps,
                                 avg_ms=avg_ms, pairs_per_launch=pairs_per_launch,
                                 tflops=flop / (avg_ms * 1e-3) / 1e12,
                                 gpairs_per_s=pairs_per_launch / (avg_ms * 1e-3) / 1e9)
    dom = max(per_kind, key=lambda k: per_kind[k]["total_ms"])
    d = per_kind[dom]
    # one wavefront (64 threads, one workgroup) per task
    grid = int(st["n_tasks"]) * 64
    # committed counter summaries of each kind's timed walk, per walk split
    # (used only when taken on the current traversal sources and this grid)
    split = ctx.split()
    for kind, dk in per_kind.items():
        sqk = load_profile(f"sq_traverse_{kind}_torusknot500k_split{split}", grid)
        trk = load_profile(f"traffic_traverse_{kind}_torusknot500k_split{split}", grid)
        if sqk and "SQ_INSTS_VALU" in sqk["per_dispatch"]:
            pdk = sqk["per_dispatch"]
            dk["counters"] = {
                "valu_insts_per_launch": pdk["SQ_INSTS_VALU"],
                "salu_insts_per_launch": pdk.get("SQ_INSTS_SALU"),
                # lane-instructions per counted pair (wave64 instructions x 64)
                "valu_lane_insts_per_pair": round(pdk["SQ_INSTS_VALU"] * 64 / dk["pairs_per_launch"], 2),
                "valu_issue_frac": round(pdk["SQ_INSTS_VALU"] / (dk["avg_ms"] * 1e-3)
                                         / sqk["valu_issue_peak_per_s"], 4),
                "VALUBusy": pdk.get("VALUBusy"), "VALUUtilization": pdk.get("VALUUtilization")}
        if trk:
            dk["hbm_bytes_per_launch"] = trk["bytes_per_launch"]
            dk["hbm_gb_per_s"] = round(trk["bytes_per_launch"] / (dk["avg_ms"] * 1e-3) / 1e9, 1)
    tr = load_profile(f"traffic_traverse_{dom}_torusknot500k_split{split}", grid)
    roofline = {"bound": "alu", "achieved": round(d["tflops"], 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(d["tflops"] / PEAK_FP32_TFLOPS, 4),
                # without packed FP32 (the library is compiled without it) the ceiling is half
                "frac_nonpacked": round(d["tflops"] / (PEAK_FP32_TFLOPS / 2), 4),
                "traffic": tr["bytes_per_launch"] if tr else None,
                "kernel": f"k_traverse<{dom}>",
                "grid_threads": grid,
                "avg_launch_ms": round(d["avg_ms"], 4),
                "flop_per_launch": round(d["pairs_per_launch"] * FLOPS_PER_PAIR[{"A": 0, "AT": 1, "G": 2}[dom]])}
    sq = load_profile(f"sq_traverse_{dom}_torusknot500k_split{split}", grid)
    if sq and "SQ_INSTS_VALU" in sq["per_dispatch"]:
        # the instruction-issue view: wave64 vector instructions per launch
        # (committed counters) over this run's launch time
        vi = sq["per_dispatch"]["SQ_INSTS_VALU"]
        roofline["valu_issue"] = {"insts_per_launch": vi,
                                  "frac": round(vi / (d["avg_ms"] * 1e-3) / sq["valu_issue_peak_per_s"], 4),
                                  "peak_per_s": sq["valu_issue_peak_per_s"]}
        for k in ("VALUBusy", "VALUUtilization"):
            if k in sq["per_dispatch"]:
                roofline["valu_issue"][k] = sq["per_dispatch"][k]

    # random initial vectors (the generator's unit vectors) scaled by the
    # mean area weight in the normalized frame
    sig = cloud.area * cs0[1] ** 2 / cloud.n
    mu0_rnd = (cloud.mu0.astype(np.float64) * sig).astype(np.float32)
    warm = None if args.core_only else warm_start_section(ctx, w, mu, stream, args.iters, w1, w2,
                                                          cloud.normals, mu0_rnd)

    from paper_2405_16634_amd.metrics import ae_pcd, p_co
    nrm_h = nrm.cpu().numpy()
    pco = p_co(nrm_h, cloud.normals)
    ae = ae_pcd(nrm_h, cloud.normals)
    far = leaf = batched = union = None
    if not args.core_only:
        union = union50k_section(w, stream, args.iters, c, depth, 5)
        far = far_field_section(ctx, w, step, mu, stream, max(1, min(args.steps, 3)),
                                cloud.normals)
        leaf = leaf_cap_section(w, P, stream, args.iters, w1, w2, c, depth,
                                max(1, min(args.steps, 3)), cloud.normals)
        batched = batched_section(w, stream, args.iters, w1, w2, c, depth)

    out = {
        "metric": METRIC,
        "value": round(total_pairs / (ms_step * 1e-3) / 1e9, 3),
        "unit": "Gpair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"torusknot{args.n // 1000}k", "n_points": args.n, "iters": args.iters,
                   "w1": w1, "w2": w2, "c": c, "max_depth": depth, "outlier_frac": 0.02,
                   "tube_radius": 0.05, "density_ratio": 10, "seed": 3},
        "time_40iter_s": round(ms_step / 1e3, 4),
        "t_pre_ms": round(t_pre, 3),
        "t_main_ms": round(t_main, 3),
        "pairs_per_step": total_pairs,
        "pairs_per_kind": {KIND[k]: int(pairs[k]) for k in range(3)},
        "operator_calls": {KIND[k]: int(calls_per_run[k]) for k in range(3)},
        "traversal": per_kind,
        "tile": {"targets_per_lane": ctx.tile(), "prefetch": ctx.prefetch(),
                 "split_visits": ctx.split(), "groups": int(st["n_groups"]),
                 "tasks_per_launch": int(st["n_tasks"]),
                 "prefetch_by_op": {KIND[k]: bool((st["prefetch_ops"] >> k) & 1) for k in range(3)}},
        "tile_autotune_ms": {f"tpl{k[0]}_pf{k[1]}_split{k[2]}": round(v, 4)
                             for k, v in tile_ms.items()},
        # (the moment passes that read a split walk's output also run its
        # combining pass; moments_separate times both as launches of their own)
        "moments_ms_per_step": round(st_all["moments_ms"], 3),
        "combine_ms_per_step": round(st_all["combine_ms"], 3),
        "moments_separate": {"moments_ms_per_step": round(st_sep["moments_ms"], 3),
                             "combine_ms_per_step": round(st_sep["combine_ms"], 3)},
        "moments_counters": moments_counters(st_sep, calls_per_run),
        "host_wall_s_per_step": round((t_host1 - t_host0) / args.steps, 4),
        "accuracy_vs_generator": {"P_co": round(pco, 5), "AE_pcd": round(ae, 6)},
        "context_paper_rtx3090_s": {"N=50k": 1.25, "N=500k": 31.63},
        "roofline": roofline,
        "warm_start": warm,
        "far_field_order2_wsafe": far,
        "tree_leaf_cap_8": leaf,
        "batched64": batched,
        "ellipsoids50k": union,
    }
    if rank == 0 and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cloud, w1, c)
        # the full plan is long: its last run on this kind of host, as committed
        plan = os.path.join(ROOT, "profiles", "cpu_oracle_plan.json")
        if os.path.exists(plan):
            out["cpu_baseline"]["plan_record"] = json.load(open(plan))
    ctx.close()
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
