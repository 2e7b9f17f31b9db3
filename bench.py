#!/usr/bin/env python3
"""Benchmark of the L-GPDF hot path on one MI355X.

One step is one LiDAR frame through the whole path, on inputs already
resident in HBM:
  gpdf_fuse_frame      keys, voxel downsampling, 8^3-voxel leaves, FP64
                       training of every local GP, band test voxels of the
                       global grid, their signed L-GPDF query, fusion
  gpdf_query_distance  signed distance + gradient + variance at every 0.1 m
                       voxel within 1 m of the scan (~4.9M queries)
  gpdf_query_global    trilinear query of the fused grid at 4M points jittered
                       around the scan (N(0, 5 cm))

``value`` counts only the band queries (distance + gradient) per second of
the whole step; the fusion test points are extra work inside the step.
The roofline object describes the dominant kernel, the FP32 evaluation
kernel of the band query, timed with HIP events on the context stream;
roofline_test_voxels the other evaluation launch of the step (the fusion's
test voxels, no gradient).  frac_of_measured prices the same work at the
FMA and exp2 rates the probe kernels sustain on this device (measured_peaks:
HBM copy, FP32 VALU, exp2, BF16 / FP32 / FP64 MFMA).  query_only_shuffled
times the band query with its queries in a random order.  cpu_baseline also
reports one host thread.
The cpu_baseline leg runs the same step with the FP64 oracle on the host
cores and checks every GPU output of the last step against it.

The ``extensions`` object reports, on the same GPU:
  precision   the band query of the same frame with the variance product on
              BF16 MFMA, on FP32 MFMA, and in FP64, rate and errors against
              the oracle;
  batched     8,192 local GPs of 8-256 points on planar patches with 524,288
              queries: autotuned launch shapes, FP64 training, FP32, BF16 and
              FP32-MFMA queries, error against the oracle on a sample of the
              patches;
  sequence    100 frames of a moving sensor fused eagerly and through the
              per-frame HIP graph (bitwise compared), then 4M global queries;
              the first 5 frames fused again and compared with the oracle
              (grid, and global queries at observed voxels and uniform
              points), the G-GPDF on their zero crossings, and 20 frames with
              the paper's ray-cast test points beside the band (test voxels,
              time, the first frames against the oracle);
  correction  the learned correction trained on the GPU on pairs the method
              generates (GP output vs brute-force nearest point), its held-out
              gain, and its fused inference rate;
  properties  the frame with a surface property per return (Eq. (6)):
              training, the band query with the property, one fused frame,
              and 20,000 sampled queries against the oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extensions] [--legs precision,properties,batched,sequence,correction]
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

METRIC = "GP distance+gradient queries/sec at <=1e-4 m error vs FP64 oracle, 1 GPU"
PEAK_FP32_VECTOR = 157.3e12     # MI355X published FP32 vector peak (packed FMA), flop/s
PEAK_FP32_NONPACKED = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, the issuable peak here
PEAK_HBM = 8.0e12               # bytes/s
# VALU roofline of the evaluation: FMA work at the FMA rate plus the
# transcendentals (exp, sqrt, log, rcp) at quarter rate, per CU and clock
CUS, CLOCK = 256, 2.4e9
FMA_CLK_PACKED, FMA_CLK, TRANS_CLK = 128, 64, 16
ORIGIN = (0.0, 0.0, 1.5)


def workload():
    from paper_2407_09649_amd import scenes as S
    scene = S.lidar_scene(1)
    pts = S.lidar_frame(scene, ORIGIN, np.random.default_rng(1))
    q = S.lidar_band_queries(pts)
    qg = S.jitter_points(pts, 4_000_000, 0.05, seed=2)
    return pts, q, qg


def algorithmic_work(st, grad=True):
    """Counted work of the FP32 evaluation pass (Matern-3/2): per (query,
    cluster) pair of n points, n^2 + 25 n + 40 flops (kernel values,
    occupancy, gradient sum, the triangular variance product, reverting and
    combination) and 2 n + 4 transcendentals (sqrt and exp per point, the
    reverting).  With tri = sum n (n + 1) / 2: sum n^2 = 2 tri - sum n.
    Without a gradient the gradient sum (8 flops per point) is not counted."""
    per_point = 24 if grad else 16
    flops = 2 * st["eval_tri"] + per_point * st["eval_points"] + 40 * st["eval_pairs"]
    trans = 2 * st["eval_points"] + 4 * st["eval_pairs"]
    return flops, trans


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_lidar_frame_step.md")
EVAL_SOURCE = os.path.join(ROOT, "paper_2407_09649_amd", "csrc", "query.hip")


def profiled_traffic():
    """HBM bytes of one band evaluation launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the evaluation source has
    changed since the counters were taken (the summary records its sha256)."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(EVAL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("band-eval-traffic-bytes:"):
            f = line.split()
            if len(f) >= 4 and f[2] == "query.hip-sha256:" and f[3] == src:
                return int(f[1])
    return None


def valu_roofline_s(flops, trans, fma_clk):
    """Time of the work at 100 % VALU: FMAs (2 flops) at fma_clk per CU and
    clock, transcendentals at quarter rate."""
    return (flops / 2) / (fma_clk * CUS * CLOCK) + trans / (TRANS_CLK * CUS * CLOCK)


class Timer:
    """HIP events on a stream, median of repeated calls."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def median(self, fn, reps=5, warm=1):
        torch = self.torch
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(self.stream)
            fn()
            b.record(self.stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--legs", default="precision,properties,batched,sequence,correction",
                    help="extension legs to run (comma-separated subset)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_09649_amd as P

    dev = torch.device("cuda:0")
    t0 = time.time()
    pts, q, qg = workload()
    gen_s = time.time() - t0
    x = torch.from_numpy(pts).to(dev)
    qd = torch.from_numpy(q).to(dev)
    qgd = torch.from_numpy(qg).to(dev)
    m = q.shape[0]
    params = P.Params.default(voxel_size=0.1, timing=1)
    ctx = P.Context(params, device=dev)
    out = dict(dist=torch.empty(m, device=dev), grad=torch.empty((m, 3), device=dev),
               var=torch.empty(m, device=dev), valid=torch.empty(m, dtype=torch.uint8, device=dev),
               aux=torch.empty((m, 3), device=dev))

    glob = {}

    def step():
        ctx.fuse(x, ORIGIN)
        ctx.query(qd, origin=ORIGIN, out=out)
        glob.update(ctx.query_global(qgd))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stage_sum = {}
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
        st = ctx.stats()  # synchronises; reads this step's HIP-event stage times
        for k, v in st["ms"].items():
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    stages = {k: v / args.steps for k, v in stage_sum.items()}
    value = m / (ms_per_step / 1e3)

    # query-only rate: the whole gpdf_query_distance call, median of 20 runs,
    # on the queries in lattice order and in a random order
    timer = Timer(torch, ctx.stream)
    q_ms = timer.median(lambda: ctx.query(qd, origin=ORIGIN, out=out), reps=20)
    qs = torch.from_numpy(q[np.random.default_rng(11).permutation(m)]).to(dev)
    out_s = {k: torch.empty_like(v) for k, v in out.items()}
    q_ms_shuffled = timer.median(lambda: ctx.query(qs, origin=ORIGIN, out=out_s), reps=20)
    del qs, out_s

    # dominant kernel: the FP32 evaluation of the band query
    # frac = time of the counted work at 100 % VALU (published packed-FMA
    # rate) / measured time; achieved = frac x peak, in flop-equivalents
    # (a transcendental costs 16 flops of packed-FMA issue)
    flops, trans = algorithmic_work(st)
    eval_s = stages["eval"] / 1e3
    frac = valu_roofline_s(flops, trans, FMA_CLK_PACKED) / eval_s
    roofline = {"bound": "alu", "achieved": frac * PEAK_FP32_VECTOR / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": frac, "traffic": profiled_traffic(),
                "frac_issuable": valu_roofline_s(flops, trans, FMA_CLK) / eval_s,
                "flops_only_tflops": flops / eval_s / 1e12,
                "kernel": "k_query_cells<float, Matern-3/2>",
                "flops_per_launch": flops, "transcendentals_per_launch": trans,
                "pairs": st["eval_pairs"], "kernel_evals": st["eval_points"],
                "variance_fmas": st["eval_tri"], "avg_launch_ms": stages["eval"]}
    # the second evaluation launch of the step: the test voxels of the fusion
    # (their query asks for no gradient), measured on a fusion call alone
    ev_ms = []
    for _ in range(5):
        ctx.fuse(x, ORIGIN)
        st_tv = ctx.stats()
        ev_ms.append(st_tv["ms"]["eval"])
    f2, t2 = algorithmic_work(st_tv, grad=False)
    tv_s = float(np.median(ev_ms)) / 1e3
    frac2 = valu_roofline_s(f2, t2, FMA_CLK_PACKED) / tv_s
    roofline_tv = {"bound": "alu", "achieved": frac2 * PEAK_FP32_VECTOR / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                   "unit": "TFLOP/s", "frac": frac2, "frac_issuable": valu_roofline_s(f2, t2, FMA_CLK) / tv_s,
                   "flops_only_tflops": f2 / tv_s / 1e12, "kernel": "k_query_cells<float, Matern-3/2, no gradient>",
                   "flops_per_launch": f2, "transcendentals_per_launch": t2, "pairs": st_tv["eval_pairs"],
                   "queries": st_tv["queries"], "avg_launch_ms": tv_s * 1e3}
    # what this device sustains (probe kernels): the same work at the
    # measured FMA and exp2 rates
    peaks = ctx.measure_peaks()
    meas_fma = peaks["fp32_valu_tflops"] * 1e12 / 2
    meas_trans = peaks["exp2_gops"] * 1e9

    def frac_measured(fl, tr, sec):
        return ((fl / 2) / meas_fma + tr / meas_trans) / sec

    roofline["frac_of_measured"] = frac_measured(flops, trans, eval_s)
    roofline_tv["frac_of_measured"] = frac_measured(f2, t2, tv_s)
    res = {
        "metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one 64x1024 LiDAR frame (ground + 20 boxes, seed 1): "
                               "voxel 0.1 m, 8^3-voxel leaves, Matern-3/2 l=0.2 s=0.01, "
                               "27-cell smooth minimum, signed; fused at 0.05 m with a 0.2 m band",
                   "raw_points": int(pts.shape[0]), "training_points": st["points"],
                   "clusters": st["clusters"], "band_queries": m, "global_queries": int(qg.shape[0]),
                   "test_points": st["test_points"], "global_voxels": st["global_voxels"]},
        "stages_ms": stages,
        "query_only_ms": q_ms,
        "query_only_rate": m / (q_ms / 1e3),
        "query_only_shuffled_ms": q_ms_shuffled,
        "query_only_shuffled_rate": m / (q_ms_shuffled / 1e3),
        "refined_fraction": st["refined_queries"] / max(st["valid_queries"], 1),
        "refine_pairs": {"small_clusters": st["refine_pairs_small"], "large_clusters": st["refine_pairs_large"],
                         "large_cluster_items": st["refine_items_large"]},
        "fp64_share_of_band_query": stages["refine"] / max(stages["group"] + stages["eval"] + stages["refine"], 1e-9),
        "roofline": roofline,
        "roofline_test_voxels": roofline_tv,
        "measured_peaks": peaks,
        "input_generation_s": gen_s,
    }
    gpu_out = {k: v.cpu().numpy() for k, v in out.items()}
    others = {}
    ext = {}
    legs = set() if args.no_extensions else set(args.legs.split(","))
    if "precision" in legs:
        ext["precision"], others = precision_leg(P, torch, dev, x, qd, timer)
    if "properties" in legs:
        ext["properties"] = properties_leg(P, torch, dev, pts, q, x, qd, q_ms)
    if not args.no_cpu_baseline:
        res["cpu_baseline"], res["parity"], ref = run_cpu_baseline(
            pts, q, qg, gpu_out, {k: v.cpu().numpy() for k, v in glob.items()}, st["test_points"])
        for name, g in others.items():
            ext["precision"][name].update(dist_errors(g, ref))
    ctx.close()
    if "batched" in legs:
        ext["batched"] = batched_leg(P, torch, dev)
    if "sequence" in legs:
        ext["sequence"] = sequence_leg(P, torch, dev)
    if "correction" in legs:
        ext["correction"] = correction_leg(P, torch, dev)
    if legs:
        res["extensions"] = ext
    print(json.dumps(res))


def dist_errors(g, ref):
    """Errors against the oracle with the sign aligned at the oracle's sign
    near-ties (the only queries where a sign may differ; counted)."""
    v = ref["valid"]
    tie = ref.get("sign_tie", np.zeros(len(v), bool))[v]
    flip = np.sign(g["dist"][v]) != np.sign(ref["dist"][v])
    sg = np.where(flip, -1.0, 1.0)
    e = np.abs(sg * g["dist"][v].astype(np.float64) - ref["dist"][v])
    ge = np.abs(sg[:, None] * g["grad"][v].astype(np.float64) - ref["grad"][v]).max(axis=1)
    return {"validity_equal": bool((g["valid"].astype(bool) == v).all()),
            "sign_flips": int(flip.sum()), "sign_flips_outside_near_ties": int((flip & ~tie).sum()),
            "median_dist_err_m": float(np.median(e)), "p99_dist_err_m": float(np.quantile(e, 0.99)),
            "max_dist_err_m": float(e.max()), "max_grad_err": float(ge.max())}


def precision_leg(P, torch, dev, x, qd, timer):
    """The band query of the same frame with BF16 and FP32 MFMA products and in FP64."""
    m = qd.shape[0]
    rep, outs = {}, {}
    for name, prec in (("bf16", P.PREC_BF16), ("fp32_mfma", P.PREC_FP32_MFMA), ("fp64", P.PREC_FP64)):
        c = P.Context(P.Params.default(voxel_size=0.1, precision=prec), device=dev)
        c.train(x)
        o = dict(dist=torch.empty(m, device=dev), grad=torch.empty((m, 3), device=dev),
                 var=torch.empty(m, device=dev), valid=torch.empty(m, dtype=torch.uint8, device=dev))
        t = Timer(torch, c.stream).median(lambda: c.query(qd, origin=ORIGIN, aux=False, out=o), reps=10)
        rep[name] = {"query_ms": t, "query_rate": m / (t / 1e3)}
        outs[name] = {k: v.cpu().numpy() for k, v in o.items()}
        c.close()
    return rep, outs


def properties_leg(P, torch, dev, pts, q, x, qd, q_plain_ms, n_sample=20000):
    """The same frame with one surface property per return (a smooth
    intensity texture plus N(0, 0.01) noise, Eq. (6)): training with it, the
    band query with property and property variance, one fused frame with
    the property (Sec. IV-C), and a sample of the band queries against the
    FP64 oracle."""
    import oracle as O
    from paper_2407_09649_amd import scenes as S
    prop = S.surface_intensity(pts, 11)
    cp = torch.from_numpy(prop).to(dev)
    c = P.Context(P.Params.default(voxel_size=0.1, properties=1), device=dev)
    tm = Timer(torch, c.stream)
    rep = {"train_ms": tm.median(lambda: c.train_prop(x, cp), reps=5)}
    out = {}
    rep["query_ms"] = tm.median(lambda: out.update(c.query_prop(qd, origin=ORIGIN, aux=False)), reps=10)
    rep["query_rate"] = q.shape[0] / (rep["query_ms"] / 1e3)
    rep["query_ms_without_property"] = q_plain_ms
    rep["fuse_frame_ms"] = tm.median(lambda: c.fuse_prop(x, cp, ORIGIN), reps=5)
    st = c.stats()
    rep["refined_queries"] = st["refined_queries"]
    idx = np.random.default_rng(12).choice(q.shape[0], n_sample, replace=False)
    g = {k: v.cpu().numpy()[idx] for k, v in out.items()}
    c.close()
    t0 = time.perf_counter()
    ref = O.Model(O.Params(voxel=0.1), pts, prop=prop).query(q[idx], origin=np.asarray(ORIGIN, np.float32))
    rep["oracle_sample_s"] = time.perf_counter() - t0
    v = ref["valid"]
    rep.update(dist_errors(g, ref))
    rep["sample"] = n_sample
    rep["max_prop_err"] = float(np.abs(g["prop"][v] - ref["prop"][v]).max())
    rep["max_prop_var_rel_err"] = float(np.abs(g["prop_var"][v] / ref["prop_var"][v] - 1).max())
    return rep


def batched_leg(P, torch, dev):
    """8,192 local GPs of U{8..256} points on planar patches, 64 queries each:
    autotuned launch shapes, then FP32, BF16 and FP32-MFMA queries; the error against the
    oracle is taken on a sample of 256 patches (each query's 27 neighbour
    cells hold only its own patch, so a model of the sampled patches gives
    the oracle value of their queries)."""
    import oracle as O
    from paper_2407_09649_amd import scenes as S
    ps = S.planar_patches(3)
    x = torch.from_numpy(ps.points).to(dev)
    q = torch.from_numpy(ps.queries).to(dev)
    base = dict(cluster_size=0.8, max_points=1 << 21, max_factor_elems=(1 << 31) - 1, max_queries=1 << 20)
    rep = {"gps": int(len(ps.sizes)), "points": int(ps.points.shape[0]), "queries": int(ps.queries.shape[0]),
           "fp64_train_flop": float((ps.sizes.astype(np.float64) ** 3 / 3 + 2 * ps.sizes ** 2).sum())}
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(len(ps.sizes), 256, replace=False))
    starts = np.concatenate([[0], np.cumsum(ps.sizes)])
    sp = np.concatenate([ps.points[starts[i]:starts[i + 1]] for i in sample])
    qi = np.concatenate([np.arange(64 * i, 64 * i + 64) for i in sample])
    ref = O.Model(O.Params(cell=0.8), sp).query(ps.queries[qi])
    for name, prec in (("fp32", P.PREC_FP32), ("bf16", P.PREC_BF16), ("fp32_mfma", P.PREC_FP32_MFMA)):
        c = P.Context(P.Params.default(precision=prec, timing=1, **base), device=dev)
        tune = c.autotune(x, q)
        t = Timer(torch, c.stream)
        train_ms = t.median(lambda: c.train(x), reps=3)
        r = {}
        q_ms = t.median(lambda: r.update(c.query(q)), reps=5)
        g = {k: v.cpu().numpy()[qi] for k, v in r.items()}
        st = c.stats()
        rep[name] = {"tuning": c.get_tuning(), "autotune_ms": tune, "train_ms": train_ms,
                     "query_ms": q_ms, "query_rate": ps.queries.shape[0] / (q_ms / 1e3),
                     "refined_queries": st["refined_queries"], **dist_errors(g, ref)}
        c.close()
    return rep


def sequence_leg(P, torch, dev, n_frames=100):
    """100 frames of the LiDAR scene from a sensor moving 0.5 m per frame,
    fused eagerly and through the per-frame HIP graph; then 4M global queries
    at observed voxels jittered within the voxel."""
    from paper_2407_09649_amd import scenes as S
    t0 = time.time()
    path = S.sensor_path(4, n_frames=n_frames)
    scene = S.lidar_scene(4, keep_clear_xy=path[:, :2], clearance=1.5)
    rng = np.random.default_rng(4)
    frames = [torch.from_numpy(S.lidar_frame(scene, o, rng)).to(dev) for o in path]
    gen = time.time() - t0
    prm = dict(voxel_size=0.1, max_points=1 << 16, max_queries=3_600_000, global_capacity=1 << 26)
    rep = {"frames": n_frames, "input_generation_s": gen, "max_points": prm["max_points"]}
    grids = {}
    for mode in ("eager", "graph"):
        c = P.Context(P.Params.default(**prm), device=dev)
        if mode == "graph":
            c.fuse_graph(frames[0], path[0].astype(np.float32))  # capture + frame 0
        else:
            c.fuse(frames[0], path[0].astype(np.float32))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(1, n_frames):
            o = path[i].astype(np.float32)
            (c.fuse_graph if mode == "graph" else c.fuse)(frames[i], o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = c.stats()
        rep[mode] = {"ms_per_frame": 1e3 * dt / (n_frames - 1), "global_voxels": st["global_voxels"],
                     "status_bits": st["status_bits"]}
        grids[mode] = c.export_global()
        if mode == "graph":
            keys = grids[mode]["key"]
            r = np.random.default_rng(5)
            kk = keys[r.integers(0, len(keys), 4_000_000)]
            cc = np.stack([(kk >> np.uint64(42)) & np.uint64(0x1FFFFF), (kk >> np.uint64(21)) & np.uint64(0x1FFFFF),
                           kk & np.uint64(0x1FFFFF)], 1).astype(np.int64) - (1 << 20)
            qg = torch.from_numpy(((cc + 0.5 + r.uniform(-0.5, 0.5, size=cc.shape)) * 0.05).astype(np.float32)).to(dev)
            out = {}
            tq = Timer(torch, c.stream).median(lambda: out.update(c.query_global(qg)), reps=10)
            rep["global_query"] = {"queries": 4_000_000, "ms": tq, "rate": 4e6 / (tq / 1e3),
                                   "valid_fraction": float(out["valid"].float().mean())}
        c.close()
    rep["graph_equals_eager"] = all(np.array_equal(grids["eager"][k], grids["graph"][k])
                                    for k in ("key", "D", "V", "stamp"))
    rep["oracle_check"] = sequence_oracle_check(P, torch, dev, frames, path, prm)
    rep["raycast"] = raycast_check(P, torch, dev, frames, path, prm)
    return rep


def raycast_check(P, torch, dev, frames, path, prm, n_frames=20, k_oracle=2):
    """The paper's test points (Sec. IV-B: rays against the grid, measured
    voxels, normals) on the first frames of the sequence, beside the band:
    test voxels and time per frame, and the first frames' test-voxel sets
    and grid against the oracle."""
    import oracle as O
    rep = {"frames": n_frames}
    for mode, tp in (("band", P.TEST_BAND), ("raycast", P.TEST_RAYCAST)):
        c = P.Context(P.Params.default(timing=1, test_points=tp, **prm), device=dev)
        c.fuse(frames[0], path[0].astype(np.float32))
        torch.cuda.synchronize()
        tests, tp_ms = 0, 0.0
        t = time.perf_counter()
        for i in range(1, n_frames):
            c.fuse(frames[i], path[i].astype(np.float32))
            st = c.stats()
            tests += st["test_points"]
            tp_ms += st["ms"]["testpts"]
        dt = time.perf_counter() - t
        rep[mode] = {"ms_per_frame": 1e3 * dt / (n_frames - 1), "test_voxels_per_frame": tests / (n_frames - 1),
                     "test_voxel_generation_ms": tp_ms / (n_frames - 1), "global_voxels": c.stats()["global_voxels"]}
        c.close()
    # the first frames against the oracle (host cores)
    c = P.Context(P.Params.default(test_points=P.TEST_RAYCAST, **prm), device=dev)
    omap = O.Map()
    op = O.Params(voxel=0.1, tp_mode=1, normal_reach=0.2)
    same = True
    t0 = time.perf_counter()
    for i in range(k_oracle):
        o = path[i].astype(np.float32)
        om = O.Model(op, frames[i].cpu().numpy())
        expect = om.test_points_ray(omap, o)
        c.fuse(frames[i], o)
        same = same and bool(np.array_equal(c.export_test_points(), expect))
        omap.fuse(om, o, i)
    g, r = c.export_global(), omap.export()
    t = r["sign_tie"]
    rep["oracle"] = {"frames": k_oracle, "test_voxel_sets_equal": same, "oracle_s": time.perf_counter() - t0,
                     "keys_and_stamps_equal": bool(np.array_equal(g["key"], r["key"]) and
                                                   np.array_equal(g["stamp"], r["stamp"]))}
    if rep["oracle"]["keys_and_stamps_equal"]:
        rep["oracle"]["max_D_err_m"] = float(np.abs(g["D"][~t] - r["D"][~t]).max())
        rep["oracle"]["max_V_rel_err"] = float(np.abs(g["V"] / r["V"] - 1).max())
    c.close()
    return rep


def sequence_oracle_check(P, torch, dev, frames, path, prm, k_frames=5):
    """The first frames of the sequence fused by the GPU and by the FP64
    oracle on the host cores: the grids after the last of them, and global
    queries at observed voxels and at uniform points of the scene volume."""
    import oracle as O
    c = P.Context(P.Params.default(**prm), device=dev)
    op = O.Params(voxel=0.1)
    omap = O.Map()
    t0 = time.perf_counter()
    for i in range(k_frames):
        o = path[i].astype(np.float32)
        c.fuse(frames[i], o)
        omap.fuse(O.Model(op, frames[i].cpu().numpy()), o, i)
    torch.cuda.synchronize()
    oracle_s = time.perf_counter() - t0
    g, r = c.export_global(), omap.export()
    t = r["sign_tie"]
    same = bool(np.array_equal(g["key"], r["key"]) and np.array_equal(g["stamp"], r["stamp"]))
    out = {"frames": k_frames, "voxels": int(len(r["key"])), "keys_and_stamps_equal": same,
           "near_tie_voxels": int(t.sum()), "oracle_s": oracle_s}
    if same:
        out["max_D_err_m"] = float(np.abs(g["D"][~t] - r["D"][~t]).max())
        out["max_V_rel_err"] = float(np.abs(g["V"] / r["V"] - 1).max())
    rng = np.random.default_rng(6)
    kk = r["key"][rng.integers(0, len(r["key"]), 200_000)]
    cc = np.stack([(kk >> np.uint64(42)) & np.uint64(0x1FFFFF), (kk >> np.uint64(21)) & np.uint64(0x1FFFFF),
                   kk & np.uint64(0x1FFFFF)], 1).astype(np.int64) - (1 << 20)
    qo = ((cc + 0.5 + rng.uniform(-0.5, 0.5, size=cc.shape)) * 0.05).astype(np.float32)
    qu = rng.uniform([-20, -20, -1], [20, 20, 5], size=(200_000, 3)).astype(np.float32)
    for name, qq in (("observed", qo), ("uniform", qu)):
        gq = {k: v.cpu().numpy() for k, v in c.query_global(torch.from_numpy(qq).to(dev)).items()}
        rq = omap.query(0.05, qq)
        v = rq["valid"]
        ok = v & ~rq["sign_tie"]
        out[name] = {"queries": int(len(qq)), "valid_fraction": float(v.mean()),
                     "validity_equal": bool((gq["valid"].astype(bool) == v).all()),
                     "max_dist_err_m": float(np.abs(gq["dist"][ok] - rq["dist"][ok]).max()) if ok.any() else 0.0,
                     "max_grad_err": float(np.abs(gq["grad"][ok] - rq["grad"][ok]).max()) if ok.any() else 0.0}
    out["ggpdf"] = ggpdf_check(P, torch, dev, c, omap, qo)
    c.close()
    return out


def ggpdf_check(P, torch, dev, c, omap, qo, n_sample=2000):
    """The global GP distance field (G-GPDF, Sec. IV-D) of the fused grid: its
    zero crossings, one lazily trained GP per leaf of the grid (0.4 m), the
    Q = 8 nearest leaves per query combined by the smooth minimum; timed on
    the GPU for the observed-voxel queries, and checked against the FP64
    oracle (crossings of the same grid, every leaf trained) on a sample."""
    import oracle as O
    rep = {}
    timer = Timer(torch, c.stream)
    zc = {}
    rep["zero_crossings_ms"] = timer.median(lambda: zc.update(p=c.zero_crossings()), reps=3)
    pts = zc["p"]
    rep["zero_crossings"] = int(pts.shape[0])
    prm = dict(cluster_size=0.4, selection=P.SEL_KNN, knn_q=8, max_cluster_points=1024,
               max_points=max(1 << 20, int(pts.shape[0]) + 1), max_clusters=1 << 20,
               max_factor_elems=1 << 29, max_queries=len(qo), lazy_train=1, timing=1)
    g = P.Context(P.Params.default(**prm), device=dev)
    qd = torch.from_numpy(qo).to(dev)
    t0 = time.perf_counter()
    g.train(pts)
    r = g.query(qd)               # trains the leaves these queries select
    torch.cuda.synchronize()
    rep["first_query_with_lazy_training_ms"] = 1e3 * (time.perf_counter() - t0)
    st = g.stats()
    rep["leaves"], rep["trained_leaves"] = st["clusters"], st["trained_clusters"]
    out = {}
    q_ms = Timer(torch, g.stream).median(lambda: out.update(g.query(qd)), reps=5)
    rep["queries"] = int(len(qo))
    rep["query_ms"] = q_ms
    rep["query_rate"] = len(qo) / (q_ms / 1e3)
    # oracle: the crossings of the oracle's own fused grid (FP64 fusion), so
    # the comparison also covers the fusion; every leaf trained
    op = O.Params(cell=0.4, selection=1, knn_q=8)
    zo = omap.zero_crossings(0.05)
    rep["oracle_zero_crossings"] = int(len(zo))
    # the GPU field on the oracle's crossings, against the oracle field
    g2 = P.Context(P.Params.default(**{**prm, "max_points": max(1 << 20, len(zo) + 1)}), device=dev)
    g2.train(torch.from_numpy(zo).to(dev))
    idx = np.random.default_rng(8).choice(len(qo), n_sample, replace=False)
    gs = {k: v.cpu().numpy() for k, v in g2.query(torch.from_numpy(qo[idx]).to(dev)).items()}
    t1 = time.perf_counter()
    ref = O.Model(op, zo).query(qo[idx])
    rep["oracle_sample_s"] = time.perf_counter() - t1
    v = ref["valid"]
    rep["sample"] = n_sample
    rep["validity_equal"] = bool((gs["valid"].astype(bool) == v).all())
    rep["max_dist_err_m"] = float(np.abs(gs["dist"][v] - ref["dist"][v]).max())
    rep["max_grad_err"] = float(np.abs(gs["grad"][v] - ref["grad"][v]).max())
    g.close()
    g2.close()
    return rep


def correction_leg(P, torch, dev, n_train_scenes=40, n_eval_scenes=32, per_scene=250_000):
    """The learned correction: pairs (GP output, brute-force nearest training
    point) from sphere scenes with new seeds, KNN Q = 8, queries 0.1-3 m
    outside the sphere; trained on the GPU (BF16 MFMA, FP32 master weights)
    and evaluated on held-out scenes, gated and ungated."""
    from paper_2407_09649_amd import scenes as S
    c = P.Context(P.Params.default(selection=P.SEL_KNN, knn_q=8, cluster_size=0.4, max_queries=1 << 20),
                  device=dev)

    def pairs(seed0, n):
        fs, ts, ds, trs, vs = [], [], [], [], []
        for i in range(n):
            sc = S.sphere_scene(seed0 + i, n_queries=0)
            p = torch.from_numpy(sc.points).to(dev)
            qq = torch.from_numpy(S.sphere_eval_queries(seed0 + 50_000 + i, per_scene)).to(dev)
            c.train(p)
            r = c.query(qq)
            f = c.mlp_features(r)
            tr = c.nearest_distance(p, qq)
            ok = r["valid"].bool() & torch.isfinite(f).all(1)
            fs.append(f[ok]); ts.append((tr - r["dist"])[ok]); ds.append(r["dist"][ok])
            trs.append(tr[ok]); vs.append(r["var"][ok])
        return torch.cat(fs), torch.cat(ts), torch.cat(ds), torch.cat(trs), torch.cat(vs)

    t0 = time.time()
    f, t, _, _, _ = pairs(10_000, n_train_scenes)
    torch.cuda.synchronize()
    gen = time.time() - t0
    c.mlp_init(seed=0)
    epochs, batch = 2, 4096
    t1 = time.perf_counter()
    loss = c.mlp_train(f, t, epochs=epochs, batch=batch, lr=2e-3, seed=1)
    train_s = time.perf_counter() - t1
    fe, te, de, tre, ve = pairs(20_000, n_eval_scenes)
    r = {}
    tm = Timer(torch, c.stream).median(lambda: r.update(rr=c.mlp_forward(fe)), reps=5)
    rr = r["rr"]
    gate = c.params.mlp_gate
    g = ve <= gate

    def err(mask):
        e0 = (de - tre)[mask].double()
        e1 = (de + rr - tre)[mask].double()
        return {"n": int(mask.sum()), "mse_plain": float((e0 ** 2).mean()), "mse_corrected": float((e1 ** 2).mean()),
                "mae_plain": float(e0.abs().mean()), "mae_corrected": float(e1.abs().mean())}

    rep = {"train_pairs": int(f.shape[0]), "pair_generation_s": gen, "epochs": epochs, "batch": batch,
           "train_s": train_s, "train_samples_per_s": epochs * f.shape[0] / train_s, "final_loss": loss,
           "eval_queries": int(fe.shape[0]), "forward_ms": tm, "forward_rate": fe.shape[0] / (tm / 1e3),
           "gate": gate, "gated_fraction": float(g.float().mean()),
           "gated": err(g), "ungated": err(torch.ones_like(g))}
    c.close()
    return rep


def run_cpu_baseline(pts, q, qg, g, gg, n_test):
    """The same step with the FP64 oracle on the host cores (OpenMP over
    clusters and queries): training, fusion of the band test voxels, all band
    queries and the global query.  Every GPU output of the last step is
    compared with the oracle's on the way (the GPU grid has fused the frame
    once per step; repeated fusion of one observation leaves D unchanged)."""
    import oracle as O
    prm = O.Params(voxel=0.1)
    o = np.asarray(ORIGIN, np.float32)
    threads = O.max_threads()
    t = [time.perf_counter()]
    model = O.Model(prm, pts)
    t.append(time.perf_counter())
    gmap = O.Map()
    ntp, _ = gmap.fuse(model, o, 0)
    t.append(time.perf_counter())
    ref = model.query(q, origin=o)
    t.append(time.perf_counter())
    rg = gmap.query(0.05, qg)
    t.append(time.perf_counter())
    dt = np.diff(t)
    v = ref["valid"]
    gv = g["valid"].astype(bool)
    vg = rg["valid"]
    # the sign may differ only at the oracle's sign near-ties (nearest training
    # points on different sides within FP32 rounding); magnitudes and
    # gradients are compared with the sign aligned
    tie = ref["sign_tie"][v]
    flip = np.sign(g["dist"][v]) != np.sign(ref["dist"][v])
    sg = np.where(flip, -1.0, 1.0)
    gt = vg & ~rg["sign_tie"]
    parity = {"band_queries_compared": int(q.shape[0]),
              "validity_equal": bool((gv == v).all()),
              "max_dist_err_m": float(np.abs(sg * g["dist"][v] - ref["dist"][v]).max()),
              "max_grad_err": float(np.abs(sg[:, None] * g["grad"][v] - ref["grad"][v]).max()),
              "max_var_rel_err": float(np.abs(g["var"][v] / ref["var"][v] - 1).max()),
              "sign_near_ties": int(tie.sum()), "sign_flips": int(flip.sum()),
              "sign_flips_outside_near_ties": int((flip & ~tie).sum()),
              "test_points_gpu": int(n_test), "test_points_oracle": int(ntp),
              "global_validity_equal": bool((gg["valid"].astype(bool) == vg).all()),
              "global_queries_touching_a_near_tie_voxel": int((vg & rg["sign_tie"]).sum()),
              "global_max_dist_err_m": float(np.abs(gg["dist"][gt] - rg["dist"][gt]).max()),
              "global_max_grad_err": float(np.abs(gg["grad"][gt] - rg["grad"][gt]).max())}
    # one host thread: training and a fixed sample of the band queries,
    # median of three runs after a warm-up
    sub = q[np.random.default_rng(12).choice(q.shape[0], 100_000, replace=False)]
    one = []
    for r in range(4):
        t1 = time.perf_counter()
        m1 = O.Model(prm, pts, nthreads=1)
        m1.query(sub, origin=o, nthreads=1)
        if r:
            one.append(time.perf_counter() - t1)
    O.Model(prm, pts[:1], nthreads=threads)   # restore the thread count
    cpu = {"value": q.shape[0] / dt.sum(), "unit": "queries/s", "cores": int(threads),
           "kind": "oracle",
           "sample": (f"the whole step, no sampling: training {dt[0]:.2f} s, fusion of "
                      f"{ntp} test voxels {dt[1]:.2f} s, {q.shape[0]} band queries "
                      f"{dt[2]:.2f} s, {qg.shape[0]} global queries {dt[3]:.2f} s"),
           "one_thread": {"value": sub.shape[0] / float(np.median(one)), "unit": "queries/s", "cores": 1,
                          "sample": "training + 100,000 band queries, median of 3 after a warm-up"},
           "host_cpu": _cpu_model()}
    return cpu, parity, ref


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
