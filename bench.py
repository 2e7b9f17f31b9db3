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
kernel of the band query, timed with HIP events on the context stream.
The cpu_baseline leg runs the same step with the FP64 oracle on the host
cores and checks every GPU output of the last step against it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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
PEAK_FP32_VECTOR = 157.3e12     # MI355X published FP32 vector peak, flop/s
PEAK_HBM = 8.0e12               # bytes/s
ORIGIN = (0.0, 0.0, 1.5)


def workload():
    from paper_2407_09649_amd import scenes as S
    scene = S.lidar_scene(1)
    pts = S.lidar_frame(scene, ORIGIN, np.random.default_rng(1))
    q = S.lidar_band_queries(pts)
    qg = S.jitter_points(pts, 4_000_000, 0.05, seed=2)
    return pts, q, qg


def algorithmic_flops(st):
    """Counted work of the FP32 evaluation pass: per (query, cluster) pair of
    n points, n^2 + 25 n + 40 flops (kernel values, occupancy, gradient sum,
    the triangular variance product and the reverting).  With
    tri = sum n (n + 1) / 2: sum n^2 = 2 tri - sum n."""
    return 2 * st["eval_tri"] + 24 * st["eval_points"] + 40 * st["eval_pairs"]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
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

    # dominant kernel: the FP32 evaluation of the band query
    flops = algorithmic_flops(st)
    eval_s = stages["eval"] / 1e3
    achieved = flops / eval_s
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
                "kernel": "k_query_cells<float, Matern-3/2>",
                "flops_per_launch": flops, "pairs": st["eval_pairs"],
                "kernel_evals": st["eval_points"], "variance_fmas": st["eval_tri"],
                "avg_launch_ms": stages["eval"]}
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
        "query_only_rate": m / ((stages["group"] + stages["eval"] + stages["refine"]) / 1e3),
        "refined_fraction": st["refined_queries"] / max(st["valid_queries"], 1),
        "roofline": roofline,
        "input_generation_s": gen_s,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"], res["parity"] = run_cpu_baseline(
            pts, q, qg, {k: v.cpu().numpy() for k, v in out.items()},
            {k: v.cpu().numpy() for k, v in glob.items()}, st["test_points"])
    ctx.close()
    print(json.dumps(res))


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
    parity = {"band_queries_compared": int(q.shape[0]),
              "validity_equal": bool((gv == v).all()),
              "max_dist_err_m": float(np.abs(g["dist"][v] - ref["dist"][v]).max()),
              "max_grad_err": float(np.abs(g["grad"][v] - ref["grad"][v]).max()),
              "max_var_rel_err": float(np.abs(g["var"][v] / ref["var"][v] - 1).max()),
              "sign_equal": bool((np.sign(g["dist"][v]) == np.sign(ref["dist"][v])).all()),
              "test_points_gpu": int(n_test), "test_points_oracle": int(ntp),
              "global_validity_equal": bool((gg["valid"].astype(bool) == vg).all()),
              "global_max_dist_err_m": float(np.abs(gg["dist"][vg] - rg["dist"][vg]).max()),
              "global_max_grad_err": float(np.abs(gg["grad"][vg] - rg["grad"][vg]).max())}
    cpu = {"value": q.shape[0] / dt.sum(), "unit": "queries/s", "cores": int(threads),
           "kind": "oracle",
           "sample": (f"the whole step, no sampling: training {dt[0]:.2f} s, fusion of "
                      f"{ntp} test voxels {dt[1]:.2f} s, {q.shape[0]} band queries "
                      f"{dt[2]:.2f} s, {qg.shape[0]} global queries {dt[3]:.2f} s"),
           "host_cpu": _cpu_model()}
    return cpu, parity


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
