"""GPU checks of the batching extension: every launch shape the autotuner
can pick gives bitwise the same results (each output element goes through
the same arithmetic, only its assignment to threads changes), the autotuner
returns a shape among its candidates, and the batched uneven-size workload
stays in parity with the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import compare, gpu_query, oracle_params, small_params

pytestmark = pytest.mark.gpu


def _patches(n_patches=160):
    ps = S.planar_patches(3, n_patches=n_patches, grid=(6, 6, 6), q_per=48)
    return ps.points, ps.queries


def _run(ctx, pts, q, dev):
    ctx.train(torch.from_numpy(pts).to(dev))
    r = gpu_query(ctx, q)
    model = ctx.export_model()
    return r, model


def test_launch_shapes_bitwise_identical(dev):
    pts, q = _patches()
    p = small_params(cluster_size=0.8, max_factor_elems=1 << 24)
    ref = None
    for tt in (256, 512, 1024):
        for ep in (0, 1, 2, 4):
            ctx = P.Context(p, device=dev)
            ctx.set_tuning(train_threads=tt, eval_persistent=ep)
            assert ctx.get_tuning() == {"train_threads": tt, "eval_persistent": ep, "mfma_min_n": 0}
            r, model = _run(ctx, pts, q, dev)
            st = ctx.stats()
            ctx.close()
            if ref is None:
                ref = (r, model, st)
                continue
            for k in r:
                assert np.array_equal(r[k], ref[0][k], equal_nan=True), (tt, ep, k)
            assert np.array_equal(model["alpha"], ref[1]["alpha"]), (tt, ep)
            assert st["refined_queries"] == ref[2]["refined_queries"]


def test_autotune_picks_a_candidate_and_keeps_parity(dev, tmp_path):
    P.tuning_cache_clear()
    pts, q = _patches(96)
    p = small_params(cluster_size=0.8, max_factor_elems=1 << 24)
    x, qd = torch.from_numpy(pts).to(dev), torch.from_numpy(q).to(dev)
    ctx = P.Context(p, device=dev)
    ms = ctx.autotune(x, qd)
    assert not ms.pop("cached")
    assert len(ms) == 11 and all(v > 0 for v in ms.values()), ms
    t = ctx.get_tuning()
    assert t["train_threads"] in (256, 512, 1024) and t["eval_persistent"] in (0, 1, 2, 4)
    assert t["mfma_min_n"] in (0, 17, 33, 65, 129)
    # the context is left trained on the tuning input
    g = gpu_query(ctx, q)
    o = O.Model(oracle_params(p), pts).query(q)
    compare(g, o, label="autotuned")
    # the same workload shape again: served from the cache, same shapes
    c2 = P.Context(p, device=dev)
    ms2 = c2.autotune(x, qd)
    assert ms2.pop("cached") and all(v == -1 for v in ms2.values())
    assert c2.get_tuning() == t
    # written, cleared, read back
    f = tmp_path / "tuning.txt"
    P.tuning_cache_save(f)
    P.tuning_cache_clear()
    P.tuning_cache_load(f)
    c3 = P.Context(p, device=dev)
    assert c3.autotune(x, qd)["cached"] and c3.get_tuning() == t
    for c in (ctx, c2, c3):
        c.close()
    P.tuning_cache_clear()


@pytest.mark.parametrize("min_n", [17, 33, 65])
def test_mfma_size_buckets_keep_parity(dev, min_n):
    # every MFMA bucket boundary the autotuner can pick keeps the FP32 path's
    # tolerances (the product's summation order changes, nothing else)
    pts, q = _patches(96)
    p = small_params(cluster_size=0.8, max_factor_elems=1 << 24)
    ctx = P.Context(p, device=dev)
    ctx.set_tuning(train_threads=1024, eval_persistent=0, mfma_min_n=min_n)
    ctx.train(torch.from_numpy(pts).to(dev))
    g = gpu_query(ctx, q)
    ctx.close()
    compare(g, O.Model(oracle_params(p), pts).query(q), label=f"mfma from {min_n}")


def test_rejects_unknown_shape(dev):
    ctx = P.Context(small_params(), device=dev)
    with pytest.raises(P.GpdfError):
        ctx.set_tuning(train_threads=300, eval_persistent=0)
    with pytest.raises(P.GpdfError):
        ctx.set_tuning(train_threads=256, eval_persistent=3)
    with pytest.raises(P.GpdfError):
        ctx.set_tuning(train_threads=256, eval_persistent=0, mfma_min_n=40)
