"""GPU checks of the per-frame graph (batching extension): a sequence of
frames fused through gpdf_fuse_frame_graph gives bitwise the same global grid
as gpdf_fuse_frame after every frame, with eager library work between the
replays; the graph reports capacity overflows in the status bits."""
import numpy as np
import pytest
import torch

import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import small_params

pytestmark = pytest.mark.gpu


def _frames(seed, n, beams=16, az=256):
    path = S.sensor_path(seed, n_frames=n)
    scene = S.lidar_scene(seed, keep_clear_xy=path[:, :2], clearance=1.5)
    rng = np.random.default_rng(seed)
    return path, [S.lidar_frame(scene, o, rng, n_beams=beams, n_azimuth=az) for o in path]


def _params(**kw):
    base = dict(voxel_size=0.1, max_points=8192, max_queries=1 << 21, global_capacity=1 << 22)
    base.update(kw)
    return small_params(**base)


def test_graph_replays_equal_eager_frames(dev):
    path, frames = _frames(5, 5)
    p = _params()
    eager = P.Context(p, device=dev)
    graph = P.Context(p, device=dev)
    probe = torch.from_numpy(S.lidar_band_queries(frames[0], radius_cells=2)[:5000]).to(dev)
    for i, (pts, o) in enumerate(zip(frames, path)):
        x = torch.from_numpy(pts).to(dev)
        o32 = np.asarray(o, np.float32)
        eager.fuse(x, o32)
        graph.fuse_graph(x, o32)
        # eager work on the graph's context and stream between replays
        graph.query_global(probe)
        torch.cuda.synchronize()
        a, b = eager.export_global(), graph.export_global()
        for k in ("key", "D", "V", "stamp"):
            assert np.array_equal(a[k], b[k]), (i, k)
        sa, sb = eager.stats(), graph.stats()
        assert sa["test_points"] == sb["test_points"] and sa["clusters"] == sb["clusters"], (i, sa, sb)
        assert sb["status_bits"] & P.STATUS_CAPACITY == 0
    ra = eager.query_global(probe)
    rb = graph.query_global(probe)
    for k in ra:
        assert torch.equal(ra[k], rb[k]), k
    eager.close()
    graph.close()


def test_graph_replays_with_growing_frames_equal_eager(dev):
    # the graph's evaluation runs one workgroup per chunk over a grid sized
    # from the previous replay's chunk count, the rest persistent: a frame
    # with a quarter of the points, then full frames (about four times the
    # chunks), puts most of a replay's chunks beyond that grid; a last
    # quarter frame runs on a grid over twice its count, which is then reset
    path, frames = _frames(7, 5)
    frames[0] = frames[0][::4].copy()
    frames[4] = frames[4][::4].copy()
    p = _params()
    eager = P.Context(p, device=dev)
    graph = P.Context(p, device=dev)
    tp = []
    for i, (pts, o) in enumerate(zip(frames, path)):
        x = torch.from_numpy(pts).to(dev)
        o32 = np.asarray(o, np.float32)
        eager.fuse(x, o32)
        graph.fuse_graph(x, o32)
        torch.cuda.synchronize()
        a, b = eager.export_global(), graph.export_global()
        for k in ("key", "D", "V", "stamp"):
            assert np.array_equal(a[k], b[k]), (i, k)
        sa, sb = eager.stats(), graph.stats()
        assert sa["test_points"] == sb["test_points"], (i, sa["test_points"], sb["test_points"])
        tp.append(sb["test_points"])
    print("test voxels per frame", tp, flush=True)
    assert tp[1] > 2 * tp[0] and tp[3] > 2 * tp[4]
    eager.close()
    graph.close()


@pytest.mark.parametrize("kw", [dict(precision=P.PREC_FP64), dict(kernel=P.KERNEL_SE, length_scale=0.15)],
                         ids=["fp64", "se-kernel"])
def test_graph_other_precision_and_kernel_equal_eager(dev, kw):
    # the FP64 evaluation takes the persistent instance in a captured frame;
    # the squared-exponential kernel has its own recording instance
    path, frames = _frames(8, 3)
    p = _params(**kw)
    eager = P.Context(p, device=dev)
    graph = P.Context(p, device=dev)
    for i, (pts, o) in enumerate(zip(frames, path)):
        x = torch.from_numpy(pts).to(dev)
        o32 = np.asarray(o, np.float32)
        eager.fuse(x, o32)
        graph.fuse_graph(x, o32)
        torch.cuda.synchronize()
        a, b = eager.export_global(), graph.export_global()
        for k in ("key", "D", "V", "stamp"):
            assert np.array_equal(a[k], b[k]), (i, k)
    eager.close()
    graph.close()


def test_graph_reports_capacity_overflow(dev):
    path, frames = _frames(6, 2)
    ctx = P.Context(_params(max_clusters=32), device=dev)
    for pts, o in zip(frames, path):
        ctx.fuse_graph(torch.from_numpy(pts).to(dev), np.asarray(o, np.float32))
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["status_bits"] & P.STATUS_CAPACITY
    assert st["clusters"] == 32
    ctx.close()


def test_graph_rejects_knn(dev):
    ctx = P.Context(_params(selection=P.SEL_KNN, knn_q=8), device=dev)
    with pytest.raises(P.GpdfError):
        ctx.fuse_graph(torch.zeros((10, 3), device=dev), np.zeros(3, np.float32))
    ctx.close()
