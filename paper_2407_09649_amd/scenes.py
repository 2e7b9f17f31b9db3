"""Seeded synthetic scenes standing in for the paper's datasets.

The paper evaluates on Cow and Lady, Newer College, Mai City and KITTI
(Sec. V, opening paragraph); none of them is available here, so every input is
generated from a seed with the shapes and structure of those workloads: a
noisy sampled sphere (RGB-D-like object scale), a spinning 64-beam LiDAR scan
of a ground plane with boxes (the LiDAR datasets), a sequence of such scans
along a smooth path (online fusion), and planar patches of uneven size
(batched local GPs).

This module holds no part of the method: no keys, hashing, kernels, GP
algebra, reverting or fusion.  It draws random numbers, ray-casts an analytic
scene and enumerates lattice points near the hits.  Every array it returns is
rounded once from FP64 to FP32, and both the HIP library and the CPU oracle
read the same arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "SphereScene", "sphere_scene", "lidar_scene", "LidarScene", "lidar_frame",
    "lidar_band_queries", "planar_patches", "PatchScene", "sensor_path",
    "sphere_eval_queries", "shuffle_rows", "jitter_points", "surface_intensity",
]


# --------------------------------------------------------------------------
# Noisy sphere: a small object scanned densely (RGB-D scale).
# --------------------------------------------------------------------------
@dataclasses.dataclass
class SphereScene:
    points: np.ndarray   # float32 [n, 3] surface samples
    queries: np.ndarray  # float32 [m, 3]
    radius: float


def sphere_scene(seed: int = 0, n_points: int = 2048, n_queries: int = 10000,
                 radius: float = 1.0, radial_sigma: float = 0.005,
                 box: float = 2.0) -> SphereScene:
    """Surface points uniform on a sphere with Gaussian radial noise, and
    queries uniform in the cube [-box, box]^3."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_points, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius + rng.normal(0.0, radial_sigma, size=n_points)
    pts = (d * r[:, None]).astype(np.float32)
    q = rng.uniform(-box, box, size=(n_queries, 3)).astype(np.float32)
    return SphereScene(points=pts, queries=q, radius=radius)


def sphere_eval_queries(seed: int, n: int, radius: float = 1.0,
                        dmin: float = 0.1, dmax: float = 3.0) -> np.ndarray:
    """Points outside the sphere at a uniform offset in [dmin, dmax] along a
    uniform direction: x = u * (radius + delta)."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    delta = rng.uniform(dmin, dmax, size=n)
    return (u * (radius + delta)[:, None]).astype(np.float32)


# --------------------------------------------------------------------------
# Spinning LiDAR over a ground plane with axis-aligned boxes.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class LidarScene:
    boxes_lo: np.ndarray  # float64 [B, 3]
    boxes_hi: np.ndarray  # float64 [B, 3]


def _footprint_distance(lo, hi, xy):
    """Distance in the xy plane from point xy to the rectangle [lo, hi]."""
    dx = np.maximum(np.maximum(lo[0] - xy[..., 0], 0.0), xy[..., 0] - hi[0])
    dy = np.maximum(np.maximum(lo[1] - xy[..., 1], 0.0), xy[..., 1] - hi[1])
    return np.hypot(dx, dy)


def lidar_scene(seed: int = 1, n_boxes: int = 20, half_extent: float = 20.0,
                side_lo: float = 0.5, side_hi: float = 4.0,
                keep_clear_xy: np.ndarray | None = None,
                clearance: float = 3.0) -> LidarScene:
    """Ground z = 0 plus boxes resting on it, sides U(side_lo, side_hi)^3 and
    footprint centres U(-half_extent, half_extent)^2.  A box whose footprint
    comes within ``clearance`` of any point of ``keep_clear_xy`` is redrawn."""
    rng = np.random.default_rng(seed)
    if keep_clear_xy is None:
        keep_clear_xy = np.zeros((1, 2))
    keep = np.asarray(keep_clear_xy, dtype=np.float64).reshape(-1, 2)
    lo, hi = [], []
    while len(lo) < n_boxes:
        side = rng.uniform(side_lo, side_hi, size=3)
        c = rng.uniform(-half_extent, half_extent, size=2)
        blo = np.array([c[0] - side[0] / 2, c[1] - side[1] / 2, 0.0])
        bhi = np.array([c[0] + side[0] / 2, c[1] + side[1] / 2, side[2]])
        if np.min(_footprint_distance(blo, bhi, keep)) < clearance:
            continue
        lo.append(blo)
        hi.append(bhi)
    return LidarScene(boxes_lo=np.array(lo), boxes_hi=np.array(hi))


def _beam_directions(n_beams: int, n_azimuth: int, elev_lo_deg: float,
                     elev_hi_deg: float) -> np.ndarray:
    el = np.deg2rad(np.linspace(elev_lo_deg, elev_hi_deg, n_beams))
    az = 2.0 * np.pi * np.arange(n_azimuth) / n_azimuth
    el, az = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az),
                  np.sin(el)], axis=-1)
    return d.reshape(-1, 3)


def lidar_frame(scene: LidarScene, origin, rng: np.random.Generator,
                n_beams: int = 64, n_azimuth: int = 1024,
                elev_lo_deg: float = -24.9, elev_hi_deg: float = 2.0,
                max_range: float = 50.0, range_sigma: float = 0.02
                ) -> np.ndarray:
    """One spinning scan from ``origin``: ray-cast against the ground and the
    boxes, keep the nearest hit within ``max_range`` and perturb its range by
    N(0, range_sigma).  Returns float32 [n_hits, 3] world-frame points."""
    o = np.asarray(origin, dtype=np.float64)
    d = _beam_directions(n_beams, n_azimuth, elev_lo_deg, elev_hi_deg)
    t_best = np.full(d.shape[0], np.inf)
    # ground plane z = 0
    down = d[:, 2] < 0
    t_best[down] = -o[2] / d[down, 2]
    # boxes: slab test
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        for blo, bhi in zip(scene.boxes_lo, scene.boxes_hi):
            t1 = (blo[None, :] - o[None, :]) * inv
            t2 = (bhi[None, :] - o[None, :]) * inv
            tn = np.nanmax(np.minimum(t1, t2), axis=1)
            tf = np.nanmin(np.maximum(t1, t2), axis=1)
            hit = (tn <= tf) & (tn > 0)
            t_best = np.where(hit & (tn < t_best), tn, t_best)
    keep = t_best <= max_range
    rng_noise = rng.normal(0.0, range_sigma, size=int(keep.sum()))
    t = t_best[keep] + rng_noise
    pts = o[None, :] + t[:, None] * d[keep]
    return pts.astype(np.float32)


def lidar_band_queries(points: np.ndarray, lattice: float = 0.1,
                       radius_cells: int = 10) -> np.ndarray:
    """All lattice-cell centres whose integer cell index lies within
    ``radius_cells`` (Euclidean, in cells) of the cell of some hit point:
    the 0.1 m cells within 1 m of the scan.  Returned in lexicographic cell
    order as float32 [m, 3]."""
    p = points.astype(np.float64)
    cell = np.floor(p / lattice).astype(np.int64)
    cell = np.unique(cell, axis=0)
    lo = cell.min(axis=0) - radius_cells
    hi = cell.max(axis=0) + radius_cells
    shape = tuple((hi - lo + 1).tolist())
    mask = np.zeros(shape, dtype=bool)
    rel = cell - lo
    r = radius_cells
    rng1 = np.arange(-r, r + 1)
    ox, oy, oz = np.meshgrid(rng1, rng1, rng1, indexing="ij")
    inside = ox * ox + oy * oy + oz * oz <= r * r
    offs = np.stack([ox[inside], oy[inside], oz[inside]], axis=1)
    for o in offs:
        t = rel + o
        mask[t[:, 0], t[:, 1], t[:, 2]] = True
    ix, iy, iz = np.nonzero(mask)
    c = np.stack([ix, iy, iz], axis=1) + lo
    return ((c.astype(np.float64) + 0.5) * lattice).astype(np.float32)


def sensor_path(seed: int, n_frames: int = 100, start=(0.0, 0.0, 1.5),
                step: float = 0.5, heading_sigma_deg: float = 10.0,
                bound: float = 18.0) -> np.ndarray:
    """Smooth random planar path: the heading changes by N(0, sigma) per step
    and the path reflects at +-bound.  float64 [n_frames, 3]."""
    rng = np.random.default_rng(seed)
    p = np.array(start, dtype=np.float64)
    th = rng.uniform(0.0, 2.0 * np.pi)
    out = [p.copy()]
    for _ in range(n_frames - 1):
        th += np.deg2rad(rng.normal(0.0, heading_sigma_deg))
        q = p + step * np.array([np.cos(th), np.sin(th), 0.0])
        if abs(q[0]) > bound:
            q[0] = math.copysign(2 * bound, q[0]) - q[0]
            th = np.pi - th
        if abs(q[1]) > bound:
            q[1] = math.copysign(2 * bound, q[1]) - q[1]
            th = -th
        p = q
        out.append(p.copy())
    return np.array(out)


# --------------------------------------------------------------------------
# Planar patches of uneven size, one per well-separated cell.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class PatchScene:
    points: np.ndarray     # float32 [N, 3], patch after patch
    sizes: np.ndarray      # int64 [G] points per patch
    queries: np.ndarray    # float32 [G * q_per, 3]
    cell: float


def planar_patches(seed: int = 3, n_patches: int = 8192, n_lo: int = 8,
                   n_hi: int = 256, cell: float = 0.8, half_width: float = 0.2,
                   noise: float = 0.01, q_per: int = 64,
                   grid=(16, 16, 32)) -> PatchScene:
    """One planar patch per cell of a sparse lattice whose occupied cells sit
    two cells apart (so no two patches are neighbours).  Patch i has
    U{n_lo..n_hi} points c + u e1 + v e2 + N(0, noise) n with u, v uniform in
    [-half_width, half_width] and a random unit normal n; ``q_per`` queries
    are drawn uniformly inside each occupied cell."""
    rng = np.random.default_rng(seed)
    gx, gy, gz = grid
    assert gx * gy * gz >= n_patches
    idx = np.stack(np.meshgrid(np.arange(gx), np.arange(gy), np.arange(gz),
                               indexing="ij"), axis=-1).reshape(-1, 3)
    idx = idx[:n_patches] * 2
    sizes = rng.integers(n_lo, n_hi + 1, size=n_patches)
    pts, qs = [], []
    for i in range(n_patches):
        lo = idx[i] * cell
        c = lo + 0.5 * cell
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        a = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(nrm, a)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        n = int(sizes[i])
        uv = rng.uniform(-half_width, half_width, size=(n, 2))
        h = rng.normal(0.0, noise, size=n)
        pts.append(c + uv[:, :1] * e1 + uv[:, 1:] * e2 + h[:, None] * nrm)
        qs.append(lo + rng.uniform(0.0, cell, size=(q_per, 3)))
    return PatchScene(points=np.concatenate(pts).astype(np.float32),
                      sizes=sizes.astype(np.int64),
                      queries=np.concatenate(qs).astype(np.float32),
                      cell=cell)


def jitter_points(points: np.ndarray, n: int, sigma: float, seed: int) -> np.ndarray:
    """n points drawn around randomly chosen input points with isotropic
    N(0, sigma^2) offsets (queries of the fused field near the surface)."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, points.shape[0], size=n)
    p = points[idx].astype(np.float64) + rng.normal(0.0, sigma, size=(n, 3))
    return p.astype(np.float32)


def shuffle_rows(a: np.ndarray, seed: int) -> np.ndarray:
    """A seeded row permutation (used to check order independence)."""
    return a[np.random.default_rng(seed).permutation(a.shape[0])]


# --------------------------------------------------------------------------
# A surface property per point (LiDAR intensity, a colour channel).
# --------------------------------------------------------------------------
def surface_intensity(points: np.ndarray, seed: int, sigma: float = 0.01) -> np.ndarray:
    """A smooth texture over space plus N(0, sigma) noise per point:
    0.5 + 0.3 sin(1.3 x) cos(0.9 y) + 0.1 tanh(z), as float32 [n]."""
    rng = np.random.default_rng(seed)
    x = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    v = 0.5 + 0.3 * np.sin(1.3 * x[:, 0]) * np.cos(0.9 * x[:, 1]) + 0.1 * np.tanh(x[:, 2])
    return (v + rng.normal(0.0, sigma, size=x.shape[0])).astype(np.float32)
