"""Pins of the oracle's ray-cast test points (Sec. IV-B).

The walk from the sensor's voxel to the measured voxel is checked against an
exact segment/voxel intersection test in rational arithmetic; the normal
direction against planes whose normal is known; the selection of previously
observed voxels against the map's contents.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

HF = 0.05   # global voxel
HV = 0.1    # training voxel


def _pack(c):
    return ((int(c[0]) + (1 << 20)) << 42) | ((int(c[1]) + (1 << 20)) << 21) | (int(c[2]) + (1 << 20))


def _unpack(k):
    k = int(k)
    return ((k >> 42) & 0x1FFFFF) - (1 << 20), ((k >> 21) & 0x1FFFFF) - (1 << 20), (k & 0x1FFFFF) - (1 << 20)


def _fine(x):
    return tuple(int(np.floor(np.float64(v) / HF)) for v in x)


def _segment_voxels(O_, E_):
    """Voxels whose interior the segment between the centres of O_ and E_
    (voxel units) passes through, by exact slab intersection."""
    D = [E_[a] - O_[a] for a in range(3)]
    lo = [min(O_[a], E_[a]) for a in range(3)]
    hi = [max(O_[a], E_[a]) for a in range(3)]
    out = set()
    for x in range(lo[0], hi[0] + 1):
        for y in range(lo[1], hi[1] + 1):
            for z in range(lo[2], hi[2] + 1):
                v = (x, y, z)
                t0, t1 = Fraction(0), Fraction(1)
                ok = True
                for a in range(3):
                    if D[a] == 0:
                        ok = ok and v[a] == O_[a]
                        continue
                    u1 = Fraction(2 * (v[a] - O_[a]) - 1, 2 * D[a])
                    u2 = Fraction(2 * (v[a] + 1 - O_[a]) - 1, 2 * D[a])
                    a1, a2 = min(u1, u2), max(u1, u2)
                    t0, t1 = max(t0, a1), min(t1, a2)
                if ok and t0 < t1:
                    out.add(v)
    return out


def _block_map(lo, hi):
    """A map holding every global voxel of the box [lo, hi] (voxel units)."""
    cc = np.stack(np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in range(3)], indexing="ij"), -1).reshape(-1, 3)
    keys = np.array(sorted(_pack(c) for c in cc), np.uint64)
    g = O.Map()
    n = len(keys)
    g.merge(keys, np.full(n, 0.1), np.full(n, 0.01), np.ones(n, np.uint8), 0)
    return g


@pytest.mark.parametrize("delta", [(7, 2, 4), (-5, 12, -2), (3, -6, 0), (0, 0, 9), (-11, -4, 8)])
def test_ray_walk_visits_exactly_the_voxels_of_the_segment(delta):
    # Deltas with no two components tying (an odd and an even, or two even
    # ones of different powers of two), so that the segment never passes
    # exactly through a voxel edge or corner and the visited set is unique.
    # A single training voxel has no normal (fewer than 3 neighbours), and
    # with every voxel of the box in the map its test voxels are the walk.
    # the training point is the centre of a 0.1 m voxel, which lies on a
    # corner of the 0.05 m voxels: its global voxel E is the upper one
    E_ = (12, 5, -7)
    O_ = tuple(E_[a] - delta[a] for a in range(3))
    origin = np.array([(O_[a] + 0.5) * HF for a in range(3)], np.float32)
    x = np.array([[(E_[a] // 2 + 0.5) * HV for a in range(3)]], np.float32)
    m = O.Model(O.Params(voxel=HV, fuse_voxel=HF, tp_mode=1), x)
    assert _fine(origin) == O_ and _fine(m.export()["points"][0]) == E_
    lo = [min(O_[a], E_[a]) - 1 for a in range(3)]
    hi = [max(O_[a], E_[a]) + 1 for a in range(3)]
    g = _block_map(lo, hi)
    got = {_unpack(k) for k in m.test_points_ray(g, origin)}
    expect = _segment_voxels(O_, E_)
    assert got == expect
    assert len(expect) == sum(abs(d) for d in delta) + 1   # a face-connected walk
    # an empty map keeps only the measured voxel
    assert {_unpack(k) for k in m.test_points_ray(None, origin)} == {E_}


def test_ray_walk_through_edges_steps_the_lower_axis_first():
    # (3, 3, 0): the segment runs through voxel edges; at equal crossing
    # parameters the walk steps x before y: a staircase x, y, x, y, ...
    E_ = (12, 5, -7)
    O_ = (9, 2, -7)
    origin = np.array([(O_[a] + 0.5) * HF for a in range(3)], np.float32)
    x = np.array([[(E_[a] // 2 + 0.5) * HV for a in range(3)]], np.float32)
    m = O.Model(O.Params(voxel=HV, fuse_voxel=HF, tp_mode=1), x)
    g = _block_map([8, 1, -8], [13, 6, -6])
    got = {_unpack(k) for k in m.test_points_ray(g, origin)}
    expect = {(9, 2, -7), (10, 2, -7), (10, 3, -7), (11, 3, -7), (11, 4, -7), (12, 4, -7), (12, 5, -7)}
    assert got == expect


def test_ray_keeps_only_previously_observed_voxels():
    x = np.array([[0.45, 0.25, 0.15]], np.float32)
    m = O.Model(O.Params(voxel=HV, fuse_voxel=HF, tp_mode=1), x)
    E_ = _fine(m.export()["points"][0])
    O_ = tuple(E_[a] - (9, 4, 2)[a] for a in range(3))   # a delta with no ties
    origin = np.array([(O_[a] + 0.5) * HF for a in range(3)], np.float32)
    walk = _segment_voxels(O_, E_)
    rng = np.random.default_rng(3)
    held = {v for v in walk if rng.random() < 0.4} | {(20, 20, 20)}
    keys = np.array(sorted(_pack(v) for v in held), np.uint64)
    g = O.Map()
    g.merge(keys, np.full(len(keys), 0.1), np.full(len(keys), 0.01), np.ones(len(keys), np.uint8), 0)
    got = {_unpack(k) for k in m.test_points_ray(g, origin)}
    assert got == (held & walk) | {E_}


@pytest.mark.parametrize("normal,span", [((0, 0, 1), ((0, 1, 0), (1, 0, 0))),
                                         ((1, 1, 0), ((1, -1, 0), (0, 0, 1))),
                                         ((1, 0, 2), ((2, 0, -1), (0, 1, 0)))])
def test_normal_voxels_of_a_plane(normal, span):
    # Training voxels on a lattice plane spanned by two integer vectors: the
    # least-spread direction is the plane's normal, and every measured voxel
    # gets the voxels E + k n with k^2 |n|^2 <= R^2, R = reach / h_f = 4.
    a, b = np.array(span[0]), np.array(span[1])
    base = np.array([40, -30, 12])
    vox = np.array([base + i * a + j * b for i in range(-3, 4) for j in range(-3, 4)])
    x = ((vox + 0.5) * HV).astype(np.float32)
    origin = np.array([0.0, 0.0, 30.0], np.float32)   # far: the empty map keeps no ray voxel
    m = O.Model(O.Params(voxel=HV, fuse_voxel=HF, tp_mode=1, normal_reach=0.2), x)
    got = {_unpack(k) for k in m.test_points_ray(None, origin)}
    n = np.array(normal)
    R = 4
    expect = set()
    for p in m.export()["points"]:
        E = np.array(_fine(p))
        expect.add(tuple(E))
        for k in range(-R, R + 1):
            if k != 0 and k * k * int(n @ n) <= R * R:
                expect.add(tuple(E + k * n))
    assert got == expect


def test_few_neighbours_give_no_normal_voxels():
    x = np.array([[1.05, 2.05, 0.55], [1.15, 2.05, 0.55]], np.float32)   # two voxels
    m = O.Model(O.Params(voxel=HV, fuse_voxel=HF, tp_mode=1), x)
    got = {_unpack(k) for k in m.test_points_ray(None, np.zeros(3, np.float32))}
    assert got == {_fine(p) for p in m.export()["points"]}


def test_fusion_uses_the_ray_test_points():
    rng = np.random.default_rng(5)
    pts = np.concatenate([np.stack([rng.uniform(-1, 1, 400), rng.uniform(-1, 1, 400), np.full(400, 0.03)], 1),
                          np.stack([np.full(200, 0.83), rng.uniform(-1, 1, 200), rng.uniform(0, 1, 200)], 1)])
    pts = pts.astype(np.float32)
    origin = np.array([-0.5, 0.2, 1.2], np.float32)
    prm = O.Params(voxel=HV, fuse_voxel=HF, tp_mode=1, normal_reach=0.2)
    m = O.Model(prm, pts)
    g = O.Map()
    k0 = m.test_points_ray(g, origin)
    n, _ = g.fuse(m, origin, 0)
    assert n == len(k0) and g.size() <= n
    # the wall is gone in the next frame (a dynamic object): the rays to the
    # ground behind it cross the voxels fused around the wall, which are
    # tested again (and only voxels the map holds are added by the rays)
    origin2 = np.array([-0.2, 0.0, 0.8], np.float32)
    ground = np.stack([rng.uniform(-1, 2, 900), rng.uniform(-1, 1, 900), np.full(900, 0.03)], 1).astype(np.float32)
    m2 = O.Model(prm, ground)
    own = m2.test_points_ray(None, origin2)
    k1 = m2.test_points_ray(g, origin2)
    extra = np.setdiff1d(k1, own)
    held = set(g.export()["key"].tolist())
    assert len(extra) > 0 and all(int(k) in held for k in extra)
    wall = np.array([_unpack(k)[0] for k in extra])
    assert ((wall >= 14) & (wall <= 19)).mean() > 0.5   # mostly around the wall at x = 0.83 m
