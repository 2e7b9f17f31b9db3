"""FP64 CPU oracle of the L-GPDF hot path (VDB-GPDF, arXiv:2407.09649).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never loads it and it never loads the product library: the two share no code.

The arithmetic lives in ``gpdf_oracle.c`` (plain C, double precision, no
fast-math, no FP contraction), and ``mlp.py`` (NumPy float64).  This module
only marshals NumPy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpdf_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile the C oracle in place (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-Wno-unused-parameter", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(C.CDLL(_LIB))
    return _lib


class Params(C.Structure):
    """Mirror of ``orc_params``.  Defaults: the noisy-sphere configuration
    (Matern-3/2, l = 0.2 m, s = 0.01, raw points in 0.4 m cells, 27-cell
    selection, smooth minimum with lambda = 100)."""
    _fields_ = [
        ("kernel", C.c_int32), ("selection", C.c_int32), ("knn_q", C.c_int32),
        ("combine", C.c_int32), ("grad_mode", C.c_int32), ("pad_", C.c_int32),
        ("l", C.c_double), ("s", C.c_double), ("voxel", C.c_double),
        ("cell", C.c_double), ("lam", C.c_double), ("occ_min", C.c_double),
        ("occ_max", C.c_double), ("fuse_voxel", C.c_double),
        ("fuse_band", C.c_double), ("fuse_rule", C.c_int32),
        ("tp_mode", C.c_int32), ("normal_reach", C.c_double),
    ]

    def __init__(self, **kw):
        d = dict(kernel=0, selection=0, knn_q=8, combine=0, grad_mode=0,
                 pad_=0, l=0.2, s=0.01, voxel=0.0, cell=0.4, lam=100.0,
                 occ_min=1e-15, occ_max=1.0 - 1e-5, fuse_voxel=0.05,
                 fuse_band=0.2, fuse_rule=0, tp_mode=0, normal_reach=0.2)
        d.update(kw)
        super().__init__(**d)

    def copy(self, **kw):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d.update(kw)
        return Params(**d)


_P = C.c_void_p
_I64 = C.c_int64
_D = C.c_double


def _bind(L):
    L.orc_keys.argtypes = [_P, _I64, _D, _P, _P]
    L.orc_keys.restype = _I64
    L.orc_matern_t.argtypes = [_D]
    L.orc_matern_t.restype = _D
    L.orc_revert.argtypes = [C.POINTER(Params), _D, C.POINTER(_D), C.POINTER(_D)]
    L.orc_revert.restype = None
    L.orc_cholesky.argtypes = [_P, _I64]
    L.orc_cholesky.restype = C.c_int
    L.orc_train.argtypes = [C.POINTER(Params), _P, _I64, C.c_int]
    L.orc_train_prop.argtypes = [C.POINTER(Params), _P, _P, _I64, C.c_int]
    L.orc_train_prop.restype = _P
    L.orc_model_props.argtypes = [_P, _P, _P]
    L.orc_query_prop.argtypes = [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_int]
    L.orc_map_merge_prop.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _I64, C.c_uint32, C.c_int]
    L.orc_map_merge_prop.restype = _I64
    L.orc_map_export_prop.argtypes = [_P, _P, _P]
    L.orc_query_global_prop.argtypes = [_P, _D, _P, _I64, _P, _P]
    L.orc_train.restype = _P
    L.orc_free.argtypes = [_P]
    L.orc_model_sizes.argtypes = [_P, _P]
    L.orc_model_export.argtypes = [_P, _P, _P, _P, _P, _P]
    L.orc_model_factor.argtypes = [_P, _I64, _P]
    L.orc_query.argtypes = [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, C.c_int]
    L.orc_test_points.argtypes = [_P, _P, _I64]
    L.orc_test_points_ray.argtypes = [_P, _P, _P, _P, _I64]
    L.orc_test_points_ray.restype = _I64
    L.orc_test_points.restype = _I64
    L.orc_voxel_centres.argtypes = [_P, _I64, _D, _P]
    L.orc_map_new.restype = _P
    L.orc_map_free.argtypes = [_P]
    L.orc_map_size.argtypes = [_P]
    L.orc_map_size.restype = _I64
    L.orc_map_export.argtypes = [_P, _P, _P, _P, _P, _P]
    L.orc_map_merge.argtypes = [_P, _P, _P, _P, _P, _P, _I64, C.c_uint32, C.c_int]
    L.orc_map_merge.restype = _I64
    L.orc_fuse.argtypes = [_P, _P, _P, C.c_uint32, C.POINTER(_I64), C.c_int]
    L.orc_fuse.restype = _I64
    L.orc_query_global.argtypes = [_P, _D, _P, _I64, _P, _P, _P, _P]
    L.orc_nearest_distance.argtypes = [_P, _I64, _P, _I64, _P, C.c_int]
    L.orc_zero_crossings.argtypes = [_P, _D, _P, _I64]
    L.orc_zero_crossings.restype = _I64
    L.orc_max_threads.restype = C.c_int
    return L


class _Alt(C.Structure):
    """Mirror of ``orc_alt``: the second-closest node's results."""
    _fields_ = [("tie", C.c_void_p), ("dist", C.c_void_p), ("grad", C.c_void_p),
                ("var", C.c_void_p), ("prop", C.c_void_p), ("prop_var", C.c_void_p)]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def keys(xyz, h):
    """Packed voxel keys of FP32 points at edge h (and a validity mask)."""
    x = _f32(xyz).reshape(-1, 3)
    k = np.empty(x.shape[0], np.uint64)
    ok = np.empty(x.shape[0], np.uint8)
    lib().orc_keys(_ptr(x), x.shape[0], float(h), _ptr(k), _ptr(ok))
    return k, ok.astype(bool)


def matern_t(o: float) -> float:
    return float(lib().orc_matern_t(float(o)))


def revert(params: Params, o: float):
    d, lam = _D(), _D()
    lib().orc_revert(C.byref(params), float(o), C.byref(d), C.byref(lam))
    return d.value, lam.value


def cholesky(A):
    """Lower Cholesky factor of A (copy) and the positive-definiteness flag."""
    A = np.array(A, dtype=np.float64, order="C")
    ok = lib().orc_cholesky(_ptr(A), A.shape[0])
    return np.tril(A), bool(ok)


class Model:
    """The local GPs of one point cloud (one per leaf cluster)."""

    def __init__(self, params: Params, xyz, nthreads: int = 0, prop=None):
        """prop: optional surface property per input point (Eq. (6))."""
        self.params = params.copy()
        x = _f32(xyz).reshape(-1, 3)
        self.has_props = prop is not None
        if prop is None:
            self._h = lib().orc_train(C.byref(self.params), _ptr(x), x.shape[0],
                                      int(nthreads))
        else:
            c = _f32(prop).reshape(-1)
            assert c.shape[0] == x.shape[0]
            self._h = lib().orc_train_prop(C.byref(self.params), _ptr(x), _ptr(c),
                                           x.shape[0], int(nthreads))
        s = np.zeros(4, np.int64)
        lib().orc_model_sizes(self._h, _ptr(s))
        self.nclusters, self.npoints, self.nonpd, self.skipped = map(int, s)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def export(self):
        nc, npt = self.nclusters, self.npoints
        ck = np.empty(nc, np.uint64)
        off = np.empty(nc + 1, np.int64)
        pts = np.empty((npt, 3), np.float32)
        al = np.empty(npt, np.float64)
        pd = np.empty(nc, np.uint8)
        lib().orc_model_export(self._h, _ptr(ck), _ptr(off), _ptr(pts),
                               _ptr(al), _ptr(pd))
        return dict(ckey=ck, off=off, points=pts, alpha=al, pd=pd.astype(bool))

    def props(self):
        """Property c and beta = (K + s^2 I)^{-1} c of every training point."""
        c = np.empty(self.npoints)
        b = np.empty(self.npoints)
        if not lib().orc_model_props(self._h, _ptr(c), _ptr(b)):
            raise ValueError("model trained without properties")
        return dict(prop=c, beta=b)

    def factor(self, c: int):
        e = self.export()
        n = int(e["off"][c + 1] - e["off"][c])
        L = np.empty((n, n), np.float64)
        lib().orc_model_factor(self._h, int(c), _ptr(L))
        return L

    def query(self, q, origin=None, nthreads: int = 0):
        """Distance, gradient, variance, validity and aux (occupancy and
        latent variance of the closest node, points used) per query.  With an
        origin the result is signed and ``sign_tie`` marks the queries whose
        sign an FP32 evaluation could decide the other way.  ``node_tie``
        marks the queries whose second-closest node lies within 2e-4 m of the
        closest, and ``alt`` holds their results with that node taken as the
        closest (the other valid answer of the closest-node rule)."""
        x = _f32(q).reshape(-1, 3)
        m = x.shape[0]
        out = dict(dist=np.empty(m), grad=np.empty((m, 3)), var=np.empty(m),
                   valid=np.empty(m, np.uint8), aux=np.empty((m, 3)),
                   sign_tie=np.zeros(m, np.uint8))
        o = None if origin is None else _f32(origin).reshape(3)
        if self.has_props:
            out["prop"] = np.empty(m)
            out["prop_var"] = np.empty(m)
        alt = dict(tie=np.zeros(m, np.uint8), dist=np.zeros(m), grad=np.zeros((m, 3)), var=np.zeros(m),
                   prop=np.zeros(m), prop_var=np.zeros(m))
        ab = _Alt(*[_ptr(alt[k]) for k in ("tie", "dist", "grad", "var", "prop", "prop_var")])
        lib().orc_query_prop(self._h, _ptr(x), m, _ptr(o), _ptr(out["dist"]),
                             _ptr(out["grad"]), _ptr(out["var"]),
                             _ptr(out["valid"]), _ptr(out["aux"]), _ptr(out["sign_tie"]),
                             _ptr(out.get("prop")), _ptr(out.get("prop_var")), C.byref(ab), int(nthreads))
        alt["tie"] = alt["tie"].astype(bool)
        out["node_tie"] = alt["tie"]
        out["alt"] = alt
        out["valid"] = out["valid"].astype(bool)
        out["sign_tie"] = out["sign_tie"].astype(bool)
        return out

    def test_points(self):
        n = int(lib().orc_test_points(self._h, None, 0))
        k = np.empty(n, np.uint64)
        lib().orc_test_points(self._h, _ptr(k), n)
        return k

    def test_points_ray(self, gmap, origin):
        """Ray-cast test voxels (Sec. IV-B) against the map ``gmap`` (None:
        an empty map): sorted unique keys."""
        o = _f32(origin).reshape(3)
        g = None if gmap is None else gmap._h
        n = int(lib().orc_test_points_ray(self._h, g, _ptr(o), None, 0))
        k = np.empty(n, np.uint64)
        lib().orc_test_points_ray(self._h, g, _ptr(o), _ptr(k), n)
        return k


def voxel_centres(keys_, h):
    k = np.ascontiguousarray(keys_, dtype=np.uint64)
    x = np.empty((k.shape[0], 3), np.float32)
    lib().orc_voxel_centres(_ptr(k), k.shape[0], float(h), _ptr(x))
    return x


class Map:
    """The fused global grid: sorted (key, D, V, stamp) records."""

    def __init__(self):
        self._h = lib().orc_map_new()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_map_free(h)
            self._h = None

    def fuse(self, model: Model, origin, frame: int, nthreads: int = 0):
        sk = _I64(0)
        o = _f32(origin).reshape(3)
        n = lib().orc_fuse(self._h, model._h, _ptr(o), int(frame),
                           C.byref(sk), int(nthreads))
        return int(n), int(sk.value)

    def merge(self, keys_, d, v, ok, frame: int, tie=None, rule: int = 0, prop=None, prop_var=None):
        k = np.ascontiguousarray(keys_, np.uint64)
        d = np.ascontiguousarray(d, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        ok = np.ascontiguousarray(ok, np.uint8)
        t = None if tie is None else np.ascontiguousarray(tie, np.uint8)
        c = None if prop is None else np.ascontiguousarray(prop, np.float64)
        cv = None if prop is None else np.ascontiguousarray(prop_var, np.float64)
        return int(lib().orc_map_merge_prop(self._h, _ptr(k), _ptr(d), _ptr(v), _ptr(ok), _ptr(t),
                                            _ptr(c), _ptr(cv), k.shape[0], int(frame), int(rule)))

    def size(self) -> int:
        return int(lib().orc_map_size(self._h))

    def export(self):
        n = self.size()
        k = np.empty(n, np.uint64)
        D = np.empty(n)
        V = np.empty(n)
        s = np.empty(n, np.uint32)
        t = np.empty(n, np.uint8)
        lib().orc_map_export(self._h, _ptr(k), _ptr(D), _ptr(V), _ptr(s), _ptr(t))
        out = dict(key=k, D=D, V=V, stamp=s, sign_tie=t.astype(bool))
        Cp, W = np.empty(n), np.empty(n)
        if lib().orc_map_export_prop(self._h, _ptr(Cp), _ptr(W)):
            out["C"], out["W"] = Cp, W
        return out

    def zero_crossings(self, h):
        """Surface points on the grid edges where D changes sign (linear
        interpolation along the edge), ascending voxel key then axis."""
        n = int(lib().orc_zero_crossings(self._h, float(h), None, 0))
        out = np.empty((n, 3), np.float32)
        lib().orc_zero_crossings(self._h, float(h), _ptr(out), n)
        return out

    def query(self, h, q):
        x = _f32(q).reshape(-1, 3)
        m = x.shape[0]
        d = np.empty(m)
        g = np.empty((m, 3))
        ok = np.empty(m, np.uint8)
        t = np.empty(m, np.uint8)
        lib().orc_query_global(self._h, float(h), _ptr(x), m, _ptr(d), _ptr(g),
                               _ptr(ok), _ptr(t))
        return dict(dist=d, grad=g, valid=ok.astype(bool), sign_tie=t.astype(bool))

    def query_prop(self, h, q):
        """Trilinear interpolation of the fused property; valid where the
        eight voxels around q exist and hold a property."""
        x = _f32(q).reshape(-1, 3)
        m = x.shape[0]
        c = np.empty(m)
        ok = np.empty(m, np.uint8)
        lib().orc_query_global_prop(self._h, float(h), _ptr(x), m, _ptr(c), _ptr(ok))
        return dict(prop=c, valid=ok.astype(bool))


def nearest_distance(points, q, nthreads: int = 0):
    p = _f32(points).reshape(-1, 3)
    x = _f32(q).reshape(-1, 3)
    out = np.empty(x.shape[0])
    lib().orc_nearest_distance(_ptr(p), p.shape[0], _ptr(x), x.shape[0],
                               _ptr(out), int(nthreads))
    return out
