"""MI355X L-GPDF: local Gaussian-process distance fields (VDB-GPDF,
arXiv:2407.09649) on hand-written HIP kernels behind a C ABI.

This module only marshals arguments to ``libvdbgpdf.so`` (``include/vdbgpdf.h``):
torch tensors supply device memory and the current HIP stream; every step of
the computation runs in the library's kernels.  There is no CPU fallback: if
the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = ["Params", "Stats", "Context", "load_library", "library_path",
           "KERNEL_MATERN32", "KERNEL_SE", "SEL_NEIGHBOR27", "SEL_KNN",
           "COMB_SMOOTHMIN", "COMB_HARDMIN", "GRAD_WEIGHTED", "GRAD_PAPER_MEAN",
           "PREC_FP32", "PREC_BF16", "PREC_FP64", "PREC_FP32_MFMA", "MLP_NPARAM", "GpdfError",
           "FUSE_INVVAR", "FUSE_TSDF", "TEST_BAND", "TEST_RAYCAST",
           "STATUS_HASH_FULL", "STATUS_GLOBAL_FULL", "STATUS_NONFINITE", "STATUS_NONPD",
           "STATUS_CAPACITY"]

ABI_VERSION = 4
KERNEL_MATERN32, KERNEL_SE = 0, 1
SEL_NEIGHBOR27, SEL_KNN = 0, 1
COMB_SMOOTHMIN, COMB_HARDMIN = 0, 1
GRAD_WEIGHTED, GRAD_PAPER_MEAN = 0, 1
PREC_FP32, PREC_BF16, PREC_FP64, PREC_FP32_MFMA = 0, 1, 2, 3
FUSE_INVVAR, FUSE_TSDF = 0, 1
TEST_BAND, TEST_RAYCAST = 0, 1
MLP_NPARAM = 8897
STATUS_HASH_FULL, STATUS_GLOBAL_FULL, STATUS_NONFINITE, STATUS_NONPD, STATUS_CAPACITY = 1, 2, 4, 8, 16

_HERE = os.path.dirname(os.path.abspath(__file__))
_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "HIP", 4: "CAPACITY", 5: "NOT_TRAINED"}

EXPORTS = [
    "gpdf_params_default", "gpdf_create", "gpdf_destroy", "gpdf_train_local_gps",
    "gpdf_query_distance", "gpdf_fuse_frame", "gpdf_query_global", "gpdf_get_stats",
    "gpdf_last_error", "gpdf_export_model", "gpdf_export_global",
    "gpdf_export_test_points", "gpdf_save_global", "gpdf_load_global",
    "gpdf_nearest_distance", "gpdf_mlp_init", "gpdf_mlp_set_weights",
    "gpdf_set_tuning", "gpdf_get_tuning", "gpdf_autotune", "gpdf_fuse_frame_graph",
    "gpdf_mlp_get_weights", "gpdf_mlp_set_norm", "gpdf_mlp_get_norm", "gpdf_mlp_features",
    "gpdf_mlp_forward", "gpdf_mlp_grad", "gpdf_mlp_train", "gpdf_query_distance_noalloc",
    "gpdf_zero_crossings", "gpdf_train_local_gps_prop", "gpdf_query_distance_prop",
    "gpdf_fuse_frame_prop", "gpdf_query_global_prop", "gpdf_export_global_prop",
    "gpdf_tuning_cache_save", "gpdf_tuning_cache_load", "gpdf_tuning_cache_clear",
    "gpdf_measure_peaks",
]


class GpdfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gpdf status {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    """Mirror of ``gpdf_params``; defaults from ``gpdf_params_default``."""
    _fields_ = [
        ("abi_version", C.c_uint32), ("kernel", C.c_int32),
        ("length_scale", C.c_double), ("noise_sigma", C.c_double),
        ("voxel_size", C.c_double), ("cluster_size", C.c_double),
        ("selection", C.c_int32), ("knn_q", C.c_int32),
        ("combine", C.c_int32), ("grad_mode", C.c_int32),
        ("smooth_min_lambda", C.c_double), ("occ_min", C.c_double),
        ("occ_max", C.c_double), ("precision", C.c_int32), ("timing", C.c_int32),
        ("fuse_voxel_size", C.c_double), ("fuse_band", C.c_double),
        ("mlp_gate", C.c_double),
        ("max_points", C.c_int64), ("max_clusters", C.c_int64),
        ("max_cluster_points", C.c_int64), ("max_factor_elems", C.c_int64),
        ("max_queries", C.c_int64), ("global_capacity", C.c_int64),
        ("fuse_rule", C.c_int32), ("test_points", C.c_int32), ("normal_reach", C.c_double),
        ("lazy_train", C.c_int32), ("properties", C.c_int32),
    ]

    @classmethod
    def default(cls, **kw) -> "Params":
        p = cls()
        _check(load_library().gpdf_params_default(C.byref(p)), None)
        for k, v in kw.items():
            if not hasattr(p, k):
                raise AttributeError(k)
            setattr(p, k, v)
        return p


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "clusters", "points", "nonpd_clusters", "skipped_points", "queries",
        "valid_queries", "refined_queries", "test_points", "fused",
        "fuse_skipped", "global_voxels", "gated", "eval_pairs", "eval_points",
        "eval_tri", "refine_dist", "refine_grad", "refine_var")] + [
        ("status_bits", C.c_uint32), ("pad0", C.c_uint32), ("ms", C.c_float * 8),
        ("trained_clusters", C.c_int64), ("refine_pairs_small", C.c_int64),
        ("refine_pairs_large", C.c_int64), ("refine_items_large", C.c_int64)]

    STAGES = ("train", "group", "eval", "refine", "testpts", "fuse", "global", "mlp")

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("pad0", "ms")}
        d["ms"] = {k: float(self.ms[i]) for i, k in enumerate(self.STAGES)}
        return d


_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "libvdbgpdf.so")


def load_library():
    """Load libvdbgpdf.so (built by ``paper_2407_09649_amd.build``)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "python -m paper_2407_09649_amd.build")
        _lib = _bind(C.CDLL(path))
    return _lib


def _bind(L):
    P, I64, F, U64 = C.c_void_p, C.c_int64, C.c_float, C.c_uint64
    sig = {
        "gpdf_params_default": [P],
        "gpdf_create": [P, P, P],
        "gpdf_train_local_gps": [P, P, I64],
        "gpdf_query_distance": [P, P, I64, P, P, P, P, P, P, C.c_int32],
        "gpdf_query_distance_noalloc": [P, P, I64, P, P, P, P, P, P, C.c_int32],
        "gpdf_fuse_frame": [P, P, I64, P],
        "gpdf_train_local_gps_prop": [P, P, P, I64],
        "gpdf_query_distance_prop": [P, P, I64, P, P, P, P, P, P, P, P],
        "gpdf_fuse_frame_prop": [P, P, P, I64, P],
        "gpdf_query_global_prop": [P, P, I64, P, P],
        "gpdf_export_global_prop": [P, P, P, P, I64, P],
        "gpdf_query_global": [P, P, I64, P, P, P],
        "gpdf_get_stats": [P, P],
        "gpdf_export_model": [P, P, P, P, P, P],
        "gpdf_export_global": [P, P, P, P, P, I64, P],
        "gpdf_export_test_points": [P, P, I64, P],
        "gpdf_save_global": [P, C.c_char_p],
        "gpdf_load_global": [P, C.c_char_p],
        "gpdf_nearest_distance": [P, P, I64, P, I64, P],
        "gpdf_fuse_frame_graph": [P, P, I64, P],
        "gpdf_zero_crossings": [P, P, I64, P],
        "gpdf_set_tuning": [P, C.c_int32, C.c_int32, C.c_int32],
        "gpdf_get_tuning": [P, P, P, P],
        "gpdf_autotune": [P, P, I64, P, I64, P, P, P],
        "gpdf_tuning_cache_save": [C.c_char_p],
        "gpdf_tuning_cache_load": [C.c_char_p],
        "gpdf_tuning_cache_clear": [],
        "gpdf_measure_peaks": [P, P, C.c_int32],
        "gpdf_mlp_init": [P, U64],
        "gpdf_mlp_set_weights": [P, P, I64],
        "gpdf_mlp_get_weights": [P, P, I64],
        "gpdf_mlp_set_norm": [P, P, P],
        "gpdf_mlp_get_norm": [P, P, P],
        "gpdf_mlp_features": [P, P, P, P, P, I64, P],
        "gpdf_mlp_forward": [P, P, I64, P],
        "gpdf_mlp_grad": [P, P, P, I64, P, P],
        "gpdf_mlp_train": [P, P, P, I64, C.c_int32, C.c_int32, F, U64, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.gpdf_destroy.argtypes = [P]
    L.gpdf_destroy.restype = None
    L.gpdf_last_error.argtypes = [P]
    L.gpdf_last_error.restype = C.c_char_p
    return L


def _check(status, ctx):
    if status != 0:
        msg = ""
        if ctx is not None:
            m = load_library().gpdf_last_error(ctx)
            msg = m.decode() if m else ""
        raise GpdfError(status, msg)


def _dptr(t, dtype=None, shape_last=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a tensor on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"expected shape [n, {shape_last}]")
    return C.c_void_p(t.data_ptr())


def _host3(v):
    if v is None:
        return None
    a = (C.c_float * 3)(*[float(x) for x in v])
    return a


class Context:
    """One library context bound to the current HIP stream of a device."""

    def __init__(self, params: Params | None = None, device=None, stream=None, **kw):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device(device if device is not None else "cuda:0")
        self.params = params if params is not None else Params.default()
        for k, v in kw.items():
            setattr(self.params, k, v)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            _check(self.lib.gpdf_create(C.byref(self.params),
                                        C.c_void_p(self.stream.cuda_stream),
                                        C.byref(h)), None)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.gpdf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- core calls ---------------------------------------------------------
    def train(self, xyz):
        torch = self._torch
        n = 0 if xyz is None else xyz.shape[0]
        _check(self.lib.gpdf_train_local_gps(self._h, _dptr(xyz, torch.float32, 3) if n else None, n),
               self._h)

    def train_prop(self, xyz, prop):
        """gpdf_train_local_gps_prop: training with a surface property per point."""
        torch = self._torch
        n = xyz.shape[0]
        _check(self.lib.gpdf_train_local_gps_prop(self._h, _dptr(xyz, torch.float32, 3) if n else None,
                                                  _dptr(prop, torch.float32) if n else None, n), self._h)

    def query_prop(self, q, origin=None, grad=True, var=True, aux=True):
        """gpdf_query_distance_prop: query() plus prop and prop_var."""
        torch = self._torch
        m = q.shape[0]
        dev = self.device
        r = {"dist": torch.empty(m, dtype=torch.float32, device=dev),
             "valid": torch.empty(m, dtype=torch.uint8, device=dev),
             "prop": torch.empty(m, dtype=torch.float32, device=dev),
             "prop_var": torch.empty(m, dtype=torch.float32, device=dev)}
        if grad:
            r["grad"] = torch.empty((m, 3), dtype=torch.float32, device=dev)
        if var:
            r["var"] = torch.empty(m, dtype=torch.float32, device=dev)
        if aux:
            r["aux"] = torch.empty((m, 3), dtype=torch.float32, device=dev)
        _check(self.lib.gpdf_query_distance_prop(
            self._h, _dptr(q, torch.float32, 3) if m else None, m, _host3(origin), _dptr(r["dist"]),
            _dptr(r.get("grad")), _dptr(r.get("var")), _dptr(r["valid"]), _dptr(r.get("aux")),
            _dptr(r["prop"]), _dptr(r["prop_var"])), self._h)
        return r

    def query(self, q, origin=None, grad=True, var=True, aux=True, correct=False, out=None):
        torch = self._torch
        m = q.shape[0]
        dev = self.device
        o = out or {}
        dist = o.get("dist", torch.empty(m, dtype=torch.float32, device=dev))
        valid = o.get("valid", torch.empty(m, dtype=torch.uint8, device=dev))
        g = o.get("grad", torch.empty((m, 3), dtype=torch.float32, device=dev)) if grad else None
        v = o.get("var", torch.empty(m, dtype=torch.float32, device=dev)) if var else None
        a = o.get("aux", torch.empty((m, 3), dtype=torch.float32, device=dev)) if aux else None
        _check(self.lib.gpdf_query_distance(
            self._h, _dptr(q, torch.float32, 3) if m else None, m, _host3(origin),
            _dptr(dist), _dptr(g), _dptr(v), _dptr(valid), _dptr(a), int(bool(correct))), self._h)
        r = {"dist": dist, "valid": valid}
        if grad:
            r["grad"] = g
        if var:
            r["var"] = v
        if aux:
            r["aux"] = a
        return r

    def query_noalloc(self, q, out, origin=None, correct=False):
        """gpdf_query_distance_noalloc: the query into caller-provided
        buffers (``out``: dist, valid and optionally grad, var, aux), with no
        device allocation in the library."""
        torch = self._torch
        m = q.shape[0]
        _check(self.lib.gpdf_query_distance_noalloc(
            self._h, _dptr(q, torch.float32, 3) if m else None, m, _host3(origin),
            _dptr(out["dist"]), _dptr(out.get("grad")), _dptr(out.get("var")), _dptr(out["valid"]),
            _dptr(out.get("aux")), int(bool(correct))), self._h)
        return out

    def fuse(self, xyz, origin):
        torch = self._torch
        n = 0 if xyz is None else xyz.shape[0]
        _check(self.lib.gpdf_fuse_frame(
            self._h, _dptr(xyz, torch.float32, 3) if xyz is not None and n else None, n,
            _host3(origin)), self._h)

    def fuse_prop(self, xyz, prop, origin):
        """gpdf_fuse_frame_prop: train with a property per point and fuse it."""
        torch = self._torch
        n = xyz.shape[0]
        _check(self.lib.gpdf_fuse_frame_prop(self._h, _dptr(xyz, torch.float32, 3),
                                             _dptr(prop, torch.float32) if n else None, n,
                                             _host3(origin)), self._h)

    def query_global_prop(self, q):
        torch = self._torch
        m = q.shape[0]
        prop = torch.empty(m, dtype=torch.float32, device=self.device)
        valid = torch.empty(m, dtype=torch.uint8, device=self.device)
        _check(self.lib.gpdf_query_global_prop(self._h, _dptr(q, torch.float32, 3) if m else None, m,
                                               _dptr(prop), _dptr(valid)), self._h)
        return {"prop": prop, "valid": valid}

    def export_global_prop(self):
        import numpy as np
        cnt = C.c_int64(0)
        _check(self.lib.gpdf_export_global_prop(self._h, None, None, None, 0, C.byref(cnt)), self._h)
        n = cnt.value
        k = np.empty(n, np.uint64)
        Cp = np.empty(n, np.float32)
        W = np.empty(n, np.float32)
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(self.lib.gpdf_export_global_prop(self._h, P(k), P(Cp), P(W), n, C.byref(cnt)), self._h)
        return dict(key=k, C=Cp, W=W)

    def fuse_graph(self, xyz, origin):
        """fuse() as one replay of a captured HIP graph (captured on the first
        call); the counts stay on the device."""
        torch = self._torch
        n = xyz.shape[0]
        _check(self.lib.gpdf_fuse_frame_graph(self._h, _dptr(xyz, torch.float32, 3) if n else None, n,
                                              _host3(origin)), self._h)

    def query_global(self, q, grad=True):
        torch = self._torch
        m = q.shape[0]
        dist = torch.empty(m, dtype=torch.float32, device=self.device)
        valid = torch.empty(m, dtype=torch.uint8, device=self.device)
        g = torch.empty((m, 3), dtype=torch.float32, device=self.device) if grad else None
        _check(self.lib.gpdf_query_global(self._h, _dptr(q, torch.float32, 3) if m else None, m,
                                          _dptr(dist), _dptr(g), _dptr(valid)), self._h)
        r = {"dist": dist, "valid": valid}
        if grad:
            r["grad"] = g
        return r

    def nearest_distance(self, pts, q):
        torch = self._torch
        out = torch.empty(q.shape[0], dtype=torch.float32, device=self.device)
        _check(self.lib.gpdf_nearest_distance(self._h, _dptr(pts, torch.float32, 3), pts.shape[0],
                                              _dptr(q, torch.float32, 3), q.shape[0],
                                              _dptr(out)), self._h)
        return out

    # -- inspection ------------------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        _check(self.lib.gpdf_get_stats(self._h, C.byref(s)), self._h)
        return s.as_dict()

    def export_model(self):
        import numpy as np
        st = self.stats()
        nc, npt = st["clusters"], st["points"]
        ck = np.empty(nc, np.uint64)
        off = np.empty(nc + 1, np.int64)
        pts = np.empty((npt, 3), np.float32)
        al = np.empty(npt, np.float64)
        pd = np.empty(nc, np.uint8)
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(self.lib.gpdf_export_model(self._h, P(ck), P(off), P(pts), P(al), P(pd)), self._h)
        return dict(ckey=ck, off=off, points=pts, alpha=al, pd=pd.astype(bool))

    def export_global(self):
        import numpy as np
        cnt = C.c_int64(0)
        _check(self.lib.gpdf_export_global(self._h, None, None, None, None, 0, C.byref(cnt)), self._h)
        n = cnt.value
        k = np.empty(n, np.uint64)
        D = np.empty(n, np.float32)
        V = np.empty(n, np.float32)
        s = np.empty(n, np.uint32)
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(self.lib.gpdf_export_global(self._h, P(k), P(D), P(V), P(s), n, C.byref(cnt)), self._h)
        return dict(key=k, D=D, V=V, stamp=s)

    def export_test_points(self):
        import numpy as np
        cnt = C.c_int64(0)
        _check(self.lib.gpdf_export_test_points(self._h, None, 0, C.byref(cnt)), self._h)
        k = np.empty(cnt.value, np.uint64)
        _check(self.lib.gpdf_export_test_points(self._h, k.ctypes.data_as(C.c_void_p), cnt.value,
                                                C.byref(cnt)), self._h)
        return k

    def zero_crossings(self):
        """The surface points of the fused grid (gpdf_zero_crossings) as a
        device tensor [n, 3]."""
        torch = self._torch
        cnt = C.c_int64(0)
        _check(self.lib.gpdf_zero_crossings(self._h, None, 0, C.byref(cnt)), self._h)
        out = torch.empty((cnt.value, 3), dtype=torch.float32, device=self.device)
        if cnt.value:
            _check(self.lib.gpdf_zero_crossings(self._h, _dptr(out), cnt.value, C.byref(cnt)), self._h)
        return out

    def save_global(self, path):
        _check(self.lib.gpdf_save_global(self._h, os.fsencode(path)), self._h)

    def load_global(self, path):
        _check(self.lib.gpdf_load_global(self._h, os.fsencode(path)), self._h)

    # -- batching: tuned launch shapes ----------------------------------------
    def set_tuning(self, train_threads=256, eval_persistent=0, mfma_min_n=0):
        _check(self.lib.gpdf_set_tuning(self._h, int(train_threads), int(eval_persistent), int(mfma_min_n)),
               self._h)

    def get_tuning(self):
        t, p, mm = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _check(self.lib.gpdf_get_tuning(self._h, C.byref(t), C.byref(p), C.byref(mm)), self._h)
        return {"train_threads": t.value, "eval_persistent": p.value, "mfma_min_n": mm.value}

    def autotune(self, xyz, q, origin=None):
        """Times the launch-shape candidates on this workload (or takes them
        from the process-wide cache when its shape was tuned before), keeps
        the fastest and leaves the context trained on xyz.  Returns the
        median times (ms) of every candidate (-1: not run) and ``cached``."""
        import numpy as np
        torch = self._torch
        ms = np.zeros(11, np.float32)
        cached = C.c_int32(0)
        _check(self.lib.gpdf_autotune(self._h, _dptr(xyz, torch.float32, 3), xyz.shape[0],
                                      _dptr(q, torch.float32, 3), q.shape[0], _host3(origin),
                                      ms.ctypes.data_as(C.c_void_p), C.byref(cached)), self._h)
        names = ["train_256", "train_512", "train_1024", "eval_grid", "eval_persist1",
                 "eval_persist2", "eval_persist4", "eval_mfma_from17", "eval_mfma_from33",
                 "eval_mfma_from65", "eval_mfma_from129"]
        out = dict(zip(names, ms.tolist()))
        out["cached"] = bool(cached.value)
        return out

    def measure_peaks(self):
        """What this device sustains, from probe kernels: HBM copy GB/s, FP32
        FMA TFLOP/s (VOP2 register form; the VOP3 and literal forms beside
        it), exp2 Gop/s, BF16 / FP32 / FP64 MFMA TFLOP/s."""
        import numpy as np
        out = np.zeros(9, np.float64)
        _check(self.lib.gpdf_measure_peaks(self._h, out.ctypes.data_as(C.c_void_p), 9), self._h)
        names = ["hbm_copy_gbs", "fp32_valu_tflops", "exp2_gops", "mfma_bf16_tflops",
                 "mfma_f32_tflops", "mfma_f64_tflops", "copy_gib", "fp32_fma_vop3_tflops",
                 "fp32_fma_literal_tflops"]
        return dict(zip(names, out.tolist()))

    # -- learned correction ---------------------------------------------------
    def mlp_init(self, seed=0):
        _check(self.lib.gpdf_mlp_init(self._h, int(seed)), self._h)

    def mlp_set_weights(self, w):
        import numpy as np
        a = np.ascontiguousarray(w, np.float32)
        _check(self.lib.gpdf_mlp_set_weights(self._h, a.ctypes.data_as(C.c_void_p), a.size), self._h)

    def mlp_get_weights(self):
        import numpy as np
        a = np.empty(MLP_NPARAM, np.float32)
        _check(self.lib.gpdf_mlp_get_weights(self._h, a.ctypes.data_as(C.c_void_p), a.size), self._h)
        return a

    def mlp_set_norm(self, mean, std):
        import numpy as np
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(std, np.float32)
        _check(self.lib.gpdf_mlp_set_norm(self._h, m.ctypes.data_as(C.c_void_p),
                                          s.ctypes.data_as(C.c_void_p)), self._h)

    def mlp_get_norm(self):
        import numpy as np
        m = np.empty(7, np.float32)
        s = np.empty(7, np.float32)
        _check(self.lib.gpdf_mlp_get_norm(self._h, m.ctypes.data_as(C.c_void_p),
                                          s.ctypes.data_as(C.c_void_p)), self._h)
        return m, s

    def mlp_features(self, res):
        torch = self._torch
        n = res["dist"].shape[0]
        f = torch.empty((n, 7), dtype=torch.float32, device=self.device)
        _check(self.lib.gpdf_mlp_features(self._h, _dptr(res["dist"]), _dptr(res["var"]),
                                          _dptr(res["grad"]), _dptr(res["aux"]), n, _dptr(f)),
               self._h)
        return f

    def mlp_forward(self, feat):
        torch = self._torch
        r = torch.empty(feat.shape[0], dtype=torch.float32, device=self.device)
        _check(self.lib.gpdf_mlp_forward(self._h, _dptr(feat, torch.float32, 7), feat.shape[0],
                                         _dptr(r)), self._h)
        return r

    def mlp_grad(self, feat, target):
        torch = self._torch
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=self.device)
        loss = C.c_float(0)
        _check(self.lib.gpdf_mlp_grad(self._h, _dptr(feat, torch.float32, 7),
                                      _dptr(target, torch.float32), feat.shape[0], _dptr(g),
                                      C.byref(loss)), self._h)
        return g, loss.value

    def mlp_train(self, feat, target, epochs=1, batch=1024, lr=1e-3, seed=0):
        torch = self._torch
        loss = C.c_float(0)
        _check(self.lib.gpdf_mlp_train(self._h, _dptr(feat, torch.float32, 7),
                                       _dptr(target, torch.float32), feat.shape[0], int(epochs),
                                       int(batch), float(lr), int(seed), C.byref(loss)), self._h)
        return loss.value


def tuning_cache_save(path):
    """Write the process-wide tuning cache (gpdf_tuning_cache_save)."""
    _check(load_library().gpdf_tuning_cache_save(str(path).encode()), None)


def tuning_cache_load(path):
    """Add the entries of a tuning cache file (gpdf_tuning_cache_load)."""
    _check(load_library().gpdf_tuning_cache_load(str(path).encode()), None)


def tuning_cache_clear():
    _check(load_library().gpdf_tuning_cache_clear(), None)
