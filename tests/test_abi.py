"""The C-ABI library loads and exports every entry point of include/vdbgpdf.h.

CPU only: no call here touches the GPU.
"""
import ctypes
import os
import re

import paper_2407_09649_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vdbgpdf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(gpdf_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ["gpdf_train_local_gps", "gpdf_query_distance", "gpdf_fuse_frame",
              "gpdf_query_global", "gpdf_create", "gpdf_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.library_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(P.EXPORTS)


def test_params_default_layout_and_values():
    p = P.Params.default()
    assert p.abi_version == 4
    assert p.kernel == P.KERNEL_MATERN32
    assert p.length_scale == 0.2 and p.noise_sigma == 0.01
    assert p.cluster_size == 0.4 and p.voxel_size == 0.0
    assert p.selection == P.SEL_NEIGHBOR27 and p.knn_q == 8
    assert p.smooth_min_lambda == 100.0
    assert p.occ_min == 1e-15 and p.occ_max == 1.0 - 1e-5
    assert p.precision == P.PREC_FP32
    assert p.fuse_voxel_size == 0.05 and p.fuse_band == 0.2 and p.mlp_gate == 0.05
    assert p.max_cluster_points == 1024
    # the last field lands where the C struct puts it
    assert p.global_capacity == 1 << 24
    assert p.fuse_rule == P.FUSE_INVVAR and p.test_points == P.TEST_BAND and p.normal_reach == 0.2
    assert p.lazy_train == 0 and p.properties == 0
    assert ctypes.sizeof(P.Params) == 184


def test_create_rejects_bad_parameters_without_touching_the_gpu():
    lib = P.load_library()
    h = ctypes.c_void_p()
    bad = [dict(abi_version=7), dict(length_scale=0.0), dict(length_scale=float("nan")),
           dict(occ_max=1.0), dict(knn_q=0, selection=P.SEL_KNN), dict(kernel=9),
           dict(max_cluster_points=2048), dict(precision=5), dict(fuse_rule=2),
           dict(test_points=2), dict(test_points=P.TEST_RAYCAST, voxel_size=0.0),
           dict(normal_reach=-1.0), dict(lazy_train=2), dict(properties=2),
           dict(properties=1, precision=P.PREC_BF16), dict(properties=1, selection=P.SEL_KNN),
           dict(properties=1, lazy_train=1), dict(precision=4),
           dict(precision=P.PREC_FP32_MFMA, selection=P.SEL_KNN),
           dict(properties=1, precision=P.PREC_FP32_MFMA)]
    for kw in bad:
        p = P.Params.default(**kw)
        assert lib.gpdf_create(ctypes.byref(p), None, ctypes.byref(h)) == 1, kw
    assert lib.gpdf_create(None, None, ctypes.byref(h)) == 1
    s = P.Stats()
    assert lib.gpdf_get_stats(None, ctypes.byref(s)) == 1
    assert lib.gpdf_last_error(None) == b"null context"
