"""The peak-measurement probes: every figure is positive and no figure is
above the device's published peak (HBM 8 TB/s; FP32 vector 157.3 TFLOP/s;
dense MFMA BF16 2.5 PFLOP/s, FP32 157.3 and FP64 78.6 TFLOP/s; exp2 at
most at half the non-packed FMA issue rate, 256 CU x 64 lanes x 2.4 GHz / 2,
twice the quarter rate of earlier CDNA parts)."""
import pytest

import paper_2407_09649_amd as P

from parity import small_params

pytestmark = pytest.mark.gpu

CEILING = {"hbm_copy_gbs": 8000.0, "fp32_valu_tflops": 157.3, "fp32_fma_vop3_tflops": 157.3,
           "fp32_fma_literal_tflops": 157.3, "exp2_gops": 256 * 64 * 2.4 / 2 * 1.01,
           "mfma_bf16_tflops": 2500.0, "mfma_f32_tflops": 157.3, "mfma_f64_tflops": 78.6}


def test_measured_peaks_are_positive_and_below_the_published_ones(dev):
    with P.Context(small_params(), device=dev) as ctx:
        pk = ctx.measure_peaks()
    print(pk, flush=True)
    assert pk["copy_gib"] == 1.0
    for k, hi in CEILING.items():
        assert 0 < pk[k] <= hi, (k, pk[k])
