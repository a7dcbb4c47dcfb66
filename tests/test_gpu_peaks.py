"""The library's own ceiling microbenchmarks (rfd_measure_peaks): positive,
finite and below the published MI355X peaks they are compared with (FP32
vector 157.3 and FP64 78.6 TFLOP/s, dense BF16 MFMA 2.5 PFLOP/s, HBM 8 TB/s of
read + write)."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_measured_ceilings_are_plausible(rfd):
    p = rfd.rfd_measure_peaks()
    print(f"\n[peaks] {p}")
    for v in p.values():
        assert math.isfinite(v) and v > 0
    assert p["fp32_fma_TFLOPs"] <= 157.3 * 1.05
    assert p["fp64_fma_TFLOPs"] <= 78.6 * 1.05
    assert p["bf16_mfma_TFLOPs"] <= 2500 * 1.05
    assert p["copy_GBs"] <= 8000 * 1.05
