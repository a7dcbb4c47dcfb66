"""Least-squares ratio taps (Sec. V.A) against the FP64 oracle at tap counts
that reach every shape of the triangular solves (one wavefront per template
owning 4, 8, 16 or 32 rows per lane: T <= 256, 512, 1024, 2048), with one and
several templates per sub-bank.  At N = 2^13 (128 x 64) the correlation lags of
T = 64 come from per-workgroup lag shares, those of the larger T from the
row-limited column transform and direct lag sums, so both routes are checked."""
import numpy as np
import pytest

import synth
from gpu_cases import SB, Case, gpu_search, oracle_case

pytestmark = pytest.mark.gpu

FS, F_LOW = 2048.0, 30.0
SIZES = [(64, -32, 3), (300, -150, 2), (700, -350, 2), (1500, -750, 1)]


@pytest.fixture(scope="module")
def sized(rfd):
    n = 1 << 13
    w = synth.Workload("tapsizes", 9, n, FS, F_LOW, 0, 1, 0, "fp32", "nonspin")
    rng = np.random.default_rng(11)
    psd = synth.psd_array(n, FS)
    s = synth.make_noise_spectrum(w, rng)
    h_ref = synth.taylorf2(synth.WaveformParams(6.0, 5.0), n, FS, F_LOW)
    subbanks = []
    for T, k0, count in SIZES:
        params = [synth.WaveformParams(*m) for m in rng.uniform(5.0, 7.5, size=(count, 2))]
        subbanks.append(SB(0, T, k0, synth.template_batch(w, params), "ls"))
    case = Case("tapsizes", n, FS, F_LOW, psd, synth.spectrum_to_time(s, n, FS), {0: h_ref}, subbanks)
    oracle_case(case)
    srch = gpu_search(case)
    yield case, srch
    srch.close()


def test_ls_taps_every_solve_shape(rfd, sized):
    case, s = sized
    j = 0
    for sb in case.subbanks:
        worst = 0.0
        for _ in range(sb.H.shape[0]):
            tt = case.oracle["taps"][j]
            a, sig, T, k0 = s.tap(j)
            assert T == sb.T and k0 == sb.k0
            worst = max(worst, np.max(np.abs(a - tt.a)) / np.max(np.abs(tt.a)))
            assert abs(sig - tt.sigma_fit) <= 1e-9 * tt.sigma_fit
            j += 1
        print(f"\n[taps T={sb.T}] max rel |da| = {worst:.3e}")
        assert worst <= 1e-8
