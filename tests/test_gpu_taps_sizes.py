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


# Long segments: N2 = 1024 (N = 2^20, four columns per workgroup) and N2 = 2048
# (N = 2^22, two columns per workgroup) of the per-workgroup lag shares.
@pytest.mark.parametrize("log2n", [20, 22])
def test_ls_taps_long_segments(rfd, log2n):
    from oracle import pipeline as orc
    from oracle import taps as otaps
    n, T, k0 = 1 << log2n, 128, -64
    w = synth.Workload(f"taps{log2n}", 9, n, FS, F_LOW, 0, 1, 0, "fp32", "nonspin")
    rng = np.random.default_rng(log2n)
    psd = synth.psd_array(n, FS)
    s = synth.make_noise_spectrum(w, rng)
    h_ref = synth.taylorf2(synth.WaveformParams(3.0, 2.5), n, FS, F_LOW)
    params = [synth.WaveformParams(*m) for m in rng.uniform(2.7, 3.3, size=(2, 2))]
    H = synth.template_batch(w, params)
    data = synth.spectrum_to_time(s, n, FS)
    case = Case(f"taps{log2n}", n, FS, F_LOW, psd, data, {0: h_ref}, [SB(0, T, k0, H, "ls")])
    p = orc.prepare(psd, data, FS, F_LOW)
    M = otaps.gram(h_ref, p.w, T)
    srch = gpu_search(case)
    try:
        for j in range(H.shape[0]):
            tt = orc.make_taps(p, H[j], h_ref, T, k0, method="ls", M=M)
            a, sig, Tg, k0g = srch.tap(j)
            rel = np.max(np.abs(a - tt.a)) / np.max(np.abs(tt.a))
            print(f"\n[taps N=2^{log2n}] template {j}: max rel |da| = {rel:.3e}")
            assert rel <= 1e-8
            assert abs(sig - tt.sigma_fit) <= 1e-9 * tt.sigma_fit
    finally:
        srch.close()


def test_ls_taps_reject_singular_gram(rfd):
    """A reference that vanishes in band gives g = 0: the ridge normal matrix
    M + eps g[0] I is zero, so the factorisation must report that it is not
    positive definite (RFD_E_INVALID) instead of returning taps; the same
    taps object then accepts a proper reference."""
    import torch
    n = 1 << 13
    psd = synth.psd_array(n, FS)
    rng = np.random.default_rng(5)
    w = synth.Workload("tapsingular", 9, n, FS, F_LOW, 0, 1, 0, "fp32", "nonspin")
    params = [synth.WaveformParams(*m) for m in rng.uniform(5.0, 7.5, size=(2, 2))]
    H = torch.from_numpy(synth.template_batch(w, params)).cuda()
    plan = rfd.rfd_plan_create(psd, F_LOW, FS, n, 1)
    taps = rfd.rfd_taps_create(plan, [0, 2], [0], [64], [-32])
    try:
        zero = torch.zeros(n // 2 + 1, dtype=torch.complex128, device="cuda")
        with pytest.raises(rfd.RfdError) as err:
            rfd.rfd_make_taps(plan, taps, 0, zero, H)
        assert err.value.code == rfd.RFD_E_INVALID
        assert "positive definite" in str(err.value)
        h_ref = torch.from_numpy(synth.taylorf2(synth.WaveformParams(6.0, 5.0), n, FS, F_LOW)).cuda()
        rfd.rfd_make_taps(plan, taps, 0, h_ref, H)
        a, sig, T, k0 = rfd.rfd_taps_get(taps, 0)
        assert T == 64 and np.isfinite(sig) and sig > 0
    finally:
        rfd.rfd_taps_destroy(taps)
        rfd.rfd_plan_destroy(plan)
