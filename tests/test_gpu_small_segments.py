"""The shortest segments (2^10 ... 2^12 samples), where a workgroup's Hankel
window, an overlap-save block and the tap span all wrap around the whole
segment: every FIR form against the FP64 oracle in validation mode, and
trigger identity with a single window covering the segment."""
import numpy as np
import pytest

import synth
from gpu_cases import SB, Case, compare_triggers, fir_tolerance, gpu_search, oracle_case, rho_matrix

pytestmark = pytest.mark.gpu

FS, F_LOW = 2048.0, 30.0
FORMS = ["fp32", "bf16x3", "fp16x3", "ols32"]


def _case(n):
    w = synth.Workload(f"short{n}", 9, n, FS, F_LOW, 0, 1, 0, "fp32", "nonspin")
    rng = np.random.default_rng(n)
    psd = synth.psd_array(n, FS)
    s = synth.make_noise_spectrum(w, rng)
    h_ref = synth.taylorf2(synth.WaveformParams(3.0, 2.5), n, FS, F_LOW)
    subbanks = []
    for T, k0, count in [(16, -8, 3), (300, -150, 5)]:
        params = [synth.WaveformParams(*m) for m in rng.uniform(2.4, 3.2, size=(count, 2))]
        subbanks.append(SB(0, T, k0, synth.template_batch(w, params)))
    h = subbanks[1].H[2]
    amp = synth.workloads.optimal_snr_amplitude(h, w, 16.0)
    k = np.arange(n // 2 + 1)
    n0 = n // 3
    s = s + amp * h * np.exp(-2j * np.pi * ((k * n0) % n) / n)
    return Case(f"short{n}", n, FS, F_LOW, psd, synth.spectrum_to_time(s, n, FS), {0: h_ref}, subbanks)


@pytest.fixture(scope="module", params=[1 << 10, 1 << 11, 1 << 12])
def short(rfd, request):
    case = _case(request.param)
    oracle_case(case)
    s = gpu_search(case)
    yield case, s
    s.close()


@pytest.mark.parametrize("precision", FORMS)
def test_short_segment_series(rfd, short, precision):
    case, s = short
    buf, n = s.filter(precision, 0.0, 1, case.n_templates * case.n)
    rho = rho_matrix(rfd.triggers_to_numpy(buf, n), case.n_templates, case.n)
    assert not np.isnan(rho).any()
    want = np.abs(case.oracle["z"])
    err = np.max(np.abs(rho - want), axis=1)
    tol = fir_tolerance(case, precision, 1e-5 if precision in ("fp32", "ols32") else 1e-3)
    print(f"\n[N={case.n}] {precision}: max |drho| = {err.max():.3e}, worst err/tol = {np.max(err / tol):.2f}")
    assert (err <= tol).all()


@pytest.mark.parametrize("precision", FORMS)
def test_short_segment_one_window(rfd, short, precision):
    """W = N: one peak per template over the whole segment."""
    case, s = short
    buf, n = s.filter(precision, 3.0, case.n, 64)
    trig = rfd.triggers_to_numpy(buf, n)
    tol = fir_tolerance(case, precision, 1e-5 if precision in ("fp32", "ols32") else 1e-3)
    ncmp, namb, dmax = compare_triggers(trig, np.abs(case.oracle["z"]), 3.0, case.n, tol)
    assert ncmp + namb == case.n_templates
    assert len(trig) >= 1
