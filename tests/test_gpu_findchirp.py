"""FINDCHIRP baseline (Eq. 1, one full-length inverse FFT per template)
against the FP64 oracle at every transform geometry: segments of at most
4096 samples (one pass, no column transform), column transforms of 2 to 256
points held in registers (2^13 ... 2^20 samples), and the LDS column
transform of 2^21 samples; template counts that leave a ragged last batch."""
import numpy as np
import pytest

import synth
from gpu_cases import compare_triggers, rho_matrix
from oracle import pipeline as orc

pytestmark = pytest.mark.gpu

FS, F_LOW = 2048.0, 30.0


def _case(n, count, seed):
    w = synth.Workload(f"fc{n}", 9, n, FS, F_LOW, count, 1, 0, "fp32", "nonspin")
    rng = np.random.default_rng(seed)
    psd = synth.psd_array(n, FS)
    s = synth.make_noise_spectrum(w, rng)
    params = [synth.WaveformParams(*m) for m in rng.uniform(1.2, 3.0, size=(count, 2))]
    H = synth.template_batch(w, params)
    amp = synth.workloads.optimal_snr_amplitude(H[0], w, 14.0)
    k = np.arange(n // 2 + 1)
    n0 = int(rng.integers(0, n))
    s = s + amp * H[0] * np.exp(-2j * np.pi * ((k * n0) % n) / n)
    data = synth.spectrum_to_time(s, n, FS)
    p = orc.prepare(psd, data, FS, F_LOW)
    want = np.array([np.abs(orc.findchirp_snr(p, H[j])) for j in range(count)])
    return psd, data, H, want, n0


def _run(rfd, n, count, threshold, window, seed=3):
    import torch
    psd, data, H, want, n0 = _case(n, count, seed)
    plan = rfd.rfd_plan_create(psd, F_LOW, FS, n)
    try:
        filt, _ = rfd.rfd_findchirp_prepare(plan, torch.from_numpy(H).to("cuda"))
        d = torch.from_numpy(data).to("cuda")
        cap = count * ((n + window - 1) // window)
        buf, m = rfd.findchirp_filter(plan, d, filt, threshold, window, cap)
        trig = rfd.triggers_to_numpy(buf, m)
        torch.cuda.synchronize()
    finally:
        rfd.rfd_plan_destroy(plan)
    return trig, want, n0


# (segment length, templates): batches hold 64 templates up to 2^19 samples,
# 256 MiB / (8 N) above, so the counts below end on a partial batch
FULL = [(1 << 10, 7), (1 << 11, 6), (1 << 12, 5), (1 << 13, 67), (1 << 14, 3), (1 << 15, 4), (1 << 16, 3),
        (1 << 17, 2)]


@pytest.mark.parametrize("n,count", FULL)
def test_full_series_matches_oracle(rfd, n, count):
    trig, want, _ = _run(rfd, n, count, 0.0, 1)
    rho = rho_matrix(trig, count, n)
    assert not np.isnan(rho).any(), "threshold 0 and window 1 must report every sample"
    err = np.max(np.abs(rho - want))
    print(f"\n[findchirp N={n}] {count} templates, max |drho| = {err:.3e}")
    assert err <= 1e-5


# larger segments: one peak per window of 4096 samples, every window compared
WINDOWED = [(1 << 19, 67), (1 << 20, 35), (1 << 21, 17), (1 << 22, 9)]


@pytest.mark.parametrize("n,count", WINDOWED)
def test_window_peaks_match_oracle(rfd, n, count):
    trig, want, n0 = _run(rfd, n, count, 0.0, 4096)
    ncmp, namb, dmax = compare_triggers(trig, want, 0.0, 4096, 1e-5)
    print(f"\n[findchirp N={n}] {count} templates: {ncmp} windows identical, {namb} ambiguous, "
          f"max |drho| {dmax:.2e}")
    assert ncmp >= count * (n // 4096) - namb
    assert dmax <= 1e-5


def test_threshold_keeps_only_loud_windows(rfd):
    """At theta = 6 only windows whose peak exceeds it are reported, each with
    the oracle's sample; the injection is among them."""
    n, count = 1 << 17, 6
    trig, want, n0 = _run(rfd, n, count, 6.0, 2048)
    ncmp, namb, dmax = compare_triggers(trig, want, 6.0, 2048, 1e-5)
    assert np.all(trig["rho"] > 6.0)
    hit = trig[(trig["tmpl"] == 0)]
    assert np.any(np.abs(hit["sample"].astype(np.int64) - n0) <= 2)
    print(f"\n[findchirp N={n}] theta=6: {len(trig)} triggers, {ncmp} windows identical, {namb} ambiguous")
