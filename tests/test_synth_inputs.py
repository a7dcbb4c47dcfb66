"""Sanity of the seeded input generator (shapes, determinism, noise level)."""
import numpy as np

import synth


def test_noise_level_matches_one_sided_psd():
    w = synth.get_workload("bns64s")
    s = synth.make_noise_spectrum(w)
    psd = synth.psd_array(w.n, w.fs)
    i0, i1 = synth.workloads.band(w)
    ratio = np.abs(s[i0:i1 + 1]) ** 2 * 2 * w.df / psd[i0:i1 + 1]
    assert abs(ratio.mean() - 1.0) < 0.02
    assert np.all(s[:i0] == 0) and s[-1] == 0


def test_time_series_round_trip():
    w = synth.get_workload("bns64s")
    seg = synth.make_segment(w, synth.make_bank(w))
    back = np.fft.rfft(seg.data) / w.fs
    assert seg.data.dtype == np.float64 and seg.data.size == w.n
    assert w.n // 4 <= seg.inj_sample < 3 * w.n // 4


def test_determinism_and_shapes():
    w = synth.get_workload("spin256s")
    b1, b2 = synth.make_bank(w), synth.make_bank(w)
    assert b1.n_templates == 4096 and b1.params(17) == b2.params(17)
    w3 = synth.get_workload("tidal256s")
    b3 = synth.make_bank(w3)
    assert len(b3.subbanks) == 64
    assert all(256 <= sb.size <= 2048 and 32 <= sb.taps <= 1024 for sb in b3.subbanks)
    w4 = synth.get_workload("ecc512s")
    b4 = synth.make_bank(w4)
    assert b4.n_templates == 16384 and all(sb.size == 512 and sb.taps == 1024 for sb in b4.subbanks)


def test_taylorf2_support_and_isco():
    p = synth.WaveformParams(3.0, 3.0)
    n, fs = 1 << 14, 2048.0
    h = synth.taylorf2(p, n, fs, 20.0)
    f = np.arange(n // 2 + 1) * fs / n
    nz = f[np.abs(h) > 0]
    assert nz.min() >= 20.0 and nz.max() <= synth.f_isco(6.0) < fs / 2
    assert abs(synth.f_isco(1.0) - 4397.0) < 1.0
    k = np.nonzero(np.abs(h) > 0)[0]
    assert np.allclose(np.abs(h[k]), f[k] ** (-7 / 6))


def test_device_batches_equal_host_waveforms():
    """synth.device evaluates the same TaylorF2 formulas with torch tensors
    (here on the CPU): same band edges, values equal to FP64 rounding of the
    phase (which reaches ~1e6 rad for the lightest eccentric systems)."""
    torch = __import__("pytest").importorskip("torch")
    from synth.device import template_batch_device
    for name, tol in [("ecc512s", 5e-9), ("tidal256s", 1e-9), ("spin256s", 1e-9), ("surr512s", 1e-9),
                      ("bns64s", 1e-9)]:
        w = synth.get_workload(name)
        bank = synth.make_bank(w)
        ps = [bank.params(j) for j in range(0, bank.n_templates, max(1, bank.n_templates // 5))][:5]
        host = synth.template_batch(w, ps)
        dev = template_batch_device(w, ps, "cpu").numpy()
        assert np.array_equal(dev == 0, host == 0), name
        assert np.max(np.abs(dev - host)) <= tol * np.max(np.abs(host)), name
