"""Pins for the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: a
brute-force sum, a closed form, a statistical law of Gaussian noise, an exact
identity between two routes, or hand-built cases.  They run on the CPU.
"""
import numpy as np
import pytest

import synth
from oracle import cluster, fir, pipeline, spectral, taps

RNG = np.random.default_rng(12345)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_data_transform_matches_defining_sum(n):
    fs = 4.0
    x = RNG.standard_normal(n)
    got = spectral.data_transform(x, fs)
    m = np.arange(n)
    want = np.array([np.sum(x * np.exp(-2j * np.pi * k * m / n)) for k in range(n // 2 + 1)]) / fs
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    assert np.allclose(spectral.dft_brute(x)[: n // 2 + 1] / fs, want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("n", [8, 32, 64])
def test_one_sided_inverse_matches_defining_sum(n):
    q = crandn(n // 2 + 1)
    got = spectral.one_sided_ifft(q, n)
    i = np.arange(n // 2 + 1)
    want = np.array([np.sum(q * np.exp(2j * np.pi * i * t / n)) for t in range(n)])
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_matched_filter_matches_double_sum():
    n, fs, f_low = 64, 64.0, 3.0
    s, h = crandn(n // 2 + 1), crandn(n // 2 + 1)
    psd = 1.0 + RNG.random(n // 2 + 1)
    w = spectral.psd_weights(psd, n, fs, f_low)
    i0, i1 = spectral.band_limits(n, fs, f_low)
    df = fs / n
    want = np.zeros(n, dtype=complex)
    for t in range(n):
        for i in range(i0, i1 + 1):
            want[t] += 4 * df * s[i] * np.conj(h[i]) / psd[i] * np.exp(2j * np.pi * i * t / n)
    got = spectral.matched_filter(s, h, w)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.allclose(spectral.matched_filter_at(s, h, w, [0, 5, 63]), want[[0, 5, 63]], atol=1e-12 * np.abs(want).max())
    assert w[0] == 0 and w[n // 2] == 0 and w[i0 - 1] == 0 and w[i0] > 0


def test_parseval_data_transform():
    n, fs = 1024, 256.0
    x = RNG.standard_normal(n)
    s = spectral.data_transform(x, fs)
    full = np.concatenate([s, np.conj(s[-2:0:-1])])
    assert abs(np.sum(x * x) - fs * fs / n * np.sum(np.abs(full) ** 2)) <= 1e-10 * np.sum(x * x)


# ------------------------------------------------------- matched filter laws

@pytest.fixture(scope="module")
def small():
    w = synth.get_workload("bns64s")
    bank = synth.make_bank(w)
    psd = synth.psd_array(w.n, w.fs)
    noise = synth.make_segment(w, bank, noise=True, inject=False)
    clean = synth.make_segment(w, bank, noise=False, inject=True)
    hr = synth.reference_waveform(w, bank.subbanks[0])
    H = synth.template_batch(w, bank.subbanks[0].params)
    return dict(w=w, bank=bank, psd=psd, noise=noise, clean=clean, hr=hr, H=H)


def test_noise_rho_squared_mean_two_and_exponential_tail(small):
    from scipy import stats
    w = small["w"]
    p = pipeline.prepare(small["psd"], small["noise"].data, w.fs, w.f_low)
    z = pipeline.findchirp_snr(p, small["hr"])
    r2 = np.abs(z) ** 2
    assert abs(r2.mean() - 2.0) < 0.03          # sd of the mean here is ~0.006
    dec = r2[::97]                              # decorrelated subsample
    assert stats.kstest(dec, stats.expon(scale=2.0).cdf).pvalue > 1e-3
    assert abs(np.mean(r2 > 6.0) - np.exp(-3.0)) < 0.01


def test_noise_free_injection_recovered_exactly(small):
    w, clean = small["w"], small["clean"]
    p = pipeline.prepare(small["psd"], clean.data, w.fs, w.f_low)
    h = small["H"][clean.inj_template]
    rho = np.abs(pipeline.findchirp_snr(p, h))
    assert int(np.argmax(rho)) == clean.inj_sample
    assert abs(rho[clean.inj_sample] - w.injection_snr) < 1e-9


# ----------------------------------------------------------------------- taps

def tiny_case(n=512, fs=256.0, f_low=20.0):
    psd = synth.psd_array(n, fs * 8)[: n // 2 + 1] * 0 + 1.0 + RNG.random(n // 2 + 1)
    w = spectral.psd_weights(psd, n, fs, f_low)
    i = np.arange(n // 2 + 1)
    hr = np.where(w > 0, (1 + i) ** (-7 / 6.0) * np.exp(-1j * 0.002 * i * i), 0)
    hj = np.where(w > 0, (1 + i) ** (-7 / 6.0) * np.exp(-1j * 0.0021 * i * i + 0.3j), 0)
    return n, w, hr, hj


def test_normal_equations_hold_for_direct_chi2_minimiser():
    n, w, hr, hj = tiny_case()
    T, k0, eps = 24, -12, 1e-6
    a = taps.ls_taps_direct(hj, hr, w, T, k0, eps)
    M = taps.gram(hr, w, T)
    b = taps.crosscorr(hj, hr, w, T, k0)
    lam = eps * np.real(M[0, 0])
    res = (M + lam * np.eye(T)) @ a - b
    assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(b)
    a2 = taps.ls_taps_normal(hj, hr, w, T, k0, eps)
    assert np.max(np.abs(a - a2)) <= 1e-8 * np.max(np.abs(a))


def test_chi2_quadratic_identity_for_any_taps():
    n, w, hr, hj = tiny_case()
    T, k0 = 16, -8
    R, u = taps.ratio_and_weight(hj, hr, w)
    M = taps.gram(hr, w, T)
    b = taps.crosscorr(hj, hr, w, T, k0)
    for _ in range(3):
        a = crandn(T) * 0.3
        direct = taps.chi2(hj, hr, w, a, k0, eps=0.0)
        quad = np.sum(u * np.abs(R) ** 2) - 2 * np.real(np.conj(a) @ b) + np.real(np.conj(a) @ M @ a)
        assert abs(direct - quad) <= 1e-10 * abs(direct)


def test_random_perturbations_never_lower_objective():
    n, w, hr, hj = tiny_case()
    T, k0, eps = 20, -10, 1e-6
    a = taps.ls_taps_normal(hj, hr, w, T, k0, eps)
    base = taps.chi2(hj, hr, w, a, k0, eps)
    for scale in (1e-2, 1e-4):
        for _ in range(10):
            assert taps.chi2(hj, hr, w, a + scale * crandn(T), k0, eps) >= base * (1 - 1e-12)


def test_time_shifted_target_gives_tap_at_the_shift():
    n, fs, f_low = 4096, 2048.0, 30.0
    psd = synth.psd_array(n, fs)
    w = spectral.psd_weights(psd, n, fs, f_low)
    hr = synth.taylorf2(synth.WaveformParams(1.4, 1.4), n, fs, f_low)
    T, k0, tau = 32, -16, 5
    i = np.arange(n // 2 + 1)
    hj = hr * np.exp(-2j * np.pi * ((i * tau) % n) / n)      # delayed by tau samples
    a = taps.ls_taps_normal(hj, hr, w, T, k0, 1e-6)
    assert int(np.argmax(np.abs(a))) == tau - k0
    R, u = taps.ratio_and_weight(hj, hr, w)
    assert taps.chi2(hj, hr, w, a, k0, 0.0) <= 1e-6 * np.sum(u * np.abs(R) ** 2)
    # the ratio filter of the reference series reproduces the shifted series
    s = crandn(n // 2 + 1)
    zr = spectral.matched_filter(s, hr, w)
    zj = fir.fir_direct(zr, np.conj(a), k0)
    assert np.linalg.norm(zj - np.roll(zr, -tau)) <= 1e-3 * np.linalg.norm(zr)


def test_full_length_taps_without_ridge_reproduce_findchirp():
    n, w, hr, hj = tiny_case(n=64, fs=64.0, f_low=4.0)
    s = crandn(n // 2 + 1)
    a = taps.ls_taps_direct(hj, hr, w, n, 0, eps=0.0)          # T = N circular taps
    zr = spectral.matched_filter(s, hr, w)
    zj = fir.fir_direct(zr, np.conj(a), 0)
    want = spectral.matched_filter(s, hj, w)
    assert np.max(np.abs(zj - want)) <= 1e-10 * np.max(np.abs(want))


def test_fir_equals_matched_filter_of_fitted_template():
    n, w, hr, hj = tiny_case()
    T, k0 = 16, -5
    s = crandn(n // 2 + 1)
    a = crandn(T)
    zr = spectral.matched_filter(s, hr, w)
    got = fir.fir_direct(zr, np.conj(a), k0)
    want = spectral.matched_filter(s, hr * taps.response(a, k0, n), w)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # direct double loop
    brute = np.array([sum(np.conj(a[k]) * zr[(t + k0 + k) % n] for k in range(T)) for t in range(n)])
    assert np.max(np.abs(brute - got)) <= 1e-12 * np.max(np.abs(got))
    assert np.allclose(fir.fir_at(zr, np.conj(a), k0, [0, 7, n - 1]), got[[0, 7, n - 1]], rtol=0,
                       atol=1e-12 * np.abs(got).max())


def test_fitted_norm_two_forms_agree():
    n, w, hr, hj = tiny_case()
    T, k0 = 24, -12
    M = taps.gram(hr, w, T)
    for _ in range(3):
        a = crandn(T)
        f = taps.fitted_sigma_sq_freq(a, hr, w, k0)
        l = taps.fitted_sigma_sq_lag(a, M)
        assert abs(f - l) <= 1e-11 * f


def test_gram_is_hermitian_toeplitz_with_g0_on_diagonal():
    n, w, hr, hj = tiny_case()
    M = taps.gram(hr, w, 12)
    assert np.allclose(M, M.conj().T, atol=1e-14 * abs(M[0, 0]))
    assert np.allclose(np.diag(M), np.sum(w * np.abs(hr) ** 2))
    assert np.allclose(M[3, 1], M[5, 3])


def test_tukey_matches_scipy():
    from scipy.signal.windows import tukey
    for T in (5, 64, 251):
        assert np.allclose(taps.tukey(T, 0.25), tukey(T, 0.25, sym=True), atol=1e-15)


def test_window_taps_closed_form_for_shift():
    n, w, hr, _ = tiny_case()
    T, k0, tau = 40, -20, 3
    i = np.arange(n // 2 + 1)
    hj = hr * np.exp(-2j * np.pi * ((i * tau) % n) / n)
    a = taps.window_taps(hj, hr, w, T, k0)
    R, u = taps.ratio_and_weight(hj, hr, w)
    sel = np.nonzero(u > 0)[0]
    i0, m = int(sel[0]), len(sel)
    assert np.all(np.diff(sel) == 1)
    want = np.empty(T, dtype=complex)
    for l in range(T):
        d = k0 + l - tau
        r = np.exp(2j * np.pi * d / n)
        want[l] = m if d % n == 0 else r ** i0 * (1 - r ** m) / (1 - r)
    want = taps.tukey(T, 0.25) * want / n
    assert np.max(np.abs(a - want)) <= 1e-12


def test_ratio_filter_noise_normalisation(small):
    w = small["w"]
    p = pipeline.prepare(small["psd"], small["noise"].data, w.fs, w.f_low)
    sb = small["bank"].subbanks[0]
    ref = pipeline.dechirp(p, small["hr"])
    tt = pipeline.make_taps(p, small["H"][3], small["hr"], sb.taps, sb.k0)
    z = pipeline.ratio_snr(ref, tt)
    assert abs(np.mean(np.abs(z) ** 2) - 2.0) < 0.04


def test_direct_and_normal_solvers_agree_at_workload_size(small):
    w = small["w"]
    p = pipeline.prepare(small["psd"], small["noise"].data, w.fs, w.f_low)
    sb = small["bank"].subbanks[0]
    a1 = pipeline.make_taps(p, small["H"][0], small["hr"], sb.taps, sb.k0, solver="normal").a
    a2 = pipeline.make_taps(p, small["H"][0], small["hr"], sb.taps, sb.k0, solver="direct").a
    assert np.max(np.abs(a1 - a2)) <= 1e-8 * np.max(np.abs(a1))


# -------------------------------------------------------------- clustering

def test_cluster_hand_built_ties_and_strict_threshold():
    rho = np.array([1.0, 5.0, 5.0, 2.0, 6.0, 6.0, 0.0, 6.0])
    assert cluster.cluster(rho, 0.0, 4) == [(1, 5.0), (4, 6.0)]
    assert cluster.cluster(rho, 5.0, 4) == [(4, 6.0)]          # 5.0 is not > 5.0
    assert cluster.cluster(rho, 6.0, 4) == []
    assert cluster.cluster(rho, 0.0, 3) == [(1, 5.0), (4, 6.0), (7, 6.0)]
    assert cluster.cluster(rho, 0.5, 1) == [(i, v) for i, v in enumerate(rho) if v > 0.5]


def test_cluster_matches_brute_force_loop():
    for _ in range(20):
        n = int(RNG.integers(1, 300))
        rho = np.round(RNG.random(n) * 8, 1)         # many exact ties
        W = int(RNG.integers(1, 50))
        th = float(RNG.random() * 8)
        assert cluster.cluster(rho, th, W) == cluster.cluster_brute(rho, th, W)


def test_window_ambiguity_cases():
    rho = np.array([6.0000001, 1, 1, 1, 7.0, 6.9999995, 0, 0, 3.0, 2.9999999, 0, 0])
    flags = cluster.window_ambiguity(rho, 6.0, 4, 1e-5)
    assert flags.tolist() == [True, True, False]


def test_zero_lag_match_and_tap_selection():
    """The zero-lag match equals the overlap series of pipeline.match at lag 0,
    equals |a^H b| / (sigma_j sqrt(a^H M a)) in the tap domain, and the
    selection is the first ladder entry reaching the target."""
    import synth
    from oracle import pipeline, spectral, taps as tp
    n, fs, f_low = 8192, 2048.0, 30.0
    w = spectral.psd_weights(synth.psd_array(n, fs), n, fs, f_low)
    h_r = synth.taylorf2(synth.WaveformParams(6.0, 5.0), n, fs, f_low)
    h_j = synth.taylorf2(synth.WaveformParams(6.4, 4.7), n, fs, f_low)
    T, k0 = 48, -24
    M = tp.gram(h_r, w, T)
    a = tp.ls_taps_normal(h_j, h_r, w, T, k0, M=M)
    m = tp.zero_lag_match(h_j, h_r, w, a, k0)
    h_fit = h_r * tp.response(a, k0, n)
    series = spectral.matched_filter(h_j, h_fit, w)
    want = abs(series[0]) / np.sqrt(spectral.sigma_sq(h_j, w) * spectral.sigma_sq(h_fit, w))
    assert abs(m - want) <= 1e-12
    b = tp.crosscorr(h_j, h_r, w, T, k0)
    alt = abs(np.conj(a) @ b) / np.sqrt(spectral.sigma_sq(h_j, w) * np.real(np.conj(a) @ M @ a))
    assert abs(m - alt) <= 1e-10
    # the time-maximised match bounds it from above
    assert m <= pipeline.match(pipeline.Prepared(n, fs, f_low, w, None), h_j, h_r,
                               pipeline.TemplateTaps(a, k0, 1.0)) + 1e-12
    ladder = [8, 16, 32, 64, 128, 256]
    ms = []
    for TT in ladder:
        aa = tp.ls_taps_normal(h_j, h_r, w, TT, -(TT // 2))
        ms.append(tp.zero_lag_match(h_j, h_r, w, aa, -(TT // 2)))
    for target in (0.5, 0.9, 0.99, 0.999, 2.0):
        T_sel, m_sel = tp.select_taps(h_j, h_r, w, target, ladder)
        first = next((TT for TT, mm in zip(ladder, ms) if mm >= target), ladder[-1])
        assert T_sel == first and abs(m_sel - ms[ladder.index(T_sel)]) <= 1e-14


@pytest.mark.parametrize("T,k0", [(8, -4), (33, 5), (16, -40), (2048, -1024)])
def test_response_fft_equals_the_defining_sum(T, k0):
    """response_fft (one FFT of the taps at their lags) equals response, the
    defining sum sum_k a_k exp(-2 pi i i (k0 + k) / N) written as a matrix
    product, bin by bin."""
    from oracle import taps as tp
    n = 4096
    rng = np.random.default_rng(T)
    a = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    want = tp.response(a, k0, n)
    got = tp.response_fft(a, k0, n)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


# ------------------------------------------------------- lag centring

@pytest.mark.parametrize("n", [16, 64])
def test_peak_lag_matches_brute_force_correlation(n):
    """peak_lag is the argmax over every lag of |sum_i u_i R_i e^{+2 pi i i l/N}|^2,
    written as a double loop, mapped into (-N/2, N/2]."""
    rng = np.random.default_rng(n)
    nb = n // 2 + 1
    h_r = rng.standard_normal(nb) + 1j * rng.standard_normal(nb)
    h_j = rng.standard_normal(nb) + 1j * rng.standard_normal(nb)
    w = rng.random(nb)
    w[0] = w[-1] = 0.0
    best, bl = -1.0, None
    for lag in range(n):
        acc = 0j
        for i in range(nb):
            u = w[i] * abs(h_r[i]) ** 2
            if u > 0:
                acc += u * (h_j[i] / h_r[i]) * np.exp(2j * np.pi * i * lag / n)
        p = acc.real ** 2 + acc.imag ** 2
        if p > best * (1 + 1e-12):
            best, bl = p, lag
    want = bl if bl <= n // 2 else bl - n
    assert taps.peak_lag(h_j, h_r, w) == want
    assert taps.centred_k0(h_j, h_r, w, 9) == want - 4


@pytest.mark.parametrize("tau", [-300, -37, 0, 5, 700])
def test_peak_lag_of_a_delayed_reference_is_the_delay(tau):
    """A target equal to the reference delayed by tau samples has R = e^{-2 pi i i tau/N},
    so every term of b[tau] is real and positive: the peak sits at lag tau
    exactly, and the centred taps (T = 32) then reproduce the target (match 1)
    while lags centred on 0 miss it when |tau| > T/2."""
    n, fs, f_low = 4096, 2048.0, 30.0
    w = spectral.psd_weights(synth.psd_array(n, fs), n, fs, f_low)
    hr = synth.taylorf2(synth.WaveformParams(1.4, 1.4), n, fs, f_low)
    i = np.arange(n // 2 + 1)
    hj = hr * np.exp(-2j * np.pi * ((i * tau) % n) / n)
    assert taps.peak_lag(hj, hr, w) == tau
    T = 32
    k0c = taps.centred_k0(hj, hr, w, T)
    a = taps.ls_taps_normal(hj, hr, w, T, k0c, 1e-6)
    assert taps.zero_lag_match(hj, hr, w, a, k0c) >= 1 - 1e-6
    if abs(tau) > T // 2:
        a0 = taps.ls_taps_normal(hj, hr, w, T, -(T // 2), 1e-6)
        assert taps.zero_lag_match(hj, hr, w, a0, -(T // 2)) < 0.9
    T_sel, m_sel = taps.select_taps(hj, hr, w, 0.999, [8, 16, 32], 1e-6, centre=True)
    assert T_sel == 8 and m_sel >= 0.999


@pytest.mark.parametrize("shift", [-5, 3, 17])
def test_shifted_window_grid_matches_brute_force(shift):
    """triggers(..., shift=d): windows on the filter index m = n + d. A loop
    over every sample n assigns it to window ((n + d) mod N) // W, keeps the
    largest rho^2 (lowest m on exact ties) and reports n; same list."""
    n, W, thr = 64, 16, 1.0
    rng = np.random.default_rng(7 + shift)
    z = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 1.3
    z[10] = z[11] = 3.0          # an exact tie in one window
    got = sorted(pipeline.triggers(z, thr, W, shift))
    best = {}
    for s in range(n):
        m = (s + shift) % n
        q = m // W
        r2 = abs(z[s]) ** 2
        if q not in best or r2 > best[q][0] or (r2 == best[q][0] and m < best[q][1]):
            best[q] = (r2, m, s)
    want = sorted((s, float(np.sqrt(r2))) for r2, m, s in best.values() if np.sqrt(r2) > thr)
    assert [g[0] for g in got] == [x[0] for x in want]
    assert np.allclose([g[1] for g in got], [x[1] for x in want], rtol=1e-15)
    assert pipeline.triggers(z, thr, W, 0) == cluster.cluster(np.abs(z), thr, W)
