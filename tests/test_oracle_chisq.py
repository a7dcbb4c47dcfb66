"""Pins for the ratio-filtered chi^2 oracle (oracle/chisq.py, Sec. VI.C):
the band split, the band identity of Eq. 3 (FIR of the reference's band
series = band matched filter of the fitted template), the shares in two
independent forms, zero chi^2 on a noise-free fitted-template signal, the
noise mean 2 (p - 1), and the statistic by explicit loops."""
import numpy as np
import pytest

import synth
from oracle import chisq as ocq
from oracle import fir, pipeline, spectral
from oracle import taps as otaps

N, FS, F_LOW, T = 8192, 2048.0, 30.0, 64
K0 = -(T // 2)
P = 8


@pytest.fixture(scope="module")
def setup():
    w_ = synth.Workload("chisq-pin", 9, N, FS, F_LOW, 0, 1, T, "fp32", "nonspin")
    psd = synth.psd_array(N, FS)
    w = spectral.psd_weights(psd, N, FS, F_LOW)
    i_low, i_high = spectral.band_limits(N, FS, F_LOW)
    h_ref = synth.taylorf2(synth.WaveformParams(6.0, 5.0), N, FS, F_LOW)
    h_j = synth.taylorf2(synth.WaveformParams(6.3, 4.8), N, FS, F_LOW)
    rng = np.random.default_rng(11)
    s_noise = synth.make_noise_spectrum(w_, rng)
    edges = ocq.band_edges(h_ref, w, i_low, i_high, P)
    M = otaps.gram(h_ref, w, T)
    a = otaps.ls_taps_normal(h_j, h_ref, w, T, K0, M=M)
    return dict(w=w, i_low=i_low, i_high=i_high, h_ref=h_ref, h_j=h_j, s_noise=s_noise, edges=edges, M=M, a=a)


def test_band_edges_split_the_reference_power(setup):
    c = setup
    e = c["edges"]
    assert e[0] == c["i_low"] and e[-1] == c["i_high"] + 1 and np.all(np.diff(e) >= 1)
    u = c["w"] * np.abs(c["h_ref"]) ** 2
    total = u[c["i_low"]:c["i_high"] + 1].sum()
    # brute force: walk the bins with a running sum
    acc, want, b = 0.0, [c["i_low"]], 1
    for i in range(c["i_low"], c["i_high"] + 1):
        while b < P and acc >= (total * b) / P:
            want.append(i)
            b += 1
        acc += u[i]
    want.append(c["i_high"] + 1)
    assert np.array_equal(e, want)
    shares = np.array([u[e[k]:e[k + 1]].sum() for k in range(P)]) / total
    assert np.all(np.abs(shares - 1.0 / P) <= u.max() / total + 1e-12)


def test_band_identity_of_eq3(setup):
    """FIR of the reference's band series with conj(a)/sigma_fit equals the band
    matched filter of the fitted template, band by band; the bands sum to z."""
    c = setup
    stilde = c["s_noise"]
    zr = ocq.reference_band_series(stilde, c["h_ref"], c["w"], c["edges"])
    sig_ref = np.sqrt(spectral.sigma_sq(c["h_ref"], c["w"]))
    full_ref = spectral.matched_filter(stilde, c["h_ref"], c["w"]) / sig_ref
    np.testing.assert_allclose(zr.sum(axis=0), full_ref, atol=1e-12 * np.abs(full_ref).max())
    zb = ocq.fitted_band_snr(stilde, c["h_ref"], c["w"], c["a"], K0, c["edges"])
    sig_fit = np.sqrt(otaps.fitted_sigma_sq_lag(c["a"], c["M"]))
    for b in range(P):
        via_fir = fir.fir_direct(zr[b] * sig_ref, np.conj(c["a"]), K0) / sig_fit
        np.testing.assert_allclose(via_fir, zb[b], atol=1e-10 * np.abs(zb[b]).max())
    ref = pipeline.Reference(c["h_ref"], sig_ref, full_ref * sig_ref)
    z = pipeline.ratio_snr(ref, pipeline.TemplateTaps(c["a"], K0, sig_fit))
    np.testing.assert_allclose(zb.sum(axis=0), z, atol=1e-10 * np.abs(z).max())


def test_shares_two_ways(setup):
    """f_b from frequency sums equals a^H M_b a / a^H M a with M_b the Toeplitz
    Gram of the band-masked weight."""
    c = setup
    f = ocq.band_fractions(c["h_ref"], c["w"], c["a"], K0, c["edges"])
    assert abs(f.sum() - 1.0) <= 1e-12 and np.all(f > 0)
    den = np.real(np.conj(c["a"]) @ c["M"] @ c["a"])
    for b in range(P):
        Mb = otaps.gram(c["h_ref"], c["w"] * ocq.band_mask(c["w"].size, c["edges"], b), T)
        num = np.real(np.conj(c["a"]) @ Mb @ c["a"])
        assert abs(num / den - f[b]) <= 1e-10


def test_noise_free_fitted_signal_has_zero_chisq(setup):
    c = setup
    n0 = 3001
    A = otaps.response(c["a"], K0, N)
    k = np.arange(N // 2 + 1)
    h_fit = c["h_ref"] * A
    stilde = 7.0 * h_fit * np.exp(-2j * np.pi * ((k * n0) % N) / N)
    zb = ocq.fitted_band_snr(stilde, c["h_ref"], c["w"], c["a"], K0, c["edges"])
    f = ocq.band_fractions(c["h_ref"], c["w"], c["a"], K0, c["edges"])
    x = ocq.chisq(zb[:, n0:n0 + 1], f)[0]
    z = zb[:, n0].sum()
    sig_fit = np.sqrt(spectral.sigma_sq(h_fit, c["w"]))
    assert abs(abs(z) - 7.0 * sig_fit) <= 1e-9 * 7.0 * sig_fit
    assert x <= 1e-18 * abs(z) ** 2


def test_noise_mean_is_two_p_minus_one(setup):
    c = setup
    zb = ocq.fitted_band_snr(c["s_noise"], c["h_ref"], c["w"], c["a"], K0, c["edges"])
    f = ocq.band_fractions(c["h_ref"], c["w"], c["a"], K0, c["edges"])
    x = ocq.chisq(zb, f)
    # 8192 samples, correlated over a few taps: 6% is several standard errors
    assert abs(x.mean() / (2 * (P - 1)) - 1.0) <= 0.06
    rho2 = np.abs(zb.sum(axis=0)) ** 2
    assert abs(rho2.mean() / 2.0 - 1.0) <= 0.06


def test_statistic_by_loops():
    rng = np.random.default_rng(5)
    p, n = 5, 7
    zb = rng.standard_normal((p, n)) + 1j * rng.standard_normal((p, n))
    f = rng.uniform(0.1, 1.0, size=p)
    f /= f.sum()
    got = ocq.chisq(zb, f)
    for t in range(n):
        z = sum(zb[b, t] for b in range(p))
        want = sum(abs(zb[b, t] - f[b] * z) ** 2 / f[b] for b in range(p))
        assert abs(got[t] - want) <= 1e-12 * want
    eq = np.full(p, 1.0 / p)
    z = zb.sum(axis=0)
    np.testing.assert_allclose(ocq.chisq(zb, eq), p * np.sum(np.abs(zb - z / p) ** 2, axis=0), rtol=1e-12)
