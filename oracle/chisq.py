"""Ratio-filtered chi^2 signal-consistency test (Sec. VI.C), FP64.

Test infrastructure only (see package header).

Sec. VI.C describes the time-frequency chi^2 test: the analysis band is split
into frequency bands, the SNR accumulated in each band is compared with the
share the template predicts, and, with ratio filtering, a target's band SNRs
come from the band SNR series of its reference passed through the target's
taps.  Readings (the section gives no formulas):

  * Bands: p contiguous bin ranges of the analysis band, each holding 1/p of
    the reference's power sum_i u_i, u_i = w_i |h_ref(f_i)|^2 (the classic
    equal-power split, taken on the reference so that its band series serve
    every target).  Edge b (0 < b < p) is the first bin i with
    sum_{i_low <= i' < i} u_i' >= (total * b) / p (sequential FP64 sums),
    edge 0 = i_low, edge p = i_high + 1.
  * Band SNR of target j: the matched filter (Eq. 1) of the fitted template
    h_fit = h_ref * A_j (A_j the taps' response) restricted to band b,
    normalised by sigma_fit:  z_b(t) = (s | h_fit)_b(t) / sigma_fit.
    By Eq. 3 applied band by band this is the FIR of the reference's band
    series, which is how the GPU computes it.
  * Predicted shares: f_b = (h_fit|h_fit)_b / (h_fit|h_fit), the fitted
    template's own power split over the reference's bands.
  * Statistic: chi^2(t) = sum_b |z_b(t) - f_b z(t)|^2 / f_b with
    z = sum_b z_b; it is p sum_b |z_b - z/p|^2 when every f_b = 1/p, and its
    mean in Gaussian noise is 2 (p - 1) (complex SNRs).
"""
import numpy as np

from . import spectral
from . import taps as taps_mod


def band_edges(h_ref, w, i_low, i_high, p):
    """Bin edges e_0 < e_1 < ... < e_p of the equal-reference-power split."""
    hr = np.asarray(h_ref)[i_low:i_high + 1]
    u = w[i_low:i_high + 1] * (hr.real ** 2 + hr.imag ** 2)
    prefix = np.concatenate([[0.0], np.cumsum(u)])     # prefix[k] = sum of the first k
    total = prefix[-1]
    edges = [i_low]
    for b in range(1, p):
        thr = (total * b) / p
        edges.append(i_low + int(np.searchsorted(prefix, thr, side="left")))
    edges.append(i_high + 1)
    edges = np.array(edges, dtype=np.int64)
    if np.any(np.diff(edges) < 1):
        raise ValueError("band split produced an empty band")
    return edges


def band_mask(nb, edges, b):
    m = np.zeros(nb, dtype=np.float64)
    m[edges[b]:edges[b + 1]] = 1.0
    return m


def reference_band_series(stilde, h_ref, w, edges):
    """[p, N] band series of the reference, normalised by sigma_ref:
    zhat_b[n] = sum_{i in band b} w_i s_i conj(h_ref,i) e^{+2 pi i i n/N} / sigma_ref."""
    sig = np.sqrt(spectral.sigma_sq(h_ref, w))
    p = len(edges) - 1
    return np.stack([spectral.matched_filter(stilde, h_ref, w * band_mask(stilde.size, edges, b)) / sig
                     for b in range(p)])


def fitted_band_snr(stilde, h_ref, w, a, k0, edges):
    """[p, N] band SNRs of the fitted template h_fit = h_ref A, by the
    frequency-domain definition, normalised by sigma_fit."""
    n = 2 * (stilde.size - 1)
    h_fit = h_ref * taps_mod.response(a, k0, n)
    sig_fit = np.sqrt(spectral.sigma_sq(h_fit, w))
    p = len(edges) - 1
    return np.stack([spectral.matched_filter(stilde, h_fit, w * band_mask(stilde.size, edges, b)) / sig_fit
                     for b in range(p)])


def band_fractions(h_ref, w, a, k0, edges):
    """f_b = (h_fit|h_fit)_b / (h_fit|h_fit), frequency-domain sums."""
    n = 2 * (np.asarray(h_ref).size - 1)
    pw = w * np.abs(h_ref * taps_mod.response(a, k0, n)) ** 2
    parts = np.array([np.sum(pw[edges[b]:edges[b + 1]]) for b in range(len(edges) - 1)])
    return parts / np.sum(pw)


def chisq(zb, f):
    """chi^2 = sum_b |z_b - f_b z|^2 / f_b with z = sum_b z_b; zb [p, ...]."""
    z = np.sum(zb, axis=0)
    f = np.asarray(f, dtype=np.float64).reshape((-1,) + (1,) * (zb.ndim - 1))
    return np.sum(np.abs(zb - f * z) ** 2 / f, axis=0)
