"""Sec. V.A: ratio FIR taps by weighted ridge least squares; Sec. VI.B norms.

Test infrastructure only (see package header).

Notation (Sec. V.A, with the readings below):
  R_i   = h_j(f_i) / h_ref(f_i)           the ratio of Eq. 2
  t_k   = (k0 + k) / fs, k = 0..T-1        tap times at the data rate
  A_i   = sum_k a_k exp(-2 pi i f_i t_k)  the taps' frequency response
  chi^2 = sum_i u_i |R_i - A_i|^2 + lam sum_k |a_k|^2

Readings (the paper leaves these open):
  * weight: u_i = w_i |h_ref(f_i)|^2 with w_i = 4 df / S_n, i.e. the
    reference's signal power over the noise PSD; bins with u_i = 0 (out of
    band, or where h_ref vanishes) drop out, so R is never divided by zero;
  * frequency grid: every in-band bin f_i = i df of the analysis segment;
  * tap times: k0 = -floor(T/2) unless given; with per-template lag
    centring, k0_j = (lag of the largest |b_j[l]| over every lag) -
    floor(T/2), b_j the full weighted cross-correlation of target and
    reference (the normal equations' right-hand side at every lag);
  * ridge: lam = eps * g[0] with g[0] = sum_i u_i and eps = 1e-4 by default.
    The paper adds the ridge so that taps stay bounded where the weight is
    small and numerical error does not accumulate in band; eps sets that
    bound.  With eps = 1e-6 the normalised taps reach ||c||_2 ~ 50-95 on
    the BNS workloads, so white rounding noise in the reference series is
    amplified ~100x; eps = 1e-4 keeps ||c||_2 ~ 5-10 for a match change
    below 0.01.  eps is a parameter everywhere;
  * the FIR applies conj(a) as a correlation (Eq. 3 after substituting
    Eq. 2 into Eq. 1, which correlates with the conjugate template);
  * windowed variant: the exact inverse transform of R, truncated to the T
    lags and tapered by a Tukey(0.25) window.
"""
import numpy as np

from .spectral import one_sided_ifft

DEFAULT_RIDGE_EPS = 1e-4


def phase_frac(i, m, n):
    """((i * m) mod N) / N computed exactly in integers."""
    return ((np.asarray(i, dtype=np.int64) * np.int64(m)) % n) / n


def ratio_and_weight(h_j, h_r, w):
    """(R, u): the ratio of Eq. 2 and the chi^2 weight, on the rfft grid."""
    u = w * np.abs(h_r) ** 2
    R = np.zeros_like(h_j)
    nz = u > 0
    R[nz] = h_j[nz] / h_r[nz]
    return R, u


def design_matrix(bins, T, k0, n):
    """E[i, k] = exp(-2 pi i f_i t_k) = exp(-2 pi i bin_i (k0 + k) / N)."""
    lag = (k0 + np.arange(T, dtype=np.int64)) % n
    ph = (np.outer(np.asarray(bins, dtype=np.int64), lag) % n) / n
    return np.exp(-2j * np.pi * ph)


def ls_taps_direct(h_j, h_r, w, T, k0, eps=DEFAULT_RIDGE_EPS):
    """Minimise chi^2 + ridge (Sec. V.A) as a stacked least-squares problem.

        [ sqrt(u) E ]       [ sqrt(u) R ]
        [ sqrt(lam) I ] a = [     0     ]

    The defining form; O(n_band T^2), so for tiny and moderate sizes.
    """
    n = 2 * (h_j.size - 1)
    R, u = ratio_and_weight(h_j, h_r, w)
    bins = np.nonzero(u > 0)[0]
    lam = eps * float(np.sum(u))
    E = design_matrix(bins, T, k0, n)
    su = np.sqrt(u[bins])
    A = np.vstack([su[:, None] * E, np.sqrt(lam) * np.eye(T)])
    y = np.concatenate([su * R[bins], np.zeros(T, dtype=np.complex128)])
    a, *_ = np.linalg.lstsq(A, y, rcond=None)
    return a


def autocorr(h_r, w, lags):
    """g[m] = sum_i u_i exp(+2 pi i i m / N): the reference autocorrelation
    (h_ref|h_ref)(t_m) of Sec. VI.B, at integer lags m (any sign)."""
    n = 2 * (h_r.size - 1)
    full = one_sided_ifft(w * np.abs(h_r) ** 2, n)
    return full[np.asarray(lags, dtype=np.int64) % n]


def crosscorr(h_j, h_r, w, T, k0):
    """b[l] = sum_i u_i R_i exp(+2 pi i f_i t_l), l = 0..T-1 (normal-equation
    right-hand side; equals sum_i w_i h_j conj(h_ref) exp(...))."""
    n = 2 * (h_j.size - 1)
    R, u = ratio_and_weight(h_j, h_r, w)
    full = one_sided_ifft(u * R, n)
    return full[(k0 + np.arange(T, dtype=np.int64)) % n]


def peak_lag(h_j, h_r, w):
    """Lag l in (-N/2, N/2] of the largest |b[l]|^2 = Re^2 + Im^2 over all N
    lags of b[l] = sum_i u_i R_i exp(+2 pi i i l / N), the weighted
    cross-correlation of target and reference (the right-hand side of the
    normal equations at every lag).  On exact ties the lowest index
    0..N-1 wins."""
    n = 2 * (h_j.size - 1)
    R, u = ratio_and_weight(h_j, h_r, w)
    full = one_sided_ifft(u * R, n)
    i = int(np.argmax(full.real * full.real + full.imag * full.imag))
    return i if i <= n // 2 else i - n


def centred_k0(h_j, h_r, w, T):
    """Per-template lag centring (Sec. V.A's tap tuning, with the tap window
    placed per template): the T lags centred on the peak of |b|."""
    return peak_lag(h_j, h_r, w) - T // 2


def toeplitz_gram(g_pos_neg, T):
    """M[l, k] = g[l - k] from g sampled at lags -(T-1)..(T-1)."""
    idx = np.arange(T)[:, None] - np.arange(T)[None, :] + (T - 1)
    return g_pos_neg[idx]


def gram(h_r, w, T):
    """The normal-equation matrix M (T x T, Hermitian Toeplitz)."""
    g = autocorr(h_r, w, np.arange(-(T - 1), T))
    return toeplitz_gram(g, T)


def ls_taps_normal(h_j, h_r, w, T, k0, eps=DEFAULT_RIDGE_EPS, M=None):
    """Same minimiser through the normal equations (M + lam I) a = b.

    d chi^2 / d conj(a_l) = 0 gives sum_k M[l,k] a_k + lam a_l = b[l] with
    M[l,k] = sum_i u_i exp(2 pi i f_i (t_l - t_k)) = g[l - k].
    """
    if M is None:
        M = gram(h_r, w, T)
    lam = eps * float(np.real(M[0, 0]))
    b = crosscorr(h_j, h_r, w, T, k0)
    return np.linalg.solve(M + lam * np.eye(T), b)


def tukey(T, alpha=0.25):
    """Tukey (tapered cosine) window of T points."""
    if T == 1:
        return np.ones(1)
    x = np.arange(T, dtype=np.float64) / (T - 1)
    out = np.ones(T)
    if alpha <= 0:
        return out
    lo = x < alpha / 2
    hi = x > 1 - alpha / 2
    out[lo] = 0.5 * (1 + np.cos(np.pi * (2 * x[lo] / alpha - 1)))
    out[hi] = 0.5 * (1 + np.cos(np.pi * (2 * x[hi] / alpha - 2 / alpha + 1)))
    return out


def window_taps(h_j, h_r, w, T, k0, alpha=0.25):
    """The windowing-and-truncation route the paper contrasts with the fit
    (Sec. V): a[l] = win[l] (1/N) sum_i R_i exp(+2 pi i f_i t_l)."""
    n = 2 * (h_j.size - 1)
    R, _ = ratio_and_weight(h_j, h_r, w)
    full = one_sided_ifft(R, n) / n
    return tukey(T, alpha) * full[(k0 + np.arange(T, dtype=np.int64)) % n]


def chi2(h_j, h_r, w, a, k0, eps=DEFAULT_RIDGE_EPS):
    """The objective of Sec. V.A (plus ridge) summed directly over bins."""
    n = 2 * (h_j.size - 1)
    R, u = ratio_and_weight(h_j, h_r, w)
    bins = np.nonzero(u > 0)[0]
    A = design_matrix(bins, a.size, k0, n) @ a
    lam = eps * float(np.sum(u))
    return float(np.sum(u[bins] * np.abs(R[bins] - A) ** 2) + lam * np.sum(np.abs(a) ** 2))


def response(a, k0, n):
    """A_i = sum_k a_k exp(-2 pi i i (k0 + k) / N) for i = 0..N/2."""
    bins = np.arange(n // 2 + 1, dtype=np.int64)
    return design_matrix(bins, a.size, k0, n) @ a


def response_fft(a, k0, n):
    """The same A_i as `response`, by one length-N FFT of the taps placed at
    their lags (k0 + k) mod N: A_i = sum_m x[m] exp(-2 pi i i m / N) with
    x[(k0 + k) mod N] = a_k.  O(N log N) memory-light form for long segments."""
    x = np.zeros(n, dtype=np.complex128)
    lag = (k0 + np.arange(a.size, dtype=np.int64)) % n
    np.add.at(x, lag, a)
    return np.fft.fft(x)[: n // 2 + 1]


def fitted_sigma_sq_freq(a, h_r, w, k0):
    """(h_fit|h_fit) = sum_i w_i |h_ref A|^2: the frequency-domain form of
    Sec. VI.B for the fitted template h_fit = h_ref * A."""
    n = 2 * (h_r.size - 1)
    return float(np.sum(w * np.abs(h_r * response(a, k0, n)) ** 2))


def fitted_sigma_sq_lag(a, M):
    """The same norm in the tap domain (Sec. VI.B via Parseval): a^H M a,
    with M built from the reference autocorrelation."""
    return float(np.real(np.conj(a) @ (M @ a)))


def zero_lag_match(h_j, h_r, w, a, k0):
    """|(h_j|h_fit)(0)| / (sigma_j sigma_fit), h_fit = h_ref A: the fitted
    template's phase-maximised overlap with its target at zero lag, by
    frequency sums (Eq. 1 inner products).  Reading of Sec. V.A's target
    match: the filter reproduces the target at the target's own time, so the
    overlap is taken there."""
    n = 2 * (h_j.size - 1)
    h_fit = h_r * response(a, k0, n)
    num = abs(np.sum(w * h_j * np.conj(h_fit)))
    return float(num / np.sqrt(np.sum(w * np.abs(h_j) ** 2) * np.sum(w * np.abs(h_fit) ** 2)))


def select_taps(h_j, h_r, w, target, ladder, eps=DEFAULT_RIDGE_EPS, centre=False):
    """Sec. V.A's dynamic tap count: the first T of the ascending ladder whose
    least-squares taps (lags centred on lag 0, k0 = -floor(T/2), or with
    centre=True on the peak of |b|: k0 = centred_k0) reach the target
    zero-lag match; the last T if none does.  Returns (T, match)."""
    m = 0.0
    for T in ladder:
        k0 = centred_k0(h_j, h_r, w, T) if centre else -(T // 2)
        a = ls_taps_normal(h_j, h_r, w, T, k0, eps)
        m = zero_lag_match(h_j, h_r, w, a, k0)
        if m >= target:
            return T, m
    return ladder[-1], m
