"""Eq. 1 discretised: the complex matched filter (FINDCHIRP definition).

Test infrastructure only (see package header).

Discretisation (Reading, the paper gives the continuous integral only):
  * segment of N samples at rate fs, dt = 1/fs, df = fs/N, f_i = i df;
  * Fourier convention s(f_i) = dt * sum_m s[m] exp(-2 pi i i m / N);
  * the one-sided integral over f >= 0 becomes a sum over the analysis band
    i_low = ceil(f_low/df) <= i <= N/2 - 1 (DC and Nyquist excluded), with
    the factor 4 df folded into the weight w_i = 4 df / S_n(f_i);
  * the output is complex and sampled at t_n = n dt:
        z[n] = sum_i w_i s(f_i) conj(h(f_i)) exp(+2 pi i i n / N).
"""
import numpy as np


def band_limits(n, fs, f_low):
    """(i_low, i_high), inclusive bin range of the analysis band."""
    df = fs / n
    return int(np.ceil(f_low / df)), n // 2 - 1


def psd_weights(psd, n, fs, f_low):
    """w_i = 4 df / S_n(f_i) in band, 0 elsewhere (Eq. 1's 4/S_n times df)."""
    df = fs / n
    i0, i1 = band_limits(n, fs, f_low)
    w = np.zeros(n // 2 + 1, dtype=np.float64)
    w[i0:i1 + 1] = 4.0 * df / psd[i0:i1 + 1]
    return w


def data_transform(x, fs):
    """s(f_i) = dt * DFT(x)[i] for i = 0..N/2 (x real, float64)."""
    return np.fft.rfft(np.asarray(x, dtype=np.float64)) / fs


def dft_brute(x, sign=-1):
    """O(N^2) DFT by the defining sum, for pinning on tiny N."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.size
    k = np.arange(n)
    e = np.exp(sign * 2j * np.pi * ((np.outer(k, k) % n) / n))
    return e @ x


def one_sided_ifft(q, n):
    """sum_{i=0}^{N/2} q[i] exp(+2 pi i i n / N), n = 0..N-1 (no 1/N)."""
    full = np.zeros(n, dtype=np.complex128)
    full[:q.size] = q
    return np.fft.ifft(full) * n


def matched_filter(stilde, h, w):
    """Complex SNR series z[n] = sum_i w_i s_i conj(h_i) exp(+2 pi i i n/N).

    Eq. 1 with the discretisation above; used for FINDCHIRP and, with h the
    reference template, for the dechirped reference series (Eq. 3, Fig. 2).
    """
    n = 2 * (stilde.size - 1)
    return one_sided_ifft(w * stilde * np.conj(h), n)


def sigma_sq(h, w):
    """(h|h) = sum_i w_i |h_i|^2 (Eq. 1 with s = h at t = 0)."""
    return float(np.sum(w * np.abs(h) ** 2))


def matched_filter_at(stilde, h, w, samples):
    """z at selected samples by the defining sum (no FFT), for spot checks."""
    n = 2 * (stilde.size - 1)
    q = w * stilde * np.conj(h)
    idx = np.nonzero(q)[0]
    out = np.empty(len(samples), dtype=np.complex128)
    for t, s in enumerate(samples):
        ph = ((idx.astype(np.int64) * int(s)) % n) / n
        out[t] = np.sum(q[idx] * np.exp(2j * np.pi * ph))
    return out
