"""Eq. 3: the target's SNR series from the reference series by a short FIR.

Test infrastructure only (see package header).

Substituting Eq. 2 into Eq. 1 with the fitted ratio A_i = sum_k a_k
exp(-2 pi i f_i t_k) gives, for the fitted template h_fit = h_ref * A,

    (s|h_fit)(t_n) = sum_k conj(a_k) z_ref(t_n + t_k),

a correlation of the reference series with the conjugated taps (Reading:
the paper writes the ratio without the conjugate; Eq. 1 conjugates the
template, so conj(R) is what multiplies the reference filter output).
Segments are periodic, so the lag index wraps modulo N.
"""
import numpy as np


def fir_direct(z_ref, c, k0):
    """out[n] = sum_k c[k] z_ref[(n + k0 + k) mod N] by direct summation."""
    z_ref = np.asarray(z_ref, dtype=np.complex128)
    out = np.zeros_like(z_ref)
    for k in range(len(c)):
        out += c[k] * np.roll(z_ref, -(k0 + k))
    return out


def fir_at(z_ref, c, k0, samples):
    """The same sum at selected output samples only."""
    n = z_ref.size
    samples = np.asarray(samples, dtype=np.int64)
    idx = (samples[:, None] + k0 + np.arange(len(c))[None, :]) % n
    return z_ref[idx] @ np.asarray(c, dtype=np.complex128)


def ratio_filter_snr(z_ref, a, k0, sigma_fit):
    """Normalised SNR series of the target: |sum_k conj(a_k) z_ref| / sigma_fit."""
    return np.abs(fir_direct(z_ref, np.conj(a), k0)) / sigma_fit
