"""Analytic one-sided noise PSD used by every synthetic workload.

S(f) = 1e-46 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)],
x = f / 215 Hz.  It is positive on [10, 1024] Hz (minimum 3.24e-45 at 228 Hz)
and stands in for the Advanced LIGO O3 PSD the paper's BNS bank was built with
(Sec. IV), which is not available here.
"""
import numpy as np

F0_HZ = 215.0


def analytic_psd(f):
    """S_n(f) in 1/Hz for f > 0 (float64)."""
    x = np.asarray(f, dtype=np.float64) / F0_HZ
    x2 = x * x
    return 1e-46 * (x ** -4.14 - 5.0 / x2 + 111.0 * (1.0 - x2 + 0.5 * x2 * x2) / (1.0 + 0.5 * x2))


def psd_array(n, fs):
    """PSD sampled on the rfft grid f_i = i fs / n, i = 0..n/2.

    The DC bin has no finite value; it is filled with the i = 1 value.  DC is
    outside every analysis band, so the value never enters a computation.
    """
    df = fs / n
    f = np.arange(n // 2 + 1, dtype=np.float64) * df
    out = np.empty_like(f)
    out[1:] = analytic_psd(f[1:])
    out[0] = out[1]
    return out
