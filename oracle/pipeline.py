"""End-to-end FP64 evaluation of the two-step procedure (Fig. 2).

Test infrastructure only (see package header).

Step 1 (dechirp): the reference matched filter z_ref = (s|h_ref) of Eq. 1.
Step 2 (ratio filter): taps from Sec. V.A, then Eq. 3 by direct summation,
normalised by the fitted template's norm (Sec. VI.B).  Reading: the ratio
filter reconstructs the SNR of the fitted template h_fit = h_ref * A, so its
own norm (not the exact template's) normalises it; with that choice
<rho^2> = 2 in Gaussian noise holds exactly.
Step 3: threshold and per-window peak (Table II's last two stages).
FINDCHIRP (the baseline): Eq. 1 per template, normalised by its own sigma.
"""
from dataclasses import dataclass

import numpy as np

from . import spectral, taps as taps_mod, fir, cluster


@dataclass
class Prepared:
    n: int
    fs: float
    f_low: float
    w: np.ndarray          # PSD weights 4 df / S_n in band
    stilde: np.ndarray     # data transform, bins 0..N/2


def prepare(psd, data, fs, f_low):
    n = len(data)
    return Prepared(n, fs, f_low, spectral.psd_weights(psd, n, fs, f_low),
                    spectral.data_transform(data, fs))


@dataclass
class Reference:
    h: np.ndarray
    sigma: float
    z: np.ndarray          # complex reference SNR series (unnormalised)


def dechirp(p: Prepared, h_ref):
    """Reference series z_ref = (s|h_ref)(t_n) and sigma_ref (Eq. 1, Eq. 3)."""
    return Reference(h_ref, np.sqrt(spectral.sigma_sq(h_ref, p.w)),
                     spectral.matched_filter(p.stilde, h_ref, p.w))


@dataclass
class TemplateTaps:
    a: np.ndarray          # Sec. V.A taps (device applies conj(a))
    k0: int
    sigma_fit: float       # sqrt(a^H M a)


def make_taps(p: Prepared, h_j, h_ref, T, k0, method="ls", eps=taps_mod.DEFAULT_RIDGE_EPS,
              M=None, solver="normal"):
    """Taps and fitted norm for one template.

    method "ls": the weighted ridge fit (solver "normal": normal equations;
    "direct": stacked least squares).  method "window": truncated inverse
    transform of the ratio with a Tukey taper.
    """
    if M is None:
        M = taps_mod.gram(h_ref, p.w, T)
    if method == "ls":
        if solver == "direct":
            a = taps_mod.ls_taps_direct(h_j, h_ref, p.w, T, k0, eps)
        else:
            a = taps_mod.ls_taps_normal(h_j, h_ref, p.w, T, k0, eps, M=M)
    elif method == "window":
        a = taps_mod.window_taps(h_j, h_ref, p.w, T, k0)
    else:
        raise ValueError(method)
    return TemplateTaps(a, k0, np.sqrt(taps_mod.fitted_sigma_sq_lag(a, M)))


def ratio_snr(ref: Reference, tt: TemplateTaps):
    """Normalised SNR series rho_j[n] of the ratio filter (complex z too)."""
    z = fir.fir_direct(ref.z, np.conj(tt.a), tt.k0) / tt.sigma_fit
    return z


def ratio_snr_at(ref: Reference, tt: TemplateTaps, samples):
    return fir.fir_at(ref.z, np.conj(tt.a), tt.k0, samples) / tt.sigma_fit


def findchirp_snr(p: Prepared, h_j):
    """Normalised complex SNR series of the standard matched filter."""
    return spectral.matched_filter(p.stilde, h_j, p.w) / np.sqrt(spectral.sigma_sq(h_j, p.w))


def triggers(z_norm, threshold, window, shift=0):
    """[(sample, rho)] for one template from its normalised complex series.

    shift d: the template's taps start d lags after its sub-bank's k0 (per
    template lag centring).  Reading: its windows lie on the filter index
    m = n + d, i.e. [qW - d, (q+1)W - d) in samples n (taken mod N), so one
    window grid serves every template of a sub-bank in filter-index terms;
    samples are reported as n.  d = 0 is the plain grid aligned to n = 0."""
    if shift == 0:
        return cluster.cluster(np.abs(z_norm), threshold, window)
    n = z_norm.size
    y = np.roll(np.abs(z_norm), shift)        # y[m] = |z[(m - shift) mod N]|
    return [((m - shift) % n, r) for m, r in cluster.cluster(y, threshold, window)]


def match(p: Prepared, h_j, h_ref, tt: TemplateTaps):
    """Fidelity of the fitted template: max_t |(h_j|h_fit)(t)| / (sigma_j sigma_fit)."""
    A = taps_mod.response(tt.a, tt.k0, p.n)
    h_fit = h_ref * A
    z = spectral.matched_filter(h_j, h_fit, p.w)
    return float(np.max(np.abs(z)) / np.sqrt(spectral.sigma_sq(h_j, p.w) * spectral.sigma_sq(h_fit, p.w)))
