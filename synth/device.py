"""TaylorF2 template batches generated in device memory (inputs only).

The same stationary-phase formulas as `synth.waveforms` (3.5PN point-particle
phase, aligned-spin beta / sigma terms, leading tidal and eccentric
corrections, f^(-7/6) amplitude cut at f_ISCO), evaluated in FP64 with torch
tensor operations on whatever device the caller names.  Banks of tens of
thousands of templates at 2^20 samples then take seconds instead of minutes
of host time.  Values agree with `synth.waveforms.taylorf2` to FP64 rounding
(the phase reaches 1e5-1e6 rad for the lightest eccentric systems, so the
agreement is ~1e-10 relative there, checked in tests/test_synth_inputs.py).

Inputs for the GPU path only: the oracle consumes host waveforms, and every
parity comparison gives both sides the same host waveforms.
"""
import math

import numpy as np

from .waveforms import EULER_GAMMA, MSUN_S


def _columns(params):
    a = np.array([[p.m1, p.m2, p.chi1, p.chi2, p.lambda1, p.lambda2, p.e0, p.f_e0] for p in params],
                 dtype=np.float64)
    return a.T


def template_batch_device(w, params, device, out=None):
    """complex128 tensor [len(params), N/2+1] on `device`; bins outside
    [f_low, min(f_ISCO, fs/2)] are exactly zero (as taylorf2)."""
    import torch
    k = len(params)
    n, fs, f_low = w.n, w.fs, w.f_low
    nb = n // 2 + 1
    df = fs / n
    if out is None:
        out = torch.zeros((k, nb), dtype=torch.complex128, device=device)
    else:
        out.zero_()
    if k == 0:
        return out
    m1, m2, c1, c2, l1, l2, e0, fe0 = (torch.from_numpy(c).to(device)[:, None] for c in _columns(params))
    mtot = m1 + m2
    eta = m1 * m2 / mtot ** 2
    # band per template: [ceil(f_low/df), floor(min(f_isco, fs/2)/df)], as taylorf2
    f_isco = 1.0 / (6.0 ** 1.5 * math.pi * mtot * MSUN_S)
    i0 = int(math.ceil(f_low / df))
    i1 = torch.clamp(torch.floor(torch.clamp(f_isco, max=fs / 2.0) / df), max=nb - 1)
    i1_max = int(i1.max().item())
    if i1_max < i0:
        return out
    idx = torch.arange(i0, i1_max + 1, dtype=torch.float64, device=device)[None, :]
    f = idx * df
    keep = idx <= i1
    M = mtot * MSUN_S
    v = torch.pow(math.pi * M * f, 1.0 / 3.0)
    x1, x2 = m1 / mtot, m2 / mtot
    beta = (113.0 * x1 * x1 / 12.0 + 25.0 * eta / 4.0) * c1 + (113.0 * x2 * x2 / 12.0 + 25.0 * eta / 4.0) * c2
    sig = 79.0 / 8.0 * eta * c1 * c2
    pi = math.pi
    phi2 = 3715.0 / 756.0 + 55.0 * eta / 9.0
    phi3 = -16.0 * pi + 4.0 * beta
    phi4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta ** 2 / 72.0 - 10.0 * sig
    vlso = 6.0 ** -0.5
    phi5 = pi * (38645.0 / 756.0 - 65.0 * eta / 9.0) * (1.0 + 3.0 * torch.log(v / vlso))
    phi6 = (11583231236531.0 / 4694215680.0 - 640.0 * pi ** 2 / 3.0 - 6848.0 * EULER_GAMMA / 21.0
            - 6848.0 / 21.0 * torch.log(4.0 * v)
            + (-15737765635.0 / 3048192.0 + 2255.0 * pi ** 2 / 12.0) * eta
            + 76055.0 * eta ** 2 / 1728.0 - 127825.0 * eta ** 3 / 1296.0)
    phi7 = pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta ** 2 / 756.0)
    newt = 1.0 - 2355.0 / 1462.0 * e0 ** 2 * torch.pow(fe0 / f, 19.0 / 9.0)
    v2 = v * v
    series = (newt + phi2 * v2 + phi3 * v2 * v + phi4 * v2 * v2 + phi5 * v2 * v2 * v
              + phi6 * v2 * v2 * v2 + phi7 * v2 * v2 * v2 * v)
    lt = (16.0 / 13.0) * ((m1 + 12 * m2) * m1 ** 4 * l1 + (m2 + 12 * m1) * m2 ** 4 * l2) / mtot ** 5
    series = series - 39.0 / 2.0 * lt * v2 ** 5
    psi = -pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * series
    amp = torch.pow(f, -7.0 / 6.0)
    h = torch.polar(amp.expand_as(psi).contiguous(), -psi)
    h = torch.where(keep, h, torch.zeros((), dtype=h.dtype, device=device))
    out[:, i0:i1_max + 1] = h
    return out
