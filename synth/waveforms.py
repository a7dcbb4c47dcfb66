"""TaylorF2 frequency-domain inspiral waveforms (inputs, FP64).

The paper gives no waveform formulas.  These are the standard stationary-phase
post-Newtonian expressions:

* point-particle phase to 3.5PN: Buonanno, Iyer, Ochsner, Pan & Sathyaprakash,
  Phys. Rev. D 80, 084043 (2009), Table I (TaylorF2 column);
* aligned-spin spin-orbit (beta) and spin-spin (sigma) terms: Kidder (1995),
  Poisson & Will (1995);
* leading (5PN) tidal term in Lambda-tilde: Flanagan & Hinderer (2008),
  Favata (2014);
* leading-order eccentric correction to the Newtonian phase: Yunes & Arun
  (2009), Moore et al. (2016).

h(f) = f^(-7/6) exp(-i Psi(f)) for f_low <= f <= min(f_ISCO, fs/2), else 0,
with t_c = phi_c = 0.  The amplitude constant is dropped: every consumer
normalises by sigma.
"""
from dataclasses import dataclass

import numpy as np

MSUN_S = 4.925490947641267e-6          # G M_sun / c^3 in seconds
EULER_GAMMA = 0.5772156649015329


@dataclass(frozen=True)
class WaveformParams:
    m1: float                 # solar masses
    m2: float
    chi1: float = 0.0         # aligned dimensionless spins
    chi2: float = 0.0
    lambda1: float = 0.0      # dimensionless tidal deformabilities
    lambda2: float = 0.0
    e0: float = 0.0           # eccentricity at f_e0
    f_e0: float = 10.0        # Hz

    @property
    def mtot(self):
        return self.m1 + self.m2

    @property
    def eta(self):
        return self.m1 * self.m2 / self.mtot ** 2

    @property
    def mchirp(self):
        return self.mtot * self.eta ** 0.6


def f_isco(mtot_msun):
    """Schwarzschild ISCO gravitational-wave frequency (Hz)."""
    return 1.0 / (6.0 ** 1.5 * np.pi * mtot_msun * MSUN_S)


def lambda_tilde(p: WaveformParams):
    m1, m2, M = p.m1, p.m2, p.mtot
    return (16.0 / 13.0) * ((m1 + 12 * m2) * m1 ** 4 * p.lambda1
                            + (m2 + 12 * m1) * m2 ** 4 * p.lambda2) / M ** 5


def phase(f, p: WaveformParams):
    """Psi(f) for the parameters p, f in Hz (array, f > 0)."""
    f = np.asarray(f, dtype=np.float64)
    M = p.mtot * MSUN_S
    eta = p.eta
    v = np.cbrt(np.pi * M * f)
    x1, x2 = p.m1 / p.mtot, p.m2 / p.mtot
    beta = (113.0 * x1 * x1 / 12.0 + 25.0 * eta / 4.0) * p.chi1 \
        + (113.0 * x2 * x2 / 12.0 + 25.0 * eta / 4.0) * p.chi2
    sig = 79.0 / 8.0 * eta * p.chi1 * p.chi2
    pi = np.pi
    phi2 = 3715.0 / 756.0 + 55.0 * eta / 9.0
    phi3 = -16.0 * pi + 4.0 * beta
    phi4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta ** 2 / 72.0 - 10.0 * sig
    vlso = 6.0 ** -0.5
    phi5 = pi * (38645.0 / 756.0 - 65.0 * eta / 9.0) * (1.0 + 3.0 * np.log(v / vlso))
    phi6 = (11583231236531.0 / 4694215680.0 - 640.0 * pi ** 2 / 3.0 - 6848.0 * EULER_GAMMA / 21.0
            - 6848.0 / 21.0 * np.log(4.0 * v)
            + (-15737765635.0 / 3048192.0 + 2255.0 * pi ** 2 / 12.0) * eta
            + 76055.0 * eta ** 2 / 1728.0 - 127825.0 * eta ** 3 / 1296.0)
    phi7 = pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta ** 2 / 756.0)
    newt = 1.0
    if p.e0 != 0.0:
        newt = 1.0 - 2355.0 / 1462.0 * p.e0 ** 2 * (p.f_e0 / f) ** (19.0 / 9.0)
    v2 = v * v
    series = (newt + phi2 * v2 + phi3 * v2 * v + phi4 * v2 * v2 + phi5 * v2 * v2 * v
              + phi6 * v2 * v2 * v2 + phi7 * v2 * v2 * v2 * v)
    lt = lambda_tilde(p)
    if lt != 0.0:
        series = series - 39.0 / 2.0 * lt * v2 ** 5
    return -pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * series


def taylorf2(p: WaveformParams, n, fs, f_low, out=None):
    """Frequency-domain template on the rfft grid of an n-sample segment.

    Returns complex128 [n/2 + 1].  Bins outside [f_low, min(f_ISCO, fs/2)]
    are exactly zero.
    """
    df = fs / n
    nb = n // 2 + 1
    if out is None:
        out = np.zeros(nb, dtype=np.complex128)
    else:
        out[:] = 0
    f_hi = min(f_isco(p.mtot), fs / 2.0)
    i0 = int(np.ceil(f_low / df))
    i1 = min(int(np.floor(f_hi / df)), nb - 1)
    if i1 < i0:
        return out
    f = np.arange(i0, i1 + 1, dtype=np.float64) * df
    psi = phase(f, p)
    amp = f ** (-7.0 / 6.0)
    out[i0:i1 + 1] = amp * np.exp(-1j * psi)
    return out
