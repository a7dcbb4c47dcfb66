"""Seeded synthetic workloads: segment, noise, bank, reference association.

Five workloads, sized like the searches the paper targets (dense BNS banks
with a coarse reference bank, Sec. IV; eccentric and subsolar banks, Secs. I
and V.B).  The paper's own inputs (O3 PSD, stochastic-placement banks) are not
available; these synthetic stand-ins have the same shapes:

=========  =======  =====  ==========================================  ====  ========
name        N        f_low  bank                                        T     FIR form
=========  =======  =====  ==========================================  ====  ========
bns64s      2^17     30     16 non-spinning, m1,m2 in [1.3,1.5], 1 ref  64    fp32
spin256s    2^19     20     4096 aligned-spin, m in [1,3], |chi|<=.05   256   bf16x3
tidal256s   2^19     20     64 sub-banks of 256..2048 tidal templates   32..  fp16x3
                             (Lambda in [0,2000], m in [1,2])            1024
ecc512s     2^20     15     16384 eccentric, e0 in [0,.3] at 10 Hz,     1024  bf16x3
                             m in [0.2,1.0], 32 references
surr512s    2^20     20     65536 (m1,m2,chi,e0) for the tap surrogate   1024  bf16x3
=========  =======  =====  ==========================================  ====  ========

All draws come from numpy ``SeedSequence(260118835 + index).spawn(4)``:
stream 0 noise, 1 bank parameters, 2 sub-bank sizes and tap counts,
3 injection.  Noise is generated in the frequency domain, so every segment is
exactly periodic and circular correlation is exact.
"""
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
import os
from typing import List, Optional

import numpy as np

from .psd import psd_array
from .waveforms import WaveformParams, taylorf2

MASTER_SEED = 260118835


@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    n: int
    fs: float
    f_low: float
    n_templates: int          # total over all sub-banks (nominal for tidal256s)
    n_refs: int
    taps: int                 # tap count (maximum for tidal256s)
    precision: str            # "fp32" | "bf16x3" | "fp16x3"
    family: str
    threshold: float = 6.0    # on normalised SNR rho
    window: int = 2048        # cluster window in samples (1 s)
    injection_snr: float = 12.0

    @property
    def df(self):
        return self.fs / self.n

    @property
    def n_bins(self):
        return self.n // 2 + 1


WORKLOADS = {
    "bns64s": Workload("bns64s", 1, 1 << 17, 2048.0, 30.0, 16, 1, 64, "fp32", "nonspin"),
    "spin256s": Workload("spin256s", 2, 1 << 19, 2048.0, 20.0, 4096, 1, 256, "bf16x3", "alignedspin"),
    "tidal256s": Workload("tidal256s", 3, 1 << 19, 2048.0, 20.0, 64 * 1152, 64, 1024, "fp16x3", "tidal"),
    "ecc512s": Workload("ecc512s", 4, 1 << 20, 2048.0, 15.0, 16384, 32, 1024, "bf16x3", "eccentric"),
    "surr512s": Workload("surr512s", 5, 1 << 20, 2048.0, 20.0, 65536, 32, 1024, "bf16x3", "surrogate"),
}


def get_workload(name):
    return WORKLOADS[name]


def _streams(w: Workload):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(MASTER_SEED + w.index).spawn(4)]


def band(w: Workload):
    """(i_low, i_high) inclusive: in-band bins exclude DC and Nyquist."""
    i_low = int(np.ceil(w.f_low / w.df))
    return i_low, w.n // 2 - 1


def make_noise_spectrum(w: Workload, rng=None):
    """Coloured Gaussian noise in the frequency domain.

    s(f_i) = sqrt(S_n(f_i) / (4 df)) (x + i y), x, y ~ N(0, 1), in band;
    zero elsewhere.  So <|s|^2> = S_n / (2 df), the one-sided convention.
    """
    if rng is None:
        rng = _streams(w)[0]
    psd = psd_array(w.n, w.fs)
    i0, i1 = band(w)
    s = np.zeros(w.n_bins, dtype=np.complex128)
    m = i1 - i0 + 1
    g = rng.standard_normal((m, 2))
    s[i0:i1 + 1] = np.sqrt(psd[i0:i1 + 1] / (4.0 * w.df)) * (g[:, 0] + 1j * g[:, 1])
    return s


def spectrum_to_time(s, n, fs):
    """Real time series whose transform Delta_t * DFT equals s on bins 0..n/2."""
    return fs * np.fft.irfft(s, n)


def optimal_snr_amplitude(h, w: Workload, snr):
    """Amplitude A such that A*h has optimal SNR `snr` in the analytic PSD.

    Optimal SNR^2 = 4 df sum |A h|^2 / S_n over the band (the usual inner
    product); used only to scale injections.
    """
    psd = psd_array(w.n, w.fs)
    i0, i1 = band(w)
    hh = 4.0 * w.df * np.sum(np.abs(h[i0:i1 + 1]) ** 2 / psd[i0:i1 + 1])
    return snr / np.sqrt(hh)


@dataclass
class SubBank:
    ref: WaveformParams
    params: List[WaveformParams]
    taps: int
    k0: int

    @property
    def size(self):
        return len(self.params)


@dataclass
class Bank:
    workload: Workload
    subbanks: List[SubBank]
    offsets: np.ndarray = field(default=None)   # [n_subbanks + 1] template offsets

    def __post_init__(self):
        if self.offsets is None:
            sizes = np.array([sb.size for sb in self.subbanks], dtype=np.int64)
            self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    @property
    def n_templates(self):
        return int(self.offsets[-1])

    def params(self, j):
        b = int(np.searchsorted(self.offsets, j, side="right") - 1)
        return self.subbanks[b].params[j - int(self.offsets[b])]

    def subbank_of(self, j):
        return int(np.searchsorted(self.offsets, j, side="right") - 1)


def _draw_params(w: Workload, rng, count):
    u = rng.uniform
    out = []
    if w.family == "nonspin":
        m = u(1.3, 1.5, size=(count, 2))
        out = [WaveformParams(a, b) for a, b in m]
    elif w.family == "alignedspin":
        m = u(1.0, 3.0, size=(count, 2))
        c = u(-0.05, 0.05, size=(count, 2))
        out = [WaveformParams(a, b, x, y) for (a, b), (x, y) in zip(m, c)]
    elif w.family == "tidal":
        m = u(1.0, 2.0, size=(count, 2))
        lam = u(0.0, 2000.0, size=count)
        out = [WaveformParams(a, b, lambda1=l, lambda2=l) for (a, b), l in zip(m, lam)]
    elif w.family == "eccentric":
        m = u(0.2, 1.0, size=(count, 2))
        e = u(0.0, 0.3, size=count)
        out = [WaveformParams(a, b, e0=x) for (a, b), x in zip(m, e)]
    elif w.family == "surrogate":
        m = u(1.0, 2.0, size=(count, 2))
        c = u(-0.05, 0.05, size=count)
        e = u(0.0, 0.3, size=count)
        out = [WaveformParams(a, b, x, x, e0=y) for (a, b), x, y in zip(m, c, e)]
    else:
        raise ValueError(w.family)
    return out


def draw_in_chirp_mass_range(w: Workload, lo, hi, count, stream=5):
    """`count` parameter draws of workload w's family whose chirp mass lies in
    [lo, hi] (rejection from the family's distribution; a seeded stream of
    its own, so the bank's draws are untouched)."""
    rng = np.random.default_rng(np.random.SeedSequence(MASTER_SEED + w.index).spawn(stream + 1)[stream])
    out = []
    while len(out) < count:
        out += [p for p in _draw_params(w, rng, 8192) if lo <= p.mchirp <= hi]
    return out[:count]


def _equal_mass_with_mchirp(mc):
    m = mc * 2.0 ** 0.2          # equal masses: Mc = m * 2^(-1/5)
    return WaveformParams(m, m)


def make_bank(w: Workload, max_templates: Optional[int] = None):
    """Draw the bank of workload w and group it into reference sub-banks.

    Single-reference workloads use the centre of the mass range as reference.
    Multi-reference workloads sort templates by chirp mass, cut them into
    consecutive groups (equal sizes, or the seeded uneven sizes of tidal256s)
    and put an equal-mass reference at each group's median chirp mass.  This
    stands in for the paper's association of each template with its
    best-matching reference (Sec. IV), which needs per-pair matches from a
    placement tool that is not available here.

    ``max_templates`` truncates each sub-bank proportionally (for tests); the
    draws themselves do not depend on it.
    """
    rs = _streams(w)
    rng_bank, rng_sizes = rs[1], rs[2]
    if w.name == "bns64s":
        sbs = [SubBank(WaveformParams(1.4, 1.4), _draw_params(w, rng_bank, w.n_templates), w.taps, -(w.taps // 2))]
    elif w.name == "spin256s":
        sbs = [SubBank(WaveformParams(2.0, 2.0), _draw_params(w, rng_bank, w.n_templates), w.taps, -(w.taps // 2))]
    else:
        if w.name == "tidal256s":
            sizes = rng_sizes.integers(256, 2049, size=w.n_refs)
            taps = rng_sizes.integers(32, 1025, size=w.n_refs)
        else:
            sizes = np.full(w.n_refs, w.n_templates // w.n_refs)
            taps = np.full(w.n_refs, w.taps)
        total = int(sizes.sum())
        params = _draw_params(w, rng_bank, total)
        order = np.argsort([p.mchirp for p in params], kind="stable")
        params = [params[i] for i in order]
        sbs = []
        o = 0
        for b in range(w.n_refs):
            grp = params[o:o + int(sizes[b])]
            o += int(sizes[b])
            mc = float(np.median([p.mchirp for p in grp]))
            ref = _equal_mass_with_mchirp(mc)
            if w.family == "tidal":
                lam = float(np.median([p.lambda1 for p in grp]))
                ref = WaveformParams(ref.m1, ref.m2, lambda1=lam, lambda2=lam)
            elif w.family == "eccentric" or w.family == "surrogate":
                e = float(np.median([p.e0 for p in grp]))
                ref = WaveformParams(ref.m1, ref.m2, e0=e)
            T = int(taps[b])
            sbs.append(SubBank(ref, grp, T, -(T // 2)))
    if max_templates is not None:
        per = max(1, max_templates // len(sbs))
        sbs = [SubBank(sb.ref, sb.params[:per], sb.taps, sb.k0) for sb in sbs]
    return Bank(w, sbs)


def _nthreads():
    return max(1, min(16, os.cpu_count() or 1))


def template_batch(w: Workload, params: List[WaveformParams], out=None, threads=None):
    """complex128 [len(params), N/2+1] TaylorF2 templates (threaded over templates)."""
    k = len(params)
    if out is None:
        out = np.zeros((k, w.n_bins), dtype=np.complex128)
    threads = threads or _nthreads()

    def one(i):
        taylorf2(params[i], w.n, w.fs, w.f_low, out=out[i])

    if k == 1 or threads == 1:
        for i in range(k):
            one(i)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(k)))
    return out


def reference_waveform(w: Workload, sb: SubBank):
    return taylorf2(sb.ref, w.n, w.fs, w.f_low)


@dataclass
class Segment:
    workload: Workload
    data: np.ndarray               # float64 [N] time series
    noise_spectrum: np.ndarray     # complex128 [N/2+1], before injection
    inj_template: int              # template index (-1: none)
    inj_sample: int
    inj_amplitude: float


def make_segment(w: Workload, bank: Optional[Bank] = None, noise=True, inject=True):
    """One analysis segment: coloured noise plus one SNR-12 injection.

    The injected template j is drawn from the bank and placed at an integer
    sample n0 in [N/4, 3N/4):  s += A h_j exp(-2 pi i f n0 / fs), with A
    such that its optimal SNR is `injection_snr`.
    """
    rs = _streams(w)
    rng_noise, rng_inj = rs[0], rs[3]
    s = make_noise_spectrum(w, rng_noise) if noise else np.zeros(w.n_bins, dtype=np.complex128)
    s0 = s.copy()
    j, n0, amp = -1, 0, 0.0
    if inject and bank is not None:
        j = int(rng_inj.integers(0, bank.n_templates))
        n0 = int(rng_inj.integers(w.n // 4, 3 * w.n // 4))
        h = taylorf2(bank.params(j), w.n, w.fs, w.f_low)
        amp = optimal_snr_amplitude(h, w, w.injection_snr)
        k = np.arange(w.n_bins, dtype=np.int64)
        frac = ((k * n0) % w.n).astype(np.float64) / w.n      # exact phase reduction
        s = s + amp * h * np.exp(-2j * np.pi * frac)
    return Segment(w, spectrum_to_time(s, w.n, w.fs), s0, j, n0, amp)
