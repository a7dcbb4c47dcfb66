"""A small search driver over the C ABI: device buffers and call order.

It takes host arrays (PSD, segment, waveforms), places them in torch device
tensors and runs the library's entry points on the current stream.  All
arithmetic of the path happens inside librfd.
"""
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import rfd


@dataclass
class SubBankSpec:
    ref_id: int
    taps: int
    k0: int
    count: int


class RatioFilterSearch:
    """Plan + taps for one bank of reference sub-banks."""

    def __init__(self, psd, f_low, fs, n, subbanks: List[SubBankSpec], max_refs: Optional[int] = None, stream=None):
        import torch
        self.torch = torch
        self.n = n
        self.subbanks = list(subbanks)
        nref = max_refs or (max(s.ref_id for s in subbanks) + 1)
        self.plan = rfd.rfd_plan_create(psd, f_low, fs, n, nref, stream)
        self.info = rfd.rfd_plan_info_get(self.plan)
        self.offsets = np.concatenate([[0], np.cumsum([s.count for s in subbanks])]).astype(np.int64)
        self.taps = rfd.rfd_taps_create(self.plan, self.offsets, [s.ref_id for s in subbanks],
                                        [s.taps for s in subbanks], [s.k0 for s in subbanks])
        self.h_ref = {}
        self.data = None

    @property
    def n_templates(self):
        return int(self.offsets[-1])

    def to_dev(self, a, dtype=None):
        t = self.torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        return t.to("cuda")

    def set_reference(self, ref_id, h_ref):
        self.h_ref[ref_id] = self.to_dev(np.asarray(h_ref, dtype=np.complex128))

    def make_taps(self, subbank, h_tmpl, first=0, method=rfd.RFD_TAPS_LS, ridge_eps=1e-4):
        spec = self.subbanks[subbank]
        ht = h_tmpl if isinstance(h_tmpl, self.torch.Tensor) else self.to_dev(np.asarray(h_tmpl, np.complex128))
        rfd.rfd_make_taps(self.plan, self.taps, subbank, self.h_ref[spec.ref_id], ht, first, method, ridge_eps)

    def set_segment(self, data):
        self.data = data if isinstance(data, self.torch.Tensor) else self.to_dev(np.asarray(data, np.float64))

    def dechirp_all(self, want_sigma=False):
        """Transform the segment once, then dechirp every reference (batched)."""
        sig = rfd.rfd_dechirp_refs(self.plan, self.data, self.h_ref, want_sigma)
        return sig if want_sigma else {r: None for r in self.h_ref}

    def filter(self, precision, threshold, window, capacity, out=None, raise_overflow=True):
        return rfd.rfd_filter_bank(self.plan, self.taps, precision, threshold, window, capacity, out,
                                   raise_overflow)

    def filter_range(self, precision, threshold, window, n_start, n_len, capacity, out=None):
        return rfd.rfd_filter_range(self.plan, self.taps, precision, threshold, window, n_start, n_len, capacity, out)

    def bands(self, n_bands):
        """Band series of every reference and band shares of every sub-bank
        (the chi^2 test's inputs); returns the edges per reference."""
        edges = {r: rfd.rfd_dechirp_bands(self.plan, h, r, n_bands) for r, h in self.h_ref.items()}
        for b, spec in enumerate(self.subbanks):
            if spec.count:
                rfd.rfd_taps_band_fractions(self.plan, self.taps, b, self.h_ref[spec.ref_id], n_bands)
        return edges

    def chisq(self, triggers, n):
        return rfd.rfd_chisq(self.plan, self.taps, triggers, n)

    def zref(self, ref_id):
        return rfd.rfd_get_zref(self.plan, ref_id)

    def tap(self, tmpl):
        return rfd.rfd_taps_get(self.taps, tmpl)

    def close(self):
        if self.taps is not None:
            rfd.rfd_taps_destroy(self.taps)
            self.taps = None
        if self.plan is not None:
            rfd.rfd_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TapSurrogate:
    """A learned tap generator for one (reference, T, k0) of a plan.

    Training taps are exact least-squares taps (Sec. V.A) made by librfd
    from training waveforms; the network maps scaled features to the
    coefficients of their phase-aligned, whitened form.  Inference fills a
    sub-bank of a search's taps; validation against exact taps and the
    per-template fallback use rfd_taps_match and rfd_taps_fallback.
    """

    def __init__(self, search, ref_id, T, k0, n_train, n_basis=64, hidden=256, seed=2601):
        import torch
        self.torch = torch
        self.search = search
        self.ref_id, self.T, self.k0 = ref_id, T, k0
        self.n_train = n_train
        self.n_basis, self.hidden, self.seed = n_basis, hidden, seed
        self.train_taps = rfd.rfd_taps_create(search.plan, np.array([0, n_train], np.int64), [ref_id], [T], [k0])
        self.sur = None
        self.params_dev = None

    def add_training_waveforms(self, h_tmpl, first, ridge_eps=1e-4):
        ht = h_tmpl if isinstance(h_tmpl, self.torch.Tensor) else self.search.to_dev(
            np.asarray(h_tmpl, np.complex128))
        rfd.rfd_make_taps(self.search.plan, self.train_taps, 0, self.search.h_ref[self.ref_id], ht, first,
                          rfd.RFD_TAPS_LS, ridge_eps)

    def _phys_dev(self, params):
        if isinstance(params, self.torch.Tensor):
            return params.to(device="cuda", dtype=self.torch.float64).reshape(-1, 4).contiguous()
        return self.search.to_dev(np.asarray(params, np.float64).reshape(-1, 4))

    def scale_dev(self, params):
        """Network inputs (dev float32 [n, 4]) of physical (m1, m2, chi, e0), by librfd."""
        return rfd.rfd_surrogate_features(self.sur, self._phys_dev(params))

    def scale(self, params):
        return self.scale_dev(params).cpu().numpy()

    def fit(self, train_params, basis_iters=20):
        """Input range from the training parameters, whitened training taps and
        the basis; returns the captured fraction."""
        self.sur = rfd.rfd_surrogate_create(self.search.plan, self.train_taps, 0, self.n_basis, self.hidden,
                                            self.seed)
        phys = self._phys_dev(train_params)
        rfd.rfd_surrogate_set_feature_range(self.sur, phys)
        self.params_dev = rfd.rfd_surrogate_features(self.sur, phys)
        return rfd.rfd_surrogate_fit_basis(self.sur, basis_iters)

    def train(self, epochs, batch=256, lr=2e-3, lr_end=2e-5, stages=10, progress=None):
        """Adam with a geometric learning-rate decay over `stages` calls;
        progress(stage, epochs_done, last_loss) after each."""
        losses = []
        per = max(1, epochs // stages)
        done = 0
        for s in range(stages):
            e = per if s < stages - 1 else epochs - done
            if e <= 0:
                break
            rate = lr * (lr_end / lr) ** (s / max(1, stages - 1))
            losses.append(rfd.rfd_surrogate_train(self.sur, self.params_dev, e, batch, rate))
            done += e
            if progress is not None:
                progress(s, done, float(losses[-1][-1]))
        return np.concatenate(losses)

    def make_taps(self, target_taps, subbank, params, first=0):
        rfd.rfd_surrogate_make_taps(self.sur, self.scale_dev(params), target_taps, subbank, first)

    def close(self):
        if self.sur is not None:
            rfd.rfd_surrogate_destroy(self.sur)
            self.sur = None
        if self.train_taps is not None:
            rfd.rfd_taps_destroy(self.train_taps)
            self.train_taps = None
