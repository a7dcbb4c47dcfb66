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
        """Transform the segment once, then dechirp every reference."""
        sig = {}
        first = True
        for ref_id in sorted(self.h_ref):
            sig[ref_id] = rfd.rfd_dechirp(self.plan, self.data if first else None, self.h_ref[ref_id], ref_id,
                                          want_sigma)
            first = False
        return sig

    def filter(self, precision, threshold, window, capacity, out=None, raise_overflow=True):
        return rfd.rfd_filter_bank(self.plan, self.taps, precision, threshold, window, capacity, out,
                                   raise_overflow)

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
