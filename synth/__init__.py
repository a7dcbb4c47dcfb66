"""Seeded synthetic inputs for ratio-filter dechirping (arXiv:2601.18835).

This package produces *inputs only*: the analytic noise PSD, coloured Gaussian
noise, TaylorF2 frequency-domain waveforms, template banks with their
reference association, and SNR-12 injections.  It holds none of the method's
arithmetic (no matched filter, no taps, no FIR, no clustering), so the FP64
oracle and the GPU path may both consume what it generates without sharing
any method code.

The paper states no waveform model, PSD or worked example; every formula here
is from the published post-Newtonian literature named in the docstrings, and
the workload sizes follow the paper's BNS / eccentric / subsolar search setting
(Secs. IV and V, Fig. 4 and 5 captions).
"""
from .psd import analytic_psd, psd_array
from .waveforms import taylorf2, f_isco, WaveformParams
from .workloads import (Workload, WORKLOADS, get_workload, make_noise_spectrum,
                        spectrum_to_time, make_segment, SubBank, Bank, make_bank,
                        template_batch, reference_waveform)

__all__ = ["analytic_psd", "psd_array", "taylorf2", "f_isco", "WaveformParams",
           "Workload", "WORKLOADS", "get_workload", "make_noise_spectrum",
           "spectrum_to_time", "make_segment", "SubBank", "Bank", "make_bank",
           "template_batch", "reference_waveform"]
