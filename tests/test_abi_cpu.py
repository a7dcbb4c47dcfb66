"""Host-side checks of the C ABI: exports, and errors forced from the host.

No kernel runs here: every call below fails validation before touching the
device, or (without a GPU) fails at its first device allocation.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT, gpu_available

rfd = pytest.importorskip("paper_2601_18835_amd.rfd", reason="librfd.so not built")


def header_functions():
    txt = open(os.path.join(ROOT, "include", "rfd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert "rfd_filter_bank" in names and "findchirp_filter" in names and len(names) >= 14
    lib = C.CDLL(rfd.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(rfd.EXPORTED)


def psd_for(n, fs=2048.0):
    import synth
    return synth.psd_array(n, fs)


def create(psd, f_low=20.0, fs=2048.0, n=4096, max_refs=1):
    h = C.c_void_p()
    rc = rfd._lib.rfd_plan_create(np.ascontiguousarray(psd).ctypes.data, psd.size, f_low, fs, n, max_refs, None,
                                  C.byref(h))
    return rc, h


@pytest.mark.parametrize("n", [1000, 512, 1 << 23, 0, -4096])
def test_plan_rejects_bad_segment_length(n):
    psd = psd_for(4096)
    rc, _ = create(psd, n=n)
    assert rc == rfd.RFD_E_INVALID
    assert "seg_len" in rfd.rfd_last_error() or "n_psd" in rfd.rfd_last_error()


def test_plan_rejects_inconsistent_arguments():
    psd = psd_for(4096)
    assert create(psd[:-1])[0] == rfd.RFD_E_INVALID
    assert create(psd, f_low=1024.0)[0] == rfd.RFD_E_INVALID
    assert create(psd, f_low=0.0)[0] == rfd.RFD_E_INVALID
    assert create(psd, fs=-1.0)[0] == rfd.RFD_E_INVALID
    assert create(psd, max_refs=0)[0] == rfd.RFD_E_INVALID
    bad = psd.copy()
    bad[100] = np.nan
    assert create(bad)[0] == rfd.RFD_E_INVALID
    assert "bin 100" in rfd.rfd_last_error()
    bad = psd.copy()
    bad[2047] = 0.0
    assert create(bad)[0] == rfd.RFD_E_INVALID
    ok_out_of_band = psd.copy()
    ok_out_of_band[0] = np.nan            # DC is outside every band: ignored
    ok_out_of_band[2048] = -1.0           # Nyquist too
    rc, h = create(ok_out_of_band)
    assert rc != rfd.RFD_E_INVALID
    if rc == rfd.RFD_OK:
        rfd.rfd_plan_destroy(h)


def test_null_arguments_are_rejected():
    assert rfd._lib.rfd_plan_create(None, 2049, 20.0, 2048.0, 4096, 1, None, None) == rfd.RFD_E_INVALID
    assert rfd._lib.rfd_dechirp(None, None, None, 0, None) == rfd.RFD_E_INVALID
    assert rfd._lib.rfd_filter_bank(None, None, 0, 6.0, 2048, None, 0, None) == rfd.RFD_E_INVALID
    assert rfd._lib.rfd_make_taps(None, None, 0, None, None, 0, 0, 0, 1e-6) == rfd.RFD_E_INVALID
    assert rfd._lib.findchirp_filter(None, None, None, 0, 6.0, 2048, None, 0, None) == rfd.RFD_E_INVALID
    assert rfd._lib.rfd_plan_destroy(None) == rfd.RFD_OK
    assert rfd._lib.rfd_taps_destroy(None) == rfd.RFD_OK
    b = C.c_size_t(7)
    assert rfd._lib.rfd_plan_workspace_size(None, 16, 2048, 1, C.byref(b)) == rfd.RFD_E_INVALID
    assert b.value == 7
    assert rfd._lib.rfd_plan_set_workspace(None, None, 0, 0, 1, 0) == rfd.RFD_E_INVALID
    assert rfd._lib.rfd_dechirp_refs(None, None, 1, None, None, None) == rfd.RFD_E_INVALID


@pytest.mark.skipif(gpu_available(), reason="forces an allocation failure by having no device")
def test_device_allocation_failure_is_reported_without_gpu():
    psd = psd_for(4096)
    rc, h = create(psd)
    assert rc in (rfd.RFD_E_NOMEM, rfd.RFD_E_DEVICE)
    assert h.value is None
    assert rfd.rfd_last_error()


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The binding has no fallback: a copy of it next to no librfd.so refuses
    to import (the product path never degrades to a host implementation)."""
    import importlib.util
    import shutil
    src = os.path.join(ROOT, "paper_2601_18835_amd", "rfd.py")
    dst = tmp_path / "rfd_nolib.py"
    shutil.copy(src, dst)
    spec = importlib.util.spec_from_file_location("rfd_nolib", str(dst))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="librfd.so is missing"):
        spec.loader.exec_module(mod)
