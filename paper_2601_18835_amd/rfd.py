"""Thin ctypes binding of librfd (include/rfd.h): argument marshalling only.

Every step of the path runs in the HIP library; torch supplies device memory
and the stream.  Functions keep the C names.  Importing this module loads
librfd.so and raises if it is missing: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np
# torch first: it loads its bundled HIP runtime (soname libamdhip64.so.7), and
# librfd then binds to that same runtime instead of loading a second copy.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_18835_amd.build` "
                      "(or __graft_entry__.build()); there is no non-HIP fallback")
_lib = C.CDLL(LIB_PATH)

RFD_OK, RFD_E_INVALID, RFD_E_NOMEM, RFD_E_DEVICE, RFD_E_OVERFLOW, RFD_E_STATE, RFD_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
RFD_FP32, RFD_BF16X3, RFD_FP16X3, RFD_OLS32 = 0, 1, 2, 3
RFD_TAPS_LS, RFD_TAPS_WINDOW = 0, 1
RFD_TAPS_CENTRE = 0x100          # flag: per-template lag windows (or-ed into a method)
RFD_MAX_TAPS = 2048
PRECISIONS = {"fp32": RFD_FP32, "bf16x3": RFD_BF16X3, "fp16x3": RFD_FP16X3, "ols32": RFD_OLS32}

TRIGGER_DTYPE = np.dtype([("sample", "<i8"), ("tmpl", "<i4"), ("subbank", "<i4"), ("rho", "<f4"),
                          ("z_re", "<f4"), ("z_im", "<f4"), ("flags", "<u4")])
assert TRIGGER_DTYPE.itemsize == 32


class rfd_plan_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_bins", C.c_int64), ("i_low", C.c_int64), ("i_high", C.c_int64),
                ("n_band", C.c_int64), ("fs", C.c_double), ("f_low", C.c_double), ("df", C.c_double),
                ("data_scale", C.c_double), ("max_refs", C.c_int32), ("fft_n1", C.c_int32), ("fft_n2", C.c_int32)]


class rfd_timing(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("data_fft_ms", "dechirp_ms", "fir_ms", "compact_ms", "findchirp_ms",
                                          "taps_ms", "sur_net_ms", "sur_expand_ms", "sur_pack_ms", "match_ms")] + \
               [(k, C.c_int64) for k in ("n_data_fft", "n_dechirp", "n_fir", "n_compact", "n_findchirp", "n_taps",
                                         "n_sur_net", "n_sur_expand", "n_sur_pack", "n_match")] + \
               [("fir_kernel_ms", C.c_double), ("n_fir_kernel", C.c_int64)]


class rfd_fir_config(C.Structure):
    _fields_ = [("col_blocks", C.c_int32), ("mode", C.c_int32), ("max_tiles", C.c_int32), ("wg_per_cu", C.c_int32),
                ("ols_block", C.c_int32), ("ols_aligned", C.c_int32)]


class rfd_tune_result(C.Structure):
    _fields_ = [("best", rfd_fir_config), ("best_ms", C.c_double), ("before_ms", C.c_double),
                ("n_candidates", C.c_int32)]


_P = C.c_void_p
_i64, _i32, _d, _f = C.c_int64, C.c_int32, C.c_double, C.c_float
_SIGS = {
    "rfd_plan_create": [_P, _i64, _d, _d, _i64, _i32, _P, C.POINTER(_P)],
    "rfd_plan_info_get": [_P, C.POINTER(rfd_plan_info)],
    "rfd_plan_set_stream": [_P, _P],
    "rfd_plan_destroy": [_P],
    "rfd_plan_workspace_size": [_P, _i64, _i64, _i32, C.POINTER(C.c_size_t)],
    "rfd_measure_peaks": [_P, _P],
    "rfd_plan_set_workspace": [_P, _P, C.c_size_t, _i64, _i64, _i32],
    "rfd_plan_set_timing": [_P, _i32],
    "rfd_plan_set_fir_config": [_P, C.POINTER(rfd_fir_config)],
    "rfd_plan_get_fir_config": [_P, C.POINTER(rfd_fir_config)],
    "rfd_autotune_fir": [_P, _P, _i32, _i64, _i32, C.POINTER(rfd_tune_result)],
    "rfd_segment_graph_create": [_P, _P, _i32, _f, _i64, _P, _i32, _P, _P, _P, _i64, C.POINTER(_P)],
    "rfd_segment_graph_launch": [_P, C.POINTER(_i64)],
    "rfd_range_graph_create": [_P, _P, _i32, _f, _i64, _P, _i32, _P, _P, _i64, _i64, _P, _i64, C.POINTER(_P)],
    "rfd_graph_destroy": [_P],
    "rfd_surrogate_create": [_P, _P, _i32, _i32, _i32, C.c_uint64, C.POINTER(_P)],
    "rfd_surrogate_fit_basis": [_P, _i32, C.POINTER(_d)],
    "rfd_surrogate_train": [_P, _P, _i32, _i32, _f, _P],
    "rfd_surrogate_train_many": [_P, _P, _i32, _i32, _i32, _f, _P],
    "rfd_surrogate_set_graphs": [_P, _i32],
    "rfd_surrogate_loss_grad": [_P, _P, _P, _i32, _P, C.POINTER(_d)],
    "rfd_surrogate_get_state": [_P, _P, _P, _P, _P],
    "rfd_surrogate_set_state": [_P, _P, _P],
    "rfd_surrogate_make_taps": [_P, _P, _P, _i32, _i64, _i64],
    "rfd_taps_match": [_P, _P, _i32, _i64, _i64, _P],
    "rfd_taps_fallback": [_P, _P, _i32, _i64, _i64, _P, _d, C.POINTER(_i64)],
    "rfd_dechirp_bands": [_P, _P, _i32, _i32, _P],
    "rfd_taps_band_fractions": [_P, _P, _i32, _P, _i32],
    "rfd_taps_get_band_fractions": [_P, _i64, _P, C.POINTER(_i32)],
    "rfd_chisq": [_P, _P, _P, _i64, _P],
    "rfd_select_taps": [_P, _P, _P, _i64, _d, _P, _i32, _d, _i32, _P, _P, _P],
    "rfd_plan_set_psd": [_P, _P, _i64],
    "rfd_filter_range": [_P, _P, _i32, _f, _i64, _i64, _i64, _P, _i64, C.POINTER(_i64)],
    "rfd_taps_renormalize": [_P, _P, _i32, _P],
    "rfd_surrogate_destroy": [_P],
    "rfd_plan_get_timing": [_P, C.POINTER(rfd_timing)],
    "rfd_dechirp": [_P, _P, _P, _i32, C.POINTER(_d)],
    "rfd_dechirp_refs": [_P, _P, _i32, _P, _P, _P],
    "rfd_get_zref": [_P, _i32, _P],
    "rfd_taps_create": [_P, _i32, _P, _P, _P, _P, C.POINTER(_P)],
    "rfd_make_taps": [_P, _P, _i32, _P, _P, _i64, _i64, _i32, _d],
    "rfd_taps_get": [_P, _i64, _P, C.POINTER(_d), C.POINTER(_i32), C.POINTER(_i32)],
    "rfd_taps_destroy": [_P],
    "rfd_filter_bank": [_P, _P, _i32, _f, _i64, _P, _i64, C.POINTER(_i64)],
    "rfd_filter_bank_noalloc": [_P, _P, _i32, _f, _i64, _P, _i64, C.POINTER(_i64)],
    "rfd_stream_create": [_P, _P, _i32, _P, _P, _i64, C.POINTER(_P)],
    "rfd_stream_prime": [_P, _P],
    "rfd_stream_push": [_P, _P, _i32, _f, _i64, _P, _i64, C.POINTER(_i64), C.POINTER(_i64)],
    "rfd_stream_info": [_P, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)],
    "rfd_stream_destroy": [_P],
    "rfd_debug_fail_allocation": [_i64],
    "rfd_ols_shape": [_P, _i32, C.POINTER(_i32), C.POINTER(_i32)],
    "rfd_plan_set_dechirp_fp64": [_P, _i32],
    "rfd_surrogate_set_feature_range": [_P, _P, _i64],
    "rfd_surrogate_features": [_P, _P, _i64, _P],
    "rfd_findchirp_prepare": [_P, _P, _i64, _P, _P],
    "findchirp_filter": [_P, _P, _P, _i64, _f, _i64, _P, _i64, C.POINTER(_i64)],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int
_lib.rfd_last_error.argtypes = []
_lib.rfd_last_error.restype = C.c_char_p

EXPORTED = sorted(list(_SIGS) + ["rfd_last_error"])


class RfdError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} -> {code}: {msg}")
        self.code = code


def rfd_last_error():
    return _lib.rfd_last_error().decode()


def _check(rc, fn):
    if rc != RFD_OK:
        raise RfdError(rc, fn, rfd_last_error())


def _ptr(t):
    """Device (or host numpy) pointer of a buffer, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


def _dev_check(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


# ------------------------------------------------------------------ plan
def rfd_plan_create(psd, f_low, fs, seg_len, max_refs=1, stream=None):
    psd = np.ascontiguousarray(psd, dtype=np.float64)
    h = _P()
    _check(_lib.rfd_plan_create(psd.ctypes.data, psd.size, f_low, fs, seg_len, max_refs, _stream(stream),
                                C.byref(h)), "rfd_plan_create")
    return h


def rfd_plan_info_get(plan):
    info = rfd_plan_info()
    _check(_lib.rfd_plan_info_get(plan, C.byref(info)), "rfd_plan_info_get")
    return {k: getattr(info, k) for k, _ in rfd_plan_info._fields_}


def rfd_plan_set_stream(plan, stream=None):
    _check(_lib.rfd_plan_set_stream(plan, _stream(stream)), "rfd_plan_set_stream")


def rfd_plan_set_timing(plan, enable=True):
    _check(_lib.rfd_plan_set_timing(plan, 1 if enable else 0), "rfd_plan_set_timing")


def rfd_plan_get_timing(plan):
    t = rfd_timing()
    _check(_lib.rfd_plan_get_timing(plan, C.byref(t)), "rfd_plan_get_timing")
    return {k: getattr(t, k) for k, _ in rfd_timing._fields_}


def _cfg_dict(c):
    return {k: getattr(c, k) for k, _ in rfd_fir_config._fields_}


def rfd_plan_set_fir_config(plan, col_blocks=8, mode=0, max_tiles=16, wg_per_cu=0, ols_block=0, ols_aligned=1):
    c = rfd_fir_config(col_blocks, mode, max_tiles, wg_per_cu, ols_block, ols_aligned)
    _check(_lib.rfd_plan_set_fir_config(plan, C.byref(c)), "rfd_plan_set_fir_config")


def rfd_plan_get_fir_config(plan):
    c = rfd_fir_config()
    _check(_lib.rfd_plan_get_fir_config(plan, C.byref(c)), "rfd_plan_get_fir_config")
    return _cfg_dict(c)


def rfd_ols_shape(plan, taps):
    """(K, L): overlap-save block size and outputs kept per block for `taps` taps."""
    k, l = C.c_int32(0), C.c_int32(0)
    _check(_lib.rfd_ols_shape(plan, taps, C.byref(k), C.byref(l)), "rfd_ols_shape")
    return k.value, l.value


def rfd_autotune_fir(plan, taps, precision, cluster_window, reps=3):
    r = rfd_tune_result()
    _check(_lib.rfd_autotune_fir(plan, taps, PRECISIONS.get(precision, precision), cluster_window, reps, C.byref(r)),
           "rfd_autotune_fir")
    return {"best": _cfg_dict(r.best), "best_ms": r.best_ms, "before_ms": r.before_ms,
            "n_candidates": r.n_candidates}


def rfd_segment_graph_create(plan, taps, precision, threshold, cluster_window, data, refs, out, capacity):
    """refs: {ref_id: complex128 device tensor}.  data: float64 device tensor [N] (read at replay)."""
    ids = np.array(sorted(refs), dtype=np.int32)
    ptrs = (C.c_void_p * len(ids))(*[refs[int(i)].data_ptr() for i in ids])
    g = _P()
    _check(_lib.rfd_segment_graph_create(plan, taps, PRECISIONS.get(precision, precision), threshold, cluster_window,
                                         _ptr(data), len(ids), ids.ctypes.data, ptrs, _ptr(out), capacity,
                                         C.byref(g)), "rfd_segment_graph_create")
    return g


def rfd_range_graph_create(plan, taps, precision, threshold, cluster_window, data, refs, n_start, n_len, out,
                           capacity):
    """As rfd_segment_graph_create, FIR and triggers over outputs [n_start, n_start + n_len) only."""
    ids = np.array(sorted(refs), dtype=np.int32)
    ptrs = (C.c_void_p * len(ids))(*[refs[int(i)].data_ptr() for i in ids])
    g = _P()
    _check(_lib.rfd_range_graph_create(plan, taps, PRECISIONS.get(precision, precision), threshold, cluster_window,
                                       _ptr(data), len(ids), ids.ctypes.data, ptrs, n_start, n_len, _ptr(out),
                                       capacity, C.byref(g)), "rfd_range_graph_create")
    return g


def rfd_segment_graph_launch(graph, want_count=True, raise_overflow=True):
    n = C.c_int64(0)
    rc = _lib.rfd_segment_graph_launch(graph, C.byref(n) if want_count else None)
    if rc == RFD_E_OVERFLOW and not raise_overflow:
        return n.value
    _check(rc, "rfd_segment_graph_launch")
    return n.value if want_count else None


def rfd_graph_destroy(graph):
    _check(_lib.rfd_graph_destroy(graph), "rfd_graph_destroy")


def rfd_plan_workspace_size(plan, max_templates, min_cluster_window=1, with_findchirp=False):
    b = C.c_size_t()
    _check(_lib.rfd_plan_workspace_size(plan, max_templates, min_cluster_window, 1 if with_findchirp else 0,
                                        C.byref(b)), "rfd_plan_workspace_size")
    return b.value


def rfd_plan_set_workspace(plan, workspace, max_templates=0, min_cluster_window=1, with_findchirp=False):
    """workspace: a device tensor the plan carves its per-call scratch from
    (kept alive by the caller), or None for library-owned scratch."""
    if workspace is None:
        _check(_lib.rfd_plan_set_workspace(plan, None, 0, 0, 1, 0), "rfd_plan_set_workspace")
        return
    nbytes = workspace.numel() * workspace.element_size()
    _check(_lib.rfd_plan_set_workspace(plan, _ptr(workspace), nbytes, max_templates, min_cluster_window,
                                       1 if with_findchirp else 0), "rfd_plan_set_workspace")


def rfd_measure_peaks(stream=None):
    """This GPU's measured ceilings: FP32 / FP64 FMA and BF16 MFMA TFLOP/s, copy GB/s."""
    out = np.zeros(4, dtype=np.float64)
    _check(_lib.rfd_measure_peaks(_stream(stream), out.ctypes.data), "rfd_measure_peaks")
    return {"fp32_fma_TFLOPs": float(out[0]), "fp64_fma_TFLOPs": float(out[1]), "bf16_mfma_TFLOPs": float(out[2]),
            "copy_GBs": float(out[3])}


def rfd_plan_destroy(plan):
    _check(_lib.rfd_plan_destroy(plan), "rfd_plan_destroy")


# --------------------------------------------------------------- dechirp
def rfd_dechirp(plan, data, h_ref, ref_id=0, want_sigma=True):
    """data: float64 [N] tensor or None; h_ref: complex128 [N/2+1] tensor."""
    import torch
    info = rfd_plan_info_get(plan)
    if data is not None:
        _dev_check(data, torch.float64, info["n"], "data")
    _dev_check(h_ref, torch.complex128, info["n_bins"], "h_ref")
    sig = C.c_double(0.0)
    _check(_lib.rfd_dechirp(plan, _ptr(data), _ptr(h_ref), ref_id, C.byref(sig) if want_sigma else None),
           "rfd_dechirp")
    return sig.value if want_sigma else None


def rfd_dechirp_refs(plan, data, refs, want_sigma=True):
    """data: float64 [N] tensor or None; refs: {ref_id: complex128 [N/2+1]
    tensor}.  Returns {ref_id: sigma_ref} (or None)."""
    import torch
    info = rfd_plan_info_get(plan)
    if data is not None:
        _dev_check(data, torch.float64, info["n"], "data")
    ids = sorted(refs)
    for r in ids:
        _dev_check(refs[r], torch.complex128, info["n_bins"], "h_ref")
    id_arr = (C.c_int32 * len(ids))(*ids)
    ptr_arr = (C.c_void_p * len(ids))(*[_ptr(refs[r]) for r in ids])
    sig = np.zeros(len(ids), dtype=np.float64)
    _check(_lib.rfd_dechirp_refs(plan, _ptr(data), len(ids), id_arr, ptr_arr,
                                 sig.ctypes.data if want_sigma else None), "rfd_dechirp_refs")
    return dict(zip(ids, sig.tolist())) if want_sigma else None


def rfd_get_zref(plan, ref_id, out=None):
    import torch
    info = rfd_plan_info_get(plan)
    if out is None:
        out = torch.empty(info["n"], dtype=torch.complex64, device="cuda")
    _dev_check(out, torch.complex64, info["n"], "out")
    _check(_lib.rfd_get_zref(plan, ref_id, _ptr(out)), "rfd_get_zref")
    return out


# ------------------------------------------------------------------ taps
def rfd_taps_create(plan, offsets, ref_id, taps, k0):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    nsb = offsets.size - 1
    ref_id = np.ascontiguousarray(ref_id, dtype=np.int32)
    taps = np.ascontiguousarray(taps, dtype=np.int32)
    k0 = np.ascontiguousarray(k0, dtype=np.int32)
    if not (ref_id.size == taps.size == k0.size == nsb):
        raise ValueError("offsets must have n_subbanks+1 entries and the others n_subbanks")
    h = _P()
    _check(_lib.rfd_taps_create(plan, nsb, offsets.ctypes.data, ref_id.ctypes.data, taps.ctypes.data,
                                k0.ctypes.data, C.byref(h)), "rfd_taps_create")
    return h


def rfd_make_taps(plan, taps, subbank, h_ref, h_tmpl, first=0, method=RFD_TAPS_LS, ridge_eps=1e-4):
    """h_ref: complex128 [N/2+1]; h_tmpl: complex128 [count, N/2+1] (templates first.. of the sub-bank)."""
    import torch
    info = rfd_plan_info_get(plan)
    _dev_check(h_ref, torch.complex128, info["n_bins"], "h_ref")
    if h_tmpl.dim() != 2 or h_tmpl.shape[1] != info["n_bins"]:
        raise ValueError("h_tmpl must be [count, N/2+1]")
    _dev_check(h_tmpl, torch.complex128, None, "h_tmpl")
    _check(_lib.rfd_make_taps(plan, taps, subbank, _ptr(h_ref), _ptr(h_tmpl), first, h_tmpl.shape[0], method,
                              ridge_eps), "rfd_make_taps")


def rfd_taps_get(taps, tmpl, max_taps=RFD_MAX_TAPS):
    a = np.zeros(max_taps, dtype=np.complex128)
    sig = C.c_double(0)
    T = C.c_int32(0)
    k0 = C.c_int32(0)
    _check(_lib.rfd_taps_get(taps, tmpl, a.ctypes.data, C.byref(sig), C.byref(T), C.byref(k0)), "rfd_taps_get")
    return a[:T.value].copy(), sig.value, T.value, k0.value


def rfd_taps_destroy(taps):
    _check(_lib.rfd_taps_destroy(taps), "rfd_taps_destroy")


# ---------------------------------------------------------------- filter
def _trigger_buffer(capacity):
    import torch
    return torch.empty(max(capacity, 1) * 32, dtype=torch.uint8, device="cuda")


def triggers_to_numpy(buf, n):
    if n <= 0:
        return np.zeros(0, dtype=TRIGGER_DTYPE)
    return buf[: n * 32].cpu().numpy().view(TRIGGER_DTYPE).copy()


def rfd_filter_bank(plan, taps, precision, threshold, cluster_window, capacity, out=None, raise_overflow=True):
    """Returns (trigger buffer, n).  precision: name or rfd_precision value."""
    prec = PRECISIONS.get(precision, precision)
    if out is None:
        out = _trigger_buffer(capacity)
    n = C.c_int64(0)
    rc = _lib.rfd_filter_bank(plan, taps, prec, threshold, cluster_window, _ptr(out), capacity, C.byref(n))
    if rc == RFD_E_OVERFLOW and not raise_overflow:
        return out, n.value
    _check(rc, "rfd_filter_bank")
    return out, n.value


def rfd_filter_bank_noalloc(plan, taps, precision, threshold, cluster_window, capacity, out, raise_overflow=True):
    """As rfd_filter_bank, with the library's static scratch (no device
    allocation inside the call).  `out` must be given: (out, n)."""
    prec = PRECISIONS.get(precision, precision)
    n = C.c_int64(0)
    rc = _lib.rfd_filter_bank_noalloc(plan, taps, prec, threshold, cluster_window, _ptr(out), capacity, C.byref(n))
    if rc == RFD_E_OVERFLOW and not raise_overflow:
        return out, n.value
    _check(rc, "rfd_filter_bank_noalloc")
    return out, n.value


def rfd_debug_fail_allocation(after):
    """The allocation after `after` further successful ones fails once (-1: off)."""
    _check(_lib.rfd_debug_fail_allocation(after), "rfd_debug_fail_allocation")


# ---------------------------------------------------------------- stream
def rfd_stream_create(plan, taps, refs, increment):
    """refs: {ref_id: dev complex128 tensor [N/2+1]}."""
    ids = sorted(refs)
    id_arr = (C.c_int32 * len(ids))(*ids)
    ptr_arr = (C.c_void_p * len(ids))(*[_ptr(refs[r]) for r in ids])
    h = C.c_void_p()
    _check(_lib.rfd_stream_create(plan, taps, len(ids), id_arr, ptr_arr, increment, C.byref(h)), "rfd_stream_create")
    return h


def rfd_stream_prime(stream, data):
    _check(_lib.rfd_stream_prime(stream, _ptr(data)), "rfd_stream_prime")


def rfd_stream_push(stream, data, precision, threshold, cluster_window, capacity, out=None, raise_overflow=True):
    """Returns (trigger buffer, n, first output position)."""
    prec = PRECISIONS.get(precision, precision)
    if out is None:
        out = _trigger_buffer(capacity)
    n, start = C.c_int64(0), C.c_int64(0)
    rc = _lib.rfd_stream_push(stream, _ptr(data), prec, threshold, cluster_window, _ptr(out), capacity, C.byref(n),
                              C.byref(start))
    if rc == RFD_E_OVERFLOW and not raise_overflow:
        return out, n.value, start.value
    _check(rc, "rfd_stream_push")
    return out, n.value, start.value


def rfd_stream_info(stream):
    head, lag, zlen = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    _check(_lib.rfd_stream_info(stream, C.byref(head), C.byref(lag), C.byref(zlen)), "rfd_stream_info")
    return {"head": head.value, "lag": lag.value, "zlen": zlen.value}


def rfd_stream_destroy(stream):
    _check(_lib.rfd_stream_destroy(stream), "rfd_stream_destroy")


def rfd_findchirp_prepare(plan, h_tmpl, filt=None, sigma=None):
    """FINDCHIRP filters of h_tmpl [count, N/2+1] into filt [count, n_band] (complex64)."""
    import torch
    info = rfd_plan_info_get(plan)
    _dev_check(h_tmpl, torch.complex128, None, "h_tmpl")
    count = h_tmpl.shape[0]
    if filt is None:
        filt = torch.empty((count, info["n_band"]), dtype=torch.complex64, device="cuda")
    _dev_check(filt, torch.complex64, count * info["n_band"], "filt")
    if sigma is None:
        sigma = torch.empty(count, dtype=torch.float64, device="cuda")
    _dev_check(sigma, torch.float64, count, "sigma")
    _check(_lib.rfd_findchirp_prepare(plan, _ptr(h_tmpl), count, _ptr(filt), _ptr(sigma)), "rfd_findchirp_prepare")
    return filt, sigma


def findchirp_filter(plan, data, filt, threshold, cluster_window, capacity, out=None, raise_overflow=True):
    import torch
    if data is not None:
        _dev_check(data, torch.float64, None, "data")
    _dev_check(filt, torch.complex64, None, "filt")
    if out is None:
        out = _trigger_buffer(capacity)
    n = C.c_int64(0)
    rc = _lib.findchirp_filter(plan, _ptr(data), _ptr(filt), filt.shape[0], threshold, cluster_window, _ptr(out),
                               capacity, C.byref(n))
    if rc == RFD_E_OVERFLOW and not raise_overflow:
        return out, n.value
    _check(rc, "findchirp_filter")
    return out, n.value


# ------------------------------------------------------------- surrogate
def rfd_surrogate_create(plan, taps, subbank, n_basis=64, hidden=256, seed=2601):
    h = _P()
    _check(_lib.rfd_surrogate_create(plan, taps, subbank, n_basis, hidden, seed, C.byref(h)), "rfd_surrogate_create")
    return h


def rfd_surrogate_fit_basis(sur, iters=20):
    cap = C.c_double(0)
    _check(_lib.rfd_surrogate_fit_basis(sur, iters, C.byref(cap)), "rfd_surrogate_fit_basis")
    return cap.value


def rfd_surrogate_train(sur, params, epochs, batch=256, lr=1e-3):
    """params: float32 device tensor [n_train, 4] (training templates, same order)."""
    import torch
    sizes = np.zeros(6, dtype=np.int64)
    _check(_lib.rfd_surrogate_get_state(sur, None, None, None, sizes.ctypes.data), "rfd_surrogate_get_state")
    _dev_check(params, torch.float32, 4 * (int(sizes[2]) // int(sizes[4])), "params")
    losses = np.zeros(epochs, dtype=np.float32)
    _check(_lib.rfd_surrogate_train(sur, _ptr(params), epochs, batch, lr, losses.ctypes.data), "rfd_surrogate_train")
    return losses


def rfd_surrogate_train_many(surs, params, epochs, batch=256, lr=1e-3):
    """Train len(surs) surrogates together; params[i]: float32 device tensor
    [n_train, 4] of surrogate i.  Returns losses [len(surs), epochs]."""
    import torch
    count = len(surs)
    if len(params) != count:
        raise ValueError("one parameter tensor per surrogate")
    for sur, prm in zip(surs, params):
        sizes = np.zeros(6, dtype=np.int64)
        _check(_lib.rfd_surrogate_get_state(sur, None, None, None, sizes.ctypes.data), "rfd_surrogate_get_state")
        _dev_check(prm, torch.float32, 4 * (int(sizes[2]) // int(sizes[4])), "params")
    hs = (C.c_void_p * max(count, 1))(*[C.c_void_p(s if isinstance(s, int) else getattr(s, "value", s))
                                        for s in surs])
    ps = (C.c_void_p * max(count, 1))(*[C.c_void_p(p.data_ptr()) for p in params])
    losses = np.zeros((count, epochs), dtype=np.float32)
    _check(_lib.rfd_surrogate_train_many(hs, ps, count, epochs, batch, lr, losses.ctypes.data),
           "rfd_surrogate_train_many")
    return losses


def rfd_surrogate_state(sur):
    sizes = np.zeros(6, dtype=np.int64)
    _check(_lib.rfd_surrogate_get_state(sur, None, None, None, sizes.ctypes.data), "rfd_surrogate_get_state")
    w = np.zeros(sizes[0], dtype=np.float32)
    b = np.zeros(sizes[1], dtype=np.float32)
    t = np.zeros(sizes[2], dtype=np.float32)
    _check(_lib.rfd_surrogate_get_state(sur, w.ctypes.data, b.ctypes.data, t.ctypes.data, None),
           "rfd_surrogate_get_state")
    D, K, H = int(sizes[3]), int(sizes[4]), int(sizes[5])
    return {"weights": w, "basis": b.reshape(K, D), "targets": t.reshape(-1, K), "D": D, "K": K, "H": H}


def rfd_surrogate_set_state(sur, weights=None, basis=None):
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    b = None if basis is None else np.ascontiguousarray(basis, dtype=np.float32)
    _check(_lib.rfd_surrogate_set_state(sur, None if w is None else w.ctypes.data,
                                        None if b is None else b.ctypes.data), "rfd_surrogate_set_state")


def rfd_surrogate_set_feature_range(sur, phys):
    """phys: dev float64 tensor [n, 4] (m1, m2, chi, e0) of the training set."""
    import torch
    _dev_check(phys, torch.float64, None, "phys")
    _check(_lib.rfd_surrogate_set_feature_range(sur, _ptr(phys), phys.shape[0]), "rfd_surrogate_set_feature_range")


def rfd_surrogate_features(sur, phys, out=None):
    """Scaled network inputs (dev float32 [n, 4]) of physical parameters (dev float64 [n, 4])."""
    import torch
    _dev_check(phys, torch.float64, None, "phys")
    if out is None:
        out = torch.empty((phys.shape[0], 4), dtype=torch.float32, device=phys.device)
    _check(_lib.rfd_surrogate_features(sur, _ptr(phys), phys.shape[0], _ptr(out)), "rfd_surrogate_features")
    return out


def rfd_surrogate_set_graphs(sur, enable=True):
    _check(_lib.rfd_surrogate_set_graphs(sur, 1 if enable else 0), "rfd_surrogate_set_graphs")


def rfd_surrogate_loss_grad(sur, params, targets=None):
    import torch
    sizes = np.zeros(6, dtype=np.int64)
    _check(_lib.rfd_surrogate_get_state(sur, None, None, None, sizes.ctypes.data), "rfd_surrogate_get_state")
    _dev_check(params, torch.float32, None, "params")
    if params.dim() != 2 or params.shape[1] != 4:
        raise ValueError("params must be [n, 4]")
    if targets is not None:
        _dev_check(targets, torch.float32, params.shape[0] * int(sizes[4]), "targets")
    g = torch.empty(int(sizes[0]), dtype=torch.float32, device="cuda")
    loss = C.c_double(0)
    _check(_lib.rfd_surrogate_loss_grad(sur, _ptr(params), _ptr(targets), params.shape[0], _ptr(g), C.byref(loss)),
           "rfd_surrogate_loss_grad")
    return loss.value, g.cpu().numpy()


def rfd_surrogate_make_taps(sur, params, target_taps, subbank, first=0):
    import torch
    _dev_check(params, torch.float32, None, "params")
    if params.dim() != 2 or params.shape[1] != 4:
        raise ValueError("params must be [count, 4]")
    _check(_lib.rfd_surrogate_make_taps(sur, _ptr(params), target_taps, subbank, first, params.shape[0]),
           "rfd_surrogate_make_taps")


def rfd_taps_match(taps_a, taps_b, subbank, first, count):
    import torch
    out = torch.empty(max(count, 1), dtype=torch.float64, device="cuda")
    _check(_lib.rfd_taps_match(taps_a, taps_b, subbank, first, count, _ptr(out)), "rfd_taps_match")
    return out[:count].cpu().numpy()


def rfd_taps_fallback(target, exact, subbank, first, match, min_match=0.99):
    """match: float64 device tensor [count]; returns the number of templates replaced."""
    import torch
    _dev_check(match, torch.float64, None, "match")
    n = C.c_int64(0)
    _check(_lib.rfd_taps_fallback(target, exact, subbank, first, match.numel(), _ptr(match), min_match, C.byref(n)),
           "rfd_taps_fallback")
    return n.value


def rfd_surrogate_destroy(sur):
    _check(_lib.rfd_surrogate_destroy(sur), "rfd_surrogate_destroy")


# ------------------------------------------------------------------ chi^2
def rfd_dechirp_bands(plan, h_ref, ref_id, n_bands):
    """Band series of slot ref_id; returns the band edges (int64 [n_bands + 1])."""
    import torch
    info = rfd_plan_info_get(plan)
    _dev_check(h_ref, torch.complex128, info["n_bins"], "h_ref")
    edges = np.zeros(n_bands + 1, dtype=np.int64)
    _check(_lib.rfd_dechirp_bands(plan, _ptr(h_ref), ref_id, n_bands, edges.ctypes.data), "rfd_dechirp_bands")
    return edges


def rfd_taps_band_fractions(plan, taps, subbank, h_ref, n_bands):
    import torch
    info = rfd_plan_info_get(plan)
    _dev_check(h_ref, torch.complex128, info["n_bins"], "h_ref")
    _check(_lib.rfd_taps_band_fractions(plan, taps, subbank, _ptr(h_ref), n_bands), "rfd_taps_band_fractions")


def rfd_taps_get_band_fractions(taps, tmpl, max_bands=64):
    f = np.zeros(max_bands, dtype=np.float32)
    p = C.c_int32(0)
    _check(_lib.rfd_taps_get_band_fractions(taps, tmpl, f.ctypes.data, C.byref(p)), "rfd_taps_get_band_fractions")
    return f[:p.value].copy()


def rfd_chisq(plan, taps, triggers, n):
    """chi^2 at the first n triggers of a device trigger buffer; float32 numpy [n]."""
    import torch
    out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    _check(_lib.rfd_chisq(plan, taps, _ptr(triggers), n, _ptr(out)), "rfd_chisq")
    return out[:n].cpu().numpy()


# ---------------------------------------------------------- tap selection
def rfd_select_taps(plan, h_ref, h_tmpl, target, ladder, ridge_eps=1e-4, centre=False):
    """Per-template tap counts reaching `target` (zero-lag match); returns
    (T int32 [count], match float64 [count]), and with centre=True (lags
    centred on each template's correlation peak) also k0 int32 [count]."""
    import torch
    info = rfd_plan_info_get(plan)
    _dev_check(h_ref, torch.complex128, info["n_bins"], "h_ref")
    if h_tmpl.dim() != 2 or h_tmpl.shape[1] != info["n_bins"]:
        raise ValueError("h_tmpl must be [count, N/2+1]")
    _dev_check(h_tmpl, torch.complex128, None, "h_tmpl")
    lad = np.ascontiguousarray(ladder, dtype=np.int32)
    count = h_tmpl.shape[0]
    T = np.zeros(count, dtype=np.int32)
    m = np.zeros(count, dtype=np.float64)
    k0 = np.zeros(count, dtype=np.int32)
    _check(_lib.rfd_select_taps(plan, _ptr(h_ref), _ptr(h_tmpl), count, target, lad.ctypes.data, lad.size,
                                ridge_eps, RFD_TAPS_CENTRE if centre else 0, T.ctypes.data, m.ctypes.data,
                                k0.ctypes.data), "rfd_select_taps")
    return (T, m, k0) if centre else (T, m)


# --------------------------------------------------------------- PSD drift
def rfd_plan_set_psd(plan, psd):
    psd = np.ascontiguousarray(psd, dtype=np.float64)
    _check(_lib.rfd_plan_set_psd(plan, psd.ctypes.data, psd.size), "rfd_plan_set_psd")


def rfd_taps_renormalize(plan, taps, subbank, h_ref):
    import torch
    info = rfd_plan_info_get(plan)
    _dev_check(h_ref, torch.complex128, info["n_bins"], "h_ref")
    _check(_lib.rfd_taps_renormalize(plan, taps, subbank, _ptr(h_ref)), "rfd_taps_renormalize")


# ------------------------------------------------------------ low latency
def rfd_filter_range(plan, taps, precision, threshold, cluster_window, n_start, n_len, capacity, out=None):
    prec = PRECISIONS.get(precision, precision)
    if out is None:
        out = _trigger_buffer(capacity)
    n = C.c_int64(0)
    _check(_lib.rfd_filter_range(plan, taps, prec, threshold, cluster_window, n_start, n_len, _ptr(out), capacity,
                                 C.byref(n)), "rfd_filter_range")
    return out, n.value


def rfd_plan_set_dechirp_fp64(plan, enable=True):
    """Reference transform passes in FP64 (True) or FP32 (False, the default)."""
    _check(_lib.rfd_plan_set_dechirp_fp64(plan, 1 if enable else 0), "rfd_plan_set_dechirp_fp64")
