"""ctypes binding of libbg_mi355x.so (include/bg.h), same names as the C ABI.

Argument marshalling only: every step of the amplitude computation runs in
the library's HIP kernels.  Tensors are torch tensors on the GPU; the
binding checks dtype, shape and device, then passes raw device pointers and
the current HIP stream.  If the library has not been built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbg_mi355x.so")
_lib = None

BG_OK = 0
BG_EINVAL = -1
BG_EDOMAIN = -2
BG_ENOTPRIME = -3
BG_EHIP = -4
BG_ENOTIMPL = -5
BG_ENOMEM = -6
BG_EBUSY = -7
BG_PT_OK, BG_PT_SINGULAR, BG_PT_BADRESIDUE = 0, 1, 2
BG_FIELD_C128, BG_FIELD_FP = 0, 1
BG_METRIC_MOSTLY_MINUS, BG_METRIC_ALTERNATING = 0, 1
BG_MAX_N, BG_MAX_D = 14, 10
BG_BATCH_QUEUE = 1
(BG_PROBE_MAD_I64_I32, BG_PROBE_MAD_U64_U32, BG_PROBE_FMA_F64, BG_PROBE_MUL_LO_U32,
 BG_PROBE_DPP_MOV_B32) = range(5)
FP_SENTINEL = 0xFFFFFFFF

# every symbol include/bg.h declares, with its ctypes signature
_SIGNATURES = {
    "bg_amplitudes_c128": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "bg_amplitudes_fp": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_amplitudes_c128_metric": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_amplitudes_fp_metric": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                               ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_fp_from_rational": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_rational_reconstruct": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "bg_fp_contract": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_fp_divide": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_fp_divide_scalar": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_currents_c128": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "bg_currents_fp": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "bg_state_sum_c128": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "bg_state_sum_fp": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_states_c128": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "bg_states_fp": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "bg_variants": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "bg_select_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "bg_select_variant_metric": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int]),
    "bg_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_int64,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "bg_autotune_metric": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                          ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_void_p]),
    "bg_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "bg_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "bg_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "bg_batch_run_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "bg_batch_run_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "bg_batch_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "bg_batch_plan_create_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "bg_batch_plan_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bg_batch_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "bg_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]),
    "bg_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bg_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "bg_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p]),
    "bg_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bg_server_now_ns": (ctypes.c_int64, []),
    "bg_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "bg_issue_rate": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "bg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "bg_version": (ctypes.c_int, []),
}


class BGError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


def lib():
    """Load the shared library (no GPU access happens here)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with `python -m paper_2502_07060_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def library_path() -> str:
    return _LIB_PATH


def strerror(code: int) -> str:
    return lib().bg_strerror(int(code)).decode()


def bg_version() -> int:
    return lib().bg_version()


class bg_variant_info(ctypes.Structure):
    _fields_ = [("index", ctypes.c_int), ("lanes", ctypes.c_int), ("comps_per_lane", ctypes.c_int),
                ("lds_tables", ctypes.c_int), ("generic", ctypes.c_int), ("padded", ctypes.c_int),
                ("max_d", ctypes.c_int), ("selected", ctypes.c_int)]


def bg_variants(field: int, n: int, d: int):
    """List of dicts describing the kernels compiled for (field, n, d)."""
    cnt = lib().bg_variants(field, n, d, None, 0)
    if cnt < 0:
        raise BGError(cnt, "bg_variants")
    arr = (bg_variant_info * max(cnt, 1))()
    lib().bg_variants(field, n, d, ctypes.cast(arr, ctypes.c_void_p), cnt)
    return [{k: getattr(arr[i], k) for k, _ in bg_variant_info._fields_} for i in range(cnt)]


def bg_select_variant(field: int, n: int, d: int, index: int, metric=None) -> None:
    """Pin variant `index` for (field, n, d): for the mostly-minus metric, or
    for `metric` (BG_METRIC_*) when given."""
    if metric is None:
        rc = lib().bg_select_variant(field, n, d, index)
    else:
        rc = lib().bg_select_variant_metric(int(metric), field, n, d, index)
    if rc != BG_OK:
        raise BGError(rc, "bg_select_variant" if metric is None else "bg_select_variant_metric")


def bg_autotune(field: int, n: int, d: int, p: int = 0, npts: int = 1 << 18, reps: int = 5, stream=None,
                metric=None):
    """Time every variant for (field, n, d), pin the fastest; returns
    (chosen index, [(variant dict, ms per launch), ...]).  With `metric`
    (BG_METRIC_*) the launches run in that metric and the pin is that
    metric's (bg_autotune_metric)."""
    vs = bg_variants(field, n, d)
    ms = (ctypes.c_double * max(len(vs), 1))()
    if metric is None:
        rc = lib().bg_autotune(field, n, d, ctypes.c_uint32(p), npts, reps, ctypes.cast(ms, ctypes.c_void_p),
                               len(vs), _stream_ptr(stream))
    else:
        rc = lib().bg_autotune_metric(int(metric), field, n, d, ctypes.c_uint32(p), npts, reps,
                                      ctypes.cast(ms, ctypes.c_void_p), len(vs), _stream_ptr(stream))
    if rc < 0:
        raise BGError(rc, "bg_autotune" if metric is None else "bg_autotune_metric")
    return rc, [(v, ms[i]) for i, v in enumerate(vs)]


def bg_issue_rate(kind: int, blocks: int = 8192, iters: int = 2048, reps: int = 5, stream=None):
    """(lane-operations per second, ms per launch) of one instruction class
    (BG_PROBE_*) measured on the current device."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    rc = lib().bg_issue_rate(kind, blocks, iters, reps, ctypes.byref(rate), ctypes.byref(ms), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_issue_rate")
    return rate.value, ms.value


def bg_tune_save(path: str) -> None:
    rc = lib().bg_tune_save(path.encode())
    if rc != BG_OK:
        raise BGError(rc, "bg_tune_save")


def bg_tune_load(path: str) -> int:
    rc = lib().bg_tune_load(path.encode())
    if rc < 0:
        raise BGError(rc, "bg_tune_load")
    return rc


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_soa(name, t, n, d, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 3 or t.shape[0] != n or t.shape[1] != d or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous [n][d][ld], got {tuple(t.shape)}")
    return t.shape[2]


def bg_amplitudes_c128(momenta, pols, out=None, status=None, npts=None, stream=None, check=True,
                       metric=None):
    """M = eps_n . K([1..n-1]) per point over complex128.

    momenta, pols: complex128 tensors [n][d][ld] on the GPU.  Returns
    (out complex128 [npts], status uint8 [npts]).  ``metric`` (BG_METRIC_*)
    selects bg_amplitudes_c128_metric; None is the mostly-minus call.
    """
    import torch
    n, d = momenta.shape[0], momenta.shape[1]
    ld = _check_soa("momenta", momenta, n, d, torch.complex128)
    if _check_soa("pols", pols, n, d, torch.complex128) != ld:
        raise ValueError("momenta and pols must share ld")
    npts = ld if npts is None else int(npts)
    dev = momenta.device
    if out is None:
        out = torch.empty(npts, dtype=torch.complex128, device=dev)
    if status is None:
        status = torch.empty(npts, dtype=torch.uint8, device=dev)
    if metric is None:
        rc = lib().bg_amplitudes_c128(n, d, npts, ld, _ptr(momenta), _ptr(pols), _ptr(out), _ptr(status),
                                      _stream_ptr(stream))
    else:
        rc = lib().bg_amplitudes_c128_metric(int(metric), n, d, npts, ld, _ptr(momenta), _ptr(pols), _ptr(out),
                                             _ptr(status), _stream_ptr(stream))
    if check and rc != BG_OK:
        raise BGError(rc, "bg_amplitudes_c128" if metric is None else "bg_amplitudes_c128_metric")
    return out, status


def bg_amplitudes_c128_metric(metric, momenta, pols, **kw):
    """bg_amplitudes_c128 in the metric BG_METRIC_MOSTLY_MINUS or BG_METRIC_ALTERNATING."""
    return bg_amplitudes_c128(momenta, pols, metric=metric, **kw)


def bg_amplitudes_fp(momenta, pols, p, out=None, status=None, npts=None, stream=None, check=True,
                     metric=None):
    """M mod p per point over Z_p (``metric`` as for bg_amplitudes_c128).

    momenta, pols: tensors of uint32 residues [n][d][ld] (torch.uint32, or
    int32 holding the same bits).  Returns (out uint32-bits int32 [npts],
    status uint8 [npts]).
    """
    import torch
    n, d = momenta.shape[0], momenta.shape[1]
    dt = momenta.dtype
    if dt not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        raise TypeError("momenta must hold 32-bit residues")
    ld = _check_soa("momenta", momenta, n, d, dt)
    if _check_soa("pols", pols, n, d, dt) != ld:
        raise ValueError("momenta and pols must share ld")
    npts = ld if npts is None else int(npts)
    dev = momenta.device
    if out is None:
        out = torch.empty(npts, dtype=dt, device=dev)
    if status is None:
        status = torch.empty(npts, dtype=torch.uint8, device=dev)
    if metric is None:
        rc = lib().bg_amplitudes_fp(n, d, npts, ld, ctypes.c_uint32(p), _ptr(momenta), _ptr(pols), _ptr(out),
                                    _ptr(status), _stream_ptr(stream))
    else:
        rc = lib().bg_amplitudes_fp_metric(int(metric), n, d, npts, ld, ctypes.c_uint32(p), _ptr(momenta),
                                           _ptr(pols), _ptr(out), _ptr(status), _stream_ptr(stream))
    if check and rc != BG_OK:
        raise BGError(rc, "bg_amplitudes_fp" if metric is None else "bg_amplitudes_fp_metric")
    return out, status


def bg_amplitudes_fp_metric(metric, momenta, pols, p, **kw):
    """bg_amplitudes_fp in the metric BG_METRIC_MOSTLY_MINUS or BG_METRIC_ALTERNATING."""
    return bg_amplitudes_fp(momenta, pols, p, metric=metric, **kw)


# ----------------------------------------------------------------------------
# polarisation states
# ----------------------------------------------------------------------------

def _check_rows(name, t, rows, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.shape[0] != rows or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous [{rows}][ld], got {tuple(t.shape)}")
    return t.shape[1]


def bg_states_c128(momenta, chi, npts=None, stream=None):
    """States and duals of massless d-vectors over complex128.

    momenta: [d][ld], chi: [4][ld] complex128 on the GPU.  Returns views
    (eps [d-2][d][npts], epst [d-2][d][npts], status [npts]) of outputs laid
    out with the inputs' leading dimension."""
    import torch
    d = momenta.shape[0]
    ld = _check_rows("momenta", momenta, d, torch.complex128)
    if _check_rows("chi", chi, 4, torch.complex128) != ld:
        raise ValueError("momenta and chi must share ld")
    npts = ld if npts is None else int(npts)
    eps = torch.empty((max(d - 2, 0), d, ld), dtype=torch.complex128, device=momenta.device)
    epst = torch.empty_like(eps)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=momenta.device)
    rc = lib().bg_states_c128(d, npts, ld, _ptr(momenta), _ptr(chi), _ptr(eps), _ptr(epst), _ptr(st),
                              _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_states_c128")
    return eps[..., :npts], epst[..., :npts], st[:npts]


def bg_states_fp(momenta, chi, p, npts=None, stream=None):
    """States and duals of massless d-vectors over Z_p (p = 1 mod 4).

    momenta: [d][ld], chi: [4][ld] 32-bit residues on the GPU.  Returns
    views (eps [d-2][d][npts], epst [d-2][d][npts], status [npts])."""
    import torch
    d = momenta.shape[0]
    dt = momenta.dtype
    ld = _check_rows("momenta", momenta, d, dt)
    if _check_rows("chi", chi, 4, dt) != ld:
        raise ValueError("momenta and chi must share ld")
    npts = ld if npts is None else int(npts)
    eps = torch.empty((max(d - 2, 0), d, ld), dtype=dt, device=momenta.device)
    epst = torch.empty_like(eps)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=momenta.device)
    rc = lib().bg_states_fp(d, npts, ld, ctypes.c_uint32(p), _ptr(momenta), _ptr(chi), _ptr(eps), _ptr(epst),
                            _ptr(st), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_states_fp")
    return eps[..., :npts], epst[..., :npts], st[:npts]


# ----------------------------------------------------------------------------
# root currents and sums over the states of a cut leg
# ----------------------------------------------------------------------------

def bg_currents_c128(momenta, pols, npts=None, stream=None):
    """Root currents K([1..n-1]) over complex128: returns (cur [d][ld], status [npts])."""
    import torch
    n, d = momenta.shape[0], momenta.shape[1]
    ld = _check_soa("momenta", momenta, n, d, torch.complex128)
    if _check_soa("pols", pols, n, d, torch.complex128) != ld:
        raise ValueError("momenta and pols must share ld")
    npts = ld if npts is None else int(npts)
    cur = torch.empty((d, ld), dtype=torch.complex128, device=momenta.device)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=momenta.device)
    rc = lib().bg_currents_c128(n, d, npts, ld, _ptr(momenta), _ptr(pols), _ptr(cur), _ptr(st), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_currents_c128")
    return cur, st[:npts]


def bg_currents_fp(momenta, pols, p, npts=None, stream=None):
    """Root currents K([1..n-1]) mod p: returns (cur [d][ld] 32-bit, status [npts])."""
    import torch
    n, d = momenta.shape[0], momenta.shape[1]
    dt = momenta.dtype
    ld = _check_soa("momenta", momenta, n, d, dt)
    if _check_soa("pols", pols, n, d, dt) != ld:
        raise ValueError("momenta and pols must share ld")
    npts = ld if npts is None else int(npts)
    cur = torch.empty((d, ld), dtype=dt, device=momenta.device)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=momenta.device)
    rc = lib().bg_currents_fp(n, d, npts, ld, ctypes.c_uint32(p), _ptr(momenta), _ptr(pols), _ptr(cur), _ptr(st),
                              _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_currents_fp")
    return cur, st[:npts]


def bg_state_sum(kl, kr, eps, epst, p=None, npts=None, stream=None):
    """sum_s (e_s . K_L)(e~_s . K_R) per point: kl, kr [d][ld]; eps, epst
    [d-2][d][ld] (complex128, or 32-bit residues with prime p)."""
    import torch
    d, ld = kl.shape
    npts = ld if npts is None else int(npts)
    for name, t in (("kl", kl), ("kr", kr), ("eps", eps), ("epst", epst)):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != kl.dtype or t.shape[-1] != ld:
            raise TypeError(f"{name}: contiguous HIP tensor of kl's dtype and ld")
    out = torch.empty(max(ld, 1), dtype=kl.dtype, device=kl.device)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=kl.device)
    if kl.dtype == torch.complex128:
        rc = lib().bg_state_sum_c128(d, npts, ld, _ptr(kl), _ptr(kr), _ptr(eps), _ptr(epst), _ptr(out), _ptr(st),
                                     _stream_ptr(stream))
        name = "bg_state_sum_c128"
    else:
        rc = lib().bg_state_sum_fp(d, npts, ld, ctypes.c_uint32(p), _ptr(kl), _ptr(kr), _ptr(eps), _ptr(epst),
                                   _ptr(out), _ptr(st), _stream_ptr(stream))
        name = "bg_state_sum_fp"
    if rc != BG_OK:
        raise BGError(rc, name)
    return out[:npts], st[:npts]


# ----------------------------------------------------------------------------
# from Z_p samples back to rationals
# ----------------------------------------------------------------------------

BG_RR_MAX_PRIMES = 32


def bg_rr_limbs(nprimes: int) -> int:
    """Limbs per value of bg_rational_reconstruct's outputs (BG_RR_LIMBS)."""
    return (nprimes + 2) // 2


def bg_fp_from_rational(p, num, den, out=None, status=None, stream=None):
    """num / den mod p elementwise for int64 device tensors of one shape;
    returns (out uint32 bits in int32, status uint8) of the same shape."""
    import torch
    if num.dtype != torch.int64 or den.dtype != torch.int64 or num.shape != den.shape:
        raise TypeError("num and den must be int64 tensors of one shape")
    if not (num.is_cuda and den.is_cuda and num.is_contiguous() and den.is_contiguous()):
        raise TypeError("num and den must be contiguous HIP tensors")
    if out is None:
        out = torch.empty(num.shape, dtype=torch.int32, device=num.device)
    if status is None:
        status = torch.empty(num.shape, dtype=torch.uint8, device=num.device)
    rc = lib().bg_fp_from_rational(ctypes.c_uint32(p), num.numel(), _ptr(num), _ptr(den), _ptr(out),
                                   _ptr(status), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_fp_from_rational")
    return out, status


def bg_rational_reconstruct(primes, residues, npts=None, stream=None):
    """Rationals from residues [nprimes][ld] (32-bit, one row per prime).
    Returns (num int32 [L][npts] two's complement limbs, den int32 [L][npts]
    holding uint32 limbs, status uint8 [npts]); L = bg_rr_limbs(nprimes)."""
    import torch
    k = len(primes)
    if residues.dim() != 2 or residues.shape[0] != k or not residues.is_contiguous():
        raise ValueError("residues must be a contiguous [nprimes][ld] tensor")
    if residues.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        raise TypeError("residues must hold 32-bit values")
    ld = residues.shape[1]
    npts = ld if npts is None else int(npts)
    L = bg_rr_limbs(k)
    num = torch.zeros((L, max(ld, 1)), dtype=torch.int32, device=residues.device)
    den = torch.zeros_like(num)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=residues.device)
    parr = (ctypes.c_uint32 * max(k, 1))(*[int(p) for p in primes])
    rc = lib().bg_rational_reconstruct(k, ctypes.cast(parr, ctypes.c_void_p), npts, ld, _ptr(residues), _ptr(num),
                                       _ptr(den), _ptr(st), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_rational_reconstruct")
    return num[:, :npts], den[:, :npts], st[:npts]


def limbs_to_ints(limbs, signed: bool):
    """Python ints from a host array of 32-bit limbs [L][npts] (least
    significant first), two's complement when signed."""
    import numpy as np
    a = np.asarray(limbs).astype(np.uint32)
    L = a.shape[0]
    out = []
    for q in range(a.shape[1]):
        v = 0
        for k in range(L - 1, -1, -1):
            v = (v << 32) | int(a[k, q])
        if signed and v >> (32 * L - 1):
            v -= 1 << (32 * L)
        out.append(v)
    return out


# ----------------------------------------------------------------------------
# standalone Z_p operations
# ----------------------------------------------------------------------------

BG_FP_MAX_DIM = 4096


def _u32(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous HIP tensor")
    if t.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        raise TypeError(f"{name} must hold 32-bit residues")


def bg_fp_contract(p, x, y, y_batched=True, npts=None, stream=None):
    """z[i][k][q] = sum_j x[i][j][q] y[j][k](q) mod p.  x: [I][J][ld];
    y: [J][K][ld] (batched) or [J][K] (shared).  Returns (z [I][K][ld], status [npts])."""
    import torch
    _u32(x, "x")
    _u32(y, "y")
    I, J, ld = x.shape
    if y_batched:
        if y.dim() != 3 or y.shape[0] != J or y.shape[2] != ld:
            raise ValueError("y must be [J][K][ld]")
    elif y.dim() != 2 or y.shape[0] != J:
        raise ValueError("y must be [J][K]")
    K = y.shape[1]
    npts = ld if npts is None else int(npts)
    z = torch.empty((I, K, ld), dtype=x.dtype, device=x.device)
    st = torch.empty(max(ld, 1), dtype=torch.uint8, device=x.device)
    rc = lib().bg_fp_contract(ctypes.c_uint32(p), I, J, K, npts, ld, _ptr(x), _ptr(y), 1 if y_batched else 0,
                              _ptr(z), _ptr(st), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_fp_contract")
    return z, st[:npts]


def bg_fp_divide(p, x, y, stream=None):
    """Elementwise x / y mod p (y a tensor of x's shape, or a Python int);
    returns (z, status) of x's shape."""
    import torch
    _u32(x, "x")
    z = torch.empty_like(x)
    st = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    if isinstance(y, int):
        rc = lib().bg_fp_divide_scalar(ctypes.c_uint32(p), x.numel(), _ptr(x), ctypes.c_uint32(y), _ptr(z),
                                       _ptr(st), _stream_ptr(stream))
        name = "bg_fp_divide_scalar"
    else:
        _u32(y, "y")
        if y.shape != x.shape:
            raise ValueError("x and y must have one shape")
        rc = lib().bg_fp_divide(ctypes.c_uint32(p), x.numel(), _ptr(x), _ptr(y), _ptr(z), _ptr(st),
                                _stream_ptr(stream))
        name = "bg_fp_divide"
    if rc != BG_OK:
        raise BGError(rc, name)
    return z, st


# ----------------------------------------------------------------------------
# batched form
# ----------------------------------------------------------------------------

class bg_group(ctypes.Structure):
    _fields_ = [("field", ctypes.c_int), ("n", ctypes.c_int), ("d", ctypes.c_int), ("p", ctypes.c_uint32),
                ("npts", ctypes.c_int64), ("ld", ctypes.c_int64), ("momenta", ctypes.c_void_p),
                ("pols", ctypes.c_void_p), ("out", ctypes.c_void_p), ("status", ctypes.c_void_p)]


def make_group(momenta, pols, out, status=None, p=0, npts=None):
    """A bg_group for device tensors laid out as for bg_amplitudes_* (field
    from the dtype: complex128 -> C, 32-bit integers -> F_p with prime p)."""
    import torch
    n, d, ld = momenta.shape
    field = BG_FIELD_C128 if momenta.dtype == torch.complex128 else BG_FIELD_FP
    return bg_group(field, n, d, p if field == BG_FIELD_FP else 0, ld if npts is None else int(npts), ld,
                    momenta.data_ptr(), pols.data_ptr(), out.data_ptr(),
                    status.data_ptr() if status is not None else None)


def _group_array(groups):
    arr = (bg_group * max(len(groups), 1))(*groups)
    return arr


def bg_batch_run(groups, stream=None) -> None:
    arr = _group_array(groups)
    rc = lib().bg_batch_run(ctypes.cast(arr, ctypes.c_void_p), len(groups), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_batch_run")


def bg_batch_run_ex(groups, flags=0, stream=None) -> None:
    arr = _group_array(groups)
    rc = lib().bg_batch_run_ex(ctypes.cast(arr, ctypes.c_void_p), len(groups), int(flags), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_batch_run_ex")


def bg_batch_run_noalloc(groups, stream=None) -> None:
    arr = _group_array(groups)
    rc = lib().bg_batch_run_noalloc(ctypes.cast(arr, ctypes.c_void_p), len(groups), _stream_ptr(stream))
    if rc != BG_OK:
        raise BGError(rc, "bg_batch_run_noalloc")


class BatchPlan:
    """A recorded batch (hipGraph); launch() replays it on a stream."""

    def __init__(self, groups, flags=0):
        self._groups = _group_array(groups)   # keep the descriptors alive with the plan
        self._h = ctypes.c_void_p()
        rc = lib().bg_batch_plan_create_ex(ctypes.cast(self._groups, ctypes.c_void_p), len(groups), int(flags),
                                           ctypes.byref(self._h))
        if rc != BG_OK:
            raise BGError(rc, "bg_batch_plan_create_ex")

    def launch(self, stream=None) -> None:
        rc = lib().bg_batch_plan_launch(self._h, _stream_ptr(stream))
        if rc != BG_OK:
            raise BGError(rc, "bg_batch_plan_launch")

    def close(self) -> None:
        if self._h:
            lib().bg_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# serving loop
# ----------------------------------------------------------------------------

BG_SERVER_PLAIN = 1


class bg_request_times(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64),
                ("batch_requests", ctypes.c_int32)]


class bg_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "rejected", "batches", "points", "queued",
                                               "inflight_batches", "arena_bytes", "arena_in_use", "arena_peak")]


def _host_ptr(x):
    """Address of a host buffer: a CPU torch tensor or a numpy array (contiguous)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        if x.is_cuda or not x.is_contiguous():
            raise ValueError("server requests take contiguous host tensors")
        return x.data_ptr()
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("server requests take contiguous host arrays")
    return x.ctypes.data


def _is_complex(x):
    return str(x.dtype).endswith("complex128")


def bg_server_now_ns() -> int:
    return lib().bg_server_now_ns()


class Server:
    """A serving loop on the current device (bg_server_*).  Requests are host
    buffers laid out as for bg_amplitudes_*: momenta and pols [n][d][ld],
    out [npts], status [npts]; pinned torch tensors let copies overlap."""

    def __init__(self, hbm_budget_bytes: int, plain: bool = False):
        self._h = ctypes.c_void_p()
        rc = lib().bg_server_create(int(hbm_budget_bytes), BG_SERVER_PLAIN if plain else 0, ctypes.byref(self._h))
        if rc != BG_OK:
            raise BGError(rc, "bg_server_create")
        self._live = {}

    def submit(self, momenta, pols, out, status=None, p: int = 0, npts=None) -> int:
        n, d, ld = momenta.shape
        field = BG_FIELD_C128 if _is_complex(momenta) else BG_FIELD_FP
        g = bg_group(field, n, d, p if field == BG_FIELD_FP else 0, ld if npts is None else int(npts), ld,
                     _host_ptr(momenta), _host_ptr(pols), _host_ptr(out), _host_ptr(status))
        rid = ctypes.c_uint64()
        rc = lib().bg_server_submit(self._h, ctypes.byref(g), ctypes.byref(rid))
        if rc != BG_OK:
            raise BGError(rc, "bg_server_submit")
        self._live[rid.value] = (momenta, pols, out, status)   # the buffers outlive the request
        return rid.value

    def poll(self, rid: int) -> bool:
        rc = lib().bg_server_poll(self._h, rid)
        if rc < 0:
            raise BGError(rc, "bg_server_poll")
        return rc == 1

    def wait(self, rid: int, timeout: float = -1.0):
        """Waits for a request; returns its times (dict) and forgets it."""
        t = bg_request_times()
        rc = lib().bg_server_wait(self._h, rid, float(timeout), ctypes.byref(t))
        if rc == BG_EBUSY:
            raise TimeoutError(f"request {rid} not done after {timeout} s")
        self._live.pop(rid, None)
        if rc != BG_OK:
            raise BGError(rc, "bg_server_wait")
        return {k: getattr(t, k) for k, _ in bg_request_times._fields_}

    def stats(self) -> dict:
        s = bg_server_stats()
        rc = lib().bg_server_get_stats(self._h, ctypes.byref(s))
        if rc != BG_OK:
            raise BGError(rc, "bg_server_get_stats")
        return {k: getattr(s, k) for k, _ in bg_server_stats._fields_}

    def close(self) -> None:
        if self._h:
            lib().bg_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
