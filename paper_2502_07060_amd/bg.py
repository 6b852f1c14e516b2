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
BG_MAX_N, BG_MAX_D = 14, 10
FP_SENTINEL = 0xFFFFFFFF

# every symbol include/bg.h declares, with its ctypes signature
_SIGNATURES = {
    "bg_amplitudes_c128": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "bg_amplitudes_fp": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
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


def bg_amplitudes_c128(momenta, pols, out=None, status=None, npts=None, stream=None, check=True):
    """M = eps_n . K([1..n-1]) per point over complex128.

    momenta, pols: complex128 tensors [n][d][ld] on the GPU.  Returns
    (out complex128 [npts], status uint8 [npts]).
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
    rc = lib().bg_amplitudes_c128(n, d, npts, ld, _ptr(momenta), _ptr(pols), _ptr(out), _ptr(status),
                                  _stream_ptr(stream))
    if check and rc != BG_OK:
        raise BGError(rc, "bg_amplitudes_c128")
    return out, status


def bg_amplitudes_fp(momenta, pols, p, out=None, status=None, npts=None, stream=None, check=True):
    """M mod p per point over Z_p.

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
    rc = lib().bg_amplitudes_fp(n, d, npts, ld, ctypes.c_uint32(p), _ptr(momenta), _ptr(pols), _ptr(out),
                                _ptr(status), _stream_ptr(stream))
    if check and rc != BG_OK:
        raise BGError(rc, "bg_amplitudes_fp")
    return out, status
