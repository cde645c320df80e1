"""ctypes binding of libdfjk (include/dfjk.h), argument marshalling only.

Every function takes torch tensors that already live on the GPU (PyTorch
supplies device memory and the stream) and passes their raw pointers to the
C-ABI function of the same name.  Nothing here computes; if the library is
missing, importing ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libdfjk.so")

DFJK_F64, DFJK_F32, DFJK_BF16, DFJK_F16 = 0, 1, 2, 3
DFJK_OK = 0
DFJK_W_NOT_CONVERGED = 1

_ELEM = {DFJK_F64: torch.float64, DFJK_F32: torch.float32, DFJK_BF16: torch.bfloat16,
         DFJK_F16: torch.float16}


class DFJKError(RuntimeError):
    def __init__(self, name: str, code: int, msg: str):
        super().__init__(f"{name} returned {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("diis_space", ctypes.c_int), ("conv_tol", ctypes.c_double),
                ("conv_tol_grad", ctypes.c_double), ("max_cycle", ctypes.c_int),
                ("compensated_j", ctypes.c_int)]


_lib = None


def lib():
    """Load libdfjk.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise OSError(f"{lib_path} not found: build it with paper_2506_06661_amd/build.py")
        L = ctypes.CDLL(lib_path)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.dfjk_init.argtypes = [ctypes.POINTER(vp), vp, i32, i64, i64, i64, vp, ctypes.POINTER(Options)]
        L.dfjk_build_J.argtypes = [vp, vp, vp, vp]
        L.dfjk_build_K.argtypes = [vp, vp, i64, vp, vp]
        L.dfjk_build_K_factored.argtypes = [vp, vp, i64, vp, dbl, vp]
        L.dfjk_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.dfjk_destroy.argtypes = [vp]
        L.dfjk_destroy.restype = None
        L.dfjk_last_error.restype = ctypes.c_char_p
        L.dfjk_default_options.argtypes = [ctypes.POINTER(Options)]
        L.dfjk_default_options.restype = None
        L.dfjk_quantize.argtypes = [vp, vp, i32, i64, vp]
        L.dfjk_tile_count.argtypes = [i32]
        L.dfjk_tile_info.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.dfjk_set_tile.argtypes = [vp, i32, i32]
        L.dfjk_profile.argtypes = [vp, i32]
        L.dfjk_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32), i32]
        for name in ("dfjk_tile_count", "dfjk_tile_info", "dfjk_set_tile", "dfjk_profile", "dfjk_profile_read", "dfjk_init", "dfjk_build_J", "dfjk_build_K", "dfjk_build_K_factored",
                     "dfjk_workspace_bytes", "dfjk_quantize"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def dfjk_last_error() -> str:
    return lib().dfjk_last_error().decode()


def _check(name: str, rc: int) -> int:
    if rc < 0:
        raise DFJKError(name, rc, dfjk_last_error())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def default_options() -> Options:
    o = Options()
    lib().dfjk_default_options(ctypes.byref(o))
    return o


def dfjk_init(B, dtype: int, nao: int, naux: int, ldB: int, stream=None, opts: Options | None = None):
    h = ctypes.c_void_p()
    _check("dfjk_init", lib().dfjk_init(ctypes.byref(h), _ptr(B), dtype, nao, naux, ldB,
                                         _stream(stream), ctypes.byref(opts) if opts else None))
    return h


def dfjk_build_J(h, D, J, rho=None) -> int:
    return _check("dfjk_build_J", lib().dfjk_build_J(h, _ptr(D), _ptr(J), _ptr(rho)))


def dfjk_build_K(h, Cocc, nocc: int, D, K) -> int:
    return _check("dfjk_build_K", lib().dfjk_build_K(h, _ptr(Cocc), nocc, _ptr(D), _ptr(K)))


def dfjk_build_K_factored(h, C, ncol: int, sign, scale: float, K) -> int:
    return _check("dfjk_build_K_factored",
                  lib().dfjk_build_K_factored(h, _ptr(C), ncol, _ptr(sign), scale, _ptr(K)))


def dfjk_workspace_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check("dfjk_workspace_bytes", lib().dfjk_workspace_bytes(h, ctypes.byref(n)))
    return n.value


DFJK_TILE_GEMM1 = 0


def dfjk_tile_count(kernel: int = DFJK_TILE_GEMM1) -> int:
    return _check("dfjk_tile_count", lib().dfjk_tile_count(kernel))


def dfjk_tile_info(kernel: int, index: int):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check("dfjk_tile_info", lib().dfjk_tile_info(kernel, index, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def dfjk_set_tile(h, kernel: int, index: int) -> int:
    return _check("dfjk_set_tile", lib().dfjk_set_tile(h, kernel, index))


PHASES = ("J", "J_rho", "J_out", "K", "K_gemm1", "K_syrk", "K_finish")


def dfjk_profile(h, capacity: int) -> int:
    return _check("dfjk_profile", lib().dfjk_profile(h, capacity))


def dfjk_profile_read(h) -> dict:
    """{phase: (total_ms, launches)} since the last read."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    _check("dfjk_profile_read", lib().dfjk_profile_read(h, ms, cnt, n))
    return {p: (ms[i], cnt[i]) for i, p in enumerate(PHASES)}


def dfjk_destroy(h) -> None:
    lib().dfjk_destroy(h)


def dfjk_quantize(src, dst, dtype: int, n: int, stream=None) -> int:
    return _check("dfjk_quantize", lib().dfjk_quantize(_ptr(src), _ptr(dst), dtype, n, _stream(stream)))


class Handle:
    """Owns a dfjk handle over a device-resident B (a torch tensor of shape
    (naux, ldB)) and allocates J/K outputs with torch."""

    def __init__(self, B: torch.Tensor, nao: int, dtype: int | None = None, stream=None,
                 opts: Options | None = None):
        if dtype is None:
            dtype = {v: k for k, v in _ELEM.items()}[B.dtype]
        if B.dtype != _ELEM[dtype]:
            raise ValueError(f"B has element type {B.dtype}, dtype {dtype} needs {_ELEM[dtype]}")
        self.B = B  # keep the borrowed buffer alive
        self.nao, self.naux, self.ldB = nao, B.shape[0], B.shape[1]
        self.dtype = dtype
        self.h = dfjk_init(B, dtype, nao, self.naux, self.ldB, stream, opts)

    def J(self, D: torch.Tensor, rho: torch.Tensor | None = None) -> torch.Tensor:
        J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=D.device)
        dfjk_build_J(self.h, D, J, rho)
        return J

    def K(self, C: torch.Tensor | None = None, D: torch.Tensor | None = None) -> torch.Tensor:
        dev = (C if C is not None else D).device
        K = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
        dfjk_build_K(self.h, C, 0 if C is None else C.shape[1], D, K)
        return K

    def workspace_bytes(self) -> int:
        return dfjk_workspace_bytes(self.h)

    def close(self) -> None:
        if self.h:
            dfjk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
