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


class ScfInfo(ctypes.Structure):
    _fields_ = [("e_tot", ctypes.c_double), ("e_1e", ctypes.c_double), ("e_j", ctypes.c_double),
                ("e_k", ctypes.c_double), ("err_norm", ctypes.c_double), ("d_e", ctypes.c_double),
                ("iter", ctypes.c_int), ("converged", ctypes.c_int)]


DFJK_SCF_C_VALID = 1


class Mol(ctypes.Structure):
    _fields_ = [("B", ctypes.c_void_p), ("nao", ctypes.c_int64), ("naux", ctypes.c_int64),
                ("ldB", ctypes.c_int64), ("nocc", ctypes.c_int64), ("D", ctypes.c_void_p),
                ("Cocc", ctypes.c_void_p), ("J", ctypes.c_void_p), ("K", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("diis_space", ctypes.c_int), ("conv_tol", ctypes.c_double),
                ("conv_tol_grad", ctypes.c_double), ("max_cycle", ctypes.c_int),
                ("compensated_j", ctypes.c_int), ("k16", ctypes.c_int), ("max_ncol", ctypes.c_int),
                ("max_ndm", ctypes.c_int)]


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
        L.dfjk_build_J_diag.argtypes = [vp, vp, vp, vp, vp]
        L.dfjk_build_J_static.argtypes = [vp, i32, i64, i64, i64, vp, ctypes.POINTER(Options), vp, vp, vp]
        L.dfjk_build_J_static.restype = i32
        L.dfjk_static_scratch_bytes.argtypes = []
        L.dfjk_static_scratch_bytes.restype = ctypes.c_size_t
        L.dfjk_build_J_multi.argtypes = [vp, i64, vp, vp, vp]
        L.dfjk_form_B.argtypes = [i64, i64, vp, vp, i64, vp]
        L.dfjk_build_K.argtypes = [vp, vp, i64, vp, vp]
        L.dfjk_build_K_factored.argtypes = [vp, vp, i64, vp, dbl, vp]
        L.dfjk_build_K_pair.argtypes = [vp, vp, vp, i64, i32, dbl, vp]
        L.dfjk_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.dfjk_update_B.argtypes = [vp]
        L.dfjk_update_B.restype = i32
        L.dfjk_destroy.argtypes = [vp]
        L.dfjk_destroy.restype = None
        L.dfjk_last_error.restype = ctypes.c_char_p
        L.dfjk_default_options.argtypes = [ctypes.POINTER(Options)]
        L.dfjk_default_options.restype = None
        L.dfjk_quantize.argtypes = [vp, vp, i32, i64, vp]
        L.dfjk_batch_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Mol), i32, i32, vp]
        for name in ("dfjk_batch_build", "dfjk_batch_capture", "dfjk_batch_launch"):
            getattr(L, name).argtypes = [vp]
        L.dfjk_batch_autotune.argtypes = [vp, i32, ctypes.c_char_p, ctypes.POINTER(dbl)]
        L.dfjk_batch_get_tile.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.dfjk_batch_set_tile.argtypes = [vp, i32, i32]
        L.dfjk_batch_set_k16.argtypes = [vp, i32]
        L.dfjk_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.dfjk_batch_destroy.argtypes = [vp]
        L.dfjk_batch_destroy.restype = None
        L.dfjk_batch_scf_guess.argtypes = [vp, ctypes.POINTER(vp)]
        L.dfjk_batch_scf_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(ScfInfo)]
        L.dfjk_batch_scf_reset.argtypes = [vp]
        for name in ("dfjk_batch_scf_guess", "dfjk_batch_scf_step", "dfjk_batch_scf_reset"):
            getattr(L, name).restype = i32
        for name in ("dfjk_batch_init", "dfjk_batch_build", "dfjk_batch_capture", "dfjk_batch_launch",
                     "dfjk_batch_autotune", "dfjk_batch_get_tile", "dfjk_batch_set_tile",
                     "dfjk_batch_set_k16", "dfjk_batch_workspace_bytes"):
            getattr(L, name).restype = i32
        L.dfjk_mlp_init.argtypes = [ctypes.POINTER(vp), i32, i32, i64, vp]
        L.dfjk_mlp_nparam.argtypes = [vp]
        L.dfjk_mlp_nparam.restype = i64
        fp = ctypes.POINTER(ctypes.c_float)
        L.dfjk_mlp_set_params.argtypes = [vp, fp]
        L.dfjk_mlp_get.argtypes = [vp, i32, fp]
        L.dfjk_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.dfjk_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp]
        L.dfjk_mlp_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        L.dfjk_mlp_set_compute.argtypes = [vp, i32]
        L.dfjk_mlp_set_compute.restype = i32
        L.dfjk_mlp_destroy.argtypes = [vp]
        L.dfjk_mlp_destroy.restype = None
        L.dfjk_guess_features.argtypes = [vp, vp, vp, i64, vp, vp]
        L.dfjk_guess_assemble.argtypes = [vp, vp, i64, vp, vp]
        L.dfjk_guess_target.argtypes = [vp, vp, i64, vp, vp]
        L.dfjk_guess_check.argtypes = [vp, i64, vp, vp]
        L.dfjk_gather_rows.argtypes = [vp, vp, i64, i32, vp, vp]
        for name in ("dfjk_guess_target", "dfjk_guess_check", "dfjk_gather_rows"):
            getattr(L, name).restype = i32
        for name in ("dfjk_mlp_init", "dfjk_mlp_set_params", "dfjk_mlp_get", "dfjk_mlp_forward",
                     "dfjk_mlp_loss_grad", "dfjk_mlp_adam", "dfjk_guess_features", "dfjk_guess_assemble"):
            getattr(L, name).restype = i32
        L.dfjk_scf_step.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.POINTER(ScfInfo)]
        L.dfjk_scf_reset.argtypes = [vp]
        L.dfjk_probe_mfma.argtypes = [i32, ctypes.POINTER(dbl)]
        L.dfjk_probe_mfma.restype = i32
        L.dfjk_probe_hbm_read.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(dbl)]
        L.dfjk_probe_hbm_read.restype = i32
        L.dfjk_aufbau.argtypes = [vp, vp, i64, vp, vp]
        L.dfjk_aufbau.restype = i32
        L.dfjk_tile_count.argtypes = [i32]
        L.dfjk_tile_info.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.dfjk_set_tile.argtypes = [vp, i32, i32]
        L.dfjk_profile.argtypes = [vp, i32]
        L.dfjk_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32), i32]
        for name in ("dfjk_scf_step", "dfjk_scf_reset", "dfjk_tile_count", "dfjk_tile_info", "dfjk_set_tile", "dfjk_profile", "dfjk_profile_read", "dfjk_init", "dfjk_build_J", "dfjk_build_K", "dfjk_build_K_factored", "dfjk_build_K_pair",
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


def dfjk_build_J_static(B, dtype: int, nao: int, naux: int, ldB: int, D, J, rho=None, stream=None,
                        opts: Options | None = None) -> int:
    """dfjk_build_J on the library's fixed scratch array (no device allocation)."""
    return _check("dfjk_build_J_static", lib().dfjk_build_J_static(
        _ptr(B), dtype, nao, naux, ldB, _stream(stream), ctypes.byref(opts) if opts else None, _ptr(D),
        _ptr(J), _ptr(rho)))


def dfjk_static_scratch_bytes() -> int:
    return int(lib().dfjk_static_scratch_bytes())


def dfjk_form_B(naux: int, ncol: int, M, Q, ldQ: int, stream=None) -> int:
    """B = L^-1 Q in place of Q, L = Cholesky factor of M (M overwritten)."""
    return _check("dfjk_form_B", lib().dfjk_form_B(naux, ncol, _ptr(M), _ptr(Q), ldQ, _stream(stream)))


def dfjk_build_J_multi(h, ndm: int, D, J, rho=None) -> int:
    return _check("dfjk_build_J_multi", lib().dfjk_build_J_multi(h, ndm, _ptr(D), _ptr(J), _ptr(rho)))


def dfjk_build_J_diag(h, D, J, rho, diag) -> int:
    return _check("dfjk_build_J_diag", lib().dfjk_build_J_diag(h, _ptr(D), _ptr(J), _ptr(rho), _ptr(diag)))


def dfjk_build_K(h, Cocc, nocc: int, D, K) -> int:
    return _check("dfjk_build_K", lib().dfjk_build_K(h, _ptr(Cocc), nocc, _ptr(D), _ptr(K)))


def dfjk_build_K_factored(h, C, ncol: int, sign, scale: float, K) -> int:
    return _check("dfjk_build_K_factored",
                  lib().dfjk_build_K_factored(h, _ptr(C), ncol, _ptr(sign), scale, _ptr(K)))


def dfjk_build_K_pair(h, L, R, ncol: int, sym: int, scale: float, K) -> int:
    return _check("dfjk_build_K_pair",
                  lib().dfjk_build_K_pair(h, _ptr(L), _ptr(R), ncol, sym, scale, _ptr(K)))


def dfjk_update_B(h) -> int:
    return _check("dfjk_update_B", lib().dfjk_update_B(h))


def dfjk_workspace_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check("dfjk_workspace_bytes", lib().dfjk_workspace_bytes(h, ctypes.byref(n)))
    return n.value


DFJK_TILE_GEMM1 = 0
DFJK_TILE_J_OUT = 1
DFJK_TILE_K16 = 2
DFJK_TILE_K16_SYRK = 3


def dfjk_scf_step(h, H, D, Cocc, nocc: int, flags: int = 0, want_info: bool = True):
    """One SCF iteration; returns (rc, ScfInfo or None)."""
    info = ScfInfo() if want_info else None
    rc = lib().dfjk_scf_step(h, _ptr(H), _ptr(D), _ptr(Cocc), nocc, flags,
                             ctypes.byref(info) if want_info else None)
    return _check("dfjk_scf_step", rc), info


def dfjk_aufbau(h, F, nocc: int, Cocc, D=None) -> int:
    return _check("dfjk_aufbau", lib().dfjk_aufbau(h, _ptr(F), nocc, _ptr(Cocc), _ptr(D)))


def dfjk_probe_hbm_read(buf, nbytes: int | None = None) -> float:
    """Sustained HBM read rate (GB/s) of a streaming kernel over a device tensor."""
    out = ctypes.c_double()
    n = buf.numel() * buf.element_size() if nbytes is None else nbytes
    _check("dfjk_probe_hbm_read", lib().dfjk_probe_hbm_read(_ptr(buf), n, ctypes.byref(out)))
    return out.value


def dfjk_probe_mfma(dtype: int) -> float:
    """Sustained matrix-core TFLOP/s for the dtype's instruction."""
    out = ctypes.c_double()
    _check("dfjk_probe_mfma", lib().dfjk_probe_mfma(dtype, ctypes.byref(out)))
    return out.value


def dfjk_scf_reset(h) -> int:
    return _check("dfjk_scf_reset", lib().dfjk_scf_reset(h))


def dfjk_tile_count(kernel: int = DFJK_TILE_GEMM1) -> int:
    return _check("dfjk_tile_count", lib().dfjk_tile_count(kernel))


def dfjk_tile_info(kernel: int, index: int):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check("dfjk_tile_info", lib().dfjk_tile_info(kernel, index, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def dfjk_set_tile(h, kernel: int, index: int) -> int:
    return _check("dfjk_set_tile", lib().dfjk_set_tile(h, kernel, index))


class Batch:
    """Batched J/K over molecules given as dicts with device tensors
    B (naux x ldB), D, J, K (nao x nao FP64), C (nao x nocc FP64)."""

    def __init__(self, mols, dtype: int, stream=None):
        self.mols = mols  # keep the tensors alive
        arr = (Mol * len(mols))()
        for i, m in enumerate(mols):
            B = m["B"]
            arr[i] = Mol(_ptr(B), m["nao"], B.shape[0], B.shape[1], m["C"].shape[1], _ptr(m["D"]),
                         _ptr(m["C"]), _ptr(m["J"]), _ptr(m["K"]))
        self.h = ctypes.c_void_p()
        _check("dfjk_batch_init", lib().dfjk_batch_init(ctypes.byref(self.h), arr, len(mols), dtype,
                                                         _stream(stream)))

    def build(self):
        return _check("dfjk_batch_build", lib().dfjk_batch_build(self.h))

    def capture(self):
        return _check("dfjk_batch_capture", lib().dfjk_batch_capture(self.h))

    def launch(self):
        return _check("dfjk_batch_launch", lib().dfjk_batch_launch(self.h))

    def autotune(self, reps: int = 3, cache_path: str | None = None):
        ms = (ctypes.c_double * 8)()
        _check("dfjk_batch_autotune", lib().dfjk_batch_autotune(
            self.h, reps, cache_path.encode() if cache_path else None, ms))
        return list(ms)

    def tile(self, bucket: int) -> int:
        t = ctypes.c_int()
        _check("dfjk_batch_get_tile", lib().dfjk_batch_get_tile(self.h, bucket, ctypes.byref(t)))
        return t.value

    def set_tile(self, bucket: int, tile: int):
        return _check("dfjk_batch_set_tile", lib().dfjk_batch_set_tile(self.h, bucket, tile))

    def set_k16(self, on: bool = True):
        """Exchange on the 16-bit matrix cores (BF16 / FP16 B only)."""
        return _check("dfjk_batch_set_k16", lib().dfjk_batch_set_k16(self.h, int(bool(on))))

    def _hlist(self, H_list):
        if len(H_list) != len(self.mols):
            raise ValueError("one H per molecule")
        return (ctypes.c_void_p * len(H_list))(*[_ptr(H) for H in H_list])

    def scf_guess(self, H_list):
        self._H = self._hlist(H_list)
        return _check("dfjk_batch_scf_guess", lib().dfjk_batch_scf_guess(self.h, self._H))

    def scf_step(self, H_list, want_info: bool = True):
        """One SCF iteration for every molecule; returns (rc, [ScfInfo] or None)."""
        self._H = self._hlist(H_list)
        info = (ScfInfo * len(self.mols))() if want_info else None
        rc = lib().dfjk_batch_scf_step(self.h, self._H, info)
        return _check("dfjk_batch_scf_step", rc), (list(info) if want_info else None)

    def scf_reset(self):
        return _check("dfjk_batch_scf_reset", lib().dfjk_batch_scf_reset(self.h))

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check("dfjk_batch_workspace_bytes", lib().dfjk_batch_workspace_bytes(self.h, ctypes.byref(n)))
        return n.value

    def close(self):
        if self.h:
            lib().dfjk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The learned-guess perceptron on the GPU (parameters live in the library)."""

    def __init__(self, d_in: int = 8, hidden: int = 256, max_batch: int = 65536, stream=None):
        import numpy as np
        self._np = np
        self.d_in, self.hidden = d_in, hidden
        self.h = ctypes.c_void_p()
        _check("dfjk_mlp_init", lib().dfjk_mlp_init(ctypes.byref(self.h), d_in, hidden, max_batch,
                                                     _stream(stream)))
        self.nparam = int(lib().dfjk_mlp_nparam(self.h))

    def shapes(self):
        H, d = self.hidden, self.d_in
        return [(H, d), (H,), (H, H), (H,), (1, H), (1,)]

    def set_params(self, flat):
        a = self._np.ascontiguousarray(flat, dtype=self._np.float32)
        assert a.size == self.nparam
        _check("dfjk_mlp_set_params", lib().dfjk_mlp_set_params(
            self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def _get(self, which):
        a = self._np.empty(self.nparam, dtype=self._np.float32)
        _check("dfjk_mlp_get", lib().dfjk_mlp_get(self.h, which, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a

    def params(self):
        return self._get(0)

    def grads(self):
        return self._get(1)

    def unflatten(self, flat):
        out, o = [], 0
        for s in self.shapes():
            n = int(self._np.prod(s))
            out.append(flat[o:o + n].reshape(s))
            o += n
        return out

    def forward(self, X, y):
        return _check("dfjk_mlp_forward", lib().dfjk_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(y)))

    def loss_grad(self, X, t, loss=None):
        return _check("dfjk_mlp_loss_grad", lib().dfjk_mlp_loss_grad(self.h, _ptr(X), _ptr(t), X.shape[0],
                                                                      _ptr(loss)))

    def set_compute(self, dtype: int):
        """DFJK_F32 (default) or DFJK_BF16 for the hidden-layer products."""
        return _check("dfjk_mlp_set_compute", lib().dfjk_mlp_set_compute(self.h, dtype))

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        return _check("dfjk_mlp_adam", lib().dfjk_mlp_adam(self.h, lr, b1, b2, eps))

    def close(self):
        if self.h:
            lib().dfjk_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dfjk_guess_features(H, Dcore, R, nao, X, stream=None):
    return _check("dfjk_guess_features", lib().dfjk_guess_features(_ptr(H), _ptr(Dcore), _ptr(R), nao,
                                                                    _ptr(X), _stream(stream)))


def dfjk_guess_assemble(y, Dcore, nao, D, stream=None):
    return _check("dfjk_guess_assemble", lib().dfjk_guess_assemble(_ptr(y), _ptr(Dcore), nao, _ptr(D),
                                                                    _stream(stream)))


def dfjk_guess_target(D, Dcore, nao, t, stream=None):
    return _check("dfjk_guess_target", lib().dfjk_guess_target(_ptr(D), _ptr(Dcore), nao, _ptr(t),
                                                                _stream(stream)))


def dfjk_guess_check(D, nao, out, stream=None):
    return _check("dfjk_guess_check", lib().dfjk_guess_check(_ptr(D), nao, _ptr(out), _stream(stream)))


def dfjk_gather_rows(X, idx, n, d, Y, stream=None):
    return _check("dfjk_gather_rows", lib().dfjk_gather_rows(_ptr(X), _ptr(idx), n, d, _ptr(Y),
                                                              _stream(stream)))


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

    def K_pair(self, L: torch.Tensor, R: torch.Tensor, sym: bool = False, scale: float = 1.0) -> torch.Tensor:
        """K of the density D = L R^T (plus its transpose when sym)."""
        K = torch.empty((self.nao, self.nao), dtype=torch.float64, device=L.device)
        dfjk_build_K_pair(self.h, L, R, L.shape[1], int(sym), scale, K)
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
