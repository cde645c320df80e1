"""Plain FP64 CPU oracle for the density-fitted J/K build and the SCF around it.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the GPU path (no kernels, headers, helpers or tables);
the only thing both sides use is the input generator in ``synth``.

Contents, each following the passage it cites:

* ``df_diagonal`` -- sum_P T[P, mu nu]^2 per packed pair (Sec. IV.C.2).
* ``form_B`` -- T = L^-1 Q from the metric Cholesky factor (Sec. IV.C.2).
* ``K_pair_rows`` -- row-sampled K of a two-factor density D = L R^T.
* ``rho``, ``J``, ``K_C``, ``K_D``, ``K_C_rows`` -- the J/K contractions of
  Sec. IV.C.2, Eq. eq:df:eri, written as plain loops in ``oracle.c``.
* ``energies`` -- E_J = 1/2 sum_P rho_P^2 = 1/2 tr(DJ) and E_K = -1/4 tr(DK).
* ``scf`` -- restricted closed-shell SCF with Pulay DIIS (the default
  accelerator of Sec. IV.B), core-Hamiltonian or user ``dm0`` start (Sec.
  IV.A.1: dm0 need not be idempotent), eigh via ``numpy.linalg.eigh``.
* ``quantize_bf16`` / ``quantize_f16`` -- one round-to-nearest-even step from
  FP64 to a 16-bit format (a reading: the paper fixes no reduced format).
* ``mlp_*`` -- FP64 forward/backward of the initial-guess network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile ``liboracle.so``: gcc -O2, OpenMP, no FMA contraction."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", _LIB, _SRC])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_rho.argtypes = [dp, i64, i64, i64, dp, dp]
        L.oracle_rho.restype = ctypes.c_int
        L.oracle_J_acc.argtypes = [dp, i64, i64, i64, dp, dp]
        L.oracle_J_acc.restype = ctypes.c_int
        L.oracle_K_C_acc.argtypes = [dp, i64, i64, i64, dp, i64, dp]
        L.oracle_K_C_acc.restype = ctypes.c_int
        L.oracle_K_D_acc.argtypes = [dp, i64, i64, i64, dp, dp]
        L.oracle_K_D_acc.restype = ctypes.c_int
        L.oracle_unpack.argtypes = [dp, i64, dp]
        L.oracle_K_C_rows.argtypes = [dp, i64, i64, i64, dp, i64, dp]
        L.oracle_K_C_rows.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for the following oracle calls."""
    lib().oracle_set_num_threads(int(n))


def nao_of(ldB_or_npair: int) -> int:
    n = int((np.sqrt(8 * ldB_or_npair + 1) - 1) / 2)
    return n


# ----------------------------------------------------------- J / K (Eq. eq:df:eri)
def rho(B: np.ndarray, nao: int, D: np.ndarray) -> np.ndarray:
    """rho_P = sum_{ka,la} B_P[ka,la] D[ka,la]."""
    B = _f64(B)
    D = _f64(D)
    out = np.empty(B.shape[0])
    if lib().oracle_rho(_dp(B), B.shape[1], nao, B.shape[0], _dp(D), _dp(out)) != 0:
        raise MemoryError("oracle_rho")
    return out


def J_acc(B: np.ndarray, nao: int, rho_: np.ndarray, J: np.ndarray) -> None:
    """J += sum_P rho_P B_P over the rows of this block of B."""
    B = _f64(B)
    if lib().oracle_J_acc(_dp(B), B.shape[1], nao, B.shape[0], _dp(_f64(rho_)), _dp(J)) != 0:
        raise MemoryError("oracle_J_acc")


def J(B: np.ndarray, nao: int, D: np.ndarray, return_rho: bool = False):
    """Coulomb matrix J = sum_P rho_P B_P."""
    r = rho(B, nao, D)
    out = np.zeros((nao, nao))
    J_acc(B, nao, r, out)
    return (out, r) if return_rho else out


def K_C_acc(B: np.ndarray, nao: int, C: np.ndarray, K: np.ndarray) -> None:
    B = _f64(B)
    C = _f64(C)
    rc = lib().oracle_K_C_acc(_dp(B), B.shape[1], nao, B.shape[0], _dp(C), C.shape[1], _dp(K))
    if rc != 0:
        raise MemoryError("oracle_K_C_acc")


def K_C(B: np.ndarray, nao: int, C: np.ndarray) -> np.ndarray:
    """Exchange for D = 2 C C^T: K = 2 sum_P (B_P C)(B_P C)^T."""
    out = np.zeros((nao, nao))
    K_C_acc(B, nao, C, out)
    return out


def K_D(B: np.ndarray, nao: int, D: np.ndarray) -> np.ndarray:
    """Exchange for any D: K = sum_P B_P D B_P."""
    B = _f64(B)
    out = np.zeros((nao, nao))
    rc = lib().oracle_K_D_acc(_dp(B), B.shape[1], nao, B.shape[0], _dp(_f64(D)), _dp(out))
    if rc != 0:
        raise MemoryError("oracle_K_D_acc")
    return out


def unpack(Brow: np.ndarray, nao: int) -> np.ndarray:
    out = np.empty((nao, nao))
    lib().oracle_unpack(_dp(_f64(Brow)), nao, _dp(out))
    return out


def K_C_rows(Bsel: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Exchange entries among a set of rows mu_r for D = 2CC^T, from the row
    slices Bsel[r, P, ka] = B_P[mu_r, ka]: returns Ksel[r, s] = K[mu_r, mu_s]."""
    Bsel = _f64(Bsel)
    C = _f64(C)
    nsel, naux, nao = Bsel.shape
    out = np.zeros((nsel, nsel))
    if lib().oracle_K_C_rows(_dp(Bsel), nsel, nao, naux, _dp(C), C.shape[1], _dp(out)) != 0:
        raise MemoryError("oracle_K_C_rows")
    return out


def K_pair_rows(Bsel: np.ndarray, L: np.ndarray, R: np.ndarray, sym: bool = False) -> np.ndarray:
    """Exchange entries among a set of rows mu_r for the two-factor density
    D = L R^T (plus R L^T when sym), from the row slices Bsel[r, P, ka] =
    B_P[mu_r, ka]: K[mu_r, mu_s] = sum_P sum_i (B_P L)[mu_r, i] (B_P R)[mu_s, i],
    i.e. sum_P (B_P D B_P) restricted to those rows (Sec. IV.C.2)."""
    Bsel = _f64(Bsel)
    XL = Bsel @ _f64(L)  # (nsel, naux, ncol)
    XR = Bsel @ _f64(R)
    nsel = Bsel.shape[0]
    out = np.zeros((nsel, nsel))
    for P in range(Bsel.shape[1]):  # plain sum over the auxiliary index
        out += XL[:, P, :] @ XR[:, P, :].T
    return out + out.T if sym else out


def form_B(M: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """The 3-index factor of Eq. eq:df:eri: M = L L^T (Cholesky of the
    auxiliary metric, lower L), T = L^-1 Q with Q the 3-index integrals
    (P|mu nu), one column per packed pair (Sec. IV.C.2)."""
    import scipy.linalg

    L = np.linalg.cholesky(_f64(M))
    return scipy.linalg.solve_triangular(L, _f64(Q), lower=True)


def df_diagonal(B: np.ndarray, nao: int) -> np.ndarray:
    """DF approximation of the diagonal integrals (mu nu|mu nu) = sum_P
    T[P, mu nu]^2, in packed pair order: the fitted half of the diagonal error
    measure of Sec. IV.C.2 (the exact half needs an integral engine)."""
    npair = nao * (nao + 1) // 2
    Bp = _f64(B)[:, :npair]
    out = np.zeros(npair)
    for P in range(Bp.shape[0]):  # plain sum over the auxiliary index
        out += Bp[P] * Bp[P]
    return out


def energies(rho_: np.ndarray, D: np.ndarray, K: np.ndarray):
    """E_J = 1/2 sum_P rho_P^2 and E_K = -1/4 tr(D K)."""
    return 0.5 * float(np.dot(rho_, rho_)), -0.25 * float(np.sum(D * K))


# ----------------------------------------------------------- reduced formats
def quantize_bf16(x: np.ndarray) -> np.ndarray:
    """One round-to-nearest-even step from FP64 to bfloat16 (8-bit exponent,
    7 stored mantissa bits, gradual underflow below 2^-126).  Returns the
    rounded values as FP64 (bfloat16 values are exact in FP64)."""
    return _quantize(x, emin=-126, mant=7, emax=127)


def quantize_f16(x: np.ndarray) -> np.ndarray:
    """One round-to-nearest-even step from FP64 to IEEE binary16 (5-bit
    exponent, 10 stored mantissa bits, subnormals below 2^-14)."""
    return _quantize(x, emin=-14, mant=10, emax=15)


def quantize_f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def _quantize(x, emin, mant, emax):
    x = np.asarray(x, np.float64)
    out = np.empty(x.shape, np.float64)
    xf, of = x.reshape(-1), out.reshape(-1)
    step = 1 << 16  # elementwise; pieces only keep the temporaries in cache
    for s in range(0, xf.size, step):
        of[s:s + step] = _quantize_piece(xf[s:s + step], emin, mant, emax)
    return out


def _quantize_piece(x, emin, mant, emax):
    _, e = np.frexp(x)  # x = f * 2^e, 0.5 <= |f| < 1, so the leading bit has weight 2^(e-1)
    lead = np.maximum(e - 1, emin)
    quantum = np.ldexp(1.0, lead - mant)
    r = np.rint(x / quantum) * quantum  # rint rounds half to even
    maxval = (2.0 - 2.0 ** -mant) * 2.0 ** emax
    r = np.where(np.abs(r) > maxval, np.copysign(np.inf, x), r)
    return np.where(x == 0, x, r)


def bf16_bits(q: np.ndarray) -> np.ndarray:
    """Bit patterns of values already rounded to bfloat16."""
    return (np.asarray(q, np.float64).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def f16_bits(q: np.ndarray) -> np.ndarray:
    """Bit patterns of values already rounded to binary16."""
    return np.asarray(q, np.float64).astype(np.float16).view(np.uint16)


# ----------------------------------------------------------- SCF (Sec. IV.A, IV.B)
DIIS_SPACE = 8


def aufbau(F: np.ndarray, nocc: int):
    """Lowest-nocc eigenvectors of symmetric F; D = 2 C C^T."""
    eps, U = np.linalg.eigh(F)
    C = np.ascontiguousarray(U[:, :nocc])
    return eps, C, 2.0 * C @ C.T


DIIS_MAX_COND = 1e12


def diis_prune(Fs, es, max_cond: float = DIIS_MAX_COND) -> int:
    """Drop the oldest stored (F, e) pairs, in place, while the Gram matrix
    <e_i, e_j> of the error vectors is worse conditioned than max_cond (2-norm
    condition number; a singular Gram matrix counts as infinitely bad).  At
    least one pair stays.  Returns the number dropped.  This is the reading
    taken of the DIIS the paper names as default (Sec. IV.B), which it does
    not detail: the usual safeguard against a near-singular subspace."""
    dropped = 0
    while len(es) > 1:
        G = np.array([[float(np.sum(a * b)) for b in es] for a in es])
        w = np.linalg.eigvalsh(G)
        if w[0] > 0 and w[-1] / w[0] <= max_cond:
            break
        Fs.pop(0)
        es.pop(0)
        dropped += 1
    return dropped


def diis_extrapolate(Fs, es):
    """Pulay DIIS: minimise |sum_i c_i e_i| subject to sum_i c_i = 1 via the
    bordered system [[<e_i,e_j>, -1], [-1, 0]] [c; lam] = [0; -1]."""
    m = len(Fs)
    A = np.zeros((m + 1, m + 1))
    for i in range(m):
        for j in range(m):
            A[i, j] = float(np.sum(es[i] * es[j]))
    A[:m, m] = -1.0
    A[m, :m] = -1.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    try:
        c = np.linalg.solve(A, rhs)[:m]
    except np.linalg.LinAlgError:
        c = np.zeros(m)
        c[-1] = 1.0
    F = np.zeros_like(Fs[0])
    for ci, Fi in zip(c, Fs):
        F += ci * Fi
    return F, c


def scf(B: np.ndarray, H: np.ndarray, nocc: int, dm0: np.ndarray | None = None,
        max_cycle: int = 100, conv_tol: float = 1e-9, conv_tol_grad: float = 3e-5,
        diis_space: int = DIIS_SPACE):
    """Restricted closed-shell SCF in an orthonormal AO basis (S = I).

    Iteration k with density D_k: J, K from D_k (K via C when D_k = 2CC^T);
    F = H + J - K/2; E_k = 1/2 tr(D_k (H + F)); e = F D - D F; DIIS over the
    last ``diis_space`` (F, e) pairs; aufbau on the extrapolated F gives
    D_{k+1}.  Converged when |E_k - E_{k-1}| < conv_tol and |e|_F <
    conv_tol_grad.  Returns a dict with per-iteration energies and error
    norms, the converged D and C, and the flag.
    """
    nao = H.shape[0]
    if dm0 is None:
        _, C, D = aufbau(H, nocc)
    else:
        C, D = None, _f64(dm0)
    Fs, es = [], []
    hist_E, hist_err = [], []
    E_prev = None
    converged = False
    for it in range(1, max_cycle + 1):
        Jm, r = J(B, nao, D, return_rho=True)
        Km = K_C(B, nao, C) if C is not None else K_D(B, nao, D)
        F = H + Jm - 0.5 * Km
        E = 0.5 * float(np.sum(D * (H + F)))
        err = F @ D - D @ F
        en = float(np.linalg.norm(err))
        hist_E.append(E)
        hist_err.append(en)
        Fs.append(F)
        es.append(err)
        if len(Fs) > diis_space:
            Fs.pop(0)
            es.pop(0)
        if E_prev is not None and abs(E - E_prev) < conv_tol and en < conv_tol_grad:
            converged = True
            break
        E_prev = E
        diis_prune(Fs, es)
        Fx, _ = diis_extrapolate(Fs, es)
        _, C, D = aufbau(Fx, nocc)
    return {"E": hist_E, "err": hist_err, "D": D, "C": C, "converged": converged,
            "iterations": len(hist_E)}


def builds_to(E_hist, E_ref: float, tol: float = 1e-6):
    """Number of J/K builds until |E_k - E_ref| < tol (None if never)."""
    for k, e in enumerate(E_hist):
        if abs(e - E_ref) < tol:
            return k + 1
    return None


# ----------------------------------------------------------- learned guess (FP64)
def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def mlp_forward(params, X):
    """Three linear layers with SiLU between: X (n, d_in) -> (n,)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y[:, 0], (X, z1, h1, z2, h2)


def mlp_loss_grad(params, X, t):
    """Mean squared error L = mean((y - t)^2) and its gradient by the chain
    rule, in FP64."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, h1, z2, h2) = mlp_forward(params, X)
    n = X.shape[0]
    L = float(np.mean((y - t) ** 2))
    gy = (2.0 / n) * (y - t)[:, None]            # (n, 1)
    gW3 = gy.T @ h2
    gb3 = gy.sum(0)
    gz2 = (gy @ W3) * dsilu(z2)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(0)
    gz1 = (gz2 @ W2) * dsilu(z1)
    gW1 = gz1.T @ X
    gb1 = gz1.sum(0)
    return L, [gW1, gb1, gW2, gb2, gW3, gb3]
