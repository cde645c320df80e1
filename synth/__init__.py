"""Seeded synthetic systems for the density-fitted J/K build.

Shared input source for the oracle and the GPU path.  Nothing here computes
J, K, energies or any step of the SCF: it draws random numbers (Philox-4x32-10
in ``synth.c``), places basis functions on lattices, and fills B, C_occ and H
with the distributions below.

Workloads (synthetic stand-ins for the paper's 50-100 atom density-fitting
workloads of Sec. III, whose geometries and basis sets are not available):

* ``c1``  nao=64,   naux=256,  nocc=16;  4x4x4 cubic lattice, 1.5 bohr, one
  function per site.
* ``c2``  nao=1024, naux=4096, nocc=200; 16x8x8 lattice, three functions on
  each of sites 0..339 and one on each of sites 340..343.
* ``c3``  nao=2048, naux=8192, nocc=400; 16x16x8 lattice, one per site.
* ``c4``  batches of molecules, nao ~ U{40..400}, naux=4*nao, nocc=nao//5,
  each a connected cluster grown breadth-first on a 10x10x10 lattice.
* ``c5``  nao=128, naux=512, nocc=24; 8x4x4 lattice with N(0, 0.1) bohr
  jitter and a core Hamiltonian H = -diag(U(1,5)) + 0.1 exp(-r^2) N(0,1).

B[P, mu nu] = a_P exp(-|R_mu - R_nu|^2 / 2) z, a_P ~ U(0.1, 1), z ~ N(0, 1),
symmetric in mu, nu (one draw per packed pair), stored as rows of the packed
lower triangle p(mu, nu) = nu(nu+1)/2 + mu (mu <= nu).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

SPACING = 1.5  # bohr

# stream ids (B uses 1 and 2 inside synth.c)
STREAM_COCC = 3
STREAM_H_DIAG = 4
STREAM_H_OFF = 5
STREAM_JITTER = 6
STREAM_BATCH = 7
STREAM_MLP = 8
STREAM_METRIC = 9
STREAM_ROT = 10


def build() -> str:
    """Compile ``libsynth.so`` with gcc (OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.synth_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                    ctypes.c_int64, dp]
        L.synth_normal.argtypes = L.synth_uniform.argtypes
        L.synth_B_rows.argtypes = [ctypes.c_uint64, ctypes.c_int64, dp, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int64, dp]
        L.synth_B_cols.argtypes = [ctypes.c_uint64, ctypes.c_int64, dp, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox(ctr, key):
    """Raw Philox-4x32-10 block (for known-answer tests)."""
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().synth_philox4x32_10(c, k, o)
    return list(o)


def uniform(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, np.float64)
    lib().synth_uniform(seed, stream, start, n, _dp(out))
    return out


def normal(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, np.float64)
    lib().synth_normal(seed, stream, start, n, _dp(out))
    return out


def npair(nao: int) -> int:
    return nao * (nao + 1) // 2


def pair_index(mu, nu):
    """Packed position of the pair (mu, nu): lower triangle, row max(mu,nu)."""
    a = np.maximum(mu, nu)
    b = np.minimum(mu, nu)
    return a * (a + 1) // 2 + b


# ---------------------------------------------------------------- lattices
def lattice(nx: int, ny: int, nz: int) -> np.ndarray:
    """Sites of an nx*ny*nz cubic lattice, index (ix*ny + iy)*nz + iz."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return SPACING * np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)


def positions_c1() -> np.ndarray:
    return lattice(4, 4, 4)


def positions_c2() -> np.ndarray:
    """16x8x8 lattice; 3 functions on each of the first 340 sites (1020) and
    one on each of sites 340..343 (4): nao = 1024."""
    sites = lattice(16, 8, 8)
    return np.ascontiguousarray(np.concatenate([np.repeat(sites[:340], 3, axis=0), sites[340:344]]))


def positions_c3() -> np.ndarray:
    return lattice(16, 16, 8)


def positions_c5(seed: int) -> np.ndarray:
    base = lattice(8, 4, 4)
    return np.ascontiguousarray(base + 0.1 * normal(seed, STREAM_JITTER, base.size).reshape(base.shape))


def cluster_positions(seed: int, nao: int, box: int = 10) -> np.ndarray:
    """A connected cluster of nao sites grown breadth-first on a box^3 lattice
    from a random start site; neighbours are queued in a seeded random order."""
    assert 1 <= nao <= box ** 3
    u = uniform(seed, STREAM_BATCH, 1 + 6 * box ** 3)
    start = int(u[0] * box ** 3)
    seen = np.zeros(box ** 3, bool)
    order = [start]
    seen[start] = True
    head = 0
    k = 1
    steps = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    while len(order) < nao:
        s = order[head]
        head += 1
        x, y, z = s // (box * box), (s // box) % box, s % box
        perm = np.argsort(u[k:k + 6], kind="stable")
        k += 6
        for d in perm:
            nx_, ny_, nz_ = x + steps[d, 0], y + steps[d, 1], z + steps[d, 2]
            if 0 <= nx_ < box and 0 <= ny_ < box and 0 <= nz_ < box:
                t = (nx_ * box + ny_) * box + nz_
                if not seen[t]:
                    seen[t] = True
                    order.append(t)
                    if len(order) == nao:
                        break
    idx = np.array(order[:nao])
    return np.ascontiguousarray(SPACING * np.stack([idx // (box * box), (idx // box) % box, idx % box],
                                                   axis=1).astype(np.float64))


# ---------------------------------------------------------------- tensors
def B_rows(seed: int, R: np.ndarray, P0: int, nrows: int, ldB: int | None = None) -> np.ndarray:
    nao = R.shape[0]
    ld = npair(nao) if ldB is None else ldB
    assert ld >= npair(nao)
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.empty((nrows, ld), np.float64)
    lib().synth_B_rows(seed, nao, _dp(R), P0, nrows, ld, _dp(out))
    return out


def B_full(seed: int, R: np.ndarray, naux: int, ldB: int | None = None) -> np.ndarray:
    return B_rows(seed, R, 0, naux, ldB)


def B_cols(seed: int, R: np.ndarray, naux: int, cols) -> np.ndarray:
    """B[:, cols] for all naux rows, shape (naux, len(cols))."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    out = np.empty((naux, cols.size), np.float64)
    lib().synth_B_cols(seed, R.shape[0], _dp(R), naux,
                       cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cols.size, _dp(out))
    return out


def metric(seed: int, naux: int, shift: float = 0.05) -> np.ndarray:
    """Synthetic symmetric positive definite auxiliary metric
    M = G G^T / naux + shift * I with G ~ N(0,1) (naux x naux)."""
    G = normal(seed, STREAM_METRIC, naux * naux).reshape(naux, naux)
    return np.ascontiguousarray(G @ G.T / naux + shift * np.eye(naux))


def C_occ(seed: int, nao: int, nocc: int) -> np.ndarray:
    """Orthonormal nao x nocc columns: Q of the thin QR of an N(0,1) matrix."""
    G = normal(seed, STREAM_COCC, nao * nocc).reshape(nao, nocc)
    Q, _ = np.linalg.qr(G)
    return np.ascontiguousarray(Q)


def rotation(seed: int, nvir: int, nocc: int, amp: float = 0.1) -> np.ndarray:
    """Occupied-virtual rotation amplitudes x (nvir x nocc), amp * N(0,1):
    the trial vectors of a second-order SCF step."""
    return np.ascontiguousarray(amp * normal(seed, STREAM_ROT, nvir * nocc).reshape(nvir, nocc))


def core_hamiltonian(seed: int, R: np.ndarray) -> np.ndarray:
    """H = -diag(U(1,5)) + 0.1 exp(-|R_mu-R_nu|^2) N(0,1), symmetric."""
    nao = R.shape[0]
    diag = 1.0 + 4.0 * uniform(seed, STREAM_H_DIAG, nao)
    z = normal(seed, STREAM_H_OFF, npair(nao))
    mu, nu = np.meshgrid(np.arange(nao), np.arange(nao), indexing="ij")
    r2 = ((R[:, None, :] - R[None, :, :]) ** 2).sum(-1)
    H = 0.1 * np.exp(-r2) * z[pair_index(mu, nu)]
    H[np.diag_indices(nao)] -= diag
    return np.ascontiguousarray(H)


# ---------------------------------------------------------------- configs
@dataclass(frozen=True)
class Config:
    name: str
    nao: int
    naux: int
    nocc: int
    seed: int

    @property
    def npair(self) -> int:
        return npair(self.nao)


C1 = Config("c1", 64, 256, 16, 1)
C2 = Config("c2", 1024, 4096, 200, 2)
C3 = Config("c3", 2048, 8192, 400, 3)
C5 = Config("c5", 128, 512, 24, 0)
C4_NMOL = 256
C4_SEED = 4


def positions(cfg: Config, seed: int | None = None) -> np.ndarray:
    if cfg.name == "c1":
        return positions_c1()
    if cfg.name == "c2":
        return positions_c2()
    if cfg.name == "c3":
        return positions_c3()
    if cfg.name == "c5":
        return positions_c5(cfg.seed if seed is None else seed)
    raise ValueError(cfg.name)


def batch_sizes(nmol: int = C4_NMOL, seed: int = C4_SEED, lo: int = 40, hi: int = 400) -> np.ndarray:
    """nao per molecule, uniform on {lo..hi}."""
    u = uniform(seed, STREAM_BATCH, nmol)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


def small_system(nao: int, naux: int, nocc: int, seed: int):
    """A C1-style system of any size (used for ragged parity cases): sites on
    a near-cubic lattice, one function per site."""
    n = int(np.ceil(nao ** (1 / 3)))
    R = lattice(n, n, n)[:nao].copy()
    return R, B_full(seed, R, naux), C_occ(seed, nao, nocc)


# The SCF family (c5) scales B by this factor.  With B as drawn above the
# two-electron terms are several hundred times the spread of H's spectrum and
# plain DIIS from the core guess does not converge; at 0.005 about 97% of
# seeds converge (measured over seeds 0..29).
C5_B_SCALE = 0.005


def scf_system(seed: int, cfg: Config = C5, b_scale: float = C5_B_SCALE):
    """(R, B, H) of one member of the SCF family."""
    R = positions_c5(seed)
    B = B_full(seed, R, cfg.naux) * b_scale
    H = core_hamiltonian(seed, R)
    return R, B, H
