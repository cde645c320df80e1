"""Exchange for a two-factor density D = L R^T on the GPU against the FP64
oracle's K of that D (K = sum_P B_P D B_P, Sec. IV.C.2), element by element.

The factors are those of a second-order SCF trial density: an orthonormal
basis C split into occupied and virtual columns and rotation amplitudes x,
L = C_vir x and R = C_occ; D = L R^T is not symmetric, D + D^T is.

Tolerances: FP64 B 1e-10 relative to the largest entry (as for the other
FP64 builds; the two sides differ only in summation order).  FP32 B: against
the oracle on the dequantised B with L and R rounded to FP32, the FP32
matrix-core sums (at most nao terms in GEMM1, at most 16384 per SYRK split)
bound the error by ~(nao + 16384) u32 sum|X_L||X_R|; asserted at 2e-4.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, max_rel, system

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def factors(nao, nocc, seed):
    """L = C_vir x, R = C_occ from an orthonormal basis of nao columns."""
    C = synth.C_occ(seed, nao, nao)
    x = synth.rotation(seed, nao - nocc, nocc)
    return np.ascontiguousarray(C[:, nocc:] @ x), np.ascontiguousarray(C[:, :nocc])


CASES = [
    # nao, naux, nocc, seed -- several 128-wide tiles, ragged tails, rank 1,
    # no virtual space (L = 0), contraction splits over the L/R boundary
    (64, 256, 16, 1),
    (300, 77, 37, 11),
    (129, 33, 1, 12),
    (257, 5, 257, 14),
    (200, 130, 40, 15),
    (520, 40, 100, 16),
]


@pytest.mark.parametrize("sym", [0, 1])
@pytest.mark.parametrize("nao,naux,nocc,seed", CASES)
def test_pair_parity_f64(pkg, nao, naux, nocc, seed, sym):
    print(f"case nao={nao} naux={naux} nocc={nocc} seed={seed} sym={sym}", flush=True)
    _, B, _ = system(nao, naux, nocc, seed)
    L, R = factors(nao, nocc, seed)
    D = L @ R.T
    if sym:
        D = D + D.T
    scale = -0.5
    h = pkg.Handle(dev(B), nao)
    K = host(h.K_pair(dev(L), dev(R), sym=bool(sym), scale=scale))
    ref = oracle.K_D(B, nao, scale * D)
    assert max_rel(K, ref) < TOL
    if sym:
        assert np.array_equal(K, K.T)  # exactly symmetric


def test_pair_transpose(pkg):
    """K(R L^T) = K(L R^T)^T: swapping the factors transposes K."""
    nao, naux, nocc = 300, 60, 50
    _, B, _ = system(nao, naux, nocc, 17)
    L, R = factors(nao, nocc, 17)
    h = pkg.Handle(dev(B), nao)
    K1 = host(h.K_pair(dev(L), dev(R)))
    K2 = host(h.K_pair(dev(R), dev(L)))
    assert max_rel(K2, K1.T) < TOL


def test_pair_equal_factors_is_K_C(pkg):
    """L = R = C_occ with scale 2 is the closed-shell K(C_occ)."""
    nao, naux, nocc = 260, 90, 30
    _, B, C = system(nao, naux, nocc, 18)
    h = pkg.Handle(dev(B), nao)
    Kp = host(h.K_pair(dev(C), dev(C), scale=2.0))
    Kc = host(h.K(C=dev(C)))
    ref = oracle.K_C(B, nao, C)
    assert max_rel(Kp, ref) < TOL
    assert max_rel(Kp, Kc) < TOL


def test_pair_deterministic(pkg):
    nao, naux, nocc = 260, 90, 30
    _, B, _ = system(nao, naux, nocc, 19)
    L, R = factors(nao, nocc, 19)
    h = pkg.Handle(dev(B), nao)
    a = host(h.K_pair(dev(L), dev(R), sym=True))
    b = host(h.K_pair(dev(L), dev(R), sym=True))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("sym", [0, 1])
def test_pair_f32(pkg, sym):
    nao, naux, nocc = 300, 77, 37
    _, B, _ = system(nao, naux, nocc, 20)
    L, R = factors(nao, nocc, 20)
    Bq = oracle.quantize_f32(B)
    Bd = torch.empty(B.shape, dtype=torch.float32, device="cuda")
    pkg.dfjk_quantize(dev(B), Bd, 1, B.size)
    Lq, Rq = oracle.quantize_f32(L), oracle.quantize_f32(R)
    D = Lq @ Rq.T
    if sym:
        D = D + D.T
    h = pkg.Handle(Bd, nao, dtype=1)
    K = host(h.K_pair(dev(L), dev(R), sym=bool(sym)))
    assert max_rel(K, oracle.K_D(Bq, nao, D)) < 2e-4


def test_pair_bf16_with_k16_option(pkg):
    """BF16 B on a handle with the k16 option: the two-factor K runs on the
    FP32 matrix cores (the 16-bit path takes one factor), so it matches the
    oracle on the dequantised B with L and R rounded to FP32 (2e-4)."""
    nao, naux, nocc = 300, 40, 37
    _, B, _ = system(nao, naux, nocc, 23)
    L, R = factors(nao, nocc, 23)
    Bq = oracle.quantize_bf16(B)
    Bd = torch.empty(B.shape, dtype=torch.bfloat16, device="cuda")
    pkg.dfjk_quantize(dev(B), Bd, 2, B.size)
    opts = pkg.dfjk.default_options()
    opts.k16 = 1
    h = pkg.Handle(Bd, nao, dtype=2, opts=opts)
    D = oracle.quantize_f32(L) @ oracle.quantize_f32(R).T
    K = host(h.K_pair(dev(L), dev(R), sym=True))
    assert max_rel(K, oracle.K_D(Bq, nao, D + D.T)) < 2e-4
    assert np.array_equal(K, K.T)


def test_pair_invalid(pkg):
    nao, naux, nocc = 64, 20, 8
    _, B, C = system(nao, naux, nocc, 21)
    h = pkg.Handle(dev(B), nao)
    K = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    Cd = dev(C)
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_K_pair(h.h, Cd, Cd, 0, 0, 1.0, K)
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_K_pair(h.h, Cd, Cd, nao + 1, 0, 1.0, K)
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_K_pair(h.h, Cd, Cd, nocc, 2, 1.0, K)
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_K_pair(h.h, Cd, None, nocc, 0, 1.0, K)
