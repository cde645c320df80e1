"""FP64 J/K on the GPU against the FP64 oracle, element by element.

Tolerance: 1e-10 relative (largest elementwise error over the largest
reference entry, and the Frobenius ratio), the bound set for the FP64 path.
Both sides sum the same terms in different orders with FP64 rounding, so the
observed differences are ~1e-15.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, frob_rel, host, max_rel, system

pytestmark = pytest.mark.gpu
TOL = 1e-10

CASES = [
    # nao, naux, nocc, seed, ld_pad  -- several tiles, ragged tails, odd row stride;
    # even and odd nao: the GEMM2 stages X rows with 16-byte loads when they are
    # 16-byte aligned (even nao in FP64) and one element per load otherwise
    (64, 256, 16, 1, 0),
    (300, 77, 37, 11, 3),
    (129, 33, 1, 12, 0),
    (1, 1, 1, 13, 0),
    (257, 5, 257, 14, 1),
    (200, 130, 200 // 5, 15, 0),
]


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


@pytest.mark.parametrize("nao,naux,nocc,seed,ld_pad", CASES)
def test_J_K_parity(pkg, nao, naux, nocc, seed, ld_pad):
    print(f"case nao={nao} naux={naux} nocc={nocc} seed={seed} ld_pad={ld_pad}", flush=True)
    R, B, C = system(nao, naux, nocc, seed, ld_pad)
    D = 2 * C @ C.T
    Bd = dev(B)
    h = pkg.Handle(Bd, nao)
    rho_d = torch.empty(naux, dtype=torch.float64, device="cuda")
    J = host(h.J(dev(D), rho_d))
    K = host(h.K(C=dev(C)))
    J_ref, rho_ref = oracle.J(B, nao, D, return_rho=True)
    K_ref = oracle.K_C(B, nao, C)
    assert max_rel(host(rho_d), rho_ref) < TOL
    assert max_rel(J, J_ref) < TOL and frob_rel(J, J_ref) < TOL
    assert max_rel(K, K_ref) < TOL and frob_rel(K, K_ref) < TOL
    assert np.array_equal(J, J.T) and np.array_equal(K, K.T)
    h.close()


def test_J_nonsymmetric_density(pkg):
    nao, naux = 150, 40
    R, B, _ = system(nao, naux, 1, 21)
    A = np.random.default_rng(0).standard_normal((nao, nao))
    h = pkg.Handle(dev(B), nao)
    J = host(h.J(dev(A)))
    assert max_rel(J, oracle.J(B, nao, A)) < TOL


def test_K_factored_signs(pkg):
    """K = s * sum_P B_P (C S C^T) B_P for signs S: the oracle's K of that D."""
    nao, naux, ncol = 140, 50, 23
    R, B, C = system(nao, naux, ncol, 22)
    sign = np.where(np.arange(ncol) % 3 == 0, -1.0, 1.0)
    h = pkg.Handle(dev(B), nao)
    K = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    pkg.dfjk_build_K_factored(h.h, dev(C), ncol, dev(sign), 0.75, K)
    ref = oracle.K_D(B, nao, 0.75 * (C * sign) @ C.T)
    assert max_rel(host(K), ref) < TOL


def test_deterministic(pkg):
    nao, naux, nocc = 260, 90, 30
    R, B, C = system(nao, naux, nocc, 23)
    D = 2 * C @ C.T
    h = pkg.Handle(dev(B), nao)
    Dd, Cd = dev(D), dev(C)
    J1, K1 = host(h.J(Dd)), host(h.K(C=Cd))
    J2, K2 = host(h.J(Dd)), host(h.K(C=Cd))
    assert np.array_equal(J1, J2) and np.array_equal(K1, K2)


def test_invalid_nocc(pkg):
    nao = 20
    R, B, C = system(nao, 4, 3, 24)
    h = pkg.Handle(dev(B), nao)
    K = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_K(h.h, dev(C), nao + 1, None, K)
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_K(h.h, dev(C), 0, None, K)


def test_every_gemm1_tile(pkg):
    """Each compiled GEMM1 tile gives the oracle's K (ragged nao, nocc)."""
    nao, naux, nocc = 300, 21, 37
    R, B, C = system(nao, naux, nocc, 25)
    K_ref = oracle.K_C(B, nao, C)
    h = pkg.Handle(dev(B), nao)
    Cd = dev(C)
    nf64 = 0
    for t in range(pkg.dfjk_tile_count(pkg.DFJK_TILE_GEMM1)):
        try:
            pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_GEMM1, t)
        except pkg.DFJKError as e:  # the FP32-only 32 x 32 x 2 tiles
            assert e.code == -5
            continue
        nf64 += 1
        K = host(h.K(C=Cd))
        assert max_rel(K, K_ref) < TOL, (t, pkg.dfjk_tile_info(pkg.DFJK_TILE_GEMM1, t))
    assert nf64 >= 14


@pytest.mark.parametrize("dtype", [1, 2])
def test_every_gemm1_tile_reduced(pkg, dtype):
    """Each GEMM1 tile on B stored in FP32 / BF16 (FP32 matrix cores, the
    32 x 32 x 2 tiles included) gives the oracle's K on the rounded B within
    the FP32 sums' error (1e-5 of the largest entry; the sums run over nao
    and naux * nocc terms)."""
    nao, naux, nocc = 300, 21, 101
    R, B, C = system(nao, naux, nocc, 27)
    quant = {1: oracle.quantize_f32, 2: oracle.quantize_bf16}[dtype]
    Bq = quant(B)
    K_ref = oracle.K_C(Bq, nao, C)
    Bd = torch.empty(B.shape, dtype={1: torch.float32, 2: torch.bfloat16}[dtype], device="cuda")
    pkg.dfjk_quantize(dev(B), Bd, dtype, B.size)
    h = pkg.Handle(Bd, nao, dtype=dtype)
    Cd = dev(C)
    K0 = host(h.K(C=Cd))  # default tiles
    assert max_rel(K0, K_ref) < 1e-5
    for t in range(pkg.dfjk_tile_count(pkg.DFJK_TILE_GEMM1)):
        pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_GEMM1, t)
        K = host(h.K(C=Cd))
        assert max_rel(K, K_ref) < 1e-5, (t, pkg.dfjk_tile_info(pkg.DFJK_TILE_GEMM1, t))
        assert np.array_equal(K, K.T)


@pytest.mark.parametrize("naux", [33, 1000])
def test_every_j_out_width(pkg, naux):
    """Each compiled J pass-2 variant gives the oracle's J (naux=1000 makes
    the row slices long enough for the multi-row loads and their tails)."""
    nao, nocc = 300, 5
    R, B, C = system(nao, naux, nocc, 26)
    D = 2 * C @ C.T
    J_ref = oracle.J(B, nao, D)
    h = pkg.Handle(dev(B), nao)
    Dd = dev(D)
    for t in range(pkg.dfjk_tile_count(pkg.DFJK_TILE_J_OUT)):
        pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_J_OUT, t)
        assert max_rel(host(h.J(Dd)), J_ref) < TOL, t


@pytest.mark.parametrize("nao,naux,seed,ld_pad", [(64, 256, 1, 0), (300, 77, 31, 0), (129, 40, 32, 3)])
def test_df_diagonal(pkg, nao, naux, seed, ld_pad):
    """The DF diagonal from the J pass-2 stream equals the oracle's
    sum_P B[P,p]^2 (1e-12 relative: FP64 sums of positive terms), and J and
    rho are bitwise those of dfjk_build_J."""
    print(f"df diagonal nao={nao} naux={naux} ld_pad={ld_pad}", flush=True)
    R, B, C = system(nao, naux, 4, seed, ld_pad)
    D = 2 * C @ C.T
    h = pkg.Handle(dev(B), nao)
    Dd = dev(D)
    npair = nao * (nao + 1) // 2
    J0 = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    J1 = torch.empty_like(J0)
    r0 = torch.empty(naux, dtype=torch.float64, device="cuda")
    r1 = torch.empty_like(r0)
    dg = torch.empty(npair, dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J(h.h, Dd, J0, r0)
    pkg.dfjk_build_J_diag(h.h, Dd, J1, r1, dg)
    ref = oracle.df_diagonal(B, nao)
    assert float(np.abs(host(dg) - ref).max() / ref.max()) < 1e-12
    assert torch.equal(J0, J1) and torch.equal(r0, r1)
    for t in range(pkg.dfjk_tile_count(pkg.DFJK_TILE_J_OUT)):  # every pass-2 width
        pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_J_OUT, t)
        pkg.dfjk_build_J_diag(h.h, Dd, J1, r1, dg)
        assert float(np.abs(host(dg) - ref).max() / ref.max()) < 1e-12, t
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_build_J_diag(h.h, Dd, J1, r1, None)
    h.close()


@pytest.mark.parametrize("ndm", [1, 3, 8, 11])
@pytest.mark.parametrize("nao,naux,seed,ld_pad", [(300, 77, 31, 0), (129, 40, 32, 3)])
def test_J_several_densities(pkg, ndm, nao, naux, seed, ld_pad):
    """dfjk_build_J_multi: every J (and rho) equals the oracle's for its own
    density (non-symmetric densities included); 11 densities run as 8 + 3."""
    print(f"J multi ndm={ndm} nao={nao} naux={naux}", flush=True)
    R, B, C = system(nao, naux, 4, seed, ld_pad)
    rng = np.random.default_rng(seed + ndm)
    Ds = rng.standard_normal((ndm, nao, nao))
    Ds[0] = 2 * C @ C.T
    h = pkg.Handle(dev(B), nao)
    J = torch.empty((ndm, nao, nao), dtype=torch.float64, device="cuda")
    rho = torch.empty((ndm, naux), dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J_multi(h.h, ndm, dev(Ds), J, rho)
    Jh, rh = host(J), host(rho)
    for m in range(ndm):
        J_ref, r_ref = oracle.J(B, nao, Ds[m], return_rho=True)
        assert max_rel(Jh[m], J_ref) < TOL, m
        assert max_rel(rh[m], r_ref) < TOL, m
    J1 = torch.empty_like(J)
    pkg.dfjk_build_J_multi(h.h, ndm, dev(Ds), J1, None)
    assert torch.equal(J, J1)  # deterministic
    h.close()


@pytest.mark.slow
def test_long_range_df_shape(pkg):
    """naux ~ nao/10 at nao=1024 (the long-range-DF shape): J and K against
    the oracle in full."""
    cfg = synth.C2
    naux = 103
    R = synth.positions(cfg)
    B = synth.B_rows(cfg.seed, R, 0, naux)
    C = synth.C_occ(cfg.seed, cfg.nao, cfg.nocc)
    D = 2 * C @ C.T
    h = pkg.Handle(dev(B), cfg.nao)
    assert max_rel(host(h.J(dev(D))), oracle.J(B, cfg.nao, D)) < TOL
    assert max_rel(host(h.K(C=dev(C))), oracle.K_C(B, cfg.nao, C)) < TOL
    h.close()


@pytest.mark.parametrize("nocc", [113, 150, 200, 230])
def test_gemm1_column_split(pkg, nocc):
    """The default FP64 exchange covers the first columns with one tile and
    the rest with another when that pads less (nocc=200: 112 + 96): K
    matches the oracle and the single-tile result."""
    nao, naux = 256, 12
    R, B, C = system(nao, naux, nocc, 40 + nocc)
    h = pkg.Handle(dev(B), nao)
    K = host(h.K(C=dev(C)))
    assert max_rel(K, oracle.K_C(B, nao, C)) < TOL
    pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_GEMM1, 10)  # the (7,1) tile alone
    assert max_rel(host(h.K(C=dev(C))), K) < 1e-13
    h.close()
