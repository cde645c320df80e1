"""Reduced-precision storage of B (FP32, BF16, FP16) on the GPU.

* Quantisation: the GPU's one-step RNE conversion equals the oracle's,
  bit for bit (integer decision taken by both sides from the same FP64 value).
* J and K against the FP64 oracle on the *dequantised* B (kernel error only),
  with bounds from the arithmetic:
    - J, FP64 accumulation: products of exact FP32 values with FP64 weights
      summed in FP64 -> FP64 rounding only, 1e-10.
    - J, FP32 Dot2: compensated FP32 dot products (Ogita-Rump-Oishi): error
      ~ u32 + n u32^2 relative to sum |b d|, where n <= npair; asserted at 1e-6
      against the largest entry.
    - K: C rounded to FP32 (u32 = 2^-24), FP32 matrix-core products with
      FP32 sums over nao terms (GEMM1) and over a split of up to ~16k terms
      (SYRK), split partials added in FP64: |dK| <= ~(nao + kchunk) u32 *
      sum|X||X|; asserted at 2e-4 of the largest entry.
* Against the FP64 oracle on the FP64 B the error is dominated by the
  storage rounding of B (unit roundoff u = 2^-24, 2^-8, 2^-11 for FP32,
  BF16, FP16); it is reported.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, frob_rel, host, max_rel, system

pytestmark = pytest.mark.gpu

F32, BF16, F16 = 1, 2, 3
QUANT = {F32: oracle.quantize_f32, BF16: oracle.quantize_bf16, F16: oracle.quantize_f16}
TDT = {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def gpu_quantize(pkg, x, dtype):
    src = dev(x)
    dst = torch.empty(x.shape, dtype=TDT[dtype], device="cuda")
    pkg.dfjk_quantize(src, dst, dtype, src.numel())
    return dst


def test_quantize_bit_exact(pkg):
    rng = np.random.default_rng(30)
    x = np.concatenate([
        rng.standard_normal(100000) * np.exp(rng.uniform(-60, 12, 100000)),
        [0.0, -0.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -40, 65504.0, 65520.0,
         2.0 ** -25, 3 * 2.0 ** -26, 1e-160, -1e-45, 3.4e38, 3.5e38, 1e300],
    ])
    bf = host(gpu_quantize(pkg, x, BF16).view(torch.uint16).to(torch.int32)).astype(np.uint16)
    assert np.array_equal(bf, oracle.bf16_bits(oracle.quantize_bf16(x)))
    hf = host(gpu_quantize(pkg, x, F16).view(torch.uint16).to(torch.int32)).astype(np.uint16)
    ref = oracle.quantize_f16(x)
    assert np.array_equal(hf, oracle.f16_bits(ref))
    f = host(gpu_quantize(pkg, x, F32)).astype(np.float64)
    with np.errstate(over="ignore"):
        assert np.array_equal(f, oracle.quantize_f32(x))


# nao, naux, nocc, seed, ld_pad: rows of X and C^T that are whole 16-byte
# vectors (nao, nocc multiples of 4: 16-byte staging loads) and that are not
# (element loads at the row ends), and a padded row stride of B (its
# 16-byte loads at every alignment)
CASES = [(64, 256, 16, 1, 0), (300, 77, 37, 31, 0), (129, 40, 9, 32, 3)]


@pytest.mark.parametrize("dtype", [F32, BF16, F16])
@pytest.mark.parametrize("nao,naux,nocc,seed,ld_pad", CASES)
def test_reduced_J_K(pkg, dtype, nao, naux, nocc, seed, ld_pad):
    print(f"case dtype={dtype} nao={nao} naux={naux} nocc={nocc} ld_pad={ld_pad}", flush=True)
    R, B, C = system(nao, naux, nocc, seed, ld_pad)
    D = 2 * C @ C.T
    Bq = QUANT[dtype](B)                      # dequantised storage values (exact in FP64)
    Bd = gpu_quantize(pkg, B, dtype)
    J_ii = oracle.J(Bq, nao, D)
    K_ii = oracle.K_C(Bq, nao, C)
    J_i = oracle.J(B, nao, D)
    K_i = oracle.K_C(B, nao, C)
    errs = {}
    for mode, tol in [(2, 1e-10), (1, 1e-6), (0, None)]:
        opts = pkg.dfjk.default_options()
        opts.compensated_j = mode
        h = pkg.Handle(Bd, nao, dtype=dtype, opts=opts)
        J = host(h.J(dev(D)))
        errs[f"J mode{mode} (ii)"] = max_rel(J, J_ii)
        errs[f"J mode{mode} (i)"] = frob_rel(J, J_i)
        if tol is not None:
            assert max_rel(J, J_ii) < tol, (mode, max_rel(J, J_ii))
        if mode == 2:
            K = host(h.K(C=dev(C)))
            errs["K (ii)"] = max_rel(K, K_ii)
            errs["K (i)"] = frob_rel(K, K_i)
            assert max_rel(K, K_ii) < 2e-4
            assert np.array_equal(K, K.T)
        h.close()
    print({k: f"{v:.2e}" for k, v in errs.items()})


@pytest.mark.parametrize("dtype,bound", [(BF16, 2 * 2.0 ** -8 + 5e-4), (F16, 2 * 2.0 ** -11 + 5e-4)])
@pytest.mark.parametrize("nao,naux,nocc,seed", [(64, 256, 16, 1), (300, 40, 37, 33), (129, 20, 40, 34),
                                              (1, 3, 1, 35), (65, 7, 65, 36)])
def test_k16_exchange(pkg, dtype, bound, nao, naux, nocc, seed):
    """K on the 16-bit matrix cores (dense 16-bit copy of B).  Reference: the
    oracle on the dequantised B with C rounded once to the same format.  X is
    rounded to 16 bits (unit roundoff u = 2^-8 bf16, 2^-11 fp16) after FP32
    accumulation; to first order the rounding of X gives, by Cauchy-Schwarz,
    |dK_mn| <= 2u sqrt(K_mm K_nn) <= 2u max|K|, and the FP32 sums add less
    than 5e-4 of max|K| (probabilistic bound, lambda = 10, for sums of up to
    ~2e5 terms): asserted at 2u + 5e-4."""
    print(f"k16 dtype={dtype} nao={nao} naux={naux} nocc={nocc}", flush=True)
    R, B, C = system(nao, naux, nocc, seed)
    Bq = QUANT[dtype](B)
    Cq = QUANT[dtype](C)
    opts = pkg.dfjk.default_options()
    opts.k16 = 1
    h = pkg.Handle(gpu_quantize(pkg, B, dtype), nao, dtype=dtype, opts=opts)
    K = host(h.K(C=dev(C)))
    K_ref = oracle.K_C(Bq, nao, Cq)
    err = max_rel(K, K_ref)
    print(f"  k16 err vs rounded-input oracle {err:.2e}; vs FP64 {frob_rel(K, oracle.K_C(B, nao, C)):.2e}")
    assert err < bound
    assert np.array_equal(K, K.T)
    K2 = host(h.K(C=dev(C)))  # the dense copy is made once and reused
    assert np.array_equal(K, K2)
    for t in range(pkg.dfjk_tile_count(pkg.DFJK_TILE_K16)):  # every GEMM1 tile
        pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_K16, t)
        assert max_rel(host(h.K(C=dev(C))), K_ref) < bound, t
    pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_K16, -1)
    for t in range(pkg.dfjk_tile_count(pkg.DFJK_TILE_K16_SYRK)):  # every GEMM2 tile (128, 256)
        pkg.dfjk_set_tile(h.h, pkg.DFJK_TILE_K16_SYRK, t)
        Kt = host(h.K(C=dev(C)))
        assert max_rel(Kt, K_ref) < bound, t
        assert np.array_equal(Kt, Kt.T)


@pytest.mark.parametrize("dtype", [F32, BF16, F16])
def test_reduced_df_diagonal(pkg, dtype):
    """DF diagonal with B stored in FP32/BF16/FP16: FP64 sums of the exact
    squares of the stored values, so it matches the oracle on the rounded B
    to 1e-12; J is bitwise that of dfjk_build_J."""
    nao, naux = 300, 77
    R, B, C = system(nao, naux, 5, 31)
    D = 2 * C @ C.T
    Bq = QUANT[dtype](B)
    h = pkg.Handle(gpu_quantize(pkg, B, dtype), nao, dtype=dtype)
    Dd = dev(D)
    J0 = h.J(Dd)
    J1 = torch.empty_like(J0)
    dg = torch.empty(nao * (nao + 1) // 2, dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J_diag(h.h, Dd, J1, None, dg)
    ref = oracle.df_diagonal(Bq, nao)
    assert float(np.abs(host(dg) - ref).max() / ref.max()) < 1e-12
    assert torch.equal(J0, J1)
    h.close()


def test_reduced_several_densities(pkg):
    """Reduced B streams the densities one after another: each J is bitwise
    dfjk_build_J's."""
    nao, naux = 129, 40
    R, B, C = system(nao, naux, 5, 32)
    rng = np.random.default_rng(5)
    Ds = rng.standard_normal((3, nao, nao))
    h = pkg.Handle(gpu_quantize(pkg, B, BF16), nao, dtype=BF16)
    J = torch.empty((3, nao, nao), dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J_multi(h.h, 3, dev(Ds), J, None)
    for m in range(3):
        assert torch.equal(J[m], h.J(dev(Ds[m])))
    h.close()
