"""Parity at the full workload sizes, in the launch configuration the
benchmark times (default tiles, options and split factors).

* nao=1024, naux=4096, nocc=200, FP64 B: rho, J and the whole K against the
  oracle in full; the Coulomb energy E_J = 1/2 sum_P rho_P^2.  Tolerance
  1e-10 relative to the largest reference entry.
* The same workload, K of a two-factor density D = L R^T (with and without
  its transpose) on the same 12 rows, 1e-10.
* The same workload with B stored in FP32 (one rounding from FP64): rho and
  J in full against the oracle on the rounded B (FP64 accumulation: 1e-10);
  the whole K against the oracle on the rounded B within a probabilistic
  bound for the FP32 matrix-core sums (below).
* nao=2048, naux=8192, nocc=400, B stored in BF16 and FP16 (34 GB each, made
  in row blocks): the oracle cannot hold B, so
    - rho and J are checked elementwise against the FP64 oracle on the FP64 B
      within the a-priori bound of one rounding of every B element (below),
      the oracle streaming the same row blocks;
    - rho on sampled rows against the oracle on the rounded rows (1e-10);
    - K (FP32 matrix cores, and the 16-bit matrix-core option) on 4 rows
      against the oracle on the rounded B;
    - the whole K built from the first 64 auxiliary rows against the oracle
      on those rows, rounded (asserted) and FP64 (Frobenius and exchange
      energy errors in Eh, reported).

Bound for one rounding of B (unit roundoff u, absolute floor a for gradual
underflow: |dB| <= u|B| + a; u = 2^-8 bf16, 2^-11 fp16, 2^-24 fp32; a =
2^-25 fp16, 2^-134 bf16).  With r_P = sum_q |B_Pq||dt_q| and s = sum_q |dt_q|
(dt the packed density):
    |d rho_P| <= u r_P + a s
    |d J_p|   <= u sum_P |B_Pp| (|rho_P| + r_P) + a (sum_P |rho_P| + s sum_P |B_Pp|)
to first order; asserted with a factor (1 + 4u) and an FP64 slack of
1e-12 of the largest entry.

FP32 sums of n terms: the probabilistic bound of Higham & Mary (SIAM J. Sci.
Comput. 41(5), 2019), |err| <= lambda sqrt(n) u32 sum|x y| with failure
probability below 2 exp(-lambda^2 (1-u32)^2 / 2); lambda = 10.  K sums nao
terms in GEMM1 and naux*nocc/nsplit in each SYRK split (at most ~2.2e5 at
these sizes); sum|X_m||X_n| <= sqrt(K_mm K_nn) <= max|K|, so the FP32 path is
asserted at 10 (sqrt(nao) + sqrt(2.2e5)) 2^-24 (plus the rounding of C to
FP32) < 5e-4 of the largest entry.  The 16-bit option rounds C and X to the
storage format: first order 2u max|K| from X, plus the same FP32 term:
asserted at 2u + 5e-4.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import frob_rel, host, max_rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

F64, F32, BF16, F16 = 0, 1, 2, 3
U = {F32: 2.0 ** -24, BF16: 2.0 ** -8, F16: 2.0 ** -11}
AFLOOR = {F32: 2.0 ** -150, BF16: 2.0 ** -134, F16: 2.0 ** -25}
QUANT = {F32: oracle.quantize_f32, BF16: oracle.quantize_bf16, F16: oracle.quantize_f16}
TDT = {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}
FP32_SUM_BOUND = 5e-4
SLICE = 64  # auxiliary rows over which the oracle builds the whole K at nao=2048


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def sample_rows(nao):
    rows = [0, 1, 2, 63, 64, 127, 128, nao // 3, nao // 2, nao - 65, nao - 2, nao - 1]
    return np.array(sorted(set(r for r in rows if 0 <= r < nao)))


def row_slices(cfg, R, rows, quant=None):
    """Bsel[r, P, ka] = B_P[mu_r, ka] (optionally rounded), for the oracle's
    row-sampled exchange."""
    out = np.empty((len(rows), cfg.naux, cfg.nao))
    for k, mu in enumerate(rows):
        cols = synth.B_cols(cfg.seed, R, cfg.naux, synth.pair_index(mu, np.arange(cfg.nao)))
        out[k] = cols if quant is None else quant(cols)
    return out


# ---------------------------------------------------------------- C2 sizes
@pytest.fixture(scope="module")
def c2():
    cfg = synth.C2
    print(f"generating nao={cfg.nao} naux={cfg.naux} nocc={cfg.nocc}", flush=True)
    R = synth.positions(cfg)
    B = synth.B_full(cfg.seed, R, cfg.naux)
    C = synth.C_occ(cfg.seed, cfg.nao, cfg.nocc)
    return cfg, R, B, C, 2.0 * C @ C.T


def _c2_build(pkg, cfg, Bd, dtype, C, D):
    h = pkg.Handle(Bd, cfg.nao, dtype=dtype)
    Dd = torch.from_numpy(D).cuda()
    Cd = torch.from_numpy(C).cuda()
    J = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    rho = torch.empty(cfg.naux, dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J(h.h, Dd, J, rho)
    pkg.dfjk_build_K(h.h, Cd, cfg.nocc, None, K)
    out = host(J), host(K), host(rho)
    h.close()
    return out


def test_c2_fp64_full(pkg, c2):
    cfg, R, B, C, D = c2
    Bd = torch.from_numpy(B).cuda()
    J, K, rho = _c2_build(pkg, cfg, Bd, F64, C, D)
    del Bd
    J_o, rho_o = oracle.J(B, cfg.nao, D, return_rho=True)
    assert max_rel(rho, rho_o) < 1e-10
    assert max_rel(J, J_o) < 1e-10
    print("oracle K over all rows", flush=True)
    K_o = oracle.K_C(B, cfg.nao, C)
    err_k = max_rel(K, K_o)
    assert err_k < 1e-10 and frob_rel(K, K_o) < 1e-10, err_k
    assert np.array_equal(K, K.T)
    ej, ej_o = 0.5 * float(rho @ rho), 0.5 * float(rho_o @ rho_o)
    assert abs(ej - ej_o) < 1e-10 * abs(ej_o)
    # K from the density itself (two factors (D, I) at this size): the whole K
    # against the same oracle K, and an indefinite density on sampled rows
    h = pkg.Handle(torch.from_numpy(B).cuda(), cfg.nao)
    K_d = host(h.K(D=torch.from_numpy(D).cuda()))
    err_kd = max_rel(K_d, K_o)
    assert err_kd < 1e-10 and np.array_equal(K_d, K_d.T), err_kd
    rng = np.random.default_rng(11)
    A = rng.standard_normal((cfg.nao, cfg.nao))
    A = A + A.T
    K_a = host(h.K(D=torch.from_numpy(A).cuda()))
    h.close()
    rows = sample_rows(cfg.nao)
    K_a_o = oracle.K_pair_rows(row_slices(cfg, R, rows), A, np.eye(cfg.nao))
    err_ka = float(np.abs(K_a[np.ix_(rows, rows)] - K_a_o).max() / np.abs(K_a_o).max())
    assert err_ka < 1e-10, err_ka
    # DF diagonal from the same J stream
    h = pkg.Handle(torch.from_numpy(B).cuda(), cfg.nao)
    Jd = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
    dg = torch.empty(cfg.npair, dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J_diag(h.h, torch.from_numpy(D).cuda(), Jd, None, dg)
    h.close()
    d_o = oracle.df_diagonal(B, cfg.nao)
    err_d = float(np.abs(host(dg) - d_o).max() / d_o.max())
    assert err_d < 1e-12 and np.array_equal(host(Jd), J)
    # two densities through one pass: D and a random symmetric matrix
    rng = np.random.default_rng(7)
    A = rng.standard_normal((cfg.nao, cfg.nao))
    Ds = np.stack([D, A + A.T])
    h = pkg.Handle(torch.from_numpy(B).cuda(), cfg.nao)
    Jm = torch.empty((2, cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J_multi(h.h, 2, torch.from_numpy(Ds).cuda(), Jm, None)
    h.close()
    Jm = host(Jm)
    assert max_rel(Jm[0], J_o) < 1e-10
    assert max_rel(Jm[1], oracle.J(B, cfg.nao, Ds[1])) < 1e-10
    print(f"C2 FP64: K from D {err_kd:.1e}, indefinite D rows {err_ka:.1e}")
    print(f"C2 FP64: rho {max_rel(rho, rho_o):.1e} J {max_rel(J, J_o):.1e} K {err_k:.1e} "
          f"E_J {ej_o:.10f} Eh, diff {ej - ej_o:.1e}; DF diagonal {err_d:.1e}")


def test_c2_fp32_full(pkg, c2):
    cfg, R, B, C, D = c2
    Bd = torch.from_numpy(B).cuda()
    Bf = torch.empty(Bd.shape, dtype=torch.float32, device="cuda")
    pkg.dfjk_quantize(Bd, Bf, F32, Bd.numel())
    del Bd
    J, K, rho = _c2_build(pkg, cfg, Bf, F32, C, D)
    del Bf
    Bq = oracle.quantize_f32(B)
    J_o, rho_o = oracle.J(Bq, cfg.nao, D, return_rho=True)
    assert max_rel(rho, rho_o) < 1e-10
    assert max_rel(J, J_o) < 1e-10
    print("oracle K over all rows of the rounded B", flush=True)
    K_o = oracle.K_C(Bq, cfg.nao, C)
    del Bq
    err_k = max_rel(K, K_o)
    assert err_k < FP32_SUM_BOUND, err_k
    assert np.array_equal(K, K.T)
    rows = sample_rows(cfg.nao)
    K_i = oracle.K_C_rows(row_slices(cfg, R, rows), C)
    err_i = float(np.abs(K[np.ix_(rows, rows)] - K_i).max() / np.abs(K_i).max())
    print(f"C2 FP32 B: rho {max_rel(rho, rho_o):.1e} J {max_rel(J, J_o):.1e} K (ii) {err_k:.1e} "
          f"Frobenius {frob_rel(K, K_o):.1e}, K rows (i) {err_i:.1e}")


def test_c2_pair_K(pkg, c2):
    """K of a second-order SCF trial density D = C_vir x C_occ^T (+ D^T) from
    its two factors at nao=1024, naux=4096, nocc=200, FP64 B, sampled rows."""
    cfg, R, B, _, _ = c2
    Cb = synth.C_occ(cfg.seed, cfg.nao, cfg.nao)
    x = synth.rotation(cfg.seed, cfg.nao - cfg.nocc, cfg.nocc)
    L, Rm = np.ascontiguousarray(Cb[:, cfg.nocc:] @ x), np.ascontiguousarray(Cb[:, :cfg.nocc])
    h = pkg.Handle(torch.from_numpy(B).cuda(), cfg.nao)
    Ld, Rd = torch.from_numpy(L).cuda(), torch.from_numpy(Rm).cuda()
    rows = sample_rows(cfg.nao)
    Bsel = row_slices(cfg, R, rows)
    for sym in (0, 1):
        print(f"case pair K sym={sym}", flush=True)
        K = host(h.K_pair(Ld, Rd, sym=bool(sym)))
        K_o = oracle.K_pair_rows(Bsel, L, Rm, sym=bool(sym))
        err = float(np.abs(K[np.ix_(rows, rows)] - K_o).max() / np.abs(K_o).max())
        assert err < 1e-10, err
        if sym:
            assert np.array_equal(K, K.T)
    h.close()


def test_c2_form_B(pkg, c2):
    """B = L^-1 Q at naux=4096 with 524800 columns (the lattice-decay B of
    this workload standing in for the 3-index integrals Q, a synthetic SPD
    metric): sampled columns against the oracle (columns are independent)."""
    cfg, R, B, C, D = c2
    M = synth.metric(cfg.seed, cfg.naux)
    Md = torch.from_numpy(M).cuda()
    Qd = torch.from_numpy(B).cuda()
    pkg.dfjk_form_B(cfg.naux, cfg.npair, Md, Qd, cfg.npair)
    cols = np.array([0, 1, 2, 1000, 65535, 262144, cfg.npair - 2, cfg.npair - 1])
    got = host(Qd[:, torch.from_numpy(cols).cuda()])
    del Qd
    ref = oracle.form_B(M, B[:, cols])
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    assert err < 1e-10, err
    print(f"C2 form_B: sampled columns {err:.1e}")


# ---------------------------------------------------------------- C3 sizes
@pytest.fixture(scope="module")
def c3(pkg):
    """Both 16-bit copies of B on the device, and the FP64 oracle's rho, J and
    the first-order bound terms, accumulated over the same row blocks."""
    cfg = synth.C3
    print(f"generating nao={cfg.nao} naux={cfg.naux} nocc={cfg.nocc}", flush=True)
    torch.cuda.empty_cache()
    R = synth.positions(cfg)
    C = synth.C_occ(cfg.seed, cfg.nao, cfg.nocc)
    D = 2.0 * C @ C.T
    Dabs = np.abs(D)
    bufs = {dt: torch.empty((cfg.naux, cfg.npair), dtype=TDT[dt], device="cuda") for dt in (BF16, F16)}
    nao = cfg.nao
    rho = np.empty(cfg.naux)
    r_abs = np.empty(cfg.naux)
    J = np.zeros((nao, nao))
    JB = np.zeros((nao, nao))   # sum_P |B_Pp| (|rho_P| + r_P)
    NB = np.zeros((nao, nao))   # sum_P |B_Pp|
    step = 256
    for P0 in range(0, cfg.naux, step):
        blk = synth.B_rows(cfg.seed, R, P0, step)
        src = torch.from_numpy(blk).cuda()
        for dt, buf in bufs.items():
            pkg.dfjk_quantize(src, buf[P0:P0 + step], dt, src.numel())
        rho[P0:P0 + step] = oracle.rho(blk, nao, D)
        oracle.J_acc(blk, nao, rho[P0:P0 + step], J)
        np.abs(blk, out=blk)
        r_abs[P0:P0 + step] = oracle.rho(blk, nao, Dabs)
        oracle.J_acc(blk, nao, np.abs(rho[P0:P0 + step]) + r_abs[P0:P0 + step], JB)
        oracle.J_acc(blk, nao, np.ones(step), NB)
        torch.cuda.synchronize()
        del src
    s = float(np.abs(D).sum())  # sum_q |dt_q| for symmetric D
    slice_B = synth.B_rows(cfg.seed, R, 0, SLICE)
    K_slice = oracle.K_C(slice_B, nao, C)
    return dict(cfg=cfg, R=R, C=C, D=D, bufs=bufs, rho=rho, r_abs=r_abs, J=J, JB=JB, NB=NB, s=s,
                slice_B=slice_B, K_slice=K_slice)


def _k(pkg, B, nao, dtype, C, nocc, k16=False):
    opts = pkg.dfjk.default_options()
    opts.k16 = 1 if k16 else 0
    h = pkg.Handle(B, nao, dtype=dtype, opts=opts)
    K = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    pkg.dfjk_build_K(h.h, torch.from_numpy(C).cuda(), nocc, None, K)
    out = host(K)
    h.close()
    return out


@pytest.mark.parametrize("dtype", [BF16, F16])
def test_c3_16bit_full(pkg, c3, dtype):
    cfg, C, D = c3["cfg"], c3["C"], c3["D"]
    nao, u, a = cfg.nao, U[dtype], AFLOOR[dtype]
    buf = c3["bufs"][dtype]
    Cd, Dd = torch.from_numpy(C).cuda(), torch.from_numpy(D).cuda()
    h = pkg.Handle(buf, nao, dtype=dtype)
    Jt = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    Kt = torch.empty_like(Jt)
    rt = torch.empty(cfg.naux, dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J(h.h, Dd, Jt, rt)
    pkg.dfjk_build_K(h.h, Cd, cfg.nocc, None, Kt)
    J, K, rho = host(Jt), host(Kt), host(rt)
    h.close()

    # rho and J within one rounding of B, against the FP64 oracle on the FP64 B
    rho_o, J_o = c3["rho"], c3["J"]
    bound_rho = (1 + 4 * u) * (u * c3["r_abs"] + a * c3["s"]) + 1e-12 * np.abs(rho_o).max()
    assert np.all(np.abs(rho - rho_o) <= bound_rho)
    bound_J = (1 + 4 * u) * (u * c3["JB"] + a * (np.abs(rho_o).sum() + c3["s"] * c3["NB"])) \
        + 1e-12 * np.abs(J_o).max()
    assert np.all(np.abs(J - J_o) <= bound_J)
    ej, ej_o = 0.5 * float(rho @ rho), 0.5 * float(rho_o @ rho_o)

    # rho on sampled rows against the oracle on the rounded rows
    prow = [0, 1, 255, 256, cfg.naux // 2, cfg.naux - 1]
    for P in prow:
        brow = QUANT[dtype](synth.B_rows(cfg.seed, c3["R"], P, 1))
        r_ii = oracle.rho(brow, nao, D)[0]
        assert abs(rho[P] - r_ii) <= 1e-10 * c3["r_abs"][P], P  # FP64 sums of npair terms

    # K on 4 rows against the oracle on the rounded B
    rows = np.array([0, 1023, 1024, nao - 1])
    Bsel_q = row_slices(cfg, c3["R"], rows, QUANT[dtype])
    K_ii = oracle.K_C_rows(Bsel_q, C)
    scale = np.abs(K_ii).max()
    err_k = float(np.abs(K[np.ix_(rows, rows)] - K_ii).max() / scale)
    assert err_k < FP32_SUM_BOUND, err_k
    assert np.array_equal(K, K.T)

    # K on the 16-bit matrix cores (C and X rounded to the storage format)
    opts = pkg.dfjk.default_options()
    opts.k16 = 1
    h16 = pkg.Handle(buf, nao, dtype=dtype, opts=opts)
    pkg.dfjk_build_K(h16.h, Cd, cfg.nocc, None, Kt)
    K16 = host(Kt)
    h16.close()
    K16_ii = oracle.K_C_rows(Bsel_q, QUANT[dtype](C))
    err16 = float(np.abs(K16[np.ix_(rows, rows)] - K16_ii).max() / np.abs(K16_ii).max())
    assert err16 < 2 * u + FP32_SUM_BOUND, err16
    assert np.array_equal(K16, K16.T)

    # whole K over the first SLICE auxiliary rows: Frobenius and energy errors
    # against the oracle on the FP64 rows (i) and on the rounded rows (ii)
    Ks_i = c3["K_slice"]
    Bs_q = QUANT[dtype](c3["slice_B"])
    Ks_ii = oracle.K_C(Bs_q, nao, C)
    Ks16_ii = oracle.K_C(Bs_q, nao, QUANT[dtype](C))
    Ks = _k(pkg, buf[:SLICE], nao, dtype, C, cfg.nocc)
    Ks16 = _k(pkg, buf[:SLICE], nao, dtype, C, cfg.nocc, k16=True)
    assert max_rel(Ks, Ks_ii) < FP32_SUM_BOUND
    assert max_rel(Ks16, Ks16_ii) < 2 * u + FP32_SUM_BOUND

    def ek(K_):
        return -0.25 * float(np.sum(D * K_))

    report = {
        "J_maxrel_i": float(np.abs(J - J_o).max() / np.abs(J_o).max()), "J_frob_i": frob_rel(J, J_o),
        "J_bound_use": float((np.abs(J - J_o) / bound_J).max()), "E_J_Eh": ej_o, "E_J_err_i_Eh": ej - ej_o,
        "K_rows_maxrel_ii": err_k, "K16_rows_maxrel_ii": err16,
        "slice_K_frob_i": frob_rel(Ks, Ks_i), "slice_K_frob_ii": frob_rel(Ks, Ks_ii),
        "slice_E_K_Eh": ek(Ks_i), "slice_E_K_err_i_Eh": ek(Ks) - ek(Ks_i),
        "slice_E_K_err_ii_Eh": ek(Ks) - ek(Ks_ii),
        "slice_K16_frob_i": frob_rel(Ks16, Ks_i), "slice_K16_frob_ii": frob_rel(Ks16, Ks16_ii),
        "slice_E_K16_err_i_Eh": ek(Ks16) - ek(Ks_i), "slice_E_K16_err_ii_Eh": ek(Ks16) - ek(Ks16_ii)}
    print(f"C3 dtype {dtype}: " + ", ".join(f"{k} {v:.3e}" for k, v in report.items()))
    assert math.isfinite(ej)


# ---------------------------------------------------------------- C4 size
def test_c4_full_batch_sampled(pkg):
    """The 256-molecule batch as the batch bench builds it (nao ~ U{40..400},
    naux = 4 nao, nocc = nao // 5, BF16 B, graph-captured), with the FP32
    exchange and with the 16-bit one: J and K of sampled molecules (the two
    largest, the two smallest, two in between) against the oracle on the
    stored B, at the bounds of the small batch tests (FP32 exchange 2e-4;
    16-bit exchange 2u + 5e-4 with C rounded to BF16)."""
    sizes = synth.batch_sizes()
    order = np.argsort(sizes, kind="stable")
    picks = sorted(set([int(order[-1]), int(order[-2]), int(order[0]), int(order[1]),
                        int(order[len(order) // 3]), int(order[2 * len(order) // 3])]))
    print(f"c4 batch: {len(sizes)} molecules, checking {[int(sizes[i]) for i in picks]}", flush=True)
    mols = []
    for i, nao in enumerate(sizes):
        nao = int(nao)
        seed = 4000 + i
        R = synth.cluster_positions(seed, nao)
        B = torch.from_numpy(synth.B_full(seed, R, 4 * nao)).cuda()
        C = synth.C_occ(seed, nao, max(nao // 5, 1))
        Cd = torch.from_numpy(C).cuda()
        Bq = torch.empty(B.shape, dtype=torch.bfloat16, device="cuda")
        pkg.dfjk_quantize(B, Bq, BF16, B.numel())
        del B
        mols.append({"B": Bq, "nao": nao, "D": 2.0 * Cd @ Cd.T, "C": Cd,
                     "J": torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                     "K": torch.empty((nao, nao), dtype=torch.float64, device="cuda")})
    torch.cuda.synchronize()
    bt = pkg.Batch(mols, BF16)
    refs = {}
    for i in picks:
        nao = int(sizes[i])
        R = synth.cluster_positions(4000 + i, nao)
        Bq = oracle.quantize_bf16(synth.B_full(4000 + i, R, 4 * nao))
        C = host(mols[i]["C"])
        refs[i] = (oracle.J(Bq, nao, 2.0 * C @ C.T), oracle.K_C(Bq, nao, C),
                   oracle.K_C(Bq, nao, oracle.quantize_bf16(C)))
    for k16 in (False, True):
        bt.set_k16(k16)
        bt.capture()
        bt.launch()
        torch.cuda.synchronize()
        for i in picks:
            J_o, K_o, K_o16 = refs[i]
            ej = max_rel(host(mols[i]["J"]), J_o)
            ek = max_rel(host(mols[i]["K"]), K_o16 if k16 else K_o)
            print(f"  k16={k16} nao={int(sizes[i])}: J {ej:.1e} K {ek:.1e}", flush=True)
            assert ej < 1e-10
            assert ek < (2 * 2.0 ** -8 + 5e-4 if k16 else 2e-4)
    bt.close()
