"""Batched J/K over molecules of uneven size (one launch per phase, graph
replay) against the FP64 oracle on each molecule's dequantised B.

Bounds as for single builds with reduced-precision storage: J accumulates in
FP64 (1e-10); K runs on the FP32 matrix cores (2e-4 of the largest entry).
Graph replays equal the eager build bit for bit, across several replays with
other device work in between.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, max_rel

pytestmark = pytest.mark.gpu
TDT = {1: torch.float32, 2: torch.bfloat16, 3: torch.float16}
QUANT = {1: oracle.quantize_f32, 2: oracle.quantize_bf16, 3: oracle.quantize_f16}


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def make_batch(pkg, sizes, dtype, seed0):
    mols, refs = [], []
    for i, nao in enumerate(sizes):
        seed = seed0 + i
        naux, nocc = 4 * nao, max(nao // 5, 1)
        R = synth.cluster_positions(seed, nao)
        B = synth.B_full(seed, R, naux)
        C = synth.C_occ(seed, nao, nocc)
        D = 2 * C @ C.T
        Bd = torch.empty(B.shape, dtype=TDT[dtype], device="cuda")
        pkg.dfjk_quantize(dev(B), Bd, dtype, B.size)
        mols.append({"B": Bd, "nao": nao, "D": dev(D), "C": dev(C),
                     "J": torch.zeros((nao, nao), dtype=torch.float64, device="cuda"),
                     "K": torch.zeros((nao, nao), dtype=torch.float64, device="cuda")})
        refs.append((QUANT[dtype](B), C, D))
    return pkg.Batch(mols, dtype), mols, refs


@pytest.mark.parametrize("dtype", [1, 2])
def test_batch_matches_oracle(pkg, dtype):
    # nocc buckets 0..4 (ceil(nocc/16) - 1), i.e. every bucket the 256-molecule
    # workload (nao up to 400, nocc up to 80) uses
    sizes = [40, 97, 130, 41, 256, 72, 150, 64, 33, 200, 345, 400]
    print(f"batch dtype={dtype} sizes={sizes}", flush=True)
    bt, mols, refs = make_batch(pkg, sizes, dtype, 4100)
    bt.build()
    torch.cuda.synchronize()
    for m, (Bq, C, D) in zip(mols, refs):
        nao = m["nao"]
        J_ref = oracle.J(Bq, nao, D)
        K_ref = oracle.K_C(Bq, nao, C)
        assert max_rel(host(m["J"]), J_ref) < 1e-10, nao
        assert max_rel(host(m["K"]), K_ref) < 2e-4, nao
    bt.close()


def test_graph_replay_equals_eager(pkg):
    sizes = [60, 170, 45, 120]
    bt, mols, _ = make_batch(pkg, sizes, 1, 4200)
    bt.build()
    eager = [(host(m["J"]).copy(), host(m["K"]).copy()) for m in mols]
    bt.capture()
    for rep in range(3):
        for m in mols:
            m["J"].zero_()
            m["K"].zero_()
        torch.cuda.synchronize()
        bt.launch()
        torch.cuda.synchronize()
        for m, (J0, K0) in zip(mols, eager):
            assert np.array_equal(host(m["J"]), J0), rep
            assert np.array_equal(host(m["K"]), K0), rep
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * 2).sum().item()
    bt.close()


def _check_all(mols, refs, what):
    for m, (Bq, C, D) in zip(mols, refs):
        nao = m["nao"]
        ej = max_rel(host(m["J"]), oracle.J(Bq, nao, D))
        ek = max_rel(host(m["K"]), oracle.K_C(Bq, nao, C))
        assert ej < 1e-10 and ek < 2e-4, (what, nao, ej, ek)


@pytest.mark.parametrize("dtype", [1, 2])
def test_autotune_keeps_parity(pkg, tmp_path, dtype):
    """Default tiles and autotuned tiles over buckets 0..4 (nao up to 380),
    every molecule against the oracle; a second batch reads the cache (and
    re-checks those tiles) instead of timing."""
    sizes = [50, 90, 140, 210, 260, 380]
    print(f"autotune dtype={dtype} sizes={sizes}", flush=True)
    bt, mols, refs = make_batch(pkg, sizes, dtype, 4300)
    bt.build()
    torch.cuda.synchronize()
    _check_all(mols, refs, "default tiles")
    cache = str(tmp_path / "tiles.txt")
    ms = bt.autotune(reps=1, cache_path=cache)
    tiles = [bt.tile(b) for b in range(8)]
    print("tiles", tiles, "ms", ms)
    for m in mols:
        m["J"].zero_()
        m["K"].zero_()
    bt.build()
    torch.cuda.synchronize()
    _check_all(mols, refs, "tuned tiles")
    # graph replay of the tuned build equals the eager one
    eager = [host(m["K"]).copy() for m in mols]
    bt.capture()
    bt.launch()
    torch.cuda.synchronize()
    for m, K0 in zip(mols, eager):
        assert np.array_equal(host(m["K"]), K0)
    bt.close()
    # a second batch reads the cache instead of timing
    bt2, mols2, _ = make_batch(pkg, sizes, dtype, 4300)
    bt2.autotune(reps=1, cache_path=cache)
    assert [bt2.tile(b) for b in range(8)] == tiles
    bt2.build()
    torch.cuda.synchronize()
    _check_all(mols2, refs, "cached tiles")
    bt2.close()


@pytest.mark.parametrize("dtype,bound", [(2, 2 * 2.0 ** -8 + 5e-4), (3, 2 * 2.0 ** -11 + 5e-4)])
def test_batch_k16_matches_oracle(pkg, dtype, bound):
    """Exchange on the 16-bit matrix cores over the batch (GEMM1 on the packed
    triangle, buckets of 32, 64 and 96 padded orbital columns, all present
    here).  Reference: the oracle on the stored B with C rounded once to the
    same format; bound as for the single-molecule 16-bit exchange (X rounded
    to 16 bits: |dK| <= 2u max|K| to first order, FP32 sums < 5e-4).  J is
    the FP64-accumulated one (1e-10).  Graph replays equal the eager build
    bit for bit; switching back gives the FP32 exchange's K bit for bit."""
    sizes = [40, 97, 130, 41, 256, 72, 150, 64, 33, 200, 345, 400]
    print(f"batch k16 dtype={dtype} sizes={sizes}", flush=True)
    bt, mols, refs = make_batch(pkg, sizes, dtype, 4100)
    bt.build()
    torch.cuda.synchronize()
    k32 = [host(m["K"]).copy() for m in mols]
    bt.set_k16(True)
    bt.build()
    torch.cuda.synchronize()
    for m, (Bq, C, D) in zip(mols, refs):
        nao = m["nao"]
        K = host(m["K"])
        err = max_rel(K, oracle.K_C(Bq, nao, QUANT[dtype](C)))
        assert err < bound, (nao, err)
        assert np.array_equal(K, K.T), nao
        assert max_rel(host(m["J"]), oracle.J(Bq, nao, D)) < 1e-10, nao
    eager = [host(m["K"]).copy() for m in mols]
    bt.capture()
    for rep in range(2):
        for m in mols:
            m["K"].zero_()
        torch.cuda.synchronize()
        bt.launch()
        torch.cuda.synchronize()
        for m, K0 in zip(mols, eager):
            assert np.array_equal(host(m["K"]), K0), rep
    bt.set_k16(False)
    bt.build()
    torch.cuda.synchronize()
    for m, K0 in zip(mols, k32):
        assert np.array_equal(host(m["K"]), K0)
    bt.close()


def test_batch_k16_needs_16bit_storage(pkg):
    bt, _, _ = make_batch(pkg, [40, 60], 1, 4400)
    with pytest.raises(RuntimeError, match="16-bit exchange"):
        bt.set_k16(True)
    bt.close()
