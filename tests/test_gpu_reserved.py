"""Workspace reserved at init (dfjk_options.max_ncol > 0): no call allocates,
so J and K builds can be captured in a HIP graph; replays equal the eager
builds bitwise.  Calls beyond the reservation are refused.  With the k16
option the dense 16-bit copy of B follows B's contents only through
dfjk_update_B.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfjk():
    from paper_2506_06661_amd import dfjk as d
    return d


def _opts(dfjk, max_ncol, k16=0):
    o = dfjk.default_options()
    o.max_ncol = max_ncol
    o.k16 = k16
    return o


@pytest.mark.parametrize("dtype_name", ["f64", "f32", "bf16_k16"])
def test_graph_capture_replays_bitwise(dfjk, dtype_name):
    nao, naux, nocc = 300, 600, 60
    print(f"reserved-mode capture: {dtype_name} nao={nao} naux={naux} nocc={nocc}", flush=True)
    R, B, C = system(nao, naux, nocc, 81)
    D = 2 * C @ C.T
    s = torch.cuda.Stream()
    if dtype_name == "f64":
        dt, Bd, o = dfjk.DFJK_F64, dev(B), _opts(dfjk, 64)
    else:
        dt = dfjk.DFJK_F32 if dtype_name == "f32" else dfjk.DFJK_BF16
        Bd = torch.empty(B.shape, dtype=dfjk._ELEM[dt], device="cuda")
        dfjk.dfjk_quantize(dev(B), Bd, dt, B.size)
        o = _opts(dfjk, 64, k16=1 if dtype_name == "bf16_k16" else 0)
    torch.cuda.synchronize()
    h = dfjk.dfjk_init(Bd, dt, nao, naux, B.shape[1], stream=s, opts=o)
    ws0 = dfjk.dfjk_workspace_bytes(h)
    Dd, Cd = dev(D), dev(C)
    Je = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    Ke = torch.empty_like(Je)
    Jg = torch.empty_like(Je)
    Kg = torch.empty_like(Je)
    with torch.cuda.stream(s):
        dfjk.dfjk_build_J(h, Dd, Je)
        dfjk.dfjk_build_K(h, Cd, nocc, None, Ke)
    s.synchronize()
    J_eager, K_eager = host(Je), host(Ke)
    assert dfjk.dfjk_workspace_bytes(h) == ws0  # nothing grew

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        dfjk.dfjk_build_J(h, Dd, Jg)
        dfjk.dfjk_build_K(h, Cd, nocc, None, Kg)
    for rep in range(3):
        Jg.fill_(np.nan)
        Kg.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(Jg), J_eager), rep
        assert np.array_equal(host(Kg), K_eager), rep
        # eager work of the program's own between replays
        Je.zero_()
        torch.cuda.synchronize()
    assert dfjk.dfjk_workspace_bytes(h) == ws0
    del g
    dfjk.dfjk_destroy(h)


def test_refuses_beyond_reservation(dfjk):
    nao, naux = 120, 240
    R, B, C = system(nao, naux, 40, 82)
    h = dfjk.dfjk_init(dev(B), dfjk.DFJK_F64, nao, naux, B.shape[1], opts=_opts(dfjk, 32))
    K = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    with pytest.raises(dfjk.DFJKError) as e:
        dfjk.dfjk_build_K(h, dev(C), 40, None, K)
    assert e.value.code == -1 and "max_ncol" in str(e.value)
    with pytest.raises(dfjk.DFJKError):
        dfjk.dfjk_build_K(h, None, 0, dev(2 * C @ C.T), K)  # K from D needs max_ncol = nao
    with pytest.raises(dfjk.DFJKError):
        dfjk.dfjk_build_K_pair(h, dev(C[:, :20]), dev(C[:, :20]), 20, 1, 1.0, K)  # 40 > 32
    dfjk.dfjk_build_K(h, dev(C[:, :32].copy()), 32, None, K)  # within the reservation
    torch.cuda.synchronize()
    dfjk.dfjk_destroy(h)


def test_k16_copy_follows_update_B(dfjk):
    nao, naux, nocc = 200, 300, 40
    print(f"k16 update_B: nao={nao} naux={naux} nocc={nocc}", flush=True)
    R, B, C = system(nao, naux, nocc, 83)
    Bd = torch.empty(B.shape, dtype=torch.bfloat16, device="cuda")
    dfjk.dfjk_quantize(dev(B), Bd, dfjk.DFJK_BF16, B.size)
    o = dfjk.default_options()
    o.k16 = 1
    h = dfjk.dfjk_init(Bd, dfjk.DFJK_BF16, nao, naux, B.shape[1], opts=o)
    Cd = dev(C)
    K = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    dfjk.dfjk_build_K(h, Cd, nocc, None, K)
    K1 = host(K)
    Bd.mul_(2.0)  # exact in BF16: K of the new B is exactly 4 K1
    torch.cuda.synchronize()
    dfjk.dfjk_build_K(h, Cd, nocc, None, K)
    assert np.array_equal(host(K), K1)  # the copy still holds the old contents
    dfjk.dfjk_update_B(h)
    dfjk.dfjk_build_K(h, Cd, nocc, None, K)
    assert np.array_equal(host(K), 4.0 * K1)
    dfjk.dfjk_destroy(h)
