"""dfjk_build_J_static (J on the library's fixed scratch array, no device
allocation) against dfjk_build_J on a handle made from the same arguments.

Both run the same kernels with the same launch geometry, so J and rho must be
bitwise equal; the smaller FP64 case is also held to the FP64 bound (1e-10
relative) against the oracle.  Two calls in a row, the second on a smaller
system, show that what the first call leaves in the shared scratch does not
leak into the second.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, max_rel, system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def _pair(pkg, nao, naux, seed, dtype, opts=None):
    """(J_static, rho_static, J_handle, rho_handle, B64, D) for one seeded system."""
    from paper_2506_06661_amd import dfjk
    R, B, C = system(nao, naux, max(1, nao // 5), seed)
    D = 2 * C @ C.T
    if dtype == dfjk.DFJK_F64:
        Bd = dev(B)
    else:
        Bd = torch.empty(B.shape, dtype=dfjk._ELEM[dtype], device="cuda")
        dfjk.dfjk_quantize(dev(B), Bd, dtype, B.size)
    Dd = dev(D)
    Js = torch.full((nao, nao), np.nan, dtype=torch.float64, device="cuda")
    rs = torch.full((naux,), np.nan, dtype=torch.float64, device="cuda")
    print(f"static J: nao={nao} naux={naux} dtype={dtype} seed={seed}", flush=True)
    dfjk.dfjk_build_J_static(Bd, dtype, nao, naux, B.shape[1], Dd, Js, rs, opts=opts)
    Js_h, rs_h = host(Js), host(rs)
    h = dfjk.dfjk_init(Bd, dtype, nao, naux, B.shape[1], opts=opts)
    Jh = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    rh = torch.empty(naux, dtype=torch.float64, device="cuda")
    dfjk.dfjk_build_J(h, Dd, Jh, rh)
    Jh_h, rh_h = host(Jh), host(rh)
    dfjk.dfjk_destroy(h)
    return Js_h, rs_h, Jh_h, rh_h, B, D


def test_static_J_f64_two_calls(pkg):
    from paper_2506_06661_amd import dfjk
    for nao, naux, seed in ((700, 1500, 71), (130, 300, 72)):
        Js, rs, Jh, rh, B, D = _pair(pkg, nao, naux, seed, dfjk.DFJK_F64)
        assert np.array_equal(Js, Jh) and np.array_equal(rs, rh), (nao, naux)
    J_ref, rho_ref = oracle.J(B, 130, D, return_rho=True)
    assert max_rel(Js, J_ref) < 1e-10 and max_rel(rs, rho_ref) < 1e-10


def test_static_J_bf16_compensated_two_calls(pkg):
    from paper_2506_06661_amd import dfjk
    o = dfjk.default_options()
    o.compensated_j = 1
    for nao, naux, seed in ((200, 500, 73), (90, 200, 74)):
        Js, rs, Jh, rh, _, _ = _pair(pkg, nao, naux, seed, dfjk.DFJK_BF16, opts=o)
        assert np.array_equal(Js, Jh) and np.array_equal(rs, rh), (nao, naux)


def test_static_J_rejects_oversize(pkg):
    from paper_2506_06661_amd import dfjk
    nao, naux = 4096, 1
    ld = nao * (nao + 1) // 2
    B = torch.zeros((naux, ld), dtype=torch.float64, device="cuda")
    D = torch.zeros((nao, nao), dtype=torch.float64, device="cuda")
    J = torch.zeros((nao, nao), dtype=torch.float64, device="cuda")
    with pytest.raises(dfjk.DFJKError) as e:
        dfjk.dfjk_build_J_static(B, dfjk.DFJK_F64, nao, naux, ld, D, J)
    assert e.value.code == -1 and "scratch" in str(e.value)
    assert dfjk.dfjk_static_scratch_bytes() == 128 << 20
