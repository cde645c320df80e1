"""The 3-index factor on the GPU (dfjk_form_B) against the oracle's
Cholesky + triangular solve, Sec. IV.C.2: B = L^-1 Q with M = L L^T.

Tolerance: 1e-10 of the largest entry (FP64; the synthetic metrics have
condition numbers below 1e3, the explicit 64 x 64 block inverses and the
blocked updates change only the rounding order)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, max_rel, system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


@pytest.mark.parametrize("naux,ncol,pad,seed", [(1, 5, 0, 1), (64, 64, 0, 2), (100, 257, 3, 3),
                                                (300, 1000, 0, 4), (129, 77, 5, 5), (300, 300, 1, 6)])
def test_form_B(pkg, naux, ncol, pad, seed):
    print(f"form_B naux={naux} ncol={ncol} pad={pad}", flush=True)
    M = synth.metric(seed, naux)
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((naux, ncol + pad))
    Md, Qd = dev(M), dev(Q)
    pkg.dfjk_form_B(naux, ncol, Md, Qd, ncol + pad)
    B = host(Qd)
    ref = oracle.form_B(M, Q[:, :ncol])
    assert max_rel(B[:, :ncol], ref) < 1e-10
    assert np.array_equal(B[:, ncol:], Q[:, ncol:])  # padding untouched
    L = host(Md)
    assert max_rel(L, np.linalg.cholesky(M)) < 1e-12
    assert np.all(np.triu(L, 1) == 0)
    # deterministic
    Md2, Qd2 = dev(M), dev(Q)
    pkg.dfjk_form_B(naux, ncol, Md2, Qd2, ncol + pad)
    assert torch.equal(Qd, Qd2) and torch.equal(Md, Md2)


def test_form_B_not_positive_definite(pkg):
    naux = 80
    M = synth.metric(6, naux)
    M[70, 70] = -1.0  # breaks positive definiteness
    with pytest.raises(pkg.DFJKError) as e:
        pkg.dfjk_form_B(naux, 10, dev(M), dev(np.ones((naux, 10))), 10)
    assert e.value.code == -6  # DFJK_E_NONFINITE


def test_formed_B_drives_J_and_K(pkg):
    """B made on the GPU from a synthetic metric and 3-index integrals gives
    the oracle's J and K of the oracle's B."""
    nao, naux, nocc = 40, 120, 8
    R, Q, C = system(nao, naux, nocc, 7)
    M = synth.metric(7, naux)
    Qd = dev(Q)
    pkg.dfjk_form_B(naux, Q.shape[1], dev(M), Qd, Q.shape[1])
    B_ref = oracle.form_B(M, Q)
    D = 2 * C @ C.T
    h = pkg.Handle(Qd, nao)
    assert max_rel(host(h.J(dev(D))), oracle.J(B_ref, nao, D)) < 1e-10
    assert max_rel(host(h.K(C=dev(C))), oracle.K_C(B_ref, nao, C)) < 1e-10
    h.close()
