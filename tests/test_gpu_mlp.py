"""Learned-guess network on the GPU against the FP64 CPU oracle.

* Forward values and gradients of the mean-squared loss: the GPU computes in
  FP32 (matrix-core products over d_in and hidden = 256 terms, batch sums in
  slabs) on parameters, inputs and targets that are exactly representable in
  FP32; the oracle (pinned by finite differences) computes in FP64.  Bound:
  |g_gpu - g_ref| <= 1e-4 * max |g_ref| per parameter block, |y| likewise.
* Adam: one step moves every parameter by at most lr (Kingma & Ba's bound
  for the bias-corrected first step) and against the gradient sign.
* Guess features and assembly: a symmetric density Dcore + y.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def glorot(shapes, seed):
    out = []
    for k, s in enumerate(shapes):
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            u = synth.uniform(seed, synth.STREAM_MLP, int(np.prod(s)), start=k << 32)
            out.append(((2 * u - 1) * lim).reshape(s))
        else:
            out.append(np.zeros(s))
    return out


def test_mlp_gradients_match_oracle(pkg):
    m = pkg.MLP(d_in=8, hidden=256, max_batch=4096)
    shapes = m.shapes()
    params = [p.astype(np.float32).astype(np.float64) for p in glorot(shapes, 7)]
    params[1] = (0.05 * synth.normal(7, 9, 256)).astype(np.float32).astype(np.float64)
    flat = np.concatenate([p.ravel() for p in params])
    m.set_params(flat)
    rng = np.random.default_rng(5)
    n = 3000
    X = rng.standard_normal((n, 8)).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    Xd, td = dev(X, torch.float32), dev(t, torch.float32)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(Xd, y)
    y_ref, _ = oracle.mlp_forward(params, X.astype(np.float64))
    assert np.abs(host(y) - y_ref).max() <= 1e-4 * np.abs(y_ref).max()
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m.loss_grad(Xd, td, loss)
    L_ref, g_ref = oracle.mlp_loss_grad(params, X.astype(np.float64), t.astype(np.float64))
    assert abs(float(host(loss)[0]) - L_ref) <= 1e-5 * L_ref
    g = m.unflatten(m.grads())
    for k, (a, b) in enumerate(zip(g, g_ref)):
        err = np.abs(a.reshape(b.shape) - b).max()
        print(f"block {k}: max|g| {np.abs(b).max():.3e} err {err:.3e}")
        assert err <= 1e-4 * np.abs(b).max() + 1e-12, k
    # one Adam step: |dp| <= lr, opposite to the gradient where it is nonzero
    lr = 1e-3
    m.adam(lr)
    p1 = m.params()
    d = p1 - flat.astype(np.float32)
    gf = np.concatenate([x.ravel() for x in g])
    assert np.abs(d).max() <= lr * (1 + 1e-5)
    big = np.abs(gf) > 1e-6 * np.abs(gf).max()
    assert np.all(np.sign(d[big]) == -np.sign(gf[big]))
    m.close()


def test_guess_features_and_assembly(pkg):
    nao = 128
    R, B, H = synth.scf_system(11)
    eps, U = np.linalg.eigh(H)
    C = U[:, :24]
    Dc = 2 * C @ C.T
    npair = synth.npair(nao)
    X = torch.empty((npair, 8), dtype=torch.float32, device="cuda")
    pkg.dfjk_guess_features(dev(H), dev(Dc), dev(R), nao, X)
    Xh = host(X)
    mu, nu = 3, 17
    p = synth.pair_index(mu, nu)
    r = np.linalg.norm(R[mu] - R[nu])
    assert np.allclose(Xh[p, :7], [Dc[mu, nu], H[mu, nu], 0.5 * (H[mu, mu] + H[nu, nu]),
                                   abs(H[mu, mu] - H[nu, nu]), 0.1 * r, np.exp(-r * r), 0.0],
                       rtol=1e-6, atol=1e-7)
    ranks = np.argsort(np.argsort(np.diag(H), kind="stable"), kind="stable")
    assert abs(Xh[p, 7] - (ranks[mu] + ranks[nu]) / (2 * nao)) < 1e-6
    y = torch.linspace(-1, 1, npair, dtype=torch.float32, device="cuda")
    D = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    pkg.dfjk_guess_assemble(y, dev(Dc), nao, D)
    Dh = host(D)
    yh = host(y).astype(np.float64)
    assert np.array_equal(Dh, Dh.T)
    assert Dh[mu, nu] == Dc[mu, nu] + yh[p]
