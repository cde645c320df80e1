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


def bf16_sigmas(params, X, t, u=2.0 ** -8):
    """Standard deviations of the BF16 network's errors against the FP64 one
    under the probabilistic model of rounding (independent relative errors,
    uniform in [-u, u], variance u^2/3; Higham & Mary 2019).

    Only the three hidden x hidden products round their operands (to
    bfloat16, u = 2^-8): an entry a(1 + d_a) b(1 + d_b) errs by a b (d_a +
    d_b), variance (a b)^2 2u^2/3, summed over the product's terms.  Those
    errors are carried through the chain rule with the exact first and second
    derivatives of SiLU at the oracle's pre-activations."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, h1, z2, h2) = oracle.mlp_forward(params, X)
    n = X.shape[0]
    v = 2.0 * u * u / 3.0

    def d2silu(x):
        s = 1.0 / (1.0 + np.exp(-x))
        return s * (1 - s) * (2 + x * (1 - 2 * s))

    s_z2 = np.sqrt(v * (h1 ** 2) @ (W2 ** 2).T)                 # forward product
    s_h2 = np.abs(oracle.dsilu(z2)) * s_z2
    s_y = np.sqrt((s_h2 ** 2) @ (W3 ** 2).T)[:, 0]
    gy = (2.0 / n) * (y - t)
    s_gy = (2.0 / n) * s_y
    gz2 = (gy[:, None] * W3) * oracle.dsilu(z2)
    s_gz2 = np.sqrt((s_gy[:, None] * W3 * oracle.dsilu(z2)) ** 2 + (gy[:, None] * W3 * d2silu(z2) * s_z2) ** 2)
    s_gW2 = np.sqrt(v * (gz2 ** 2).T @ (h1 ** 2) + (s_gz2 ** 2).T @ (h1 ** 2))   # weight-gradient product
    s_gb2 = np.sqrt((s_gz2 ** 2).sum(0))
    s_ga1 = np.sqrt(v * (gz2 ** 2) @ (W2 ** 2) + (s_gz2 ** 2) @ (W2 ** 2))      # input-gradient product
    s_gz1 = np.abs(oracle.dsilu(z1)) * s_ga1
    s_gW1 = np.sqrt((s_gz1 ** 2).T @ (X ** 2))
    s_gb1 = np.sqrt((s_gz1 ** 2).sum(0))
    s_gW3 = np.sqrt((s_gy[:, None] ** 2).T @ (h2 ** 2) + (gy[:, None] ** 2).T @ (s_h2 ** 2))
    s_gb3 = np.array([np.sqrt((s_gy ** 2).sum())])
    return s_y, [s_gW1, s_gb1, s_gW2, s_gb2, s_gW3, s_gb3]


# The rounding of W2 is shared by every row of the batch, so batch sums of its
# effects are partly correlated and the model's variances somewhat low: a
# host emulation of the BF16 products (oracle arithmetic on rounded operands)
# reaches up to 6 standard deviations; the assertion allows 16.
LAMBDA = 16.0


def test_mlp_bf16_gradients_within_bound(pkg):
    """BF16 compute mode: forward values and every gradient entry within
    LAMBDA standard deviations of bf16_sigmas plus the FP32 test's 1e-4 of the
    largest entry (FP32 sums and the FP32 steps); the errors must also be
    visibly larger than FP32's, showing the 16-bit products in use."""
    from paper_2506_06661_amd import dfjk
    m = pkg.MLP(d_in=8, hidden=256, max_batch=4096)
    m.set_compute(dfjk.DFJK_BF16)
    shapes = m.shapes()
    params = [p.astype(np.float32).astype(np.float64) for p in glorot(shapes, 8)]
    params[3] = (0.05 * synth.normal(8, 9, 256)).astype(np.float32).astype(np.float64)
    m.set_params(np.concatenate([p.ravel() for p in params]))
    rng = np.random.default_rng(6)
    n = 3000
    X = rng.standard_normal((n, 8)).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    Xd, td = dev(X, torch.float32), dev(t, torch.float32)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(Xd, y)
    y_ref, _ = oracle.mlp_forward(params, X.astype(np.float64))
    dy, dg = bf16_sigmas(params, X.astype(np.float64), t.astype(np.float64))
    err_y = np.abs(host(y) - y_ref)
    print(f"y: max err {err_y.max():.3e}, max sigma {dy.max():.3e}, max |y| {np.abs(y_ref).max():.3e}")
    assert np.all(err_y <= LAMBDA * dy + 1e-4 * np.abs(y_ref).max())
    assert err_y.max() > 5e-4 * np.abs(y_ref).max()  # far above FP32 rounding: the 16-bit products are in use
    m.loss_grad(Xd, td)
    _, g_ref = oracle.mlp_loss_grad(params, X.astype(np.float64), t.astype(np.float64))
    g = m.unflatten(m.grads())
    for k, (a, b, bd) in enumerate(zip(g, g_ref, dg)):
        err = np.abs(a.reshape(b.shape) - b)
        bd = bd.reshape(b.shape)
        print(f"block {k}: max|g| {np.abs(b).max():.3e} err {err.max():.3e} max sigma {bd.max():.3e}")
        assert np.all(err <= LAMBDA * bd + 1e-4 * np.abs(b).max() + 1e-12), k
    m.close()
