"""Learned initial guess end to end on the GPU (small scale).

Training data come from the plain DIIS SCF on the GPU (core guess); the
network is trained with the library's kernels; on held-out systems the SCF
from the learned guess (with the core guess as fallback) must reach the same
converged energy as the plain SCF (1e-6 Eh), and the J/K build counts of
both are reported.  Fallback logic is exercised with a corrupted network.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def system(pkg, seed):
    cfg = synth.C5
    R, B, H = synth.scf_system(seed, cfg)
    h = pkg.Handle(dev(B), cfg.nao)
    return h, dev(H), dev(R)


def test_learned_guess_pipeline(pkg):
    from paper_2506_06661_amd import guess
    cfg = synth.C5
    Xs, ts = [], []
    for seed in range(40):
        h, H, R = system(pkg, seed)
        recs, D, C = guess.run_scf(h, H, cfg.nocc)
        if not recs[-1][2]:
            continue
        _, Dc = guess.core_guess(h, H, cfg.nocc)
        Xs.append(guess.features(H, Dc, R))
        ts.append(guess.target(D, Dc))
        h.close()
    assert len(Xs) >= 30
    X = torch.cat(Xs).contiguous()
    t = torch.cat(ts).contiguous()
    mlp = pkg.MLP(8, 256, 65536)
    tr = guess.Trainer(mlp, synth.uniform(1, synth.STREAM_MLP, mlp.nparam))
    order = synth.uniform(2, synth.STREAM_MLP, X.shape[0] * 3)
    hist = tr.fit(X, t, epochs=3, batch=65536, lr=1e-3, order_uniform=order)
    print("loss samples", hist)
    core, learned, projected, fallbacks, wrong = [], [], [], 0, 0
    for seed in range(2000, 2010):
        h, H, R = system(pkg, seed)
        ref, _, _ = guess.run_scf(h, H, cfg.nocc)
        if not ref[-1][2]:
            continue
        e_ref = ref[-1][0]
        core.append(guess.builds_to(ref, e_ref))
        out = guess.solve(h, tr, H, R, cfg.nocc)  # no reference energy in the run
        acc = guess.account(out, e_ref, ref)
        learned.append(acc["builds"])
        fallbacks += out["fallback"]
        wrong += acc["wrong_state"]
        final = (out["fallback_records"] or out["records"])[-1]
        assert final[2]
        if not acc["wrong_state"]:
            assert abs(final[0] - e_ref) < 1e-6
        outp = guess.solve(h, tr, H, R, cfg.nocc, projected=True)
        projected.append(guess.account(outp, e_ref, ref)["builds"])
        h.close()
    print(f"builds to 1e-6 Eh: core {np.mean(core):.2f}, learned {np.mean(learned):.2f}, "
          f"projected {np.mean(projected):.2f}, fallbacks {fallbacks}/{len(learned)}, other state {wrong}")
    assert len(learned) >= 8


def test_fallback_on_corrupted_network(pkg):
    from paper_2506_06661_amd import guess
    cfg = synth.C5
    mlp = pkg.MLP(8, 256, 65536)
    tr = guess.Trainer(mlp, synth.uniform(3, synth.STREAM_MLP, mlp.nparam))
    p = mlp.params()
    p[-1] = np.float32(np.nan)  # output bias
    mlp.set_params(p)
    h, H, R = system(pkg, 2001)
    ref, _, _ = guess.run_scf(h, H, cfg.nocc)
    out = guess.solve(h, tr, H, R, cfg.nocc)
    assert out["fallback"] and out["reason"] == "non-finite guess" and out["records"] == []
    assert out["fallback_records"][-1][2]
    assert abs(out["fallback_records"][-1][0] - ref[-1][0]) < 1e-10
    acc = guess.account(out, ref[-1][0], ref)
    assert acc["builds"] == guess.builds_to(ref, ref[-1][0]) and not acc["wrong_state"]
