"""Learned initial guess: data from the plain SCF, training, and use.

The paper's mean-field runs take any guess density (Sec. IV.A.1); the
default accelerator is DIIS (Sec. IV.B).  This module drives the library:

* ``run_scf``      -- DIIS SCF on the GPU through ``dfjk_scf_step`` from the
                      core-Hamiltonian guess or a given density.
* ``run_scf_mixed``-- the same SCF with J/K from B stored at reduced
                      precision until the commutator norm is small, then
                      from the FP64 B.
* ``Trainer``      -- fits the perceptron (library kernels: forward, backward,
                      Adam) to converged densities, as corrections of the
                      core guess on the packed pairs.
* ``guess_density``-- features -> network -> D0 = Dcore + correction.
* ``solve``        -- SCF from the learned guess with the core guess as the
                      fallback, decided from the run's own signals only
                      (non-finite D0, electron count off by more than 25%, no
                      convergence within max_iter).
* ``account``      -- J/K builds to a reference energy for a ``solve`` result,
                      computed after the run: a run that converged to another
                      state counts as a failure with a core-guess run on top.

Systems are passed in as arrays (H, packed B, positions R); nothing here
draws random inputs except the seeded parameter initialisation, whose
uniform numbers are supplied by the caller.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dfjk as _d


def core_guess(handle: _d.Handle, H: torch.Tensor, nocc: int):
    """Aufbau on the core Hamiltonian (the library's eigensolver): (C, D)."""
    nao = H.shape[0]
    C = torch.empty((nao, nocc), dtype=torch.float64, device=H.device)
    D = torch.empty((nao, nao), dtype=torch.float64, device=H.device)
    _d.dfjk_aufbau(handle.h, H, nocc, C, D)
    return C, D


def run_scf(handle: _d.Handle, H: torch.Tensor, nocc: int, D0: torch.Tensor | None = None,
            C0: torch.Tensor | None = None, max_iter: int = 100):
    """DIIS SCF from D0 (K through C0 when given, else through D0's
    eigen-factors on the first iteration).  Returns (records, D, C) with one
    (e_tot, err_norm, converged) record per J/K build."""
    nao = H.shape[0]
    _d.dfjk_scf_reset(handle.h)
    if D0 is None:
        C0, D0 = core_guess(handle, H, nocc)
    D = D0.clone().contiguous()
    C = (C0.clone() if C0 is not None else torch.zeros((nao, nocc), dtype=torch.float64,
                                                       device=H.device)).contiguous()
    flags = _d.DFJK_SCF_C_VALID if C0 is not None else 0
    recs = []
    for _ in range(max_iter):
        _, info = _d.dfjk_scf_step(handle.h, H, D, C, nocc, flags)
        flags = _d.DFJK_SCF_C_VALID
        recs.append((info.e_tot, info.err_norm, bool(info.converged)))
        if info.converged or not math.isfinite(info.e_tot):
            break
    return recs, D, C


def run_scf_mixed(h_low: _d.Handle, h64: _d.Handle, H: torch.Tensor, nocc: int, switch: float = 1e-4,
                  max_iter: int = 100):
    """SCF that builds J/K from B stored at reduced precision (h_low) until
    the commutator norm |FD - DF|_F falls below `switch` (or that SCF
    converges), then from the FP64 B (h64) with a fresh DIIS history,
    continuing from the same density and orbitals.  Both handles describe the
    same system.  Returns (records, D, C); each record is (e_tot, err_norm,
    converged, reduced) with `reduced` True for builds from h_low."""
    _d.dfjk_scf_reset(h_low.h)
    _d.dfjk_scf_reset(h64.h)
    C, D = core_guess(h64, H, nocc)
    flags = _d.DFJK_SCF_C_VALID
    recs = []
    h, low = h_low, True
    for _ in range(max_iter):
        _, info = _d.dfjk_scf_step(h.h, H, D, C, nocc, flags)
        recs.append((info.e_tot, info.err_norm, bool(info.converged) and not low, low))
        if not math.isfinite(info.e_tot):
            break
        if low and (info.err_norm < switch or info.converged):
            h, low = h64, False
        elif not low and info.converged:
            break
    return recs, D, C


def builds_to(recs, e_ref: float, tol: float = 1e-6):
    """J/K builds until |E_k - E_ref| < tol, or None.  Builds from B stored
    at reduced precision (a fourth record field that is True) do not count as
    reaching it: their energies are not FP64 energies of the system."""
    for k, rec in enumerate(recs):
        if len(rec) > 3 and rec[3]:
            continue
        if abs(rec[0] - e_ref) < tol:
            return k + 1
    return None


def features(H: torch.Tensor, Dcore: torch.Tensor, R: torch.Tensor) -> torch.Tensor:
    nao = H.shape[0]
    X = torch.empty((nao * (nao + 1) // 2, 8), dtype=torch.float32, device=H.device)
    _d.dfjk_guess_features(H, Dcore, R, nao, X)
    return X


def target(D: torch.Tensor, Dcore: torch.Tensor) -> torch.Tensor:
    """Training target D - Dcore on the packed pairs (FP32, library kernel)."""
    nao = D.shape[0]
    t = torch.empty(nao * (nao + 1) // 2, dtype=torch.float32, device=D.device)
    _d.dfjk_guess_target(D, Dcore, nao, t)
    return t


class Trainer:
    """Mean-squared-error fit of the perceptron with Adam (library kernels)."""

    def __init__(self, mlp: _d.MLP, init_uniform: np.ndarray):
        """init_uniform: nparam uniforms in [0, 1) for Glorot initialisation
        of the weight matrices (biases start at zero)."""
        self.mlp = mlp
        flat, o = [], 0
        for s in mlp.shapes():
            n = int(np.prod(s))
            if len(s) == 2:  # weight matrix: Glorot-uniform
                lim = math.sqrt(6.0 / (s[0] + s[1]))
                flat.append((2.0 * init_uniform[o:o + n] - 1.0) * lim)
            else:
                flat.append(np.zeros(n))
            o += n
        mlp.set_params(np.concatenate(flat))

    def fit(self, X: torch.Tensor, t: torch.Tensor, epochs: int, batch: int, lr: float,
            order_uniform: np.ndarray | None = None, log=None):
        """X (n x 8), t (n) on the device.  order_uniform: one uniform per row
        and epoch for the shuffle (or None: fixed order)."""
        n = X.shape[0]
        loss = torch.zeros(1, dtype=torch.float32, device=X.device)
        hist = []
        for ep in range(epochs):
            if order_uniform is not None:
                # the shuffle order is data preparation (a sort of the supplied
                # uniforms); the rows are gathered by the library
                perm = torch.from_numpy(np.argsort(order_uniform[ep * n:(ep + 1) * n], kind="stable")).to(X.device)
                Xe, te = torch.empty_like(X), torch.empty_like(t)
                _d.dfjk_gather_rows(X, perm, n, X.shape[1], Xe)
                _d.dfjk_gather_rows(t, perm, n, 1, te)
            else:
                Xe, te = X, t
            tot = 0.0
            nb = 0
            for b0 in range(0, n, batch):
                xb, tb = Xe[b0:b0 + batch], te[b0:b0 + batch]
                self.mlp.loss_grad(xb, tb, loss)
                self.mlp.adam(lr)
                tot += float(loss.item()) if (nb % 64 == 0) else 0.0
                nb += 1
            hist.append(tot)
            if log:
                log(f"epoch {ep + 1}/{epochs}")
        return hist

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self.mlp.forward(X, y)
        return y


def guess_density(handle: _d.Handle, trainer: Trainer, H: torch.Tensor, R: torch.Tensor, nocc: int):
    """D0 = Dcore + network correction on the packed pairs."""
    _, Dc = core_guess(handle, H, nocc)
    X = features(H, Dc, R)
    y = trainer.predict(X)
    D0 = torch.empty_like(Dc)
    _d.dfjk_guess_assemble(y, Dc, H.shape[0], D0)
    return D0


def project(handle: _d.Handle, D0: torch.Tensor, nocc: int):
    """Closest idempotent density of rank nocc: D = 2 C C^T with C the
    eigenvectors of the nocc largest eigenvalues of D0."""
    nao = D0.shape[0]
    C = torch.empty((nao, nocc), dtype=torch.float64, device=D0.device)
    D = torch.empty_like(D0)
    _d.dfjk_aufbau(handle.h, (-D0).contiguous(), nocc, C, D)
    return C, D


def solve(handle: _d.Handle, trainer: Trainer, H: torch.Tensor, R: torch.Tensor, nocc: int,
          max_iter: int = 100, projected: bool = False):
    """SCF from the learned guess with the core guess as fallback.  With
    `projected`, the guess is first replaced by the closest idempotent density
    of rank nocc (then the first exchange goes through C).  The fallback is
    decided from this run's own signals: a guess with non-finite entries or an
    electron count off by more than 25%, or an SCF that does not converge
    within max_iter.  Returns a dict with the records of the learned run, the
    records of the fallback run ([] if none), whether it ran and why."""
    D0 = guess_density(handle, trainer, H, R, nocc)
    chk = torch.empty(2, dtype=torch.float64, device=H.device)
    _d.dfjk_guess_check(D0, H.shape[0], chk)
    tr_d, bad = (float(v) for v in chk.cpu())
    reason = None
    if bad > 0:
        reason = "non-finite guess"
    elif abs(tr_d - 2 * nocc) > 0.25 * 2 * nocc:
        reason = "electron count"
    recs = []
    if reason is None:
        C0 = None
        if projected:
            C0, D0 = project(handle, D0, nocc)
        recs = run_scf(handle, H, nocc, D0=D0, C0=C0, max_iter=max_iter)[0]
        if not (recs and recs[-1][2]):
            reason = "not converged"
    if reason is None:
        return {"records": recs, "fallback": False, "reason": None, "fallback_records": []}
    fb = run_scf(handle, H, nocc, max_iter=max_iter)[0]
    return {"records": recs, "fallback": True, "reason": reason, "fallback_records": fb}


def account(out: dict, e_ref: float, core_records, tol: float = 1e-6) -> dict:
    """J/K builds to |E - e_ref| < tol for a ``solve`` result, counted after
    the run (e_ref, the plain SCF's converged energy, is the judge and takes
    no part in the run).  A run that converged to another state counts as a
    failure, with the plain core-guess run's builds added on top."""
    recs = out["records"]
    if out["fallback"]:
        nb = builds_to(out["fallback_records"], e_ref, tol)
        fb_len = len(out["fallback_records"])
        return {"builds": len(recs) + (nb if nb is not None else fb_len), "wrong_state": False}
    nb = builds_to(recs, e_ref, tol)
    if nb is not None and abs(recs[-1][0] - e_ref) < tol:
        return {"builds": nb, "wrong_state": False}
    nc = builds_to(core_records, e_ref, tol)
    return {"builds": len(recs) + (nc if nc is not None else len(core_records)), "wrong_state": True}
