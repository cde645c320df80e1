"""Helpers shared by the GPU tests: seeded systems on the device."""
import numpy as np
import torch

import synth


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def system(nao, naux, nocc, seed, ld_pad=0):
    """Lattice positions, packed B (naux x (npair+ld_pad)) and C_occ."""
    n = int(np.ceil(nao ** (1 / 3) - 1e-9))
    R = np.ascontiguousarray(synth.lattice(n, n, n)[:nao])
    B = synth.B_full(seed, R, naux, ldB=synth.npair(nao) + ld_pad)
    C = synth.C_occ(seed, nao, nocc)
    return R, B, C


def max_rel(a, ref):
    """Largest elementwise error relative to the largest reference entry."""
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300))


def frob_rel(a, ref):
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))
