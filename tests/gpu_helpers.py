"""Shared helpers of the GPU parity tests (device marshalling via torch)."""
import numpy as np

from oracle import mdp_oracle as O


def torch_mod():
    import torch
    return torch


def dev_vec(x, dtype="float64"):
    torch = torch_mod()
    return torch.tensor(np.asarray(x), dtype=getattr(torch, dtype), device="cuda")


def zeros(n, dtype="float64"):
    torch = torch_mod()
    return torch.zeros(n, dtype=getattr(torch, dtype), device="cuda")


def host(t):
    torch_mod().cuda.synchronize()
    return t.detach().cpu().numpy()


def tol_par(mdp, vstar_inf):
    """Outer tolerance that certifies rel. error <= 1e-8 and a policy match
    wherever the action gap exceeds 1e-9 (certificate ||V-V*|| <= res/(1-gamma))."""
    g = mdp.gamma
    return min(0.5e-8 * (1 - g) * vstar_inf, (1 - g) * 1e-9 / (2 * g))


def assert_policy_match(mdp, Vstar, pi_star, pi, gap_min=1e-9):
    gaps = O.action_gaps(mdp, Vstar)
    sel = gaps > gap_min
    bad = np.nonzero(pi[sel] != pi_star[sel])[0]
    assert bad.size == 0, f"{bad.size} policy mismatches where the action gap > {gap_min}"


def rel_err(V, Vstar):
    return float(np.max(np.abs(V - Vstar)) / max(np.max(np.abs(Vstar)), 1e-300))
