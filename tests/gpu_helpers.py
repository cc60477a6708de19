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
    """pi equals the optimal policy wherever the action gap at V* exceeds
    gap_min; at the other states (near-ties, where several policies are
    optimal) the chosen action must be admissible and gap_min-optimal at V*:
    Q*(s, pi(s)) - min_a Q*(s, a) <= gap_min (up to rounding of Q*).  A
    policy greedy for V with 2 gamma ||V - V*||_inf <= gap_min meets both."""
    Q = O.q_values(mdp, Vstar)
    srt = np.sort(Q, axis=1)
    gaps = srt[:, 1] - srt[:, 0] if mdp.m > 1 else np.full(mdp.n, np.inf)
    sel = gaps > gap_min
    bad = np.nonzero(pi[sel] != pi_star[sel])[0]
    assert bad.size == 0, f"{bad.size} policy mismatches where the action gap > {gap_min}"
    pi = np.asarray(pi, np.int64)
    assert np.all((pi >= 0) & (pi < mdp.m)), "policy entry out of range"
    q_pi = Q[np.arange(mdp.n), pi]
    assert np.all(np.isfinite(q_pi)), "policy picks an action outside A(s)"
    slack = gap_min + 1e-13 * max(1.0, float(np.max(np.abs(srt[:, 0]))))
    sub = q_pi - srt[:, 0]
    worst = float(np.max(sub)) if sub.size else 0.0
    assert worst <= slack, f"an action {worst:.3e} above the optimum at a near-tie state"


def rel_err(V, Vstar):
    return float(np.max(np.abs(V - Vstar)) / max(np.max(np.abs(Vstar)), 1e-300))


def residual_floor(mdp, Vstar):
    """Absolute rounding error of one FP64 evaluation of g^pi - (V - gamma
    P^pi V) near V*: each component sums k products and three terms, each
    rounded at unit roundoff eps, on operands bounded by max|g| + 2 max|V|."""
    k = int(np.max(np.diff(mdp.row_ptr))) if mdp.fmt == "csr" else mdp.n
    eps = np.finfo(np.float64).eps / 2
    return (k + 3) * eps * (float(np.max(np.abs(mdp.cost))) + 2 * float(np.max(np.abs(Vstar))))


def assert_inner_parity(st, sto, trace, replay, floor=0.0, rel_band=1e-4):
    """The GPU's Arnoldi step count against the oracle's literal stopping
    index.  Equal totals pass.  Otherwise, at the first outer step whose
    counts differ (replay(k) returns the GPU's cumulative count after k
    outer steps), the two may differ by one step only where the decision is
    not resolvable in FP64: the oracle's residual at the disputed iterate
    lies within rel_band of the threshold, or within `floor` (the rounding
    error of an evaluated residual, residual_floor) of it, as happens when a
    forcing sequence drives the threshold to the rounding level.  Later steps
    start from different iterates, and only the outer count and V* compare."""
    if st["inner"] == sto.inner:
        return
    prev = 0
    for k, tr in enumerate(trace):
        cum = replay(k + 1)
        got, want = cum - prev, len(tr["res"])
        prev = cum
        if got == want:
            continue
        assert abs(got - want) == 1, f"outer step {k}: {got} inner steps against the oracle's {want}"
        # GPU one longer: it went past the oracle's stop; one shorter: it
        # stopped at an iterate where the oracle did not
        q = tr["res"][want - 1] if got > want else tr["res"][got - 1]
        thr = tr["thr"]
        assert abs(q - thr) <= max(rel_band * thr, floor), (
            f"outer step {k}: a one-step difference at a resolvable decision (residual "
            f"{q:.3e}, threshold {thr:.3e}, rounding floor {floor:.1e})")
        return
    raise AssertionError("totals differ but every replayed outer step agrees")
