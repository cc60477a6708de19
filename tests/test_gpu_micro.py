"""Every solver entry point on tiny MDPs against what needs no solver:
brute force over all deterministic policies (eq. 2: V* is their
componentwise minimum, and the returned policy must be one of those that
attain it) and closed forms (self-loops: V*(s) = min_a g(s,a)/(1-gamma);
constant costs: V* = g0/(1-gamma), the equality case of Lemma 3; cyclic
moves, whose P^pi has its spectrum on the circle of radius gamma and forces
restarts of GMRES(W) when W is small)."""
import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import host, zeros

pytestmark = pytest.mark.gpu

METHODS = [("igmres_pi_solve", 1), ("igmres_pi_solve", 2), ("pi_solve", 0), ("opi_solve", 0),
           ("ipi_vi_solve", 0)]


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


def run(mdp, method, engine, **kw):
    I = igm()
    kw.setdefault("tol", 1e-12)
    kw.setdefault("restart", 8)
    with I.mdp_create(mdp) as h:
        V = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        st = getattr(h, method)(V, pi, I.params_default(mdp.gamma, engine=engine, **kw))
        return host(V), host(pi), st


@pytest.mark.parametrize("method,engine", METHODS)
@pytest.mark.parametrize("n,m,seed", [(5, 3, 1), (7, 2, 2), (6, 3, 3), (8, 2, 4)])
def test_micro_brute_force(n, m, seed, method, engine):
    mdp = synth.random_micro(n, m, 0.9, seed)
    Vstar, optimal = O.brute_force(mdp)
    V, pi, st = run(mdp, method, engine)
    assert st["converged"] == 1
    assert np.max(np.abs(V - Vstar)) <= 1e-9 * np.max(np.abs(Vstar))
    assert any(np.array_equal(pi, np.asarray(p)) for p in optimal), (pi, optimal)


@pytest.mark.parametrize("method,engine", METHODS)
def test_self_loops_closed_form(method, engine):
    mdp = synth.self_loops(300, 4, 0.95, seed=6)
    c = np.asarray(mdp.cost).reshape(mdp.n, mdp.m)
    V, pi, st = run(mdp, method, engine)
    assert st["converged"] == 1
    assert np.allclose(V, c.min(axis=1) / (1 - mdp.gamma), rtol=1e-10, atol=0)
    assert np.array_equal(pi, np.argmin(c, axis=1))


@pytest.mark.parametrize("method,engine", METHODS)
def test_constant_costs_closed_form(method, engine):
    base = synth.sparse_uniform(500, 3, 6, 0.99, 8)
    mdp = synth.MDP(base.n, base.m, base.gamma, np.full(base.n * base.m, 0.25), "csr",
                    base.row_ptr, base.col, base.val, None, "const", dict(base.meta))
    V, _, st = run(mdp, method, engine)
    assert st["converged"] == 1
    assert np.allclose(V, 0.25 / (1 - mdp.gamma), rtol=1e-10, atol=0)


@pytest.mark.parametrize("engine", [1, 2])
def test_cyclic_forces_restarts(engine):
    """A deterministic cycle: GMRES(4) on a 64-cycle needs restarts; the
    result is still the LU value of the returned policy, and that policy is
    greedy with respect to it."""
    mdp = synth.cyclic(64, 2, 0.9, seed=9)
    V, pi, st = run(mdp, "igmres_pi_solve", engine, restart=4, tol=1e-11)
    assert st["converged"] == 1 and st["restarts"] > 0
    Vpi = O.policy_eval_lu(mdp, pi)
    assert np.max(np.abs(V - Vpi)) <= 1e-9 * np.max(np.abs(Vpi))
    Vs, pis, _ = O.policy_iteration(mdp)
    assert np.max(np.abs(V - Vs)) <= 1e-9 * np.max(np.abs(Vs))
