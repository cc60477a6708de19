"""policy_eval_gmres (inner loop of Algorithm 2) against the oracle's literal
GMRES(W) with modified Gram-Schmidt and an explicit residual test every step:
same stopping step, same iterate; and against LU at alpha -> 0."""
import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import dev_vec, host

pytestmark = pytest.mark.gpu


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


def gpu_eval(mdp, pi, x0, alpha, W, store="fp64", mode="fp64", max_inner=100000):
    I = igm()
    with I.mdp_create(mdp, store=store) as h:
        V = dev_vec(x0)
        p = I.params_default(mdp.gamma, alpha=alpha, restart=W, mode=mode, max_inner=max_inner)
        st = h.policy_eval_gmres(dev_vec(pi, "int32"), V, p, allow_noconv=True)
        return host(V), st


@pytest.mark.parametrize("n,m,k,gamma,alpha,W", [
    (100, 4, 5, 0.9, 0.0263, 20),
    (100, 4, 5, 0.9, 1e-3, 5),
    (1000, 3, 6, 0.99, 0.1, 30),
    (2500, 8, 20, 0.99, 2.5e-3, 30),
    (333, 2, 4, 0.95, 1e-4, 3),
])
def test_eval_matches_literal_algorithm(n, m, k, gamma, alpha, W):
    mdp = synth.sparse_uniform(n, m, k, gamma, seed=n)
    rng = np.random.default_rng(n)
    pi = rng.integers(0, m, size=n).astype(np.int32)
    x0 = rng.normal(size=n)
    Vg, st = gpu_eval(mdp, pi, x0, alpha, W)
    Vo, info = O.gmres_inner(mdp, pi, x0, alpha, W)
    assert st["status"] == 0 and st["converged"] == 1
    assert st["inner"] == info["steps"], (st, info["steps"])
    assert st["restarts"] == info["restarts"]
    scale = max(1.0, np.max(np.abs(Vo)))
    np.testing.assert_allclose(Vg, Vo, rtol=0, atol=1e-9 * scale)
    # the rule itself holds on the returned iterate
    b = O.policy_cost(mdp, pi)
    r0 = np.max(np.abs(b - O.j_apply(mdp, pi, x0)))
    assert np.max(np.abs(b - O.j_apply(mdp, pi, Vg))) <= alpha * r0 * (1 + 1e-9)


@pytest.mark.parametrize("W", [2, 7, 40])
def test_eval_tight_matches_lu(W):
    mdp = synth.sparse_uniform(300, 3, 5, 0.95, seed=W)
    pi = np.random.default_rng(W).integers(0, 3, size=300).astype(np.int32)
    Vg, st = gpu_eval(mdp, pi, np.zeros(300), 1e-12, W)
    Vlu = O.policy_eval_lu(mdp, pi)
    np.testing.assert_allclose(Vg, Vlu, rtol=1e-10)


def test_eval_breakdown_uniform_transitions():
    # Krylov space of dimension <= 2: exact after at most two steps
    mdp = synth.uniform_transitions(64, 2, 0.95, seed=3)
    pi = np.zeros(64, np.int32)
    Vg, st = gpu_eval(mdp, pi, np.zeros(64), 1e-10, 10)
    assert st["inner"] <= 2
    np.testing.assert_allclose(Vg, O.policy_eval_lu(mdp, pi), rtol=1e-12)


def test_eval_mixed_precision_fp32_basis():
    mdp = synth.sparse_uniform(3000, 4, 10, 0.99, seed=9)
    stored = mdp.with_values(val=synth.upcast_values(synth.round_values(mdp.val, "fp32"), "fp32"))
    pi = np.random.default_rng(9).integers(0, 4, size=3000).astype(np.int32)
    Vg, st = gpu_eval(mdp, pi, np.zeros(3000), 1e-3, 30, store="fp32", mode="mixed")
    b = O.policy_cost(stored, pi)
    r0 = np.max(np.abs(b))
    # FP64 residual on the stored MDP decides the rule, so it holds exactly there
    assert np.max(np.abs(b - O.j_apply(stored, pi, Vg))) <= 1e-3 * r0 * (1 + 1e-9)


def test_eval_rejects_bad_policy():
    I = igm()
    mdp = synth.sparse_uniform(100, 3, 4, 0.9, seed=1)
    with I.mdp_create(mdp) as h:
        pi = np.zeros(100, np.int32)
        pi[5] = 3
        with pytest.raises(I.IgError) as e:
            h.policy_eval_gmres(dev_vec(pi, "int32"), dev_vec(np.zeros(100)),
                                I.params_default(0.9))
        assert e.value.status == I.IG_E_INVALID
