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


def test_eval_matches_literal_algorithm_past_one_grid_stride():
    """n = 140003 is more rows than the Gram-Schmidt passes have threads
    (256 blocks of 512), so some threads take a second row and the last rows
    form a ragged tail; 54 steps with W = 36 run past the 32 columns the fused
    FP64 passes hold (later columns take the separate projection kernels).
    Same stopping step, restarts and iterate as the literal algorithm."""
    n, W, alpha = 140003, 36, 1e-4
    mdp = synth.sparse_band(n, 2, 8, 0.995, seed=5)
    pi = np.random.default_rng(5).integers(0, 2, size=n).astype(np.int32)
    x0 = np.zeros(n)
    Vg, st = gpu_eval(mdp, pi, x0, alpha, W)
    Vo, info = O.gmres_inner(mdp, pi, x0, alpha, W)
    print(f"fp64 n={n}: inner={st['inner']} restarts={st['restarts']} oracle steps={info['steps']}")
    assert info["steps"] > 32 and info["restarts"] >= 1
    assert st["status"] == 0 and st["converged"] == 1
    assert st["inner"] == info["steps"], (st, info["steps"])
    assert st["restarts"] == info["restarts"]
    scale = max(1.0, np.max(np.abs(Vo)))
    np.testing.assert_allclose(Vg, Vo, rtol=0, atol=1e-9 * scale)
    b = O.policy_cost(mdp, pi)
    assert np.max(np.abs(b - O.j_apply(mdp, pi, Vg))) <= alpha * np.max(np.abs(b)) * (1 + 1e-9)


def test_eval_mixed_widest_fused_passes_past_two_grid_strides():
    """Mixed path (FP32 basis) at n = 300007 (threads take two or three rows,
    ragged tail) with W = 64 and a tight rule, so that cycles run into the
    48- and 64-column fused passes; the FP64 residual on the stored MDP
    decides the stop, so the rule holds exactly there, and the error from
    the policy's value is at most ||residual||_inf / (1 - gamma)."""
    n, W, alpha = 300007, 64, 1e-9
    mdp = synth.sparse_band(n, 2, 8, 0.995, seed=6)
    stored = mdp.with_values(val=synth.upcast_values(synth.round_values(mdp.val, "fp32"), "fp32"))
    pi = np.random.default_rng(6).integers(0, 2, size=n).astype(np.int32)
    Vg, st = gpu_eval(mdp, pi, np.zeros(n), alpha, W, store="fp32", mode="mixed")
    print(f"mixed n={n}: inner={st['inner']} restarts={st['restarts']}")
    assert st["status"] == 0 and st["converged"] == 1
    # some cycle is at least this long, so it ran through columns 32..48 and past 48
    assert -(-st["inner"] // (st["restarts"] + 1)) > 48, st
    b = O.policy_cost(stored, pi)
    res = np.max(np.abs(b - O.j_apply(stored, pi, Vg)))
    assert res <= alpha * np.max(np.abs(b)) * (1 + 1e-9)


@pytest.mark.parametrize("alpha,W", [(1e-6, 30), (1e-12, 3), (1e-9, 2)])
def test_eval_dense_c3_full_size_matches_literal_algorithm(alpha, W):
    """Dense P^pi products at the full c3 size (n = 1e4, FP64): the same
    stopping step, restarts and iterate as the literal algorithm, with and
    without restarts (W = 2 restarts 24 times)."""
    mdp = synth.config("c3", seed=0)
    pi = np.random.default_rng(7).integers(0, mdp.m, size=mdp.n).astype(np.int32)
    x0 = np.zeros(mdp.n)
    Vg, st = gpu_eval(mdp, pi, x0, alpha, W)
    Vo, info = O.gmres_inner(mdp, pi, x0, alpha, W)
    assert st["status"] == 0 and st["converged"] == 1
    assert st["inner"] == info["steps"], (st, info["steps"])
    assert st["restarts"] == info["restarts"]
    scale = max(1.0, np.max(np.abs(Vo)))
    np.testing.assert_allclose(Vg, Vo, rtol=0, atol=1e-9 * scale)
