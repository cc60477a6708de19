"""bellman_apply (fused Bellman operator + GreedyPolicy + residual) against
the FP64 oracle, element by element, over several ELL slices with a ragged
tail, edge shapes, ties, dense input and narrow storage."""
import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import dev_vec, host, zeros

pytestmark = pytest.mark.gpu


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


def run_bellman(h, V):
    n = len(V)
    Vd = dev_vec(V)
    TV, pi, res = zeros(n), zeros(n, "int32"), zeros(1)
    h.bellman_apply(Vd, TV, pi, res)
    return host(TV), host(pi), float(host(res)[0])


def check(mdp, V, store="fp64", rtol=1e-14):
    I = igm()
    ref = mdp
    if store != "fp64":
        if mdp.fmt == "csr":
            ref = mdp.with_values(val=synth.upcast_values(synth.round_values(mdp.val, store), store))
        else:
            ref = mdp.with_values(P=synth.upcast_values(synth.round_values(mdp.P, store), store))
    with I.mdp_create(mdp, store=store, validate=(store == "fp64")) as h:
        TV, pi, res = run_bellman(h, V)
    TVo, pio, reso = O.bellman(ref, V)
    scale = max(1.0, np.max(np.abs(TVo)))
    np.testing.assert_allclose(TV, TVo, rtol=0, atol=rtol * scale * 10)
    gaps = O.action_gaps(ref, V)
    sel = gaps > 1e-12 * scale
    assert np.array_equal(pi[sel], pio[sel])
    # where the gap is tiny the chosen action must still attain the minimum
    Q = O.q_values(ref, V)
    np.testing.assert_allclose(Q[np.arange(mdp.n), pi], Q.min(axis=1), rtol=0, atol=1e-12 * scale)
    assert res == pytest.approx(reso, rel=1e-12, abs=1e-13 * scale)


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (1, 3, 1), (63, 2, 4), (64, 4, 5), (65, 4, 5),
                                   (100, 4, 5), (777, 3, 7), (2000, 8, 20), (130, 17, 3),
                                   (300, 300, 3), (70, 1000, 2)])
def test_bellman_shapes(n, m, k):
    mdp = synth.sparse_uniform(n, m, min(k, n), 0.9, seed=n + m)
    V = np.random.default_rng(1).normal(size=n) * 5
    check(mdp, V)


def test_bellman_c2_full_size():
    mdp = synth.config("c2", seed=0)
    V = np.random.default_rng(2).normal(size=mdp.n)
    check(mdp, V)
    check(mdp, np.zeros(mdp.n))


def test_bellman_ragged_rows():
    mdp = synth.random_micro(90, 3, 0.95, seed=5)  # row lengths 1..90
    check(mdp, np.random.default_rng(3).normal(size=90))


def test_bellman_ties_lowest_index():
    rows, cost = [], []
    for s in range(70):
        rows += [[(s, 1.0)], [((s + 1) % 70, 1.0)], [(s, 1.0)]]
        cost += [0.25, 0.25, 0.25]
    mdp = synth.from_rows(70, 3, 0.9, rows, cost)
    V = np.ones(70)  # all three actions tie exactly
    I = igm()
    with I.mdp_create(mdp) as h:
        _, pi, _ = run_bellman(h, V)
    assert np.all(pi == 0)


def test_bellman_dense_fp64():
    mdp = synth.dense_exp(150, 3, 0.95, seed=4)
    check(mdp, np.random.default_rng(4).normal(size=150))


@pytest.mark.parametrize("store", ["fp32", "bf16"])
def test_bellman_narrow_storage(store):
    mdp = synth.sparse_uniform(500, 4, 8, 0.99, seed=6)
    check(mdp, np.random.default_rng(5).normal(size=500) * 10, store=store)
    dm = synth.dense_exp(130, 2, 0.99, seed=7)
    check(dm, np.random.default_rng(6).normal(size=130), store=store)


def test_bellman_nan_reported():
    I = igm()
    mdp = synth.sparse_uniform(100, 2, 3, 0.9, seed=8)
    with I.mdp_create(mdp) as h:
        V = np.zeros(100)
        V[7] = np.nan
        p = I.params_default(0.9)
        Vd = dev_vec(V)
        pi = zeros(100, "int32")
        with pytest.raises(I.IgError) as e:
            h.igmres_pi_solve(Vd, pi, p)
        assert e.value.status == I.IG_E_NUMERIC


@pytest.mark.parametrize("m,store,sets", [(5, "fp32", False), (6, "bf16", False), (5, "fp32", True),
                                          (7, "fp64", True)])
def test_bellman_dense_action_groups(m, store, sets):
    """Dense rows streamed several states and four actions at a time: action
    counts that are not a multiple of four, excluded actions inside a
    group, and group tails (n not a multiple of the states per group)."""
    n = 208 if store == "bf16" else 204
    mdp = synth.dense_exp(n, m, 0.97, seed=11 + m)
    if sets:
        mdp = synth.with_action_sets(mdp, 0.5, 12 + m)
    check(mdp, np.random.default_rng(m).normal(size=n) * 5, store=store)


@pytest.mark.parametrize("name,store", [("c4", "fp32"), ("c3", "fp32"), ("c3", "bf16")])
def test_bellman_full_size(name, store):
    """The full c3 (dense, n = 1e4, m = 4) and c4 (sparse, n = 4e6, m = 8,
    k = 16) workloads through the kernels and launch shapes the bench times,
    every state against the FP64 oracle's Bellman operator on the stored
    values, for a V on the scale of V* (costs in [0, 1)).  Dense rows sum
    1e4 products, so their tolerance allows for a different summation order."""
    mdp = synth.config(name, seed=0)
    V = np.random.default_rng(3).uniform(0.0, 1.0 / (1.0 - mdp.gamma), size=mdp.n)
    check(mdp, V, store=store, rtol=1e-12 if mdp.fmt == "dense" else 1e-14)


@pytest.mark.parametrize("store", ["fp64", "fp32", "bf16"])
def test_bellman_dense_many_actions(store):
    """Dense rows with 200 actions per state (50 groups of four actions)."""
    mdp = synth.dense_exp(64, 200, 0.95, seed=3)
    check(mdp, np.random.default_rng(9).normal(size=64) * 5, store=store)
