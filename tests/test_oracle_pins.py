"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(not against the oracle itself): a hand-solved example, closed forms,
operator properties (Section 2), Lemmas 1-3, brute force over all policies
(eq. 2), and the GMRES minimum-residual property (eq. 13)."""
import json
import os

import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def two_state():
    d = json.load(open(os.path.join(GOLD, "two_state.json")))
    mdp = synth.from_rows(d["n"], d["m"], d["gamma"], [[tuple(e) for e in r] for r in d["rows"]],
                          d["cost"])
    return mdp, d


# ---------------------------------------------------------------- hand example

def test_two_state_bellman_and_greedy():
    mdp, d = two_state()
    V = np.array(d["V"])
    np.testing.assert_allclose(O.q_values(mdp, V), d["Q_of_V"], rtol=0, atol=1e-15)
    TV, pi, res = O.bellman(mdp, V)
    np.testing.assert_allclose(TV, d["TV"], rtol=0, atol=1e-15)
    assert pi.tolist() == d["greedy"]
    assert res == pytest.approx(d["res_inf"], abs=1e-15)


def test_two_state_policy_values_and_optimum():
    mdp, d = two_state()
    for key, want in d["V_pi"].items():
        pi = np.array([int(x) for x in key.split(",")], dtype=np.int32)
        np.testing.assert_allclose(O.policy_eval_lu(mdp, pi), want, rtol=1e-14)
        np.testing.assert_allclose(O.policy_eval_neumann(mdp, pi), want, rtol=1e-13)
    Vs, opt = O.brute_force(mdp)
    np.testing.assert_allclose(Vs, d["V_star"], rtol=1e-14)
    assert [p.tolist() for p in opt] == [d["pi_star"]]
    V, pi, _ = O.policy_iteration(mdp)
    np.testing.assert_allclose(V, d["V_star"], rtol=1e-14)
    assert pi.tolist() == d["pi_star"]
    V, _ = O.value_iteration(mdp)
    np.testing.assert_allclose(V, d["V_star"], rtol=1e-11)
    V, pi, st = O.igmres_pi(mdp, W=2, tol=1e-13)
    np.testing.assert_allclose(V, d["V_star"], rtol=1e-12)
    assert st.converged


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("gamma", [0.5, 0.9, 0.99])
def test_constant_cost_lemma3_equality(gamma):
    # g == c0 gives V^pi = c0/(1-gamma) 1 for every policy (row-stochastic P^pi)
    mdp = synth.sparse_uniform(60, 3, 4, gamma, seed=3)
    mdp.cost = np.full(mdp.n * mdp.m, 0.7)
    want = np.full(mdp.n, 0.7 / (1 - gamma))
    pi = np.random.default_rng(0).integers(0, 3, size=60).astype(np.int32)
    np.testing.assert_allclose(O.policy_eval_lu(mdp, pi), want, rtol=1e-12)
    V, _, _ = O.policy_iteration(mdp)
    np.testing.assert_allclose(V, want, rtol=1e-12)
    V, _, _ = O.igmres_pi(mdp, W=5, tol=1e-12 * want[0])
    np.testing.assert_allclose(V, want, rtol=1e-11)


def test_self_loops_closed_form():
    mdp = synth.self_loops(30, 4, 0.9, seed=1)
    cmin = mdp.cost.reshape(30, 4).min(axis=1)
    want = cmin / (1 - 0.9)
    V, pi, _ = O.policy_iteration(mdp)
    np.testing.assert_allclose(V, want, rtol=1e-13)
    assert np.array_equal(pi, mdp.cost.reshape(30, 4).argmin(axis=1))
    V, _ = O.value_iteration(mdp)
    np.testing.assert_allclose(V, want, rtol=1e-10)


def test_uniform_transitions_closed_form_and_breakdown():
    n, m, g = 25, 3, 0.95
    mdp = synth.uniform_transitions(n, m, g, seed=2)
    cmin = mdp.cost.reshape(n, m).min(axis=1)
    want = cmin + g / (1 - g) * cmin.mean()
    V, pi, _ = O.policy_iteration(mdp)
    np.testing.assert_allclose(V, want, rtol=1e-13)
    # J = I - gamma/n 11^T: the Krylov space of any residual has dimension <= 2
    pi = np.zeros(n, dtype=np.int32)
    x, info = O.gmres_inner(mdp, pi, np.zeros(n), alpha=1e-14, W=10)
    assert info["steps"] <= 2
    np.testing.assert_allclose(x, O.policy_eval_neumann(mdp, pi), rtol=1e-12)


def test_cycle_closed_form():
    # single action, deterministic n-cycle: V(s) = sum_t gamma^t c(s+t) / (1 - gamma^n)
    n, g = 7, 0.8
    mdp = synth.cyclic(n, 1, g, seed=4)
    c = mdp.cost
    want = np.array([sum(g ** t * c[(s + t) % n] for t in range(n)) / (1 - g ** n)
                     for s in range(n)])
    np.testing.assert_allclose(O.policy_eval_lu(mdp, np.zeros(n, np.int32)), want, rtol=1e-13)
    # GMRES needs the full Krylov dimension n here (Lemma 1: spectrum on a circle)
    x, info = O.gmres_inner(mdp, np.zeros(n, np.int32), np.zeros(n), alpha=1e-13, W=n)
    np.testing.assert_allclose(x, want, rtol=1e-11)
    assert info["steps"] == n


def test_tie_rule_lowest_index():
    # actions 0 and 2 identical and best; GreedyPolicy must return 0
    rows, cost = [], []
    for s in range(3):
        rows += [[(s, 1.0)], [((s + 1) % 3, 1.0)], [(s, 1.0)]]
        cost += [0.1, 0.5, 0.1]
    mdp = synth.from_rows(3, 3, 0.9, rows, cost)
    _, pi, _ = O.bellman(mdp, np.zeros(3))
    assert pi.tolist() == [0, 0, 0]
    # PI keeps the incumbent on a tie
    newpi = O.greedy_keep(mdp, np.full(3, 1.0), np.array([2, 0, 2], np.int32))
    assert newpi.tolist() == [2, 0, 2]


# ---------------------------------------------------------------- properties

@pytest.fixture(scope="module")
def small():
    return synth.sparse_uniform(80, 4, 6, 0.9, seed=11)


def test_operator_properties(small):
    rng = np.random.default_rng(5)
    g = small.gamma
    for _ in range(5):
        V1, V2 = rng.normal(size=80) * 3, rng.normal(size=80) * 3
        T1, _, _ = O.bellman(small, V1)
        T2, _, _ = O.bellman(small, V2)
        assert np.max(np.abs(T1 - T2)) <= g * np.max(np.abs(V1 - V2)) * (1 + 1e-12)   # contraction
        r1, r2 = V1 - T1, V2 - T2
        assert np.max(np.abs(r1 - r2)) <= (1 + g) * np.max(np.abs(V1 - V2)) * (1 + 1e-12)  # Lemma 2
        Tup, _, _ = O.bellman(small, np.maximum(V1, V2))
        assert np.all(Tup >= np.maximum(T1, T2) - 1e-13)                           # monotone
        c = rng.normal()
        Ts, _, _ = O.bellman(small, V1 + c)
        np.testing.assert_allclose(Ts, T1 + g * c, rtol=0, atol=1e-13)             # shift


def test_lemma1_and_lemma3(small):
    g = small.gamma
    pi = np.random.default_rng(1).integers(0, 4, size=80).astype(np.int32)
    A = np.eye(80) - g * O.policy_matrix_dense(small, pi)
    ev = np.linalg.eigvals(A)
    assert np.all(np.abs(ev - 1.0) <= g * (1 + 1e-10))
    Ainv = np.linalg.inv(A)
    assert np.max(np.abs(Ainv).sum(axis=1)) == pytest.approx(1 / (1 - g), rel=1e-12)


def test_neumann_matches_lu(small):
    pi = np.random.default_rng(2).integers(0, 4, size=80).astype(np.int32)
    np.testing.assert_allclose(O.policy_eval_lu(small, pi), O.policy_eval_neumann(small, pi),
                               rtol=1e-12)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(6))
def test_brute_force_agrees_with_pi_vi(seed):
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(2, 7)), int(rng.integers(1, 4))
    mdp = synth.random_micro(n, m, float(rng.choice([0.5, 0.9, 0.99])), seed=seed)
    Vb, opt = O.brute_force(mdp)
    Vp, pip, _ = O.policy_iteration(mdp)
    np.testing.assert_allclose(Vp, Vb, rtol=1e-12)
    assert any(np.array_equal(pip, p) for p in opt)
    Vv, _ = O.value_iteration(mdp)
    np.testing.assert_allclose(Vv, Vb, rtol=1e-10)
    TV, _, _ = O.bellman(mdp, Vb)
    np.testing.assert_allclose(TV, Vb, rtol=1e-13)                 # V* = T V*
    # GMRES(W) with W >= n is exact within one cycle (at most n steps, Sec. 2.2)
    Vg, pig, st = O.igmres_pi(mdp, W=n, tol=1e-11 * max(1.0, float(np.max(np.abs(Vb)))))
    np.testing.assert_allclose(Vg, Vb, rtol=1e-10)
    assert st.converged


# ---------------------------------------------------------------- GMRES

def test_gmres_minimum_residual_property():
    """x_i = argmin ||b - J x||_2 over x0 + K_i (eq. 13), K_i spanned by the
    explicitly formed Krylov matrix [r0, J r0, ..., J^{i-1} r0]."""
    mdp = synth.sparse_uniform(40, 3, 5, 0.95, seed=7)
    pi = np.random.default_rng(3).integers(0, 3, size=40).astype(np.int32)
    x0 = np.random.default_rng(4).normal(size=40)
    _, info = O.gmres_inner(mdp, pi, x0, alpha=1e-15, W=8, trace=True, max_inner=6)
    b = O.policy_cost(mdp, pi)
    J = lambda v: O.j_apply(mdp, pi, v)  # noqa: E731
    r0 = b - J(x0)
    K = [r0 / np.linalg.norm(r0)]
    for i, xi in enumerate(info["iterates"], start=1):
        Km = np.stack(K, axis=1)
        JK = np.stack([J(v) for v in K], axis=1)
        c, *_ = np.linalg.lstsq(JK, r0, rcond=None)
        want = x0 + Km @ c
        np.testing.assert_allclose(xi, want, rtol=1e-9, atol=1e-9)
        nxt = J(K[-1])
        K.append(nxt / np.linalg.norm(nxt))


@pytest.mark.parametrize("W", [1, 2, 5, 40])
def test_gmres_restarted_converges_to_lu(W):
    mdp = synth.sparse_uniform(50, 3, 5, 0.9, seed=8)
    pi = np.random.default_rng(9).integers(0, 3, size=50).astype(np.int32)
    x, info = O.gmres_inner(mdp, pi, np.zeros(50), alpha=1e-13, W=W)
    np.testing.assert_allclose(x, O.policy_eval_lu(mdp, pi), rtol=1e-11)
    if W < 10:
        assert info["restarts"] >= 1


def test_gmres_stagnation_guard_ends_inner_loop():
    # restarted GMRES(3) stagnates completely on this 4-state system
    mdp = synth.random_micro(4, 2, 0.99, seed=1)
    pi = np.array([1, 0, 0, 1], np.int32)
    V = np.array([-4.86186671, -5.50835827, -4.59732929, -5.18435778])
    x, info = O.gmres_inner(mdp, pi, V, alpha=1e-3, W=3)
    assert info["stagnated"] and info["steps"] < 100
    x, info = O.gmres_inner(mdp, pi, V, alpha=1e-3, W=4)
    assert not info["stagnated"] and info["res_inf"] <= info["thr"]


def test_gmres_inexact_rule_holds():
    mdp = synth.sparse_uniform(200, 4, 6, 0.99, seed=10)
    pi = np.zeros(200, np.int32)
    x0 = np.zeros(200)
    b = O.policy_cost(mdp, pi)
    r0 = np.max(np.abs(b - O.j_apply(mdp, pi, x0)))
    for alpha in (0.5, 0.1, 1e-3):
        x, info = O.gmres_inner(mdp, pi, x0, alpha=alpha, W=10)
        r = np.max(np.abs(b - O.j_apply(mdp, pi, x)))
        assert r <= alpha * r0
        # and it stopped at the first step that satisfied the rule
        if info["steps"] > 1:
            _, info2 = O.gmres_inner(mdp, pi, x0, alpha=alpha, W=10, max_inner=info["steps"] - 1)
            assert info2["res_inf"] > alpha * r0


def test_igmres_pi_matches_pi_lu_c1():
    mdp = synth.config("c1", seed=0)
    Vs, pis, _ = O.policy_iteration(mdp)
    V, pi, st = O.igmres_pi(mdp, W=20, tol=1e-11)
    assert st.converged
    assert np.max(np.abs(V - Vs)) / np.max(np.abs(Vs)) <= 1e-10
    gaps = O.action_gaps(mdp, Vs)
    assert np.array_equal(pi[gaps > 1e-9], pis[gaps > 1e-9])
    assert O.certificate(mdp, V) >= np.max(np.abs(V - Vs))


def test_opi_one_sweep_is_vi(small):
    # OPI with one sweep per outer step is VI (Section 2.1): same stopping index
    tol = 1e-6
    Vo, _, outer, total = O.opi(small, 1, tol=tol)
    assert total == outer
    g = small.gamma
    Vv, sweeps = O.value_iteration(small, eps=tol * g / (1 - g))
    # VI stops one application later (it tests the step it just took)
    assert sweeps == outer + 1
    TVo, _, _ = O.bellman(small, Vo)
    np.testing.assert_array_equal(TVo, Vv)


def test_opi_two_sweeps_hand_trajectory():
    """OPI(2) on the two-state example, every step solved by hand
    (tests/golden/two_state_opi.json): the outer step, the number of
    applications of T^pi, the iterate and the greedy policy at each stop."""
    mdp, _ = two_state()
    d = json.load(open(os.path.join(GOLD, "two_state_opi.json")))
    for row in d["stops"]:
        V, pi, outer, total = O.opi(mdp, d["sweeps"], tol=row["tol"], V0=np.array(d["V0"]))
        assert (outer, total) == (row["outer"], row["total_sweeps"]), row
        np.testing.assert_array_equal(V, row["V"])
        assert pi.tolist() == row["pi"]
        _, _, res = O.bellman(mdp, V)
        assert res == row["res"]
    # exact PI from the same start: the W -> infinity limit of OPI
    seq = []
    O.policy_iteration(mdp, V0=np.array(d["V0"]), trace=seq)
    assert [p.tolist() for p in seq] == d["pi_sequence_PI"]


@pytest.mark.parametrize("case", ["c1-0", "c1-1", "c1-2", "u200"])
def test_opi_many_sweeps_is_policy_iteration(case):
    """Sec. 2.1: as the number W of T^pi applications per step grows, OPI
    becomes PI.  With gamma^W below the rounding unit, (T^pi)^W V equals
    V^pi to rounding, so OPI's greedy policies are exact PI's (LU
    evaluation) and it stops one step after evaluating the optimal policy."""
    if case.startswith("c1"):
        mdp = synth.config("c1", int(case[-1]))
    else:
        mdp = synth.sparse_uniform(200, 4, 6, 0.99, seed=31)
    W = int(np.ceil(np.log(1e-20) / np.log(mdp.gamma)))
    seq_pi, seq_opi = [], []
    Vp, pip, it = O.policy_iteration(mdp, trace=seq_pi)
    Vo, pio, outer, total = O.opi(mdp, W, tol=1e-10 * np.max(np.abs(Vp)), trace=seq_opi)
    assert outer == it and total == it * W
    for a, b in zip(seq_pi, seq_opi[:it]):
        assert np.array_equal(a, b)
    assert np.array_equal(seq_opi[it], pip)
    np.testing.assert_allclose(Vo, Vp, rtol=1e-12)


def test_certificate_bounds_error(small):
    Vs, _, _ = O.policy_iteration(small)
    rng = np.random.default_rng(12)
    for scale in (1e-2, 1e-5, 1e-9):
        V = Vs + scale * rng.normal(size=small.n)
        assert np.max(np.abs(V - Vs)) <= O.certificate(small, V) * (1 + 1e-9) + 1e-15


# ---- state-dependent action sets A(s) (Section 2) --------------------------

def _masked(base, keep, seed, **kw):
    return synth.with_action_sets(base, keep, seed, **kw)


def _penalty_twin(base, adm):
    """The same MDP without a mask, every inadmissible action given a cost no
    optimal or greedy choice can afford: c_pen = 10 max|c| / (1 - gamma) + 1."""
    cost = np.asarray(base.cost, np.float64).copy()
    big = 10.0 * np.max(np.abs(cost)) / (1.0 - base.gamma) + 1.0
    cost[~adm] = big
    return synth.MDP(base.n, base.m, base.gamma, cost, base.fmt, base.row_ptr, base.col,
                     base.val, base.P, base.name + "-pen", dict(base.meta))


@pytest.mark.parametrize("seed", range(4))
def test_action_sets_brute_force_matches_pi(seed):
    mdp = _masked(synth.random_micro(4, 3, 0.9, seed), 0.5, seed)
    adm = mdp.adm.reshape(mdp.n, mdp.m)
    Vb, opts = O.brute_force(mdp)
    Vp, pip, _ = O.policy_iteration(mdp)
    assert np.allclose(Vp, Vb, rtol=1e-10, atol=1e-12)
    assert any(np.array_equal(pip, o) for o in opts)
    assert adm[np.arange(mdp.n), pip].all()
    # every optimal policy found by enumeration is admissible
    assert all(adm[np.arange(mdp.n), o].all() for o in opts)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_action_sets_equal_prohibitive_costs(seed):
    """A mask (with the rows and costs of inadmissible pairs removed or NaN)
    and a mask-free twin whose inadmissible actions cost too much to be
    chosen give the same PI trajectory, hence the same V* and pi*."""
    base = synth.config("c1", seed)
    mdp = _masked(base, 0.6, 7 + seed)
    twin = _penalty_twin(base, mdp.adm)
    V1, pi1, it1 = O.policy_iteration(mdp)
    V2, pi2, it2 = O.policy_iteration(twin)
    assert it1 == it2
    assert np.array_equal(pi1, pi2)
    assert np.allclose(V1, V2, rtol=1e-12, atol=0)
    Vv, _ = O.value_iteration(mdp)
    assert np.allclose(Vv, V1, rtol=1e-9)


def test_action_sets_restriction_raises_values():
    """Minimising over a subset of actions can only raise V* (eq. 2)."""
    base = synth.config("c1", 3)
    Vf, _, _ = O.policy_iteration(base)
    for keep in (0.8, 0.5, 0.3):
        Vm, _, _ = O.policy_iteration(_masked(base, keep, 11))
        assert np.all(Vm >= Vf - 1e-12 * np.max(np.abs(Vf)))


def test_action_sets_single_action_states():
    """A state with one admissible action a: pi*(s) = a and V*(s) solves the
    Bellman equation with that action alone."""
    base = synth.config("c1", 4)
    mdp = _masked(base, 0.35, 5)
    adm = mdp.adm.reshape(mdp.n, mdp.m)
    V, pi, _ = O.policy_iteration(mdp)
    single = np.nonzero(adm.sum(axis=1) == 1)[0]
    assert single.size > 0
    a = np.argmax(adm[single], axis=1)
    assert np.array_equal(pi[single], a)
    rows = O._P_rows(base)[single * mdp.m + a]
    rhs = base.cost.reshape(mdp.n, mdp.m)[single, a] + mdp.gamma * (rows @ V)
    assert np.allclose(V[single], rhs, rtol=1e-12)


def test_action_sets_full_mask_is_plain():
    base = synth.config("c1", 1)
    full = synth.MDP(base.n, base.m, base.gamma, base.cost, base.fmt, base.row_ptr, base.col,
                     base.val, base.P, "full", dict(base.meta), np.ones(base.n * base.m, bool))
    V1, pi1, _ = O.policy_iteration(base)
    V2, pi2, _ = O.policy_iteration(full)
    assert np.array_equal(pi1, pi2) and np.array_equal(V1, V2)
    TV1, p1, r1 = O.bellman(base, V1)
    TV2, p2, r2 = O.bellman(full, V1)
    assert np.array_equal(TV1, TV2) and np.array_equal(p1, p2)


def test_action_sets_igmres_pi_reaches_masked_optimum():
    base = synth.config("c1", 2)
    mdp = _masked(base, 0.5, 3)
    Vs, pis, _ = O.policy_iteration(mdp)
    V, pi, st = O.igmres_pi(mdp, W=20, tol=1e-11)
    assert st.converged
    assert np.max(np.abs(V - Vs)) <= 1e-9 * np.max(np.abs(Vs))
    gaps = O.action_gaps(mdp, Vs)
    sel = gaps > 1e-9
    assert np.array_equal(pi[sel], pis[sel])


# ---- right preconditioning with the truncated Neumann series ----------------

@pytest.mark.parametrize("d", [1, 2, 5])
def test_neumann_closed_form(d):
    """J M^{-1} = I - (gamma P^pi)^{d+1} for M^{-1} = sum_{k<=d} (gamma P^pi)^k
    (the two commute); the right side is formed by repeated products."""
    mdp = synth.sparse_uniform(60, 3, 6, 0.97, seed=21)
    pi = np.random.default_rng(2).integers(0, 3, size=60).astype(np.int32)
    x = np.random.default_rng(3).normal(size=60)
    lhs = O.j_apply(mdp, pi, O.neumann_apply(mdp, pi, x, d))
    Ppi = O.policy_matrix_dense(mdp, pi)
    p = x.copy()
    for _ in range(d + 1):
        p = mdp.gamma * (Ppi @ p)
    np.testing.assert_allclose(lhs, x - p, rtol=1e-12, atol=1e-12)
    # and M^{-1} -> J^{-1} as d grows (Lemma 3's series)
    big = O.neumann_apply(mdp, pi, x, 3000)
    np.testing.assert_allclose(O.j_apply(mdp, pi, big), x, rtol=1e-9, atol=1e-9)


def test_preconditioned_gmres_minimum_residual_property():
    """Right-preconditioned GMRES: x_i = argmin ||b - J x||_2 over
    x0 + M^{-1} K_i(J M^{-1}, r0), from an explicitly formed Krylov matrix."""
    d = 2
    mdp = synth.sparse_uniform(40, 3, 5, 0.95, seed=7)
    pi = np.random.default_rng(3).integers(0, 3, size=40).astype(np.int32)
    x0 = np.random.default_rng(4).normal(size=40)
    _, info = O.gmres_inner(mdp, pi, x0, alpha=1e-15, W=8, trace=True, max_inner=6, precond=d)
    b = O.policy_cost(mdp, pi)
    J = lambda v: O.j_apply(mdp, pi, v)  # noqa: E731
    Minv = lambda v: O.neumann_apply(mdp, pi, v, d)  # noqa: E731
    r0 = b - J(x0)
    K = [r0 / np.linalg.norm(r0)]
    for xi in info["iterates"]:
        MK = np.stack([Minv(v) for v in K], axis=1)
        JMK = np.stack([J(v) for v in MK.T], axis=1)
        c, *_ = np.linalg.lstsq(JMK, r0, rcond=None)
        np.testing.assert_allclose(xi, x0 + MK @ c, rtol=1e-9, atol=1e-9)
        nxt = J(Minv(K[-1]))
        K.append(nxt / np.linalg.norm(nxt))


def test_preconditioner_degree_zero_is_plain_gmres():
    mdp = synth.config("c1", 0)
    V1, pi1, st1 = O.igmres_pi(mdp, W=20, tol=1e-10)
    V2, pi2, st2 = O.igmres_pi(mdp, W=20, tol=1e-10, precond=0)
    assert np.array_equal(V1, V2) and np.array_equal(pi1, pi2) and st1.inner == st2.inner


@pytest.mark.parametrize("d", [1, 3])
def test_preconditioned_igmres_reaches_optimum_in_fewer_steps(d):
    mdp = synth.config("c1", 1)
    Vs, pis, _ = O.policy_iteration(mdp)
    tol = 1e-11 * np.max(np.abs(Vs))
    V0, _, st0 = O.igmres_pi(mdp, W=20, tol=tol)
    V, pi, st = O.igmres_pi(mdp, W=20, tol=tol, precond=d)
    assert st.converged
    assert np.max(np.abs(V - Vs)) <= 1e-9 * np.max(np.abs(Vs))
    sel = O.action_gaps(mdp, Vs) > 1e-9
    assert np.array_equal(pi[sel], pis[sel])
    # each preconditioned step covers d+1 products: fewer Arnoldi steps
    assert st.inner < st0.inner


# --- forcing sequence alpha_k = min(alpha, ||T V_k - V_k||_inf^(1/2)) (Theorem 1) ---

def test_forcing_equals_constant_alpha_while_alpha_is_smaller():
    """While sqrt(||T V_k - V_k||) >= alpha at every outer step, alpha_k is alpha
    and the forcing run is Algorithm 2 itself, bit for bit."""
    mdp = synth.config("c1", 0)
    alpha = 0.5 * (1 - mdp.gamma) / (1 + mdp.gamma)
    tol = 1e-3  # every residual seen before stopping stays above alpha^2 ~ 6.9e-4
    Va, pia, sta = O.igmres_pi(mdp, W=20, tol=tol)
    Vb, pib, stb = O.igmres_pi(mdp, W=20, tol=tol, forcing=True)
    assert sta.outer >= 3
    assert min(sta.res_history[:-1]) >= alpha ** 2
    assert np.array_equal(Va, Vb) and np.array_equal(pia, pib)
    assert sta.inner == stb.inner and sta.res_history == stb.res_history


def test_forcing_inexactness_condition_each_outer_step():
    """Each outer step's inner solve ends with ||g^pi - J^pi V_{k+1}||_inf <=
    alpha_k ||T V_k - V_k||_inf (eq. 11 with alpha_k), and alpha_k falls below
    the constant alpha once the residual is small; replayed step by step with
    max_outer, the runs are prefixes of each other."""
    mdp = synth.sparse_uniform(400, 4, 6, 0.99, seed=21)
    alpha = 0.5 * (1 - mdp.gamma) / (1 + mdp.gamma)
    V, pi, st = O.igmres_pi(mdp, W=15, tol=1e-11, forcing=True)
    assert st.converged
    Vk = np.zeros(mdp.n)
    for k in range(st.outer):
        _, pik, res = O.bellman(mdp, Vk)
        Vn, _, stk = O.igmres_pi(mdp, W=15, tol=0.0, max_outer=k + 1, forcing=True)
        r = np.max(np.abs(O.policy_cost(mdp, pik) - O.j_apply(mdp, pik, Vn)))
        ak = st.alpha_history[k]
        assert ak <= alpha and ak > 0.0
        assert r <= ak * res * (1 + 1e-12)
        Vk = Vn
    assert min(st.alpha_history) < alpha / 10
    np.testing.assert_array_equal(Vk, V)


@pytest.mark.parametrize("seed", [0, 1])
def test_forcing_superlinear_and_optimal(seed):
    """Theorem 1: with alpha_k -> 0 the residual ratio ||T V_{k+1} - V_{k+1}|| /
    ||T V_k - V_k|| tends to zero, while the constant-alpha run contracts at a
    steady rate; both end at PI-LU's V* with an optimal policy."""
    mdp = synth.config("c1", seed)
    Vs, pis, _ = O.policy_iteration(mdp)
    tol = 1e-11 * np.max(np.abs(Vs))
    V, pi, st = O.igmres_pi(mdp, W=20, tol=tol, forcing=True)
    V0, _, st0 = O.igmres_pi(mdp, W=20, tol=tol)
    assert st.converged and st0.converged
    assert np.max(np.abs(V - Vs)) <= 1e-9 * np.max(np.abs(Vs))
    sel = O.action_gaps(mdp, Vs) > 1e-9
    assert np.array_equal(pi[sel], pis[sel])
    rf = np.asarray(st.res_history)
    r0 = np.asarray(st0.res_history)
    ratios_f = rf[-3:] / rf[-4:-1]
    ratios_0 = r0[-3:] / r0[-4:-1]
    assert ratios_f[-1] < ratios_f[0] and ratios_f[-1] < 1e-3
    assert np.min(ratios_0) > 10 * ratios_f[-1]
    assert st.outer <= st0.outer


# --- polish: one evaluation to tol / 2 once the greedy policy repeats ---

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_polish_prefix_termination_and_optimum(seed):
    mdp = synth.config("c1", seed)
    Vs, pis, _ = O.policy_iteration(mdp)
    tol = 1e-11 * np.max(np.abs(Vs))
    V, pi, st = O.igmres_pi(mdp, W=20, tol=tol, polish=True)
    V0, _, st0 = O.igmres_pi(mdp, W=20, tol=tol)
    assert st.converged and st.polished
    # the same run as plain Algorithm 2 until the first repeated policy
    p0 = st.polished[0]
    assert st.res_history[:p0 + 1] == st0.res_history[:p0 + 1]
    Va, _, _ = O.igmres_pi(mdp, W=20, tol=0.0, max_outer=p0, polish=True)
    Vb, _, _ = O.igmres_pi(mdp, W=20, tol=0.0, max_outer=p0)
    np.testing.assert_array_equal(Va, Vb)
    # the polished evaluation meets tol / 2 on its own policy, and the
    # following Bellman residual meets tol while the policy holds
    k = st.polished[-1]
    Vk, pik, _ = O.igmres_pi(mdp, W=20, tol=0.0, max_outer=k, polish=True)
    Vn, pin, _ = O.igmres_pi(mdp, W=20, tol=0.0, max_outer=k + 1, polish=True)
    _, pik, _ = O.bellman(mdp, Vk)
    r = np.max(np.abs(O.policy_cost(mdp, pik) - O.j_apply(mdp, pik, Vn)))
    assert r <= 0.5 * tol * (1 + 1e-12)
    _, pi_next, res_next = O.bellman(mdp, Vn)
    if np.array_equal(pi_next, pik):
        assert res_next <= tol and st.outer == k + 1
    # optimum, in no more outer steps than the plain run
    assert np.max(np.abs(V - Vs)) <= 1e-9 * np.max(np.abs(Vs))
    sel = O.action_gaps(mdp, Vs) > 1e-9
    assert np.array_equal(pi[sel], pis[sel])
    assert st.outer <= st0.outer
