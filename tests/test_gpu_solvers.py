"""igmres_pi_solve, pi_solve, opi_solve and ipi_vi_solve against V* and pi*
of the FP64 oracle (PI with dense LU evaluation, pinned by brute force and
closed forms), plus iteration counts of the literal Algorithm 2."""
import os

import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import (assert_inner_parity, assert_policy_match, dev_vec, host, rel_err,
                         residual_floor, tol_par, zeros)

pytestmark = pytest.mark.gpu


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


_cache = {}


def reference(name, seed):
    key = (name, seed)
    if key not in _cache:
        mdp = synth.config(name, seed)
        Vs, pis, _ = O.policy_iteration(mdp)
        _cache[key] = (mdp, Vs, pis)
    return _cache[key]


def solve(mdp, method="igmres_pi_solve", store="fp64", V0=None, allow_noconv=False, **kw):
    I = igm()
    with I.mdp_create(mdp, store=store) as h:
        V = dev_vec(np.zeros(mdp.n) if V0 is None else V0)
        pi = zeros(mdp.n, "int32")
        p = I.params_default(mdp.gamma, **kw)
        st = getattr(h, method)(V, pi, p, allow_noconv=allow_noconv)
        return host(V), host(pi), st


ENGINES = [1, 2]  # one launch per step; one persistent launch per solve


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_igmres_c1_parity(seed, engine):
    mdp, Vs, pis = reference("c1", seed)
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    V, pi, st = solve(mdp, tol=tol, restart=20, engine=engine)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)
    assert np.max(np.abs(V - Vs)) <= st["cert_bound"] * (1 + 1e-9) + 1e-15
    # same trajectory as the literal Algorithm 2
    Vo, pio, sto = O.igmres_pi(mdp, W=20, tol=tol)
    assert st["outer"] == sto.outer
    assert st["inner"] == sto.inner  # the literal stopping index, step for step


@pytest.mark.parametrize("engine", ENGINES)
def test_igmres_c2_bench_configuration(engine):
    """The timed workload: n=1e4, m=8, k=20, gamma=0.99, W=30, tol 1e-8."""
    mdp, Vs, pis = reference("c2", 0)
    V, pi, st = solve(mdp, tol=1e-8, restart=30, engine=engine)
    assert st["converged"] == 1 and st["res_inf"] <= 1e-8
    assert rel_err(V, Vs) <= 1e-8
    Vo, pio, sto = O.igmres_pi(mdp, W=30, tol=1e-8)
    assert st["outer"] == sto.outer
    assert st["inner"] == sto.inner  # the literal stopping index, step for step


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_igmres_c2_parity_tight(seed, engine):
    mdp, Vs, pis = reference("c2", seed)
    V, pi, st = solve(mdp, tol=tol_par(mdp, np.max(np.abs(Vs))), restart=30, engine=engine)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)



@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("name,seed,W", [("c1", 0, 20), ("c1", 1, 20), ("c2", 0, 30)])
def test_igmres_forcing_parity(name, seed, W, engine):
    """forcing=1: alpha_k = min(alpha, sqrt(||T V_k - V_k||_inf)), Theorem 1's
    superlinear case; same V*, policy and outer steps as the oracle's run
    with the same forcing sequence, and no more outer steps than alpha_k = alpha."""
    mdp, Vs, pis = reference(name, seed)
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    V, pi, st = solve(mdp, tol=tol, restart=W, engine=engine, forcing=1)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)
    trace = []
    Vo, pio, sto = O.igmres_pi(mdp, W=W, tol=tol, forcing=True, inner_trace=trace)
    assert st["outer"] == sto.outer
    assert_inner_parity(st, sto, trace, lambda k: solve(
        mdp, tol=tol, restart=W, engine=engine, forcing=1, max_outer=k, allow_noconv=True)[2]["inner"],
        floor=residual_floor(mdp, Vs))
    _, _, st0 = solve(mdp, tol=tol, restart=W, engine=engine)
    assert st["outer"] <= st0["outer"]



@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("name,seed,W", [("c1", 0, 20), ("c1", 2, 20), ("c2", 0, 30)])
def test_igmres_polish_parity(name, seed, W, engine):
    """polish=1: once the greedy policy repeats, one evaluation to tol / 2;
    same V*, policy and outer steps as the oracle's run with polish, and no
    more outer steps than without it."""
    mdp, Vs, pis = reference(name, seed)
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    V, pi, st = solve(mdp, tol=tol, restart=W, engine=engine, polish=1)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)
    trace = []
    Vo, pio, sto = O.igmres_pi(mdp, W=W, tol=tol, polish=True, inner_trace=trace)
    assert sto.polished
    assert st["outer"] == sto.outer
    assert_inner_parity(st, sto, trace, lambda k: solve(
        mdp, tol=tol, restart=W, engine=engine, polish=1, max_outer=k, allow_noconv=True)[2]["inner"],
        floor=residual_floor(mdp, Vs))
    _, _, st0 = solve(mdp, tol=tol, restart=W, engine=engine)
    assert st["outer"] <= st0["outer"]


def test_igmres_polish_dense_mixed():
    """The stream engine's dense Bellman kernels count policy changes too."""
    mdp = synth.dense_exp(300, 4, 0.99, seed=5)
    stored = mdp.with_values(P=synth.upcast_values(synth.round_values(mdp.P, "fp32"), "fp32"))
    Vs, pis, _ = O.policy_iteration(stored)
    tol = tol_par(stored, np.max(np.abs(Vs)))
    V, pi, st = solve(mdp, store="fp32", mode="mixed", tol=tol, restart=20, polish=1)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-6
    Vo, _, sto = O.igmres_pi(stored, W=20, tol=tol, polish=True)
    assert sto.polished and st["outer"] == sto.outer

def test_ipi_vi_forcing_c1():
    mdp, Vs, pis = reference("c1", 1)
    V, pi, st = solve(mdp, method="ipi_vi_solve", tol=1e-10, forcing=1)
    assert st["converged"] == 1
    assert np.max(np.abs(V - Vs)) <= 1e-10 / (1 - mdp.gamma) * (1 + 1e-6)

def test_pi_solve_c2():
    mdp, Vs, pis = reference("c2", 0)
    V, pi, st = solve(mdp, method="pi_solve", restart=30)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-10
    assert_policy_match(mdp, Vs, pis, pi)


def test_opi_c2_and_c1():
    for name in ("c1", "c2"):
        mdp, Vs, pis = reference(name, 0)
        V, pi, st = solve(mdp, method="opi_solve", opi_sweeps=20, tol=1e-8)
        assert st["converged"] == 1
        assert np.max(np.abs(V - Vs)) <= 1e-8 / (1 - mdp.gamma) * (1 + 1e-6)
        Vo, _, outer, total = O.opi(mdp, 20, tol=1e-8)
        assert st["outer"] == outer
        np.testing.assert_allclose(V, Vo, rtol=1e-10)


def test_ipi_vi_c1():
    mdp, Vs, pis = reference("c1", 1)
    V, pi, st = solve(mdp, method="ipi_vi_solve", tol=1e-10)
    assert st["converged"] == 1
    assert np.max(np.abs(V - Vs)) <= 1e-10 / (1 - mdp.gamma) * (1 + 1e-6)


def test_dense_fp64_igmres():
    mdp = synth.dense_exp(400, 4, 0.99, seed=3)
    Vs, pis, _ = O.policy_iteration(mdp)
    V, pi, st = solve(mdp, tol=tol_par(mdp, np.max(np.abs(Vs))), restart=30)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("store", ["fp32", "bf16"])
def test_mixed_precision_against_stored_mdp_oracle(store, engine):
    mdp = synth.config("c2", seed=1, n=3000)
    stored = mdp.with_values(val=synth.upcast_values(synth.round_values(mdp.val, store), store))
    Vs, pis, _ = O.policy_iteration(stored)
    V, pi, st = solve(mdp, store=store, mode="mixed", restart=30, engine=engine,
                      tol=tol_par(stored, np.max(np.abs(Vs))))
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-6
    assert_policy_match(stored, Vs, pis, pi)


def test_dense_bf16_mixed():
    mdp = synth.dense_exp(300, 4, 0.99, seed=5)
    stored = mdp.with_values(P=synth.upcast_values(synth.round_values(mdp.P, "bf16"), "bf16"))
    Vs, pis, _ = O.policy_iteration(stored)
    V, pi, st = solve(mdp, store="bf16", mode="mixed", tol=tol_par(stored, np.max(np.abs(Vs))))
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-6


def test_warm_start_at_solution_does_no_inner_work():
    mdp, Vs, pis = reference("c1", 0)
    V, pi, st = solve(mdp, V0=Vs, tol=1e-8)
    assert st["outer"] == 0 and st["inner"] == 0 and st["converged"] == 1


def test_single_state_closed_form():
    mdp = synth.self_loops(1, 3, 0.9, seed=2)
    V, pi, st = solve(mdp, tol=1e-12)
    assert V[0] == pytest.approx(mdp.cost.min() / 0.1, rel=1e-12)
    assert pi[0] == int(np.argmin(mdp.cost))


@pytest.mark.parametrize("engine", ENGINES)
def test_deterministic_bits(engine):
    mdp, _, _ = reference("c2", 0)
    a = solve(mdp, tol=1e-10, engine=engine)[0]
    b = solve(mdp, tol=1e-10, engine=engine)[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [64, 65, 5000, 40000])
def test_persistent_engine_shapes(n):
    """Block ownership of 1, 2 and several slices per block, ragged tails."""
    mdp = synth.sparse_uniform(n, 5, 7, 0.97, seed=n)
    Vs, pis, _ = O.policy_iteration(mdp) if n <= 5000 else (None, None, None)
    I = igm()
    with I.mdp_create(mdp) as h:
        assert h.info().persistent_ok == 1
    Va, pia, sta = solve(mdp, tol=1e-10, engine=1)
    Vb, pib, stb = solve(mdp, tol=1e-10, engine=2)
    assert sta["converged"] == 1 and stb["converged"] == 1
    assert stb["outer"] == sta["outer"]
    assert abs(stb["inner"] - sta["inner"]) <= sta["outer"]
    np.testing.assert_allclose(Vb, Va, rtol=1e-10)
    if Vs is not None:
        assert rel_err(Vb, Vs) <= 1e-8
    else:  # too large for the LU oracle: one FP64 Bellman pass on the host
        TV, pig, res = O.bellman(mdp, Vb)
        assert res <= 1e-10 * (1 + 1e-6) + 1e-14
        assert O.certificate(mdp, Vb) <= 1e-8 * np.max(np.abs(Vb))
        gaps = O.action_gaps(mdp, Vb)
        assert np.array_equal(pib[gaps > 1e-9], pig[gaps > 1e-9])


@pytest.mark.parametrize("engine", ENGINES)
def test_noconv_and_bad_params(engine):
    I = igm()
    mdp, _, _ = reference("c1", 0)
    V, pi, st = solve(mdp, max_outer=1, tol=1e-14, allow_noconv=True, engine=engine)
    assert st["status"] == I.IG_E_NOCONV and st["converged"] == 0
    for kw, code in [(dict(alpha=0.0), I.IG_E_INVALID), (dict(restart=0), I.IG_E_INVALID),
                     (dict(restart=129), I.IG_E_TOO_LARGE), (dict(tol=0.0), I.IG_E_INVALID)]:
        with pytest.raises(I.IgError) as e:
            solve(mdp, **kw)
        assert e.value.status == code


@pytest.mark.parametrize("W,engine", [(1, 1), (1, 2), (2, 1), (2, 2), (64, 1), (64, 2), (128, 1)])
def test_restart_extremes(W, engine):
    """GMRES(1) and GMRES(2) (restart after every one or two steps), the
    persistent engine's cap of 64 and the interface's cap of 128 columns:
    V*, the optimal policy and the outer steps of the oracle's Algorithm 2
    with the same W."""
    mdp = synth.config("c1", 1) if W <= 2 else synth.sparse_uniform(3000, 4, 8, 0.99, seed=12)
    Vs, pis, _ = O.policy_iteration(mdp)
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    V, pi, st = solve(mdp, tol=tol, restart=W, engine=engine)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)
    Vo, _, sto = O.igmres_pi(mdp, W=W, tol=tol)
    assert st["outer"] == sto.outer
    if W <= 2:
        assert st["restarts"] > 0


def test_auto_engine_long_restart():
    """Engine 0 with a restart longer than the persistent engine holds runs on
    the stream engine: V*, pi* and the outer steps of the oracle's run."""
    mdp, Vs, pis = reference("c1", 0)
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    V, pi, st = solve(mdp, tol=tol, restart=100, engine=0)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)
    _, _, sto = O.igmres_pi(mdp, W=100, tol=tol)
    assert st["outer"] == sto.outer


def test_restart_caps_rejected():
    I = igm()
    mdp = synth.config("c1", 0)
    for W, engine in [(65, 2), (129, 1), (129, 0), (0, 1)]:
        with I.mdp_create(mdp) as h:
            V, pi = zeros(mdp.n), zeros(mdp.n, "int32")
            with pytest.raises(I.IgError) as ei:
                h.igmres_pi_solve(V, pi, I.params_default(mdp.gamma, restart=W, engine=engine))
            assert ei.value.status == (I.IG_E_INVALID if W == 0 else I.IG_E_TOO_LARGE)


def test_barrier_wait_limit_drains_and_reports():
    """Failure handling of the persistent engine, forced from the host: with
    a limit of zero polls per grid-barrier wait, a block that has to wait
    gives up and leaves; every other block leaves at its next barrier, so the
    launch ends, the call reports IG_E_DEVICE, and the next solve on the
    same handle is exact."""
    I = igm()
    mdp, Vs, pis = reference("c2", 0)
    with I.mdp_create(mdp) as h:
        V, pi = zeros(mdp.n), zeros(mdp.n, "int32")
        p = I.params_default(mdp.gamma, restart=30, engine=2)
        os.environ["IG_SPIN_LIMIT"] = "0"
        try:
            with pytest.raises(I.IgError) as ei:
                h.igmres_pi_solve(V, pi, p)
        finally:
            del os.environ["IG_SPIN_LIMIT"]
        assert ei.value.status == I.IG_E_DEVICE
        assert "barrier" in I.last_error()
        V.zero_()
        st = h.igmres_pi_solve(V, pi, p)
        Vh, pih = host(V), host(pi)
    assert st["converged"] == 1
    assert rel_err(Vh, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pih)


@pytest.mark.parametrize("store", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("method", ["pi_solve", "opi_solve", "ipi_vi_solve"])
def test_other_solvers_dense(method, store):
    """PI (policy gather and evaluation), OPI and inexact PI with VI sweeps on
    dense transition data: V* and the optimal policy of the stored MDP."""
    mdp = synth.dense_exp(400, 4, 0.99, seed=7)
    stored = mdp if store == "fp64" else mdp.with_values(
        P=synth.upcast_values(synth.round_values(mdp.P, store), store))
    Vs, pis, _ = O.policy_iteration(stored)
    tol = tol_par(stored, np.max(np.abs(Vs)))
    mode = "fp64" if store == "fp64" else "mixed"
    V, pi, st = solve(mdp, method=method, store=store, mode=mode, tol=tol, opi_sweeps=20)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= (1e-8 if store == "fp64" else 1e-6)
    assert_policy_match(stored, Vs, pis, pi)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n,m,k", [(300, 300, 3), (70, 1000, 2)])
def test_many_actions(n, m, k, engine):
    """Hundreds of actions per state (300 and 1000: rows of many actions per
    ELL slice and long per-state argmin chains): V* and pi* of PI with LU."""
    mdp = synth.sparse_uniform(n, m, k, 0.95, seed=m)
    Vs, pis, _ = O.policy_iteration(mdp)
    V, pi, st = solve(mdp, tol=tol_par(mdp, np.max(np.abs(Vs))), engine=engine)
    assert st["converged"] == 1
    assert rel_err(V, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pi)
