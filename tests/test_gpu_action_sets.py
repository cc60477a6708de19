"""State-dependent action sets A(s) on the GPU against the FP64 oracle
(mask on the Q-values; pinned by brute force and by a prohibitive-cost twin).
Excluded pairs have empty CSR rows and NaN costs, which must be ignored."""
import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import assert_policy_match, dev_vec, host, rel_err, tol_par, zeros

pytestmark = pytest.mark.gpu


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


_cache = {}


def case(name):
    if name not in _cache:
        if name == "c1":
            mdp = synth.with_action_sets(synth.config("c1", 5), 0.5, 5)
        elif name == "mid":
            mdp = synth.with_action_sets(synth.sparse_uniform(3000, 6, 12, 0.95, 9), 0.4, 9)
        elif name == "ragged":  # slices where only low action indices survive
            base = synth.sparse_uniform(1000, 8, 6, 0.9, 4)
            adm = np.zeros((base.n, base.m), bool)
            rng = np.random.default_rng(4)
            for s in range(base.n):
                top = 2 if (s // 64) % 2 == 0 else 8
                adm[s, rng.choice(top, size=rng.integers(1, top + 1), replace=False)] = True
            mdp = synth.MDP(base.n, base.m, base.gamma, base.cost, "csr", base.row_ptr, base.col,
                            base.val, None, "ragged", dict(base.meta), adm.reshape(-1))
        else:  # dense
            mdp = synth.with_action_sets(synth.dense_exp(300, 4, 0.9, 2), 0.5, 2)
        Vs, pis, _ = O.policy_iteration(mdp)
        _cache[name] = (mdp, Vs, pis)
    return _cache[name]


@pytest.mark.parametrize("name", ["c1", "mid", "ragged", "dense"])
def test_bellman_apply_masked(name):
    I = igm()
    mdp, Vs, _ = case(name)
    V0 = np.random.default_rng(1).random(mdp.n) * np.max(np.abs(Vs))
    TVo, pio, reso = O.bellman(mdp, V0)
    with I.mdp_create(mdp) as h:
        V = dev_vec(V0)
        TV = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        res = zeros(1)
        h.bellman_apply(V, TV, pi, res)
        TVg, pig, resg = host(TV), host(pi), host(res)[0]
    assert np.max(np.abs(TVg - TVo)) <= 1e-12 * np.max(np.abs(TVo))
    gaps = O.action_gaps(mdp, V0)
    sel = gaps > 1e-9
    assert np.array_equal(pig[sel], pio[sel])
    adm = mdp.adm.reshape(mdp.n, mdp.m)
    assert adm[np.arange(mdp.n), pig].all()
    assert abs(resg - reso) <= 1e-12 * max(1.0, reso)


@pytest.mark.parametrize("engine", [1, 2])
@pytest.mark.parametrize("name", ["c1", "mid", "ragged", "dense"])
def test_igmres_masked_parity(name, engine):
    I = igm()
    mdp, Vs, pis = case(name)
    if engine == 2 and mdp.fmt == "dense":
        pytest.skip("the persistent engine takes sparse MDPs")
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    with I.mdp_create(mdp) as h:
        V = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        st = h.igmres_pi_solve(V, pi, I.params_default(mdp.gamma, tol=tol, engine=engine))
        Vg, pig = host(V), host(pi)
    assert st["converged"] == 1
    assert rel_err(Vg, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pig)
    assert mdp.adm.reshape(mdp.n, mdp.m)[np.arange(mdp.n), pig].all()


@pytest.mark.parametrize("method", ["pi_solve", "opi_solve", "ipi_vi_solve"])
def test_other_solvers_masked(method):
    I = igm()
    mdp, Vs, pis = case("c1")
    tol = tol_par(mdp, np.max(np.abs(Vs)))
    with I.mdp_create(mdp) as h:
        V = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        getattr(h, method)(V, pi, I.params_default(mdp.gamma, tol=tol))
        Vg, pig = host(V), host(pi)
    assert rel_err(Vg, Vs) <= 1e-8
    assert_policy_match(mdp, Vs, pis, pig)


def test_policy_outside_action_set_is_rejected():
    I = igm()
    mdp, Vs, pis = case("c1")
    adm = mdp.adm.reshape(mdp.n, mdp.m)
    bad = pis.copy()
    s = int(np.nonzero(~adm.all(axis=1))[0][0])
    bad[s] = int(np.nonzero(~adm[s])[0][0])
    with I.mdp_create(mdp) as h:
        V = zeros(mdp.n)
        with pytest.raises(I.IgError) as e:
            h.policy_eval_gmres(dev_vec(bad.astype(np.int32), "int32"), V,
                                I.params_default(mdp.gamma))
        assert e.value.status == I.IG_E_INVALID
        # the optimal policy is accepted and evaluates to V*
        V2 = zeros(mdp.n)
        h.policy_eval_gmres(dev_vec(pis.astype(np.int32), "int32"), V2,
                            I.params_default(mdp.gamma, alpha=1e-12))
        assert rel_err(host(V2), Vs) <= 1e-9


def test_serving_masked_request():
    I = igm()
    mdp, Vs, pis = case("mid")
    with I.Server() as srv:
        V, pi, st = srv.result(srv.submit(mdp, I.params_default(mdp.gamma, mode="mixed"), store="fp32"))
    ref = mdp.with_values(val=synth.upcast_values(synth.round_values(mdp.val, "fp32"), "fp32"))
    TV, pio, res = O.bellman(ref, V)
    assert st["converged"] == 1 and res <= 1e-8 * (1 + 1e-6)
    assert mdp.adm.reshape(mdp.n, mdp.m)[np.arange(mdp.n), pi].all()
