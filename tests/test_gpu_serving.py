"""Continuous-batching serving (srv_* entry points).

Every served result is checked by the FP64 oracle's Bellman operator on the
stored (FP32-rounded) MDP: the contraction certificate
||V - V*||_inf <= ||T V - V||_inf / (1 - gamma) bounds the error without a
full solve, and the greedy policy must match wherever the action gap is
resolvable.  Batch invariance: each request's result is bitwise the same
served alone, in a mix, and through the direct persistent entry point with
the same workgroup count."""
import math
import os

import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import host, zeros

pytestmark = pytest.mark.gpu

TOL = 1e-8
BLOCK_SLICES = 16

# (n, m, k, gamma, seed): uneven sizes, from 2 slices to ~2000
MIX = [(1000, 4, 8, 0.9, 11), (3000, 2, 4, 0.99, 12), (20000, 16, 32, 0.95, 13),
       (7000, 8, 16, 0.99, 14), (65, 3, 5, 0.9, 15), (130000, 6, 12, 0.95, 16)]


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


_mdps = {}


def request_mdp(spec):
    if spec not in _mdps:
        n, m, k, g, seed = spec
        _mdps[spec] = synth.sparse_uniform(n, m, k, g, seed)
    return _mdps[spec]


def stored_ref(mdp):
    """The MDP the FP32-stored request defines (values as stored, in FP64)."""
    return mdp.with_values(val=synth.upcast_values(synth.round_values(mdp.val, "fp32"), "fp32"))


def params(mdp, **kw):
    I = igm()
    kw.setdefault("tol", TOL)
    kw.setdefault("mode", "mixed")
    return I.params_default(mdp.gamma, **kw)


def certify(mdp, V, pi, st):
    ref = stored_ref(mdp)
    TV, pio, res = O.bellman(ref, V)
    assert st["converged"] == 1
    assert res <= TOL * (1 + 1e-6), res
    assert res / (1 - mdp.gamma) / np.max(np.abs(TV)) <= 1e-6
    Q = O.q_values(ref, V)
    Qs = np.sort(Q, axis=1)
    sel = (Qs[:, 1] - Qs[:, 0]) > 1e-9
    assert np.array_equal(pi[sel], pio[sel])


def test_serving_batch_invariance_and_certificate():
    I = igm()
    mdps = [request_mdp(s) for s in MIX]
    with I.Server(block_slices=BLOCK_SLICES) as srv:
        alone = []
        for mdp in mdps:
            t = srv.submit(mdp, params(mdp))
            alone.append(srv.result(t))
        # the same requests all at once, in another order and twice over
        order = list(range(len(mdps)))[::-1] + list(range(len(mdps)))
        tickets = [(i, srv.submit(mdps[i], params(mdps[i]))) for i in order]
        mixed = [(i, srv.result(t)) for i, t in tickets]
        info = srv.info()
    print(f"peak solves running at once: {info['peak_running']}, arena peak "
          f"{info['arena_peak'] / 2**20:.1f} MiB")
    assert info["failed"] == 0 and info["completed"] == len(mdps) + len(order)
    for mdp, (V, pi, st) in zip(mdps, alone):
        certify(mdp, V, pi, st)
    for i, (V, pi, st) in mixed:
        Va, pia, sta = alone[i]
        assert np.array_equal(V, Va), f"request {MIX[i]}: V differs between alone and mix"
        assert np.array_equal(pi, pia)
        assert (st["outer"], st["inner"], st["explicit_residuals"]) == \
            (sta["outer"], sta["inner"], sta["explicit_residuals"])
        assert st["latency_ms"] >= st["queue_ms"] >= 0.0


@pytest.mark.parametrize("spec,opts", [(MIX[0], {}), (MIX[2], {}),
                                       (MIX[3], {"forcing": 1, "polish": 1})])
def test_serving_matches_direct_persistent_solve(spec, opts):
    """Same kernel, same workgroup count: the served result equals the
    direct igmres_pi_solve (cooperative launch, engine 2) bit for bit, also
    with the forcing sequence and polish options."""
    I = igm()
    mdp = request_mdp(spec)
    blocks = math.ceil(math.ceil(mdp.n / 64) / BLOCK_SLICES)
    with I.Server(block_slices=BLOCK_SLICES) as srv:
        Vs, pis, sts = srv.result(srv.submit(mdp, params(mdp, **opts)))
    certify(mdp, Vs, pis, sts)
    with I.mdp_create(mdp, store="fp32") as h:
        V = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        st = h.igmres_pi_solve(V, pi, params(mdp, engine=2, blocks=blocks, **opts))
        Vd, pid = host(V), host(pi)
    assert np.array_equal(Vs, Vd)
    assert np.array_equal(pis, pid)
    assert (sts["outer"], sts["inner"]) == (st["outer"], st["inner"])


def test_serving_admission_by_footprint():
    """A 64 MiB arena holds about two of these requests at a time: the rest
    wait for retirements and still finish correctly; a request larger than
    the arena fails with IG_E_TOO_LARGE without disturbing the others."""
    I = igm()
    specs = [(20000, 8, 16, 0.95, 21 + i) for i in range(5)]
    mdps = [request_mdp(s) for s in specs]
    big = request_mdp((100000, 8, 16, 0.95, 30))
    budget = 64 << 20
    with I.Server(hbm_budget=budget, block_slices=BLOCK_SLICES) as srv:
        tickets = [srv.submit(m, params(m)) for m in mdps[:2]]
        tb = srv.submit(big, params(big))
        tickets += [srv.submit(m, params(m)) for m in mdps[2:]]
        outs = [srv.result(t) for t in tickets]
        with pytest.raises(I.IgError) as ei:
            srv.result(tb)
        assert ei.value.status == I.IG_E_TOO_LARGE
        info = srv.info()
    assert info["arena_peak"] <= budget
    assert info["failed"] == 1
    for mdp, (V, pi, st) in zip(mdps, outs):
        certify(mdp, V, pi, st)


def test_serving_errors_and_v0():
    I = igm()
    good = request_mdp(MIX[0])
    bad = good.with_values(val=good.val * 1.5)  # rows no longer sum to one
    with I.Server(max_states=50000) as srv:
        with pytest.raises(I.IgError) as ei:
            srv.submit(good, params(good, restart=65))
        assert ei.value.status == I.IG_E_TOO_LARGE
        with pytest.raises(I.IgError) as ei:
            srv.submit(request_mdp(MIX[5]), params(request_mdp(MIX[5])))
        assert ei.value.status == I.IG_E_TOO_LARGE
        tb = srv.submit(bad, params(bad))
        tn = srv.submit(good, params(good, max_outer=1))
        tg = srv.submit(good, params(good))
        with pytest.raises(I.IgError) as ei:
            srv.result(tb)
        assert ei.value.status == I.IG_E_INVALID
        Vn, _, stn = srv.result(tn, allow_noconv=True)
        assert stn["status"] == I.IG_E_NOCONV and stn["outer"] == 1
        assert stn["res_inf"] > TOL and np.all(np.isfinite(Vn))
        V, pi, st = srv.result(tg)
        certify(good, V, pi, st)
        # warm start at the solution: converged before any policy step
        V2, pi2, st2 = srv.result(srv.submit(good, params(good), V0=V))
        assert st2["outer"] == 0 and st2["converged"] == 1
        assert np.array_equal(V2, V) and np.array_equal(pi2, pi)


def test_serving_arena_beyond_device_memory():
    """An arena larger than the device's memory: srv_create reports
    IG_E_NOMEM (the failed allocation leaves no error behind), and a server
    with an ordinary arena serves a request afterwards."""
    I = igm()
    with pytest.raises(I.IgError) as ei:
        I.Server(hbm_budget=1 << 50)
    assert ei.value.status == I.IG_E_NOMEM
    good = request_mdp(MIX[0])
    with I.Server(max_states=50000) as srv:
        V, pi, st = srv.result(srv.submit(good, params(good)))
    certify(good, V, pi, st)


def test_serving_action_sets_match_direct_solve():
    """Requests with state-dependent action sets (excluded rows empty, their
    costs NaN) are served like any other: bitwise the direct persistent
    solve with the same workgroup count, and certified on the stored MDP."""
    I = igm()
    mdp = synth.with_action_sets(synth.sparse_uniform(9000, 6, 10, 0.95, 41), 0.5, 41)
    blocks = math.ceil(math.ceil(mdp.n / 64) / BLOCK_SLICES)
    with I.Server(block_slices=BLOCK_SLICES) as srv:
        Vs, pis, sts = srv.result(srv.submit(mdp, params(mdp)))
    with I.mdp_create(mdp, store="fp32") as h:
        V = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        h.igmres_pi_solve(V, pi, params(mdp, engine=2, blocks=blocks))
        Vd, pid = host(V), host(pi)
    assert np.array_equal(Vs, Vd) and np.array_equal(pis, pid)
    adm = mdp.adm.reshape(mdp.n, mdp.m)
    assert adm[np.arange(mdp.n), pis].all()
    ref = stored_ref(mdp)
    _, _, res = O.bellman(ref, Vs)
    assert sts["converged"] == 1 and res <= TOL * (1 + 1e-6)


def test_serving_wide_solve_runs_alone():
    """One CU per XCD stays outside the co-residency budget; a solve asking
    for more workgroups than the budget holds runs alone and is still exact
    (the same result as the direct solve with that workgroup count)."""
    import torch
    I = igm()
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    mdp = request_mdp((130000, 6, 12, 0.95, 16))
    wide = min(256, num_cu)
    small = [request_mdp(s) for s in MIX[:2]]
    with I.Server(block_slices=BLOCK_SLICES) as srv:
        cap = srv.info()["xcd_units_cap"]
        assert cap == max(1, num_cu // 8 - 1)
        tickets = [srv.submit(m, params(m)) for m in small]
        tw = srv.submit(mdp, params(mdp, blocks=wide))
        tickets += [srv.submit(m, params(m)) for m in small]
        outs = [srv.result(t) for t in tickets]
        Vw, piw, stw = srv.result(tw)
        assert srv.info()["failed"] == 0
    assert math.ceil(wide / 8) > cap
    with I.mdp_create(mdp, store="fp32") as h:
        V = zeros(mdp.n)
        pi = zeros(mdp.n, "int32")
        h.igmres_pi_solve(V, pi, params(mdp, engine=2, blocks=wide))
        assert np.array_equal(Vw, host(V)) and np.array_equal(piw, host(pi))
    for m, (V, pi, st) in zip(small + small, outs):
        certify(m, V, pi, st)


def test_serving_storage_and_modes_mix():
    """Requests with different storage types and arithmetic modes share one
    server; each equals the direct persistent solve of the same handle
    configuration bit for bit."""
    I = igm()
    mdp = request_mdp((6000, 5, 10, 0.95, 51))
    blocks = math.ceil(math.ceil(mdp.n / 64) / BLOCK_SLICES)
    combos = [("fp64", "fp64"), ("fp64", "mixed"), ("fp32", "mixed"), ("bf16", "mixed")]
    with I.Server(block_slices=BLOCK_SLICES) as srv:
        tickets = [srv.submit(mdp, params(mdp, mode=mode), store=store) for store, mode in combos]
        served = [srv.result(t) for t in tickets]
        assert srv.info()["failed"] == 0
    for (store, mode), (Vs, pis, sts) in zip(combos, served):
        with I.mdp_create(mdp, store=store) as h:
            V = zeros(mdp.n)
            pi = zeros(mdp.n, "int32")
            h.igmres_pi_solve(V, pi, params(mdp, mode=mode, engine=2, blocks=blocks))
            assert np.array_equal(Vs, host(V)), (store, mode)
            assert np.array_equal(pis, host(pi)), (store, mode)
        assert sts["converged"] == 1


def test_serving_barrier_wait_limit():
    """A request whose grid-barrier wait runs out (limit of zero polls,
    forced from the host) fails alone with IG_E_DEVICE; a one-workgroup
    request beside it needs no grid barrier and is served exactly, and the
    server keeps serving once the limit is back."""
    I = igm()
    wide, small = request_mdp(MIX[2]), request_mdp(MIX[4])
    with I.Server(max_states=50000) as srv:
        os.environ["IG_SPIN_LIMIT"] = "0"
        try:
            tw = srv.submit(wide, params(wide))
            ts = srv.submit(small, params(small))
            with pytest.raises(I.IgError) as ei:
                srv.result(tw)
            Vs, pis, sts = srv.result(ts)
        finally:
            del os.environ["IG_SPIN_LIMIT"]
        assert ei.value.status == I.IG_E_DEVICE
        certify(small, Vs, pis, sts)
        V, pi, st = srv.result(srv.submit(wide, params(wide)))
        certify(wide, V, pi, st)
