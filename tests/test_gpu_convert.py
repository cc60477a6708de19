"""CSR -> sliced-ELL conversion on the device against the conversion on the
host.  Both routes must store the same image, checked through what reads it
(the Bellman operator over every action, and a full solve, whose P^pi
gathers read the policy's rows), bit for bit; device-resident inputs go
through the device route; and invalid inputs fail on both routes with the
same status and message."""
import contextlib
import os

import numpy as np
import pytest

from paper_2211_04299_amd import synth

from gpu_helpers import dev_vec, host, zeros

pytestmark = pytest.mark.gpu


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


@contextlib.contextmanager
def route(name):
    old = os.environ.get("IG_CONVERT")
    os.environ["IG_CONVERT"] = name
    try:
        yield
    finally:
        if old is None:
            del os.environ["IG_CONVERT"]
        else:
            os.environ["IG_CONVERT"] = old


_cache = {}


def case(name):
    if name not in _cache:
        if name == "uniform":  # 3000 states: 46 full slices and a ragged one
            mdp = synth.sparse_uniform(3000, 5, 9, 0.95, 3)
        elif name == "band":
            mdp = synth.config("c4", 2, n=5000)
        elif name == "ragged":  # row lengths from 1 to n
            mdp = synth.random_micro(150, 3, 0.9, 7)
        elif name == "sets":  # action sets with empty excluded rows
            mdp = synth.with_action_sets(synth.sparse_uniform(2000, 6, 7, 0.95, 5), 0.4, 5)
        _cache[name] = mdp
    return _cache[name]


def outputs(mdp, store, val_type, **create_kw):
    """Bellman apply at a fixed V and a full solve, on a fresh handle."""
    I = igm()
    src = mdp.with_values(val=synth.round_values(mdp.val, val_type))
    V0 = np.random.default_rng(2).random(mdp.n) * 10.0
    mode = "fp64" if store == "fp64" else "mixed"
    with I.mdp_create(src, store=store, **create_kw) as h:
        V = dev_vec(V0)
        TV, pi, res = zeros(mdp.n), zeros(mdp.n, "int32"), zeros(1)
        h.bellman_apply(V, TV, pi, res)
        Vs, pis = zeros(mdp.n), zeros(mdp.n, "int32")
        st = h.igmres_pi_solve(Vs, pis, I.params_default(mdp.gamma, tol=1e-8, mode=mode,
                                                         engine=1))
        return host(TV), host(pi), host(res), host(Vs), host(pis), st["outer"], st["inner"]


def assert_same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("store,val_type", [("fp64", "fp64"), ("fp32", "fp64"), ("fp32", "fp32"),
                                            ("bf16", "fp64"), ("bf16", "bf16")])
@pytest.mark.parametrize("name", ["uniform", "band", "ragged", "sets"])
def test_device_route_matches_host_route(name, store, val_type):
    mdp = case(name)
    with route("host"):
        a = outputs(mdp, store, val_type)
    with route("device"):
        b = outputs(mdp, store, val_type)
    assert_same(a, b)


@pytest.mark.parametrize("name,val_type", [("uniform", "fp64"), ("sets", "fp64"),
                                           ("uniform", "fp32"), ("sets", "bf16")])
def test_device_inputs(name, val_type):
    """Arrays already on the device take the device route by default; the
    result equals the host route's on the same (rounded) values."""
    import torch
    mdp = case(name)
    store = "fp64" if val_type == "fp64" else val_type
    with route("host"):
        a = outputs(mdp, store, val_type)
    vals = synth.round_values(mdp.val, val_type)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).cuda()
    if val_type == "bf16":
        dval = torch.from_numpy(vals.view(np.int16).copy()).cuda()
    else:
        dval = t(vals, vals.dtype)
    dmdp = synth.MDP(mdp.n, mdp.m, mdp.gamma, t(mdp.cost, np.float64), "csr",
                     t(mdp.row_ptr, np.int64), t(mdp.col, np.int32), dval,
                     None, mdp.name, dict(mdp.meta),
                     None if mdp.adm is None else t(mdp.adm, np.uint8))
    os.environ.pop("IG_CONVERT", None)
    b = outputs_dev(dmdp, store)
    assert_same(a, b)


def outputs_dev(dmdp, store):
    I = igm()
    V0 = np.random.default_rng(2).random(dmdp.n) * 10.0
    mode = "fp64" if store == "fp64" else "mixed"
    with I.mdp_create(dmdp, store=store, inputs_on_device=True) as h:
        V = dev_vec(V0)
        TV, pi, res = zeros(dmdp.n), zeros(dmdp.n, "int32"), zeros(1)
        h.bellman_apply(V, TV, pi, res)
        Vs, pis = zeros(dmdp.n), zeros(dmdp.n, "int32")
        st = h.igmres_pi_solve(Vs, pis, I.params_default(dmdp.gamma, tol=1e-8, mode=mode,
                                                         engine=1))
        return host(TV), host(pi), host(res), host(Vs), host(pis), st["outer"], st["inner"]


def broken(kind):
    """A copy of the uniform case with one planted defect."""
    mdp = case("uniform")
    col, val, rp = mdp.col.copy(), mdp.val.copy(), mdp.row_ptr
    gamma = mdp.gamma
    r = 1234  # a row in the middle of a slice
    lo = int(rp[r])
    if kind == "col":
        col[lo + 2] = mdp.n
    elif kind == "dup":
        col[lo + 1] = col[lo]
    elif kind == "range":  # sum kept, one entry negative
        val[lo] += val[lo + 1] + 0.25
        val[lo + 1] = -0.25
    elif kind == "sum":
        val[lo:int(rp[r + 1])] *= 1.5
    elif kind == "contraction":  # within the FP32 row-sum tolerance, but gamma*sum >= 1
        val = val.astype(np.float32)
        val[lo:int(rp[r + 1])] *= np.float32(1.01)
        gamma = 0.995
    return synth.MDP(mdp.n, mdp.m, gamma, mdp.cost, "csr", rp, col, val, None, "broken",
                     dict(mdp.meta))


@pytest.mark.parametrize("kind", ["col", "dup", "range", "sum", "contraction"])
def test_device_route_validation(kind):
    I = igm()
    mdp = broken(kind)
    msgs = []
    for r in ("host", "device"):
        with route(r):
            with pytest.raises(I.IgError) as ei:
                I.mdp_create(mdp, store="fp32")
        assert ei.value.status == I.IG_E_INVALID
        msgs.append(I.last_error())
    assert msgs[0] == msgs[1], msgs
    # without validation the columns are still range-checked
    for r in ("host", "device"):
        with route(r):
            if kind == "col":
                with pytest.raises(I.IgError):
                    I.mdp_create(mdp, store="fp32", validate=False)
            else:
                I.mdp_create(mdp, store="fp32", validate=False).close()
