"""igmres_pi_solve_noalloc (workspace in the library's static device array)
against igmres_pi_solve on the persistent engine: the same kernel with the
same workgroup count, so V, pi and every count must agree bit for bit.  Two
calls in a row, the second on a smaller MDP (the array keeps the first call's
contents), then a third at the first size again; requests the array cannot
hold, or the persistent engine cannot run, are refused."""
import numpy as np
import pytest

from oracle import mdp_oracle as O
from paper_2211_04299_amd import synth

from gpu_helpers import host, rel_err, tol_par, zeros

pytestmark = pytest.mark.gpu


def igm():
    from paper_2211_04299_amd import igmres
    return igmres


def both(mdp, store="fp64", **kw):
    """(noalloc result, igmres_pi_solve engine 2 result) on one handle."""
    I = igm()
    with I.mdp_create(mdp, store=store) as h:
        p = I.params_default(mdp.gamma, **kw)
        V1, pi1 = zeros(mdp.n), zeros(mdp.n, "int32")
        st1 = h.igmres_pi_solve_noalloc(V1, pi1, p)
        a = (host(V1), host(pi1), st1)
        p.engine = 2
        V2, pi2 = zeros(mdp.n), zeros(mdp.n, "int32")
        st2 = h.igmres_pi_solve(V2, pi2, p)
        b = (host(V2), host(pi2), st2)
    return a, b


def same(a, b):
    assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64)), "V differs"
    assert np.array_equal(a[1], b[1]), "pi differs"
    for k in ("outer", "inner", "restarts", "bellman_passes", "explicit_residuals", "converged"):
        assert a[2][k] == b[2][k], k
    assert a[2]["res_inf"] == b[2]["res_inf"]


def test_noalloc_matches_persistent_solve_then_smaller_input():
    big = synth.config("c2", 0)       # n = 1e4: 40 workgroups
    small = synth.config("c1", 0)     # n = 100: one workgroup
    a, b = both(big, tol=1e-8, restart=30)
    same(a, b)
    assert a[2]["converged"] == 1
    a, b = both(small, tol=1e-8, restart=20)
    same(a, b)
    Vs, pis, _ = O.policy_iteration(small)
    assert rel_err(a[0], Vs) <= 1e-7
    a, b = both(big, tol=1e-8, restart=30)  # back to the larger size
    same(a, b)


def test_noalloc_mixed_precision():
    mdp = synth.config("c2", 1, n=4000)
    a, b = both(mdp, store="fp32", mode="mixed", tol=1e-8, restart=30)
    same(a, b)
    assert a[2]["converged"] == 1


def test_noalloc_refusals():
    I = igm()
    mdp = synth.config("c1", 0)
    with I.mdp_create(mdp) as h:
        V, pi = zeros(mdp.n), zeros(mdp.n, "int32")
        for kw in (dict(engine=1), dict(precond=2)):
            with pytest.raises(I.IgError) as e:
                h.igmres_pi_solve_noalloc(V, pi, I.params_default(mdp.gamma, **kw))
            assert e.value.status == I.IG_E_INVALID
    # (restart + 3) * n * 8 bytes above the array: refused before any work
    n = 1 << 17
    big = synth.sparse_uniform(n, 2, 4, 0.95, seed=3)
    assert (30 + 3) * n * 8 > I.IG_NOALLOC_SCRATCH_BYTES
    with I.mdp_create(big) as h:
        V, pi = zeros(n), zeros(n, "int32")
        with pytest.raises(I.IgError) as e:
            h.igmres_pi_solve_noalloc(V, pi, I.params_default(big.gamma, restart=30))
        assert e.value.status == I.IG_E_TOO_LARGE
        # the same handle still solves through the allocating entry point
        st = h.igmres_pi_solve(V, pi, I.params_default(big.gamma, restart=30, tol=1e-8))
        assert st["converged"] == 1
