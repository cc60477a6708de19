"""FP64 CPU oracle for inexact GMRES policy iteration -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product path (the HIP library and its
Python binding) never imports, links or calls it, and it shares no code with
that path: the only thing both consume is the seeded input generator
(``paper_2211_04299_amd.synth``), which draws inputs and holds none of the
method's arithmetic.

Everything is float64, plain and unfused; library primitives (a sparse or
dense matrix-vector product, a dense LU solve, a least-squares solve) serve as
single steps.  Citations are to the paper (Gargiani, Liao-McPherson, Zanelli,
Lygeros, "Inexact GMRES Policy Iteration for Large-Scale Markov Decision
Processes", arXiv:2211.04299).

What each function follows, and what pins it (tests/test_oracle_pins.py):

  q_values, bellman        Bellman operators T^pi, T and GreedyPolicy (Sec. 2,
                           eqs. 3-4 and the greedy definition).  Pinned by a
                           hand-computed two-state example (tests/golden),
                           closed forms (self-loops, uniform transitions,
                           constant costs) and the contraction, monotonicity and
                           shift-invariance properties.
  policy_eval_lu           closed form V^pi = (I - gamma P^pi)^{-1} g^pi
                           (Sec. 2.1).  Pinned by the Neumann series, Lemma 3's
                           equality case and a hand-solved two-state chain.
  policy_iteration         PI (Sec. 2.1).  Pinned by brute force over all
                           policies (eq. 2) and agreement with value iteration.
  value_iteration          VI, eq. 6 with its gamma-contraction stopping bound.
  brute_force              V* = componentwise min over all deterministic
                           policies (eq. 2).
  gmres_inner              the inner solver of Algorithm 2 written from
                           the definition of the restarted GMRES(W) iterate
                           (minimum residual over x_c + K_i, eq. 13), not
                           from the printed pseudo-code: a Householder-QR
                           basis of K_i and a direct least-squares solve
                           over J times it.  Pinned by the minimum-residual
                           property against an explicitly formed power-basis
                           Krylov matrix, by LU at alpha -> 0, by the
                           <= 2 steps of uniform transitions and the exactly
                           n steps of the deterministic n-cycle (Lemma 1).
  igmres_pi                Algorithm 2's outer loop (greedy policy,
                           Phi_k, inexact evaluation).  Pinned by
                           agreement of the returned V with PI-LU's V*.
                           Option forcing: alpha_k = min(alpha,
                           ||T V_k - V_k||_inf^(1/2)), a forcing sequence that
                           tends to zero (Theorem 1's superlinear case).
                           Pinned by identity with the constant-alpha run while
                           alpha_k = alpha, by the inexactness condition of
                           eq. 11 at every outer step, by residual ratios that
                           tend to zero, and by PI-LU's V*.
                           Option polish: once the greedy policy repeats, one
                           evaluation to tol / 2.  Pinned by identity with the
                           plain run up to the first repeat, termination at the
                           next outer step whenever the policy holds, and
                           PI-LU's V*.
  neumann_apply            M^{-1} = sum_{k<=d} (gamma P^pi)^k, the truncated
                           series of Lemma 3's proof, as a right
                           preconditioner of the inner GMRES (future work
                           named in Sec. 5).  Pinned by the closed form
                           J M^{-1} = I - (gamma P^pi)^{d+1}, by the minimum-
                           residual property over x0 + M^{-1} K_i(J M^{-1}, r0)
                           and by degree 0 = plain GMRES.
  opi                      optimistic PI with a fixed number of VI sweeps
                           (Sec. 2.1).  Pinned by OPI(1) = VI, by a
                           hand-derived OPI(2) trajectory on the two-state
                           example (tests/golden) and by the W -> infinity
                           limit: the policy sequence and iteration count of
                           exact PI.
  certificate              ||V - V*||_inf <= ||TV - V||_inf / (1 - gamma),
                           from gamma-contraction (Sec. 2).
  action sets A(s)         every minimum runs over the admissible actions of
                           the state (Sec. 2, problem statement): q_values
                           gives +inf outside A(s), brute_force enumerates
                           A(0) x ... x A(n-1).  Pinned by brute force, by a
                           mask-free twin whose excluded actions carry a
                           prohibitive cost (same PI trajectory), by
                           monotonicity in the action sets and by the
                           one-action closed form.

Readings where the paper is silent or garbled (each is also listed in the
design notes of the repository):
  * ties in GreedyPolicy: lowest action index; PI's improvement keeps the
    incumbent action unless another is better by more than
    1e-12 * max(1, ||V||_inf);
  * outer termination of Algorithm 2: first k with ||T V_k - V_k||_inf <= tol
    (the algorithm itself runs a fixed K);
  * "||Phi||_2" in the least-squares step after a restart is the 2-norm of the
    residual that produced the current first basis vector, and the update
    "V_{k+1} <- Q y + V_k" adds to the iterate at the start of the current
    restart cycle;
  * the jump of Algorithm 2's lucky-breakdown branch ends the inner loop and
    proceeds to the next outer step;
  * Phi_k = 0 (or a zero restart residual) means the inner loop is not entered;
  * the least-squares problem uses the leading (i+1) x i block of H;
  * infinity-norm in every stopping test, 2-norm inside GMRES.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "q_values", "bellman", "greedy_keep", "policy_cost", "policy_matrix_dense",
    "policy_matrix_sparse", "j_apply", "policy_eval_lu", "policy_eval_neumann",
    "policy_iteration", "value_iteration", "brute_force", "gmres_inner",
    "igmres_pi", "opi", "certificate", "action_gaps", "OracleStats", "neumann_apply",
]


# ---------------------------------------------------------------------------
# operators (Section 2)
# ---------------------------------------------------------------------------

def _P_rows(mdp):
    """The (n*m) x n transition matrix, row r = s*m + a holds P(s, a, .)."""
    n, m = mdp.n, mdp.m
    if mdp.fmt == "dense":
        return mdp.P.reshape(n * m, n)
    return sp.csr_matrix((np.asarray(mdp.val, np.float64), mdp.col, mdp.row_ptr),
                         shape=(n * m, n))


def _adm(mdp):
    """Admissibility mask [n, m] of the action sets A(s) (Section 2), or None
    when every action is admissible."""
    adm = getattr(mdp, "adm", None)
    return None if adm is None else np.asarray(adm, bool).reshape(mdp.n, mdp.m)


def q_values(mdp, V):
    """Q[s, a] = g(s, a) + gamma * sum_s' p_ss'(a) V(s')   (the expression
    minimised in the Bellman equation for V*, eq. 4, and in GreedyPolicy);
    +inf for actions outside A(s), so that every minimum runs over A(s)."""
    V = np.asarray(V, dtype=np.float64)
    EV = _P_rows(mdp) @ V
    Q = (np.asarray(mdp.cost, np.float64) + mdp.gamma * EV).reshape(mdp.n, mdp.m)
    adm = _adm(mdp)
    return Q if adm is None else np.where(adm, Q, np.inf)


def bellman(mdp, V):
    """T V, a greedy policy w.r.t. V (lowest action index on exact ties) and
    the Bellman residual ||T V - V||_inf  (operators T and GreedyPolicy of
    Section 2; residual function r(V) = V - T V, eq. 8)."""
    Q = q_values(mdp, V)
    pi = np.argmin(Q, axis=1).astype(np.int32)  # first minimiser
    TV = Q[np.arange(mdp.n), pi]
    return TV, pi, float(np.max(np.abs(TV - V))) if mdp.n else 0.0


def action_gaps(mdp, V):
    """Per state: second-smallest minus smallest Q-value (inf if m == 1)."""
    Q = np.sort(q_values(mdp, V), axis=1)
    if mdp.m == 1:
        return np.full(mdp.n, np.inf)
    return Q[:, 1] - Q[:, 0]


def greedy_keep(mdp, V, pi_old, rel_tie=1e-12):
    """Policy improvement that keeps the incumbent action unless another action
    is better by more than rel_tie * max(1, ||V||_inf)."""
    Q = q_values(mdp, V)
    best = np.argmin(Q, axis=1)
    idx = np.arange(mdp.n)
    tie = rel_tie * max(1.0, float(np.max(np.abs(V))) if mdp.n else 1.0)
    keep = Q[idx, pi_old] <= Q[idx, best] + tie
    return np.where(keep, pi_old, best).astype(np.int32)


def policy_cost(mdp, pi):
    """g^pi(s) = g(s, pi(s))."""
    return np.asarray(mdp.cost, np.float64).reshape(mdp.n, mdp.m)[np.arange(mdp.n), pi]


def policy_matrix_sparse(mdp, pi):
    """[P^pi]_{s s'} = p_ss'(pi(s)) as a sparse matrix."""
    rows = np.arange(mdp.n) * mdp.m + np.asarray(pi)
    return _P_rows(mdp)[rows]


def policy_matrix_dense(mdp, pi):
    Ppi = policy_matrix_sparse(mdp, pi)
    return Ppi.toarray() if sp.issparse(Ppi) else np.asarray(Ppi)


def j_apply(mdp, pi, x, Ppi=None):
    """J x = (I - gamma P^pi) x   (Newton matrix, eq. 10)."""
    if Ppi is None:
        Ppi = policy_matrix_sparse(mdp, pi)
    return x - mdp.gamma * (Ppi @ x)


def neumann_apply(mdp, pi, x, degree, Ppi=None):
    """M^{-1} x = sum_{k=0}^{degree} (gamma P^pi)^k x, the truncated Neumann
    series of J^{-1} = (I - gamma P^pi)^{-1} (the series of Lemma 3's proof),
    by Horner's rule y <- x + gamma P^pi y.  degree 0 is the identity."""
    if Ppi is None:
        Ppi = policy_matrix_sparse(mdp, pi)
    x = np.asarray(x, np.float64)
    y = x.copy()
    for _ in range(degree):
        y = x + mdp.gamma * (Ppi @ y)
    return y


def policy_eval_lu(mdp, pi):
    """V^pi = (I - gamma P^pi)^{-1} g^pi by a dense LU solve (policy
    evaluation, Section 2.1)."""
    A = np.eye(mdp.n) - mdp.gamma * policy_matrix_dense(mdp, pi)
    return np.linalg.solve(A, policy_cost(mdp, pi))


def policy_eval_neumann(mdp, pi, rel=1e-15, max_terms=1_000_000):
    """V^pi = sum_k (gamma P^pi)^k g^pi (the series in the proof of Lemma 3),
    summed until the next term is below rel * ||partial sum||_inf."""
    Ppi = policy_matrix_sparse(mdp, pi)
    term = policy_cost(mdp, pi)
    V = term.copy()
    for _ in range(max_terms):
        term = mdp.gamma * (Ppi @ term)
        V += term
        if np.max(np.abs(term)) <= rel * max(np.max(np.abs(V)), 1e-300):
            break
    return V


# ---------------------------------------------------------------------------
# plain dynamic programming (Section 2.1, eq. 2)
# ---------------------------------------------------------------------------

def policy_iteration(mdp, V0=None, max_iter=1000, trace=None):
    """Exact PI: pi_0 = GreedyPolicy(V0), then alternate LU evaluation and
    improvement until the policy repeats.  Returns (V, pi, iterations);
    a list passed as `trace` receives the evaluated policies in order."""
    V = np.zeros(mdp.n) if V0 is None else np.asarray(V0, np.float64)
    _, pi, _ = bellman(mdp, V)
    for it in range(1, max_iter + 1):
        if trace is not None:
            trace.append(pi.copy())
        V = policy_eval_lu(mdp, pi)
        new = greedy_keep(mdp, V, pi)
        if np.array_equal(new, pi):
            return V, pi, it
        pi = new
    raise RuntimeError("policy iteration did not terminate")


def value_iteration(mdp, eps=None, V0=None, max_iter=10_000_000):
    """VI, V <- T V (eq. 6), until ||V_{j+1} - V_j||_inf <= eps (1-gamma)/gamma,
    which bounds ||V_{j+1} - V*||_inf by eps (gamma-contraction).  eps defaults
    to 1e-12 * ||V||_inf.  Returns (V, sweeps)."""
    V = np.zeros(mdp.n) if V0 is None else np.asarray(V0, np.float64).copy()
    g = mdp.gamma
    for j in range(1, max_iter + 1):
        TV, _, _ = bellman(mdp, V)
        d = float(np.max(np.abs(TV - V)))
        V = TV
        e = eps if eps is not None else 1e-12 * max(float(np.max(np.abs(V))), 1e-300)
        if d <= e * (1 - g) / g:
            return V, j
    raise RuntimeError("value iteration did not converge")


def brute_force(mdp, atol=1e-12):
    """V* = componentwise minimum of V^pi over all deterministic policies
    with pi(s) in A(s) (eq. 2).  Returns (V*, list of optimal policies).
    Only for tiny MDPs."""
    n, m = mdp.n, mdp.m
    adm = _adm(mdp)
    choices = [range(m) if adm is None else np.nonzero(adm[s])[0].tolist() for s in range(n)]
    if np.prod([len(c) for c in choices], dtype=float) > 200_000:
        raise ValueError("too many policies for brute force")
    vals = {}
    for pol in itertools.product(*choices):
        vals[pol] = policy_eval_lu(mdp, np.array(pol, dtype=np.int32))
    Vstar = np.min(np.stack(list(vals.values())), axis=0)
    opt = [np.array(p, dtype=np.int32) for p, v in vals.items()
           if np.all(v <= Vstar + atol * max(1.0, np.max(np.abs(Vstar))))]
    return Vstar, opt


def certificate(mdp, V):
    """Upper bound on ||V - V*||_inf from one Bellman pass:
    ||V - V*|| <= ||V - TV|| + ||TV - TV*|| <= ||V - TV|| + gamma ||V - V*||."""
    _, _, res = bellman(mdp, V)
    return res / (1.0 - mdp.gamma)


# ---------------------------------------------------------------------------
# Algorithm 2: GMRES(W) policy iteration
# ---------------------------------------------------------------------------

@dataclass
class OracleStats:
    outer: int = 0
    inner: int = 0
    restarts: int = 0
    breakdowns: int = 0
    inner_per_outer: list = field(default_factory=list)
    res_history: list = field(default_factory=list)
    alpha_history: list = field(default_factory=list)  # inner tolerance factor per outer step
    polished: list = field(default_factory=list)  # outer steps evaluated to tol / 2
    converged: bool = False


def gmres_inner(mdp, pi, x0, alpha, W, max_inner=10_000, ref_inf=None, trace=False, precond=0,
                res_trace=None):
    """Inexact policy evaluation by restarted GMRES(W): the inner solver of
    Algorithm 2 (Sec. 3.1) for J V = b with J = I - gamma P^pi, b = g^pi.

    Written from the definition of the GMRES iterate (Sec. 2.2, eq. 13), not
    from the printed pseudo-code: inside a restart cycle that starts at x_c
    with residual r_c = b - J x_c, the i-th iterate is

        x_i = x_c + M^{-1} z_i,  z_i = argmin_{z in K_i} ||r_c - J M^{-1} z||_2,
        K_i = span{r_c, A r_c, ..., A^{i-1} r_c},  A = J M^{-1},

    (M^{-1} = identity unless precond = d > 0 selects the degree-d Neumann
    polynomial of neumann_apply, a right preconditioner: the future work of
    Sec. 5).  A cycle ends after W iterates and the next one starts from the
    last iterate.  The loop returns the first iterate that meets the inexact
    rule of eq. 11 in the infinity-norm,
        || b - J x ||_inf <= alpha * ref_inf,
    where ref_inf defaults to ||b - J x0||_inf (= ||Phi_k||_inf).

    Steps (plain library primitives, no fusion):
      * an orthonormal basis of K_{i+1} is the basis of K_i plus the last
        column of the Q factor of a Householder QR (numpy.linalg.qr) of
        [basis of K_i, A q_i], q_i the newest basis vector
        (K_{i+1} = K_i + span{A q_i});
      * z_i solves the least-squares problem over the n x i matrix
        [A q_1, ..., A q_i] directly (numpy.linalg.lstsq);
      * the residual b - J x_i is formed explicitly at every step.
    When A q_i lies in K_i (the R factor's new diagonal entry is exactly
    zero) the space is invariant, x_i is the exact solution and the loop
    ends (the lucky breakdown; the paper then proceeds to the next outer
    step).  Two guards the paper leaves implicit end the loop early:
    max_inner iterates, and a restart cycle that lowers the residual 2-norm
    (the quantity GMRES minimises) by less than a factor 1 - 1e-6: restarted
    GMRES(W) with W < n can stagnate completely, and rounding puts a floor
    under the residual.
    Returns (x, info) with info = dict(steps, restarts, breakdown, iterates
    (first cycle, if trace), res_inf, thr, stagnated); a list passed as
    res_trace receives ||b - J x_i||_inf of every iterate.
    """
    Ppi = policy_matrix_sparse(mdp, pi)
    b = policy_cost(mdp, pi)
    J = lambda v: j_apply(mdp, pi, v, Ppi)  # noqa: E731
    Minv = lambda v: neumann_apply(mdp, pi, v, precond, Ppi)  # noqa: E731
    A = lambda v: J(Minv(v))  # noqa: E731

    x = np.asarray(x0, np.float64).copy()
    r = b - J(x)
    res_inf = float(np.max(np.abs(r))) if r.size else 0.0
    if ref_inf is None:
        ref_inf = res_inf
    thr = alpha * ref_inf
    steps = restarts = 0
    breakdown = stagnated = False
    iterates = []
    while res_inf > thr and steps < max_inner and not (breakdown or stagnated):
        # one restart cycle from x_c = x, r_c = r
        x_c, r_c = x.copy(), r.copy()
        beta = float(np.linalg.norm(r_c))
        basis = (r_c / beta)[:, None]      # orthonormal basis of K_1
        AK = np.zeros((mdp.n, 0))          # A applied to the basis vectors
        for _ in range(W):
            AK = np.column_stack([AK, A(basis[:, -1])])
            z, *_ = np.linalg.lstsq(AK, r_c, rcond=None)
            x = x_c + Minv(basis @ z)
            r = b - J(x)
            res_inf = float(np.max(np.abs(r)))
            steps += 1
            if res_trace is not None:
                res_trace.append(res_inf)
            if trace and restarts == 0:
                iterates.append(x.copy())
            if res_inf <= thr or steps >= max_inner:
                break
            Qf, Rf = np.linalg.qr(np.column_stack([basis, AK[:, -1]]))
            if Rf[-1, -1] == 0.0:          # K_{i+1} = K_i: x is exact
                breakdown = True
                break
            # the new direction, orthogonal to K_i; the earlier columns stay
            # as they are (AK holds A times exactly these vectors)
            basis = np.column_stack([basis, Qf[:, -1]])
        else:
            restarts += 1
            if res_inf > thr and float(np.linalg.norm(r)) > (1.0 - 1e-6) * beta:
                stagnated = True
    return x, dict(steps=steps, restarts=restarts, breakdown=breakdown, iterates=iterates,
                   res_inf=res_inf, thr=thr, stagnated=stagnated)


def igmres_pi(mdp, V0=None, alpha=None, W=30, tol=1e-8, max_outer=1000, max_inner=10_000,
              precond=0, forcing=False, polish=False, inner_trace=None):
    """Algorithm 2 with outer termination at ||T V_k - V_k||_inf <= tol.

    alpha defaults to the midpoint of Theorem 1's admissible range,
    0.5 * (1 - gamma) / (1 + gamma).  forcing: the inner tolerance of outer
    step k uses alpha_k = min(alpha, ||T V_k - V_k||_inf^(1/2)), a forcing
    sequence tending to zero (the superlinear case of Theorem 1) instead of
    the constant alpha.  polish: at an outer step k >= 1 whose greedy policy
    equals the previous one in every state, the inner threshold becomes
    min(alpha_k ||Phi_k||_inf, tol / 2): one evaluation of the (then
    usually optimal) policy to below the outer tolerance, after which the
    next Bellman residual meets it unless the greedy policy moves again.
    Both only shrink the inexactness term, so Theorem 1 still applies.
    Returns (V, pi, OracleStats); V and pi are V_k and GreedyPolicy(V_k) of
    the terminating outer step.  A list passed as inner_trace receives, per
    outer step, dict(thr=the inner threshold, res=[||g - J x_i||_inf of each
    inner iterate]).
    """
    g = mdp.gamma
    if alpha is None:
        alpha = 0.5 * (1 - g) / (1 + g)
    V = np.zeros(mdp.n) if V0 is None else np.asarray(V0, np.float64).copy()
    st = OracleStats()
    pi_prev = None
    for k in range(max_outer):
        TV, pi, res = bellman(mdp, V)
        st.res_history.append(res)
        if res <= tol:
            st.converged = True
            st.outer = k
            return V, pi, st
        Phi = policy_cost(mdp, pi) - j_apply(mdp, pi, V)
        phi_inf = float(np.max(np.abs(Phi)))
        alpha_k = min(alpha, float(np.sqrt(res))) if forcing else alpha
        if polish and pi_prev is not None and np.array_equal(pi, pi_prev):
            alpha_k = min(alpha_k, 0.5 * tol / phi_inf)
            st.polished.append(k)
        pi_prev = pi
        st.alpha_history.append(alpha_k)
        res_list = [] if inner_trace is not None else None
        V, info = gmres_inner(mdp, pi, V, alpha_k, W, max_inner, ref_inf=phi_inf,
                              precond=precond, res_trace=res_list)
        if inner_trace is not None:
            inner_trace.append(dict(thr=info["thr"], res=res_list))
        st.inner += info["steps"]
        st.restarts += info["restarts"]
        st.breakdowns += int(info["breakdown"])
        st.inner_per_outer.append(info["steps"])
    TV, pi, res = bellman(mdp, V)
    st.outer = max_outer
    st.converged = res <= tol
    return V, pi, st


def opi(mdp, sweeps, tol=1e-8, V0=None, max_outer=10_000_000, trace=None):
    """Optimistic PI: greedy policy from V_k, then `sweeps` applications of
    T^{pi_k} (the first of which equals T V_k); stop at ||T V - V||_inf <= tol.
    Returns (V, pi, outer, total_sweeps); a list passed as `trace` receives
    the greedy policy of every outer step."""
    V = np.zeros(mdp.n) if V0 is None else np.asarray(V0, np.float64).copy()
    total = 0
    for k in range(max_outer):
        TV, pi, res = bellman(mdp, V)
        if trace is not None:
            trace.append(pi.copy())
        if res <= tol:
            return V, pi, k, total
        Ppi = policy_matrix_sparse(mdp, pi)
        gpi = policy_cost(mdp, pi)
        V = TV
        total += 1
        for _ in range(sweeps - 1):
            V = gpi + mdp.gamma * (Ppi @ V)
            total += 1
    raise RuntimeError("OPI did not converge")
