"""Seeded synthetic MDP generators.

This module produces the *inputs* of the method: finite discounted-cost MDPs
{S, A, P, g, gamma} with row-stochastic transition rows and bounded stage
costs (problem setting, Section 2 of the paper).  It holds random draws and
array assembly only -- none of the method's arithmetic (no Bellman operator, no
linear algebra) -- so that the FP64 oracle and the HIP path can both be fed
from it without sharing any computational code.

The paper does not describe its benchmark MDP (Section 4 only gives n = 10000,
m = 40, gamma in {0.95, 0.99}); the shapes below are synthetic stand-ins.

Recipe (fixed, so every consumer sees bit-identical arrays):
  * NumPy PCG64 ``default_rng``.  States are generated in chunks of
    ``CHUNK`` states; chunk c draws from child c of ``SeedSequence(seed)``.
  * Within a chunk: successors first, then probabilities, then costs.
  * Successors of one (s, a) are distinct; duplicates are redrawn (with the
    same distribution) until none remain; each row is stored sorted by
    column.  A state may be its own successor.
  * Probabilities: Dirichlet(conc) drawn as normalised Gamma(conc, 1) draws,
    in float64.  Costs: U[0, 1).
  * Row r of the sparse layout is r = s * m + a (0-based), cost[s*m + a].
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

CHUNK = 1 << 16  # states per RNG chunk

__all__ = [
    "MDP", "sparse_uniform", "sparse_band", "dense_exp", "config", "CONFIGS",
    "round_values", "upcast_values", "serving_stream", "ServingRequest",
    "from_rows", "self_loops", "uniform_transitions", "cyclic", "random_micro",
    "with_action_sets",
]


@dataclass
class MDP:
    """Container for one finite MDP (0-based indices).

    fmt == "csr":   row_ptr int64[n*m+1], col int32[nnz], val float64[nnz]
    fmt == "dense": P float64[n, m, n]   (P[s, a, s'])
    cost float64[n*m] with cost[s*m + a] = g(s, a).
    adm (optional) bool[n*m]: adm[s*m + a] says whether action a is
    admissible in state s (the action set A(s)); None = every action.  Rows
    and costs of inadmissible pairs carry no meaning (CSR rows may be empty).
    """
    n: int
    m: int
    gamma: float
    cost: np.ndarray
    fmt: str = "csr"
    row_ptr: Optional[np.ndarray] = None
    col: Optional[np.ndarray] = None
    val: Optional[np.ndarray] = None
    P: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)
    adm: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        if self.fmt == "csr":
            return int(self.row_ptr[-1])
        return self.n * self.m * self.n

    def with_values(self, val=None, P=None) -> "MDP":
        """Same MDP structure with replaced probability values."""
        return MDP(self.n, self.m, self.gamma, self.cost, self.fmt, self.row_ptr,
                   self.col, val if val is not None else self.val,
                   P if P is not None else self.P, self.name, dict(self.meta), self.adm)


# ---------------------------------------------------------------------------
# storage rounding (input preparation: FP64 master values -> stored values)
# ---------------------------------------------------------------------------

def round_values(x: np.ndarray, storage: str) -> np.ndarray:
    """Round float64 probabilities to the storage type.

    "fp64": unchanged.  "fp32": IEEE round-to-nearest-even.  "bf16": first to
    fp32 (RNE), then to the upper 16 bits of the fp32 pattern with RNE;
    returned as the raw uint16 bit patterns.
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    if storage == "fp64":
        return x
    f = x.astype(np.float32)
    if storage == "fp32":
        return f
    if storage == "bf16":
        u = f.view(np.uint32).astype(np.uint64)
        lsb = (u >> np.uint64(16)) & np.uint64(1)
        u = u + np.uint64(0x7FFF) + lsb
        return (u >> np.uint64(16)).astype(np.uint16)
    raise ValueError(storage)


def upcast_values(x: np.ndarray, storage: str) -> np.ndarray:
    """Exact float64 value of stored probabilities."""
    if storage == "fp64":
        return np.asarray(x, dtype=np.float64)
    if storage == "fp32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    if storage == "bf16":
        u = np.asarray(x, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
        return u.view(np.float32).astype(np.float64)
    raise ValueError(storage)


# ---------------------------------------------------------------------------
# chunked drawing helpers
# ---------------------------------------------------------------------------

def _chunks(n: int):
    return [(c, c * CHUNK, min(n, (c + 1) * CHUNK)) for c in range(math.ceil(n / CHUNK))]


def _run_chunks(n, seed, fn, threads=None):
    children = np.random.SeedSequence(seed).spawn(max(1, math.ceil(n / CHUNK)))
    chunks = _chunks(n)
    if threads is None:
        threads = min(8, len(chunks))
    if threads <= 1 or len(chunks) == 1:
        return [fn(np.random.default_rng(children[c]), lo, hi) for c, lo, hi in chunks]
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda t: fn(np.random.default_rng(children[t[0]]), t[1], t[2]), chunks))


def _distinct_rows(rng, draw, rows: int, k: int):
    """rows x k successor table with distinct entries per row, rows sorted.

    draw(rng, row_index_array) -> one candidate per listed row.
    """
    idx = np.repeat(np.arange(rows), k)
    d = draw(rng, idx).reshape(rows, k)
    d.sort(axis=1)
    while True:
        dup = np.zeros_like(d, dtype=bool)
        dup[:, 1:] = d[:, 1:] == d[:, :-1]
        if not dup.any():
            return d
        r, c = np.nonzero(dup)
        d[r, c] = draw(rng, r)
        d.sort(axis=1)


def _dirichlet(rng, rows: int, k: int, conc: float) -> np.ndarray:
    g = rng.standard_gamma(conc, size=(rows, k))
    s = g.sum(axis=1, keepdims=True)
    bad = ~(s[:, 0] > 0)
    while bad.any():  # all-zero row (only possible for tiny conc): redraw it
        g[bad] = rng.standard_gamma(conc, size=(int(bad.sum()), k))
        s = g.sum(axis=1, keepdims=True)
        bad = ~(s[:, 0] > 0)
    return g / s


def _assemble_csr(n, m, k, gamma, parts, name, meta):
    col = np.concatenate([p[0].reshape(-1) for p in parts]).astype(np.int32)
    val = np.concatenate([p[1].reshape(-1) for p in parts])
    cost = np.concatenate([p[2].reshape(-1) for p in parts])
    row_ptr = np.arange(0, n * m * k + 1, k, dtype=np.int64)
    return MDP(n, m, float(gamma), cost, "csr", row_ptr, col, val, None, name, meta)


# ---------------------------------------------------------------------------
# generators
# ---------------------------------------------------------------------------

def sparse_uniform(n: int, m: int, k: int, gamma: float, seed: int,
                   conc: float = 1.0, threads=None, name="") -> MDP:
    """k distinct successors per (s, a), uniform on the state space."""
    if not (1 <= k <= n):
        raise ValueError("need 1 <= k <= n")

    def fn(rng, lo, hi):
        R = (hi - lo) * m
        succ = _distinct_rows(rng, lambda g, r: g.integers(0, n, size=r.shape[0]), R, k)
        prob = _dirichlet(rng, R, k, conc)
        cost = rng.random(size=(hi - lo) * m)
        return succ, prob, cost

    parts = _run_chunks(n, seed, fn, threads)
    return _assemble_csr(n, m, k, gamma, parts, name or f"uniform-n{n}-m{m}-k{k}",
                         dict(kind="uniform", k=k, conc=conc, seed=seed))


def sparse_band(n: int, m: int, k: int, gamma: float, seed: int, band: int = 64,
                p_band: float = 0.9, conc: float = 0.5, threads=None, name="") -> MDP:
    """k distinct successors; each draw is, with prob. p_band, uniform on the
    clipped window [max(0, s-band), min(n-1, s+band)], otherwise uniform on
    [0, n)."""
    if not (1 <= k <= min(n, 2 * band + 1)):
        raise ValueError("k too large for the band")

    def fn(rng, lo, hi):
        R = (hi - lo) * m
        state_of_row = lo + np.arange(R) // m

        def draw(g, r):
            s = state_of_row[r]
            a = np.maximum(0, s - band)
            b = np.minimum(n - 1, s + band)
            u = g.random(size=r.shape[0])
            local = a + (g.random(size=r.shape[0]) * (b - a + 1)).astype(np.int64)
            local = np.minimum(local, b)
            glob = g.integers(0, n, size=r.shape[0])
            return np.where(u < p_band, local, glob)

        succ = _distinct_rows(rng, draw, R, k)
        prob = _dirichlet(rng, R, k, conc)
        cost = rng.random(size=(hi - lo) * m)
        return succ, prob, cost

    parts = _run_chunks(n, seed, fn, threads)
    return _assemble_csr(n, m, k, gamma, parts, name or f"band-n{n}-m{m}-k{k}",
                         dict(kind="band", k=k, band=band, p_band=p_band, conc=conc, seed=seed))


def dense_exp(n: int, m: int, gamma: float, seed: int, threads=None, name="") -> MDP:
    """Dense P[s, a, :] with Exp(1) entries, normalised per row in float64."""
    def fn(rng, lo, hi):
        P = rng.exponential(size=(hi - lo, m, n))
        P /= P.sum(axis=2, keepdims=True)
        cost = rng.random(size=(hi - lo) * m)
        return P, cost

    parts = _run_chunks(n, seed, fn, threads)
    P = np.concatenate([p[0] for p in parts], axis=0)
    cost = np.concatenate([p[1] for p in parts])
    return MDP(n, m, float(gamma), cost, "dense", None, None, None, P,
               name or f"dense-n{n}-m{m}", dict(kind="dense", seed=seed))


def from_rows(n: int, m: int, gamma: float, rows, cost) -> MDP:
    """Build a CSR MDP from a list of n*m rows, each a list of (s', p)."""
    row_ptr = np.zeros(n * m + 1, dtype=np.int64)
    cols, vals = [], []
    for r, row in enumerate(rows):
        row = sorted(row)
        row_ptr[r + 1] = row_ptr[r] + len(row)
        cols += [c for c, _ in row]
        vals += [p for _, p in row]
    return MDP(n, m, float(gamma), np.asarray(cost, dtype=np.float64).reshape(-1), "csr",
               row_ptr, np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float64))


# special structures (test fixtures with known answers) ----------------------

def self_loops(n: int, m: int, gamma: float, seed: int) -> MDP:
    """Every action keeps the state: P(s, a, s) = 1."""
    rng = np.random.default_rng(seed)
    cost = rng.random(size=n * m)
    rows = [[(s, 1.0)] for s in range(n) for _ in range(m)]
    return from_rows(n, m, gamma, rows, cost)


def uniform_transitions(n: int, m: int, gamma: float, seed: int) -> MDP:
    """Every (s, a) moves to a uniformly random state: P(s, a, s') = 1/n."""
    rng = np.random.default_rng(seed)
    cost = rng.random(size=n * m)
    col = np.tile(np.arange(n, dtype=np.int32), n * m)
    val = np.full(n * n * m, 1.0 / n)
    row_ptr = np.arange(0, n * m * n + 1, n, dtype=np.int64)
    return MDP(n, m, float(gamma), cost, "csr", row_ptr, col, val, name="uniform-trans")


def cyclic(n: int, m: int, gamma: float, seed: int) -> MDP:
    """Action a moves s -> (s + a + 1) mod n deterministically."""
    rng = np.random.default_rng(seed)
    cost = rng.random(size=n * m)
    rows = [[((s + a + 1) % n, 1.0)] for s in range(n) for a in range(m)]
    return from_rows(n, m, gamma, rows, cost)


def random_micro(n: int, m: int, gamma: float, seed: int, k: Optional[int] = None) -> MDP:
    """Tiny MDP with random rows of (possibly different) lengths in [1, n]."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n * m):
        kk = k if k is not None else int(rng.integers(1, n + 1))
        succ = rng.choice(n, size=kk, replace=False)
        p = rng.random(size=kk) + 0.05
        p /= p.sum()
        rows.append(list(zip(succ.tolist(), p.tolist())))
    cost = rng.random(size=n * m)
    return from_rows(n, m, gamma, rows, cost)


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    # tiny sparse, FP64: n=100, m=4, k=5, gamma=0.9, restart 20
    "c1": dict(kind="uniform", n=100, m=4, k=5, gamma=0.9, restart=20, conc=1.0),
    # paper-scale sparse, FP64: n=1e4, m=8, k=20, gamma=0.99, restart 30
    "c2": dict(kind="uniform", n=10_000, m=8, k=20, gamma=0.99, restart=30, conc=1.0),
    # dense, mixed precision: n=1e4, m=4, gamma=0.99 (restart 30)
    "c3": dict(kind="dense", n=10_000, m=4, gamma=0.99, restart=30),
    # large banded sparse, mixed precision: n=4e6, m=8, k=16, gamma=0.995, restart 40
    "c4": dict(kind="band", n=4_000_000, m=8, k=16, gamma=0.995, restart=40, conc=0.5),
}


def config(name: str, seed: int = 0, n: Optional[int] = None, gamma: Optional[float] = None,
           m: Optional[int] = None, threads=None) -> MDP:
    """Generate a named workload (optionally with a different n, m or gamma,
    keeping the rest of the recipe)."""
    c = dict(CONFIGS[name])
    if n is not None:
        c["n"] = n
    if m is not None:
        c["m"] = m
    if gamma is not None:
        c["gamma"] = gamma
    if c["kind"] == "uniform":
        mdp = sparse_uniform(c["n"], c["m"], c["k"], c["gamma"], seed, c["conc"], threads)
    elif c["kind"] == "band":
        mdp = sparse_band(c["n"], c["m"], c["k"], c["gamma"], seed, conc=c["conc"], threads=threads)
    else:
        mdp = dense_exp(c["n"], c["m"], c["gamma"], seed, threads)
    mdp.name = f"{name}-seed{seed}"
    mdp.meta["restart"] = c["restart"]
    return mdp


def with_action_sets(mdp: MDP, keep: float, seed: int, empty_rows: bool = True,
                     nan_costs: bool = True) -> MDP:
    """State-dependent action sets: each (s, a) is admissible with
    probability `keep` (at least one action per state, drawn uniformly when
    none survives).  With empty_rows (CSR) the rows of inadmissible pairs are
    dropped from the CSR arrays; with nan_costs their costs become NaN --
    both must be ignored by every consumer."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xAC7]))
    n, m = mdp.n, mdp.m
    adm = rng.random((n, m)) < keep
    none = ~adm.any(axis=1)
    adm[np.nonzero(none)[0], rng.integers(0, m, size=int(none.sum()))] = True
    adm = adm.reshape(-1)
    cost = np.asarray(mdp.cost, np.float64).copy()
    if nan_costs:
        cost[~adm] = np.nan
    out = MDP(n, m, mdp.gamma, cost, mdp.fmt, mdp.row_ptr, mdp.col, mdp.val, mdp.P,
              (mdp.name or "mdp") + f"-A{keep:g}", dict(mdp.meta), adm)
    if mdp.fmt == "csr" and empty_rows:
        lens = np.diff(mdp.row_ptr)
        keep_e = np.repeat(adm, lens)
        out.col = np.ascontiguousarray(mdp.col[keep_e])
        out.val = np.ascontiguousarray(np.asarray(mdp.val)[keep_e])
        out.row_ptr = np.concatenate([[0], np.cumsum(np.where(adm, lens, 0))]).astype(np.int64)
    out.meta["action_keep"] = keep
    return out


@dataclass
class ServingRequest:
    index: int
    arrival: float  # seconds after stream start
    n: int
    m: int
    k: int
    gamma: float
    seed: int

    def footprint_nnz(self) -> int:
        return self.n * self.m * self.k

    def make(self, threads=None) -> MDP:
        mdp = sparse_uniform(self.n, self.m, self.k, self.gamma, self.seed, 1.0, threads)
        mdp.name = f"req{self.index}"
        return mdp


def serving_stream(count: int, rate: float, seed: int = 0, n_lo: int = 1_000,
                   n_hi: int = 200_000) -> list:
    """Poisson(rate) arrivals; n log-uniform in [n_lo, n_hi]; m uniform in
    {2..16}; k uniform in {4..32}; gamma uniform in {0.9, 0.95, 0.99};
    request i's MDP uses seed (seed + 1 + i)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5E7]))
    gaps = rng.exponential(1.0 / rate, size=count) if rate > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0]
    ln = rng.uniform(math.log(n_lo), math.log(n_hi), size=count)
    ns = np.clip(np.round(np.exp(ln)).astype(np.int64), n_lo, n_hi)
    ms = rng.integers(2, 17, size=count)
    ks = rng.integers(4, 33, size=count)
    gs = np.array([0.9, 0.95, 0.99])[rng.integers(0, 3, size=count)]
    return [ServingRequest(i, float(t[i]), int(ns[i]), int(ms[i]), int(min(ks[i], ns[i])),
                           float(gs[i]), seed + 1 + i) for i in range(count)]
