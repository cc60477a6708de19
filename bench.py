"""Benchmark: inexact GMRES policy iteration (Algorithm 2) solved to
||T V - V||_inf <= 1e-8 from V0 = 0 on the largest single-GPU workload (c4:
n = 4e6 states, m = 8 actions, k = 16 successors per (s, a), 90% in the band
|s' - s| <= 64 and 10% uniform, Dirichlet(0.5) probabilities, c ~ U[0,1],
gamma = 0.995, GMRES restart 40; P stored in FP32 with int32 columns, FP32
Krylov basis and products, FP64 Bellman residual, solution update and
Hessenberg/Givens solve).  One step = one full solve with the MDP already
resident in HBM.  --workload picks another (c2: the paper-scale n = 1e4,
m = 8, k = 20 FP64 workload; c1; c3 dense; c3-bf16; c3-bf16r with the FP32
refinement copy).

Prints one JSON line.  Extra keys: "roofline" for the dominant kernel (HIP
events on its launch stream around about four of its launches per solve
during the timed steps, the first and then one in every "sampled_every", so
that the events' own cost stays out of the timed throughput; algorithmic
bytes per launch from the kernel's definition), "cpu_baseline" (the FP64 oracle's
literal Algorithm 2 on the host, a bounded sample of solves) and "serving"
(continuous batching of the serving stream, 2000 requests: uneven sparse
requests, n log-uniform in [1e3, 2e5], m in 2..16, k in 4..32, gamma in
{0.9, 0.95, 0.99}, FP32-stored P, mixed precision, W = 30, tol 1e-8;
saturated throughput with every request queued at once, then p50/p99
latency under Poisson arrivals at 0.5, 0.8 and 1.0x that throughput, beside
the same requests solved one at a time by the plain FP64 path).

The roofline also names its regime ("regime": HBM streaming, or latency-bound
when the stored MDP fits the 256 MB last-level cache and repeated passes
are served from it) and carries the rate of a plain 1 GiB device copy measured
in the same run ("copy_GBps", read + write bytes per second), context for
the published peak.

Also reported: per-solve device time p50/p90, the upload (mdp_create)
time, and under "compare" the same workload by exact-evaluation PI and by
OPI with 20 sweeps (FP64 workloads) or with FP64 storage and arithmetic
(mixed workloads), each timed from V0 = 0 to the same tolerance.  Under
"extra" the other single-GPU workloads are timed in the same run (c2 with
its PI and OPI comparisons; c3 with FP32, BF16 and BF16 + FP32 refinement
storage against FP64), under "preconditioned" (c4) the same solve with the
truncated-Neumann right preconditioner of degree 1 and 3 in the inner GMRES
(the paper's future work, not the headline method), and "cpu_baseline" carries the oracle's times on one
host core and on all of them, with the host's CPU model and core count, plus
the oracle's PI with LU evaluation, value iteration and Algorithm 2 on c2.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c4|c3|c3-bf16|c5]
                    [--serve-requests R] [--no-serving] [--no-compare]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "iGMRES-PI time-to-1e-8 Bellman residual, HBM GB/s; p50/p99 batched latency"
HBM_PEAK_GBPS = 8000.0
KSRC = os.path.join(ROOT, "paper_2211_04299_amd", "csrc")

WORKLOADS = {
    "c2": dict(cfg="c2", store="fp64", mode="fp64",
               desc="sparse n=10000 m=8 k=20 gamma=0.99 W=30 FP64 (CSR int32 cols), tol 1e-8, V0=0"),
    "c1": dict(cfg="c1", store="fp64", mode="fp64",
               desc="sparse n=100 m=4 k=5 gamma=0.9 W=20 FP64, tol 1e-8, V0=0"),
    "c3": dict(cfg="c3", store="fp32", mode="mixed",
               desc="dense n=10000 m=4 gamma=0.99 W=30 FP32-stored P, mixed, tol 1e-8, V0=0"),
    "c3-bf16": dict(cfg="c3", store="bf16", mode="mixed",
                    desc="dense n=10000 m=4 gamma=0.99 W=30 BF16-stored P, mixed, tol 1e-8, V0=0"),
    "c3-bf16r": dict(cfg="c3", store="bf16", mode="mixed", refine=True,
                     desc="dense n=10000 m=4 gamma=0.99 W=30 BF16 P inside GMRES, FP32 copy for "
                          "Bellman passes and residuals, mixed, tol 1e-8, V0=0"),
    "c4": dict(cfg="c4", store="fp32", mode="mixed",
               desc="banded sparse n=4e6 m=8 k=16 (90% within +-64, 10% uniform) Dirichlet(0.5) "
                    "gamma=0.995 W=40; P in FP32 (int32 cols), FP32 basis and P^pi products, "
                    "FP64 Bellman residual, update and Givens; tol 1e-8, V0=0"),
}


# sources that define the kernels of a dominant class (plus the shared
# device helpers): stored counter figures stay valid while these are unchanged
KERNEL_FILES = {
    "persistent": ["kernels_persist.hip", "common.hpp"],
    "sparse": ["kernels_sparse.hip", "common.hpp"],
    "dense": ["kernels_dense.hip", "common.hpp"],
}


def kernel_source_hash(group):
    h = hashlib.sha256()
    for f in KERNEL_FILES[group]:
        with open(os.path.join(KSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def kernel_group(dom, fmt):
    return "persistent" if dom == "persistent" else ("sparse" if fmt == 0 else "dense")


def per_launch_bytes(info, cls, fp32):
    """Algorithmic bytes one launch of a kernel class must move."""
    idx = 4 if info.fmt == 0 else 0
    refine = getattr(info, "refine", 0)
    # refine mode: the Bellman pass and residuals read the FP32 copy
    entry = (8 if info.store == 0 else 4 if (info.store == 1 or refine) else 2) + idx
    n, m = info.n, info.m
    xb = 4 if fp32 else 8
    nnz_pi = info.nnz / m
    if cls == "bellman":  # P (all actions), g, V; Phi, pi and g^pi out
        return info.nnz * entry + n * m * 8 + n * 8 + n * (8 + 4 + 8)
    if cls == "japply":   # P^pi (the BF16 copy in refine mode), x in, y out
        return nnz_pi * ((2 + idx) if refine else entry) + n * xb * 2
    if cls == "residual":
        return nnz_pi * entry + n * 8 * 3
    return None  # classes whose bytes depend on the step (persistent, Gram-Schmidt)


def copy_bandwidth(torch, mib=1024, reps=10):
    """Achievable HBM rate of a plain device-to-device copy on this GPU
    (bytes read + written per second), the practical ceiling beside the
    published peak."""
    a = torch.empty(mib << 17, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbps


def timed_solves(h, fn, V, pi, params, runs, torch):
    """Wall time of `runs` solves from V0 = 0 (synchronised each), with the
    last solve's counts."""
    ts, st = [], None
    for _ in range(runs):
        V.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = fn(V, pi, params)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return {"ms_p50": round(float(np.median(ts)), 4), "ms_p90": round(float(np.percentile(ts, 90)), 4),
            "runs": runs, "outer": st["outer"], "inner": st["inner"], "res_inf": st["res_inf"],
            "converged": st["converged"]}


def comparisons(igmres, torch, mdp, wl, restart, igmres_ms, runs, V_main=None):
    """The same workload by the other methods (sparse FP64: exact-evaluation
    PI and OPI with 20 sweeps) or the other precision (mixed workloads: FP64
    storage and arithmetic), each from V0 = 0 to the same tolerance."""
    out = {}
    dev = torch.device("cuda:0")
    V = torch.zeros(mdp.n, dtype=torch.float64, device=dev)
    pi = torch.zeros(mdp.n, dtype=torch.int32, device=dev)
    if wl["mode"] == "fp64":
        with igmres.mdp_create(mdp, store="fp64") as h:
            p = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8, mode="fp64")
            out["pi"] = timed_solves(h, h.pi_solve, V, pi, p, runs, torch)
            p = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8, mode="fp64", opi_sweeps=20)
            out["opi20"] = timed_solves(h, h.opi_solve, V, pi, p, runs, torch)
        for k in ("pi", "opi20"):
            out[k]["igmres_pi_speedup"] = round(out[k]["ms_p50"] / igmres_ms, 2)
    else:
        t0 = time.perf_counter()
        with igmres.mdp_create(mdp, store="fp64") as h:
            create = (time.perf_counter() - t0) * 1e3
            p = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8, mode="fp64")
            out["fp64"] = timed_solves(h, h.igmres_pi_solve, V, pi, p, runs, torch)
            out["fp64"]["create_ms"] = round(create, 1)
        out["fp64"]["mixed_speedup"] = round(out["fp64"]["ms_p50"] / igmres_ms, 2)
        if V_main is not None:
            # the mixed result against the FP64 one: stored-value rounding of P
            # (reported, not gated) plus both solves' tolerance
            vf = V.double()
            out["fp64"]["mixed_rel_diff"] = float((V_main - vf).abs().max() / vf.abs().max())
            out["fp64"]["fp64_cert_bound"] = float(out["fp64"]["res_inf"] / (1 - mdp.gamma))
    return out


CPU_FULL_NNZ = 50_000_000  # above this, the oracle is timed on a reduced instance


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "nproc": cores, "logical_cpus": os.cpu_count()}


def _oracle_rate(O, mdp, restart, threads, budget_s):
    """Solves per second of the oracle's Algorithm 2 on `threads` threads."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(threads):
        t0 = time.perf_counter()
        count = 0
        while True:
            O.igmres_pi(mdp, W=restart, tol=1e-8)
            count += 1
            el = time.perf_counter() - t0
            if el >= budget_s or count >= 1000:
                break
    return count, el


def cpu_baseline(mdp, restart, synth=None, wl_cfg=None, seed=0, budget_s=8.0, c2_legs=True):
    """The oracle's literal Algorithm 2 on the host for about budget_s seconds
    on all cores (the reported value) and again on one core.  Workloads with
    more than CPU_FULL_NNZ entries are sampled by solves of the same recipe
    with a tenth of the states, scaled to the full size by the entry count
    (the oracle's work per iteration is linear in it).  c2_legs: the oracle's
    PI with LU evaluation, value iteration and Algorithm 2 on c2, once each,
    on all cores."""
    from oracle import mdp_oracle as O
    host = host_cpu()
    scale, what = 1.0, "the same workload"
    if synth is not None and mdp.fmt == "csr" and mdp.nnz > CPU_FULL_NNZ:
        small = synth.config(wl_cfg, seed=seed, n=max(1000, mdp.n // 10))
        scale = mdp.nnz / small.nnz
        what = (f"the same recipe at n={small.n} ({small.nnz} entries), scaled by the entry "
                f"ratio {scale:.1f} to the full workload")
        mdp = small
    allc = host["nproc"]
    n_all, t_all = _oracle_rate(O, mdp, restart, allc, budget_s)
    n_one, t_one = _oracle_rate(O, mdp, restart, 1, budget_s)
    out = {"value": n_all / t_all / scale, "unit": "solves/s", "cores": allc, "kind": "oracle",
           "sample": f"{n_all} full solves of {what} by the oracle's literal Algorithm 2 "
                     f"(NumPy/SciPy FP64, BLAS on {allc} threads) in {t_all:.1f} s",
           "single_core": {"value": n_one / t_one / scale, "cores": 1,
                           "sample": f"{n_one} solves in {t_one:.1f} s, BLAS on 1 thread"},
           "host": host}
    if c2_legs:
        from threadpoolctl import threadpool_limits
        c2 = synth.config("c2", seed=seed)
        legs = {}
        with threadpool_limits(allc):
            for name, fn in (("pi_lu", lambda: O.policy_iteration(c2)),
                             ("vi", lambda: O.value_iteration(c2, eps=1e-8 * c2.gamma / (1 - c2.gamma))),
                             ("igmres_pi", lambda: O.igmres_pi(c2, W=30, tol=1e-8))):
                t0 = time.perf_counter()
                fn()
                legs[name + "_s"] = round(time.perf_counter() - t0, 3)
        legs["note"] = ("c2 (n=1e4, m=8, k=20, gamma=0.99) by the oracle on all host cores, one run "
                        "each: PI with LU evaluation to a repeated policy, value iteration to "
                        "||T V - V||_inf <= 1e-8, Algorithm 2 to tol 1e-8")
        out["c2_legs"] = legs
    return out


def class_rooflines(igmres, torch, h, V, pi, params, fp32, runs=3):
    """Average launch time of the streaming kernel classes over `runs`
    solves (HIP events on the launch stream) and their algorithmic bytes per
    launch over that time, against the HBM peak."""
    info = h.info()
    h.profile_enable((1 << igmres.IG_PROFILE_CLASSES) - 1)
    for _ in range(runs):
        V.zero_()
        h.igmres_pi_solve(V, pi, params)
    torch.cuda.synchronize()
    prof = h.profile_read(reset=True)
    h.profile_enable(0)
    out = {}
    for cls in ("bellman", "japply", "residual"):
        ms, cnt = prof.get(cls, (0.0, 0))
        b = per_launch_bytes(info, cls, fp32)
        if not cnt or not b:
            continue
        avg = ms / cnt
        gbps = b / (avg * 1e-3) / 1e9
        out[cls] = {"avg_us": round(avg * 1e3, 2), "alg_bytes_per_launch": round(b),
                    "achieved_GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4)}
    return out


def extra_leg(igmres, synth, torch, name, seed):
    """Another single-GPU workload timed in the same run: c2 (FP64,
    persistent engine) with exact-evaluation PI and OPI(20) beside it; c3
    (dense) with FP32, BF16 and BF16 + FP32-refinement storage beside FP64,
    each with its relative difference from the FP64 result."""
    dev = torch.device("cuda:0")
    mdp = synth.config(name, seed=seed)
    restart = mdp.meta["restart"]
    V = torch.zeros(mdp.n, dtype=torch.float64, device=dev)
    pi = torch.zeros(mdp.n, dtype=torch.int32, device=dev)
    out = {"workload": WORKLOADS[name]["desc"]}
    if name == "c2":
        with igmres.mdp_create(mdp, store="fp64") as h:
            info = h.info()
            p = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8)
            timed_solves(h, h.igmres_pi_solve, V, pi, p, 20, torch)  # warm-up
            r = timed_solves(h, h.igmres_pi_solve, V, pi, p, 200, torch)
            out["igmres_pi"] = r
            out["solves_per_s"] = round(1e3 / r["ms_p50"], 2)
            out["engine"] = (f"persistent, {info.persistent_blocks} blocks" if info.persistent_ok
                             else "stream")
            out["regime"] = "latency-bound: the 19 MB stored MDP is cache-resident"
        out.update(comparisons(igmres, torch, mdp, WORKLOADS["c2"], restart, r["ms_p50"], 5))
        return out
    variants = [("fp64", "fp64", "fp64", False), ("fp32", "fp32", "mixed", False),
                ("bf16", "bf16", "mixed", False), ("bf16+fp32 refine", "bf16", "mixed", True)]
    ref = None
    for label, store, mode, refine in variants:
        with igmres.mdp_create(mdp, store=store, refine=refine) as h:
            p = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8, mode=mode)
            timed_solves(h, h.igmres_pi_solve, V, pi, p, 3, torch)
            r = timed_solves(h, h.igmres_pi_solve, V, pi, p, 20, torch)
            r["kernels"] = class_rooflines(igmres, torch, h, V, pi, p, mode == "mixed")
        Vh = V.double().cpu()
        if ref is None:
            ref = Vh
        else:
            r["rel_diff_vs_fp64"] = float((Vh - ref).abs().max() / ref.abs().max())
            r["speedup_vs_fp64"] = round(out["fp64"]["ms_p50"] / r["ms_p50"], 2)
        out[label] = r
    return out


SERVE_W = 30
SERVE_TOL = 1e-8


def serving_requests(synth, count, seed):
    """The first `count` requests of the seeded serving stream, generated in
    parallel on the host (values rounded to FP32, as stored)."""
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.serving_stream(count, 1.0, seed)

    def make(r):
        m = r.make(threads=1)
        m.val = m.val.astype(np.float32)
        return m
    mdps = []
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        for i, m in enumerate(ex.map(make, specs)):
            mdps.append(m)
            if (i + 1) % 250 == 0:
                print(f"[bench] serving: {i + 1} of {count} requests generated", file=sys.stderr, flush=True)
    return specs, mdps


def serve_once(igmres, mdps, arrivals, prep_threads):
    """Submit request i at arrivals[i] seconds; returns per-request
    (latency_s, completion_s, stats) and the server's counters."""
    srv = igmres.Server(prep_threads=prep_threads)
    params = [igmres.params_default(m.gamma, restart=SERVE_W, tol=SERVE_TOL, mode="mixed") for m in mdps]
    t0 = time.perf_counter()
    tickets, late = [], []
    for i, mdp in enumerate(mdps):
        target = t0 + arrivals[i]
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(target - now, 0.0005))
        tickets.append(srv.submit(mdp, params[i], store="fp32", validate=True))
        late.append(time.perf_counter() - target)
    out = []
    for i, t in enumerate(tickets):
        _, _, st = srv.result(t)
        lat = late[i] + st["latency_ms"] * 1e-3
        out.append((lat, arrivals[i] + lat, st))
    info = srv.info()
    srv.close()
    return out, info


def sequential_fp64(igmres, torch, mdps, budget_s=15.0):
    """The plain FP64 path, one request at a time: mdp_create (the stored
    values in FP64, without the host validation the served requests get),
    igmres_pi_solve (engine chosen by the library), mdp_destroy."""
    t0 = time.perf_counter()
    done = 0
    for m in mdps:
        m64 = m.with_values(val=m.val.astype(np.float64))
        with igmres.mdp_create(m64, store="fp64", validate=False) as h:
            V = torch.zeros(m.n, dtype=torch.float64, device="cuda")
            pi = torch.zeros(m.n, dtype=torch.int32, device="cuda")
            st = h.igmres_pi_solve(V, pi, igmres.params_default(m.gamma, restart=SERVE_W, tol=SERVE_TOL))
            assert st["converged"] == 1
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return done, el


def h2d_bandwidth(torch, mib=512, reps=5):
    """Host-to-device rate of one pinned 512 MiB copy (GB/s): the link every
    served request's transition data has to cross."""
    a = torch.empty(mib << 18, dtype=torch.float32, pin_memory=True)
    a.fill_(1.0)
    b = torch.empty(a.numel(), dtype=torch.float32, device="cuda")
    b.copy_(a, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a, non_blocking=True)
    torch.cuda.synchronize()
    gbps = a.numel() * 4 * reps / (time.perf_counter() - t0) / 1e9
    del a, b
    return gbps


def request_upload_bytes(m):
    """Bytes of one served request that cross the host-device link: its raw
    CSR (int64 row pointers, int32 columns, FP32 values) and FP64 costs."""
    R = m.n * m.m
    return 8 * (R + 1) + m.nnz * (4 + 4) + 8 * R


def serving_leg(igmres, synth, torch, count, seed, loads=(0.5, 0.8, 1.0), prep_threads=12):
    print(f"[bench] serving: generating {count} requests", file=sys.stderr, flush=True)
    specs, mdps = serving_requests(synth, count, seed)
    nnz = np.array([m.nnz for m in mdps], dtype=np.float64)
    up = np.array([request_upload_bytes(m) for m in mdps], dtype=np.float64)
    # saturated: every request queued at t = 0
    print("[bench] serving: saturation run", file=sys.stderr, flush=True)
    sat, info_sat = serve_once(igmres, mdps, np.zeros(count), prep_threads)
    makespan = max(c for _, c, _ in sat)
    lam_sat = count / makespan
    assert all(st["converged"] == 1 for _, _, st in sat), "a served request did not converge"
    dev_ms = sum(st["time_ms"] for _, _, st in sat)
    alg = sum(st["alg_bytes"] for _, _, st in sat)
    link = h2d_bandwidth(torch)
    # Poisson arrivals at each offered load x the saturated throughput
    at_load = {}
    for load in loads:
        rate = load * lam_sat
        arr = np.array([r.arrival for r in synth.serving_stream(count, rate, seed)])
        print(f"[bench] serving: {lam_sat:.1f} solves/s saturated; Poisson run at {rate:.1f}/s",
              file=sys.stderr, flush=True)
        res, _ = serve_once(igmres, mdps, arr, prep_threads)
        lat_ms = np.array([lt for lt, _, _ in res]) * 1e3
        span = max(c for _, c, _ in res)
        sts = [st for _, _, st in res]
        assert all(st["converged"] == 1 for st in sts), "a served request did not converge"
        at_load[str(load)] = {
            "arrival_rate_per_s": round(rate, 2), "solves_per_s": round(count / span, 2),
            "p50_latency_ms": round(float(np.percentile(lat_ms, 50)), 3),
            "p99_latency_ms": round(float(np.percentile(lat_ms, 99)), 3),
            "mean_queue_ms": round(float(np.mean([st["queue_ms"] for st in sts])), 3),
            "mean_prep_ms": round(float(np.mean([st["prep_ms"] for st in sts])), 3),
            "mean_device_ms": round(float(np.mean([st["time_ms"] for st in sts])), 3),
            "max_res_inf": float(max(st["res_inf"] for st in sts))}
    print("[bench] serving: sequential FP64 baseline", file=sys.stderr, flush=True)
    nseq, tseq = sequential_fp64(igmres, torch, mdps)
    main_load = at_load.get("0.8", next(iter(at_load.values())))
    return {
        "workload": f"first {count} requests of the seeded serving stream (seed {seed}): "
                    "n log-uniform in [1e3, 2e5], m in 2..16, k in 4..32 uniform successors, "
                    "Dirichlet(1), gamma in {0.9,0.95,0.99}; FP32-stored P, mixed, W=30, tol 1e-8, "
                    "host CSR in, V and pi back to the host",
        "requests": count, "nnz_mean": round(float(nnz.mean())), "nnz_max": int(nnz.max()),
        "saturated_solves_per_s": round(lam_sat, 2),
        "offered_load": 0.8, "arrival_rate_per_s": main_load["arrival_rate_per_s"],
        "solves_per_s": main_load["solves_per_s"],
        "p50_latency_ms": main_load["p50_latency_ms"], "p99_latency_ms": main_load["p99_latency_ms"],
        "at_load": at_load,
        "saturated_overlap": round(dev_ms / (makespan * 1e3), 3),
        "saturated_alg_GBps": round(alg / makespan / 1e9, 2),
        # the link bound: every request's CSR crosses host->device once
        "upload_MB_mean": round(float(up.mean()) / 1e6, 2),
        "saturated_upload_GBps": round(float(up.sum()) / makespan / 1e9, 2),
        "h2d_link_GBps": round(link, 2),
        "link_bound_solves_per_s": round(link * 1e9 / float(up.mean()), 2),
        "peak_running": info_sat["peak_running"], "prep_threads": prep_threads,
        "arena_peak_GiB": round(info_sat["arena_peak"] / 2**30, 3),
        "sequential_fp64_solves_per_s": round(nseq / tseq, 2), "sequential_fp64_requests": nseq,
        "speedup_vs_sequential_fp64": round(lam_sat / (nseq / tseq), 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed solves (default: 20 for c4, 50 for c3, 200 for c1/c2)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed solves (default 5 for c4, else 20)")
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS) + ["c5"])
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other single-GPU workloads (c2, c3) timed beside the main one")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving stream (2000: the whole stream; its CSR arrays take "
                         "about 115 GB of host memory)")
    ap.add_argument("--prep-threads", type=int, default=12)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--precond", type=int, default=0,
                    help="degree of the Neumann right preconditioner of the inner GMRES (stream engine)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip PI/OPI (FP64 workloads) or the FP64 run (mixed workloads)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration << 17, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "copies": 5}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a solve would shard by contiguous state blocks with all-gathers and all-reduces)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2211_04299_amd import igmres, synth

    if args.workload == "c5":
        torch.cuda.set_device(0)
        sv = serving_leg(igmres, synth, torch, args.serve_requests, args.seed,
                         prep_threads=args.prep_threads)
        out = {"metric": METRIC, "value": sv["solves_per_s"], "unit": "solves/s",
               "n_gpus": 1, "steps": sv["requests"], "warmup": 0,
               "ms_per_step": round(1e3 / sv["solves_per_s"], 4), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
               "config": {"workload": "c5 serving stream: " + sv["workload"]},
               "p50_latency_ms": sv["p50_latency_ms"], "p99_latency_ms": sv["p99_latency_ms"],
               "serving": sv, "roofline": None, "cpu_baseline": None}
        print(json.dumps(out), flush=True)
        return

    wl = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = 20 if args.workload == "c4" else 50 if wl["cfg"] == "c3" else 200
    if args.warmup is None:
        args.warmup = 5 if args.workload == "c4" else 20
    print(f"[bench] generating {args.workload} seed {args.seed}", file=sys.stderr, flush=True)
    mdp = synth.config(wl["cfg"], seed=args.seed)
    restart = mdp.meta["restart"]
    fp32 = wl["mode"] == "mixed"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print("[bench] uploading", file=sys.stderr, flush=True)
    t_up = time.perf_counter()
    h = igmres.mdp_create(mdp, store=wl["store"], refine=wl.get("refine", False))
    create_ms = (time.perf_counter() - t_up) * 1e3
    info = h.info()
    V = torch.zeros(mdp.n, dtype=torch.float64, device=dev)
    pi = torch.zeros(mdp.n, dtype=torch.int32, device=dev)
    params = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8, mode=wl["mode"],
                                   precond=args.precond)

    def step():
        V.zero_()
        return h.igmres_pi_solve(V, pi, params)

    # warmup, with every kernel class timed to find the dominant one
    h.profile_enable((1 << igmres.IG_PROFILE_CLASSES) - 1)
    for _ in range(max(1, args.warmup)):
        st = step()
    prof = h.profile_read(reset=True)
    dom = max(prof, key=lambda k: prof[k][0])
    dom_bit = igmres.PROFILE_CLASS_NAMES.index(dom)
    print(f"[bench] warmup done; per-class ms {json.dumps({k: round(v[0], 3) for k, v in prof.items()})};"
          f" dominant {dom}", file=sys.stderr, flush=True)

    # timed region: only the dominant class carries events, and only about
    # four of its launches per solve (the first, then one in every `every`):
    # a bracketed launch costs two event records on the stream, which would
    # otherwise add to every one of the class's launches (c4: 180 per solve)
    per_solve = prof[dom][1] / max(1, args.warmup)
    every = max(1, int(per_solve) // 4)
    h.profile_enable(1 << dom_bit)
    h.profile_sample(every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile_read(reset=True)
    h.profile_enable(0)
    h.profile_sample(1)
    ms_step = (t1 - t0) * 1e3 / args.steps
    st = stats[-1]
    assert all(s["converged"] == 1 for s in stats), "a timed solve did not converge"

    dom_ms, dom_n = prof[dom]
    dom_avg_ms = dom_ms / max(dom_n, 1)
    if dom == "persistent":  # one launch = one whole solve: its algorithmic bytes
        b = float(np.mean([s["alg_bytes"] for s in stats]))
    else:
        b = per_launch_bytes(info, dom, fp32)
    roof = None
    if b is not None and dom_avg_ms > 0:
        ach = b / (dom_avg_ms * 1e-3) / 1e9
        traffic = None
        tfile = os.path.join(ROOT, "profiles", f"traffic_{dom}_{args.workload}.json")
        if os.path.exists(tfile):
            t = json.load(open(tfile))
            if t.get("kernel_source_hash") == kernel_source_hash(kernel_group(dom, info.fmt)):
                traffic = t.get("hbm_bytes_per_launch")
        cbw = copy_bandwidth(torch)
        # the stored MDP against the 256 MB last-level cache: below it, repeated
        # passes are served from cache and the solve is bound by latency
        # (grid barriers, dependent loads), not by HBM bandwidth
        p_bytes = info.nnz * ((8 if info.store == 0 else 4 if info.store == 1 else 2)
                              + (4 if info.fmt == 0 else 0))
        regime = ("latency-bound; the stored MDP (%.0f MB) is cache-resident" % (p_bytes / 1e6)
                  if p_bytes < 256e6 else "HBM streaming")
        roof = {"bound": "hbm" if p_bytes >= 256e6 else "latency", "achieved": round(ach, 2),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": traffic,
                # the measured HBM-side bytes per launch at the same duration:
                # how close the launch runs to the peak with the bytes it moves
                "traffic_GBps": round(traffic / (dom_avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                "traffic_frac": round(traffic / (dom_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
                if traffic else None,
                "kernel": dom, "launches": dom_n, "sampled_every": every,
                "avg_us": round(dom_avg_ms * 1e3, 3),
                "alg_bytes_per_launch": b, "copy_GBps": round(cbw, 1), "regime": regime}

    dev_ms = np.array([s["time_ms"] for s in stats])
    # the same workload with the truncated-Neumann right preconditioner in
    # the inner GMRES (the paper's future work; not the headline method)
    precond_leg = None
    if not args.no_extra and args.workload == "c4" and args.precond == 0:
        print("[bench] preconditioned c4", file=sys.stderr, flush=True)
        V_main = V.clone()
        precond_leg = {}
        for deg in (1, 3):
            pp = igmres.params_default(mdp.gamma, restart=restart, tol=1e-8, mode=wl["mode"],
                                       precond=deg)
            timed_solves(h, h.igmres_pi_solve, V, pi, pp, 1, torch)
            r = timed_solves(h, h.igmres_pi_solve, V, pi, pp, 3, torch)
            r["speedup_vs_plain"] = round(ms_step / r["ms_p50"], 3)
            r["rel_diff_vs_plain"] = float((V - V_main).abs().max() / V_main.abs().max())
            precond_leg[f"neumann_degree_{deg}"] = r
        V.copy_(V_main)
    cmp = None
    if not args.no_compare:
        print("[bench] comparisons", file=sys.stderr, flush=True)
        runs = 5 if args.workload in ("c1", "c2", "c3", "c3-bf16") else 2
        try:
            cmp = comparisons(igmres, torch, mdp, wl, restart, ms_step, runs, V_main=V.clone())
        except igmres.IgError as e:  # reported, never fatal to the main line
            cmp = {"error": str(e)}

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(mdp, restart, synth, wl["cfg"], args.seed)

    h.close()
    del h
    extra = None
    if not args.no_extra and args.workload == "c4":
        extra = {}
        for name in ("c2", "c3"):
            print(f"[bench] extra workload {name}", file=sys.stderr, flush=True)
            try:
                extra[name] = extra_leg(igmres, synth, torch, name, args.seed)
            except igmres.IgError as e:  # reported, never fatal to the main line
                extra[name] = {"error": str(e)}
    sv = None
    if not args.no_serving:
        sv = serving_leg(igmres, synth, torch, args.serve_requests, args.seed,
                         prep_threads=args.prep_threads)

    out = {
        "metric": METRIC, "value": round(1e3 / ms_step, 3), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if not fp32 else "f64+f32", "data": "synthetic",
        "precision": ("FP64 throughout" if not fp32 else
                      f"P stored in {wl['store'].upper()}" +
                      (" for the products inside GMRES, with an FP32 copy for the Bellman passes "
                       "and residuals" if wl.get("refine") else "") +
                      "; FP32 Krylov basis and P^pi products with FP32 accumulation; FP64 Bellman "
                      "pass, residuals, dot products, solution update and Hessenberg/Givens solve"),
        "config": {"workload": f"{args.workload}: {wl['desc']}", "seed": args.seed,
                   "n": mdp.n, "m": mdp.m, "nnz": int(info.nnz), "restart": restart,
                   "engine": ("persistent (one cooperative launch per solve, "
                              f"{info.persistent_blocks} blocks)") if info.persistent_ok and not args.precond
                   else "stream (one launch per step)",
                   "precond_degree": args.precond},
        "time_to_tol_ms": round(ms_step, 4),
        "solve_ms_p50": round(float(np.median(dev_ms)), 4),
        "solve_ms_p90": round(float(np.percentile(dev_ms, 90)), 4),
        "create_ms": round(create_ms, 2),
        "compare": cmp,
        "preconditioned": precond_leg,
        "solve": {"outer": st["outer"], "inner": st["inner"], "restarts": st["restarts"],
                  "explicit_residuals": st["explicit_residuals"], "res_inf": st["res_inf"],
                  "device_ms": round(st["time_ms"], 4),
                  "alg_GB": round(st["alg_bytes"] / 1e9, 5),
                  "alg_GBps_solve": round(st["alg_bytes"] / (ms_step * 1e-3) / 1e9, 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
        "serving": sv,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
