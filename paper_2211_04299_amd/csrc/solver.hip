// Solver drivers: Algorithm 2 (GMRES(W) policy iteration), its inner policy
// evaluation, policy iteration, optimistic policy iteration and inexact policy
// iteration with a value-iteration inner solver (Algorithm 1).  All vector
// work runs in the HIP kernels; the host only sequences launches and reads
// the few scalars that decide the control flow.
#include <cmath>
#include <cstring>
#include <utility>

#include "internal.hpp"

namespace ig {

Mdp* handle_of(ig_mdp_t h);

namespace {

constexpr double kStagnation = 1e-6;  // min relative 2-norm decrease per restart cycle

// ---- format dispatch ------------------------------------------------------
void k_bellman(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
               const int32_t* pi_old, double tie, hipStream_t s) {
  if (d.fmt == IG_FMT_CSR)
    launch_bellman_sparse(d, V, TV, Phi, pi, pi_old, tie, true, s);
  else
    launch_bellman_dense(d, V, TV, Phi, pi, pi_old, tie, s);
}
void k_japply(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* eta, void* y,
              hipStream_t s) {
  if (d.fmt == IG_FMT_CSR)
    launch_japply_sparse(d, fp32, x, eta, y, s);
  else
    launch_japply_dense(d, fp32, pi, x, eta, y, s);
}
void k_pstep(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* sx, const void* z,
             const double* sz, void* y, hipStream_t s) {
  if (d.fmt == IG_FMT_CSR)
    launch_pstep_sparse(d, fp32, x, sx, z, sz, y, s);
  else
    launch_pstep_dense(d, fp32, pi, x, sx, z, sz, y, s);
}
void k_residual(Mdp& d, const int32_t* pi, const double* V, double* r, hipStream_t s) {
  if (d.fmt == IG_FMT_CSR)
    launch_residual_sparse(d, V, r, s);
  else
    launch_residual_dense(d, pi, V, r, s);
}
// one application of T^pi; `finish` reduces its difference norms (not
// needed by OPI's fixed sweeps)
void k_vi(Mdp& d, const int32_t* pi, const double* Vin, double* Vout, hipStream_t s,
          bool finish = true) {
  if (d.fmt == IG_FMT_CSR)
    launch_vi_sweep_sparse(d, Vin, Vout, s, finish);
  else
    launch_vi_sweep_dense(d, pi, Vin, Vout, s, finish);
}
void k_gather(Mdp& d, const int32_t* pi, hipStream_t s) {
  if (d.fmt == IG_FMT_CSR)
    launch_gather_policy_sparse(d, pi, s);
  else
    launch_gather_policy_dense(d, pi, s);
}

// ---- algorithmic byte counts (what each pass must move) --------------------
struct Bytes {
  const Mdp& d;
  double entry() const { return d.vb + (d.fmt == IG_FMT_CSR ? 4.0 : 0.0); }
  // entries of the products inside GMRES (the BF16 copy in refine mode)
  double entry_in() const { return d.in_vb + (d.fmt == IG_FMT_CSR ? 4.0 : 0.0); }
  double nnz_pi() const { return (double)d.nnz / d.m; }
  // refine mode, sparse: the compact P^pi is rounded to BF16 after the pass
  double bellman() const {
    return d.nnz * entry() + d.n * (double)d.m * 8 + d.n * (8.0 + 8 + 4) +
           (d.refine && d.fmt == IG_FMT_CSR ? nnz_pi() * (d.vb + d.in_vb) : 0.0);
  }
  double japply(bool fp32) const { return nnz_pi() * entry_in() + d.n * (fp32 ? 4.0 : 8.0) * 2; }
  // Orthogonalisation against Q_0..Q_c: the method's basis traffic (each
  // column read twice, as modified Gram-Schmidt does) and four more vectors.
  // The passes run here move more (the fused form reads the basis in both
  // of its passes); that extra is an implementation cost, not counted.
  double gs(bool fp32, int c) const {
    const double xb = fp32 ? 4 : 8;
    return d.n * xb * (2.0 * (c + 1) + 4.0);
  }
  double update(bool fp32, int i) const { return d.n * (i * (fp32 ? 4.0 : 8.0) + 16); }
  double residual() const { return nnz_pi() * entry() + d.n * 24.0; }
  double vi() const { return nnz_pi() * entry() + d.n * 24.0; }
};

struct Inner {
  int steps = 0, restarts = 0, expl = 0, breakdowns = 0;
  bool stagnated = false, met = false;
  double res_inf = 0.0, bytes = 0.0;
};

// Inner while-loop of Algorithm 2 for the policy whose P^pi / g^pi are in
// place.  On entry V = x0 and d.ws.r holds g - J x0 with infinity-norm r_inf
// and squared 2-norm r_l2sq (host copy) / *r_l2sq_dev (device copy).
// Stops when ||g - J V||_inf <= thr.
//
// Column c's Arnoldi step is y = J w1 / eta (w1 the previous once-orthogonal
// vector), then two Gram-Schmidt passes and the Givens update; the residual
// of column c-1's iterate, ||Q z||_inf, arrives with the step of column c.
// A stop is always confirmed on the true FP64 residual g - J V.
//
// precond = d > 0: right preconditioning with the truncated Neumann series
// M^{-1} = sum_{k<=d} (gamma P^pi)^k (Horner steps).  Arnoldi runs on
// J M^{-1} and iterates are V = Vb + M^{-1} Q y; the residual and every test
// stay those of J, so the implicit residual Q z is still g - J V.
ig_status gmres_inner(Mdp& d, const int32_t* pi, double* V, double r_inf, double r_l2sq,
                      const double* r_l2sq_dev, double thr, int W, int max_inner, bool fp32,
                      int precond, hipStream_t s, Inner& out) {
  Workspace& ws = d.ws;
  const Bytes B{d};
  if (precond > 0)
    if (ig_status e = ensure_precond(d)) return e;
  // M^{-1}(src * sc) by `precond` Horner steps into ws.pa / ws.pb
  auto minv = [&](bool f32, const void* src, const double* sc) -> const void* {
    void* a = ws.pa;
    void* b = ws.pb;
    k_pstep(d, f32, pi, src, sc, src, sc, a, s);
    for (int k = 1; k < precond; ++k) {
      k_pstep(d, f32, pi, src, sc, a, nullptr, b, s);
      std::swap(a, b);
    }
    return a;
  };
  out.res_inf = r_inf;
  if (r_inf <= thr) {
    out.met = true;
    return IG_OK;
  }
  const double xb = fp32 ? 4 : 8;
  double cycle_beta = std::sqrt(r_l2sq);
  IG_HIP(hipMemcpyAsync(ws.Vb, V, (size_t)d.n * 8, hipMemcpyDeviceToDevice, s));
  launch_form_q0(d, fp32, ws.r, r_l2sq_dev, s);
  out.bytes += d.n * (8.0 + xb + 16);
  void* y = ws.wA;   // J times the newest basis vector
  void* w1 = ws.wB;  // once-orthogonalised Arnoldi vector
  const double* eta_dev = &d.st->eta;

  // a new cycle from the true residual at the current iterate (in ws.r, its
  // squared 2-norm in the status); `stop` when the last cycle lowered the
  // residual 2-norm by less than the stagnation factor
  bool stop = false;
  auto restart = [&]() -> ig_status {
    const double nb = std::sqrt(d.hst->res_l2sq);
    if (nb > (1.0 - kStagnation) * cycle_beta) {
      out.stagnated = true;
      stop = true;
      return IG_OK;
    }
    cycle_beta = nb;
    ++out.restarts;
    IG_HIP(hipMemcpyAsync(ws.Vb, V, (size_t)d.n * 8, hipMemcpyDeviceToDevice, s));
    launch_form_q0(d, fp32, ws.r, &d.st->res_l2sq, s);
    out.bytes += d.n * (8.0 + xb + 16);
    return IG_OK;
  };

  // V = Vb + Q_{0..cnt-1} y and its true residual (FP64)
  auto explicit_residual = [&](int cnt) -> ig_status {
    if (precond == 0) {
      launch_update(d, fp32, cnt, ws.Vb, V, s);
    } else {  // V = Vb + M^{-1} (Q y), the products in FP64
      launch_update(d, fp32, cnt, nullptr, V, s);
      launch_vadd(d, ws.Vb, (const double*)minv(false, V, nullptr), V, s);
      out.bytes += precond * B.japply(false);
    }
    k_residual(d, pi, V, ws.r, s);
    out.bytes += B.update(fp32, cnt) + B.residual();
    ++out.expl;
    if (ig_status e = sync_status(d, s)) return e;
    out.res_inf = d.hst->res_inf;
    return IG_OK;
  };

  // y = J M^{-1} (column c's input): Q_0 at c = 0, else w1 / eta
  auto product = [&](int c) {
    if (precond > 0)
      k_japply(d, fp32, pi, minv(fp32, c == 0 ? ws.Q : w1, c == 0 ? nullptr : eta_dev), nullptr, y, s);
    else if (c == 0)
      k_japply(d, fp32, pi, ws.Q, nullptr, y, s);
    else
      k_japply(d, fp32, pi, w1, eta_dev, y, s);
  };
  // The product of column c+1 reads only w1 and eta of column c and writes
  // only y, which nothing reads until the next Gram-Schmidt pass.  It is
  // queued before the host waits for column c's scalars, so the device
  // does not idle while the host decides; when the decision ends the cycle
  // or the solve, the queued product is simply not used.  The scalars come
  // from the pinned snapshot the Givens kernel writes.
  const bool pipe = d.hsnap != nullptr && d.ev_step != nullptr;
  bool queued = false;  // the product of column c is already on the stream
  // 2-norm residual of the last finished column and the infinity- to 2-norm
  // ratio of the residual before it (negative: not known yet); they tell
  // when the step now running will likely end the inner solve, and then the
  // next product is not queued (it would be thrown away)
  double last_rho = -1.0, inf_ratio = -1.0;
  auto leave = [&](ig_status e) {
    if (queued) (void)hipStreamSynchronize(s);
    return e;
  };
  for (int c = 0;;) {
    if (!queued) product(c);
    queued = false;
    launch_gs_step(d, fp32, c, y, w1, s);
    out.bytes += (1 + precond) * B.japply(fp32) + B.gs(fp32, c);
    double eta, rho, res_impl;
    if (pipe) {
      IG_HIP(hipEventRecord(d.ev_step, s));
      // the step's test is on the residual of column c-1, whose 2-norm is
      // last_rho; its infinity norm is estimated with the last ratio
      const bool near_stop =
          c > 0 && last_rho >= 0.0 && last_rho * (inf_ratio >= 0.0 ? inf_ratio : 1.0) <= 2.0 * thr;
      if (c + 1 < W && out.steps + 1 < max_inner && !near_stop) {
        product(c + 1);
        queued = true;
      }
      IG_HIP(hipEventSynchronize(d.ev_step));
      const volatile StepSnap* sn = d.hsnap;
      eta = sn->eta;
      rho = sn->rho;
      res_impl = sn->res_impl;
    } else {
      if (ig_status e = sync_status(d, s)) return e;
      eta = d.hst->eta;
      rho = d.hst->rho;
      res_impl = d.hst->res_impl;
    }
    ++out.steps;
    if (c > 0 && last_rho > 0.0) inf_ratio = res_impl / last_rho;
    last_rho = rho;
    if (!std::isfinite(eta) || !std::isfinite(rho) || (c > 0 && !std::isfinite(res_impl)))
      return leave(fail(IG_E_NUMERIC, "non-finite value in the Arnoldi process"));
    // the test of Algorithm 2 for column c-1 (residual known one step late)
    if (c > 0 && res_impl <= thr) {
      if (ig_status e = explicit_residual(c)) return leave(e);
      if (out.res_inf <= thr) {  // column c was speculative: not counted
        --out.steps;
        out.met = true;
        return leave(IG_OK);
      }
      if (d.refine) {
        // refine mode: the BF16 system's residual meets the rule, the FP32
        // one does not; the next cycle solves for the correction from the
        // true residual (column c is dropped)
        --out.steps;
        if (ig_status e = restart()) return leave(e);
        queued = false;
        if (stop) return leave(IG_OK);
        c = 0;
        continue;
      }
    }
    if (eta == 0.0) {  // ||q||_2 = 0: the least-squares solution is exact; leave the loop
      ++out.breakdowns;
      if (ig_status e = explicit_residual(c + 1)) return leave(e);
      out.met = out.res_inf <= thr;
      return leave(IG_OK);
    }
    // ||r||_inf <= ||r||_2 = rho: the rule holds for column c in exact arithmetic
    if (rho <= thr || out.steps >= max_inner || c + 1 == W) {
      if (ig_status e = explicit_residual(c + 1)) return leave(e);
      if (out.res_inf <= thr) {
        out.met = true;
        return leave(IG_OK);
      }
      if (out.steps >= max_inner) return leave(IG_OK);
    }
    // restart from the residual at the current iterate at the end of a
    // cycle, and in refine mode after any explicit residual that missed
    if (c + 1 == W || (d.refine && rho <= thr)) {
      if (ig_status e = restart()) return leave(e);
      queued = false;
      if (stop) return leave(IG_OK);
      c = 0;
      continue;
    }
    ++c;
  }
}

}  // namespace

ig_status check_params(const Mdp& d, const ig_params* p, bool need_alpha) {
  if (!p) return fail(IG_E_INVALID, "params is NULL");
  if (need_alpha && !(p->alpha > 0.0 && p->alpha < 1.0)) return fail(IG_E_INVALID, "alpha must be in (0,1)");
  if (p->restart < 1) return fail(IG_E_INVALID, "restart must be >= 1");
  if (p->restart > IG_MAX_RESTART) return fail(IG_E_TOO_LARGE, "restart exceeds IG_MAX_RESTART");
  if (p->max_outer < 1 || p->max_inner < 1) return fail(IG_E_INVALID, "iteration caps must be >= 1");
  if (!(p->tol > 0.0)) return fail(IG_E_INVALID, "tol must be > 0");
  if (p->mode != IG_MODE_FP64 && p->mode != IG_MODE_MIXED) return fail(IG_E_INVALID, "bad mode");
  if (p->blocks < 0) return fail(IG_E_INVALID, "blocks must be >= 0");
  if (p->precond < 0 || p->precond > 16) return fail(IG_E_INVALID, "precond must be in 0..16");
  if (p->precond > 0 && p->engine == 2)
    return fail(IG_E_INVALID, "the persistent engine has no preconditioner (use engine 0 or 1)");
  if (d.refine && p->engine == 2)
    return fail(IG_E_INVALID, "the persistent engine does not take refine-mode handles (use engine 0 or 1)");
  return IG_OK;
}

namespace {

struct Timer {
  Mdp& d;
  hipStream_t s;
  Timer(Mdp& d_, hipStream_t s_) : d(d_), s(s_) { (void)hipEventRecord(d.ev0, s); }
  double stop() {
    (void)hipEventRecord(d.ev1, s);
    (void)hipEventSynchronize(d.ev1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, d.ev0, d.ev1);
    return ms;
  }
};

void add_inner(ig_stats& st, const Inner& in) {
  st.inner += in.steps;
  st.restarts += in.restarts;
  st.explicit_residuals += in.expl;
  st.breakdowns += in.breakdowns;
  st.stagnations += in.stagnated ? 1 : 0;
  st.alg_bytes += in.bytes;
}

// Bellman pass + status read; returns IG_E_NUMERIC on NaN/Inf.
ig_status bellman_pass(Mdp& d, const double* V, double* TV, int32_t* pi, const int32_t* pi_old,
                       double tie, ig_stats& st, hipStream_t s) {
  k_bellman(d, V, TV, d.ws.r, pi, pi_old, tie, s);
  st.alg_bytes += Bytes{d}.bellman();
  ++st.bellman_passes;
  if (ig_status e = sync_status(d, s)) return e;
  if (d.hst->nonfinite) return fail(IG_E_NUMERIC, "NaN or Inf in the Bellman pass");
  return IG_OK;
}

ig_status run_igmres(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                     hipStream_t s) {
  const bool fp32 = p.mode == IG_MODE_MIXED;
  if (p.engine < 0 || p.engine > 2) return fail(IG_E_INVALID, "engine must be 0, 1 or 2");
  if (p.engine == 2 || (p.engine == 0 && p.precond == 0 && p.restart <= kPersistMaxRestart &&
                        d.coop && persistent_fits(d)))
    return persistent_igmres(d, V, pi, p, st, s);
  if (ig_status e = ensure_workspace(d, p.restart, fp32)) return e;
  // polish: pi_{k-1}, kept in the spare vector, and the Bellman pass counts
  // the states whose greedy action differs from it (an incumbent is never
  // preferred: tie allowance -inf)
  int32_t* prev = reinterpret_cast<int32_t*>(d.ws.t);
  for (int k = 0;; ++k) {
    // pi_k = GreedyPolicy(V_k); Phi_k = g - J V_k = T V_k - V_k
    const bool cmp = p.polish && k > 0;
    if (cmp) IG_HIP(hipMemcpyAsync(prev, pi, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s));
    if (ig_status e = bellman_pass(d, V, nullptr, pi, cmp ? prev : nullptr,
                                   cmp ? -INFINITY : 0.0, st, s))
      return e;
    const double res = d.hst->phi_inf;
    st.res_inf = res;
    st.outer = k;
    if (res <= p.tol) {
      st.converged = 1;
      return IG_OK;
    }
    if (k >= p.max_outer) return fail(IG_E_NOCONV, "max_outer reached");
    const double alpha = p.forcing ? std::min(p.alpha, std::sqrt(res)) : p.alpha;
    double thr = alpha * res;
    if (cmp && d.hst->changes == 0) thr = std::min(thr, 0.5 * p.tol);
    Inner in;
    if (ig_status e = gmres_inner(d, pi, V, res, d.hst->phi_l2sq, &d.st->phi_l2sq, thr,
                                  p.restart, p.max_inner, fp32, p.precond, s, in))
      return e;
    add_inner(st, in);
  }
}

ig_status run_eval(Mdp& d, const int32_t* pi, double* V, const ig_params& p, ig_stats& st,
                   hipStream_t s) {
  const bool fp32 = p.mode == IG_MODE_MIXED;
  if (ig_status e = ensure_workspace(d, p.restart, fp32)) return e;
  k_gather(d, pi, s);
  if (ig_status e = sync_status(d, s)) return e;
  if (d.hst->changes) return fail(IG_E_INVALID, "policy entry out of range or outside A(s)");
  k_residual(d, pi, V, d.ws.r, s);
  st.alg_bytes += Bytes{d}.residual();
  if (ig_status e = sync_status(d, s)) return e;
  if (!std::isfinite(d.hst->res_inf)) return fail(IG_E_NUMERIC, "non-finite residual");
  Inner in;
  if (ig_status e = gmres_inner(d, pi, V, d.hst->res_inf, d.hst->res_l2sq, &d.st->res_l2sq,
                                p.alpha * d.hst->res_inf, p.restart, p.max_inner, fp32, p.precond, s,
                                in))
    return e;
  add_inner(st, in);
  st.res_inf = in.res_inf;
  st.converged = in.met ? 1 : 0;
  return in.met ? IG_OK : fail(IG_E_NOCONV, "inexact evaluation rule not met");
}

ig_status run_pi(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                 hipStream_t s) {
  const bool fp32 = p.mode == IG_MODE_MIXED;
  if (ig_status e = ensure_workspace(d, p.restart, fp32)) return e;
  // pi_0 = GreedyPolicy(V0)
  if (ig_status e = bellman_pass(d, V, nullptr, pi, nullptr, 0.0, st, s)) return e;
  const double thr = p.eval_rtol * std::max(d.cost_max, 1e-300);
  for (int k = 1;; ++k) {
    st.outer = k;
    // evaluation: GMRES to the residual floor
    k_residual(d, pi, V, d.ws.r, s);
    st.alg_bytes += Bytes{d}.residual();
    if (ig_status e = sync_status(d, s)) return e;
    Inner in;
    if (ig_status e = gmres_inner(d, pi, V, d.hst->res_inf, d.hst->res_l2sq, &d.st->res_l2sq, thr,
                                  p.restart, p.max_inner, fp32, p.precond, s, in))
      return e;
    add_inner(st, in);
    // improvement, keeping the incumbent unless strictly better by the tie margin
    const double tie = 1e-12 * std::max(1.0, d.hst->vmax);
    if (ig_status e = bellman_pass(d, V, nullptr, pi, pi, tie, st, s)) return e;
    st.res_inf = d.hst->phi_inf;
    if (d.hst->changes == 0) {
      st.converged = 1;
      return IG_OK;
    }
    if (k >= p.max_outer) return fail(IG_E_NOCONV, "max_outer reached");
  }
}

ig_status run_opi(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                  hipStream_t s) {
  if (p.opi_sweeps < 1) return fail(IG_E_INVALID, "opi_sweeps must be >= 1");
  if (ig_status e = ensure_workspace(d, 1, false)) return e;
  const Bytes B{d};
  for (int k = 0;; ++k) {
    if (ig_status e = bellman_pass(d, V, d.ws.t, pi, nullptr, 0.0, st, s)) return e;
    st.res_inf = d.hst->phi_inf;
    st.outer = k;
    if (d.hst->phi_inf <= p.tol) {
      st.converged = 1;
      return IG_OK;
    }
    if (k >= p.max_outer) return fail(IG_E_NOCONV, "max_outer reached");
    // the Bellman pass is the first application of T^{pi_k}; W-1 more follow
    double* cur = d.ws.t;
    double* other = V;
    for (int j = 1; j < p.opi_sweeps; ++j) {
      k_vi(d, pi, cur, other, s, false);
      st.alg_bytes += B.vi();
      std::swap(cur, other);
    }
    st.inner += p.opi_sweeps;  // applications of T^pi, the Bellman pass included
    if (cur != V) IG_HIP(hipMemcpyAsync(V, cur, (size_t)d.n * 8, hipMemcpyDeviceToDevice, s));
  }
}

ig_status run_ipi_vi(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                     hipStream_t s) {
  if (ig_status e = ensure_workspace(d, 1, false)) return e;
  const Bytes B{d};
  for (int k = 0;; ++k) {
    if (ig_status e = bellman_pass(d, V, nullptr, pi, nullptr, 0.0, st, s)) return e;
    const double res = d.hst->phi_inf;
    st.res_inf = res;
    st.outer = k;
    if (res <= p.tol) {
      st.converged = 1;
      return IG_OK;
    }
    if (k >= p.max_outer) return fail(IG_E_NOCONV, "max_outer reached");
    const double thr = (p.forcing ? std::min(p.alpha, std::sqrt(res)) : p.alpha) * res;
    // V_{k+1} <- V_k; while ||g - J V_{k+1}||_inf > thr: V_{k+1} <- T^pi V_{k+1}.
    // A sweep from x yields T^pi x and ||T^pi x - x||_inf, the residual at x.
    double* cur = V;
    double* other = d.ws.t;
    for (int j = 0; j < p.max_inner; ++j) {
      k_vi(d, pi, cur, other, s);
      st.alg_bytes += B.vi();
      ++st.inner;
      if (ig_status e = sync_status(d, s)) return e;
      if (d.hst->aux <= thr) break;  // the rule holds at cur
      std::swap(cur, other);
    }
    if (cur != V) IG_HIP(hipMemcpyAsync(V, cur, (size_t)d.n * 8, hipMemcpyDeviceToDevice, s));
  }
}

using Runner = ig_status (*)(Mdp&, double*, int32_t*, const ig_params&, ig_stats&, hipStream_t);

ig_status solve_entry(ig_mdp_t h, double* V, int32_t* pi, const ig_params* p, ig_stats* stats,
                      void* stream, Runner run, bool need_alpha) {
  Mdp* d = handle_of(h);
  if (!d) return fail(IG_E_INVALID, "NULL handle");
  if (!V) return fail(IG_E_INVALID, "V is NULL");
  if (ig_status e = check_params(*d, p, need_alpha)) return e;
  hipStream_t s = (hipStream_t)stream;
  ig_stats st;
  std::memset(&st, 0, sizeof st);
  int32_t* pol = pi ? pi : nullptr;
  if (!pol) {
    if (ig_status e = ensure_workspace(*d, 1, false)) return e;
    pol = d->ws.pi;
  }
  Timer t(*d, s);
  ig_status e;
  try {
    e = run(*d, V, pol, *p, st, s);
  } catch (...) {
    e = fail(IG_E_DEVICE, "unexpected host exception");
  }
  st.time_ms = t.stop();
  st.cert_bound = st.res_inf / (1.0 - d->gamma);
  if (stats) *stats = st;
  return e;
}

}  // namespace
}  // namespace ig

using namespace ig;

extern "C" {

ig_status bellman_apply(ig_mdp_t h, const double* V, double* TV, int32_t* pi, double* res_inf,
                        void* stream) {
  Mdp* d = handle_of(h);
  if (!d) return fail(IG_E_INVALID, "NULL handle");
  if (!V) return fail(IG_E_INVALID, "V is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (ig_status e = ensure_workspace(*d, 1, false)) return e;
  k_bellman(*d, V, TV, d->ws.r, pi ? pi : d->ws.pi, nullptr, 0.0, s);
  if (res_inf)
    IG_HIP(hipMemcpyAsync(res_inf, &d->st->phi_inf, sizeof(double), hipMemcpyDeviceToDevice, s));
  IG_HIP(hipGetLastError());
  return IG_OK;
}

ig_status policy_eval_gmres(ig_mdp_t h, const int32_t* pi, double* V, const ig_params* p,
                            ig_stats* stats, void* stream) {
  if (!pi) return fail(IG_E_INVALID, "pi is NULL");
  struct Ctx {
    static ig_status run(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                         hipStream_t s) {
      return run_eval(d, pi, V, p, st, s);
    }
  };
  return solve_entry(h, V, const_cast<int32_t*>(pi), p, stats, stream, &Ctx::run, true);
}

ig_status igmres_pi_solve(ig_mdp_t h, double* V, int32_t* pi, const ig_params* p,
                          ig_stats* stats, void* stream) {
  return solve_entry(h, V, pi, p, stats, stream, &run_igmres, true);
}

ig_status pi_solve(ig_mdp_t h, double* V, int32_t* pi, const ig_params* p, ig_stats* stats,
                   void* stream) {
  return solve_entry(h, V, pi, p, stats, stream, &run_pi, false);
}

ig_status opi_solve(ig_mdp_t h, double* V, int32_t* pi, const ig_params* p, ig_stats* stats,
                    void* stream) {
  return solve_entry(h, V, pi, p, stats, stream, &run_opi, false);
}

ig_status ipi_vi_solve(ig_mdp_t h, double* V, int32_t* pi, const ig_params* p, ig_stats* stats,
                       void* stream) {
  return solve_entry(h, V, pi, p, stats, stream, &run_ipi_vi, true);
}

}  // extern "C"
