// Streaming kernels over the sliced-ELL transition data (gfx950).
//
// Work mapping: a wavefront serves S = 64/G consecutive states of one 64-state
// slice; the G lanes of a state ("groups", lane = g*S + ls) split that
// state's actions (Bellman pass) or the entries of its P^pi row (products).
// Consecutive lanes of a group address consecutive states, so every value
// and column load is a contiguous run of S elements; the G partial results of
// a state are combined with xor-shuffles over offsets S, 2S, ..., 32.
#include "internal.hpp"

namespace ig {

namespace {

template <typename VT, int G>
__global__ __launch_bounds__(kBlock) void k_bellman(
    SellP<VT> P, const double* __restrict__ cost, int m, int64_t n, double gamma,
    const double* __restrict__ V, double* __restrict__ TV, double* __restrict__ Phi,
    int32_t* __restrict__ pi, const int32_t* __restrict__ pi_old, double tie_abs,
    double* __restrict__ cpi, SellPi<VT> Pp, RedCtx red, DevStatus* __restrict__ st) {
  constexpr int S = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int ls = lane % S, g = lane / S;
  const int64_t nw = (n + S - 1) / S;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  double pmax = 0.0, psum = 0.0, nonfin = 0.0, chg = 0.0;

  for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; w < nw;
       w += wstride) {
    const int64_t s = w * S + ls;  // < nslices*64: padded slice entries exist
    const bool valid = s < n;
    const int64_t sc = valid ? s : n - 1;
    const int64_t b = s >> 6;
    const int l = (int)(s & 63);
    const int Kb = P.width[b];
    const int64_t ob = P.off[b];
    const int inc = pi_old ? pi_old[sc] : -1;

    double best = INFINITY, qinc = INFINITY;
    int besta = m;  // sentinel: no finite candidate yet
    for (int a = g; a < m; a += G) {
      const int64_t base = ob + (((int64_t)a * Kb) << 6) + l;
      double acc = 0.0;
      for (int j = 0; j < Kb; ++j) {
        const int64_t e = base + ((int64_t)j << 6);
        acc = fma(to_d(P.val[e]), V[P.col[e]], acc);
      }
      const double q = cost[(int64_t)a * n + sc] + gamma * acc;
      if (!(q - q == 0.0)) nonfin += valid ? 1.0 : 0.0;  // NaN or +-Inf
      if (q < best) {  // actions visited in increasing order: lowest index wins ties
        best = q;
        besta = a;
      }
      if (a == inc) qinc = q;
    }
#pragma unroll
    for (int o = S; o < kWave; o <<= 1) {
      const double ob2 = __shfl_xor(best, o);
      const int oa = __shfl_xor(besta, o);
      if (ob2 < best || (ob2 == best && oa < besta)) {
        best = ob2;
        besta = oa;
      }
      qinc = fmin(qinc, __shfl_xor(qinc, o));
    }
    if (besta >= m) {  // every Q-value non-finite: keep indices in range
      besta = 0;
      best = NAN;
    }
    int astar = besta;
    double tv = best;
    if (inc >= 0 && inc < m && qinc <= best + tie_abs) {
      astar = inc;
      tv = qinc;
    }
    if (valid && g == 0) {
      const double phi = tv - V[s];
      if (TV) TV[s] = tv;
      Phi[s] = phi;
      pi[s] = astar;
      cpi[s] = cost[(int64_t)astar * n + s];
      if (!(phi - phi == 0.0)) nonfin += 1.0;  // NaN/Inf in V itself
      pmax = fmax(pmax, fabs(phi));
      psum = fma(phi, phi, psum);
      if (pi_old && astar != inc) chg += 1.0;
    }
    if (Pp.col) {  // copy the chosen row into the compact P^pi (groups split j)
      const int64_t src = ob + (((int64_t)astar * Kb) << 6) + l;
      const int64_t dst = Pp.off[b] + l;
      for (int j = g; j < Kb; j += G) {
        Pp.col[dst + ((int64_t)j << 6)] = P.col[src + ((int64_t)j << 6)];
        Pp.val[dst + ((int64_t)j << 6)] = P.val[src + ((int64_t)j << 6)];
      }
    }
  }
  double v[4] = {pmax, psum, nonfin, chg};
  const int op[4] = {1, 0, 0, 0};
  block_reduce<4>(v, op);
  if (publish_partials<4>(v, red)) {
    finish_partials<4>(v, op, red);
    if (threadIdx.x == 0) {
      st->phi_inf = v[0];
      st->phi_l2sq = v[1];
      st->nonfinite = (int32_t)v[2];
      st->changes = (int32_t)v[3];
    }
  }
}

// Row sum of the compact P^pi against x*scale, groups split j; the sum is
// complete in every lane of the state after the shuffles.
template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT row_dot(const SellPi<VT>& Pp, int64_t ob, int Kb, int l, int g,
                                      const XT* __restrict__ x, XT scale) {
  constexpr int S = kWave / G;
  AT acc = 0;
  for (int j = g; j < Kb; j += G) {
    const int64_t e = ob + ((int64_t)j << 6) + l;
    const XT xv = x[Pp.col[e]] * scale;
    if constexpr (sizeof(AT) == 8)
      acc = fma(to_d(Pp.val[e]), (AT)xv, acc);
    else
      acc = fmaf(to_f(Pp.val[e]), (AT)xv, acc);
  }
#pragma unroll
  for (int o = S; o < kWave; o <<= 1) acc += __shfl_xor(acc, o);
  return acc;
}

template <typename VT, typename XT, typename AT, int G>
__global__ __launch_bounds__(kBlock) void k_japply(SellPi<VT> Pp, int64_t n, AT gamma,
                                                   const XT* __restrict__ x,
                                                   const double* __restrict__ eta,
                                                   XT* __restrict__ q_out, XT* __restrict__ y) {
  constexpr int S = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int ls = lane % S, g = lane / S;
  const int64_t nw = (n + S - 1) / S;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  const XT scale = eta ? (XT)(1.0 / *eta) : (XT)1;
  for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; w < nw;
       w += wstride) {
    const int64_t s = w * S + ls;
    const int64_t b = s >> 6;
    const int l = (int)(s & 63);
    const AT acc = row_dot<VT, XT, AT, G>(Pp, Pp.off[b], Pp.width[b], l, g, x, scale);
    if (s < n && g == 0) {
      const XT xs = x[s] * scale;
      if (q_out) q_out[s] = xs;
      y[s] = (XT)((AT)xs - gamma * acc);
    }
  }
}

template <typename VT, int G>
__global__ __launch_bounds__(kBlock) void k_residual(SellPi<VT> Pp, int64_t n, double gamma,
                                                     const double* __restrict__ cpi,
                                                     const double* __restrict__ V,
                                                     double* __restrict__ r, RedCtx red,
                                                     DevStatus* __restrict__ st) {
  constexpr int S = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int ls = lane % S, g = lane / S;
  const int64_t nw = (n + S - 1) / S;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  double pmax = 0.0, psum = 0.0, vmax = 0.0;
  for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; w < nw;
       w += wstride) {
    const int64_t s = w * S + ls;
    const int64_t b = s >> 6;
    const int l = (int)(s & 63);
    const double acc =
        row_dot<VT, double, double, G>(Pp, Pp.off[b], Pp.width[b], l, g, V, 1.0);
    if (s < n && g == 0) {
      const double rr = cpi[s] - (V[s] - gamma * acc);
      r[s] = rr;
      pmax = fmax(pmax, fabs(rr));
      psum = fma(rr, rr, psum);
      vmax = fmax(vmax, fabs(V[s]));
    }
  }
  double v[3] = {pmax, psum, vmax};
  const int op[3] = {1, 0, 1};
  block_reduce<3>(v, op);
  if (publish_partials<3>(v, red)) {
    finish_partials<3>(v, op, red);
    if (threadIdx.x == 0) {
      st->res_inf = v[0];
      st->res_l2sq = v[1];
      st->vmax = v[2];
    }
  }
}

template <typename VT, int G>
__global__ __launch_bounds__(kBlock) void k_vi_sweep(SellPi<VT> Pp, int64_t n, double gamma,
                                                     const double* __restrict__ cpi,
                                                     const double* __restrict__ Vin,
                                                     double* __restrict__ Vout, RedCtx red,
                                                     DevStatus* __restrict__ st) {
  constexpr int S = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int ls = lane % S, g = lane / S;
  const int64_t nw = (n + S - 1) / S;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  double pmax = 0.0, psum = 0.0;
  for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; w < nw;
       w += wstride) {
    const int64_t s = w * S + ls;
    const int64_t b = s >> 6;
    const int l = (int)(s & 63);
    const double acc =
        row_dot<VT, double, double, G>(Pp, Pp.off[b], Pp.width[b], l, g, Vin, 1.0);
    if (s < n && g == 0) {
      const double vn = cpi[s] + gamma * acc;
      const double dd = vn - Vin[s];
      Vout[s] = vn;
      pmax = fmax(pmax, fabs(dd));
      psum = fma(dd, dd, psum);
    }
  }
  double v[2] = {pmax, psum};
  const int op[2] = {1, 0};
  block_reduce<2>(v, op);
  if (publish_partials<2>(v, red)) {
    finish_partials<2>(v, op, red);
    if (threadIdx.x == 0) {
      st->aux = v[0];
      st->res_l2sq = v[1];
    }
  }
}

template <typename VT, int G>
__global__ __launch_bounds__(kBlock) void k_gather_policy(SellP<VT> P, SellPi<VT> Pp,
                                                          const double* __restrict__ cost, int m,
                                                          int64_t n, const int32_t* __restrict__ pi,
                                                          double* __restrict__ cpi, RedCtx red,
                                                          DevStatus* __restrict__ st) {
  constexpr int S = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int ls = lane % S, g = lane / S;
  const int64_t nw = (n + S - 1) / S;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  double bad = 0.0;
  for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; w < nw;
       w += wstride) {
    const int64_t s = w * S + ls;
    const bool valid = s < n;
    const int64_t b = s >> 6;
    const int l = (int)(s & 63);
    int a = valid ? pi[s] : 0;
    if (a < 0 || a >= m) {
      if (g == 0) bad += 1.0;
      a = 0;
    }
    const int Kb = P.width[b];
    const int64_t src = P.off[b] + (((int64_t)a * Kb) << 6) + l;
    const int64_t dst = Pp.off[b] + l;
    for (int j = g; j < Kb; j += G) {
      Pp.col[dst + ((int64_t)j << 6)] = P.col[src + ((int64_t)j << 6)];
      Pp.val[dst + ((int64_t)j << 6)] = P.val[src + ((int64_t)j << 6)];
    }
    if (valid && g == 0) cpi[s] = cost[(int64_t)a * n + s];
  }
  double v[1] = {bad};
  const int op[1] = {0};
  block_reduce<1>(v, op);
  if (publish_partials<1>(v, red)) {
    finish_partials<1>(v, op, red);
    if (threadIdx.x == 0) st->changes = (int32_t)v[0];
  }
}

inline int grid_for(const Mdp& d, int G) {
  const int64_t waves = (d.n + (kWave / G) - 1) / (kWave / G);
  const int64_t blocks = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, kMaxBlocks));
}

template <typename VT>
SellP<VT> viewP(Mdp& d) {
  return SellP<VT>{d.col, (const VT*)d.val, d.off, d.width};
}
template <typename VT>
SellPi<VT> viewPi(Mdp& d) {
  return SellPi<VT>{d.pcol, (VT*)d.pval, d.offp, d.width};
}

// dispatch helpers over the storage type and the lanes-per-state count
template <template <typename, int> class F, typename... A>
void dispatch_vt_g(const Mdp& d, int G, A&&... a) {
  switch (d.store) {
#define IG_CASE_G(VT)                                      \
  switch (G) {                                             \
    case 1: F<VT, 1>::run(std::forward<A>(a)...); break;   \
    case 2: F<VT, 2>::run(std::forward<A>(a)...); break;   \
    case 4: F<VT, 4>::run(std::forward<A>(a)...); break;   \
    case 8: F<VT, 8>::run(std::forward<A>(a)...); break;   \
    case 16: F<VT, 16>::run(std::forward<A>(a)...); break; \
    case 32: F<VT, 32>::run(std::forward<A>(a)...); break; \
    default: F<VT, 64>::run(std::forward<A>(a)...); break; \
  }
    case IG_FP64: IG_CASE_G(double) break;
    case IG_FP32: IG_CASE_G(float) break;
    default: IG_CASE_G(bf16) break;
#undef IG_CASE_G
  }
}

template <typename VT, int G>
struct RunBellman {
  static void run(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
                  const int32_t* pi_old, double tie_abs, bool compact, hipStream_t s) {
    SellPi<VT> pp = viewPi<VT>(d);
    if (!compact) pp.col = nullptr;
    hipLaunchKernelGGL((k_bellman<VT, G>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                       viewP<VT>(d), (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi, pi,
                       pi_old, tie_abs, d.cpi, pp, red_ctx(d), d.st);
  }
};

template <typename VT, int G>
struct RunJapply {
  static void run(Mdp& d, bool fp32, const void* x, const double* eta, void* q_out, void* y,
                  hipStream_t s) {
    if (fp32)
      hipLaunchKernelGGL((k_japply<VT, float, float, G>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                         viewPi<VT>(d), d.n, (float)d.gamma, (const float*)x, eta, (float*)q_out,
                         (float*)y);
    else
      hipLaunchKernelGGL((k_japply<VT, double, double, G>), dim3(grid_for(d, G)), dim3(kBlock), 0,
                         s, viewPi<VT>(d), d.n, d.gamma, (const double*)x, eta, (double*)q_out,
                         (double*)y);
  }
};

template <typename VT, int G>
struct RunResidual {
  static void run(Mdp& d, const double* V, double* r, hipStream_t s) {
    hipLaunchKernelGGL((k_residual<VT, G>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                       viewPi<VT>(d), d.n, d.gamma, (const double*)d.cpi, V, r, red_ctx(d), d.st);
  }
};

template <typename VT, int G>
struct RunVi {
  static void run(Mdp& d, const double* Vin, double* Vout, hipStream_t s) {
    hipLaunchKernelGGL((k_vi_sweep<VT, G>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                       viewPi<VT>(d), d.n, d.gamma, (const double*)d.cpi, Vin, Vout, red_ctx(d),
                       d.st);
  }
};

template <typename VT, int G>
struct RunGather {
  static void run(Mdp& d, const int32_t* pi, hipStream_t s) {
    hipLaunchKernelGGL((k_gather_policy<VT, G>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                       viewP<VT>(d), viewPi<VT>(d), (const double*)d.cost, d.m, d.n, pi, d.cpi,
                       red_ctx(d), d.st);
  }
};

}  // namespace

void launch_bellman_sparse(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
                           const int32_t* pi_old, double tie_abs, bool compact, hipStream_t s) {
  ProfScope p(d, KC_BELLMAN, s);
  dispatch_vt_g<RunBellman>(d, d.G_bell, d, V, TV, Phi, pi, pi_old, tie_abs, compact, s);
}

void launch_japply_sparse(Mdp& d, bool fp32, const void* x, const double* eta, void* q_out,
                          void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  dispatch_vt_g<RunJapply>(d, d.G_jap, d, fp32, x, eta, q_out, y, s);
}

void launch_residual_sparse(Mdp& d, const double* V, double* r, hipStream_t s) {
  ProfScope p(d, KC_RESID, s);
  dispatch_vt_g<RunResidual>(d, d.G_jap, d, V, r, s);
}

void launch_vi_sweep_sparse(Mdp& d, const double* Vin, double* Vout, hipStream_t s) {
  ProfScope p(d, KC_VI, s);
  dispatch_vt_g<RunVi>(d, d.G_jap, d, Vin, Vout, s);
}

void launch_gather_policy_sparse(Mdp& d, const int32_t* pi, hipStream_t s) {
  ProfScope p(d, KC_OTHER, s);
  dispatch_vt_g<RunGather>(d, d.G_jap, d, pi, s);
}

}  // namespace ig
