// Streaming kernels for dense transition data P[s][a][s'] (row-major, gfx950).
//
// Bellman pass: one block per state, its four wavefronts split the actions;
// each wavefront streams a whole row with unit-stride lanes and reduces it
// with shuffles; the block picks the (value, action)-lexicographic minimum.
// Products with P^pi: one wavefront per state on row (s, pi(s)).
#include "internal.hpp"

namespace ig {

namespace {

constexpr int kWpb = kBlock / kWave;  // wavefronts per block

template <typename VT, typename XT, typename AT>
__device__ __forceinline__ AT dense_row_dot(const VT* __restrict__ row, int64_t n,
                                            const XT* __restrict__ x, XT scale, int lane) {
  AT acc = 0;
  for (int64_t e = lane; e < n; e += kWave) {
    const XT xv = x[e] * scale;
    if constexpr (sizeof(AT) == 8)
      acc = fma(to_d(row[e]), (AT)xv, acc);
    else
      acc = fmaf(to_f(row[e]), (AT)xv, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  return acc;
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_bellman_dense(
    const VT* __restrict__ P, const double* __restrict__ cost, int m, int64_t n, double gamma,
    const double* __restrict__ V, double* __restrict__ TV, double* __restrict__ Phi,
    int32_t* __restrict__ pi, const int32_t* __restrict__ pi_old, double tie_abs,
    double* __restrict__ cpi, RedCtx red, DevStatus* __restrict__ st) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __shared__ double sb[kWpb], sq[kWpb];
  __shared__ int sa[kWpb];
  double pmax = 0.0, psum = 0.0, nonfin = 0.0, chg = 0.0;
  for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
    const int inc = pi_old ? pi_old[s] : -1;
    double best = INFINITY, qinc = INFINITY;
    int besta = m;
    for (int a = wid; a < m; a += kWpb) {
      const double acc =
          dense_row_dot<VT, double, double>(P + ((int64_t)s * m + a) * n, n, V, 1.0, lane);
      const double q = cost[(int64_t)a * n + s] + gamma * acc;
      if (!(q - q == 0.0)) nonfin += 1.0;
      if (q < best) {
        best = q;
        besta = a;
      }
      if (a == inc) qinc = q;
    }
    if (lane == 0) {
      sb[wid] = best;
      sa[wid] = besta;
      sq[wid] = qinc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      best = sb[0];
      besta = sa[0];
      qinc = sq[0];
      for (int w = 1; w < kWpb; ++w) {
        if (sb[w] < best || (sb[w] == best && sa[w] < besta)) {
          best = sb[w];
          besta = sa[w];
        }
        qinc = fmin(qinc, sq[w]);
      }
      if (besta >= m) {
        besta = 0;
        best = NAN;
      }
      int astar = besta;
      double tv = best;
      if (inc >= 0 && inc < m && qinc <= best + tie_abs) {
        astar = inc;
        tv = qinc;
      }
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
    __syncthreads();
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

// mode 0: y = xs - gamma P^pi xs (+ q_out = xs)
template <typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kBlock) void k_japply_dense(const VT* __restrict__ P, int m,
                                                         int64_t n, AT gamma,
                                                         const int32_t* __restrict__ pi,
                                                         const XT* __restrict__ x,
                                                         const double* __restrict__ eta,
                                                         XT* __restrict__ q_out,
                                                         XT* __restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1);
  const XT scale = eta ? (XT)(1.0 / *eta) : (XT)1;
  for (int64_t s = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; s < n;
       s += (int64_t)gridDim.x * kWpb) {
    const AT acc = dense_row_dot<VT, XT, AT>(P + ((int64_t)s * m + pi[s]) * n, n, x, scale, lane);
    if (lane == 0) {
      const XT xs = x[s] * scale;
      if (q_out) q_out[s] = xs;
      y[s] = (XT)((AT)xs - gamma * acc);
    }
  }
}

// mode 0: residual r = g^pi - (V - gamma P^pi V); mode 1: VI sweep
// Vout = g^pi + gamma P^pi Vin with max|Vout - Vin| into status.aux.
template <typename VT, int MODE>
__global__ __launch_bounds__(kBlock) void k_policy_pass_dense(
    const VT* __restrict__ P, int m, int64_t n, double gamma, const int32_t* __restrict__ pi,
    const double* __restrict__ cpi, const double* __restrict__ V, double* __restrict__ out,
    RedCtx red, DevStatus* __restrict__ st) {
  const int lane = threadIdx.x & (kWave - 1);
  double pmax = 0.0, psum = 0.0, vmax = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; s < n;
       s += (int64_t)gridDim.x * kWpb) {
    const double acc =
        dense_row_dot<VT, double, double>(P + ((int64_t)s * m + pi[s]) * n, n, V, 1.0, lane);
    if (lane == 0) {
      double v;
      if (MODE == 0) {
        v = cpi[s] - (V[s] - gamma * acc);
        out[s] = v;
      } else {
        const double vn = cpi[s] + gamma * acc;
        v = vn - V[s];
        out[s] = vn;
      }
      pmax = fmax(pmax, fabs(v));
      psum = fma(v, v, psum);
      vmax = fmax(vmax, fabs(V[s]));
    }
  }
  double v[3] = {pmax, psum, vmax};
  const int op[3] = {1, 0, 1};
  block_reduce<3>(v, op);
  if (publish_partials<3>(v, red)) {
    finish_partials<3>(v, op, red);
    if (threadIdx.x == 0) {
      if (MODE == 0) {
        st->res_inf = v[0];
        st->res_l2sq = v[1];
        st->vmax = v[2];
      } else {
        st->aux = v[0];
        st->res_l2sq = v[1];
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_gather_dense(const double* __restrict__ cost, int m,
                                                         int64_t n, const int32_t* __restrict__ pi,
                                                         double* __restrict__ cpi, RedCtx red,
                                                         DevStatus* __restrict__ st) {
  double bad = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kBlock) {
    int a = pi[s];
    if (a < 0 || a >= m) {
      bad += 1.0;
      a = 0;
    }
    cpi[s] = cost[(int64_t)a * n + s];
  }
  double v[1] = {bad};
  const int op[1] = {0};
  block_reduce<1>(v, op);
  if (publish_partials<1>(v, red)) {
    finish_partials<1>(v, op, red);
    if (threadIdx.x == 0) st->changes = (int32_t)v[0];
  }
}

inline int grid_states(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(n, kMaxBlocks));
}
inline int grid_waves(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kWpb - 1) / kWpb, kMaxBlocks));
}

template <typename F>
void by_store(const Mdp& d, F&& f) {
  switch (d.store) {
    case IG_FP64: f(double{}); break;
    case IG_FP32: f(float{}); break;
    default: f(bf16{}); break;
  }
}

}  // namespace

void launch_bellman_dense(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
                          const int32_t* pi_old, double tie_abs, hipStream_t s) {
  ProfScope p(d, KC_BELLMAN, s);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    hipLaunchKernelGGL(k_bellman_dense<VT>, dim3(grid_states(d.n)), dim3(kBlock), 0, s,
                       (const VT*)d.P, (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi, pi,
                       pi_old, tie_abs, d.cpi, red_ctx(d), d.st);
  });
}

void launch_japply_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* eta,
                         void* q_out, void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    if (fp32)
      hipLaunchKernelGGL((k_japply_dense<VT, float, float>), dim3(grid_waves(d.n)), dim3(kBlock),
                         0, s, (const VT*)d.P, d.m, d.n, (float)d.gamma, pi, (const float*)x, eta,
                         (float*)q_out, (float*)y);
    else
      hipLaunchKernelGGL((k_japply_dense<VT, double, double>), dim3(grid_waves(d.n)),
                         dim3(kBlock), 0, s, (const VT*)d.P, d.m, d.n, d.gamma, pi,
                         (const double*)x, eta, (double*)q_out, (double*)y);
  });
}

void launch_residual_dense(Mdp& d, const int32_t* pi, const double* V, double* r, hipStream_t s) {
  ProfScope p(d, KC_RESID, s);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    hipLaunchKernelGGL((k_policy_pass_dense<VT, 0>), dim3(grid_waves(d.n)), dim3(kBlock), 0, s,
                       (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)d.cpi, V, r,
                       red_ctx(d), d.st);
  });
}

void launch_vi_sweep_dense(Mdp& d, const int32_t* pi, const double* Vin, double* Vout,
                           hipStream_t s) {
  ProfScope p(d, KC_VI, s);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    hipLaunchKernelGGL((k_policy_pass_dense<VT, 1>), dim3(grid_waves(d.n)), dim3(kBlock), 0, s,
                       (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)d.cpi, Vin, Vout,
                       red_ctx(d), d.st);
  });
}

void launch_gather_policy_dense(Mdp& d, const int32_t* pi, hipStream_t s) {
  ProfScope p(d, KC_OTHER, s);
  hipLaunchKernelGGL(k_gather_dense, dim3(grid_waves(d.n)), dim3(kBlock), 0, s,
                     (const double*)d.cost, d.m, d.n, pi, d.cpi, red_ctx(d), d.st);
}

}  // namespace ig
