// Streaming kernels for dense transition data P[s][a][s'] (row-major, gfx950).
//
// Bellman pass: one block per state, its four wavefronts split the actions;
// each wavefront streams whole rows with 16-byte loads per lane (when the row
// length keeps rows 16-byte aligned), several loads in flight, and reduces
// with shuffles; the block picks the (value, action)-lexicographic minimum.
// Products with P^pi: one wavefront per state on row (s, pi(s)).
#include "internal.hpp"

namespace ig {

namespace {

constexpr int kWpb = kBlock / kWave;  // wavefronts per block

template <typename VT>
struct Vec;  // 16 bytes of stored values
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
template <>
struct Vec<double> {
  static constexpr int N = 2;
  using T = d2v;
  __device__ static double at(const T& v, int k) { return k == 0 ? v.x : v.y; }
};
template <>
struct Vec<float> {
  static constexpr int N = 4;
  using T = f4v;
  __device__ static double at(const T& v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
  }
};
template <>
struct Vec<bf16> {
  static constexpr int N = 8;
  using T = u4v;
  __device__ static double at(const T& v, int k) {
    const unsigned w = k < 2 ? v.x : k < 4 ? v.y : k < 6 ? v.z : v.w;
    const unsigned bits = (k & 1) ? (w & 0xFFFF0000u) : (w << 16);
    return (double)__uint_as_float(bits);
  }
};
// 16-byte load of the row stream (a plain load: a non-temporal hint measured
// slower on the dense rows)
template <typename VV>
__device__ __forceinline__ VV ldv(const VV* p) { return *p; }

// sum_e row[e] * x[e] * scale over one row of length n, the whole wavefront
// cooperating; AT is the accumulation type.  Result valid in every lane.
template <typename VT, typename XT, typename AT>
__device__ __forceinline__ AT dense_row_dot(const VT* __restrict__ row, int64_t n,
                                            const XT* __restrict__ x, XT scale, int lane,
                                            bool vec_ok) {
  AT acc = 0;
  if (vec_ok) {
    constexpr int N = Vec<VT>::N;
    using VV = typename Vec<VT>::T;
    const VV* rv = reinterpret_cast<const VV*>(row);
    const int64_t nv = n / N;
    int64_t e = lane;
    for (; e + 3 * kWave < nv; e += 4 * kWave) {  // four 16-byte loads in flight per lane
      const VV p0 = ldv(rv + e), p1 = ldv(rv + e + kWave), p2 = ldv(rv + e + 2 * kWave),
               p3 = ldv(rv + e + 3 * kWave);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        acc += (AT)Vec<VT>::at(p0, k) * (AT)(x[e * N + k] * scale);
        acc += (AT)Vec<VT>::at(p1, k) * (AT)(x[(e + kWave) * N + k] * scale);
        acc += (AT)Vec<VT>::at(p2, k) * (AT)(x[(e + 2 * kWave) * N + k] * scale);
        acc += (AT)Vec<VT>::at(p3, k) * (AT)(x[(e + 3 * kWave) * N + k] * scale);
      }
    }
    for (; e < nv; e += kWave) {
      const VV p0 = ldv(rv + e);
#pragma unroll
      for (int k = 0; k < N; ++k) acc += (AT)Vec<VT>::at(p0, k) * (AT)(x[e * N + k] * scale);
    }
  } else {
    for (int64_t e = lane; e < n; e += kWave) {
      const XT xv = x[e] * scale;
      if constexpr (sizeof(AT) == 8)
        acc = fma(to_d(row[e]), (AT)xv, acc);
      else
        acc = fmaf(to_f(row[e]), (AT)xv, acc);
    }
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
    double* __restrict__ cpi, double* __restrict__ part, bool vec_ok,
    const uint8_t* __restrict__ adm) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __shared__ double sb[kWpb], sq[kWpb];
  __shared__ int sa[kWpb];
  double pmax = 0.0, psum = 0.0, nonfin = 0.0, chg = 0.0;
  for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
    const int inc = pi_old ? pi_old[s] : -1;
    double best = INFINITY, qinc = INFINITY;
    int besta = m;
    for (int a = wid; a < m; a += kWpb) {
      if (adm && !adm[(int64_t)a * n + s]) continue;  // a is not in A(s)
      const double acc = dense_row_dot<VT, double, double>(P + ((int64_t)s * m + a) * n, n, V, 1.0,
                                                           lane, vec_ok);
      const double q = cost[(int64_t)a * n + s] + gamma * acc;
      if (!(q - q == 0.0)) nonfin += lane == 0 ? 1.0 : 0.0;
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
  store_partials<4>(v, op, part);
}

template <typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kBlock) void k_japply_dense(const VT* __restrict__ P, int m,
                                                         int64_t n, AT gamma,
                                                         const int32_t* __restrict__ pi,
                                                         const XT* __restrict__ x,
                                                         const double* __restrict__ eta,
                                                         XT* __restrict__ y, bool vec_ok) {
  const int lane = threadIdx.x & (kWave - 1);
  const XT scale = eta ? (XT)(1.0 / *eta) : (XT)1;
  for (int64_t s = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; s < n;
       s += (int64_t)gridDim.x * kWpb) {
    const AT acc = dense_row_dot<VT, XT, AT>(P + ((int64_t)s * m + pi[s]) * n, n, x, scale, lane,
                                             vec_ok);
    if (lane == 0) {
      const XT xs = x[s] * scale;
      y[s] = (XT)((AT)xs - gamma * acc);
    }
  }
}

// Horner step of the Neumann preconditioner: y = x * sx + gamma * (P^pi z) * sz
template <typename VT, typename XT, typename AT>
__global__ __launch_bounds__(kBlock) void k_pstep_dense(const VT* __restrict__ P, int m,
                                                        int64_t n, AT gamma,
                                                        const int32_t* __restrict__ pi,
                                                        const XT* __restrict__ x,
                                                        const double* __restrict__ sx,
                                                        const XT* __restrict__ z,
                                                        const double* __restrict__ sz,
                                                        XT* __restrict__ y, bool vec_ok) {
  const int lane = threadIdx.x & (kWave - 1);
  const AT ax = sx ? (AT)(1.0 / *sx) : (AT)1, az = sz ? (AT)(1.0 / *sz) : (AT)1;
  for (int64_t s = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; s < n;
       s += (int64_t)gridDim.x * kWpb) {
    const AT acc = dense_row_dot<VT, XT, AT>(P + ((int64_t)s * m + pi[s]) * n, n, z, (XT)1, lane,
                                             vec_ok);
    if (lane == 0) y[s] = (XT)((AT)x[s] * ax + gamma * acc * az);
  }
}

// MODE 0: residual r = g^pi - (V - gamma P^pi V); MODE 1: VI sweep
// Vout = g^pi + gamma P^pi Vin.  Partials {max|.|, ||.||^2, max|V| (MODE 0)}.
template <typename VT, int MODE>
__global__ __launch_bounds__(kBlock) void k_policy_pass_dense(
    const VT* __restrict__ P, int m, int64_t n, double gamma, const int32_t* __restrict__ pi,
    const double* __restrict__ cpi, const double* __restrict__ V, double* __restrict__ out,
    double* __restrict__ part, bool vec_ok) {
  const int lane = threadIdx.x & (kWave - 1);
  double pmax = 0.0, psum = 0.0, vmax = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; s < n;
       s += (int64_t)gridDim.x * kWpb) {
    const double acc = dense_row_dot<VT, double, double>(P + ((int64_t)s * m + pi[s]) * n, n, V,
                                                         1.0, lane, vec_ok);
    if (lane == 0) {
      double v;
      if (MODE == 0) {
        v = cpi[s] - (V[s] - gamma * acc);
        out[s] = v;
        vmax = fmax(vmax, fabs(V[s]));
      } else {
        const double vn = cpi[s] + gamma * acc;
        v = vn - V[s];
        out[s] = vn;
      }
      pmax = fmax(pmax, fabs(v));
      psum = fma(v, v, psum);
    }
  }
  double v[3] = {pmax, psum, vmax};
  const int op[3] = {1, 0, 1};
  store_partials<3>(v, op, part);
}

__global__ __launch_bounds__(kBlock) void k_gather_dense(const double* __restrict__ cost, int m,
                                                         int64_t n, const int32_t* __restrict__ pi,
                                                         const uint8_t* __restrict__ adm,
                                                         double* __restrict__ cpi,
                                                         double* __restrict__ part) {
  double bad = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kBlock) {
    int a = pi[s];
    if (a < 0 || a >= m || (adm && !adm[(int64_t)a * n + s])) {  // not in A(s)
      bad += 1.0;
      a = 0;
    }
    cpi[s] = cost[(int64_t)a * n + s];
  }
  double v[1] = {bad};
  const int op[1] = {0};
  store_partials<1>(v, op, part);
}

inline int grid_states(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(n, kMaxBlocks));
}
inline int grid_waves(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kWpb - 1) / kWpb, kMaxBlocks));
}
inline int grid_threads(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxBlocks));
}
// rows of n stored values stay 16-byte aligned
inline bool vec_ok(const Mdp& d) { return (d.n * d.vb) % 16 == 0; }

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
  {
    ProfScope p(d, KC_BELLMAN, s);
    by_store(d, [&](auto t) {
      using VT = decltype(t);
      hipLaunchKernelGGL(k_bellman_dense<VT>, dim3(grid_states(d.n)), dim3(kBlock), 0, s,
                         (const VT*)d.P, (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi, pi,
                         pi_old, tie_abs, d.cpi, d.part, vec_ok(d), (const uint8_t*)d.adm);
    });
  }
  launch_finalize(d, FIN_BELLMAN, grid_states(d.n), s);
}

void launch_japply_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* eta,
                         void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    if (fp32)
      hipLaunchKernelGGL((k_japply_dense<VT, float, float>), dim3(grid_waves(d.n)), dim3(kBlock),
                         0, s, (const VT*)d.P, d.m, d.n, (float)d.gamma, pi, (const float*)x, eta,
                         (float*)y, vec_ok(d));
    else
      hipLaunchKernelGGL((k_japply_dense<VT, double, double>), dim3(grid_waves(d.n)),
                         dim3(kBlock), 0, s, (const VT*)d.P, d.m, d.n, d.gamma, pi,
                         (const double*)x, eta, (double*)y, vec_ok(d));
  });
}

void launch_pstep_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* sx,
                        const void* z, const double* sz, void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    if (fp32)
      hipLaunchKernelGGL((k_pstep_dense<VT, float, float>), dim3(grid_waves(d.n)), dim3(kBlock), 0,
                         s, (const VT*)d.P, d.m, d.n, (float)d.gamma, pi, (const float*)x, sx,
                         (const float*)z, sz, (float*)y, vec_ok(d));
    else
      hipLaunchKernelGGL((k_pstep_dense<VT, double, double>), dim3(grid_waves(d.n)), dim3(kBlock),
                         0, s, (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)x, sx,
                         (const double*)z, sz, (double*)y, vec_ok(d));
  });
}

void launch_residual_dense(Mdp& d, const int32_t* pi, const double* V, double* r, hipStream_t s) {
  {
    ProfScope p(d, KC_RESID, s);
    by_store(d, [&](auto t) {
      using VT = decltype(t);
      hipLaunchKernelGGL((k_policy_pass_dense<VT, 0>), dim3(grid_waves(d.n)), dim3(kBlock), 0, s,
                         (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)d.cpi, V, r, d.part,
                         vec_ok(d));
    });
  }
  launch_finalize(d, FIN_RESID, grid_waves(d.n), s);
}

void launch_vi_sweep_dense(Mdp& d, const int32_t* pi, const double* Vin, double* Vout,
                           hipStream_t s) {
  {
    ProfScope p(d, KC_VI, s);
    by_store(d, [&](auto t) {
      using VT = decltype(t);
      hipLaunchKernelGGL((k_policy_pass_dense<VT, 1>), dim3(grid_waves(d.n)), dim3(kBlock), 0, s,
                         (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)d.cpi, Vin, Vout,
                         d.part, vec_ok(d));
    });
  }
  launch_finalize(d, FIN_VI, grid_waves(d.n), s);
}

void launch_gather_policy_dense(Mdp& d, const int32_t* pi, hipStream_t s) {
  {
    ProfScope p(d, KC_OTHER, s);
    hipLaunchKernelGGL(k_gather_dense, dim3(grid_threads(d.n)), dim3(kBlock), 0, s,
                       (const double*)d.cost, d.m, d.n, pi, (const uint8_t*)d.adm, d.cpi, d.part);
  }
  launch_finalize(d, FIN_GATHER, grid_threads(d.n), s);
}

}  // namespace ig
