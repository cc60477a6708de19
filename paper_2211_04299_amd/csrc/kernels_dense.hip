// Streaming kernels for dense transition data P[s][a][s'] (row-major, gfx950).
//
// Bellman pass: one block per state, its four wavefronts split the actions;
// each wavefront streams whole rows with 16-byte loads per lane (when the row
// length keeps rows 16-byte aligned), several loads in flight, and reduces
// with shuffles; the block picks the (value, action)-lexicographic minimum.
// Products with P^pi: one wavefront per state on row (s, pi(s)).
#include <mutex>
#include <type_traits>
#include <unordered_map>

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
// 16-byte load of the row stream
template <typename VV>
__device__ __forceinline__ VV ldv(const VV* p) { return *p; }
// the same with a non-temporal hint (rows read once per pass)
template <typename VV>
__device__ __forceinline__ VV ldv_nt(const VV* p) { return __builtin_nontemporal_load(p); }

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
      const VV p0 = ldv_nt(rv + e), p1 = ldv_nt(rv + e + kWave), p2 = ldv_nt(rv + e + 2 * kWave),
               p3 = ldv_nt(rv + e + 3 * kWave);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        acc += (AT)Vec<VT>::at(p0, k) * (AT)(x[e * N + k] * scale);
        acc += (AT)Vec<VT>::at(p1, k) * (AT)(x[(e + kWave) * N + k] * scale);
        acc += (AT)Vec<VT>::at(p2, k) * (AT)(x[(e + 2 * kWave) * N + k] * scale);
        acc += (AT)Vec<VT>::at(p3, k) * (AT)(x[(e + 3 * kWave) * N + k] * scale);
      }
    }
    for (; e < nv; e += kWave) {
      const VV p0 = ldv_nt(rv + e);
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

// Bellman pass with one wavefront on SGB states at once: their action rows
// are streamed RG actions at a time (SGB * RG rows, U 16-byte loads per row
// and lane in flight) against a single load of V per element, which every
// row of the group shares.  Each row's dot product is accumulated in the
// same order as dense_row_dot, and each state's actions are visited in
// increasing order (lowest index wins ties), as in k_bellman_dense.  Rows
// must be 16-byte aligned (vec_ok).
template <typename VT, int SGB, int RG, int U>
__global__ __launch_bounds__(kBlock) void k_bellman_dense4(
    const VT* __restrict__ P, const double* __restrict__ cost, int m, int64_t n, double gamma,
    const double* __restrict__ V, double* __restrict__ TV, double* __restrict__ Phi,
    int32_t* __restrict__ pi, const int32_t* __restrict__ pi_old, double tie_abs,
    double* __restrict__ cpi, double* __restrict__ part, const uint8_t* __restrict__ adm) {
  constexpr int N = Vec<VT>::N;
  constexpr int R = SGB * RG;  // rows in flight: row q is action a0 + q % RG of state s0 + q / RG
  using VV = typename Vec<VT>::T;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nv = n / N;
  const int64_t ng = (n + SGB - 1) / SGB;
  double pmax = 0.0, psum = 0.0, nonfin = 0.0, chg = 0.0;
  for (int64_t gI = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; gI < ng;
       gI += (int64_t)gridDim.x * kWpb) {
    const int64_t s0 = gI * SGB;
    int inc[SGB], besta[SGB];
    double best[SGB], qinc[SGB];
#pragma unroll
    for (int j = 0; j < SGB; ++j) {
      const int64_t s = s0 + j < n ? s0 + j : s0;
      inc[j] = pi_old ? pi_old[s] : -1;
      best[j] = INFINITY;
      qinc[j] = INFINITY;
      besta[j] = m;
    }
    for (int a0 = 0; a0 < m; a0 += RG) {
      bool use[R];
      const VV* rv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int j = q / RG, a = a0 + q % RG;
        const bool sv = s0 + j < n;
        const int64_t s = sv ? s0 + j : s0;
        use[q] = sv && a < m && (!adm || adm[(int64_t)a * n + s]);
        // an unused slot re-reads row (s, a0) (in cache) and is dropped
        rv[q] = reinterpret_cast<const VV*>(P + ((int64_t)s * m + (a < m ? a : a0)) * n);
      }
      double acc[R];
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = 0.0;
      int64_t e = lane;
      for (; e + (U - 1) * kWave < nv; e += U * kWave) {
        VV p[R][U];
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) p[q][u] = ldv_nt(rv[q] + e + u * kWave);
#pragma unroll
        for (int k = 0; k < N; ++k) {
          double x[U];
#pragma unroll
          for (int u = 0; u < U; ++u) x[u] = V[(e + u * kWave) * N + k];
#pragma unroll
          for (int q = 0; q < R; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[q] += Vec<VT>::at(p[q][u], k) * x[u];
        }
      }
      for (; e < nv; e += kWave) {
        VV p[R];
#pragma unroll
        for (int q = 0; q < R; ++q) p[q] = ldv_nt(rv[q] + e);
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double x0 = V[e * N + k];
#pragma unroll
          for (int q = 0; q < R; ++q) acc[q] += Vec<VT>::at(p[q], k) * x0;
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if (!use[q]) continue;
        const int j = q / RG, a = a0 + q % RG;
        const double qv = cost[(int64_t)a * n + s0 + j] + gamma * acc[q];
        if (!(qv - qv == 0.0)) nonfin += lane == 0 ? 1.0 : 0.0;
        if (qv < best[j]) {
          best[j] = qv;
          besta[j] = a;
        }
        if (a == inc[j]) qinc[j] = qv;
      }
    }
#pragma unroll
    for (int j = 0; j < SGB; ++j) {
      const int64_t s = s0 + j;
      if (lane != 0 || s >= n) continue;
      int bj = besta[j];
      double bv = best[j];
      if (bj >= m) {
        bj = 0;
        bv = NAN;
      }
      int astar = bj;
      double tv = bv;
      if (inc[j] >= 0 && inc[j] < m && qinc[j] <= bv + tie_abs) {
        astar = inc[j];
        tv = qinc[j];
      }
      const double phi = tv - V[s];
      if (TV) TV[s] = tv;
      Phi[s] = phi;
      pi[s] = astar;
      cpi[s] = cost[(int64_t)astar * n + s];
      if (!(phi - phi == 0.0)) nonfin += 1.0;  // NaN/Inf in V itself
      pmax = fmax(pmax, fabs(phi));
      psum = fma(phi, phi, psum);
      if (pi_old && astar != inc[j]) chg += 1.0;
    }
  }
  double v[4] = {pmax, psum, nonfin, chg};
  const int op[4] = {1, 0, 0, 0};
  store_partials<4>(v, op, part);
}

// Dot products of SG rows (16-byte aligned, length n) with x * scale, the
// whole wavefront cooperating, U 16-byte loads per row and lane in flight
// and one load of x per element for all SG rows.  Each row is accumulated
// in the order of dense_row_dot; results valid in every lane.
template <typename VT, typename XT, typename AT, int SG, int U>
__device__ __forceinline__ void group_dot(const typename Vec<VT>::T* const (&rv)[SG], int64_t n,
                                          const XT* __restrict__ x, XT scale, int lane,
                                          AT (&acc)[SG]) {
  constexpr int N = Vec<VT>::N;
  using VV = typename Vec<VT>::T;
  const int64_t nv = n / N;
#pragma unroll
  for (int r = 0; r < SG; ++r) acc[r] = 0;
  int64_t e = lane;
  for (; e + (U - 1) * kWave < nv; e += U * kWave) {
    VV p[SG][U];
#pragma unroll
    for (int r = 0; r < SG; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) p[r][u] = ldv_nt(rv[r] + e + u * kWave);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      AT xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = (AT)(x[(e + u * kWave) * N + k] * scale);
#pragma unroll
      for (int r = 0; r < SG; ++r)
#pragma unroll
        for (int u = 0; u < U; ++u) acc[r] += (AT)Vec<VT>::at(p[r][u], k) * xv[u];
    }
  }
  for (; e < nv; e += kWave) {
    VV p[SG];
#pragma unroll
    for (int r = 0; r < SG; ++r) p[r] = ldv_nt(rv[r] + e);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const AT xv = (AT)(x[e * N + k] * scale);
#pragma unroll
      for (int r = 0; r < SG; ++r) acc[r] += (AT)Vec<VT>::at(p[r], k) * xv;
    }
  }
#pragma unroll
  for (int r = 0; r < SG; ++r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o);
  }
}

// rows (s, pi(s)) of SG consecutive states; past the end, row s0 repeated
template <typename VT, int SG>
__device__ __forceinline__ void policy_rows(const VT* __restrict__ P, int m, int64_t n,
                                            const int32_t* __restrict__ pi, int64_t s0,
                                            const typename Vec<VT>::T* (&rv)[SG]) {
#pragma unroll
  for (int r = 0; r < SG; ++r) {
    const int64_t s = s0 + r < n ? s0 + r : s0;
    rv[r] = reinterpret_cast<const typename Vec<VT>::T*>(P + ((int64_t)s * m + pi[s]) * n);
  }
}

// y = x - gamma P^pi x with one wavefront on SG states at once (group_dot).
template <typename VT, typename XT, typename AT, int SG, int U>
__global__ __launch_bounds__(kBlock) void k_japply_dense_g(const VT* __restrict__ P, int m,
                                                           int64_t n, AT gamma,
                                                           const int32_t* __restrict__ pi,
                                                           const XT* __restrict__ x,
                                                           const double* __restrict__ eta,
                                                           XT* __restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1);
  const XT scale = eta ? (XT)(1.0 / *eta) : (XT)1;
  const int64_t ng = (n + SG - 1) / SG;
  for (int64_t gI = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; gI < ng;
       gI += (int64_t)gridDim.x * kWpb) {
    const int64_t s0 = gI * SG;
    const typename Vec<VT>::T* rv[SG];
    policy_rows<VT, SG>(P, m, n, pi, s0, rv);
    AT acc[SG];
    group_dot<VT, XT, AT, SG, U>(rv, n, x, scale, lane, acc);
    if (lane < SG && s0 + lane < n) {
      AT a = acc[0];
#pragma unroll
      for (int r = 1; r < SG; ++r) a = lane == r ? acc[r] : a;
      const int64_t s = s0 + lane;
      const XT xs = x[s] * scale;
      y[s] = (XT)((AT)xs - gamma * a);
    }
  }
}

// The FP64 residual r = g^pi - J V (MODE 0, with ||V||_inf) or the policy
// sweep T^pi V (MODE 1) on SG states per wavefront (group_dot).
template <typename VT, int MODE, int SG, int U>
__global__ __launch_bounds__(kBlock) void k_policy_pass_dense_g(
    const VT* __restrict__ P, int m, int64_t n, double gamma, const int32_t* __restrict__ pi,
    const double* __restrict__ cpi, const double* __restrict__ V, double* __restrict__ out,
    double* __restrict__ part) {
  const int lane = threadIdx.x & (kWave - 1);
  double pmax = 0.0, psum = 0.0, vmax = 0.0;
  const int64_t ng = (n + SG - 1) / SG;
  for (int64_t gI = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave; gI < ng;
       gI += (int64_t)gridDim.x * kWpb) {
    const int64_t s0 = gI * SG;
    const typename Vec<VT>::T* rv[SG];
    policy_rows<VT, SG>(P, m, n, pi, s0, rv);
    double acc[SG];
    group_dot<VT, double, double, SG, U>(rv, n, V, 1.0, lane, acc);
    if (lane < SG && s0 + lane < n) {
      double a = acc[0];
#pragma unroll
      for (int r = 1; r < SG; ++r) a = lane == r ? acc[r] : a;
      const int64_t s = s0 + lane;
      double v;
      if (MODE == 0) {
        v = cpi[s] - (V[s] - gamma * a);
        out[s] = v;
        vmax = fmax(vmax, fabs(V[s]));
      } else {
        const double vn = cpi[s] + gamma * a;
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
// One wavefront per state in equal rounds: ceil(n / rounds) wavefronts,
// with the fewest rounds for which all of them are resident at once
// (`resident` blocks), so that no wave starts a late, mostly idle round.
inline int grid_rounds(int64_t n, int resident) {
  const int64_t cap = (int64_t)std::min(std::max(1, resident), kMaxBlocks) * kWpb;
  const int64_t rounds = (n + cap - 1) / cap;
  const int64_t waves = (n + rounds - 1) / rounds;
  return (int)std::max<int64_t>(1, (waves + kWpb - 1) / kWpb);
}

// blocks of a kernel resident on the whole device (the per-CU occupancy
// query is made once per kernel)
template <typename K>
int resident_blocks(const Mdp& d, K kern) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> per_cu_of;
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = per_cu_of.find((const void*)kern);
    if (it != per_cu_of.end()) {
      per_cu = it->second;
    } else {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
      }
      per_cu_of[(const void*)kern] = per_cu;
    }
  }
  return std::max(1, per_cu) * std::max(1, d.num_cu);
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
  int nb = grid_states(d.n);
  {
    ProfScope p(d, KC_BELLMAN, s);
    by_store(d, [&](auto t) {
      using VT = decltype(t);
      if (vec_ok(d)) {
        auto go = [&](auto kern, int sgb) {
          nb = grid_rounds((d.n + sgb - 1) / sgb, resident_blocks(d, kern));
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, s, (const VT*)d.P,
                             (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi, pi, pi_old,
                             tie_abs, d.cpi, d.part, (const uint8_t*)d.adm);
        };
        // FP64/FP32: two states, four actions each, two loads per row and
        // lane in flight (the best of 1-8 states x 1-4 actions x 1-4 loads
        // measured on c3: 264 against 322 us for one state x four actions x
        // four loads).  BF16, whose 16-byte loads carry eight values to widen
        // each: four states x four actions, one load per row (157 against
        // 172 us on c3; FP32 and FP64 are slower that way)
        if constexpr (std::is_same<VT, bf16>::value)
          go(k_bellman_dense4<VT, 4, 4, 1>, 4);
        else
          go(k_bellman_dense4<VT, 2, 4, 2>, 2);
      } else
        hipLaunchKernelGGL(k_bellman_dense<VT>, dim3(grid_states(d.n)), dim3(kBlock), 0, s,
                           (const VT*)d.P, (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi,
                           pi, pi_old, tie_abs, d.cpi, d.part, false, (const uint8_t*)d.adm);
    });
  }
  launch_finalize(d, FIN_BELLMAN, nb, s);
}

void launch_japply_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* eta,
                         void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  InnerView iv(d);
  by_store(d, [&](auto t) {
    using VT = decltype(t);
    auto go = [&](auto kern, auto xt, int sg) {
      using X = decltype(xt);
      const int nb = grid_rounds((d.n + sg - 1) / sg, resident_blocks(d, kern));
      hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, s, (const VT*)d.P, d.m, d.n,
                         (X)d.gamma, pi, (const X*)x, eta, (X*)y);
    };
    // two states per wavefront, four loads per row and lane in flight (the
    // best of 1-4 states x 2-4 loads measured on c3)
    if (!vec_ok(d)) {
      if (fp32)
        hipLaunchKernelGGL((k_japply_dense<VT, float, float>), dim3(grid_waves(d.n)), dim3(kBlock),
                           0, s, (const VT*)d.P, d.m, d.n, (float)d.gamma, pi, (const float*)x, eta,
                           (float*)y, false);
      else
        hipLaunchKernelGGL((k_japply_dense<VT, double, double>), dim3(grid_waves(d.n)),
                           dim3(kBlock), 0, s, (const VT*)d.P, d.m, d.n, d.gamma, pi,
                           (const double*)x, eta, (double*)y, false);
    } else if (fp32) {
      // BF16 rows: four states, one load per row and lane (1.22 against
      // 1.39 ms per three c3 solves)
      if constexpr (std::is_same<VT, bf16>::value)
        go(k_japply_dense_g<VT, float, float, 4, 1>, float{}, 4);
      else
        go(k_japply_dense_g<VT, float, float, 2, 4>, float{}, 2);
    } else {
      go(k_japply_dense_g<VT, double, double, 2, 4>, double{}, 2);
    }
  });
}

void launch_pstep_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* sx,
                        const void* z, const double* sz, void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  InnerView iv(d);
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
  int nb = grid_waves(d.n);
  {
    ProfScope p(d, KC_RESID, s);
    by_store(d, [&](auto t) {
      using VT = decltype(t);
      if (vec_ok(d)) {
        // four states per wavefront; with FP32 or BF16 rows one load per row
        // and lane (c3: 0.71 against 0.77 ms per three solves for FP32, 0.43
        // against 0.54 for BF16), four with FP64 rows
        auto go = [&](auto kern) {
          nb = grid_rounds((d.n + 3) / 4, resident_blocks(d, kern));
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, s, (const VT*)d.P, d.m, d.n,
                             d.gamma, pi, (const double*)d.cpi, V, r, d.part);
        };
        if constexpr (std::is_same<VT, double>::value)
          go(k_policy_pass_dense_g<VT, 0, 4, 4>);
        else
          go(k_policy_pass_dense_g<VT, 0, 4, 1>);
      } else {
        hipLaunchKernelGGL((k_policy_pass_dense<VT, 0>), dim3(nb), dim3(kBlock), 0, s,
                           (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)d.cpi, V, r,
                           d.part, false);
      }
    });
  }
  launch_finalize(d, FIN_RESID, nb, s);
}

void launch_vi_sweep_dense(Mdp& d, const int32_t* pi, const double* Vin, double* Vout,
                           hipStream_t s, bool finish) {
  int nb = grid_waves(d.n);
  {
    ProfScope p(d, KC_VI, s);
    by_store(d, [&](auto t) {
      using VT = decltype(t);
      if (vec_ok(d)) {
        // the shapes of the FP64 residual above
        auto go = [&](auto kern) {
          nb = grid_rounds((d.n + 3) / 4, resident_blocks(d, kern));
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, s, (const VT*)d.P, d.m, d.n,
                             d.gamma, pi, (const double*)d.cpi, Vin, Vout, d.part);
        };
        if constexpr (std::is_same<VT, double>::value)
          go(k_policy_pass_dense_g<VT, 1, 4, 4>);
        else
          go(k_policy_pass_dense_g<VT, 1, 4, 1>);
      } else {
        hipLaunchKernelGGL((k_policy_pass_dense<VT, 1>), dim3(nb), dim3(kBlock), 0, s,
                           (const VT*)d.P, d.m, d.n, d.gamma, pi, (const double*)d.cpi, Vin, Vout,
                           d.part, false);
      }
    });
  }
  if (finish) launch_finalize(d, FIN_VI, nb, s);
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
