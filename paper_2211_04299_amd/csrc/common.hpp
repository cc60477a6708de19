// Internal definitions shared by the HIP sources of libigmres (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/igmres.h"

namespace ig {

// ---------------------------------------------------------------------------
// storage types
// ---------------------------------------------------------------------------
struct bf16 {
  uint16_t bits;
};

// Streaming loads of transition data, which is read once per pass: the
// non-temporal hint keeps it from displacing the reused vectors (V, x) that
// the gathers hit in L2.
__device__ __forceinline__ int32_t ld_stream(const int32_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ bf16 ld_stream(const bf16* p) {
  return bf16{__builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p))};
}

__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return (double)x; }
__device__ __forceinline__ double to_d(bf16 x) {
  return (double)__uint_as_float(((uint32_t)x.bits) << 16);
}
__device__ __forceinline__ float to_f(double x) { return (float)x; }
__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(bf16 x) { return __uint_as_float(((uint32_t)x.bits) << 16); }

template <typename T>
__device__ __forceinline__ T from_d(double x);
template <>
__device__ __forceinline__ double from_d<double>(double x) { return x; }
template <>
__device__ __forceinline__ float from_d<float>(double x) { return (float)x; }

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kBlock = 256;     // threads per block for every kernel
constexpr int kSlice = 64;      // states per ELL slice
constexpr int kMaxBlocks = 2048;   // grid cap of the streaming kernels
constexpr int kGsBlocks = 512;     // grid cap of the Gram-Schmidt kernels
constexpr int kMaxW = IG_MAX_RESTART;

// ---------------------------------------------------------------------------
// sliced ELL views.  Slice b (states 64b .. 64b+63) has width K_b.
//   full P:     entry (a, j, l) at off[b] + ((a*K_b + j) << 6) + l
//   compact P^pi entry (j, l) at offp[b] + (j << 6) + l
// Padding entries have column 0 and value 0.  The full P and the compact
// P^pi arrays carry kRowPad zero entries after the last slice, so a
// wavefront may read 16 whole slots of any row (see k_bellman, row_whole).
constexpr int64_t kRowPad = 16 * 64;
// ---------------------------------------------------------------------------
template <typename VT>
struct SellP {
  const int32_t* __restrict__ col;
  const VT* __restrict__ val;
  const int64_t* __restrict__ off;   // [nslices]
  const int32_t* __restrict__ width; // [nslices]
  const int32_t* __restrict__ mcnt;  // [nslices] action blocks stored for the slice
  const uint8_t* __restrict__ adm;   // [m][n] admissibility, or null (all admissible)
};

template <typename VT>
struct SellPi {
  int32_t* __restrict__ col;
  VT* __restrict__ val;
  const int64_t* __restrict__ off;   // [nslices]
  const int32_t* __restrict__ width; // [nslices]
};

// ---------------------------------------------------------------------------
// device-side scalar state of a solve (one per handle)
// ---------------------------------------------------------------------------
struct DevStatus {
  double phi_inf;     // Bellman pass: ||T V - V||_inf
  double phi_l2sq;    //               ||T V - V||_2^2
  double res_inf;     // explicit residual ||g - J V||_inf
  double res_l2sq;    //                   ||g - J V||_2^2
  double eta;         // last Arnoldi step: ||q||_2 after orthogonalisation
  double rho;         // |g_hat(i+1)| = residual 2-norm of the LSQ problem
  double beta;        // 2-norm of the residual that started the cycle
  double aux;         // kernel-specific scalar (e.g. VI sweep difference)
  double vmax;        // ||V||_inf seen by the last residual pass
  double res_impl;    // ||Q z||_inf: residual of the previous column's iterate
  int32_t nonfinite;  // NaN/Inf seen in the last Bellman pass
  int32_t changes;    // policy entries changed by the last improvement
  uint32_t arrive;    // blocks of the running Gram-Schmidt pass that finished (reset by the last)
  uint32_t pad_;
};

// What the host needs after each Arnoldi step of the stream engine, written
// by the step's last kernel straight into pinned host memory (so the host
// can read it while the next product already runs on the stream).
struct StepSnap {
  double eta, rho, res_impl;
};

struct GivensState {
  double R[(kMaxW + 1) * kMaxW];  // column-major, leading dim kMaxW+1
  double cs[kMaxW];
  double sn[kMaxW];
  double g[kMaxW + 1];
  double h[kMaxW + 1];   // current Hessenberg column (first CGS pass, then h1 + h2)
  double h2[kMaxW + 1];  // second CGS pass coefficients (applied lazily)
  double y[kMaxW];       // least-squares solution of the current cycle
  double z[kMaxW + 2];   // residual of the LSQ problem in basis coordinates
};

// Control block of one persistent (single-launch) solve.  Zeroed before the
// launch; the block that arrives last at a grid barrier reduces the
// per-block partials, publishes the scalars below and releases the barrier.
struct PCtl {
  unsigned int count;  // arrivals at the current barrier
  unsigned int gen;    // barrier generation
  int32_t err;         // 1: a barrier wait exceeded its spin limit
  int32_t dec;         // decision published by the reducer
  double thr, inv_beta, inv_eta, eta, rho, cycle_beta;
  double phi_inf, phi_l2sq, res_inf, res_l2sq, vmax;
  double alg_bytes;
  int32_t outer, inner, restarts, expl, breakdowns, stagnations, converged, bellman;
  int32_t steps_outer, breakdown_flag, restart_req, nonfinite;
};

// Reduction context: per-block partials of the last finishing kernel.
struct RedCtx {
  double* part;  // [gridDim.x * nv]
};

// ---------------------------------------------------------------------------
// wave / block reductions (deterministic: fixed shuffle and LDS order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// op: 0 = sum, 1 = max.  Result valid in thread 0.  NT: threads per block.
template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&op)[NV]) {
  __shared__ double sh[NV][NT / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = op[k] ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double a = sh[k][0];
      for (int w = 1; w < NT / kWave; ++w) a = op[k] ? fmax(a, sh[k][w]) : a + sh[k][w];
      v[k] = a;
    }
  }
  __syncthreads();
}

// Block partials for a finishing kernel: block_reduce, then thread 0 stores
// the NV values at part[blockIdx.x * NV + k].  The reduction over blocks is
// done by a one-block kernel launched next on the same stream (the kernel
// boundary makes every block's partials visible; no fences or atomics).
template <int NV>
__device__ __forceinline__ void store_partials(double (&v)[NV], const int (&op)[NV], double* part) {
  block_reduce<NV>(v, op);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(int64_t)blockIdx.x * NV + k] = v[k];
  }
}

constexpr int kU = 8;  // entries per unrolled chunk of a sparse row stream

// Software-pipelined pass over F entries of one lane, entry f at
// base + f * step: the column and value loads of chunk k+1 are issued before
// the gathers of chunk k, so a chunk costs one memory round trip instead of
// two.  consume(v, xs) is called per entry, in order, with the value and
// the gathered x[col] * scale, both converted to AT.
template <typename VT, typename XT, typename AT, typename Consume>
__device__ __forceinline__ void ell_stream(const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, int64_t base,
                                           int64_t step, int F, const XT* __restrict__ x,
                                           XT scale, Consume&& consume) {
  if (F <= 0) return;
  int32_t c[kU], cn[kU];
  VT v[kU], vn[kU];
  auto load = [&](int f0, int32_t(&cc)[kU], VT(&vv)[kU]) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = base + (int64_t)min(f0 + u, F - 1) * step;  // clamped: in range
      cc[u] = ld_stream(col + e);
      vv[u] = ld_stream(val + e);
    }
  };
  auto use = [&](int f0, const int32_t(&cc)[kU], const VT(&vv)[kU]) {
    XT xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) xv[u] = x[cc[u]];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (f0 + u < F) {
        if constexpr (sizeof(AT) == 8)
          consume(to_d(vv[u]), (AT)(xv[u] * scale));
        else
          consume(to_f(vv[u]), (AT)(xv[u] * scale));
      }
    }
  };
  load(0, c, v);
  int f0 = 0;
  for (; f0 + kU < F; f0 += 2 * kU) {
    load(f0 + kU, cn, vn);
    use(f0, c, v);
    if (f0 + 2 * kU >= F) {
      use(f0 + kU, cn, vn);
      return;
    }
    load(f0 + 2 * kU, c, v);
    use(f0 + kU, cn, vn);
  }
  use(f0, c, v);
}

// Copy the K entries j = g, g+G, ... of one sliced-ELL row (entry j at
// src + (j << 6)) to a row of another sliced-ELL array (at dst + (j << 6)).
// kU loads of each array are issued before their kU stores (for the
// compiler a store may alias a later load, so it keeps them in program
// order otherwise).
template <typename VT, int G>
__device__ __forceinline__ void ell_copy_row(const int32_t* __restrict__ scol,
                                             const VT* __restrict__ sval, int64_t src,
                                             int32_t* __restrict__ dcol, VT* __restrict__ dval,
                                             int64_t dst, int K, int g) {
  for (int j0 = g; j0 < K; j0 += kU * G) {
    int32_t c[kU];
    VT v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = src + ((int64_t)min(j0 + u * G, K - 1) << 6);  // clamped: in range
      c[u] = scol[e];
      v[u] = sval[e];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int j = j0 + u * G;
      if (j < K) {
        dcol[dst + ((int64_t)j << 6)] = c[u];
        dval[dst + ((int64_t)j << 6)] = v[u];
      }
    }
  }
}

// row stride of the Gram-Schmidt partials (doubles per block)
constexpr int kPartStride = kMaxW + 8;

}  // namespace ig
