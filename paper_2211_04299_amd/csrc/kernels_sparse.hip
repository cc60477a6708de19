// Streaming kernels over the sliced-ELL transition data (gfx950).
//
// Work mapping: a wavefront serves S = 64/G consecutive states of one 64-state
// slice; the G lanes of a state ("groups", lane = g*S + ls) split that
// state's actions (Bellman pass) or the entries of its P^pi row (products).
// Consecutive lanes of a group address consecutive states, so every value
// and column load is a contiguous run of S elements; the G partial results of
// a state are combined with xor-shuffles over offsets S, 2S, ..., 32.
// Row entries are consumed eight at a time: the eight column and value loads
// are issued before the eight dependent gathers, so every wavefront keeps
// enough loads in flight to cover HBM latency (the number of resident
// wavefronts is capped by the hardware, so only this raises the bytes in
// flight).  Reductions end with per-block partials; a one-block finishing
// kernel (launch_finalize) combines them in a fixed order.
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "internal.hpp"

namespace ig {

namespace {

// sum_j val[e_j] * x[col[e_j]] * scale over the entries j = g, g+G, ... < K of
// one sliced-ELL row starting at `base` (entry j at base + (j << 6)).
template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT ell_row(const int32_t* __restrict__ col, const VT* __restrict__ val,
                                      int64_t base, int K, int g, const XT* __restrict__ x,
                                      XT scale) {
  AT acc = 0;
  const int F = K > g ? (K - g + G - 1) / G : 0;
  ell_stream<VT, XT, AT>(col, val, base + ((int64_t)g << 6), (int64_t)G << 6, F, x, scale,
                         [&](AT pv, AT xv) {
                           if constexpr (sizeof(AT) == 8)
                             acc = fma(pv, xv, acc);
                           else
                             acc = fmaf(pv, xv, acc);
                         });
  return acc;
}

// The same sum for one lane per state and rows of K <= KR entries: all KR
// slots are loaded from one base address (immediate offsets), so every load
// of the row is in flight at once; slots past K read the next row or the
// zero tail after the last slice and are not used.  Same order and rounding
// as ell_row.
template <typename VT, typename XT, typename AT, int KR>
__device__ __forceinline__ AT row_whole(const int32_t* __restrict__ col, const VT* __restrict__ val,
                                        int64_t base, int K, const XT* __restrict__ x, XT scale) {
  int32_t c[KR];
  VT v[KR];
  const int32_t* cb = col + base;
  const VT* vb = val + base;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    c[j] = ld_stream(cb + (j << 6));
    v[j] = ld_stream(vb + (j << 6));
  }
  AT acc = 0;
#pragma unroll
  for (int h = 0; h < KR; h += KR / 2) {
    XT xv[KR / 2];
#pragma unroll
    for (int j = 0; j < KR / 2; ++j) xv[j] = h + j < K ? x[c[h + j]] : (XT)0;
#pragma unroll
    for (int j = 0; j < KR / 2; ++j)
      if (h + j < K) {
        if constexpr (sizeof(AT) == 8)
          acc = fma(to_d(v[h + j]), (AT)(xv[j] * scale), acc);
        else
          acc = fmaf(to_f(v[h + j]), (AT)(xv[j] * scale), acc);
      }
  }
  return acc;
}

// ell_row (G lanes per state) or row_whole (KR > 0: one lane, short rows)
template <typename VT, typename XT, typename AT, int G, int KR>
__device__ __forceinline__ AT pi_row(const SellPi<VT>& Pp, int64_t b, int l, int g,
                                     const XT* __restrict__ x, XT scale) {
  if constexpr (KR > 0)
    return row_whole<VT, XT, AT, KR>(Pp.col, Pp.val, Pp.off[b] + l, Pp.width[b], x, scale);
  else
    return ell_row<VT, XT, AT, G>(Pp.col, Pp.val, Pp.off[b] + l, Pp.width[b], g, x, scale);
}

template <typename AT, int G>
__device__ __forceinline__ AT group_sum(AT acc) {
  constexpr int S = kWave / G;
#pragma unroll
  for (int o = S; o < kWave; o <<= 1) acc += __shfl_xor(acc, o);
  return acc;
}

// KR > 0 (one lane per state, rows of at most KR entries): each action's row
// is loaded whole, one row ahead of the one being summed, and the entries of
// the best row so far stay in registers, so the compact P^pi row is written
// from them.  Otherwise it is re-read at the end, and since the 64 lanes of a
// wavefront choose among m blocks of a slot, that re-read fetches whole
// sectors for a few useful bytes each.
template <typename VT, int G, int KR>
__global__ __launch_bounds__(kBlock) void k_bellman(
    SellP<VT> P, const double* __restrict__ cost, int m, int64_t n, double gamma,
    const double* __restrict__ V, double* __restrict__ TV, double* __restrict__ Phi,
    int32_t* __restrict__ pi, const int32_t* __restrict__ pi_old, double tie_abs,
    double* __restrict__ cpi, SellPi<VT> Pp, double* __restrict__ part) {
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
    const int Kb = P.width[b], Mb = P.mcnt[b];
    const int64_t ob = P.off[b] + l;
    const int inc = pi_old ? pi_old[sc] : -1;

    double best = INFINITY, qinc = INFINITY;
    int besta = m;  // sentinel: no finite candidate yet
    auto candidate = [&](int a, double q) {
      if (P.adm && !P.adm[(int64_t)a * n + sc]) return;  // a is not in A(s)
      if (!(q - q == 0.0)) nonfin += valid ? 1.0 : 0.0;  // NaN or +-Inf
      if (q < best) {  // actions visited in increasing order: lowest index wins ties
        best = q;
        besta = a;
      }
      if (a == inc) qinc = q;
    };
    int rowa = -1;  // KR > 0: the action whose row is held in (bc, bv)
    int32_t bc[KR > 0 ? KR : 1];
    VT bv[KR > 0 ? KR : 1];
    if constexpr (G == 1 && KR > 0) {
      int32_t rc[KR], nc[KR];
      VT rv[KR], nv[KR];
      // all KR slots from one base address (immediate offsets); slots past
      // Kb read the next row's entries or the zero tail of kRowPad entries
      // after the last slice, and are not used
      auto load_row = [&](int a, int32_t(&cc)[KR], VT(&vv)[KR]) {
        const int32_t* cb = P.col + ob + (((int64_t)a * Kb) << 6);
        const VT* vb = P.val + ob + (((int64_t)a * Kb) << 6);
#pragma unroll
        for (int j = 0; j < KR; ++j) {
          cc[j] = ld_stream(cb + (j << 6));
          vv[j] = ld_stream(vb + (j << 6));
        }
      };
      load_row(0, rc, rv);
      double cst = cost[sc];
      for (int a = 0; a < Mb; ++a) {
        if (a + 1 < Mb) load_row(a + 1, nc, nv);
        const double cst_next = a + 1 < Mb ? cost[(int64_t)(a + 1) * n + sc] : 0.0;
        double acc = 0.0;
        // gathers in halves of KR/2 (fewer registers), summed in slot order
#pragma unroll
        for (int h = 0; h < KR; h += KR / 2) {
          double xv[KR / 2];
#pragma unroll
          for (int j = 0; j < KR / 2; ++j) xv[j] = h + j < Kb ? V[rc[h + j]] : 0.0;
#pragma unroll
          for (int j = 0; j < KR / 2; ++j)
            if (h + j < Kb) acc = fma(to_d(rv[h + j]), xv[j], acc);
        }
        candidate(a, cst + gamma * acc);
        if (besta == a) {
          rowa = a;
#pragma unroll
          for (int j = 0; j < KR; ++j) {
            bc[j] = rc[j];
            bv[j] = rv[j];
          }
        }
        cst = cst_next;
#pragma unroll
        for (int j = 0; j < KR; ++j) {
          rc[j] = nc[j];
          rv[j] = nv[j];
        }
      }
    } else if constexpr (G == 1) {
      // one lane per state: rows a = 0..m-1 of the slice are consecutive, so
      // the m*Kb entries form one pipelined stream; the cost of row a is
      // loaded when the row starts and used when it ends
      double acc = 0.0, cst = cost[sc];
      int j = 0, a = 0;
      ell_stream<VT, double, double>(P.col, P.val, ob, kSlice, Mb * Kb, V, 1.0,
                                     [&](double pv, double xv) {
                                       acc = fma(pv, xv, acc);
                                       if (++j == Kb) {
                                         candidate(a, cst + gamma * acc);
                                         acc = 0.0;
                                         j = 0;
                                         if (++a < Mb) cst = cost[(int64_t)a * n + sc];
                                       }
                                     });
    } else {
      for (int a = g; a < Mb; a += G) {
        const double acc = ell_row<VT, double, double, 1>(
            P.col, P.val, ob + (((int64_t)a * Kb) << 6), Kb, 0, V, 1.0);
        candidate(a, cost[(int64_t)a * n + sc] + gamma * acc);
      }
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
    if (Pp.col) {  // the chosen row into the compact P^pi (groups split j)
      if (KR > 0 && astar == rowa) {
        const int64_t dst = Pp.off[b] + l;
#pragma unroll
        for (int j = 0; j < (KR > 0 ? KR : 1); ++j)
          if (j < Kb) {
            Pp.col[dst + ((int64_t)j << 6)] = bc[j];
            Pp.val[dst + ((int64_t)j << 6)] = bv[j];
          }
      } else {
        ell_copy_row<VT, G>(P.col, P.val, ob + (((int64_t)astar * Kb) << 6), Pp.col, Pp.val,
                            Pp.off[b] + l, Kb, g);
      }
    }
  }
  double v[4] = {pmax, psum, nonfin, chg};
  const int op[4] = {1, 0, 0, 0};
  store_partials<4>(v, op, part);
}

// y = xs - gamma * P^pi xs, xs = x * scale (scale = 1/eta, or 1)
template <typename VT, typename XT, typename AT, int G, int KR>
__global__ __launch_bounds__(kBlock) void k_japply(SellPi<VT> Pp, int64_t n, AT gamma,
                                                   const XT* __restrict__ x,
                                                   const double* __restrict__ eta,
                                                   XT* __restrict__ y) {
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
    const AT acc = group_sum<AT, G>(pi_row<VT, XT, AT, G, KR>(Pp, b, l, g, x, scale));
    if (s < n && g == 0) {
      const XT xs = x[s] * scale;
      y[s] = (XT)((AT)xs - gamma * acc);
    }
  }
}

// One Horner step of the Neumann preconditioner M^{-1} = sum_{k<=d} (gamma
// P^pi)^k:  y = x * sx + gamma * (P^pi z) * sz  (sx, sz = 1 / *eta or 1).
template <typename VT, typename XT, typename AT, int G, int KR>
__global__ __launch_bounds__(kBlock) void k_pstep(SellPi<VT> Pp, int64_t n, AT gamma,
                                                  const XT* __restrict__ x,
                                                  const double* __restrict__ sx,
                                                  const XT* __restrict__ z,
                                                  const double* __restrict__ sz,
                                                  XT* __restrict__ y) {
  constexpr int S = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int ls = lane % S, g = lane / S;
  const int64_t nw = (n + S - 1) / S;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  const AT ax = sx ? (AT)(1.0 / *sx) : (AT)1, az = sz ? (AT)(1.0 / *sz) : (AT)1;
  for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; w < nw;
       w += wstride) {
    const int64_t s = w * S + ls;
    const int64_t b = s >> 6;
    const int l = (int)(s & 63);
    const AT acc = group_sum<AT, G>(pi_row<VT, XT, AT, G, KR>(Pp, b, l, g, z, (XT)1));
    if (s < n && g == 0) y[s] = (XT)((AT)x[s] * ax + gamma * acc * az);
  }
}

// MODE 0: r = g^pi - (V - gamma P^pi V), partials {max|r|, ||r||^2, max|V|}
// MODE 1: Vout = g^pi + gamma P^pi Vin, partials {max|Vout - Vin|, ||.||^2, 0}
template <typename VT, int G, int MODE, int KR>
__global__ __launch_bounds__(kBlock) void k_policy_pass(SellPi<VT> Pp, int64_t n, double gamma,
                                                        const double* __restrict__ cpi,
                                                        const double* __restrict__ V,
                                                        double* __restrict__ out,
                                                        double* __restrict__ part) {
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
    const double acc = group_sum<double, G>(pi_row<VT, double, double, G, KR>(Pp, b, l, g, V, 1.0));
    if (s < n && g == 0) {
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

template <typename VT, int G>
__global__ __launch_bounds__(kBlock) void k_gather_policy(SellP<VT> P, SellPi<VT> Pp,
                                                          const double* __restrict__ cost, int m,
                                                          int64_t n, const int32_t* __restrict__ pi,
                                                          double* __restrict__ cpi,
                                                          double* __restrict__ part) {
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
    const int Kb = P.width[b], Mb = P.mcnt[b];
    int a = valid ? pi[s] : 0;
    if (a < 0 || a >= Mb || (valid && P.adm && !P.adm[(int64_t)a * n + s])) {  // not in A(s)
      if (g == 0 && valid) bad += 1.0;
      a = 0;  // a stored block (zero padding when excluded): stays in bounds
    }
    ell_copy_row<VT, G>(P.col, P.val, P.off[b] + (((int64_t)a * Kb) << 6) + l, Pp.col, Pp.val,
                        Pp.off[b] + l, Kb, g);
    if (valid && g == 0) cpi[s] = cost[(int64_t)a * n + s];
  }
  double v[1] = {bad};
  const int op[1] = {0};
  store_partials<1>(v, op, part);
}

inline int grid_for(const Mdp& d, int G) {
  const int64_t waves = (d.n + (kWave / G) - 1) / (kWave / G);
  const int64_t blocks = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, kMaxBlocks));
}

template <typename VT>
SellP<VT> viewP(Mdp& d) {
  return SellP<VT>{d.col, (const VT*)d.val, d.off, d.width, d.mcnt, d.adm};
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
    // rows of at most 16 entries, narrow values: the register-held rows
    // (IG_BELLMAN_ROWS=off selects the re-read, for comparisons)
    const char* ev = std::getenv("IG_BELLMAN_ROWS");
    const bool rows = G == 1 && !std::is_same<VT, double>::value && d.maxK <= 16 &&
                      !(ev && !std::strcmp(ev, "off"));
    if (rows)
      hipLaunchKernelGGL((k_bellman<VT, 1, 16>), dim3(grid_for(d, 1)), dim3(kBlock), 0, s,
                         viewP<VT>(d), (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi, pi,
                         pi_old, tie_abs, d.cpi, pp, d.part);
    else
      hipLaunchKernelGGL((k_bellman<VT, G, 0>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                         viewP<VT>(d), (const double*)d.cost, d.m, d.n, d.gamma, V, TV, Phi, pi,
                         pi_old, tie_abs, d.cpi, pp, d.part);
  }
};

// one lane per state and rows of at most 16 entries: whole-row loads
template <int G, typename F>
void with_rows(const Mdp& d, F&& f) {
  if constexpr (G == 1) {
    if (d.maxK <= 16) {
      f(std::integral_constant<int, 16>{});
      return;
    }
  }
  f(std::integral_constant<int, 0>{});
}

template <typename VT, int G>
struct RunJapply {
  static void run(Mdp& d, bool fp32, const void* x, const double* eta, void* y, hipStream_t s) {
    with_rows<G>(d, [&](auto kr) {
      constexpr int KR = decltype(kr)::value;
      if (fp32)
        hipLaunchKernelGGL((k_japply<VT, float, float, G, KR>), dim3(grid_for(d, G)),
                           dim3(kBlock), 0, s, viewPi<VT>(d), d.n, (float)d.gamma, (const float*)x,
                           eta, (float*)y);
      else
        hipLaunchKernelGGL((k_japply<VT, double, double, G, KR>), dim3(grid_for(d, G)),
                           dim3(kBlock), 0, s, viewPi<VT>(d), d.n, d.gamma, (const double*)x, eta,
                           (double*)y);
    });
  }
};

template <typename VT, int G>
struct RunPstep {
  static void run(Mdp& d, bool fp32, const void* x, const double* sx, const void* z,
                  const double* sz, void* y, hipStream_t s) {
    with_rows<G>(d, [&](auto kr) {
      constexpr int KR = decltype(kr)::value;
      if (fp32)
        hipLaunchKernelGGL((k_pstep<VT, float, float, G, KR>), dim3(grid_for(d, G)), dim3(kBlock),
                           0, s, viewPi<VT>(d), d.n, (float)d.gamma, (const float*)x, sx,
                           (const float*)z, sz, (float*)y);
      else
        hipLaunchKernelGGL((k_pstep<VT, double, double, G, KR>), dim3(grid_for(d, G)),
                           dim3(kBlock), 0, s, viewPi<VT>(d), d.n, d.gamma, (const double*)x, sx,
                           (const double*)z, sz, (double*)y);
    });
  }
};

template <typename VT, int G>
struct RunResidual {
  static void run(Mdp& d, const double* V, double* r, hipStream_t s) {
    with_rows<G>(d, [&](auto kr) {
      hipLaunchKernelGGL((k_policy_pass<VT, G, 0, decltype(kr)::value>), dim3(grid_for(d, G)),
                         dim3(kBlock), 0, s, viewPi<VT>(d), d.n, d.gamma, (const double*)d.cpi, V,
                         r, d.part);
    });
  }
};

template <typename VT, int G>
struct RunVi {
  static void run(Mdp& d, const double* Vin, double* Vout, hipStream_t s) {
    with_rows<G>(d, [&](auto kr) {
      hipLaunchKernelGGL((k_policy_pass<VT, G, 1, decltype(kr)::value>), dim3(grid_for(d, G)),
                         dim3(kBlock), 0, s, viewPi<VT>(d), d.n, d.gamma, (const double*)d.cpi,
                         Vin, Vout, d.part);
    });
  }
};

template <typename VT, int G>
struct RunGather {
  static void run(Mdp& d, const int32_t* pi, hipStream_t s) {
    hipLaunchKernelGGL((k_gather_policy<VT, G>), dim3(grid_for(d, G)), dim3(kBlock), 0, s,
                       viewP<VT>(d), viewPi<VT>(d), (const double*)d.cost, d.m, d.n, pi, d.cpi,
                       d.part);
  }
};

}  // namespace

void launch_bellman_sparse(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
                           const int32_t* pi_old, double tie_abs, bool compact, hipStream_t s) {
  {
    ProfScope p(d, KC_BELLMAN, s);
    dispatch_vt_g<RunBellman>(d, d.G_bell, d, V, TV, Phi, pi, pi_old, tie_abs, compact, s);
  }
  launch_finalize(d, FIN_BELLMAN, grid_for(d, d.G_bell), s);
  if (compact && d.refine) launch_round_bf16((const float*)d.pval, d.in_pval, d.stored_pi, s);
}

void launch_japply_sparse(Mdp& d, bool fp32, const void* x, const double* eta, void* y,
                          hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  InnerView iv(d);
  dispatch_vt_g<RunJapply>(d, d.G_jap, d, fp32, x, eta, y, s);
}

void launch_pstep_sparse(Mdp& d, bool fp32, const void* x, const double* sx, const void* z,
                         const double* sz, void* y, hipStream_t s) {
  ProfScope p(d, KC_JAPPLY, s);
  InnerView iv(d);
  dispatch_vt_g<RunPstep>(d, d.G_jap, d, fp32, x, sx, z, sz, y, s);
}

void launch_residual_sparse(Mdp& d, const double* V, double* r, hipStream_t s) {
  {
    ProfScope p(d, KC_RESID, s);
    dispatch_vt_g<RunResidual>(d, d.G_jap, d, V, r, s);
  }
  launch_finalize(d, FIN_RESID, grid_for(d, d.G_jap), s);
}

void launch_vi_sweep_sparse(Mdp& d, const double* Vin, double* Vout, hipStream_t s, bool finish) {
  {
    ProfScope p(d, KC_VI, s);
    dispatch_vt_g<RunVi>(d, d.G_jap, d, Vin, Vout, s);
  }
  if (finish) launch_finalize(d, FIN_VI, grid_for(d, d.G_jap), s);
}

void launch_gather_policy_sparse(Mdp& d, const int32_t* pi, hipStream_t s) {
  {
    ProfScope p(d, KC_OTHER, s);
    dispatch_vt_g<RunGather>(d, d.G_jap, d, pi, s);
  }
  launch_finalize(d, FIN_GATHER, grid_for(d, d.G_jap), s);
  if (d.refine) launch_round_bf16((const float*)d.pval, d.in_pval, d.stored_pi, s);
}

}  // namespace ig
