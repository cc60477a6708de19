// Persistent single-launch GMRES(W) policy iteration (Algorithm 2) for
// sparse MDPs that fit one cooperative grid (gfx950).
//
// Layout of the work: every block owns a fixed, contiguous range of 64-state
// slices for the whole solve.  Phases are separated by grid barriers built
// from one arrival word per block (each block polls all words; no shared
// counter, so arrivals are not serialised on one address).  After a barrier
// every block reduces the per-block partials itself, in a fixed order, and
// runs the Givens update and the control decisions on its own copy of the
// (tiny) least-squares state: all blocks compute bit-identical values and so
// follow the same path without any broadcast.  Barrier waits have a spin
// limit; a wait that exceeds it flags an error and every block leaves at its
// next barrier.
//
// Arnoldi step i (two barriers; classical Gram-Schmidt applied twice):
//   [A] Q_i = (w1 - sum_j d_j Q_j) / eta_i on own rows (the second-pass
//       correction of the previous step, applied lazily);
//       w = J w1 / eta_i (gather of the complete w1);  c_j = <Q_j, w>, j <= i
//   -- barrier --
//   [B] w1 = w - sum_j c_j Q_j; d_j = <Q_j, w1>; sigma = ||w1||^2
//   -- barrier --
//   eta_{i+1} = sqrt(sigma - ||d||^2), column i of H = c + d.
// Because the second-pass coefficients d are of the order of the rounding
// error, applying J to w1 instead of to Q_{i+1} * eta_{i+1} changes the
// product only at that order, and Pythagoras gives eta without cancellation.
// When the residual bracket ||r||_inf <= rho <= sqrt(n) ||r||_inf cannot
// decide the stopping test, the iterate is formed and the true FP64 residual
// evaluated (two more barriers).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "internal.hpp"

namespace ig {

namespace {

constexpr int kPB = 1024;            // threads per block
constexpr int kPWaves = kPB / kWave;
constexpr int kPMaxBlocks = 256;
constexpr int kPMaxSpb = 32;         // slices per block
constexpr int kPMaxW = kPersistMaxRestart;  // restart cap of this engine (LDS Givens state)
constexpr int kPStride = kPMaxW + 8; // doubles per block row of partials
constexpr long kSpinLimit = 1L << 23;  // polls per barrier wait (IG_SPIN_LIMIT overrides)

template <typename VT, typename XT>
struct PArgs {
  SellP<VT> P;
  SellPi<VT> Pp;
  const double* __restrict__ cost;
  int m;
  int64_t n;
  int64_t nslices;
  int spb;
  double gamma;
  double* __restrict__ V;
  int32_t* __restrict__ pi;
  double* __restrict__ cpi;
  XT* __restrict__ Q;
  XT* __restrict__ w1;
  double* __restrict__ Vb;
  double* __restrict__ r;
  double* __restrict__ part;         // [2][gridDim.x][kPStride], by barrier parity
  unsigned int* __restrict__ flags;  // [gridDim.x] arrival epochs
  PCtl* __restrict__ ctl;
  double alpha, tol, sqrt_n;
  int W, max_outer, max_inner, forcing;
  int vlds;  // the Bellman pass gathers V from a copy in LDS (n doubles fit)
  int polish;  // evaluate to tol / 2 once the greedy policy repeats
  long spin_limit;  // polls before a barrier wait fails
  double b_bellman, b_japply, b_vec, b_resid;  // algorithmic bytes per event
};

// least-squares state of the current restart cycle (per block, LDS)
struct Lsq {
  double R[(kPMaxW + 1) * kPMaxW];  // column-major, leading dim kPMaxW+1
  double cs[kPMaxW], sn[kPMaxW], g[kPMaxW + 1], y[kPMaxW];
  double c[kPMaxW + 2], d[kPMaxW + 1];
  double z[kPMaxW + 2];  // residual of the newest column's iterate in basis coordinates
};

struct Scal {  // per-block copies of the solver scalars (identical in every block)
  double thr, beta, cycle_beta, eta, inv_eta, rho, phi_inf, res_inf, res_l2sq, alg_bytes;
  int dec, outer, inner, steps_outer, restarts, expl, breakdowns, stagnations, bellman, converged,
      nonfinite;
};

enum : int { D_NEXT = 0, D_EXPLICIT, D_LAG, D_END_INNER, D_RESTART, D_CONT, D_DONE, D_NOCONV, D_ERR };

__device__ __forceinline__ int logical_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb % 8 != 0) return b;  // round-robin XCD dispatch: contiguous slices per XCD
  return (b % 8) * (nb / 8) + b / 8;
}

__device__ __forceinline__ unsigned ld_flag(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier on per-block arrival words.  Returns false (uniformly in the
// block) if a wait exceeded the spin limit or, while this block waited,
// another block had already failed its own wait: a block that fails leaves
// without arriving at the next barrier, so every other block either finds the
// error flag during that wait or times out itself, and the grid drains.  A
// barrier whose arrivals are all seen completes without reading the flag.
// bad: two LDS words, zero at launch, used by barrier parity; each barrier
// clears the word of the next one (all threads read it before this barrier).
__device__ __forceinline__ bool gbarrier(unsigned int* flags, PCtl* ctl, unsigned epoch,
                                         int* bad, long spin_limit) {
  __syncthreads();
  if (gridDim.x == 1) return true;  // one block: the block barrier orders everything
  if (threadIdx.x == 0) {
    bad[(epoch + 1) & 1] = 0;
    __hip_atomic_store(&flags[blockIdx.x], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x < gridDim.x) {
    long spins = 0;
    while (ld_flag(&flags[threadIdx.x]) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > spin_limit) {
        __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bad[epoch & 1] = 1;
        break;
      }
      if ((spins & 1023) == 0 &&
          __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        bad[epoch & 1] = 1;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return bad[epoch & 1] == 0;
}

// out[c] = sum (or max: maxmask bit c, or c == maxcol) over blocks of
// part[b][c], c < cnt; fixed order; all threads; result in LDS `out`.
__device__ void reduce_rows(const double* __restrict__ part, int cnt, unsigned maxmask,
                            double* __restrict__ out, int maxcol = -1) {
  __shared__ double seg[16][64];
  const int nb = gridDim.x;
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const bool mx = (c0 == 0 && c < 32 && ((maxmask >> c) & 1u)) || c0 + c == maxcol;
    double acc = 0.0;
    if (c0 + c < cnt) {
      // the loads of up to 128 blocks are issued before the first add (one
      // round trip each 128 blocks); the sum still runs over b = q, q+16,
      // ... in that order
      for (int b0 = 0; b0 < nb; b0 += 128) {
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int b = b0 + q + 16 * k;
          x[k] = b < nb ? part[(int64_t)b * kPStride + c0 + c] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (b0 + q + 16 * k < nb) acc = mx ? fmax(acc, x[k]) : acc + x[k];
      }
    }
    seg[q][c] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && c0 + threadIdx.x < cnt) {
      double a = seg[0][threadIdx.x];
      for (int k = 1; k < 16; ++k) a = mx ? fmax(a, seg[k][threadIdx.x]) : a + seg[k][threadIdx.x];
      out[c0 + threadIdx.x] = a;
    }
    __syncthreads();
  }
}

template <int NV>
__device__ __forceinline__ void block_reduce_big(double (&v)[NV], const int (&op)[NV],
                                                 double* mypart) {
  __shared__ double sh[NV][kPWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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
      for (int w = 1; w < kPWaves; ++w) a = op[k] ? fmax(a, sh[k][w]) : a + sh[k][w];
      mypart[k] = a;
    }
  }
}

// (kept as a plain unrolled loop: the kernel runs 1024-thread blocks, so it
// has 128 registers per lane and a double-buffered stream would spill)
template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT prow_dot(const SellPi<VT>& Pp, int64_t b, int l, int g,
                                       const XT* __restrict__ x) {
  constexpr int S = kWave / G;
  const int Kb = Pp.width[b];
  const int64_t ob = Pp.off[b] + l;
  AT acc = 0;
#pragma unroll 8
  for (int j = g; j < Kb; j += G) {
    const int64_t e = ob + ((int64_t)j << 6);
    const XT xv = x[Pp.col[e]];
    if constexpr (sizeof(AT) == 8)
      acc = fma(to_d(Pp.val[e]), (AT)xv, acc);
    else
      acc = fmaf(to_f(Pp.val[e]), (AT)xv, acc);
  }
#pragma unroll
  for (int o = S; o < kWave; o <<= 1) acc += __shfl_xor(acc, o);
  return acc;
}

__device__ __forceinline__ int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// The block's rows of the Krylov basis: row t of column j at base[j*ld + t]
// (LDS-resident with ld = the padded own-row count, or the global basis with
// base = Q + s_lo and ld = n).
template <typename XT>
struct QView {
  XT* base;
  int64_t ld;
  __device__ __forceinline__ XT& at(int j, int t) const { return base[(int64_t)j * ld + t]; }
};

// partial dots <Q_j, wl> (own rows) for j < cnt into mypart[0..cnt); with_norm
// adds ||wl||^2 as mypart[cnt].  Groups of gsz threads (a power of two,
// 8..64) per j; every thread sums a strided subset of the own rows with its
// loads issued together, then the group reduces with shuffles.
template <typename XT>
__device__ __forceinline__ void own_dots(QView<XT> Q, int cnt, int nown,
                                         const double* __restrict__ wl, double* mypart,
                                         bool with_norm) {
  const int tot = cnt + (with_norm ? 1 : 0);
  const int gsz = max(8, min(64, kPB / pow2_ceil(tot)));
  const int sub = threadIdx.x & (gsz - 1);
  for (int j0 = 0; j0 < tot; j0 += kPB / gsz) {
    const int j = j0 + threadIdx.x / gsz;
    double a0 = 0.0, a1 = 0.0;
    if (j < cnt) {
      const XT* q = &Q.at(j, 0);
      int t = sub;
      for (; t + gsz < nown; t += 2 * gsz) {
        a0 = fma(to_d(q[t]), wl[t], a0);
        a1 = fma(to_d(q[t + gsz]), wl[t + gsz], a1);
      }
      if (t < nown) a0 = fma(to_d(q[t]), wl[t], a0);
    } else if (j == cnt && with_norm) {
      for (int t = sub; t < nown; t += gsz) a0 = fma(wl[t], wl[t], a0);
    }
    double acc = a0 + a1;
    for (int o = 1; o < gsz; o <<= 1) acc += __shfl_xor(acc, o);
    if (sub == 0 && j < tot) mypart[j] = acc;
  }
}

// out[t] = base[t] + sign * sum_{j<cnt} coef_j Q_j(s_lo + t) for the own rows
// (base and out may alias, both in LDS or global through the callbacks).
// The block splits the j range over `parts` thread groups when the own rows
// are few, and combines the partial sums in a fixed order through LDS.
template <typename XT, typename Base, typename Out>
__device__ __forceinline__ void own_axpy(QView<XT> Q, int nown, int cnt,
                                         const double* __restrict__ coef, double sign,
                                         double* psum /* LDS, kPB */, Base base, Out out) {
  const int parts = nown >= kPB ? 1 : max(1, min(8, kPB / pow2_ceil(nown)));
  const int span = kPB / parts;  // states per pass
  const int p = threadIdx.x / span, tl = threadIdx.x % span;
  for (int t0 = 0; t0 < nown; t0 += span) {
    const int t = t0 + tl;
    double acc = 0.0;
    if (t < nown) {
      double a0 = 0.0, a1 = 0.0;
      int j = p;
      for (; j + parts < cnt; j += 2 * parts) {
        a0 = fma(coef[j], to_d(Q.at(j, t)), a0);
        a1 = fma(coef[j + parts], to_d(Q.at(j + parts, t)), a1);
      }
      if (j < cnt) a0 = fma(coef[j], to_d(Q.at(j, t)), a0);
      acc = a0 + a1;
    }
    if (parts > 1) {
      psum[threadIdx.x] = acc;
      __syncthreads();
      if (p == 0 && t < nown) {
        double a = psum[tl];
        for (int q = 1; q < parts; ++q) a += psum[q * span + tl];
        out(t, fma(sign, a, base(t)));
      }
      __syncthreads();
    } else if (t < nown) {
      out(t, fma(sign, acc, base(t)));
    }
  }
}

// Q_i = (w1 - sum_{j<i} d_j Q_j) * inv on the own rows, and the implicit
// residual of column i-1, r = sum_{j<i} z_j Q_j + z_i Q_i, whose largest
// |r| over the own rows is returned (valid in every thread).  Same thread
// split as own_axpy; psum and psum2 are LDS scratch of kPB doubles each.
template <typename XT>
__device__ __forceinline__ double own_form(QView<XT> Q, int nown, int i,
                                           const double* __restrict__ d,
                                           const double* __restrict__ z, double inv,
                                           const double* __restrict__ w1l, double* psum,
                                           double* psum2) {
  const int parts = nown >= kPB ? 1 : max(1, min(8, kPB / pow2_ceil(max(nown, 1))));
  const int span = kPB / parts;
  const int p = threadIdx.x / span, tl = threadIdx.x % span;
  double rmax = 0.0;
  for (int t0 = 0; t0 < nown; t0 += span) {
    const int t = t0 + tl;
    double ad = 0.0, az = 0.0;
    if (t < nown) {
      for (int j = p; j < i; j += parts) {
        const double q = to_d(Q.at(j, t));
        ad = fma(d[j], q, ad);
        az = fma(z[j], q, az);
      }
    }
    if (parts > 1) {
      psum[threadIdx.x] = ad;
      psum2[threadIdx.x] = az;
      __syncthreads();
      if (p == 0 && t < nown) {
        double a = psum[tl], b = psum2[tl];
        for (int q = 1; q < parts; ++q) {
          a += psum[q * span + tl];
          b += psum2[q * span + tl];
        }
        ad = a;
        az = b;
      }
      __syncthreads();
    }
    if (p == 0 && t < nown) {
      const XT qx = from_d<XT>((w1l[t] - ad) * inv);
      Q.at(i, t) = qx;
      rmax = fmax(rmax, fabs(fma(z[i], to_d(qx), az)));
    }
  }
  __shared__ double wm[kPWaves];
  rmax = wave_max(rmax);
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = rmax;
  __syncthreads();
  double m = wm[0];
  for (int w = 1; w < kPWaves; ++w) m = fmax(m, wm[w]);
  __syncthreads();
  return m;
}

// y = R^{-1} g_hat over the first `cols` columns (one thread)
__device__ __forceinline__ void back_sub(Lsq& L, int cols) {
  for (int j = cols - 1; j >= 0; --j) {
    double a = L.g[j];
    for (int l2 = j + 1; l2 < cols; ++l2) a -= L.R[l2 * (kPMaxW + 1) + j] * L.y[l2];
    const double dj = L.R[j * (kPMaxW + 1) + j];
    L.y[j] = dj != 0.0 ? a / dj : 0.0;
  }
}

// QL: the block's basis rows live in LDS (dynamic shared memory, after the
// two own-row vectors); otherwise in the global basis.
template <typename VT, typename XT, int G, bool QL>
__global__ __launch_bounds__(kPB) void k_persist(PArgs<VT, XT> A) {
  using AT = XT;  // accumulation of the P^pi products inside GMRES
  constexpr int S = kWave / G;
  constexpr int SPR = S * kPWaves;  // states per round
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int ls = lane % S, g = lane / S;
  const int lb = logical_block();
  const int64_t sl0 = (int64_t)lb * A.spb;
  const int64_t sl1 = min<int64_t>(A.nslices, sl0 + A.spb);
  const int64_t s_lo = sl0 * kSlice, s_hi = sl1 * kSlice;
  const int64_t n = A.n;
  const int64_t v_hi = min<int64_t>(s_hi, n);
  const int nown = (int)max<int64_t>(0, v_hi - s_lo);
  // Partials written before barrier e are read by every block after it; a
  // fast block may already write its next partials while a slow one still
  // reads, so rows alternate between two buffers by barrier parity.
  const int64_t half = (int64_t)gridDim.x * kPStride;

  __shared__ Lsq L;
  __shared__ Scal sc;
  extern __shared__ double dsm[];   // [ldq] w, [ldq] w1 of the own rows, then the basis rows
  const int ldq = A.spb * kSlice;
  double* wl = dsm;
  double* w1l = dsm + ldq;
  QView<XT> Qv;
  if constexpr (QL)
    Qv = QView<XT>{reinterpret_cast<XT*>(dsm + 2 * ldq), ldq};
  else
    Qv = QView<XT>{A.Q + s_lo, n};
  __shared__ double red[kPMaxW + 8];
  __shared__ double coef[kPMaxW + 1];
  __shared__ double psum[kPB];
  __shared__ double psum2[kPB];

  __shared__ int s_bad[2];  // barrier failure words, by barrier parity

  if (threadIdx.x == 0) {
    sc = Scal{};
    sc.dec = D_NEXT;
    s_bad[0] = s_bad[1] = 0;
  }
  __syncthreads();
  unsigned epoch = 0;
#define MYPART (A.part + ((epoch + 1) & 1) * half + (int64_t)blockIdx.x * kPStride)
#define PARTS (A.part + (epoch & 1) * half)
  int i = 0;           // basis vectors Q_0..Q_{i-1} formed in this cycle
  bool from_r = true;  // the next basis vector is r / beta (cycle start)
  double impl_max = 0.0;

  // V = Vb + sum_{j<cols} y_j Q_j on the own rows, then the true FP64
  // residual r = g^pi - J V with its infinity- and 2-norms into sc
  // (two grid barriers; false if a barrier wait failed)
  auto explicit_resid = [&](int cols) -> bool {
    for (int j = threadIdx.x; j < cols; j += kPB) coef[j] = L.y[j];
    __syncthreads();
    own_axpy<XT>(Qv, nown, cols, coef, 1.0, psum, [&](int t) { return A.Vb[s_lo + t]; },
                 [&](int t, double v) { A.V[s_lo + t] = v; });
    if (!gbarrier(A.flags, A.ctl, ++epoch, s_bad, A.spin_limit)) return false;
    {
      double pmax = 0.0, ps = 0.0;
      for (int64_t base = s_lo + (int64_t)wid * S; base < s_hi; base += SPR) {
        const int64_t s = base + ls;
        const int64_t b = s >> 6;
        const int l = (int)(s & 63);
        const double acc = prow_dot<VT, double, double, G>(A.Pp, b, l, g, A.V);
        if (s < n && g == 0) {
          const double rr = A.cpi[s] - (A.V[s] - A.gamma * acc);
          A.r[s] = rr;
          pmax = fmax(pmax, fabs(rr));
          ps = fma(rr, rr, ps);
        }
      }
      double v[2] = {pmax, ps};
      const int op[2] = {1, 0};
      block_reduce_big<2>(v, op, MYPART);
    }
    if (!gbarrier(A.flags, A.ctl, ++epoch, s_bad, A.spin_limit)) return false;
    reduce_rows(PARTS, 2, 1u, red);
    if (threadIdx.x == 0) {
      sc.alg_bytes += A.b_resid + A.b_vec * (cols + 2.0);
      sc.expl += 1;
      sc.res_inf = red[0];
      sc.res_l2sq = red[1];
    }
    __syncthreads();
    return true;
  };

#define IG_BARRIER()                                    \
  do {                                                  \
    if (!gbarrier(A.flags, A.ctl, ++epoch, s_bad, A.spin_limit)) goto leave; \
  } while (0)

  for (int k = 0;; ++k) {
    // ---------------- Bellman pass: pi_k, Phi_k = T V_k - V_k, g^pi, P^pi
    {
      double pmax = 0.0, psum = 0.0, nonfin = 0.0, chg = 0.0;
      // The V gathers (m*k per state) read a copy of V in LDS when it fits: the
      // basis and product rows there are dead between inner solves.
      auto rows = [&](auto in_lds) {
        const double* __restrict__ Vg = decltype(in_lds)::value ? dsm : A.V;
        for (int64_t base = s_lo + (int64_t)wid * S; base < s_hi; base += SPR) {
          const int64_t s = base + ls;
          const bool valid = s < n;
          const int64_t sc2 = valid ? s : n - 1;
          const int64_t b = s >> 6;
          const int l = (int)(s & 63);
          const int Kb = A.P.width[b], Mb = A.P.mcnt[b];
          const int64_t ob = A.P.off[b];
          double best = INFINITY;
          int besta = A.m;
          auto candidate = [&](int a, double q) {
            if (A.P.adm && !A.P.adm[(int64_t)a * n + sc2]) return;  // a is not in A(s)
            if (!(q - q == 0.0)) nonfin += valid ? 1.0 : 0.0;
            if (q < best) {  // increasing a: lowest index wins ties
              best = q;
              besta = a;
            }
          };
          for (int a = g; a < Mb; a += G) {
            const int64_t bs = ob + (((int64_t)a * Kb) << 6) + l;
            double acc = 0.0;
  #pragma unroll 8
            for (int j = 0; j < Kb; ++j) {
              const int64_t e = bs + ((int64_t)j << 6);
              acc = fma(to_d(A.P.val[e]), Vg[A.P.col[e]], acc);
            }
            candidate(a, A.cost[(int64_t)a * n + sc2] + A.gamma * acc);
          }
  #pragma unroll
          for (int o = S; o < kWave; o <<= 1) {
            const double ob2 = __shfl_xor(best, o);
            const int oa = __shfl_xor(besta, o);
            if (ob2 < best || (ob2 == best && oa < besta)) {
              best = ob2;
              besta = oa;
            }
          }
          if (besta >= A.m) {
            besta = 0;
            best = NAN;
          }
          if (valid && g == 0) {
            const double phi = best - Vg[s];
            A.r[s] = phi;
            if (A.polish && k > 0 && A.pi[s] != besta) chg += 1.0;  // pi_{k-1} of this thread
            A.pi[s] = besta;
            A.cpi[s] = A.cost[(int64_t)besta * n + s];
            if (!(phi - phi == 0.0)) nonfin += 1.0;
            pmax = fmax(pmax, fabs(phi));
            psum = fma(phi, phi, psum);
          }
          ell_copy_row<VT, G>(A.P.col, A.P.val, ob + (((int64_t)besta * Kb) << 6) + l, A.Pp.col,
                              A.Pp.val, A.Pp.off[b] + l, Kb, g);
        }
      };
      if (A.vlds) {
        for (int64_t t = threadIdx.x; t < n; t += kPB) dsm[t] = A.V[t];
        __syncthreads();
        rows(std::true_type{});
      } else {
        rows(std::false_type{});
      }
      double v[4] = {pmax, psum, nonfin, chg};
      const int op[4] = {1, 0, 0, 0};
      block_reduce_big<4>(v, op, MYPART);
    }
    IG_BARRIER();
    reduce_rows(PARTS, 4, 1u, red);
    if (threadIdx.x == 0) {
      sc.bellman += 1;
      sc.alg_bytes += A.b_bellman;
      sc.outer = k;
      sc.phi_inf = red[0];
      if (red[2] != 0.0) {
        sc.nonfinite = 1;
        sc.dec = D_ERR;
      } else if (red[0] <= A.tol) {
        sc.converged = 1;
        sc.dec = D_DONE;
      } else if (k >= A.max_outer) {
        sc.dec = D_NOCONV;
      } else {
        const double alpha = A.forcing ? fmin(A.alpha, sqrt(red[0])) : A.alpha;
        sc.thr = alpha * red[0];
        if (A.polish && k > 0 && red[3] == 0.0) sc.thr = fmin(sc.thr, 0.5 * A.tol);
        sc.beta = sqrt(red[1]);
        sc.cycle_beta = sc.beta;
        sc.steps_outer = 0;
        for (int j = 0; j <= kPMaxW; ++j) L.g[j] = 0.0;
        L.g[0] = sc.beta;
        sc.dec = D_NEXT;
      }
    }
    __syncthreads();
    if (sc.dec != D_NEXT) goto leave;

    // cycle start: Vb = V on own rows; the first basis vector is r / beta
    for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) A.Vb[s] = A.V[s];
    i = 0;
    from_r = true;

    for (;;) {
      // ---------------- [A] form Q_i; w = J Q_i; c = Q^T w
      {
        if (from_r) {
          const double inv = 1.0 / sc.beta;
          for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB)
            Qv.at(i, (int)(s - s_lo)) = from_d<XT>(A.r[s] * inv);
        } else {
          // second-pass correction of the previous step, applied now, and the
          // implicit residual of column i-1 from the same basis rows
          impl_max = own_form<XT>(Qv, nown, i, L.d, L.z, sc.inv_eta, w1l, psum, psum2);
        }
        // product: gather the complete source vector (r or w1), then scale
        const double inv_src = from_r ? 1.0 / sc.beta : sc.inv_eta;
        for (int64_t base = s_lo + (int64_t)wid * S; base < s_hi; base += SPR) {
          const int64_t s = base + ls;
          const int64_t b = s >> 6;
          const int l = (int)(s & 63);
          double wv;
          if (from_r) {
            const double acc = prow_dot<VT, double, double, G>(A.Pp, b, l, g, A.r);
            wv = ((s < n ? A.r[s] : 0.0) - A.gamma * acc) * inv_src;
          } else {
            const AT acc = prow_dot<VT, XT, AT, G>(A.Pp, b, l, g, A.w1);
            const AT xs = s < n ? (AT)A.w1[s] : (AT)0;
            wv = to_d((XT)((xs - (AT)A.gamma * acc) * (AT)inv_src));
          }
          if (s < n && g == 0) wl[s - s_lo] = wv;
        }
        __syncthreads();
        __syncthreads();  // Q_i of the own rows complete before the projections
        own_dots<XT>(Qv, i + 1, nown, wl, MYPART, false);
        if (threadIdx.x == 0 && !from_r) MYPART[i + 1] = impl_max;  // reduced with max
      }
      IG_BARRIER();
      reduce_rows(PARTS, from_r ? i + 1 : i + 2, 0u, L.c, from_r ? -1 : i + 1);
      __syncthreads();
      if (!from_r) {
        // the stopping test of column i-1, one step late: when the implicit
        // residual (L.c[i+1], overwritten by the Givens update later) says it
        // may hold, confirm on the true FP64 residual with the i columns; if
        // it holds, step i was speculative and is dropped
        if (threadIdx.x == 0) {
          sc.dec = D_NEXT;
          if (!(L.c[i + 1] > sc.thr)) {
            back_sub(L, i);
            sc.dec = D_LAG;
          }
        }
        __syncthreads();
        if (sc.dec == D_LAG) {
          if (!explicit_resid(i)) goto leave;
          if (!(sc.res_inf > sc.thr)) break;  // inner loop done
        }
      }
      // ---------------- [B] w1 = w - Q c; d = Q^T w1; sigma = ||w1||^2
      own_axpy<XT>(Qv, nown, i + 1, L.c, -1.0, psum, [&](int t) { return wl[t]; },
                   [&](int t, double v) {
                     const XT vx = from_d<XT>(v);
                     A.w1[s_lo + t] = vx;
                     w1l[t] = to_d(vx);
                   });
      __syncthreads();
      own_dots<XT>(Qv, i + 1, nown, w1l, MYPART, true);
      IG_BARRIER();
      reduce_rows(PARTS, i + 2, 0u, red);
      // Givens update of column i on wave 0: the element-wise parts on its
      // lanes (j <= i <= 63), the rotation and residual recurrences on lane 0
      // with their operands loaded ahead of the dependent arithmetic
      if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        double dj = 0.0;
        if (lane <= i) {
          dj = red[lane];
          L.d[lane] = dj;
          L.c[lane] += dj;  // column i of H: c + d
        }
        const double dd = wave_sum(dj * dj);
        const double eta = sqrt(fmax(red[i + 1] - dd, 0.0));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane == 0) {
          double* h = L.c;
          h[i + 1] = eta;
          double hj = h[0];
#pragma unroll 4
          for (int j = 0; j < i; ++j) {  // previous rotations
            const double c = L.cs[j], sn = L.sn[j], h1 = h[j + 1];
            h[j] = c * hj + sn * h1;
            hj = -sn * hj + c * h1;
          }
          const double rr = hypot(hj, eta);
          double cs = 1.0, sn = 0.0;
          if (rr > 0.0) {
            cs = hj / rr;
            sn = eta / rr;
          }
          L.cs[i] = cs;
          L.sn[i] = sn;
          h[i] = rr;
          const double gi = L.g[i];
          L.g[i + 1] = -sn * gi;
          L.g[i] = cs * gi;
          // residual of this column's iterate in basis coordinates
          double v = -sn * gi;
#pragma unroll 4
          for (int j = i; j >= 0; --j) {
            const double c = L.cs[j], snj = L.sn[j];
            L.z[j + 1] = c * v;
            v = -snj * v;
          }
          L.z[0] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane <= i) L.R[i * (kPMaxW + 1) + lane] = L.c[lane];
      }
      if (threadIdx.x == 0) {
        // the product, then the method's basis traffic for Q_0..Q_i (read
        // twice, as modified Gram-Schmidt does) and four more vectors; the
        // second classical pass reads the basis once more, not counted
        sc.alg_bytes += A.b_japply + A.b_vec * (2.0 * (i + 1) + 4.0);
        const double eta = L.c[i + 1];
        const double rho = fabs(L.g[i + 1]);
        sc.eta = eta;
        sc.inv_eta = eta > 0.0 ? 1.0 / eta : 0.0;
        sc.rho = rho;
        sc.inner += 1;
        sc.steps_outer += 1;
        int dec = D_NEXT;
        if (!isfinite(eta) || !isfinite(rho)) {
          sc.nonfinite = 1;
          dec = D_ERR;
        } else if (eta == 0.0) {
          sc.breakdowns += 1;
          dec = D_EXPLICIT;
        } else if (!(rho > sc.thr) || sc.steps_outer >= A.max_inner || i + 1 == A.W) {
          // ||r||_inf <= ||r||_2 = rho: the rule holds in exact arithmetic;
          // or the cycle / step budget ends here
          dec = D_EXPLICIT;
        }
        if (dec == D_EXPLICIT) back_sub(L, i + 1);
        sc.dec = dec;
      }
      __syncthreads();
      if (sc.dec == D_ERR) goto leave;
      if (sc.dec == D_NEXT) {
        from_r = false;
        ++i;
        continue;
      }

      // ---------------- explicit test at i+1 columns
      if (!explicit_resid(i + 1)) goto leave;
      if (threadIdx.x == 0) {
        int dec;
        if (sc.eta == 0.0 || sc.res_inf <= sc.thr || sc.steps_outer >= A.max_inner) {
          dec = D_END_INNER;
        } else if (i + 1 == A.W) {
          const double nb = sqrt(sc.res_l2sq);
          if (nb > (1.0 - 1e-6) * sc.cycle_beta) {
            sc.stagnations += 1;
            dec = D_END_INNER;
          } else {
            sc.cycle_beta = nb;
            sc.beta = nb;
            sc.restarts += 1;
            for (int j = 0; j <= kPMaxW; ++j) L.g[j] = 0.0;
            L.g[0] = nb;
            dec = D_RESTART;
          }
        } else {
          dec = D_CONT;
        }
        sc.dec = dec;
      }
      __syncthreads();
      if (sc.dec == D_END_INNER) break;
      if (sc.dec == D_RESTART) {
        for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) A.Vb[s] = A.V[s];
        i = 0;
        from_r = true;
        continue;
      }
      from_r = false;  // D_CONT
      ++i;
    }
  }

leave:
#undef IG_BARRIER
#undef MYPART
#undef PARTS
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    PCtl* c = A.ctl;
    c->outer = sc.outer;
    c->inner = sc.inner;
    c->restarts = sc.restarts;
    c->expl = sc.expl;
    c->breakdowns = sc.breakdowns;
    c->stagnations = sc.stagnations;
    c->converged = sc.converged;
    c->bellman = sc.bellman;
    c->nonfinite = sc.nonfinite;
    c->phi_inf = sc.phi_inf;
    c->alg_bytes = sc.alg_bytes;
    c->dec = sc.dec;
  }
}

template <typename VT, typename XT, int G>
ig_status launch_persist(Mdp& d, const PArgs<VT, XT>& a, int nblocks, bool coop, hipStream_t s) {
  // the block's basis rows go to LDS when they fit beside the static LDS
  const size_t ldq = (size_t)a.spb * kSlice;
  const size_t dyn_w = 2 * ldq * sizeof(double), dyn_q = (size_t)(a.W + 1) * ldq * sizeof(XT);
  hipFuncAttributes fa{};
  const void* kq = (const void*)k_persist<VT, XT, G, true>;
  const void* kg = (const void*)k_persist<VT, XT, G, false>;
  const bool ql = hipFuncGetAttributes(&fa, kq) == hipSuccess &&
                  fa.sharedSizeBytes + dyn_w + dyn_q <= (size_t)d.max_lds;
  (void)hipGetLastError();
  const void* kern = ql ? kq : kg;
  size_t dyn = dyn_w + (ql ? dyn_q : 0);
  // V in LDS for the Bellman pass's gathers, over the same dynamic region
  PArgs<VT, XT> av = a;
  const size_t dyn_v = (size_t)a.n * sizeof(double);
  hipFuncAttributes fk{};
  av.vlds = hipFuncGetAttributes(&fk, kern) == hipSuccess &&
            fk.sharedSizeBytes + std::max(dyn, dyn_v) <= (size_t)d.max_lds;
  (void)hipGetLastError();
  if (av.vlds) dyn = std::max(dyn, dyn_v);
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess)
    (void)hipGetLastError();  // not needed on every runtime; the launch reports real failures
  void* args[] = {(void*)&av};
  ProfScope prof(d, KC_PERSIST, s);
  // A plain launch is used by the serving loop, which keeps every block of
  // all running solves co-resident by admission (cooperative launches are
  // serialised by the runtime).
  if (coop)
    IG_HIP(hipLaunchCooperativeKernel(kern, dim3(nblocks), dim3(kPB), args, (unsigned)dyn, s));
  else
    IG_HIP(hipLaunchKernel(kern, dim3(nblocks), dim3(kPB), args, dyn, s));
  return IG_OK;
}

// Blocks of one solve: `requested` > 0 asks for that many (clamped so that
// a block owns at most kPMaxSpb slices); otherwise a quarter of the slices,
// rounded to whole XCD groups (the measured optimum between per-block work
// and grid-barrier cost for paper-scale sizes).  Depends only on the shape, the request and the CU
// count, never on other work on the device.
int persistent_blocks(const Mdp& d, int* spb_out, int requested = 0) {
  int want = requested > 0 ? requested
                           : (int)std::max<int64_t>(1, std::min<int64_t>(d.nslices, d.nslices / 4));
  if (requested <= 0)
    if (const char* e = std::getenv("IG_PERSIST_BLOCKS")) want = std::max(1, std::atoi(e));
  if (requested <= 0 && want >= 16) want = (want + 4) / 8 * 8;  // nearest whole XCD groups
  const int cap = std::min(kPMaxBlocks, std::max(1, d.num_cu));
  int nb = (int)std::min<int64_t>(std::min<int64_t>(d.nslices, cap), want);
  nb = std::max(nb, (int)((d.nslices + kPMaxSpb - 1) / kPMaxSpb));
  nb = std::min(nb, cap);
  const int spb = (int)((d.nslices + nb - 1) / nb);
  nb = (int)((d.nslices + spb - 1) / spb);
  *spb_out = spb;
  return nb;
}

// Device buffers of one persistent solve: the handle's workspace, or the
// carve-up of the allocation-free entry point's static scratch.
struct PWork {
  void* Q;          // (W+1) x n basis
  void* w1;         // n: once-orthogonalised Arnoldi vector
  double* Vb;       // n: iterate at the start of the restart cycle
  double* r;        // n: Phi_k / explicit residual
  double* part;     // [2][blocks][kPStride] reduction partials
  unsigned* flags;  // [blocks] arrival words (zeroed before the launch)
  PCtl* ctl;        // control block (zeroed before the launch)
};

template <typename VT, typename XT>
ig_status run_typed(Mdp& d, double* V, int32_t* pi, const ig_params& p, bool coop,
                    const PWork& w, hipStream_t s) {
  int spb = 0;
  const int nb = persistent_blocks(d, &spb, p.blocks);
  PArgs<VT, XT> a;
  a.P = SellP<VT>{d.col, (const VT*)d.val, d.off, d.width, d.mcnt, d.adm};
  a.Pp = SellPi<VT>{d.pcol, (VT*)d.pval, d.offp, d.width};
  a.cost = d.cost;
  a.m = d.m;
  a.n = d.n;
  a.nslices = d.nslices;
  a.spb = spb;
  a.gamma = d.gamma;
  a.V = V;
  a.pi = pi;
  a.cpi = d.cpi;
  a.Q = (XT*)w.Q;
  a.w1 = (XT*)w.w1;
  a.Vb = w.Vb;
  a.r = w.r;
  a.part = w.part;
  a.flags = w.flags;  // arrival words, zeroed below
  a.ctl = w.ctl;
  a.alpha = p.alpha;
  a.tol = p.tol;
  a.sqrt_n = std::sqrt((double)d.n);
  a.W = p.restart;
  a.max_outer = p.max_outer;
  a.max_inner = p.max_inner;
  a.forcing = p.forcing;
  a.polish = p.polish;
  // the error path of the barrier wait can be exercised with a tiny limit
  const char* sl = std::getenv("IG_SPIN_LIMIT");
  a.spin_limit = sl ? std::max(0L, std::atol(sl)) : kSpinLimit;
  const double entry = d.vb + 4.0, xb = sizeof(XT);
  a.b_bellman = d.nnz * entry + d.n * (double)d.m * 8 + d.n * 28.0;
  a.b_japply = (double)d.nnz / d.m * entry + d.n * xb * 2;
  a.b_vec = d.n * xb;
  a.b_resid = (double)d.nnz / d.m * entry + d.n * 24.0;
  IG_HIP(hipMemsetAsync(a.flags, 0, (size_t)nb * sizeof(unsigned), s));
  // lanes per state: every thread busy on the own slices
  const int per_state = kPB / (kSlice * spb);
  const int G = per_state >= 16 ? 16 : per_state >= 8 ? 8 : per_state >= 4 ? 4 : per_state >= 2 ? 2 : 1;
  switch (G) {
    case 16: return launch_persist<VT, XT, 16>(d, a, nb, coop, s);
    case 8: return launch_persist<VT, XT, 8>(d, a, nb, coop, s);
    case 4: return launch_persist<VT, XT, 4>(d, a, nb, coop, s);
    case 2: return launch_persist<VT, XT, 2>(d, a, nb, coop, s);
    default: return launch_persist<VT, XT, 1>(d, a, nb, coop, s);
  }
}

}  // namespace

int persistent_grid(const Mdp& d, int requested) {
  int spb = 0;
  return persistent_blocks(d, &spb, requested);
}

bool persistent_fits(const Mdp& d) {
  if (d.fmt != IG_FMT_CSR || d.num_cu <= 0 || d.refine) return false;
  int spb = 0;
  persistent_blocks(d, &spb);
  return spb <= kPMaxSpb && d.n >= 1;
}

namespace {

// work == nullptr: the handle's workspace (allocated or grown here)
ig_status launch_impl(Mdp& d, double* V, int32_t* pi, const ig_params& p, bool coop, hipStream_t s,
                      const PWork* work = nullptr) {
  if (!persistent_fits(d)) return fail(IG_E_TOO_LARGE, "shape does not fit the persistent engine");
  if (p.restart > kPMaxW) return fail(IG_E_TOO_LARGE, "the persistent engine takes restart <= 64");
  if (coop && !d.coop) return fail(IG_E_DEVICE, "device does not support cooperative launches");
  const bool fp32 = p.mode == IG_MODE_MIXED;
  PWork w{};
  if (work) {
    w = *work;
  } else {
    if (ig_status e = ensure_workspace(d, p.restart, fp32)) return e;
    w = PWork{d.ws.Q, d.ws.wA, d.ws.Vb, d.ws.r, d.part, (unsigned*)d.ws.wB, d.pctl};
  }
  IG_HIP(hipMemsetAsync(w.ctl, 0, sizeof(PCtl), s));
  switch (d.store) {
    case IG_FP64:
      return fp32 ? run_typed<double, float>(d, V, pi, p, coop, w, s)
                  : run_typed<double, double>(d, V, pi, p, coop, w, s);
    case IG_FP32:
      return fp32 ? run_typed<float, float>(d, V, pi, p, coop, w, s)
                  : run_typed<float, double>(d, V, pi, p, coop, w, s);
    default:
      return fp32 ? run_typed<bf16, float>(d, V, pi, p, coop, w, s)
                  : run_typed<bf16, double>(d, V, pi, p, coop, w, s);
  }
}

}  // namespace

ig_status persistent_launch(Mdp& d, double* V, int32_t* pi, const ig_params& p, hipStream_t s) {
  if (ig_status e = launch_impl(d, V, pi, p, false, s)) return e;
  IG_HIP(hipMemcpyAsync(d.hpctl, d.pctl, sizeof(PCtl), hipMemcpyDeviceToHost, s));
  return IG_OK;
}

ig_status persistent_collect(Mdp& d, ig_stats& st) {
  const PCtl& c = *d.hpctl;
  st.outer = c.outer;
  st.inner = c.inner;
  st.restarts = c.restarts;
  st.bellman_passes = c.bellman;
  st.explicit_residuals = c.expl;
  st.breakdowns = c.breakdowns;
  st.stagnations = c.stagnations;
  st.converged = c.converged;
  st.res_inf = c.phi_inf;
  st.alg_bytes = c.alg_bytes;
  if (c.err) return fail(IG_E_DEVICE, "persistent solve: grid barrier wait exceeded its limit");
  if (c.nonfinite) return fail(IG_E_NUMERIC, "NaN or Inf during the solve");
  if (!c.converged) return fail(IG_E_NOCONV, "max_outer reached");
  return IG_OK;
}

ig_status persistent_igmres(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                            hipStream_t s) {
  if (ig_status e = launch_impl(d, V, pi, p, true, s)) return e;
  IG_HIP(hipMemcpyAsync(d.hpctl, d.pctl, sizeof(PCtl), hipMemcpyDeviceToHost, s));
  IG_HIP(hipStreamSynchronize(s));
  return persistent_collect(d, st);
}

}  // namespace ig

// ---------------------------------------------------------------------------
// Allocation-free entry point (igmres_pi_solve_noalloc): the whole device
// workspace of one persistent solve comes from a static device array.
// ---------------------------------------------------------------------------
namespace ig {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // IG_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == (size_t)IG_NOALLOC_SCRATCH_BYTES, "header and library disagree");

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of `scratch` on device `dev` (which must be current); looked
// up on the first call per device.
ig_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(IG_E_INVALID, "device ordinal out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(IG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return IG_OK;
}

// Carve the persistent solve's buffers out of [base, base + kScratchBytes);
// IG_E_TOO_LARGE when they do not fit.
ig_status carve(const Mdp& d, const ig_params& p, char* base, PWork* w, size_t* used) {
  int spb = 0;
  const int nb = persistent_blocks(d, &spb, p.blocks);
  const size_t n = (size_t)d.n, xb = p.mode == IG_MODE_MIXED ? 4 : 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base + off;
    off += round_alloc(bytes);
    return (void*)q;
  };
  w->Q = take((size_t)(p.restart + 1) * n * xb);
  w->w1 = take(n * xb);
  w->Vb = (double*)take(n * 8);
  w->r = (double*)take(n * 8);
  w->part = (double*)take((size_t)2 * nb * kPStride * 8);
  w->flags = (unsigned*)take((size_t)nb * sizeof(unsigned));
  w->ctl = (PCtl*)take(sizeof(PCtl));
  *used = off;
  if (off > kScratchBytes)
    return fail(IG_E_TOO_LARGE, "the solve's workspace exceeds IG_NOALLOC_SCRATCH_BYTES");
  return IG_OK;
}

}  // namespace
}  // namespace ig

extern "C" ig_status igmres_pi_solve_noalloc(ig_mdp_t h, double* V, int32_t* pi,
                                             const ig_params* params, ig_stats* stats,
                                             void* stream) {
  using namespace ig;
  Mdp* d = handle_of(h);
  if (!d) return fail(IG_E_INVALID, "NULL handle");
  if (!V || !pi) return fail(IG_E_INVALID, "V and pi are required");
  if (ig_status e = check_params(*d, params, true)) return e;
  const ig_params& p = *params;
  if (p.engine == 1) return fail(IG_E_INVALID, "the allocation-free solve runs the persistent engine");
  if (p.precond != 0) return fail(IG_E_INVALID, "the allocation-free solve has no preconditioner");
  if (d->prof_mask) return fail(IG_E_INVALID, "per-class timing creates events: disable it first");
  int cur = -1;
  IG_HIP(hipGetDevice(&cur));
  if (cur != d->device) return fail(IG_E_INVALID, "the handle's device must be current");
  void* base = nullptr;
  if (ig_status e = scratch_address(cur, &base)) return e;
  PWork w{};
  size_t used = 0;
  if (ig_status e = carve(*d, p, (char*)base, &w, &used)) return e;
  hipStream_t s = (hipStream_t)stream;
  ig_stats st;
  std::memset(&st, 0, sizeof st);
  IG_HIP(hipEventRecord(d->ev0, s));
  ig_status e = launch_impl(*d, V, pi, p, true, s, &w);
  if (e == IG_OK) {
    IG_HIP(hipMemcpyAsync(d->hpctl, w.ctl, sizeof(PCtl), hipMemcpyDeviceToHost, s));
    IG_HIP(hipEventRecord(d->ev1, s));
    IG_HIP(hipEventSynchronize(d->ev1));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, d->ev0, d->ev1);
    e = persistent_collect(*d, st);
    st.time_ms = ms;
    st.cert_bound = st.res_inf / (1.0 - d->gamma);
  }
  if (stats) *stats = st;
  return e;
}
