// Persistent single-launch GMRES(W) policy iteration (Algorithm 2) for
// sparse MDPs that fit one cooperative grid (gfx950).
//
// Every block owns a fixed, contiguous range of 64-state slices for the whole
// solve, so its rows of P, P^pi, Q, w, V stay close to its compute unit.
// Phases are separated by grid barriers; the block that arrives last at a
// barrier reduces the per-block partials in a fixed order, takes the
// control-flow decision, publishes it and releases the barrier, so every
// block follows the same path.  Barrier waits have a spin limit: a wait that
// exceeds it flags an error and every block leaves at its next barrier.
//
// Per Arnoldi step: [A] q = J x over own rows (x = previous vector scaled by
// 1/eta, gathered from the complete buffer), x stored as the next basis
// column, dot products with the basis -> barrier; [B] first CGS correction,
// second-pass dot products -> barrier; [C] second correction, ||w||^2 ->
// barrier (reducer: Givens update of the Hessenberg column and the
// stopping-test bracket).  When the bracket cannot decide, the iterate is
// formed and the true FP64 residual evaluated (two more barriers).
#include "internal.hpp"

namespace ig {

namespace {

constexpr int kPB = 256;             // threads per block
constexpr int kPMaxBlocks = 256;     // grid cap: the reducer tile fits LDS
constexpr int kPMaxSpb = 32;         // slices per block cap
constexpr int kPMaxOwn = kPMaxSpb * kSlice;
constexpr int kPStride = kMaxW + 8;  // doubles per block row of partials
constexpr long kSpinLimit = 1L << 23;

enum Dec : int32_t {
  D_CONTINUE = 0,
  D_DONE,
  D_NOCONV,
  D_ERR_NUMERIC,
  D_NEXT,        // next Arnoldi step
  D_EXPLICIT,    // form the iterate and test the true residual
  D_END_INNER,   // inner loop finished: next outer step
  D_RESTART,     // restart from the explicit residual
  D_CONT_STEP,   // explicit test failed mid-cycle: next Arnoldi step
};

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
  XT* __restrict__ w0;
  XT* __restrict__ w1;
  double* __restrict__ Vb;
  double* __restrict__ r;
  double* __restrict__ part;
  GivensState* __restrict__ gs;
  PCtl* __restrict__ ctl;
  double alpha, tol, sqrt_n;
  int W, max_outer, max_inner, forcing;
  // algorithmic bytes per event, for the statistics
  double b_bellman, b_japply, b_vec, b_resid;
};

struct Pub {  // scalars every block reads after a barrier
  int32_t dec;
  double thr, inv_beta, inv_eta;
};

__device__ __forceinline__ int logical_block() {
  // consecutive hardware blocks go round-robin over the 8 XCDs: give each XCD
  // a contiguous range of slices
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

__device__ __forceinline__ unsigned ld_acq(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier.  `reducer` runs in the last block to arrive (all its threads)
// before the release.  Returns false (uniformly per block) if the solve must
// be abandoned.
template <typename F>
__device__ __forceinline__ bool pbarrier(PCtl* ctl, Pub& pub, F&& reducer) {
  __shared__ unsigned s_gen;
  __shared__ int s_last, s_ok;
  __shared__ Pub s_pub;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = ld_acq(&ctl->gen);
    __threadfence();
    const unsigned a = atomicAdd(&ctl->count, 1u);
    s_gen = g;
    s_last = (a == gridDim.x - 1);
    if (s_last) {
      __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
    }
  }
  __syncthreads();
  if (s_last) {
    reducer();
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (threadIdx.x == 0) {
    long spins = 0;
    while (ld_acq(&ctl->gen) == s_gen) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __threadfence();
  }
  if (threadIdx.x == 0) {
    s_ok = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    s_pub.dec = ctl->dec;
    s_pub.thr = ctl->thr;
    s_pub.inv_beta = ctl->inv_beta;
    s_pub.inv_eta = ctl->inv_eta;
  }
  __syncthreads();
  pub = s_pub;
  return s_ok != 0;
}

// Sum (or max, per bit of maxmask for columns < 32) of part[b][c] over
// blocks, c < cnt, into dst[c]; fixed order.  All threads of the block.
__device__ void reduce_cols(const double* __restrict__ part, int cnt, unsigned maxmask,
                            double* __restrict__ dst) {
  __shared__ double tile[kPMaxBlocks * 32];
  __shared__ double seg[8 * 32];
  const int nb = gridDim.x;
  for (int c0 = 0; c0 < cnt; c0 += 32) {
    const int cw = min(32, cnt - c0);
    for (int e = threadIdx.x; e < nb * 32; e += kPB) {
      const int b = e >> 5, c = e & 31;
      tile[e] = c < cw ? part[(int64_t)b * kPStride + c0 + c] : 0.0;
    }
    __syncthreads();
    const int c = threadIdx.x & 31, q = threadIdx.x >> 5;
    const bool mx = c0 == 0 && ((maxmask >> c) & 1u);
    double acc = 0.0;
    for (int b = q; b < nb; b += 8) acc = mx ? fmax(acc, tile[b * 32 + c]) : acc + tile[b * 32 + c];
    seg[q * 32 + c] = acc;
    __syncthreads();
    if (threadIdx.x < cw) {
      double a = seg[threadIdx.x];
      for (int k = 1; k < 8; ++k) a = mx ? fmax(a, seg[k * 32 + threadIdx.x]) : a + seg[k * 32 + threadIdx.x];
      dst[c0 + threadIdx.x] = a;
    }
    __syncthreads();
  }
}

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], const int (&op)[NV], double* mypart) {
  block_reduce<NV>(v, op);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) mypart[k] = v[k];
  }
}

template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT prow_dot(const SellPi<VT>& Pp, int64_t b, int l, int g,
                                       const XT* __restrict__ x, XT scale) {
  constexpr int S = kWave / G;
  const int Kb = Pp.width[b];
  const int64_t ob = Pp.off[b] + l;
  AT acc = 0;
  for (int j = g; j < Kb; j += G) {
    const int64_t e = ob + ((int64_t)j << 6);
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

// partial dot products of the own rows of Q_0..Q_{i-1} with wl (LDS) into
// mypart[0..i): groups of 8 threads per dot, 32 dots per round
template <typename XT>
__device__ __forceinline__ void own_dots(const XT* __restrict__ Q, int64_t n, int i, int64_t s_lo,
                                         int nown, const double* __restrict__ wl, double* mypart) {
  const int sub = threadIdx.x & 7;
  for (int j0 = 0; j0 < i; j0 += kPB / 8) {
    const int j = j0 + (threadIdx.x >> 3);
    double acc = 0.0;
    if (j < i) {
      const XT* q = Q + (int64_t)j * n + s_lo;
      for (int t = sub; t < nown; t += 8) acc = fma(to_d(q[t]), wl[t], acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (sub == 0 && j < i) mypart[j] = acc;
  }
}

template <typename VT, typename XT, int G>
__global__ __launch_bounds__(kPB) void k_persist(PArgs<VT, XT> A) {
  using AT = XT;
  constexpr int S = kWave / G;
  constexpr int SPR = S * (kPB / kWave);  // states per round
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int ls = lane % S, g = lane / S;
  const int lb = logical_block();
  const int64_t sl0 = (int64_t)lb * A.spb;
  const int64_t sl1 = min<int64_t>(A.nslices, sl0 + A.spb);
  const int64_t s_lo = sl0 * kSlice, s_hi = sl1 * kSlice;  // padded own range
  const int64_t v_hi = min<int64_t>(s_hi, A.n);            // valid own states
  const int nown = (int)max<int64_t>(0, v_hi - s_lo);
  const int64_t n = A.n;
  double* mypart = A.part + (int64_t)blockIdx.x * kPStride;
  PCtl* ctl = A.ctl;
  GivensState* gs = A.gs;

  __shared__ double wl[kPMaxOwn];
  __shared__ double coef[kMaxW + 1];

  Pub pub;
  int i = 1;
  XT* wcur = A.w0;
  XT* wprev = A.w1;
  const XT* xsrc = nullptr;  // vector gathered by the next product
  XT xscale = 1;
  bool src_is_r = true;

  for (int k = 0;; ++k) {
    // ---------------- Bellman pass: pi_k, Phi_k = T V_k - V_k, g^pi, P^pi
    {
      double pmax = 0.0, psum = 0.0, nonfin = 0.0;
      for (int64_t base = s_lo + (int64_t)wid * S; base < s_hi; base += SPR) {
        const int64_t s = base + ls;
        const bool valid = s < n;
        const int64_t sc = valid ? s : n - 1;
        const int64_t b = s >> 6;
        const int l = (int)(s & 63);
        const int Kb = A.P.width[b];
        const int64_t ob = A.P.off[b];
        double best = INFINITY;
        int besta = A.m;
        for (int a = g; a < A.m; a += G) {
          const int64_t bs = ob + (((int64_t)a * Kb) << 6) + l;
          double acc = 0.0;
          for (int j = 0; j < Kb; ++j) {
            const int64_t e = bs + ((int64_t)j << 6);
            acc = fma(to_d(A.P.val[e]), A.V[A.P.col[e]], acc);
          }
          const double q = A.cost[(int64_t)a * n + sc] + A.gamma * acc;
          if (!(q - q == 0.0)) nonfin += valid ? 1.0 : 0.0;
          if (q < best) {
            best = q;
            besta = a;
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
        }
        if (besta >= A.m) {
          besta = 0;
          best = NAN;
        }
        if (valid && g == 0) {
          const double phi = best - A.V[s];
          A.r[s] = phi;
          A.pi[s] = besta;
          A.cpi[s] = A.cost[(int64_t)besta * n + s];
          if (!(phi - phi == 0.0)) nonfin += 1.0;
          pmax = fmax(pmax, fabs(phi));
          psum = fma(phi, phi, psum);
        }
        const int64_t src = ob + (((int64_t)besta * Kb) << 6) + l;
        const int64_t dst = A.Pp.off[b] + l;
        for (int j = g; j < Kb; j += G) {
          A.Pp.col[dst + ((int64_t)j << 6)] = A.P.col[src + ((int64_t)j << 6)];
          A.Pp.val[dst + ((int64_t)j << 6)] = A.P.val[src + ((int64_t)j << 6)];
        }
      }
      double v[3] = {pmax, psum, nonfin};
      const int op[3] = {1, 0, 0};
      write_partials<3>(v, op, mypart);
    }
    const int kk = k;
    if (!pbarrier(ctl, pub, [&]() {
          __shared__ double red[3];
          reduce_cols(A.part, 3, 1u, red);
          if (threadIdx.x == 0) {
            ctl->bellman += 1;
            ctl->alg_bytes += A.b_bellman;
            ctl->phi_inf = red[0];
            ctl->phi_l2sq = red[1];
            ctl->outer = kk;
            ctl->res_inf = red[0];
            int32_t dec;
            if (red[2] != 0.0) {
              ctl->nonfinite = 1;
              dec = D_ERR_NUMERIC;
            } else if (red[0] <= A.tol) {
              ctl->converged = 1;
              dec = D_DONE;
            } else if (kk >= A.max_outer) {
              dec = D_NOCONV;
            } else {
              const double alpha = A.forcing ? fmin(A.alpha, sqrt(red[0])) : A.alpha;
              const double beta = sqrt(red[1]);
              ctl->thr = alpha * red[0];
              ctl->cycle_beta = beta;
              ctl->inv_beta = 1.0 / beta;
              ctl->steps_outer = 0;
              for (int j = 0; j <= kMaxW; ++j) gs->g[j] = 0.0;
              gs->g[0] = beta;
              dec = D_CONTINUE;
            }
            ctl->dec = dec;
          }
        }))
      return;
    if (pub.dec != D_CONTINUE) return;

    // cycle start: Vb = V (own rows), x = Phi / beta
    for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) A.Vb[s] = A.V[s];
    i = 1;
    xsrc = nullptr;
    src_is_r = true;
    xscale = (XT)pub.inv_beta;
    double inv_eta = 0.0;

    for (;;) {
      // ---------------- [A] q = J x; x becomes basis column i-1
      {
        XT* qcol = A.Q + (int64_t)(i - 1) * n;
        for (int64_t base = s_lo + (int64_t)wid * S; base < s_hi; base += SPR) {
          const int64_t s = base + ls;
          const int64_t b = s >> 6;
          const int l = (int)(s & 63);
          AT acc;
          XT xs;
          if (src_is_r) {
            // first vector of a cycle: gathered from the FP64 residual
            const double* rr = A.r;
            AT a2 = 0;
            const int Kb = A.Pp.width[b];
            const int64_t ob = A.Pp.off[b] + l;
            for (int j = g; j < Kb; j += G) {
              const int64_t e = ob + ((int64_t)j << 6);
              const XT xv = (XT)(rr[A.Pp.col[e]] * (double)xscale);
              if constexpr (sizeof(AT) == 8)
                a2 = fma(to_d(A.Pp.val[e]), (AT)xv, a2);
              else
                a2 = fmaf(to_f(A.Pp.val[e]), (AT)xv, a2);
            }
#pragma unroll
            for (int o = S; o < kWave; o <<= 1) a2 += __shfl_xor(a2, o);
            acc = a2;
            xs = s < n ? (XT)(rr[s] * (double)xscale) : (XT)0;
          } else {
            acc = prow_dot<VT, XT, AT, G>(A.Pp, b, l, g, xsrc, xscale);
            xs = s < n ? xsrc[s] * xscale : (XT)0;
          }
          if (s < n && g == 0) {
            qcol[s] = xs;
            const XT wv = (XT)((AT)xs - (AT)A.gamma * acc);
            wcur[s] = wv;
            wl[s - s_lo] = to_d(wv);
          }
        }
        __syncthreads();
        own_dots<XT>(A.Q, n, i, s_lo, nown, wl, mypart);
      }
      const int ii = i;
      if (!pbarrier(ctl, pub, [&]() {
            reduce_cols(A.part, ii, 0u, gs->h);
            if (threadIdx.x == 0) ctl->alg_bytes += A.b_japply + A.b_vec * (ii + 1);
          }))
        return;

      // ---------------- [B] first correction, second-pass dots
      for (int j = threadIdx.x; j < i; j += kPB) coef[j] = gs->h[j];
      __syncthreads();
      for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) {
        double ws = wl[s - s_lo];
        for (int j = 0; j < i; ++j) ws = fma(-coef[j], to_d(A.Q[(int64_t)j * n + s]), ws);
        const XT wx = from_d<XT>(ws);
        wcur[s] = wx;
        wl[s - s_lo] = to_d(wx);
      }
      __syncthreads();
      own_dots<XT>(A.Q, n, i, s_lo, nown, wl, mypart);
      if (!pbarrier(ctl, pub, [&]() {
            reduce_cols(A.part, ii, 0u, gs->h2);
            if (threadIdx.x == 0) ctl->alg_bytes += A.b_vec * (2 * ii + 2);
          }))
        return;

      // ---------------- [C] second correction, ||w||^2
      for (int j = threadIdx.x; j < i; j += kPB) coef[j] = gs->h2[j];
      __syncthreads();
      {
        double nrm = 0.0;
        for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) {
          double ws = wl[s - s_lo];
          for (int j = 0; j < i; ++j) ws = fma(-coef[j], to_d(A.Q[(int64_t)j * n + s]), ws);
          const XT wx = from_d<XT>(ws);
          wcur[s] = wx;
          const double wd = to_d(wx);
          nrm = fma(wd, wd, nrm);
        }
        double v[1] = {nrm};
        const int op[1] = {0};
        write_partials<1>(v, op, mypart);
      }
      if (!pbarrier(ctl, pub, [&]() {
            __shared__ double red[1];
            reduce_cols(A.part, 1, 0u, red);
            if (threadIdx.x == 0) {
              ctl->alg_bytes += A.b_vec * (ii + 2);
              const double eta = sqrt(red[0]);
              const int col = ii - 1;
              double* h = gs->h;
              for (int j = 0; j < ii; ++j) h[j] += gs->h2[j];
              h[ii] = eta;
              for (int j = 0; j < col; ++j) {
                const double t = gs->cs[j] * h[j] + gs->sn[j] * h[j + 1];
                h[j + 1] = -gs->sn[j] * h[j] + gs->cs[j] * h[j + 1];
                h[j] = t;
              }
              const double rr = hypot(h[col], h[col + 1]);
              double cs = 1.0, sn = 0.0;
              if (rr > 0.0) {
                cs = h[col] / rr;
                sn = h[col + 1] / rr;
              }
              gs->cs[col] = cs;
              gs->sn[col] = sn;
              h[col] = rr;
              h[col + 1] = 0.0;
              gs->g[col + 1] = -sn * gs->g[col];
              gs->g[col] = cs * gs->g[col];
              for (int j = 0; j <= col; ++j) gs->R[(int64_t)col * (kMaxW + 1) + j] = h[j];
              const double rho = fabs(gs->g[col + 1]);
              ctl->eta = eta;
              ctl->rho = rho;
              ctl->inv_eta = eta > 0.0 ? 1.0 / eta : 0.0;
              ctl->inner += 1;
              ctl->steps_outer += 1;
              int32_t dec = D_NEXT;
              ctl->breakdown_flag = 0;
              ctl->restart_req = 0;
              if (!isfinite(eta) || !isfinite(rho)) {
                ctl->nonfinite = 1;
                dec = D_ERR_NUMERIC;
              } else if (eta == 0.0) {
                ctl->breakdown_flag = 1;
                ctl->breakdowns += 1;
                dec = D_EXPLICIT;
              } else if (!(rho > A.sqrt_n * ctl->thr) || ctl->steps_outer >= A.max_inner) {
                dec = D_EXPLICIT;
              } else if (ii == A.W) {
                ctl->restart_req = 1;
                dec = D_EXPLICIT;
              }
              if (dec == D_EXPLICIT) {
                if (ii == A.W) ctl->restart_req = 1;
                for (int j = ii - 1; j >= 0; --j) {  // R y = g_hat
                  double a = gs->g[j];
                  for (int l2 = j + 1; l2 < ii; ++l2) a -= gs->R[(int64_t)l2 * (kMaxW + 1) + j] * gs->y[l2];
                  const double dj = gs->R[(int64_t)j * (kMaxW + 1) + j];
                  gs->y[j] = dj != 0.0 ? a / dj : 0.0;
                }
              }
              ctl->dec = dec;
            }
          }))
        return;
      if (pub.dec == D_ERR_NUMERIC) return;
      inv_eta = pub.inv_eta;
      if (pub.dec == D_NEXT) {
        xsrc = wcur;
        xscale = (XT)inv_eta;
        src_is_r = false;
        XT* t = wcur;
        wcur = wprev;
        wprev = t;
        ++i;
        continue;
      }

      // ---------------- explicit test: V = Vb + Q y, r = g - J V (FP64)
      for (int j = threadIdx.x; j < i; j += kPB) coef[j] = gs->y[j];
      __syncthreads();
      for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) {
        double v = A.Vb[s];
        for (int j = 0; j < i; ++j) v = fma(coef[j], to_d(A.Q[(int64_t)j * n + s]), v);
        A.V[s] = v;
      }
      if (!pbarrier(ctl, pub, [&]() {}))
        return;
      {
        double pmax = 0.0, psum = 0.0, vmax = 0.0;
        for (int64_t base = s_lo + (int64_t)wid * S; base < s_hi; base += SPR) {
          const int64_t s = base + ls;
          const int64_t b = s >> 6;
          const int l = (int)(s & 63);
          const double acc = prow_dot<VT, double, double, G>(A.Pp, b, l, g, A.V, 1.0);
          if (s < n && g == 0) {
            const double rr = A.cpi[s] - (A.V[s] - A.gamma * acc);
            A.r[s] = rr;
            pmax = fmax(pmax, fabs(rr));
            psum = fma(rr, rr, psum);
            vmax = fmax(vmax, fabs(A.V[s]));
          }
        }
        double v[3] = {pmax, psum, vmax};
        const int op[3] = {1, 0, 1};
        write_partials<3>(v, op, mypart);
      }
      if (!pbarrier(ctl, pub, [&]() {
            __shared__ double red[3];
            reduce_cols(A.part, 3, 5u, red);
            if (threadIdx.x == 0) {
              ctl->alg_bytes += A.b_resid + A.b_vec * ii;
              ctl->expl += 1;
              ctl->res_l2sq = red[1];
              ctl->vmax = red[2];
              int32_t dec;
              if (ctl->breakdown_flag || red[0] <= ctl->thr || ctl->steps_outer >= A.max_inner) {
                dec = D_END_INNER;
              } else if (ctl->restart_req) {
                const double nb = sqrt(red[1]);
                if (nb > (1.0 - 1e-6) * ctl->cycle_beta) {
                  ctl->stagnations += 1;
                  dec = D_END_INNER;
                } else {
                  ctl->cycle_beta = nb;
                  ctl->inv_beta = 1.0 / nb;
                  ctl->restarts += 1;
                  for (int j = 0; j <= kMaxW; ++j) gs->g[j] = 0.0;
                  gs->g[0] = nb;
                  dec = D_RESTART;
                }
              } else {
                dec = D_CONT_STEP;
              }
              ctl->dec = dec;
            }
          }))
        return;
      if (pub.dec == D_END_INNER) break;
      if (pub.dec == D_RESTART) {
        for (int64_t s = s_lo + threadIdx.x; s < v_hi; s += kPB) A.Vb[s] = A.V[s];
        i = 1;
        src_is_r = true;
        xscale = (XT)pub.inv_beta;
        continue;
      }
      // D_CONT_STEP
      xsrc = wcur;
      xscale = (XT)inv_eta;
      src_is_r = false;
      XT* t = wcur;
      wcur = wprev;
      wprev = t;
      ++i;
    }
  }
}

template <typename VT, typename XT, int G>
ig_status launch_persist(Mdp& d, const PArgs<VT, XT>& a, int nblocks, hipStream_t s) {
  void* args[] = {(void*)&a};
  ProfScope prof(d, KC_PERSIST, s);
  IG_HIP(hipLaunchCooperativeKernel((const void*)k_persist<VT, XT, G>, dim3(nblocks), dim3(kPB),
                                    args, 0, s));
  return IG_OK;
}

template <typename VT, typename XT>
ig_status run_typed(Mdp& d, double* V, int32_t* pi, const ig_params& p, int nblocks, int spb,
                    hipStream_t s) {
  PArgs<VT, XT> a;
  a.P = SellP<VT>{d.col, (const VT*)d.val, d.off, d.width};
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
  a.Q = (XT*)d.ws.Q;
  a.w0 = (XT*)d.ws.wA;
  a.w1 = (XT*)d.ws.wB;
  a.Vb = d.ws.Vb;
  a.r = d.ws.r;
  a.part = d.part;
  a.gs = d.gs;
  a.ctl = d.pctl;
  a.alpha = p.alpha;
  a.tol = p.tol;
  a.sqrt_n = std::sqrt((double)d.n);
  a.W = p.restart;
  a.max_outer = p.max_outer;
  a.max_inner = p.max_inner;
  a.forcing = p.forcing;
  const double entry = d.vb + 4.0, xb = sizeof(XT);
  a.b_bellman = d.nnz * entry + d.n * (double)d.m * 8 + d.n * 28.0;
  a.b_japply = (double)d.nnz / d.m * entry + d.n * xb * 3;
  a.b_vec = d.n * xb;
  a.b_resid = (double)d.nnz / d.m * entry + d.n * 24.0;
  const int G = spb == 1 ? 4 : (spb == 2 ? 2 : 1);
  switch (G) {
    case 4: return launch_persist<VT, XT, 4>(d, a, nblocks, s);
    case 2: return launch_persist<VT, XT, 2>(d, a, nblocks, s);
    default: return launch_persist<VT, XT, 1>(d, a, nblocks, s);
  }
}

int persistent_blocks(const Mdp& d, int* spb_out) {
  const int cap = std::min(kPMaxBlocks, std::max(1, d.num_cu));
  int nb = (int)std::min<int64_t>(d.nslices, cap);
  int spb = (int)((d.nslices + nb - 1) / nb);
  nb = (int)((d.nslices + spb - 1) / spb);
  *spb_out = spb;
  return nb;
}

}  // namespace

int persistent_grid(const Mdp& d) {
  int spb = 0;
  return persistent_blocks(d, &spb);
}

bool persistent_fits(const Mdp& d) {
  if (d.fmt != IG_FMT_CSR || !d.coop || d.num_cu <= 0) return false;
  int spb = 0;
  persistent_blocks(d, &spb);
  return spb <= kPMaxSpb;
}

ig_status persistent_igmres(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                            hipStream_t s) {
  if (!persistent_fits(d)) return fail(IG_E_TOO_LARGE, "shape does not fit the persistent engine");
  const bool fp32 = p.mode == IG_MODE_MIXED;
  if (ig_status e = ensure_workspace(d, p.restart, fp32)) return e;
  int spb = 0;
  const int nb = persistent_blocks(d, &spb);
  IG_HIP(hipMemsetAsync(d.pctl, 0, sizeof(PCtl), s));
  ig_status e;
  switch (d.store) {
    case IG_FP64:
      e = fp32 ? run_typed<double, float>(d, V, pi, p, nb, spb, s)
               : run_typed<double, double>(d, V, pi, p, nb, spb, s);
      break;
    case IG_FP32:
      e = fp32 ? run_typed<float, float>(d, V, pi, p, nb, spb, s)
               : run_typed<float, double>(d, V, pi, p, nb, spb, s);
      break;
    default:
      e = fp32 ? run_typed<bf16, float>(d, V, pi, p, nb, spb, s)
               : run_typed<bf16, double>(d, V, pi, p, nb, spb, s);
      break;
  }
  if (e) return e;
  IG_HIP(hipMemcpyAsync(d.hpctl, d.pctl, sizeof(PCtl), hipMemcpyDeviceToHost, s));
  IG_HIP(hipStreamSynchronize(s));
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

}  // namespace ig
