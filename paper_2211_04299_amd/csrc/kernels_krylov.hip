// Arnoldi orthogonalisation, Givens-rotated Hessenberg least squares and the
// solution update of GMRES(W) (Algorithm 2 of the paper, inner loop), one
// kernel launch per step.
//
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2), which in
// exact arithmetic gives the Hessenberg column of the modified Gram-Schmidt
// loop of Algorithm 2 with one reduction per pass.  For column c:
//   y  = J x / eta            (x = the previous once-orthogonalised vector w1)
//   h  = Q^T y                 (k_dots + finalize)
//   w1 = y - Q h               (k_axpy)
//   d  = Q^T w1, sigma = ||w1||^2  (k_dots + finalize: Givens update)
// The second-pass correction is applied lazily when the next basis vector is
// formed, Q_{c+1} = (w1 - Q d) / eta with eta = sqrt(sigma - ||d||^2): d is of
// the order of the rounding error, so the product J w1 / eta equals J Q_{c+1}
// to that order and Pythagoras loses nothing.  The same pass evaluates the
// residual of the previous column's iterate as Q z (z = the least-squares
// residual rotated back to basis coordinates), whose infinity-norm equals the
// true residual's in exact arithmetic.
// Every dot product and norm accumulates in FP64; per-block partials are
// combined in a fixed order by one block: in the fused passes (k_gs_a,
// k_gs_b) the block that finishes last, otherwise the one-block k_finalize
// launched next.  (The lines above name the separate kernels of the path
// for columns beyond the register buckets; the fused passes do the same
// work in two launches.)
#include "internal.hpp"

namespace ig {

namespace {

constexpr int kJC = 8;       // dot products per sweep
constexpr int kFinT = 1024;  // threads of the finishing kernel
constexpr int kGsT = 512;    // threads per block of the fused Gram-Schmidt passes
constexpr int kGsB = 256;    // their grid cap (as many threads as 512 blocks of 256)
constexpr int kFinBatch = 16;  // partial rows each finishing thread loads at once
constexpr int kUpdStage = 64;  // columns of R the solution update stages in LDS

template <typename XT>
__device__ __forceinline__ const XT* qcol(const XT* Q, int64_t n, int j) {
  return Q + (int64_t)j * n;
}

// partial dot products <Q_j, v>, j < cnt, (+ ||v||^2 as column cnt when
// with_norm), written to part[blockIdx.x * kPartStride + j]
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_dots(const XT* __restrict__ Q, int64_t n, int cnt,
                                                 const XT* __restrict__ v, int with_norm,
                                                 double* __restrict__ part) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t s0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double* mypart = part + (int64_t)blockIdx.x * kPartStride;
  const int op[kJC] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int j0 = 0; j0 < cnt; j0 += kJC) {
    double acc[kJC], acc2[kJC];
#pragma unroll
    for (int k = 0; k < kJC; ++k) acc[k] = acc2[k] = 0.0;
    int64_t s = s0;
    for (; s + stride < n; s += 2 * stride) {  // two states per thread in flight
      const double v0 = to_d(v[s]), v1 = to_d(v[s + stride]);
#pragma unroll
      for (int k = 0; k < kJC; ++k)
        if (j0 + k < cnt) {
          const XT* q = qcol(Q, n, j0 + k);
          acc[k] = fma(to_d(q[s]), v0, acc[k]);
          acc2[k] = fma(to_d(q[s + stride]), v1, acc2[k]);
        }
    }
    if (s < n) {
      const double v0 = to_d(v[s]);
#pragma unroll
      for (int k = 0; k < kJC; ++k)
        if (j0 + k < cnt) acc[k] = fma(to_d(qcol(Q, n, j0 + k)[s]), v0, acc[k]);
    }
#pragma unroll
    for (int k = 0; k < kJC; ++k) acc[k] += acc2[k];
    block_reduce<kJC>(acc, op);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < kJC; ++k)
        if (j0 + k < cnt) mypart[j0 + k] = acc[k];
    }
  }
  if (with_norm) {
    double nrm[1] = {0.0};
    for (int64_t s = s0; s < n; s += stride) {
      const double vs = to_d(v[s]);
      nrm[0] = fma(vs, vs, nrm[0]);
    }
    const int op1[1] = {0};
    block_reduce<1>(nrm, op1);
    if (threadIdx.x == 0) mypart[cnt] = nrm[0];
  }
}

// w1 = y - sum_{j<cnt} h_j Q_j
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_axpy(const XT* __restrict__ Q, int64_t n, int cnt,
                                                 const GivensState* __restrict__ gs,
                                                 const XT* __restrict__ y, XT* __restrict__ w1) {
  __shared__ double c[kMaxW + 1];
  for (int j = threadIdx.x; j < cnt; j += kBlock) c[j] = gs->h[j];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
    double a0 = to_d(y[s]), a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
      const double q0 = to_d(qcol(Q, n, j)[s]), q1 = to_d(qcol(Q, n, j + 1)[s]);
      const double q2 = to_d(qcol(Q, n, j + 2)[s]), q3 = to_d(qcol(Q, n, j + 3)[s]);
      a0 = fma(-c[j], q0, a0);
      a1 = fma(-c[j + 1], q1, a1);
      a2 = fma(-c[j + 2], q2, a2);
      a3 = fma(-c[j + 3], q3, a3);
    }
    for (; j < cnt; ++j) a0 = fma(-c[j], to_d(qcol(Q, n, j)[s]), a0);
    w1[s] = from_d<XT>((a0 + a1) + (a2 + a3));
  }
}

// Q_c = (w1 - sum_{j<c} d_j Q_j) / eta; implicit residual of column c-1:
// r(s) = sum_{j<=c} z_j Q_j(s); the block's max|r| goes to the spare last
// column of its Gram-Schmidt partial row (reduced with the next dot pass).
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_form_qi(XT* __restrict__ Q, int64_t n, int c,
                                                    const XT* __restrict__ w1,
                                                    const GivensState* __restrict__ gs,
                                                    const DevStatus* __restrict__ st,
                                                    double* __restrict__ part) {
  __shared__ double dd[kMaxW + 1], zz[kMaxW + 2];
  for (int j = threadIdx.x; j < c; j += kBlock) dd[j] = gs->h2[j];
  for (int j = threadIdx.x; j <= c; j += kBlock) zz[j] = gs->z[j];
  __syncthreads();
  const double inv = 1.0 / st->eta;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double rmax = 0.0;
  XT* qc = Q + (int64_t)c * n;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
    double corr = 0.0, r = 0.0, corr2 = 0.0, r2 = 0.0;
    int j = 0;
    for (; j + 2 <= c; j += 2) {
      const double q0 = to_d(qcol(Q, n, j)[s]), q1 = to_d(qcol(Q, n, j + 1)[s]);
      corr = fma(dd[j], q0, corr);
      r = fma(zz[j], q0, r);
      corr2 = fma(dd[j + 1], q1, corr2);
      r2 = fma(zz[j + 1], q1, r2);
    }
    if (j < c) {
      const double q0 = to_d(qcol(Q, n, j)[s]);
      corr = fma(dd[j], q0, corr);
      r = fma(zz[j], q0, r);
    }
    const XT qx = from_d<XT>((to_d(w1[s]) - (corr + corr2)) * inv);
    qc[s] = qx;
    r = fma(zz[c], to_d(qx), r + r2);
    rmax = fmax(rmax, fabs(r));
  }
  double v[1] = {rmax};
  const int op[1] = {1};
  block_reduce<1>(v, op);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kPartStride + kPartStride - 1] = v[0];
}

template <int NT>
__device__ void finish(int kind, const double* __restrict__ part, int nb, int cnt, int stride,
                       unsigned maxmask, int with_impl, DevStatus* __restrict__ st,
                       GivensState* __restrict__ gs, StepSnap* __restrict__ snap);

// True (uniformly in the block) for the block of the grid that finishes
// last.  Thread 0 has written the block's partial row; its arrival is an
// acquire-release increment of the counter, so the last block sees every
// row.  The last block resets the counter for the next launch.
__device__ __forceinline__ bool last_to_finish(uint32_t* arrive) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = old == gridDim.x - 1;
    if (s_last) __hip_atomic_store(arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (!s_last) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// ---- fused Gram-Schmidt step: two passes over the basis per column -------
// Every thread owns one state row at a time and keeps that row of the basis
// (at most JM columns) in registers, so each pass reads the basis once.
//   pass A (column c): Q_c = (w1 - sum_{j<c} d_j Q_j) / eta, the implicit
//     residual sum_{j<=c} z_j Q_j of column c-1, and h_j = <Q_j, y>, j <= c
//     (at c = 0 only h_0 = <Q_0, y>)
//   pass B: w1 = y - sum_{j<=c} h_j Q_j, d_j = <Q_j, w1>, sigma = ||w1||^2
// Partials: per block, columns 0..cnt-1 (+ sigma at cnt for B; the implicit
// residual's max in the spare last column for A).  The block that finishes
// last reduces them (no separate finishing launch): 512-thread blocks, at
// most 256 of them, so that one block sums the rows in two rounds of loads.

template <int JM, int NT>
__device__ __forceinline__ void store_cols(double (&acc)[JM], int cnt, double* mypart) {
  constexpr int op8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int j0 = 0; j0 < JM; j0 += 8) {
    if (j0 >= cnt) break;  // uniform over the block
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = acc[j0 + k];
    block_reduce<8, NT>(t, op8);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (j0 + k < cnt) mypart[j0 + k] = t[k];
    }
  }
}

// Row of the basis at state s into q[0..JM): column min(j, cnt-1) (column 0
// when cnt == 0), so every load is in bounds and finite and all JM loads are
// issued back to back without branches (the repeats hit in cache).  Callers
// give columns >= cnt zero coefficients and discard their dot products.
template <typename XT, int JM>
__device__ __forceinline__ void load_row(const XT* __restrict__ Q, int64_t n, int cnt, int64_t s,
                                         XT (&q)[JM]) {
  const int last = cnt > 0 ? cnt - 1 : 0;
#pragma unroll
  for (int j = 0; j < JM; ++j) q[j] = Q[(int64_t)min(j, last) * n + s];
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }

template <typename XT, int JM>
__global__ __launch_bounds__(kGsT) void k_gs_a(XT* __restrict__ Q, int64_t n, int c,
                                                 const XT* __restrict__ w1,
                                                 const XT* __restrict__ y,
                                                 GivensState* __restrict__ gs,
                                                 DevStatus* __restrict__ st,
                                                 double* __restrict__ part) {
  // The second-pass correction and the implicit residual accumulate in the
  // basis type: with an FP32 basis their rounding is that of the stored
  // vector they feed (the dot products below stay FP64).
  using CT = XT;
  __shared__ CT dd[JM], zz[JM];
  for (int j = threadIdx.x; j < JM; j += kGsT) {
    dd[j] = (CT)(j < c ? gs->h2[j] : 0.0);
    zz[j] = (CT)(j < c ? gs->z[j] : 0.0);
  }
  __syncthreads();
  const double zc = gs->z[c];
  const double inv = c > 0 ? 1.0 / st->eta : 0.0;
  double acc[JM];
#pragma unroll
  for (int j = 0; j < JM; ++j) acc[j] = 0.0;
  double accc = 0.0, rmax = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kGsT;
  XT* qc = Q + (int64_t)c * n;
  const int64_t s0 = (int64_t)blockIdx.x * kGsT + threadIdx.x;
  // Rows are visited from the last grid-sized chunk down to the first, the
  // opposite order of pass B and of the product before this pass: the rows
  // one pass touched last are still in the memory-side cache when the next
  // pass starts on them.
  // y and w1 of the next row are loaded one iteration ahead (index clamped
  // into range), so that their latency overlaps the basis loads; for rows of
  // up to 128 bytes (32 FP32 or 16 FP64 columns) the next row of the basis
  // is loaded ahead too (the grid keeps two wavefronts per SIMD, so the
  // registers are there)
  constexpr bool PF = JM * sizeof(XT) <= 128;
  int64_t sb = ((n + stride - 1) / stride - 1) * stride + s0;  // s0 + k*stride < n, k largest
  if (sb >= n) sb -= stride;
  const int64_t s1 = max<int64_t>(0, min(sb, n - 1));
  XT yn = y[s1], wn = w1[s1];
  XT qn[PF ? JM : 1];
  if constexpr (PF) load_row<XT, JM>(Q, n, c, s1, qn);
  for (int64_t s = sb; s >= 0; s -= stride) {
    // re-read the LDS coefficients per row instead of holding 2*JM doubles
    // in registers
    asm volatile("" ::: "memory");
    const XT yv = yn, wv = wn, q0v = Q[s];
    const int64_t sn = max<int64_t>(0, s - stride);
    yn = y[sn];
    wn = w1[sn];
    XT q[JM];
    if constexpr (PF) {
#pragma unroll
      for (int j = 0; j < JM; ++j) q[j] = qn[j];
      load_row<XT, JM>(Q, n, c, sn, qn);
    } else {
      load_row<XT, JM>(Q, n, c, s, q);
    }
    const double ys = to_d(yv);
    CT corr0 = 0, corr1 = 0, r0 = 0, r1 = 0;
#pragma unroll
    for (int g = 0; g < JM; g += 8) {
      asm volatile("" ::: "memory");  // at most 8 coefficient pairs live
#pragma unroll
      for (int j = g; j < g + 8; j += 2) {
        corr0 = fma_t(dd[j], q[j], corr0);
        r0 = fma_t(zz[j], q[j], r0);
        corr1 = fma_t(dd[j + 1], q[j + 1], corr1);
        r1 = fma_t(zz[j + 1], q[j + 1], r1);
      }
    }
    const XT qx = from_d<XT>((to_d(wv) - to_d(corr0 + corr1)) * inv);
    if (c > 0) qc[s] = qx;
    const double qcs = c > 0 ? to_d(qx) : to_d(q0v);
    const double rr = fabs(fma(zc, qcs, to_d(r0 + r1)));
    rmax = c > 0 ? fmax(rmax, rr) : rmax;
#pragma unroll
    for (int j = 0; j < JM; ++j) acc[j] = fma(to_d(q[j]), ys, acc[j]);
    accc = fma(qcs, ys, accc);
  }
#pragma unroll
  for (int j = 0; j < JM; ++j)
    if (j == c) acc[j] = accc;
  double* mypart = part + (int64_t)blockIdx.x * kPartStride;
  store_cols<JM, kGsT>(acc, c + 1, mypart);
  if (c > 0) {
    double v[1] = {rmax};
    const int op[1] = {1};
    block_reduce<1, kGsT>(v, op);
    if (threadIdx.x == 0) mypart[kPartStride - 1] = v[0];
  }
  // the block that finishes last reduces h (and the implicit residual)
  if (last_to_finish(&st->arrive))
    finish<kGsT>(FIN_DOTS, part, gridDim.x, c + 1, kPartStride, 0u, c > 0, st, gs, nullptr);
}

template <typename XT, int JM>
__global__ __launch_bounds__(kGsT) void k_gs_b(const XT* __restrict__ Q, int64_t n, int cnt,
                                                 GivensState* __restrict__ gs,
                                                 DevStatus* __restrict__ st,
                                                 const XT* __restrict__ y, XT* __restrict__ w1,
                                                 double* __restrict__ part,
                                                 StepSnap* __restrict__ snap) {
  // w1 accumulates in the basis type (the vector is stored in it); the dot
  // products and the norm stay FP64
  using CT = XT;
  __shared__ CT h[JM];
  for (int j = threadIdx.x; j < JM; j += kGsT) h[j] = (CT)(j < cnt ? -gs->h[j] : 0.0);
  __syncthreads();
  double acc[JM];
#pragma unroll
  for (int j = 0; j < JM; ++j) acc[j] = 0.0;
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kGsT;
  const int64_t s0 = (int64_t)blockIdx.x * kGsT + threadIdx.x;
  // y, and for rows of up to 128 bytes the basis row, one row ahead (index
  // clamped into range)
  constexpr bool PF = JM * sizeof(XT) <= 128;
  XT yn = y[min(s0, n - 1)];
  XT qn[PF ? JM : 1];
  if constexpr (PF) load_row<XT, JM>(Q, n, cnt, min(s0, n - 1), qn);
  for (int64_t s = s0; s < n; s += stride) {
    asm volatile("" ::: "memory");
    const XT yv = yn;
    yn = y[min(s + stride, n - 1)];
    XT q[JM];
    if constexpr (PF) {
#pragma unroll
      for (int j = 0; j < JM; ++j) q[j] = qn[j];
      load_row<XT, JM>(Q, n, cnt, min(s + stride, n - 1), qn);
    } else {
      load_row<XT, JM>(Q, n, cnt, s, q);
    }
    CT a0 = yv, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
    for (int g = 0; g < JM; g += 8) {
      asm volatile("" ::: "memory");  // at most 8 coefficients live
#pragma unroll
      for (int j = g; j < g + 8; j += 4) {
        a0 = fma_t(h[j], q[j], a0);
        a1 = fma_t(h[j + 1], q[j + 1], a1);
        a2 = fma_t(h[j + 2], q[j + 2], a2);
        a3 = fma_t(h[j + 3], q[j + 3], a3);
      }
    }
    const XT wx = (XT)((a0 + a1) + (a2 + a3));
    w1[s] = wx;
    const double wd = to_d(wx);
#pragma unroll
    for (int j = 0; j < JM; ++j) acc[j] = fma(to_d(q[j]), wd, acc[j]);
    nrm = fma(wd, wd, nrm);
  }
  double* mypart = part + (int64_t)blockIdx.x * kPartStride;
  store_cols<JM, kGsT>(acc, cnt, mypart);
  double v[1] = {nrm};
  const int op[1] = {0};
  block_reduce<1, kGsT>(v, op);
  if (threadIdx.x == 0) mypart[cnt] = v[0];
  // the block that finishes last runs the Givens update of the column
  if (last_to_finish(&st->arrive))
    finish<kGsT>(FIN_GIVENS, part, gridDim.x, cnt + 1, kPartStride, 0u, 0, st, gs, snap);
}

// Q_0 = r / beta, beta = sqrt(*l2sq); Givens state reset (block 0).
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_form_q0(const double* __restrict__ r,
                                                    const double* __restrict__ l2sq, int64_t n,
                                                    XT* __restrict__ q0,
                                                    GivensState* __restrict__ gs,
                                                    DevStatus* __restrict__ st) {
  const double beta = sqrt(*l2sq);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride)
    q0[s] = from_d<XT>(r[s] * inv);
  if (blockIdx.x == 0) {
    for (int j = threadIdx.x; j <= kMaxW; j += kBlock) gs->g[j] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      gs->g[0] = beta;
      st->beta = beta;
    }
  }
}

// V = Vb + sum_{j<i} y_j Q_j (Vb null: the sum alone), y from R y = g_hat
// (each block solves the i x i triangular system itself)
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_update(const XT* __restrict__ Q, int64_t n, int i,
                                                   const GivensState* __restrict__ gs,
                                                   const double* __restrict__ Vb,
                                                   double* __restrict__ V) {
  __shared__ double y[kMaxW];
  // up to kUpdStage columns: the triangle of R (column l holds rows 0..l,
  // packed) and g are loaded into LDS by the whole block in one round trip,
  // so that the serial back substitution reads LDS, not device memory
  __shared__ double Rs[kUpdStage * (kUpdStage + 1) / 2], gsh[kUpdStage];
  const bool staged = i <= kUpdStage;
  if (staged) {
    for (int l = threadIdx.x / 64; l < i; l += kBlock / 64)
      for (int j = threadIdx.x % 64; j <= l; j += 64)
        Rs[l * (l + 1) / 2 + j] = gs->R[(int64_t)l * (kMaxW + 1) + j];
    for (int j = threadIdx.x; j < i; j += kBlock) gsh[j] = gs->g[j];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int j = i - 1; j >= 0; --j) {
      double acc = staged ? gsh[j] : gs->g[j];
      for (int l = j + 1; l < i; ++l)
        acc -= (staged ? Rs[l * (l + 1) / 2 + j] : gs->R[(int64_t)l * (kMaxW + 1) + j]) * y[l];
      const double dj = staged ? Rs[j * (j + 1) / 2 + j] : gs->R[(int64_t)j * (kMaxW + 1) + j];
      y[j] = dj != 0.0 ? acc / dj : 0.0;
    }
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
    double v0 = Vb ? Vb[s] : 0.0, v1 = 0.0;
    // the columns in batches of 16 whose loads are issued together (the
    // last batch re-reads its last column, clamped); even columns sum into
    // v0 and odd ones into v1, each in increasing order
    for (int j = 0; j < i; j += 16) {
      const int rem = min(16, i - j);
      XT q[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) q[k] = qcol(Q, n, j + min(k, rem - 1))[s];
#pragma unroll
      for (int k = 0; k < 16; k += 2) {
        if (k < rem) v0 = fma(y[j + k], to_d(q[k]), v0);
        if (k + 1 < rem) v1 = fma(y[j + k + 1], to_d(q[k + 1]), v1);
      }
    }
    V[s] = v0 + v1;
  }
}

// out = a + b (FP64 vectors)
__global__ __launch_bounds__(kBlock) void k_vadd(const double* __restrict__ a,
                                                 const double* __restrict__ b, int64_t n,
                                                 double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride)
    out[s] = a[s] + b[s];
}

// Finishing work of a reduction, run by one block of NT threads: reduce cnt
// columns of per-block partials (row stride `stride`) over nb blocks in a
// fixed order, then write the result where the kind says.  FIN_GIVENS with
// snap: eta, rho and the implicit residual of the step also go to the
// pinned host snapshot.  Run by the one-block k_finalize, or by the block
// of a Gram-Schmidt pass that finishes last.
template <int NT>
__device__ void finish(int kind, const double* __restrict__ part, int nb, int cnt, int stride,
                       unsigned maxmask, int with_impl, DevStatus* __restrict__ st,
                       GivensState* __restrict__ gs, StepSnap* __restrict__ snap) {
  constexpr int NQ = NT / 64;  // row groups
  __shared__ double seg[NQ][64];
  __shared__ double red[kMaxW + 8];
  // The Givens state of the previous columns is loaded before the partials
  // so that both are in flight together (one memory round trip).
  const int col = cnt - 2;
  double gcs = 0.0, gsn = 0.0, gh = 0.0, gg = 0.0;
  if (kind == FIN_GIVENS) {
    const int j = threadIdx.x;
    if (j < col) {
      gcs = gs->cs[j];
      gsn = gs->sn[j];
    }
    if (j <= col) gh = gs->h[j];
    if (j == 0) gg = gs->g[col];
  }
  const double rimpl = kind == FIN_GIVENS && snap && threadIdx.x == 0 ? st->res_impl : 0.0;
  // columns 0..cnt-1 of the partial rows, plus (with_impl) the implicit
  // residual's max in the spare last column, reduced as column cnt
  const int ncol = cnt + (with_impl ? 1 : 0);
  for (int c0 = 0; c0 < ncol; c0 += 64) {
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const bool impl = with_impl && c0 + c == cnt;
    const int pc = impl ? stride - 1 : c0 + c;
    const bool mx = impl || (c0 == 0 && c < 32 && ((maxmask >> c) & 1u));
    double acc = 0.0;
    if (c0 + c < ncol)
      for (int b0 = q; b0 < nb; b0 += NQ * kFinBatch) {
        // a batch of loads in flight before the (ordered) accumulation
        double x[kFinBatch];
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u) {
          const int b = b0 + NQ * u;
          x[u] = b < nb ? part[(int64_t)b * stride + pc] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u)
          if (b0 + NQ * u < nb) acc = mx ? fmax(acc, x[u]) : acc + x[u];
      }
    seg[q][c] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && c0 + threadIdx.x < ncol) {
      double a = seg[0][threadIdx.x];
      for (int k = 1; k < NQ; ++k) a = mx ? fmax(a, seg[k][threadIdx.x]) : a + seg[k][threadIdx.x];
      red[c0 + threadIdx.x] = a;
    }
    __syncthreads();
  }
  if (with_impl && threadIdx.x == 0) st->res_impl = red[cnt];
  if (kind == FIN_GIVENS) {
    // red = [d_0..d_col, sigma]; gs->h = first-pass coefficients of column
    // col.  The state is staged in LDS so that the serial rotation sweep
    // touches no global memory.
    __shared__ double h[kMaxW + 2], cs[kMaxW + 1], sn[kMaxW + 1], z[kMaxW + 2], g2[2];
    __shared__ double eta_s;
    {
      const int j = threadIdx.x;
      if (j < col) {
        cs[j] = gcs;
        sn[j] = gsn;
      }
      if (j <= col) h[j] = gh + red[j];
    }
    if (threadIdx.x == 0) {
      g2[0] = gg;
      double dd = 0.0;
      for (int j = 0; j <= col; ++j) dd = fma(red[j], red[j], dd);
      eta_s = sqrt(fmax(red[col + 1] - dd, 0.0));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      h[col + 1] = eta_s;
      for (int j = 0; j < col; ++j) {  // previous rotations
        const double t = cs[j] * h[j] + sn[j] * h[j + 1];
        h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
        h[j] = t;
      }
      const double r = hypot(h[col], h[col + 1]);
      double c = 1.0, s = 0.0;
      if (r > 0.0) {
        c = h[col] / r;
        s = h[col + 1] / r;
      }
      cs[col] = c;
      sn[col] = s;
      h[col] = r;
      h[col + 1] = 0.0;
      const double gc = g2[0];
      g2[1] = -s * gc;
      g2[0] = c * gc;
      // residual of this column's iterate in basis coordinates
      double v = g2[1];
      for (int j = col; j >= 0; --j) {
        z[j + 1] = cs[j] * v;
        v = -sn[j] * v;
      }
      z[0] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= col; j += NT) {
      gs->h2[j] = red[j];
      gs->h[j] = h[j];
      gs->R[(int64_t)col * (kMaxW + 1) + j] = h[j];
    }
    for (int j = threadIdx.x; j <= col + 1; j += NT) gs->z[j] = z[j];
    if (threadIdx.x == 0) {
      gs->h[col + 1] = 0.0;
      gs->cs[col] = cs[col];
      gs->sn[col] = sn[col];
      gs->g[col] = g2[0];
      gs->g[col + 1] = g2[1];
      st->eta = eta_s;
      st->rho = fabs(g2[1]);
      if (snap) {  // system scope: the stores go to host memory, not the L2
        __hip_atomic_store(&snap->eta, eta_s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&snap->rho, fabs(g2[1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&snap->res_impl, rimpl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    return;
  }
  if (kind == FIN_DOTS) {
    for (int j = threadIdx.x; j < cnt; j += NT) gs->h[j] = red[j];
    return;
  }
  if (threadIdx.x != 0) return;
  switch (kind) {
    case FIN_BELLMAN:
      st->phi_inf = red[0];
      st->phi_l2sq = red[1];
      st->nonfinite = (int32_t)red[2];
      st->changes = (int32_t)red[3];
      break;
    case FIN_RESID:
      st->res_inf = red[0];
      st->res_l2sq = red[1];
      st->vmax = red[2];
      break;
    case FIN_VI:
      st->aux = red[0];
      st->res_l2sq = red[1];
      break;
    case FIN_GATHER:
      st->changes = (int32_t)red[0];
      break;
    case FIN_IMPL:
      st->res_impl = red[0];
      break;
    default:
      break;
  }
}

__global__ __launch_bounds__(kFinT) void k_finalize(int kind, const double* __restrict__ part,
                                                    int nb, int cnt, int stride, unsigned maxmask,
                                                    int with_impl, DevStatus* __restrict__ st,
                                                    GivensState* __restrict__ gs,
                                                    StepSnap* __restrict__ snap) {
  finish<kFinT>(kind, part, nb, cnt, stride, maxmask, with_impl, st, gs, snap);
}

inline int gs_grid(const Mdp& d) {  // grid-stride kernels
  const int64_t blocks = (d.n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, kGsBlocks));
}


}  // namespace

void launch_finalize(Mdp& d, FinKind kind, int nb, hipStream_t s, int cnt, bool with_impl,
                     StepSnap* snap) {
  int stride = 0;
  unsigned mask = 0;
  switch (kind) {
    case FIN_BELLMAN: cnt = 4; stride = 4; mask = 1u; break;
    case FIN_RESID: cnt = 3; stride = 3; mask = 5u; break;
    case FIN_VI: cnt = 3; stride = 3; mask = 5u; break;
    case FIN_GATHER: cnt = 1; stride = 1; mask = 0u; break;
    case FIN_IMPL: cnt = 1; stride = 1; mask = 1u; break;
    case FIN_DOTS: stride = kPartStride; mask = 0u; break;
    case FIN_GIVENS: stride = kPartStride; mask = 0u; break;
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinT), 0, s, (int)kind, (const double*)d.part, nb,
                     cnt, stride, mask, with_impl ? 1 : 0, d.st, d.gs, snap);
}

void launch_form_q0(Mdp& d, bool fp32, const double* r, const double* l2sq, hipStream_t s) {
  ProfScope p(d, KC_OTHER, s);
  if (fp32)
    hipLaunchKernelGGL(k_form_q0<float>, dim3(gs_grid(d)), dim3(kBlock), 0, s, r, l2sq, d.n,
                       (float*)d.ws.Q, d.gs, d.st);
  else
    hipLaunchKernelGGL(k_form_q0<double>, dim3(gs_grid(d)), dim3(kBlock), 0, s, r, l2sq, d.n,
                       (double*)d.ws.Q, d.gs, d.st);
}

void launch_form_qi(Mdp& d, bool fp32, int c, const void* w1, hipStream_t s) {
  ProfScope p(d, KC_GS, s);
  if (fp32)
    hipLaunchKernelGGL(k_form_qi<float>, dim3(gs_grid(d)), dim3(kBlock), 0, s, (float*)d.ws.Q,
                       d.n, c, (const float*)w1, (const GivensState*)d.gs, (const DevStatus*)d.st,
                       d.part);
  else
    hipLaunchKernelGGL(k_form_qi<double>, dim3(gs_grid(d)), dim3(kBlock), 0, s, (double*)d.ws.Q,
                       d.n, c, (const double*)w1, (const GivensState*)d.gs, (const DevStatus*)d.st,
                       d.part);
}

void launch_dots(Mdp& d, bool fp32, int cnt, const void* v, bool givens, bool with_impl,
                 hipStream_t s) {
  {
    ProfScope p(d, KC_GS, s);
    if (fp32)
      hipLaunchKernelGGL(k_dots<float>, dim3(gs_grid(d)), dim3(kBlock), 0, s,
                         (const float*)d.ws.Q, d.n, cnt, (const float*)v, givens ? 1 : 0, d.part);
    else
      hipLaunchKernelGGL(k_dots<double>, dim3(gs_grid(d)), dim3(kBlock), 0, s,
                         (const double*)d.ws.Q, d.n, cnt, (const double*)v, givens ? 1 : 0, d.part);
  }
  launch_finalize(d, givens ? FIN_GIVENS : FIN_DOTS, gs_grid(d), s, givens ? cnt + 1 : cnt,
                  with_impl, givens ? d.hsnap : nullptr);
}

namespace {

template <typename XT, int JM>
void gs_step_typed(Mdp& d, int c, const void* y, void* w1, hipStream_t s) {
  const int64_t blocks = (d.n + kGsT - 1) / kGsT;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(blocks, kGsB));
  ProfScope p(d, KC_GS, s);
  hipLaunchKernelGGL((k_gs_a<XT, JM>), dim3(nb), dim3(kGsT), 0, s, (XT*)d.ws.Q, d.n, c,
                     (const XT*)w1, (const XT*)y, d.gs, d.st, d.part);
  hipLaunchKernelGGL((k_gs_b<XT, JM>), dim3(nb), dim3(kGsT), 0, s, (const XT*)d.ws.Q, d.n, c + 1,
                     d.gs, d.st, (const XT*)y, (XT*)w1, d.part, d.hsnap);
}

template <typename XT>
bool gs_step_bucket(Mdp& d, int c, const void* y, void* w1, hipStream_t s) {
  const int need = c + 1;
  if (need <= 8) gs_step_typed<XT, 8>(d, c, y, w1, s);
  else if (need <= 16) gs_step_typed<XT, 16>(d, c, y, w1, s);
  else if (need <= 32) gs_step_typed<XT, 32>(d, c, y, w1, s);
  else if (sizeof(XT) == 4 && need <= 48) gs_step_typed<XT, 48>(d, c, y, w1, s);
  else if (sizeof(XT) == 4 && need <= 64) gs_step_typed<XT, 64>(d, c, y, w1, s);
  else return false;
  return true;
}

}  // namespace

int gs_fused_max(bool fp32) { return fp32 ? 64 : 32; }

void launch_gs_step(Mdp& d, bool fp32, int c, const void* y, void* w1, hipStream_t s) {
  const bool done = fp32 ? gs_step_bucket<float>(d, c, y, w1, s)
                         : gs_step_bucket<double>(d, c, y, w1, s);
  if (done) return;
  // columns beyond the register buckets: separate formation, projection,
  // update and second projection
  if (c > 0) launch_form_qi(d, fp32, c, w1, s);
  launch_dots(d, fp32, c + 1, y, false, c > 0, s);
  launch_axpy(d, fp32, c + 1, y, w1, s);
  launch_dots(d, fp32, c + 1, w1, true, false, s);
}

void launch_axpy(Mdp& d, bool fp32, int cnt, const void* y, void* w1, hipStream_t s) {
  ProfScope p(d, KC_GS, s);
  if (fp32)
    hipLaunchKernelGGL(k_axpy<float>, dim3(gs_grid(d)), dim3(kBlock), 0, s, (const float*)d.ws.Q,
                       d.n, cnt, (const GivensState*)d.gs, (const float*)y, (float*)w1);
  else
    hipLaunchKernelGGL(k_axpy<double>, dim3(gs_grid(d)), dim3(kBlock), 0, s,
                       (const double*)d.ws.Q, d.n, cnt, (const GivensState*)d.gs, (const double*)y,
                       (double*)w1);
}

void launch_vadd(Mdp& d, const double* a, const double* b, double* out, hipStream_t s) {
  ProfScope p(d, KC_UPDATE, s);
  hipLaunchKernelGGL(k_vadd, dim3(gs_grid(d)), dim3(kBlock), 0, s, a, b, d.n, out);
}

void launch_update(Mdp& d, bool fp32, int i, const double* Vb, double* V, hipStream_t s) {
  ProfScope p(d, KC_UPDATE, s);
  if (fp32)
    hipLaunchKernelGGL(k_update<float>, dim3(gs_grid(d)), dim3(kBlock), 0, s,
                       (const float*)d.ws.Q, d.n, i, d.gs, Vb, V);
  else
    hipLaunchKernelGGL(k_update<double>, dim3(gs_grid(d)), dim3(kBlock), 0, s,
                       (const double*)d.ws.Q, d.n, i, d.gs, Vb, V);
}

}  // namespace ig
