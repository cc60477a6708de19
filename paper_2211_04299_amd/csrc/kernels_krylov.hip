// Arnoldi orthogonalisation, Givens-rotated Hessenberg least squares and the
// solution update of GMRES(W) (Algorithm 2 of the paper, inner loop).
//
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2): in exact
// arithmetic it yields the same Hessenberg column as the modified
// Gram-Schmidt loop of Algorithm 2, with i+1 dot products per pass computed in
// one sweep over the basis instead of i sequential sweeps.  Every dot product
// and norm accumulates in FP64; per-block partials are combined by the last
// block in a fixed order, so results are bitwise reproducible.
#include "internal.hpp"

namespace ig {

namespace {

constexpr int kJC = 8;  // dot products accumulated per sweep

template <typename XT>
__device__ __forceinline__ const XT* qcol(const XT* Q, int64_t n, int j) {
  return Q + (int64_t)j * n;
}

// partial dot products of w with Q_0..Q_{i-1} for this block's states, written
// to part[blockIdx.x * i + j]
template <typename XT>
__device__ __forceinline__ void block_dots(const XT* __restrict__ Q, int64_t n, int i,
                                           const XT* __restrict__ w, double* __restrict__ part) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int j0 = 0; j0 < i; j0 += kJC) {
    double acc[kJC];
#pragma unroll
    for (int k = 0; k < kJC; ++k) acc[k] = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
      const double ws = to_d(w[s]);
#pragma unroll
      for (int k = 0; k < kJC; ++k)
        if (j0 + k < i) acc[k] = fma(to_d(qcol(Q, n, j0 + k)[s]), ws, acc[k]);
    }
    const int op[kJC] = {0, 0, 0, 0, 0, 0, 0, 0};
    block_reduce<kJC>(acc, op);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < kJC; ++k)
        if (j0 + k < i) part[(int64_t)blockIdx.x * i + j0 + k] = acc[k];
    }
  }
}

// ticket: true in the last block to finish
__device__ __forceinline__ bool last_block(unsigned int* ticket) {
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned t = atomicInc(ticket, gridDim.x - 1);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// in the last block: out[j] = sum_b part[b*i + j], fixed order
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int i,
                                             double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int j = wid; j < i; j += kBlock / kWave) {
    double a = 0.0;
    for (int b = lane; b < (int)gridDim.x; b += kWave) a += part[(int64_t)b * i + j];
    a = wave_sum(a);
    if (lane == 0) out[j] = a;
  }
  __syncthreads();
}

template <typename XT>
__global__ __launch_bounds__(kBlock) void k_gs_pass1(const XT* __restrict__ Q, int64_t n, int i,
                                                     const XT* __restrict__ w,
                                                     double* __restrict__ part,
                                                     unsigned int* ticket,
                                                     GivensState* __restrict__ gs) {
  block_dots<XT>(Q, n, i, w, part);
  if (last_block(ticket)) sum_partials(part, i, gs->h);
}

// w -= sum_j c_j Q_j with c taken from `coef`; then (pass 2) the dot products
// of the corrected w into gs->h2.
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_gs_pass2(const XT* __restrict__ Q, int64_t n, int i,
                                                     XT* __restrict__ w,
                                                     double* __restrict__ part,
                                                     unsigned int* ticket,
                                                     GivensState* __restrict__ gs) {
  __shared__ double c[kMaxW + 1];
  for (int j = threadIdx.x; j < i; j += kBlock) c[j] = gs->h[j];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
    double ws = to_d(w[s]);
    for (int j = 0; j < i; ++j) ws = fma(-c[j], to_d(qcol(Q, n, j)[s]), ws);
    w[s] = from_d<XT>(ws);
  }
  block_dots<XT>(Q, n, i, w, part);
  if (last_block(ticket)) sum_partials(part, i, gs->h2);
}

// w -= sum_j h2_j Q_j; eta = ||w||_2; column i-1 of H = h + h2 with
// H(i, i-1) = eta; apply the previous rotations, form rotation i-1, update
// g_hat; status.eta, status.rho = |g_hat(i)|.
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_gs_pass3(const XT* __restrict__ Q, int64_t n, int i,
                                                     XT* __restrict__ w,
                                                     double* __restrict__ part,
                                                     unsigned int* ticket,
                                                     GivensState* __restrict__ gs,
                                                     DevStatus* __restrict__ st) {
  __shared__ double c[kMaxW + 1];
  for (int j = threadIdx.x; j < i; j += kBlock) c[j] = gs->h2[j];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double nrm[1] = {0.0};
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
    double ws = to_d(w[s]);
    for (int j = 0; j < i; ++j) ws = fma(-c[j], to_d(qcol(Q, n, j)[s]), ws);
    const XT wx = from_d<XT>(ws);
    w[s] = wx;
    const double wd = to_d(wx);
    nrm[0] = fma(wd, wd, nrm[0]);
  }
  const int op[1] = {0};
  block_reduce<1>(nrm, op);
  if (threadIdx.x == 0) part[blockIdx.x] = nrm[0];
  if (last_block(ticket)) {
    __shared__ double tot;
    if (threadIdx.x < kWave) {
      double a = 0.0;
      for (int b = threadIdx.x; b < (int)gridDim.x; b += kWave) a += part[b];
      a = wave_sum(a);
      if (threadIdx.x == 0) tot = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double eta = sqrt(tot);
      const int col = i - 1;
      double* h = gs->h;
      for (int j = 0; j < i; ++j) h[j] += gs->h2[j];
      h[i] = eta;
      for (int j = 0; j < col; ++j) {  // previous rotations
        const double t = gs->cs[j] * h[j] + gs->sn[j] * h[j + 1];
        h[j + 1] = -gs->sn[j] * h[j] + gs->cs[j] * h[j + 1];
        h[j] = t;
      }
      const double r = hypot(h[col], h[col + 1]);
      double cs = 1.0, sn = 0.0;
      if (r > 0.0) {
        cs = h[col] / r;
        sn = h[col + 1] / r;
      }
      gs->cs[col] = cs;
      gs->sn[col] = sn;
      h[col] = r;
      h[col + 1] = 0.0;
      gs->g[col + 1] = -sn * gs->g[col];
      gs->g[col] = cs * gs->g[col];
      for (int j = 0; j <= col; ++j) gs->R[(int64_t)col * (kMaxW + 1) + j] = h[j];
      st->eta = eta;
      st->rho = fabs(gs->g[col + 1]);
    }
  }
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

// V = Vb + sum_{j<i} y_j Q_j, y from R y = g_hat (each block solves the
// i x i triangular system itself)
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_update(const XT* __restrict__ Q, int64_t n, int i,
                                                   const GivensState* __restrict__ gs,
                                                   const double* __restrict__ Vb,
                                                   double* __restrict__ V) {
  __shared__ double y[kMaxW];
  if (threadIdx.x == 0) {
    for (int j = i - 1; j >= 0; --j) {
      double acc = gs->g[j];
      for (int l = j + 1; l < i; ++l) acc -= gs->R[(int64_t)l * (kMaxW + 1) + j] * y[l];
      const double dj = gs->R[(int64_t)j * (kMaxW + 1) + j];
      y[j] = dj != 0.0 ? acc / dj : 0.0;
    }
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += stride) {
    double v = Vb[s];
    for (int j = 0; j < i; ++j) v = fma(y[j], to_d(qcol(Q, n, j)[s]), v);
    V[s] = v;
  }
}

inline int gs_grid(const Mdp& d) {
  const int64_t blocks = (d.n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, kGsBlocks));
}

}  // namespace

void launch_form_q0(Mdp& d, bool fp32, const double* r, const double* l2sq, hipStream_t s) {
  ProfScope p(d, KC_OTHER, s);
  if (fp32)
    hipLaunchKernelGGL(k_form_q0<float>, dim3(gs_grid(d)), dim3(kBlock), 0, s, r, l2sq, d.n,
                       (float*)d.ws.Q, d.gs, d.st);
  else
    hipLaunchKernelGGL(k_form_q0<double>, dim3(gs_grid(d)), dim3(kBlock), 0, s, r, l2sq, d.n,
                       (double*)d.ws.Q, d.gs, d.st);
}

void launch_arnoldi_orth(Mdp& d, bool fp32, int i, void* w, hipStream_t s) {
  ProfScope p(d, KC_GS, s);
  const dim3 grid(gs_grid(d)), block(kBlock);
  if (fp32) {
    const float* Q = (const float*)d.ws.Q;
    hipLaunchKernelGGL(k_gs_pass1<float>, grid, block, 0, s, Q, d.n, i, (const float*)w, d.part,
                       d.ticket, d.gs);
    hipLaunchKernelGGL(k_gs_pass2<float>, grid, block, 0, s, Q, d.n, i, (float*)w, d.part,
                       d.ticket, d.gs);
    hipLaunchKernelGGL(k_gs_pass3<float>, grid, block, 0, s, Q, d.n, i, (float*)w, d.part,
                       d.ticket, d.gs, d.st);
  } else {
    const double* Q = (const double*)d.ws.Q;
    hipLaunchKernelGGL(k_gs_pass1<double>, grid, block, 0, s, Q, d.n, i, (const double*)w,
                       d.part, d.ticket, d.gs);
    hipLaunchKernelGGL(k_gs_pass2<double>, grid, block, 0, s, Q, d.n, i, (double*)w, d.part,
                       d.ticket, d.gs);
    hipLaunchKernelGGL(k_gs_pass3<double>, grid, block, 0, s, Q, d.n, i, (double*)w, d.part,
                       d.ticket, d.gs, d.st);
  }
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
