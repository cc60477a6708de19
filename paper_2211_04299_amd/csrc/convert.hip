// Device-side conversion of a CSR MDP into the sliced-ELL image (the same
// layout, value rounding and checks as the host conversion in mdp.hip): the
// host computes only the per-slice layout from row_ptr (O(rows)); the
// entries (O(nnz)) are converted and validated here, so a request's raw
// column and value arrays only have to cross PCIe once.
#include "internal.hpp"

namespace ig {

namespace {

// stored value of an input probability, and its exact value after storage
__device__ __forceinline__ double in_val(const double* p, int64_t e) { return p[e]; }
__device__ __forceinline__ double in_val(const float* p, int64_t e) { return (double)p[e]; }
__device__ __forceinline__ double in_val(const uint16_t* p, int64_t e) {
  return (double)__uint_as_float(((uint32_t)p[e]) << 16);
}
__device__ __forceinline__ double out_val(double x, double* o) {
  *o = x;
  return x;
}
__device__ __forceinline__ double out_val(double x, float* o) {
  *o = (float)x;
  return (double)*o;
}
__device__ __forceinline__ double out_val(double x, uint16_t* o) {
  uint32_t u = __float_as_uint((float)x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  *o = (uint16_t)(u >> 16);
  return (double)__uint_as_float(((uint32_t)*o) << 16);
}

// One wavefront per 64-state slice, one lane per state: lane l writes
// entries (a, j, l) of the slice, so every store of the wavefront is
// contiguous.  err: [0] columns out of range, [1] repeated columns, [2]
// probabilities outside [0,1], [3] rows not summing to 1, [4] bits of the
// largest stored row sum (non-negative doubles order like their bits).
template <typename IN, typename OUT>
__global__ __launch_bounds__(kBlock) void k_fill_sell(
    int64_t n, int m, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
    const IN* __restrict__ val, const uint8_t* __restrict__ adm_t, const int64_t* __restrict__ off,
    const int32_t* __restrict__ width, const int32_t* __restrict__ mcnt, int32_t* __restrict__ scol,
    OUT* __restrict__ sval, int validate, double sum_tol, unsigned long long* __restrict__ err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t ns = (n + kSlice - 1) / kSlice;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / kWave);
  unsigned long long bad_col = 0, bad_dup = 0, bad_p = 0, bad_sum = 0;
  double mss = 0.0;
  for (int64_t b = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; b < ns;
       b += wstride) {
    const int Kb = width[b], Mb = mcnt[b];
    const int64_t ob = off[b];
    const int64_t s = b * kSlice + lane;
    for (int a = 0; a < Mb; ++a) {
      const int64_t base = ob + (((int64_t)a * Kb) << 6) + lane;
      const bool use = s < n && (!adm_t || adm_t[(int64_t)a * n + s]);
      int64_t lo = 0, len = 0;
      if (use) {
        lo = rp[s * m + a];
        len = rp[s * m + a + 1] - lo;
      }
      double sum = 0.0, ssum = 0.0;
      for (int64_t j = 0; j < len; ++j) {
        const int32_t c = col[lo + j];
        const bool ok = c >= 0 && c < n;
        bad_col += !ok;
        const double p = in_val(val, lo + j);
        if (validate) {
          bad_p += !(p >= 0.0 && p <= 1.0);
          for (int64_t jj = 0; jj < j; ++jj) bad_dup += col[lo + jj] == c;
        }
        sum += p;
        const int64_t pos = base + (j << 6);
        scol[pos] = ok ? c : 0;
        ssum += out_val(p, &sval[pos]);
      }
      for (int64_t j = len; j < Kb; ++j) {
        const int64_t pos = base + (j << 6);
        scol[pos] = 0;
        out_val(0.0, &sval[pos]);
      }
      if (use) {
        if (validate && !(fabs(sum - 1.0) <= sum_tol)) ++bad_sum;
        mss = fmax(mss, ssum);
      }
    }
  }
  // wavefront totals, then one atomic per wavefront
  for (int o = 32; o > 0; o >>= 1) {
    bad_col += __shfl_xor(bad_col, o);
    bad_dup += __shfl_xor(bad_dup, o);
    bad_p += __shfl_xor(bad_p, o);
    bad_sum += __shfl_xor(bad_sum, o);
    mss = fmax(mss, __shfl_xor(mss, o));
  }
  if (lane == 0) {
    if (bad_col) atomicAdd(&err[0], bad_col);
    if (bad_dup) atomicAdd(&err[1], bad_dup);
    if (bad_p) atomicAdd(&err[2], bad_p);
    if (bad_sum) atomicAdd(&err[3], bad_sum);
    atomicMax(&err[4], (unsigned long long)__double_as_longlong(mss));
  }
}

template <typename IN>
void launch_fill_in(const ConvArgs& c, ig_dtype store, hipStream_t s) {
  const int64_t ns = (c.n + kSlice - 1) / kSlice;
  const int blocks = (int)std::max<int64_t>(
      1, std::min<int64_t>((ns + kBlock / kWave - 1) / (kBlock / kWave), kMaxBlocks));
  const IN* v = (const IN*)c.val;
  switch (store) {
    case IG_FP64:
      hipLaunchKernelGGL((k_fill_sell<IN, double>), dim3(blocks), dim3(kBlock), 0, s, c.n, c.m, c.rp,
                         c.col, v, c.adm_t, c.off, c.width, c.mcnt, c.scol, (double*)c.sval,
                         c.validate, c.sum_tol, c.err);
      break;
    case IG_FP32:
      hipLaunchKernelGGL((k_fill_sell<IN, float>), dim3(blocks), dim3(kBlock), 0, s, c.n, c.m, c.rp,
                         c.col, v, c.adm_t, c.off, c.width, c.mcnt, c.scol, (float*)c.sval,
                         c.validate, c.sum_tol, c.err);
      break;
    default:
      hipLaunchKernelGGL((k_fill_sell<IN, uint16_t>), dim3(blocks), dim3(kBlock), 0, s, c.n, c.m,
                         c.rp, c.col, v, c.adm_t, c.off, c.width, c.mcnt, c.scol,
                         (uint16_t*)c.sval, c.validate, c.sum_tol, c.err);
      break;
  }
}

}  // namespace

void launch_fill_sell(const ConvArgs& c, ig_dtype val_type, ig_dtype store, hipStream_t s) {
  switch (val_type) {
    case IG_FP64: launch_fill_in<double>(c, store, s); break;
    case IG_FP32: launch_fill_in<float>(c, store, s); break;
    default: launch_fill_in<uint16_t>(c, store, s); break;
  }
}

}  // namespace ig
