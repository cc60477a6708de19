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
__device__ __forceinline__ double rounded(double x, double*) { return x; }
__device__ __forceinline__ double rounded(double x, float*) { return (double)(float)x; }
__device__ __forceinline__ uint16_t bf16_bits(double x) {
  uint32_t u = __float_as_uint((float)x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double rounded(double x, uint16_t*) {
  return (double)__uint_as_float(((uint32_t)bf16_bits(x)) << 16);
}
__device__ __forceinline__ void put(double x, double* o, int64_t e) { o[e] = x; }
__device__ __forceinline__ void put(double x, float* o, int64_t e) { o[e] = (float)x; }
__device__ __forceinline__ void put(double x, uint16_t* o, int64_t e) { o[e] = bf16_bits(x); }

constexpr int kDupLdsRows = 128;  // widths up to this test repeats in LDS (32 KiB)

// One block per (slice b, action block a): the tile of 64 rows (s, a),
// s = 64b + lane, stored as K_b x 64 entries at off[b] + a*K_b*64.  Thread
// t owns lane t & 63 and the positions j = t/64, t/64 + 4, ...: the stores
// of a wavefront are contiguous.  The row sums are then taken by one thread
// per row in the order j = 0, 1, ... (as on the host), so every check and
// the largest stored row sum agree with the host conversion bit for bit.
// err: [0] columns out of range, [1] repeated columns, [2] probabilities
// outside [0,1], [3] rows not summing to 1, [4] bits of the largest stored
// row sum (non-negative doubles order like their bit patterns).
template <typename IN, typename OUT>
__global__ __launch_bounds__(kBlock) void k_fill_sell(
    int64_t n, int m, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
    const IN* __restrict__ val, const uint8_t* __restrict__ adm_t, const int64_t* __restrict__ off,
    const int32_t* __restrict__ width, const int32_t* __restrict__ mcnt, int32_t* __restrict__ scol,
    OUT* __restrict__ sval, int validate, int dup_lds, double sum_tol,
    unsigned long long* __restrict__ err) {
  extern __shared__ int32_t tile[];  // [K_b][64] columns when dup_lds
  __shared__ int64_t lo_s[kSlice];
  __shared__ int32_t len_s[kSlice];
  __shared__ unsigned long long cnt_s[4];
  const int64_t b = blockIdx.x / m;
  const int a = (int)(blockIdx.x - b * m);
  if (a >= mcnt[b]) return;  // the whole block leaves together
  const int t = threadIdx.x, lane = t & (kSlice - 1);
  const int Kb = width[b];
  const int64_t base = off[b] + (((int64_t)a * Kb) << 6);
  if (t < kSlice) {
    const int64_t s = b * kSlice + t;
    const bool use = s < n && (!adm_t || adm_t[(int64_t)a * n + s]);
    int64_t lo = 0, len = 0;
    if (use) {
      lo = rp[s * m + a];
      len = rp[s * m + a + 1] - lo;
    }
    lo_s[t] = lo;
    len_s[t] = use ? (int32_t)len : -1;  // -1: no row (padding lane or excluded pair)
  }
  if (t < 4) cnt_s[t] = 0;
  __syncthreads();
  const int64_t lo = lo_s[lane];
  const int len = len_s[lane];
  unsigned long long bad_col = 0, bad_dup = 0, bad_p = 0;
  for (int j = t >> 6; j < Kb; j += kBlock / kSlice) {
    const int64_t pos = base + ((int64_t)j << 6) + lane;
    int32_t c = 0;
    double p = 0.0;
    if (j < len) {
      c = col[lo + j];
      p = in_val(val, lo + j);
      const bool ok = c >= 0 && c < n;
      bad_col += !ok;
      if (validate) bad_p += !(p >= 0.0 && p <= 1.0);
      c = ok ? c : 0;
      if (dup_lds) tile[(j << 6) + lane] = ok ? c : -1 - j;  // out of range: never equal
    }
    scol[pos] = c;
    put(p, sval, pos);
  }
  if (validate) {
    if (dup_lds) __syncthreads();
    for (int j = t >> 6; j < len; j += kBlock / kSlice) {
      if (dup_lds) {
        const int32_t c = tile[(j << 6) + lane];
        for (int jj = 0; jj < j; ++jj) bad_dup += tile[(jj << 6) + lane] == c;
      } else {
        const int32_t c = col[lo + j];
        for (int jj = 0; jj < j; ++jj) bad_dup += col[lo + jj] == c;
      }
    }
  }
  // row sums in the host's order, one thread per row
  unsigned long long bad_sum = 0;
  double ssum = 0.0;
  if (t < kSlice && len >= 0) {
    double sum = 0.0;
    for (int j = 0; j < len; ++j) {
      const double p = in_val(val, lo + j);
      sum += p;
      ssum += rounded(p, sval);
    }
    if (validate && !(fabs(sum - 1.0) <= sum_tol)) bad_sum = 1;
  }
  // totals: wavefront sums, then LDS, then one atomic per counter
  for (int o = 32; o > 0; o >>= 1) {
    bad_col += __shfl_xor(bad_col, o);
    bad_dup += __shfl_xor(bad_dup, o);
    bad_p += __shfl_xor(bad_p, o);
    bad_sum += __shfl_xor(bad_sum, o);
    ssum = fmax(ssum, __shfl_xor(ssum, o));
  }
  if (lane == 0) {
    if (bad_col) atomicAdd(&cnt_s[0], bad_col);
    if (bad_dup) atomicAdd(&cnt_s[1], bad_dup);
    if (bad_p) atomicAdd(&cnt_s[2], bad_p);
    if (bad_sum) atomicAdd(&cnt_s[3], bad_sum);
  }
  __syncthreads();
  if (t < 4 && cnt_s[t]) atomicAdd(&err[t], cnt_s[t]);
  if (t == 0) atomicMax(&err[4], (unsigned long long)__double_as_longlong(ssum));
}

template <typename IN, typename OUT>
void launch_fill_typed(const ConvArgs& c, hipStream_t s) {
  const int64_t ns = (c.n + kSlice - 1) / kSlice;
  const int dup_lds = c.validate && c.maxK <= kDupLdsRows;
  const size_t lds = dup_lds ? (size_t)std::max(1, c.maxK) * kSlice * sizeof(int32_t) : 0;
  hipLaunchKernelGGL((k_fill_sell<IN, OUT>), dim3((unsigned)(ns * c.m)), dim3(kBlock), lds, s, c.n,
                     c.m, c.rp, c.col, (const IN*)c.val, c.adm_t, c.off, c.width, c.mcnt, c.scol,
                     (OUT*)c.sval, c.validate, dup_lds, c.sum_tol, c.err);
}

template <typename IN>
void launch_fill_in(const ConvArgs& c, ig_dtype store, hipStream_t s) {
  switch (store) {
    case IG_FP64: launch_fill_typed<IN, double>(c, s); break;
    case IG_FP32: launch_fill_typed<IN, float>(c, s); break;
    default: launch_fill_typed<IN, uint16_t>(c, s); break;
  }
}

// BF16 copy of FP32 values (the rounding of the conversion above): four
// values per thread and step, grid-stride
__global__ __launch_bounds__(kBlock) void k_round_bf16(const float* __restrict__ src,
                                                       uint16_t* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * kBlock * 4;
  for (int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4; e < count; e += stride) {
    if (e + 4 <= count) {
      const float4 v = *reinterpret_cast<const float4*>(src + e);
      ushort4 o;
      o.x = bf16_bits(v.x);
      o.y = bf16_bits(v.y);
      o.z = bf16_bits(v.z);
      o.w = bf16_bits(v.w);
      *reinterpret_cast<ushort4*>(dst + e) = o;
    } else {
      for (int64_t k = e; k < count; ++k) dst[k] = bf16_bits(src[k]);
    }
  }
}

}  // namespace

void launch_round_bf16(const float* src, void* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const int64_t blocks = std::min<int64_t>((count + 4 * kBlock - 1) / (4 * kBlock), 4096);
  hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, (uint16_t*)dst,
                     count);
}

void launch_fill_sell(const ConvArgs& c, ig_dtype val_type, ig_dtype store, hipStream_t s) {
  switch (val_type) {
    case IG_FP64: launch_fill_in<double>(c, store, s); break;
    case IG_FP32: launch_fill_in<float>(c, store, s); break;
    default: launch_fill_in<uint16_t>(c, store, s); break;
  }
}

}  // namespace ig
