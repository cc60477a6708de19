// MDP handle: validation of the problem data (Section 2 of the paper: finite
// S and A, row-stochastic P, bounded g, gamma in (0,1)), conversion to the
// device layouts, workspace and per-class event timing.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <memory>
#include <vector>

#include "internal.hpp"

namespace ig {

thread_local std::string g_last_error = "no error";

ig_status fail(ig_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ig_status sync_status(Mdp& d, hipStream_t s) {
  IG_HIP(hipMemcpyAsync(d.hst, d.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  IG_HIP(hipStreamSynchronize(s));
  return IG_OK;
}

ProfScope::ProfScope(Mdp& d_, KClass k_, hipStream_t s_) : d(d_), k(k_), s(s_) {
  if (!(d.prof_mask & (1u << k))) return;
  if (d.prof_seen[k]++ % d.prof_every != 0) return;  // not one of the sampled launches
  auto& pool = d.prof_ev[k];
  if (d.prof_used[k] == pool.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    pool.emplace_back(a, b);
  }
  auto& pr = pool[d.prof_used[k]++];
  (void)hipEventRecord(pr.first, s);
  e1 = pr.second;
}
ProfScope::~ProfScope() {
  if (e1) (void)hipEventRecord(e1, s);
}

namespace {

inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
inline double bf16_to_f64(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}
inline int dtype_bytes(ig_dtype t) { return t == IG_FP64 ? 8 : (t == IG_FP32 ? 4 : 2); }

// value e of the caller's array as a double
struct ValReader {
  const void* p;
  ig_dtype t;
  double operator()(int64_t e) const {
    switch (t) {
      case IG_FP64: return ((const double*)p)[e];
      case IG_FP32: return (double)((const float*)p)[e];
      default: return bf16_to_f64(((const uint16_t*)p)[e]);
    }
  }
};

// store x (already representable in the input type) in the storage type,
// returning the stored value as a double
inline double store_val(void* dst, int64_t pos, ig_dtype st, double x) {
  switch (st) {
    case IG_FP64: ((double*)dst)[pos] = x; return x;
    case IG_FP32: {
      const float f = (float)x;
      ((float*)dst)[pos] = f;
      return (double)f;
    }
    default: {
      const uint16_t b = f32_to_bf16((float)x);
      ((uint16_t*)dst)[pos] = b;
      return bf16_to_f64(b);
    }
  }
}

inline size_t round256(size_t b) { return round_alloc(b); }

// the region of the handle being created (set by create_impl / ensure_workspace)
thread_local DevRegion* t_region = nullptr;

template <typename T>
ig_status dmalloc(T** p, size_t bytes) {
  *p = nullptr;
  if (t_region) {
    const size_t b = round256(bytes);
    if (t_region->used + b > t_region->size)
      return fail(IG_E_TOO_LARGE, "device region too small for the MDP");
    *p = (T*)(t_region->base + t_region->used);
    t_region->used += b;
    return IG_OK;
  }
  if (bytes == 0) bytes = 8;
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(IG_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return IG_OK;
}

// A temporary allocation from the top of the handle's region (region mode):
// `used` does not move, so the allocations made after the create has
// synchronised may reuse these bytes.  *top counts the bytes taken so far.
template <typename T>
ig_status dmalloc_top(T** p, size_t bytes, size_t* top) {
  const size_t b = round256(bytes);
  if (t_region->used + *top + b > t_region->size)
    return fail(IG_E_TOO_LARGE, "device region too small for the MDP");
  *top += b;
  *p = (T*)(t_region->base + t_region->size - *top);
  return IG_OK;
}

// host -> device copy; in region mode asynchronous on the handle's stream
// (the caller keeps `src` alive until the stream has passed the copy)
ig_status upload(Mdp* d, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return IG_OK;
  const hipError_t e = d->region ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, d->stream)
                                 : hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? IG_OK : fail(IG_E_DEVICE, "host to device copy failed");
}

// Host -> device copy of caller memory through a pinned double buffer on
// the handle's stream: the memcpy of one chunk overlaps the DMA of the
// previous one.  Pageable copies issued by several threads at once reach
// well under the link's rate; staged ones reach it.
struct Bounce {
  char* buf = nullptr;  // 2 * half pinned bytes
  size_t half = 0;
  hipEvent_t* ev = nullptr;
  int h = 0;
  bool used[2] = {false, false};
  ig_status put(hipStream_t s, void* dst, const void* src, size_t bytes) {
    for (size_t done = 0; done < bytes;) {
      const size_t c = std::min(half, bytes - done);
      if (used[h] && hipEventSynchronize(ev[h]) != hipSuccess)
        return fail(IG_E_DEVICE, "staged copy failed");
      std::memcpy(buf + h * half, (const char*)src + done, c);
      if (hipMemcpyAsync((char*)dst + done, buf + h * half, c, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipEventRecord(ev[h], s) != hipSuccess)
        return fail(IG_E_DEVICE, "staged copy failed");
      used[h] = true;
      h ^= 1;
      done += c;
    }
    return IG_OK;
  }
};
constexpr size_t kBounceHalf = (size_t)8 << 20;

// Bump allocation inside the host staging buffer of one create.
struct Staging {
  char* base = nullptr;
  size_t used = 0;
  static size_t round64(size_t b) { return (b + 63) & ~(size_t)63; }
  template <typename T>
  T* take(size_t count) {
    T* p = (T*)(base + used);
    used += round64(count * sizeof(T));
    return p;
  }
};

// value conversion of the stored transition data
template <typename T> struct VT_;
template <> struct VT_<double> {
  static double in(const double* p, int64_t e) { return p[e]; }
  static double out(double x, double* o) { *o = x; return x; }
};
template <> struct VT_<float> {
  static double in(const float* p, int64_t e) { return (double)p[e]; }
  static double out(double x, float* o) { *o = (float)x; return (double)*o; }
};
template <> struct VT_<uint16_t> {  // bf16 bit patterns
  static double in(const uint16_t* p, int64_t e) { return bf16_to_f64(p[e]); }
  static double out(double x, uint16_t* o) { *o = f32_to_bf16((float)x); return bf16_to_f64(*o); }
};

struct FillOut {
  int bad_col = 0, bad_dup = 0, bad_p = 0, bad_sum = 0;
  double max_stored_sum = 0.0;
};

// Sliced-ELL image of a CSR MDP: entry (a, j, lane) of slice b at
// off[b] + ((a*K_b + j) << 6) + lane for a < M_b (the slice's action
// blocks); padding (j >= row length, excluded pairs, lanes past n) is
// written as column 0, probability 0.  Every entry is written once; checks
// run over admissible pairs only.
template <typename IN, typename OUT>
FillOut fill_sell(int64_t n, int m, const int64_t* rp, const int32_t* col, const IN* val,
                  const int32_t* width, const int32_t* mcnt, const int64_t* off,
                  const uint8_t* adm, int32_t* scol, OUT* sval, bool validate, double sum_tol) {
  const int64_t ns = (n + kSlice - 1) / kSlice;
  FillOut F;
  int bad_col = 0, bad_dup = 0, bad_p = 0, bad_sum = 0;
  double mss = 0.0;
#pragma omp parallel reduction(+ : bad_col, bad_dup, bad_p, bad_sum) reduction(max : mss)
  {
    // duplicate test: stamp[c] == id of the row that last saw column c
    std::vector<uint32_t> stamp(validate ? (size_t)n : 0, 0u);
    uint32_t rid = 0;
#pragma omp for schedule(dynamic, 4)
    for (int64_t b = 0; b < ns; ++b) {
      const int Kb = width[b], Mb = mcnt[b];
      const int64_t ob = off[b];
      for (int l = 0; l < kSlice; ++l) {
        const int64_t s = b * kSlice + l;
        for (int a = 0; a < Mb; ++a) {
          const int64_t base = ob + (((int64_t)a * Kb) << 6) + l;
          const bool use = s < n && (!adm || adm[s * m + a]);
          int64_t lo = 0, len = 0;
          if (use) {
            lo = rp[s * m + a];
            len = rp[s * m + a + 1] - lo;
          }
          if (validate && len > 0 && ++rid == 0) {  // wrapped: forget all stamps
            std::fill(stamp.begin(), stamp.end(), 0u);
            rid = 1;
          }
          double sum = 0.0, ssum = 0.0;
          for (int64_t j = 0; j < len; ++j) {
            const int32_t c = col[lo + j];
            const bool ok = c >= 0 && c < n;
            bad_col += !ok;
            const double p = VT_<IN>::in(val, lo + j);
            if (validate) {
              bad_p += !(p >= 0.0 && p <= 1.0);
              if (ok) {
                bad_dup += stamp[c] == rid;
                stamp[c] = rid;
              }
            }
            sum += p;
            const int64_t pos = base + (j << 6);
            scol[pos] = ok ? c : 0;
            ssum += VT_<OUT>::out(p, &sval[pos]);
          }
          for (int64_t j = len; j < Kb; ++j) {
            const int64_t pos = base + (j << 6);
            scol[pos] = 0;
            VT_<OUT>::out(0.0, &sval[pos]);
          }
          if (use) {
            if (validate && !(std::fabs(sum - 1.0) <= sum_tol)) ++bad_sum;
            mss = std::max(mss, ssum);
          }
        }
      }
    }
  }
  F.bad_col = bad_col;
  F.bad_dup = bad_dup;
  F.bad_p = bad_p;
  F.bad_sum = bad_sum;
  F.max_stored_sum = mss;
  return F;
}

template <typename IN>
FillOut fill_sell_in(ig_dtype store, int64_t n, int m, const int64_t* rp, const int32_t* col,
                     const void* val, const int32_t* width, const int32_t* mcnt,
                     const int64_t* off, const uint8_t* adm, int32_t* scol, void* sval,
                     bool validate, double sum_tol) {
  const IN* v = (const IN*)val;
  switch (store) {
    case IG_FP64:
      return fill_sell<IN, double>(n, m, rp, col, v, width, mcnt, off, adm, scol, (double*)sval,
                                   validate, sum_tol);
    case IG_FP32:
      return fill_sell<IN, float>(n, m, rp, col, v, width, mcnt, off, adm, scol, (float*)sval,
                                  validate, sum_tol);
    default:
      return fill_sell<IN, uint16_t>(n, m, rp, col, v, width, mcnt, off, adm, scol,
                                     (uint16_t*)sval, validate, sum_tol);
  }
}

// zero fill on the handle's stream; plain handles wait for it
ig_status dzero(Mdp* d, void* dst, size_t bytes) {
  hipError_t e = hipMemsetAsync(dst, 0, bytes, d->stream);
  if (e == hipSuccess && !d->region) e = hipStreamSynchronize(d->stream);
  return e == hipSuccess ? IG_OK : fail(IG_E_DEVICE, "hipMemset failed");
}

void free_all(Mdp* d) {
  const bool dev = d->region == nullptr;
  auto F = [dev](void* p) {
    if (p && dev) (void)hipFree(p);
  };
  F(d->col); F(d->val); F(d->off); F(d->width); F(d->mcnt); F(d->offp); F(d->pcol); F(d->pval);
  F(d->in_pval); F(d->in_P);
  F(d->adm);
  F(d->P); F(d->cost); F(d->cpi); F(d->st); F(d->gs); F(d->part); F(d->pctl);
  F(d->ws.Q); F(d->ws.wA); F(d->ws.wB); F(d->ws.Vb); F(d->ws.r); F(d->ws.t); F(d->ws.pi);
  F(d->ws.pa); F(d->ws.pb);
  if (d->own_host_mirrors) {
    if (d->hst) (void)hipHostFree(d->hst);
    if (d->hpctl) (void)hipHostFree(d->hpctl);
    if (d->hsnap) (void)hipHostFree(d->hsnap);
  }
  if (d->ev0) (void)hipEventDestroy(d->ev0);
  if (d->ev_step) (void)hipEventDestroy(d->ev_step);
  if (d->ev1) (void)hipEventDestroy(d->ev1);
  for (auto& pool : d->prof_ev)
    for (auto& pr : pool) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
}

int pow2_at_least(int64_t x, int cap) {
  int p = 1;
  while (p < x && p < cap) p <<= 1;
  return p;
}

template <typename T>
std::vector<T> to_host(const T* p, size_t count, bool on_device, ig_status* st) {
  std::vector<T> v;
  *st = IG_OK;
  if (!on_device) return v;
  v.resize(count);
  if (count && hipMemcpy(v.data(), p, count * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    *st = fail(IG_E_DEVICE, "copy of device input to host failed");
  }
  return v;
}

}  // namespace

// partial rows: kMaxBlocks * 8 for streaming kernels, one kPartStride row per
// block of the Gram-Schmidt kernels, two sets of 256 rows for the persistent
// engine
size_t part_doubles(int64_t) {
  return (size_t)std::max<int64_t>({(int64_t)kMaxBlocks * 8, (int64_t)2 * 256 * 72,
                                    (int64_t)kGsBlocks * kPartStride});
}

ig_status ensure_workspace(Mdp& d, int W, bool fp32) {
  struct RegionScope {
    DevRegion* prev;
    explicit RegionScope(DevRegion* r) : prev(t_region) { t_region = r; }
    ~RegionScope() { t_region = prev; }
  } scope(d.region);
  Workspace& w = d.ws;
  const size_t n = (size_t)d.n;
  if (!w.Vb) {
    if (dmalloc(&w.Vb, n * 8) || dmalloc(&w.r, n * 8) || dmalloc(&w.t, n * 8) ||
        dmalloc(&w.pi, n * 4))
      return IG_E_NOMEM;
  }
  if (w.Q && w.W >= W && w.fp32 == fp32) return IG_OK;
  if (d.region && w.Q) return fail(IG_E_TOO_LARGE, "workspace of a region handle cannot grow");
  if (w.Q) (void)hipFree(w.Q);
  if (w.wA) (void)hipFree(w.wA);
  if (w.wB) (void)hipFree(w.wB);
  w.Q = w.wA = w.wB = nullptr;
  w.W = 0;
  const size_t xb = fp32 ? 4 : 8;
  if (dmalloc(&w.Q, (size_t)(W + 1) * n * xb) || dmalloc(&w.wA, n * xb) || dmalloc(&w.wB, n * xb))
    return IG_E_NOMEM;
  w.W = W;
  w.fp32 = fp32;
  return IG_OK;
}


static ig_status create_impl(const ig_mdp_desc* desc, hipStream_t stream, Mdp* d) {
  if (!desc) return fail(IG_E_INVALID, "desc is NULL");
  const int64_t n = desc->n;
  const int m = desc->m;
  if (n < 1 || m < 1) return fail(IG_E_INVALID, "need n >= 1 and m >= 1");
  if (n > (int64_t)INT32_MAX) return fail(IG_E_INVALID, "n must fit in int32 column indices");
  if (!(desc->gamma > 0.0 && desc->gamma < 1.0)) return fail(IG_E_INVALID, "gamma must be in (0,1)");
  if (desc->fmt != IG_FMT_CSR && desc->fmt != IG_FMT_DENSE) return fail(IG_E_INVALID, "bad format");
  for (ig_dtype t : {desc->val_type, desc->store})
    if (t != IG_FP64 && t != IG_FP32 && t != IG_BF16) return fail(IG_E_INVALID, "bad dtype");
  if (dtype_bytes(desc->store) > dtype_bytes(desc->val_type))
    return fail(IG_E_INVALID, "storage type wider than the input type");
  if (desc->refine != 0 && desc->refine != 1) return fail(IG_E_INVALID, "refine must be 0 or 1");
  if (desc->refine && (desc->store != IG_BF16 || desc->val_type == IG_BF16))
    return fail(IG_E_INVALID, "refine needs store IG_BF16 and FP64 or FP32 input values");
  if (!desc->val || !desc->cost) return fail(IG_E_INVALID, "val and cost are required");
  if (desc->fmt == IG_FMT_CSR && (!desc->row_ptr || !desc->col))
    return fail(IG_E_INVALID, "CSR needs row_ptr and col");

  d->n = n;
  d->m = m;
  d->gamma = desc->gamma;
  d->fmt = desc->fmt;
  // refine: the arrays built below hold the FP32 copy; the BF16 one follows
  d->refine = desc->refine != 0;
  d->store = d->refine ? IG_FP32 : desc->store;
  d->vb = dtype_bytes(d->store);
  d->in_store = desc->store;
  d->in_vb = dtype_bytes(desc->store);
  const int64_t R = n * (int64_t)m;
  const bool ondev = desc->inputs_on_device != 0;
  ig_status st;

  // ---- costs (always checked finite) ----
  std::vector<double> cost_h = to_host(desc->cost, (size_t)R, ondev, &st);
  if (st) return st;
  const double* cost = ondev ? cost_h.data() : desc->cost;
  // action sets A(s): admissibility mask [s][a] (null: every action)
  std::vector<uint8_t> adm_h;
  const uint8_t* adm = nullptr;
  if (desc->admissible) {
    adm_h = to_host(desc->admissible, (size_t)R, ondev, &st);
    if (st) return st;
    adm = ondev ? adm_h.data() : desc->admissible;
    int64_t empty = 0;
#pragma omp parallel for reduction(+ : empty)
    for (int64_t s = 0; s < n; ++s) {
      bool any = false;
      for (int a = 0; a < m; ++a) any = any || adm[s * m + a] != 0;
      empty += !any;
    }
    if (empty) return fail(IG_E_INVALID, "every state needs at least one admissible action");
  }
  auto admissible = [adm, m](int64_t s, int a) { return !adm || adm[s * m + a] != 0; };
  const double sum_tol = desc->val_type == IG_FP64 ? 1e-10 : 1.0 / 64.0;
  const bool validate = desc->validate != 0;

  // ---- host staging: one buffer for every array that is uploaded ----
  std::unique_ptr<char[]> local_stage;  // every byte is written before the upload
  Staging hs;
  auto stage_get = [&](size_t need) -> ig_status {
    if (d->stage) {
      hs.base = d->stage->get(need);
      if (!hs.base) return fail(IG_E_NOMEM, "pinned staging allocation failed");
    } else {
      local_stage.reset(new (std::nothrow) char[need]);
      if (!local_stage) return fail(IG_E_NOMEM, "host staging allocation failed");
      hs.base = local_stage.get();
    }
    return IG_OK;
  };
  double* cost_t = nullptr;
  auto transpose_costs = [&]() -> ig_status {
    cost_t = hs.take<double>((size_t)R);
    int bad_cost = 0;
    double cmax = 0.0;
#pragma omp parallel for reduction(+ : bad_cost) reduction(max : cmax)
    for (int64_t s = 0; s < n; ++s)
      for (int a = 0; a < m; ++a) {
        if (!admissible(s, a)) {  // ignored: a neutral value on the device
          cost_t[(size_t)a * n + s] = 0.0;
          continue;
        }
        const double c = cost[s * m + a];
        if (!std::isfinite(c)) ++bad_cost;
        else cmax = std::max(cmax, std::fabs(c));
        cost_t[(size_t)a * n + s] = c;
      }
    if (bad_cost) return fail(IG_E_INVALID, "costs of admissible pairs must be finite");
    d->cost_max = cmax;
    return IG_OK;
  };

  uint8_t* adm_t = nullptr;  // [m][n] on the host staging
  auto transpose_adm = [&]() {
    if (!adm) return;
    adm_t = hs.take<uint8_t>((size_t)R);
#pragma omp parallel for
    for (int64_t s = 0; s < n; ++s)
      for (int a = 0; a < m; ++a) adm_t[(size_t)a * n + s] = adm[s * m + a] != 0;
  };
  const size_t adm_bytes = adm ? Staging::round64((size_t)R) : 0;

  if (desc->fmt == IG_FMT_CSR) {
    std::vector<int64_t> rp_h = to_host(desc->row_ptr, (size_t)R + 1, ondev, &st);
    if (st) return st;
    const int64_t* rp = ondev ? rp_h.data() : desc->row_ptr;
    if (rp[0] != 0) return fail(IG_E_INVALID, "row_ptr[0] must be 0");
    int bad_rows = 0;
#pragma omp parallel for reduction(+ : bad_rows)
    for (int64_t r = 0; r < R; ++r)
      if (rp[r + 1] < rp[r] || (rp[r + 1] == rp[r] && admissible(r / m, (int)(r % m)))) ++bad_rows;
    if (bad_rows)
      return fail(IG_E_INVALID, "row_ptr must be nondecreasing and every admissible (s,a) row non-empty");
    const int64_t nnz = rp[R];

    // per 64-state slice: width (longest admissible row) and action blocks
    // (1 + largest admissible action index of its states)
    const int64_t ns = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> width((size_t)ns, 0), mblk((size_t)ns, 0);
    int64_t maxlen = 0;
#pragma omp parallel for reduction(max : maxlen)
    for (int64_t b = 0; b < ns; ++b) {
      int64_t w = 0;
      int mb = 0;
      for (int64_t s = b * kSlice; s < std::min(n, (b + 1) * kSlice); ++s)
        for (int a = 0; a < m; ++a)
          if (admissible(s, a)) {
            w = std::max(w, rp[s * m + a + 1] - rp[s * m + a]);
            mb = std::max(mb, a + 1);
          }
      width[b] = (int32_t)w;
      mblk[b] = mb;
      maxlen = std::max(maxlen, w);
    }
    if (maxlen > n) return fail(IG_E_INVALID, "a row has more entries than states");
    // The entries (O(nnz)) are converted on the device for serving, for
    // device-resident inputs and for large MDPs; only the per-slice layout
    // (O(rows)) is computed here.  The device's repeated-column test is
    // quadratic in the row length, so host inputs with long rows stay on the
    // host.  IG_CONVERT=host|device forces a route.
    bool dev_route = d->region != nullptr || ondev || nnz >= ((int64_t)1 << 22);
    if (validate && maxlen > 128 && !ondev) dev_route = false;
    if (const char* ev = std::getenv("IG_CONVERT")) {
      if (!std::strcmp(ev, "host")) dev_route = false;
      if (!std::strcmp(ev, "device")) dev_route = true;
    }
    std::vector<int32_t> col_h;
    std::vector<uint8_t> val_h;
    const int32_t* col = desc->col;
    const void* valp = desc->val;
    if (ondev && !dev_route) {
      col_h = to_host(desc->col, (size_t)nnz, ondev, &st);
      if (st) return st;
      col = col_h.data();
      val_h.resize((size_t)nnz * dtype_bytes(desc->val_type));
      if (hipMemcpy(val_h.data(), desc->val, val_h.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(IG_E_DEVICE, "copy of device values failed");
      valp = val_h.data();
    }
    int64_t tot = 0, totp = 0;
    for (int64_t b = 0; b < ns; ++b) {
      tot += (int64_t)mblk[b] * width[b] * kSlice;
      totp += (int64_t)width[b] * kSlice;
    }
    const size_t ell_host = dev_route ? 0
                                      : Staging::round64((size_t)tot * 4) +
                                            Staging::round64((size_t)tot * d->vb);
    // serving (pinned staging) bounces the raw arrays of the device route
    const bool bounce = dev_route && d->stage && !ondev;
    const size_t need = Staging::round64((size_t)R * 8) + ell_host +
                        2 * Staging::round64((size_t)ns * 8) + 2 * Staging::round64((size_t)ns * 4) +
                        adm_bytes + (bounce ? 2 * kBounceHalf : 0);
    if (ig_status e = stage_get(need)) return e;
    if (ig_status e = transpose_costs()) return e;
    transpose_adm();
    int64_t* off = hs.take<int64_t>((size_t)ns);
    int64_t* offp = hs.take<int64_t>((size_t)ns);
    int32_t* wid = hs.take<int32_t>((size_t)ns);
    int32_t* mc = hs.take<int32_t>((size_t)ns);
    Bounce bb;
    if (bounce) {
      if (!d->stage->events()) return fail(IG_E_DEVICE, "hipEventCreate failed");
      bb.buf = hs.take<char>(2 * kBounceHalf);
      bb.half = kBounceHalf;
      bb.ev = d->stage->ev;
    }
    int32_t* scol = dev_route ? nullptr : hs.take<int32_t>((size_t)tot);
    void* sval = dev_route ? nullptr : hs.take<char>((size_t)tot * d->vb);
    for (int64_t b = 0, t = 0, tp = 0; b < ns; ++b) {
      off[b] = t;
      offp[b] = tp;
      wid[b] = width[b];
      mc[b] = mblk[b];
      t += (int64_t)mblk[b] * width[b] * kSlice;
      tp += (int64_t)width[b] * kSlice;
    }
    FillOut F;
    if (!dev_route) switch (desc->val_type) {
      case IG_FP64:
        F = fill_sell_in<double>(d->store, n, m, rp, col, valp, wid, mc, off, adm, scol, sval, validate,
                                 sum_tol);
        break;
      case IG_FP32:
        F = fill_sell_in<float>(d->store, n, m, rp, col, valp, wid, mc, off, adm, scol, sval, validate,
                                 sum_tol);
        break;
      default:
        F = fill_sell_in<uint16_t>(d->store, n, m, rp, col, valp, wid, mc, off, adm, scol, sval, validate,
                                 sum_tol);
        break;
    }
    // checks, in this order for both routes (device counts arrive below)
    auto check = [&](const FillOut& F) -> ig_status {
      if (F.bad_col) return fail(IG_E_INVALID, "column index out of range");
      if (F.bad_dup) return fail(IG_E_INVALID, "repeated column inside a row");
      if (F.bad_p) return fail(IG_E_INVALID, "probabilities must lie in [0,1]");
      if (F.bad_sum) return fail(IG_E_INVALID, "a transition row does not sum to 1");
      if (validate && !(d->gamma * F.max_stored_sum < 1.0))
        return fail(IG_E_INVALID, "gamma * (largest stored row sum) must be < 1");
      return IG_OK;
    };
    if (!dev_route)
      if (ig_status e = check(F)) return e;

    d->nslices = ns;
    d->maxK = (int)maxlen;
    d->nnz = nnz;
    d->stored = tot;
    d->stored_pi = totp;
    d->h_width = width;
    if (dmalloc(&d->col, (size_t)(tot + kRowPad) * 4) ||
        dmalloc(&d->val, (size_t)(tot + kRowPad) * d->vb) ||
        dmalloc(&d->off, (size_t)ns * 8) || dmalloc(&d->offp, (size_t)ns * 8) ||
        dmalloc(&d->width, (size_t)ns * 4) || dmalloc(&d->mcnt, (size_t)ns * 4) ||
        dmalloc(&d->pcol, (size_t)(totp + kRowPad) * 4) ||
        dmalloc(&d->pval, (size_t)(totp + kRowPad) * d->vb))
      return IG_E_NOMEM;
    if (!dev_route) {
      if (ig_status e = upload(d, d->col, scol, (size_t)tot * 4)) return e;
      if (ig_status e = upload(d, d->val, sval, (size_t)tot * d->vb)) return e;
    }
    if (ig_status e = upload(d, d->off, off, (size_t)ns * 8)) return e;
    if (ig_status e = dzero(d, d->col + tot, (size_t)kRowPad * 4)) return e;
    if (ig_status e = dzero(d, (char*)d->val + (size_t)tot * d->vb, (size_t)kRowPad * d->vb)) return e;
    if (ig_status e = upload(d, d->offp, offp, (size_t)ns * 8)) return e;
    if (ig_status e = upload(d, d->width, wid, (size_t)ns * 4)) return e;
    if (ig_status e = upload(d, d->mcnt, mc, (size_t)ns * 4)) return e;
    if (dev_route) {
      // raw CSR on the device (the caller's arrays when they are already
      // there), then the conversion kernel and its counts
      if (adm_t) {
        if (dmalloc(&d->adm, (size_t)R)) return IG_E_NOMEM;
        if (ig_status e = upload(d, d->adm, adm_t, (size_t)R)) return e;
      }
      const size_t vin = dtype_bytes(desc->val_type);
      int64_t* rp_d = nullptr;
      int32_t* col_d = nullptr;
      char* val_d = nullptr;
      unsigned long long* err_d = nullptr;
      const bool temp = d->region == nullptr;  // plain allocations to free here
      size_t top = 0;                           // region mode: bytes taken from its top
      auto free_temp = [&]() {
        if (!temp) return;
        if (!ondev) {
          if (rp_d) (void)hipFree(rp_d);
          if (col_d) (void)hipFree(col_d);
          if (val_d) (void)hipFree(val_d);
        }
        if (err_d) (void)hipFree(err_d);
      };
      if (ondev) {
        rp_d = const_cast<int64_t*>(desc->row_ptr);
        col_d = const_cast<int32_t*>(desc->col);
        val_d = (char*)const_cast<void*>(desc->val);
      } else if (temp ? (dmalloc(&rp_d, ((size_t)R + 1) * 8) || dmalloc(&col_d, (size_t)nnz * 4) ||
                         dmalloc(&val_d, (size_t)nnz * vin))
                      : (dmalloc_top(&rp_d, ((size_t)R + 1) * 8, &top) ||
                         dmalloc_top(&col_d, (size_t)nnz * 4, &top) ||
                         dmalloc_top(&val_d, (size_t)nnz * vin, &top))) {
        free_temp();
        return fail(IG_E_NOMEM, "device staging of the CSR arrays");
      }
      if (temp ? dmalloc(&err_d, 5 * sizeof(unsigned long long))
               : dmalloc_top(&err_d, 5 * sizeof(unsigned long long), &top)) {
        free_temp();
        return fail(IG_E_NOMEM, "device staging of the CSR arrays");
      }
      ig_status e = IG_OK;
      if (bounce) {
        e = bb.put(d->stream, rp_d, desc->row_ptr, ((size_t)R + 1) * 8);
        if (!e) e = bb.put(d->stream, col_d, desc->col, (size_t)nnz * 4);
        if (!e) e = bb.put(d->stream, val_d, desc->val, (size_t)nnz * vin);
      } else if (!ondev) {
        e = upload(d, rp_d, desc->row_ptr, ((size_t)R + 1) * 8);
        if (!e) e = upload(d, col_d, desc->col, (size_t)nnz * 4);
        if (!e) e = upload(d, val_d, desc->val, (size_t)nnz * vin);
      }
      if (!e) e = dzero(d, err_d, 5 * sizeof(unsigned long long));
      // plain mode copied with blocking calls; order them before the kernel
      if (!e && !d->region && hipDeviceSynchronize() != hipSuccess)
        e = fail(IG_E_DEVICE, "device staging of the CSR arrays");
      if (!e) {
        ConvArgs c{n, m, rp_d, col_d, val_d, d->adm, d->off, d->width, d->mcnt, d->col, d->val,
                   (int)maxlen, validate ? 1 : 0, sum_tol, err_d};
        launch_fill_sell(c, desc->val_type, d->store, d->stream);
        if (hipGetLastError() != hipSuccess) e = fail(IG_E_DEVICE, "conversion kernel launch failed");
      }
      unsigned long long cnt[5] = {0, 0, 0, 0, 0};
      if (!e) {
        const hipError_t h = d->region ? hipStreamSynchronize(d->stream) : hipDeviceSynchronize();
        if (h != hipSuccess || hipMemcpy(cnt, err_d, sizeof cnt, hipMemcpyDeviceToHost) != hipSuccess)
          e = fail(IG_E_DEVICE, "device conversion failed");
      }
      free_temp();
      if (e) return e;
      FillOut G;
      G.bad_col = cnt[0] ? 1 : 0;
      G.bad_dup = cnt[1] ? 1 : 0;
      G.bad_p = cnt[2] ? 1 : 0;
      G.bad_sum = cnt[3] ? 1 : 0;
      double mss;
      std::memcpy(&mss, &cnt[4], 8);
      G.max_stored_sum = mss;
      if (ig_status e2 = check(G)) return e2;
    }
    if (ig_status e = dzero(d, d->pcol, (size_t)(totp + kRowPad) * 4)) return e;
    if (ig_status e = dzero(d, d->pval, (size_t)(totp + kRowPad) * d->vb)) return e;
    if (d->refine) {  // BF16 compact P^pi, rounded from the FP32 one per policy
      if (dmalloc(&d->in_pval, (size_t)(totp + kRowPad) * d->in_vb)) return IG_E_NOMEM;
      if (ig_status e = dzero(d, d->in_pval, (size_t)(totp + kRowPad) * d->in_vb)) return e;
    }

    // lanes per state: enough lanes in flight to cover latency on 256 CUs
    const int64_t target = (int64_t)1 << 18;
    const int want = pow2_at_least((target + n - 1) / n, 64);
    d->G_bell = std::min(pow2_at_least(m, 64), want);
    d->G_jap = std::min(pow2_at_least(std::max<int64_t>(1, maxlen), 64), want);
  } else {
    const int64_t total = R * n;
    std::vector<uint8_t> val_h;
    const void* valp = desc->val;
    if (ondev) {
      val_h.resize((size_t)total * dtype_bytes(desc->val_type));
      if (hipMemcpy(val_h.data(), desc->val, val_h.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(IG_E_DEVICE, "copy of device values failed");
      valp = val_h.data();
    }
    const ValReader rv{valp, desc->val_type};
    if (ig_status e = stage_get(Staging::round64((size_t)R * 8) +
                                Staging::round64((size_t)total * d->vb) + adm_bytes))
      return e;
    if (ig_status e = transpose_costs()) return e;
    transpose_adm();
    uint8_t* sval = hs.take<uint8_t>((size_t)total * d->vb);
    int bad_p = 0, bad_sum = 0;
    double max_stored_sum = 0.0;
#pragma omp parallel for reduction(+ : bad_p, bad_sum) reduction(max : max_stored_sum) schedule(dynamic, 64)
    for (int64_t r = 0; r < R; ++r) {
      const bool use = admissible(r / m, (int)(r % m));
      double sum = 0.0, ssum = 0.0;
      for (int64_t e = r * n; e < (r + 1) * n; ++e) {
        const double p = use ? rv(e) : 0.0;  // excluded rows: stored as zeros
        if (validate && !(p >= 0.0 && p <= 1.0)) ++bad_p;
        sum += p;
        ssum += store_val(sval, e, d->store, p);
      }
      if (use && validate && !(std::fabs(sum - 1.0) <= sum_tol)) ++bad_sum;
      max_stored_sum = std::max(max_stored_sum, ssum);
    }
    if (bad_p) return fail(IG_E_INVALID, "probabilities must lie in [0,1]");
    if (bad_sum) return fail(IG_E_INVALID, "a transition row does not sum to 1");
    if (validate && !(d->gamma * max_stored_sum < 1.0))
      return fail(IG_E_INVALID, "gamma * (largest stored row sum) must be < 1");
    d->nnz = total;
    d->stored = total;
    d->maxK = (int)n;
    if (dmalloc(&d->P, (size_t)total * d->vb)) return IG_E_NOMEM;
    if (ig_status e = upload(d, d->P, sval, (size_t)total * d->vb)) return e;
    if (d->refine) {  // BF16 copy of all of P, rounded from the FP32 copy
      if (dmalloc(&d->in_P, (size_t)total * d->in_vb)) return IG_E_NOMEM;
      if (!d->region) IG_HIP(hipDeviceSynchronize());
      launch_round_bf16((const float*)d->P, d->in_P, total, d->stream);
      IG_HIP(hipGetLastError());
    }
  }

  if (dmalloc(&d->cost, (size_t)R * 8) || dmalloc(&d->cpi, (size_t)n * 8) ||
      dmalloc(&d->st, sizeof(DevStatus)) || dmalloc(&d->gs, sizeof(GivensState)) ||
      dmalloc(&d->part, part_doubles(d->n) * 8) ||
      dmalloc(&d->pctl, sizeof(PCtl)))
    return IG_E_NOMEM;
  if (ig_status e = upload(d, d->cost, cost_t, (size_t)R * 8)) return e;
  if (adm_t && !d->adm) {
    if (dmalloc(&d->adm, (size_t)R)) return IG_E_NOMEM;
    if (ig_status e = upload(d, d->adm, adm_t, (size_t)R)) return e;
  }
  if (ig_status e = dzero(d, d->st, sizeof(DevStatus))) return e;
  if (ig_status e = dzero(d, d->gs, sizeof(GivensState))) return e;
  if (d->own_host_mirrors &&
      (hipHostMalloc((void**)&d->hst, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess ||
       hipHostMalloc((void**)&d->hpctl, sizeof(PCtl), hipHostMallocDefault) != hipSuccess ||
       hipHostMalloc((void**)&d->hsnap, sizeof(StepSnap), hipHostMallocDefault) != hipSuccess))
    return fail(IG_E_NOMEM, "hipHostMalloc failed");
  if (ig_status e = dzero(d, d->pctl, sizeof(PCtl))) return e;
  if (d->hst) std::memset(d->hst, 0, sizeof(DevStatus));
  if (d->hsnap) std::memset(d->hsnap, 0, sizeof(StepSnap));
  IG_HIP(hipEventCreate(&d->ev0));
  IG_HIP(hipEventCreate(&d->ev1));
  IG_HIP(hipEventCreateWithFlags(&d->ev_step, hipEventDisableTiming));
  IG_HIP(hipGetDevice(&d->device));
  int coop = 0;
  IG_HIP(hipDeviceGetAttribute(&d->num_cu, hipDeviceAttributeMultiprocessorCount, d->device));
  IG_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, d->device));
  IG_HIP(hipDeviceGetAttribute(&d->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, d->device));
  d->coop = coop != 0;
  // uploads from the local staging must finish before it goes away
  if (!d->region) IG_HIP(hipDeviceSynchronize());
  else if (!d->stage) IG_HIP(hipStreamSynchronize(d->stream));
  (void)stream;
  return IG_OK;
}

char* PinnedStage::get(size_t need) {
  if (need <= cap) return buf;
  if (buf) retired.push_back(buf);
  buf = nullptr;
  const size_t want = std::max(need, 2 * cap);
  if (hipHostMalloc((void**)&buf, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    buf = nullptr;
    cap = 0;
    return nullptr;
  }
  cap = want;
  return buf;
}

bool PinnedStage::events() {
  for (hipEvent_t& e : ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
      return false;
    }
  return true;
}

void PinnedStage::release() {
  for (hipEvent_t& e : ev)
    if (e) (void)hipEventDestroy(e), e = nullptr;
  for (char* p : retired) (void)hipHostFree(p);
  retired.clear();
  if (buf) (void)hipHostFree(buf);
  buf = nullptr;
  cap = 0;
}

// the two n-vectors of the Neumann preconditioner (stream engine only)
ig_status ensure_precond(Mdp& d) {
  if (d.ws.pa) return IG_OK;
  if (d.region) return fail(IG_E_INVALID, "a region handle has no preconditioner buffers");
  if (dmalloc(&d.ws.pa, (size_t)d.n * 8) || dmalloc(&d.ws.pb, (size_t)d.n * 8))
    return fail(IG_E_NOMEM, "preconditioner buffers");
  return IG_OK;
}

// create_impl with the handle's region (if any) as the allocation target
ig_status create_in(const ig_mdp_desc* desc, Mdp* d) {
  struct RegionScope {
    DevRegion* prev;
    explicit RegionScope(DevRegion* r) : prev(t_region) { t_region = r; }
    ~RegionScope() { t_region = prev; }
  } scope(d->region);
  try {
    return create_impl(desc, d->stream, d);
  } catch (const std::bad_alloc&) {
    return fail(IG_E_NOMEM, "host allocation failed while converting the MDP");
  }
}

// release what a handle holds (no device synchronisation; region handles
// return nothing to the allocator, their region is the owner's)
void release_handle(Mdp* d) { free_all(d); }

// one more allocation from a region handle's region
ig_status region_alloc(Mdp& d, size_t bytes, void** p) {
  if (!d.region) return fail(IG_E_INVALID, "handle has no region");
  struct RegionScope {
    DevRegion* prev;
    explicit RegionScope(DevRegion* r) : prev(t_region) { t_region = r; }
    ~RegionScope() { t_region = prev; }
  } scope(d.region);
  char* q = nullptr;
  if (ig_status e = dmalloc(&q, bytes)) return e;
  *p = q;
  return IG_OK;
}

// Device bytes that create_in + ensure_workspace(restart, fp32) allocate,
// each allocation rounded to 256 bytes.
ig_status device_footprint(const ig_mdp_desc* desc, int restart, bool fp32, size_t* bytes) {
  if (!desc || !bytes || desc->n < 1 || desc->m < 1) return fail(IG_E_INVALID, "bad description");
  const int64_t n = desc->n, R = n * (int64_t)desc->m;
  // refine: an FP32 copy of P, plus BF16 P^pi (sparse) or BF16 P (dense)
  const size_t vb = desc->refine ? 4 : dtype_bytes(desc->store);
  size_t b = 0, staging = 0;
  if (desc->fmt == IG_FMT_CSR) {
    if (desc->inputs_on_device) return fail(IG_E_INVALID, "footprint needs host CSR arrays");
    const int64_t* rp = desc->row_ptr;
    const uint8_t* adm = desc->admissible;
    const int m = desc->m;
    const int64_t ns = (n + kSlice - 1) / kSlice;
    int64_t tot = 0, totp = 0;
#pragma omp parallel for reduction(+ : tot, totp)
    for (int64_t sl = 0; sl < ns; ++sl) {
      int64_t w = 0;
      int mb = 0;
      for (int64_t s = sl * kSlice; s < std::min(n, (sl + 1) * kSlice); ++s)
        for (int a = 0; a < m; ++a)
          if (!adm || adm[s * m + a]) {
            w = std::max(w, rp[s * m + a + 1] - rp[s * m + a]);
            mb = std::max(mb, a + 1);
          }
      tot += (int64_t)mb * w * kSlice;
      totp += w * kSlice;
    }
    b += round256((tot + kRowPad) * 4) + round256((tot + kRowPad) * vb) + 2 * round256(ns * 8) +
         2 * round256(ns * 4) +
         round256((totp + kRowPad) * 4) + round256((totp + kRowPad) * vb);
    if (desc->refine) b += round256((totp + kRowPad) * 2);
    // raw CSR staging of the device conversion: taken from the top of a
    // region after the sliced-ELL arrays (and the mask), dead once the
    // conversion is done, so the later allocations may reuse its bytes
    const int64_t nnz = rp[R];
    staging = round256((R + 1) * 8) + round256(nnz * 4) + round256(nnz * dtype_bytes(desc->val_type)) +
              round256(5 * sizeof(unsigned long long));
  } else {
    b += round256((size_t)R * n * vb);
    if (desc->refine) b += round256((size_t)R * n * 2);
  }
  if (desc->admissible) b += round256(R);
  const size_t at_staging = b + staging;
  b += round256(R * 8) + round256(n * 8) + round256(sizeof(DevStatus)) +
       round256(sizeof(GivensState)) + round256(part_doubles(n) * 8) + round256(sizeof(PCtl));
  const size_t xb = fp32 ? 4 : 8;
  b += 3 * round256(n * 8) + round256(n * 4);                             // Vb, r, t, pi
  b += round256((size_t)(restart + 1) * n * xb) + 2 * round256(n * xb);  // Q, wA, wB
  *bytes = std::max(b, at_staging);
  return IG_OK;
}

}  // namespace ig

struct ig_mdp_s {
  ig::Mdp d;
};

extern "C" {

const char* ig_last_error(void) { return ig::g_last_error.c_str(); }

void ig_params_default(ig_params* p, double gamma) {
  if (!p) return;
  p->alpha = 0.5 * (1.0 - gamma) / (1.0 + gamma);
  p->restart = 30;
  p->max_outer = 1000;
  p->max_inner = 100000;
  p->tol = 1e-8;
  p->mode = IG_MODE_FP64;
  p->opi_sweeps = 20;
  p->forcing = 0;
  p->eval_rtol = 1e-13;
  p->engine = 0;
  p->blocks = 0;
  p->precond = 0;
  p->polish = 0;
}

ig_status mdp_create(const ig_mdp_desc* desc, void* stream, ig_mdp_t* out) {
  if (!out) return ig::fail(IG_E_INVALID, "out is NULL");
  *out = nullptr;
  std::unique_ptr<ig_mdp_s> h;
  try {
    h.reset(new ig_mdp_s());
  } catch (...) {
    return ig::fail(IG_E_NOMEM, "host allocation failed");
  }
  ig_status st;
  try {
    st = ig::create_impl(desc, (hipStream_t)stream, &h->d);
  } catch (const std::bad_alloc&) {
    st = ig::fail(IG_E_NOMEM, "host allocation failed while converting the MDP");
  } catch (...) {
    st = ig::fail(IG_E_INVALID, "unexpected failure while converting the MDP");
  }
  if (st != IG_OK) {
    ig::free_all(&h->d);
    return st;
  }
  *out = h.release();
  return IG_OK;
}

void mdp_destroy(ig_mdp_t mdp) {
  if (!mdp) return;
  (void)hipDeviceSynchronize();
  ig::free_all(&mdp->d);
  delete mdp;
}

ig_status mdp_get_info(ig_mdp_t mdp, ig_mdp_info* info) {
  if (!mdp || !info) return ig::fail(IG_E_INVALID, "NULL argument");
  const ig::Mdp& d = mdp->d;
  info->n = d.n;
  info->m = d.m;
  info->max_width = d.maxK;
  info->nnz = d.nnz;
  info->stored_entries = d.stored;
  info->p_bytes = d.stored * (int64_t)(d.vb + (d.fmt == IG_FMT_CSR ? 4 : 0));
  info->store = d.store;
  info->fmt = d.fmt;
  info->gamma = d.gamma;
  info->persistent_ok = (d.coop && ig::persistent_fits(d)) ? 1 : 0;
  info->persistent_blocks = info->persistent_ok ? ig::persistent_grid(d) : 0;
  info->refine = d.refine ? 1 : 0;
  info->inner_p_bytes =
      !d.refine ? 0 : (d.fmt == IG_FMT_CSR ? d.stored_pi : d.stored) * (int64_t)d.in_vb;
  return IG_OK;
}

ig_status ig_profile_enable(ig_mdp_t mdp, unsigned mask) {
  if (!mdp) return ig::fail(IG_E_INVALID, "NULL handle");
  mdp->d.prof_mask = mask;
  for (auto& c : mdp->d.prof_seen) c = 0;
  return IG_OK;
}

ig_status ig_profile_sample(ig_mdp_t mdp, int every) {
  if (!mdp) return ig::fail(IG_E_INVALID, "NULL handle");
  if (every < 1) return ig::fail(IG_E_INVALID, "every must be >= 1");
  mdp->d.prof_every = (uint32_t)every;
  for (auto& c : mdp->d.prof_seen) c = 0;
  return IG_OK;
}

ig_status ig_profile_read(ig_mdp_t mdp, double* ms, int64_t* launches, int reset) {
  if (!mdp || !ms || !launches) return ig::fail(IG_E_INVALID, "NULL argument");
  ig::Mdp& d = mdp->d;
  for (int k = 0; k < ig::KC_COUNT; ++k) {
    double tot = 0.0;
    for (size_t i = 0; i < d.prof_used[k]; ++i) {
      auto& pr = d.prof_ev[k][i];
      if (hipEventSynchronize(pr.second) != hipSuccess) return ig::fail(IG_E_DEVICE, "event sync");
      float t = 0.f;
      if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess)
        return ig::fail(IG_E_DEVICE, "event elapsed");
      tot += t;
    }
    ms[k] = tot;
    launches[k] = (int64_t)d.prof_used[k];
    if (reset) {
      d.prof_used[k] = 0;
      d.prof_seen[k] = 0;
    }
  }
  return IG_OK;
}

}  // extern "C"

// access for the solver translation unit
namespace ig {
Mdp* handle_of(ig_mdp_t h) { return h ? &h->d : nullptr; }
}  // namespace ig
