// Continuous-batching serving of Algorithm 2 solves on one GPU.
//
// Life of a request:
//   srv_submit            queued (arrays borrowed from the caller)
//   prep thread           device footprint; first-fit allocation in the
//                         arena, strictly in submission order (a request
//                         that does not fit waits for retirements); host
//                         conversion to the sliced-ELL layout and upload on
//                         the thread's own stream, into the allocation
//   scheduler thread      launch of the persistent solve on a free slot
//                         stream once its workgroups fit the co-residency
//                         budget; D2H of V, pi and the control block into
//                         the slot's pinned buffers; completion event
//   scheduler thread      retirement: results copied to the request, arena
//                         space, slot and budget returned, waiters woken
// Admission and retirement run while other solves are on the device.
//
// Co-residency: the persistent solve synchronises its workgroups with grid
// barriers, so every workgroup of every running solve must be resident.  A
// plain launch is dispatched round-robin over the 8 XCDs, so a solve of b
// workgroups places at most ceil(b/8) on any XCD; the scheduler keeps the sum
// of ceil(b/8) over running solves within the workgroups one XCD holds at
// once (one 1024-thread workgroup per CU: the solve's LDS exceeds half a CU).
// The barrier's bounded wait turns any violation into an error, not a hang.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include <omp.h>

#include "internal.hpp"

namespace ig {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
    total_ = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_alloc(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_alloc(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t total() const { return total_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0, used_ = 0, peak_ = 0;
};

enum RState { R_QUEUED, R_PREP, R_READY, R_RUNNING, R_DONE };

struct Req {
  uint64_t ticket = 0;
  ig_mdp_desc desc{};
  ig_params p{};
  const double* V0 = nullptr;
  Clock::time_point t_submit, t_launch, t_done;
  RState state = R_QUEUED;
  ig_status status = IG_OK;
  std::string err;
  DevRegion region;
  std::unique_ptr<Mdp> mdp;
  size_t off = 0, bytes = 0;
  bool has_chunk = false;
  int blocks = 0, units = 0;
  double* V = nullptr;  // device, in the request's chunk
  int32_t* pi = nullptr;
  hipEvent_t uploaded = nullptr;
  std::vector<double> Vh;
  std::vector<int32_t> pih;
  ig_stats st{};
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double* hV = nullptr;
  int32_t* hpi = nullptr;
  PCtl* hctl = nullptr;
  Req* req = nullptr;
};

}  // namespace

struct Server {
  ig_server_config cfg{};
  int num_cu = 0, units_cap = 0, units_used = 0;
  char* base = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  std::vector<std::thread> preps;
  std::thread sched;
  std::mutex mu;
  std::condition_variable cv_prep, cv_sched, cv_done;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::deque<Req*> queued;
  std::map<uint64_t, Req*> ready;
  uint64_t next_ticket = 1, next_alloc = 1;
  int n_prep = 0, n_running = 0, peak_running = 0;
  int64_t submitted = 0, completed = 0, failed = 0;
  bool stop = false;
};

namespace {

// status + message of the calling thread's last failure, for the request
void set_error(Req* r, ig_status e) {
  r->status = e;
  r->err = ig_last_error();
}

// Conversion and upload of one request (prep thread, outside the lock).
ig_status prepare(Server& S, Req* r, hipStream_t ps, PinnedStage* stage) {
  auto d = std::make_unique<Mdp>();
  d->device = S.cfg.device;
  d->region = &r->region;
  d->stream = ps;
  d->stage = stage;
  d->own_host_mirrors = false;
  if (ig_status e = create_in(&r->desc, d.get())) {
    (void)hipStreamSynchronize(ps);  // copies out of the staging may be in flight
    release_handle(d.get());
    return e;
  }
  const bool fp32 = r->p.mode == IG_MODE_MIXED;
  ig_status e = ensure_workspace(*d, r->p.restart, fp32);
  void *v = nullptr, *pv = nullptr;
  if (!e) e = region_alloc(*d, (size_t)d->n * 8, &v);
  if (!e) e = region_alloc(*d, (size_t)d->n * 4, &pv);
  if (!e) {
    r->V = (double*)v;
    r->pi = (int32_t*)pv;
    const hipError_t h = r->V0 ? hipMemcpyAsync(r->V, r->V0, (size_t)d->n * 8, hipMemcpyHostToDevice, ps)
                               : hipMemsetAsync(r->V, 0, (size_t)d->n * 8, ps);
    if (h != hipSuccess) e = fail(IG_E_DEVICE, "upload of V0 failed");
  }
  if (!e && hipEventCreateWithFlags(&r->uploaded, hipEventDisableTiming) != hipSuccess)
    e = fail(IG_E_DEVICE, "hipEventCreate failed");
  if (!e && hipEventRecord(r->uploaded, ps) != hipSuccess) e = fail(IG_E_DEVICE, "hipEventRecord failed");
  // the staging buffer (and the borrowed V0) is reused / returned only
  // after the uploads are done
  if (hipStreamSynchronize(ps) != hipSuccess && !e) e = fail(IG_E_DEVICE, "upload failed");
  d->stage = nullptr;
  if (!e && !persistent_fits(*d)) e = fail(IG_E_TOO_LARGE, "shape does not fit the persistent engine");
  if (e) {
    release_handle(d.get());
    return e;
  }
  int want = r->p.blocks;
  if (want <= 0) {
    want = (int)((d->nslices + S.cfg.block_slices - 1) / S.cfg.block_slices);
    want = std::min(want, 8 * S.units_cap);  // runs beside others when the shape allows
  }
  r->p.blocks = std::max(1, want);
  r->blocks = persistent_grid(*d, r->p.blocks);
  r->units = (r->blocks + 7) / 8;
  r->mdp = std::move(d);
  return IG_OK;
}

void prep_loop(Server* Sp, int omp_threads) {
  Server& S = *Sp;
  (void)hipSetDevice(S.cfg.device);
  omp_set_num_threads(std::max(1, omp_threads));
  hipStream_t ps = nullptr;
  (void)hipStreamCreateWithFlags(&ps, hipStreamNonBlocking);
  PinnedStage stage;  // this thread's staging, reused for every request
  std::unique_lock<std::mutex> lk(S.mu);
  for (;;) {
    S.cv_prep.wait(lk, [&] { return S.stop || !S.queued.empty(); });
    if (S.queued.empty()) break;  // stop requested and nothing left
    Req* r = S.queued.front();
    S.queued.pop_front();
    r->state = R_PREP;
    ++S.n_prep;
    lk.unlock();

    const bool fp32 = r->p.mode == IG_MODE_MIXED;
    size_t bytes = 0;
    ig_status e = device_footprint(&r->desc, r->p.restart, fp32, &bytes);
    if (!e) bytes += round_alloc((size_t)r->desc.n * 8) + round_alloc((size_t)r->desc.n * 4);
    if (!e && ps == nullptr) e = fail(IG_E_DEVICE, "stream creation failed");
    if (e) set_error(r, e);

    lk.lock();
    // allocations in submission order; wait while the arena is too full
    S.cv_prep.wait(lk, [&] {
      if (S.next_alloc != r->ticket) return false;
      if (r->status) return true;
      if (bytes > S.arena.total()) return true;
      return S.arena.alloc(bytes, &r->off);
    });
    if (!r->status && bytes > S.arena.total()) {
      fail(IG_E_TOO_LARGE, "device footprint of the request exceeds the server's hbm_budget");
      set_error(r, IG_E_TOO_LARGE);
    } else if (!r->status) {
      r->has_chunk = true;
      r->bytes = bytes;
    }
    ++S.next_alloc;
    S.cv_prep.notify_all();
    lk.unlock();

    if (!r->status) {
      r->region.base = S.base + r->off;
      r->region.size = bytes;
      r->region.used = 0;
      const Clock::time_point tp = Clock::now();
      if (ig_status e2 = prepare(S, r, ps, &stage)) set_error(r, e2);
      r->st.prep_ms = ms_between(tp, Clock::now());
    }

    lk.lock();
    --S.n_prep;
    if (r->status) {
      if (r->has_chunk) S.arena.release(r->off, r->bytes);
      r->has_chunk = false;
      if (r->uploaded) (void)hipEventDestroy(r->uploaded);
      r->uploaded = nullptr;
      r->t_done = Clock::now();
      r->state = R_DONE;
      ++S.completed;
      ++S.failed;
      S.cv_prep.notify_all();
      S.cv_done.notify_all();
      S.cv_sched.notify_all();
    } else {
      r->state = R_READY;
      S.ready[r->ticket] = r;
      S.cv_sched.notify_all();
    }
  }
  lk.unlock();
  if (ps) {
    (void)hipStreamSynchronize(ps);
    (void)hipStreamDestroy(ps);
  }
  stage.release();
}

// Enqueue request r on slot k (scheduler thread, outside the lock).
void launch_on(Server& S, Req* r, int k) {
  Slot& sl = S.slots[k];
  Mdp& d = *r->mdp;
  d.hpctl = sl.hctl;
  ig_status e = IG_OK;
  if (hipStreamWaitEvent(sl.s, r->uploaded, 0) != hipSuccess ||
      hipEventRecord(sl.ev0, sl.s) != hipSuccess)
    e = fail(IG_E_DEVICE, "stream ordering failed");
  if (!e) e = persistent_launch(d, r->V, r->pi, r->p, sl.s);
  if (!e && (hipMemcpyAsync(sl.hV, r->V, (size_t)d.n * 8, hipMemcpyDeviceToHost, sl.s) != hipSuccess ||
             hipMemcpyAsync(sl.hpi, r->pi, (size_t)d.n * 4, hipMemcpyDeviceToHost, sl.s) != hipSuccess))
    e = fail(IG_E_DEVICE, "result copy failed");
  if (e) set_error(r, e);
  // recorded in every case, so that retirement waits for whatever was enqueued
  (void)hipEventRecord(sl.ev1, sl.s);
}

// Completion of the request on slot k (scheduler thread, outside the lock).
void retire(Server& S, int k, hipError_t q) {
  Slot& sl = S.slots[k];
  Req* r = sl.req;
  Mdp& d = *r->mdp;
  if (q != hipSuccess && !r->status) {
    fail(IG_E_DEVICE, std::string("solve failed on the device: ") + hipGetErrorString(q));
    set_error(r, IG_E_DEVICE);
  }
  if (!r->status) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, sl.ev0, sl.ev1);
    const ig_status e = persistent_collect(d, r->st);
    if (e) set_error(r, e);
    r->st.time_ms = ms;
    r->st.cert_bound = r->st.res_inf / (1.0 - d.gamma);
    if (r->status == IG_OK || r->status == IG_E_NOCONV) {
      r->Vh.assign(sl.hV, sl.hV + d.n);
      r->pih.assign(sl.hpi, sl.hpi + d.n);
    }
  }
  r->t_done = Clock::now();
  r->st.latency_ms = ms_between(r->t_submit, r->t_done);
  r->st.queue_ms = ms_between(r->t_submit, r->t_launch);
  (void)hipEventDestroy(r->uploaded);
  r->uploaded = nullptr;
  d.hpctl = nullptr;
  release_handle(&d);
  r->mdp.reset();
}

void sched_loop(Server* Sp) {
  Server& S = *Sp;
  (void)hipSetDevice(S.cfg.device);
  const int ns = (int)S.slots.size();
  std::unique_lock<std::mutex> lk(S.mu);
  for (;;) {
    // retire finished solves
    bool progress = false;
    for (int k = 0; k < ns; ++k) {
      Req* r = S.slots[k].req;
      if (!r) continue;
      lk.unlock();
      const hipError_t q = hipEventQuery(S.slots[k].ev1);
      const bool done = q != hipErrorNotReady;
      if (done) retire(S, k, q);
      lk.lock();
      if (!done) continue;
      S.arena.release(r->off, r->bytes);
      r->has_chunk = false;
      S.units_used -= r->units;
      --S.n_running;
      S.slots[k].req = nullptr;
      r->state = R_DONE;
      ++S.completed;
      if (r->status && r->status != IG_E_NOCONV) ++S.failed;
      progress = true;
      S.cv_prep.notify_all();
      S.cv_done.notify_all();
    }
    // admit ready requests in submission order
    while (!S.ready.empty()) {
      int k = 0;
      while (k < ns && S.slots[k].req) ++k;
      if (k == ns) break;
      Req* r = S.ready.begin()->second;
      // within the budget; a solve wider than it runs alone (on up to every CU)
      const bool fits = S.units_used + r->units <= S.units_cap ||
                        (S.units_used == 0 && r->units <= std::max(1, S.num_cu / 8));
      if (!fits) break;
      S.ready.erase(S.ready.begin());
      S.slots[k].req = r;
      S.units_used += r->units;
      ++S.n_running;
      S.peak_running = std::max(S.peak_running, S.n_running);
      r->state = R_RUNNING;
      r->t_launch = Clock::now();
      lk.unlock();
      launch_on(S, r, k);
      lk.lock();
      progress = true;
    }
    if (S.stop && S.queued.empty() && S.n_prep == 0 && S.ready.empty() && S.n_running == 0) break;
    if (progress) continue;
    if (S.n_running == 0) {
      S.cv_sched.wait(lk, [&] {
        return !S.ready.empty() || (S.stop && S.queued.empty() && S.n_prep == 0);
      });
    } else {
      // running solves finish on the device: poll their events
      S.cv_sched.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

}  // namespace
}  // namespace ig

struct ig_server_s {
  ig::Server S;
};

extern "C" {

void ig_server_config_default(ig_server_config* cfg) {
  if (!cfg) return;
  cfg->device = 0;
  cfg->slots = 4;
  cfg->prep_threads = 4;
  cfg->block_slices = 16;
  cfg->max_states = (int64_t)1 << 19;
  cfg->hbm_budget = (size_t)32 << 30;
}

ig_status srv_create(const ig_server_config* cfg, ig_server_t* out) {
  using namespace ig;
  if (!cfg || !out) return fail(IG_E_INVALID, "NULL argument");
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 16) return fail(IG_E_INVALID, "slots must be in 1..16");
  if (cfg->prep_threads < 1 || cfg->prep_threads > 16)
    return fail(IG_E_INVALID, "prep_threads must be in 1..16");
  if (cfg->block_slices < 1) return fail(IG_E_INVALID, "block_slices must be >= 1");
  if (cfg->max_states < 1) return fail(IG_E_INVALID, "max_states must be >= 1");
  if (cfg->hbm_budget < ((size_t)1 << 20)) return fail(IG_E_INVALID, "hbm_budget below 1 MiB");
  auto h = std::make_unique<ig_server_s>();
  Server& S = h->S;
  S.cfg = *cfg;
  auto cleanup = [&S]() {
    for (Slot& sl : S.slots) {
      if (sl.s) (void)hipStreamDestroy(sl.s);
      if (sl.ev0) (void)hipEventDestroy(sl.ev0);
      if (sl.ev1) (void)hipEventDestroy(sl.ev1);
      if (sl.hV) (void)hipHostFree(sl.hV);
      if (sl.hpi) (void)hipHostFree(sl.hpi);
      if (sl.hctl) (void)hipHostFree(sl.hctl);
    }
    if (S.base) (void)hipFree(S.base);
  };
  if (hipSetDevice(cfg->device) != hipSuccess) return fail(IG_E_DEVICE, "hipSetDevice failed");
  if (hipDeviceGetAttribute(&S.num_cu, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess)
    return fail(IG_E_DEVICE, "device query failed");
  // one CU per XCD stays outside the budget: the conversion and fill
  // kernels of requests being prepared run there instead of waiting for a
  // running solve to end
  S.units_cap = std::max(1, S.num_cu / 8 - 1);
  if (hipMalloc((void**)&S.base, cfg->hbm_budget) != hipSuccess) {
    (void)hipGetLastError();
    return fail(IG_E_NOMEM, "hipMalloc of the serving arena failed");
  }
  S.arena.init(cfg->hbm_budget);
  S.slots.resize(cfg->slots);
  for (Slot& sl : S.slots) {
    const size_t nb = (size_t)cfg->max_states;
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&sl.ev0) != hipSuccess || hipEventCreate(&sl.ev1) != hipSuccess) {
      cleanup();
      return fail(IG_E_DEVICE, "stream or event creation failed");
    }
    if (hipHostMalloc((void**)&sl.hV, nb * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.hpi, nb * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.hctl, sizeof(PCtl), hipHostMallocDefault) != hipSuccess) {
      cleanup();
      return fail(IG_E_NOMEM, "hipHostMalloc of result buffers failed");
    }
  }
  const int hw = std::max(1, omp_get_max_threads());
  const int per = std::max(1, hw / cfg->prep_threads);
  try {
    for (int t = 0; t < cfg->prep_threads; ++t) S.preps.emplace_back(prep_loop, &S, per);
    S.sched = std::thread(sched_loop, &S);
  } catch (...) {
    {
      std::lock_guard<std::mutex> g(S.mu);
      S.stop = true;
    }
    S.cv_prep.notify_all();
    S.cv_sched.notify_all();
    for (auto& t : S.preps) t.join();
    if (S.sched.joinable()) S.sched.join();
    cleanup();
    return fail(IG_E_NOMEM, "thread creation failed");
  }
  *out = h.release();
  return IG_OK;
}

ig_status srv_submit(ig_server_t srv, const ig_mdp_desc* desc, const double* V0,
                     const ig_params* params, uint64_t* ticket) {
  using namespace ig;
  if (!srv || !desc || !params || !ticket) return fail(IG_E_INVALID, "NULL argument");
  Server& S = srv->S;
  if (desc->fmt != IG_FMT_CSR) return fail(IG_E_INVALID, "serving takes CSR MDPs");
  if (desc->inputs_on_device) return fail(IG_E_INVALID, "serving takes host arrays");
  if (desc->refine) return fail(IG_E_INVALID, "serving runs the persistent engine: refine must be 0");
  if (desc->n < 1 || desc->m < 1 || !desc->row_ptr || !desc->col || !desc->val || !desc->cost)
    return fail(IG_E_INVALID, "malformed MDP description");
  if (desc->n > S.cfg.max_states) return fail(IG_E_TOO_LARGE, "n exceeds the server's max_states");
  const ig_params& p = *params;
  if (!(p.alpha > 0.0 && p.alpha < 1.0)) return fail(IG_E_INVALID, "alpha must be in (0,1)");
  if (p.restart < 1) return fail(IG_E_INVALID, "restart must be >= 1");
  if (p.restart > kPersistMaxRestart) return fail(IG_E_TOO_LARGE, "serving takes restart <= 64");
  if (p.max_outer < 1 || p.max_inner < 1) return fail(IG_E_INVALID, "iteration caps must be >= 1");
  if (!(p.tol > 0.0)) return fail(IG_E_INVALID, "tol must be > 0");
  if (p.mode != IG_MODE_FP64 && p.mode != IG_MODE_MIXED) return fail(IG_E_INVALID, "bad mode");
  if (p.blocks < 0) return fail(IG_E_INVALID, "blocks must be >= 0");
  if (p.precond != 0) return fail(IG_E_INVALID, "serving runs the persistent engine: precond must be 0");
  auto r = std::make_unique<Req>();
  r->desc = *desc;
  r->p = p;
  r->V0 = V0;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(S.mu);
    if (S.stop) return fail(IG_E_INVALID, "server is shutting down");
    r->ticket = S.next_ticket++;
    *ticket = r->ticket;
    S.queued.push_back(r.get());
    S.reqs[r->ticket] = std::move(r);
    ++S.submitted;
  }
  S.cv_prep.notify_one();
  return IG_OK;
}

ig_status srv_poll(ig_server_t srv, uint64_t ticket, int32_t* done) {
  using namespace ig;
  if (!srv || !done) return fail(IG_E_INVALID, "NULL argument");
  Server& S = srv->S;
  std::lock_guard<std::mutex> g(S.mu);
  auto it = S.reqs.find(ticket);
  if (it == S.reqs.end()) return fail(IG_E_INVALID, "unknown ticket");
  *done = it->second->state == R_DONE ? 1 : 0;
  return IG_OK;
}

ig_status srv_result(ig_server_t srv, uint64_t ticket, double* V, int32_t* pi, ig_stats* stats) {
  using namespace ig;
  if (!srv) return fail(IG_E_INVALID, "NULL server");
  Server& S = srv->S;
  std::unique_ptr<Req> r;
  {
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(IG_E_INVALID, "unknown ticket");
    Req* q = it->second.get();
    S.cv_done.wait(lk, [&] { return q->state == R_DONE; });
    r = std::move(it->second);
    S.reqs.erase(it);
  }
  if (!r->Vh.empty()) {
    if (V) std::copy(r->Vh.begin(), r->Vh.end(), V);
    if (pi) std::copy(r->pih.begin(), r->pih.end(), pi);
  }
  if (stats) *stats = r->st;
  if (r->status) return fail(r->status, r->err);
  return IG_OK;
}

ig_status srv_get_info(ig_server_t srv, ig_server_info* info) {
  using namespace ig;
  if (!srv || !info) return fail(IG_E_INVALID, "NULL argument");
  Server& S = srv->S;
  std::lock_guard<std::mutex> g(S.mu);
  info->submitted = S.submitted;
  info->completed = S.completed;
  info->failed = S.failed;
  info->queued = (int32_t)S.queued.size();
  info->preparing = S.n_prep;
  info->ready = (int32_t)S.ready.size();
  info->running = S.n_running;
  info->peak_running = S.peak_running;
  info->xcd_units_cap = S.units_cap;
  info->arena_bytes = S.arena.total();
  info->arena_used = S.arena.used();
  info->arena_peak = S.arena.peak();
  return IG_OK;
}

void srv_destroy(ig_server_t srv) {
  using namespace ig;
  if (!srv) return;
  Server& S = srv->S;
  {
    std::lock_guard<std::mutex> g(S.mu);
    S.stop = true;
  }
  S.cv_prep.notify_all();
  S.cv_sched.notify_all();
  for (auto& t : S.preps) t.join();
  {
    std::lock_guard<std::mutex> g(S.mu);
  }
  S.cv_sched.notify_all();
  if (S.sched.joinable()) S.sched.join();
  for (Slot& sl : S.slots) {
    if (sl.s) {
      (void)hipStreamSynchronize(sl.s);
      (void)hipStreamDestroy(sl.s);
    }
    if (sl.ev0) (void)hipEventDestroy(sl.ev0);
    if (sl.ev1) (void)hipEventDestroy(sl.ev1);
    if (sl.hV) (void)hipHostFree(sl.hV);
    if (sl.hpi) (void)hipHostFree(sl.hpi);
    if (sl.hctl) (void)hipHostFree(sl.hctl);
  }
  if (S.base) (void)hipFree(S.base);
  delete srv;
}

}  // extern "C"
