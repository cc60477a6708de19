// Host-side internals of libigmres: the MDP handle, its workspace and the
// kernel launchers (one .hip file per kernel family).
#pragma once

#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace ig {

// Error helper: sets the thread-local message and returns the status.
ig_status fail(ig_status s, const std::string& msg);
#define IG_HIP(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::ig::fail(IG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// kinds of the one-block finishing reduction
enum FinKind { FIN_BELLMAN = 0, FIN_RESID, FIN_VI, FIN_GATHER, FIN_IMPL, FIN_DOTS, FIN_GIVENS };

// kernel classes for the optional per-class event timing
enum KClass { KC_BELLMAN = 0, KC_JAPPLY, KC_GS, KC_UPDATE, KC_RESID, KC_VI, KC_OTHER, KC_PERSIST, KC_COUNT };

struct Workspace {
  int W = 0;           // restart capacity
  bool fp32 = false;   // basis type
  double* pa = nullptr;  // preconditioner ping-pong vectors (n doubles each;
  double* pb = nullptr;  // hold FP32 values in mixed mode)
  void* Q = nullptr;   // (W+1) x n basis, column j at Q + j*n
  void* wA = nullptr;  // Arnoldi vectors (ping-pong)
  void* wB = nullptr;
  double* Vb = nullptr;   // iterate at the start of the restart cycle
  double* r = nullptr;    // Phi_k / explicit residual
  double* t = nullptr;    // spare n-vector (VI ping-pong, evaluation)
  int32_t* pi = nullptr;  // internal policy buffer
};

// Bump allocation inside a caller-owned device region (serving): handles
// created in a region never call hipMalloc/hipFree and upload on `stream`.
struct DevRegion {
  char* base = nullptr;
  size_t size = 0, used = 0;
};

// Grow-only pinned host buffer that a serving thread reuses for the staging
// of every request it converts (pinned: the uploads are DMA copies).
// Buffers outgrown are kept until release() (freeing pinned memory may wait
// for the device).
struct PinnedStage {
  char* buf = nullptr;
  size_t cap = 0;
  std::vector<char*> retired;
  hipEvent_t ev[2] = {nullptr, nullptr};  // the bounce halves' last copies
  char* get(size_t need);  // nullptr if the allocation fails
  bool events();           // creates ev on first use; false on failure
  void release();
};

struct Mdp {
  int device = 0;
  DevRegion* region = nullptr;          // non-null: allocate from the region
  hipStream_t stream = nullptr;         // stream of the region-mode uploads
  PinnedStage* stage = nullptr;         // region mode: host staging to use
  bool own_host_mirrors = true;         // hst / hpctl allocated by the handle
  int64_t n = 0;
  int m = 0;
  double gamma = 0;
  ig_format fmt = IG_FMT_CSR;
  ig_dtype store = IG_FP64;
  int vb = 8;  // bytes per stored value

  // sliced ELL (CSR input)
  int64_t nslices = 0;
  int maxK = 0;
  int64_t nnz = 0, stored = 0, stored_pi = 0;
  int32_t* col = nullptr;
  void* val = nullptr;
  int64_t* off = nullptr;
  int32_t* width = nullptr;
  int32_t* mcnt = nullptr;  // action blocks stored per slice (1 + largest admissible action)
  int64_t* offp = nullptr;
  int32_t* pcol = nullptr;  // compact P^pi
  void* pval = nullptr;
  std::vector<int32_t> h_width;

  // dense input: P[s][a][s'] row-major
  void* P = nullptr;

  // residual-corrected evaluation: store/vb/val/pval/P above are the FP32
  // copy that the Bellman passes, residuals, gathers and sweeps read; the
  // P^pi products inside GMRES read these BF16 arrays (sparse: the compact
  // P^pi rounded after each Bellman pass or gather; dense: all of P)
  bool refine = false;
  ig_dtype in_store = IG_FP64;
  int in_vb = 8;
  void* in_pval = nullptr;
  void* in_P = nullptr;

  uint8_t* adm = nullptr;  // [m][n] admissibility (null: all actions admissible)
  double* cost = nullptr;  // [m][n] (transposed; 0 for excluded pairs)
  double* cpi = nullptr;   // g^pi

  DevStatus* st = nullptr;      // device
  DevStatus* hst = nullptr;     // pinned host mirror
  GivensState* gs = nullptr;    // device
  double* part = nullptr;       // reduction partials
  PCtl* pctl = nullptr;         // persistent-solve control block (device)
  PCtl* hpctl = nullptr;        // pinned host mirror
  StepSnap* hsnap = nullptr;    // pinned; written by each Arnoldi step's Givens kernel
  hipEvent_t ev_step = nullptr; // recorded after each Arnoldi step
  int num_cu = 0;
  int max_lds = 65536;          // LDS bytes a workgroup may use
  bool coop = false;            // cooperative launch supported
  Workspace ws;

  // lanes per state of the streaming kernels
  int G_bell = 1, G_jap = 1;
  int grid_stream = 1, grid_gs = 1;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // optional per-class kernel timing
  unsigned prof_mask = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[KC_COUNT];
  size_t prof_used[KC_COUNT] = {0};
  uint32_t prof_every = 1;                 // bracket one launch in prof_every per class
  uint64_t prof_seen[KC_COUNT] = {0};      // launches of each class since the counters restarted
  double cost_max = 0;  // max |g(s, a)|
};

// per-class timing around one launch (no-op unless the class is enabled)
struct ProfScope {
  Mdp& d;
  KClass k;
  hipStream_t s;
  hipEvent_t e1 = nullptr;
  ProfScope(Mdp& d_, KClass k_, hipStream_t s_);
  ~ProfScope();
};

// For the P^pi products inside GMRES: with refine set, the handle's storage
// fields name the BF16 copy for the lifetime of this object.
struct InnerView {
  Mdp& d;
  explicit InnerView(Mdp& d_) : d(d_) { flip(); }
  ~InnerView() { flip(); }
  void flip() {
    if (!d.refine) return;
    std::swap(d.store, d.in_store);
    std::swap(d.vb, d.in_vb);
    std::swap(d.pval, d.in_pval);
    std::swap(d.P, d.in_P);
  }
};

// FP32 -> BF16 (round to nearest even) of `count` values, for the BF16 copy
// of the refine mode
void launch_round_bf16(const float* src, void* dst, int64_t count, hipStream_t s);

ig_status ensure_workspace(Mdp& d, int W, bool fp32);
ig_status sync_status(Mdp& d, hipStream_t s);
Mdp* handle_of(ig_mdp_t h);
// solver parameters against the handle (IG_E_INVALID / IG_E_TOO_LARGE)
ig_status check_params(const Mdp& d, const ig_params* p, bool need_alpha);

// ---- sparse (sliced ELL) launchers --------------------------------------
// Bellman pass: TV (nullable), Phi = TV - V, pi, g^pi, compact P^pi and the
// reductions max|Phi|, ||Phi||^2, #nonfinite, #changes into the status.
// pi_old != nullptr: keep the incumbent unless another action is better by
// more than tie_abs.
void launch_bellman_sparse(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
                           const int32_t* pi_old, double tie_abs, bool compact, hipStream_t s);
// y = xs - gamma P^pi xs with xs = x * scale, scale = 1/(*eta) (eta == nullptr:
// scale 1).  fp32: vectors in float.
void launch_japply_sparse(Mdp& d, bool fp32, const void* x, const double* eta, void* y,
                          hipStream_t s);
// r = g^pi - (V - gamma P^pi V) in FP64, with max|r| and ||r||^2 into status.
void launch_residual_sparse(Mdp& d, const double* V, double* r, hipStream_t s);
// Vout = g^pi + gamma P^pi Vin (FP64), max|Vout - Vin| into status.aux.
void launch_vi_sweep_sparse(Mdp& d, const double* Vin, double* Vout, hipStream_t s,
                            bool finish = true);
// compact P^pi and g^pi for a given policy; #invalid entries into status.changes
void launch_gather_policy_sparse(Mdp& d, const int32_t* pi, hipStream_t s);

// ---- dense launchers (same contracts) ------------------------------------
void launch_bellman_dense(Mdp& d, const double* V, double* TV, double* Phi, int32_t* pi,
                          const int32_t* pi_old, double tie_abs, hipStream_t s);
void launch_japply_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* eta,
                         void* y, hipStream_t s);
void launch_residual_dense(Mdp& d, const int32_t* pi, const double* V, double* r, hipStream_t s);
void launch_vi_sweep_dense(Mdp& d, const int32_t* pi, const double* Vin, double* Vout,
                           hipStream_t s, bool finish = true);
void launch_gather_policy_dense(Mdp& d, const int32_t* pi, hipStream_t s);

// ---- persistent single-launch solver (sparse, up to kPMaxBlocks*kPMaxSpb slices)
// Longest restart cycle the persistent engine holds (its Givens state lives
// in LDS); longer cycles run on the stream engine.
constexpr int kPersistMaxRestart = 64;
// Returns IG_E_TOO_LARGE (without side effects) when the shape does not fit
// the persistent engine; the caller then uses the stream engine.
ig_status persistent_igmres(Mdp& d, double* V, int32_t* pi, const ig_params& p, ig_stats& st,
                            hipStream_t s);
bool persistent_fits(const Mdp& d);
int persistent_grid(const Mdp& d, int requested = 0);
// asynchronous form for serving: enqueue the solve on `s` (V already holds
// V0), then the copy of the control block into d.hpctl; collect after the
// stream has passed that point.
ig_status persistent_launch(Mdp& d, double* V, int32_t* pi, const ig_params& p, hipStream_t s);
ig_status persistent_collect(Mdp& d, ig_stats& st);
// device bytes mdp_create + ensure_workspace(restart, mode) would allocate
ig_status device_footprint(const ig_mdp_desc* desc, int restart, bool fp32, size_t* bytes);
ig_status create_in(const ig_mdp_desc* desc, Mdp* d);
ig_status region_alloc(Mdp& d, size_t bytes, void** p);
void release_handle(Mdp* d);
inline size_t round_alloc(size_t b) { return ((b < 8 ? 8 : b) + 255) & ~(size_t)255; }

// ---- Krylov (Gram-Schmidt, Givens, update) -------------------------------
// reduce the partials of the last nb-block finishing kernel into status /
// Givens state (cnt: number of columns for FIN_DOTS / FIN_GIVENS)
void launch_finalize(Mdp& d, FinKind kind, int nb, hipStream_t s, int cnt = 0,
                     bool with_impl = false, StepSnap* snap = nullptr);
// Q_0 = r / sqrt(*l2sq); Givens state reset with g_hat = beta e_1.
void launch_form_q0(Mdp& d, bool fp32, const double* r, const double* l2sq, hipStream_t s);
// Q_c = (w1 - sum_{j<c} h2_j Q_j) / eta and the per-block maxima of the
// implicit residual |Q z| of column c-1 (reduced by the next launch_dots with
// with_impl into status.res_impl)
void launch_form_qi(Mdp& d, bool fp32, int c, const void* w1, hipStream_t s);
// first pass (givens = false): gs->h = Q_{0..cnt-1}^T v;  second pass
// (givens = true): d = Q^T v, sigma = ||v||^2, then the Givens update of
// column cnt-1 (status.eta, status.rho, gs->z).
void launch_dots(Mdp& d, bool fp32, int cnt, const void* v, bool givens, bool with_impl,
                 hipStream_t s);
// w1 = y - sum_{j<cnt} gs->h_j Q_j
// device conversion of CSR entries into the sliced-ELL image (layout from
// the host; see convert.hip)
struct ConvArgs {
  int64_t n;
  int m;
  const int64_t* rp;
  const int32_t* col;
  const void* val;
  const uint8_t* adm_t;  // [m][n] or null
  const int64_t* off;
  const int32_t* width;
  const int32_t* mcnt;
  int32_t* scol;
  void* sval;
  int maxK;  // longest stored row (the largest slice width)
  int validate;
  double sum_tol;
  unsigned long long* err;  // 5 counters, zeroed by the caller
};
void launch_fill_sell(const ConvArgs& c, ig_dtype val_type, ig_dtype store, hipStream_t s);

// one Arnoldi step's orthogonalisation (after the J-apply): fused two-pass
// form for columns up to gs_fused_max, else the four-kernel sequence
// Horner step of the Neumann preconditioner: y = x*sx + gamma*(P^pi z)*sz,
// sx/sz = 1 / *ptr (null: 1)
void launch_pstep_sparse(Mdp& d, bool fp32, const void* x, const double* sx, const void* z,
                         const double* sz, void* y, hipStream_t s);
void launch_pstep_dense(Mdp& d, bool fp32, const int32_t* pi, const void* x, const double* sx,
                        const void* z, const double* sz, void* y, hipStream_t s);
void launch_vadd(Mdp& d, const double* a, const double* b, double* out, hipStream_t s);
ig_status ensure_precond(Mdp& d);
void launch_gs_step(Mdp& d, bool fp32, int c, const void* y, void* w1, hipStream_t s);
int gs_fused_max(bool fp32);
void launch_axpy(Mdp& d, bool fp32, int cnt, const void* y, void* w1, hipStream_t s);
// V = Vb + sum_{j<i} y_j Q_j with R y = g_hat (back substitution per block)
void launch_update(Mdp& d, bool fp32, int i, const double* Vb, double* V, hipStream_t s);

}  // namespace ig
