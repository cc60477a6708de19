/*
 * igmres.h -- C-ABI of the MI355X (gfx950) inexact GMRES policy iteration
 * library, libigmres.so.
 *
 * The method is the one of Gargiani, Liao-McPherson, Zanelli and Lygeros,
 * "Inexact GMRES Policy Iteration for Large-Scale Markov Decision Processes"
 * (arXiv:2211.04299): finite discounted-cost MDPs {S, A, P, g, gamma}
 * (Section 2), the Bellman operators T^pi, T and GreedyPolicy (Section 2),
 * policy evaluation V^pi = (I - gamma P^pi)^{-1} g^pi, and Algorithm 2
 * (GMRES(W) policy iteration) with the inexact stopping rule of eq. 11 in the
 * infinity-norm.
 *
 * Conventions
 *   - States and actions are 0-based.  Row r = s*m + a of the transition data
 *     holds P(s, a, .); cost[s*m + a] = g(s, a).  Every state has all m
 *     actions unless ig_mdp_desc.admissible restricts them (action sets).
 *   - Vectors passed to the solver entry points (V, TV, pi) are DEVICE
 *     pointers owned by the caller (e.g. torch tensors); work is enqueued on
 *     the caller's HIP stream `stream` (hipStream_t passed as void*, NULL =
 *     the null stream).  Solver calls return after the solve has finished on
 *     that stream; bellman_apply is stream-ordered and returns immediately.
 *   - The MDP handle owns a device copy of P and g (re-laid-out for the
 *     GPU) plus all solver workspace; the caller may free its own arrays when
 *     mdp_create returns.  A handle is not re-entrant: calls on one handle
 *     must not overlap.  Distinct handles are independent.
 *   - Every entry point returns an ig_status; nothing throws across the ABI.
 *     On IG_E_INVALID outputs are untouched.  ig_last_error() returns a
 *     thread-local description of the last failure.
 */
#ifndef IGMRES_H
#define IGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IG_OK = 0,
  IG_E_INVALID = -1,   /* bad argument or malformed MDP; nothing was written */
  IG_E_NOMEM = -2,     /* device or host allocation failed                   */
  IG_E_DEVICE = -3,    /* a HIP call failed                                  */
  IG_E_NOCONV = -4,    /* iteration cap reached; last iterate and stats kept */
  IG_E_NUMERIC = -5,   /* NaN or Inf met in a Bellman pass                   */
  IG_E_TOO_LARGE = -6  /* request exceeds a capacity (restart > IG_MAX_RESTART,
                          serving budget)                                     */
} ig_status;

typedef enum { IG_FMT_CSR = 0, IG_FMT_DENSE = 1 } ig_format;
typedef enum { IG_FP64 = 0, IG_FP32 = 1, IG_BF16 = 2 } ig_dtype;
/* FP64: every vector and product in double.  MIXED: Krylov basis and the
 * P^pi products inside GMRES in single precision with float accumulation;
 * Bellman passes, residuals, dot products, the solution update and the
 * Hessenberg/Givens solve stay double. */
typedef enum { IG_MODE_FP64 = 0, IG_MODE_MIXED = 1 } ig_mode;

#define IG_MAX_RESTART 128

/* MDP description (problem setting, Section 2).
 *   fmt == IG_FMT_CSR:   row_ptr int64[n*m+1] (row_ptr[0] == 0, nondecreasing,
 *                        every row non-empty), col int32[nnz] in [0, n) with
 *                        no repeats inside a row, val[nnz] probabilities.
 *   fmt == IG_FMT_DENSE: val[n*m*n], val[(s*m + a)*n + s'] = P(s, a, s');
 *                        row_ptr and col are ignored.
 * val_type is the type of the val array as passed (IG_BF16 = raw bfloat16
 * bit patterns, uint16).  store is the type P is kept in on the device; it
 * may be narrower than val_type (conversion rounds to nearest even, through
 * fp32 for bf16) but not wider.
 * Validation (when `validate` != 0), over admissible pairs: 0 <= P <= 1;
 * no column repeated inside a row; every row sums to 1 within 1e-10 (FP64
 * input) or 1/64 (FP32 or BF16 input), and gamma * (largest stored row sum)
 * < 1.  Always checked: sizes, row_ptr (nondecreasing), column range and
 * non-empty rows of admissible pairs, finite costs of admissible pairs, a
 * nonempty A(s) for every state. */
typedef struct {
  int64_t n;
  int32_t m;
  double gamma;            /* discount factor, in (0, 1) */
  ig_format fmt;
  const int64_t* row_ptr;
  const int32_t* col;
  const void* val;
  ig_dtype val_type;
  const double* cost;      /* n*m */
  ig_dtype store;
  int32_t inputs_on_device;/* 1: row_ptr, col, val, cost, admissible are
                              device pointers                                 */
  int32_t validate;
  const uint8_t* admissible;/* NULL: every action is admissible in every
                              state.  Else n*m bytes, admissible[s*m + a] != 0
                              iff a is in A(s), the action set of s (Section
                              2); every state needs one.  Costs and CSR rows
                              of excluded pairs are ignored (the rows may be
                              empty); the Bellman operator, greedy policies
                              and every solver minimise over A(s) only, and
                              policies passed in must lie in A(s).            */
  int32_t refine;          /* 0: one stored copy of P, in `store`.  1
                              (residual-corrected evaluation; needs store ==
                              IG_BF16 and val_type FP64 or FP32): the P^pi
                              products inside GMRES (and the preconditioner
                              steps) read P^pi rounded to BF16, while every
                              Bellman pass, every true residual of the
                              stopping tests and restarts, the policy gather
                              and the value-iteration sweeps read an FP32
                              copy of P.  The outer iteration then converges
                              to the optimum of the FP32-stored MDP; an
                              explicit residual that misses the inexact rule
                              restarts the GMRES cycle from that residual
                              (iterative refinement of the BF16 solve).
                              Stream engine only (igmres_pi_solve with
                              engine 0 takes it; engine 2 and serving refuse
                              such a handle).                                 */
} ig_mdp_desc;

/* Solver parameters.  Algorithm 2's inputs are V0 (the V argument), alpha,
 * K (max_outer) and W (restart). */
typedef struct {
  double alpha;        /* forcing term, in (0, 1); Theorem 1 asks for
                          alpha < (1 - gamma) / (1 + gamma)                   */
  int32_t restart;     /* GMRES restart length W, 1..IG_MAX_RESTART          */
  int32_t max_outer;   /* K: outer (policy) iterations                        */
  int32_t max_inner;   /* cap on Arnoldi steps per policy evaluation          */
  double tol;          /* outer stop: ||T V - V||_inf <= tol (absolute)       */
  ig_mode mode;
  int32_t opi_sweeps;  /* opi_solve: applications of T^pi per outer step      */
  int32_t forcing;     /* igmres_pi_solve and ipi_vi_solve: 0: alpha_k =
                          alpha (Algorithm 2); 1: alpha_k = min(alpha,
                          sqrt(||T V_k - V_k||_inf)) (a forcing sequence
                          tending to zero, Theorem 1)                          */
  double eval_rtol;    /* pi_solve: evaluation residual target relative to
                          max |g(s,a)| (exact evaluation taken as GMRES to
                          this level or to stagnation)                        */
  int32_t engine;      /* igmres_pi_solve: 0 auto, 1 one kernel launch per
                          step (any size, dense or sparse), 2 a single
                          persistent launch for the whole solve (sparse,
                          up to 256*32 slices of 64 states, restart <= 64,
                          no preconditioner); auto picks 2 when all of
                          these hold and 1 otherwise.  Engine 2's grid
                          barriers wait
                          a bounded number of polls (environment variable
                          IG_SPIN_LIMIT overrides, for tests of the error
                          path); a wait that runs out ends the solve with
                          IG_E_DEVICE after every workgroup has left.       */
  int32_t blocks;      /* persistent engine: workgroups of the launch (0 =
                          from the shape); clamped so that a workgroup owns
                          1..32 slices.  The result depends on this count
                          (reduction order), never on other device work.      */
  int32_t precond;     /* inner GMRES right-preconditioned by the truncated
                          Neumann series M^{-1} = sum_{k<=precond} (gamma
                          P^pi)^k (the preconditioner Section 5 leaves to
                          future work); 0..16, 0 = none.  Stopping tests stay
                          on the true residual of J.  Stream engine only:
                          engine 0 then takes it, engine 2 is rejected.       */
  int32_t polish;      /* igmres_pi_solve: 1 = at an outer step k >= 1 whose
                          greedy policy equals the previous one in every
                          state, evaluate it to min(alpha_k ||Phi_k||_inf,
                          tol / 2) instead, so that the next outer step
                          stops unless the policy moves again (only a
                          smaller inexactness term: Theorem 1 still holds).
                          Both engines; 0 = off.                              */
} ig_params;

typedef struct {
  int32_t outer;          /* outer iterations performed (Bellman passes - 1)  */
  int32_t inner;          /* Arnoldi steps of the returned iterates (the stop
                             test of a column is known one step later; that
                             speculative step is not counted)                */
  int32_t restarts;
  int32_t bellman_passes;
  int32_t explicit_residuals; /* true-residual evaluations made for the
                                 stopping test                                */
  int32_t breakdowns;     /* Arnoldi steps with ||q||_2 == 0                   */
  int32_t stagnations;    /* inner loops ended by the stagnation guard        */
  int32_t converged;      /* 1 if the outer stopping test was met             */
  double res_inf;         /* ||T V - V||_inf at return                        */
  double cert_bound;      /* res_inf / (1 - gamma) >= ||V - V*||_inf          */
  double time_ms;         /* device time of the call (HIP events)             */
  double alg_bytes;       /* algorithmic HBM bytes the call had to move       */
  double latency_ms;      /* serving: submission to result ready (host clock);
                             0 for the direct entry points                    */
  double queue_ms;        /* serving: submission to launch                    */
  double prep_ms;         /* serving: host conversion + upload of the request */
} ig_stats;

typedef struct ig_mdp_s* ig_mdp_t;

/* Fill `p` with defaults for discount gamma: alpha = (1-gamma)/(2(1+gamma))
 * (midpoint of Theorem 1's range), restart 30, max_outer 1000,
 * max_inner 100000, tol 1e-8, FP64 mode, opi_sweeps 20, forcing 0,
 * eval_rtol 1e-13, engine 0, blocks 0, precond 0, polish 0. */
void ig_params_default(ig_params* p, double gamma);

/* Copy P and g to the device in the GPU layout (sliced ELL, 64 states per
 * slice, for CSR input; row-major for dense input) and allocate the solver
 * buffers the solvers share; the Krylov workspace is allocated on the first
 * solve and grown when a later call asks for a longer restart or the FP64
 * basis.  Problem setting: Section 2.  CSR entries are converted on the host
 * or, for device-resident inputs and from 2^22 entries on, by a device
 * kernel after one copy of the raw arrays (the environment variable
 * IG_CONVERT=host|device forces a route); both routes store the same bytes
 * and report the same first error.  On success *out owns all device memory
 * until mdp_destroy.  Errors: IG_E_INVALID (malformed description, see
 * ig_mdp_desc), IG_E_NOMEM, IG_E_DEVICE. */
ig_status mdp_create(const ig_mdp_desc* desc, void* stream, ig_mdp_t* out);

/* Release the handle and its device memory (synchronises the device).
 * NULL is ignored. */
void mdp_destroy(ig_mdp_t mdp);

/* Layout facts of a handle, for byte accounting. */
typedef struct {
  int64_t n;
  int32_t m;
  int32_t max_width;      /* widest ELL slice (CSR) or n (dense)               */
  int64_t nnz;            /* stored transition entries                         */
  int64_t stored_entries; /* nnz plus ELL padding                              */
  int64_t p_bytes;        /* device bytes of P (values + column indices)       */
  ig_dtype store;
  ig_format fmt;
  double gamma;
  int32_t persistent_ok;  /* igmres_pi_solve with engine 0 uses one persistent
                             launch per solve on this handle                */
  int32_t persistent_blocks;
  int32_t refine;         /* 1: BF16 products inside GMRES beside an FP32
                             copy for every other pass (store and p_bytes
                             then describe the FP32 copy; inner_p_bytes the
                             BF16 one)                                       */
  int64_t inner_p_bytes;  /* device bytes of the BF16 copy (0 without refine)*/
} ig_mdp_info;
ig_status mdp_get_info(ig_mdp_t mdp, ig_mdp_info* info);

/* One application of the Bellman operator T with greedy policy extraction
 * (Section 2: T V = min_pi {g^pi + gamma P^pi V}; GreedyPolicy(V)).
 *   V[n] in, TV[n] out (may be NULL), pi[n] out (int32, may be NULL),
 *   res_inf out: ||T V - V||_inf as one double (may be NULL).
 * All four are device pointers.  Ties go to the lowest action index.
 * Stream-ordered: returns once the work is enqueued. */
ig_status bellman_apply(ig_mdp_t mdp, const double* V, double* TV, int32_t* pi,
                        double* res_inf, void* stream);

/* Inexact policy evaluation by restarted GMRES(W) (the inner loop of
 * Algorithm 2, Section 3.1): starting from x0 = V, solve
 * (I - gamma P^pi) V = g^pi until
 *     ||g^pi - (I - gamma P^pi) V||_inf <= alpha * ||g^pi - (I - gamma P^pi) x0||_inf,
 * or params->max_inner Arnoldi steps, or a restart cycle that lowers the
 * residual 2-norm by less than a factor 1 - 1e-6 (stagnation).
 *   pi[n] int32 in (device), V[n] in/out (device).
 * Returns IG_E_NOCONV (with V = last iterate) if the rule was not met. */
ig_status policy_eval_gmres(ig_mdp_t mdp, const int32_t* pi, double* V, const ig_params* params,
                            ig_stats* stats, void* stream);

/* Algorithm 2 (GMRES(W) policy iteration): V[n] in V0 / out V_k, pi[n] out
 * GreedyPolicy(V_k), for the first k with ||T V_k - V_k||_inf <= params->tol.
 * IG_E_NOCONV after max_outer outer steps (V, pi = last iterate). */
ig_status igmres_pi_solve(ig_mdp_t mdp, double* V, int32_t* pi, const ig_params* params,
                          ig_stats* stats, void* stream);

/* Allocation-free Algorithm 2, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc).  The same
 * solve as igmres_pi_solve on the persistent engine (same kernel, same
 * workgroup count, bitwise the same V, pi and counts), except that its
 * device workspace -- Krylov basis, Arnoldi vector, cycle base, residual,
 * reduction partials, barrier arrival words and control block -- lives in a
 * static device array of IG_NOALLOC_SCRATCH_BYTES that every GPU holds from
 * the library's load until the process ends; the call allocates nothing.
 * Every call on one GPU shares that array: calls that overlap on a GPU (any
 * handle, any stream) race and must be serialised by the caller.  What must
 * start at zero (arrival words, control block) is cleared by each call.
 * The handle comes from mdp_create (which allocates); V (n doubles) and pi
 * (n int32) are device pointers, both required.  The call is host-synchronous
 * (not capturable into a HIP graph).
 * Errors: IG_E_TOO_LARGE when the workspace, about (restart+3) * n * 8 bytes
 * (FP64) or (restart+2) * n * 4 + 16 * n bytes (MIXED), exceeds the array, or
 * the shape does not fit the persistent engine (sparse, restart <= 64, no
 * refine); IG_E_INVALID for engine 1, a preconditioner, per-class timing
 * enabled on the handle (its events are created on demand), or a handle whose
 * device is not current; otherwise as igmres_pi_solve. */
#define IG_NOALLOC_SCRATCH_BYTES (32u << 20)
ig_status igmres_pi_solve_noalloc(ig_mdp_t mdp, double* V, int32_t* pi, const ig_params* params,
                                  ig_stats* stats, void* stream);

/* Policy iteration (Section 2.1): pi_0 = GreedyPolicy(V0); evaluation by
 * GMRES driven to ||residual||_inf <= eval_rtol * ||g^pi||_inf (or
 * stagnation); improvement keeps the incumbent action unless another is
 * better by more than 1e-12 * max(1, ||V||_inf); stops when the policy
 * repeats.  V out = V^pi of the final policy, pi out. */
ig_status pi_solve(ig_mdp_t mdp, double* V, int32_t* pi, const ig_params* params,
                   ig_stats* stats, void* stream);

/* Optimistic policy iteration (Section 2.1): per outer step a greedy policy
 * and params->opi_sweeps applications of T^pi (the first equals T V_k),
 * until ||T V - V||_inf <= tol. */
ig_status opi_solve(ig_mdp_t mdp, double* V, int32_t* pi, const ig_params* params,
                    ig_stats* stats, void* stream);

/* Inexact policy iteration with value iteration as the inner solver
 * (Algorithm 1 with IterativeLinearSolver = one application of T^pi_k):
 * sweeps until ||g^pi - J V_{k+1}||_inf <= alpha ||g^pi - J V_k||_inf. */
ig_status ipi_vi_solve(ig_mdp_t mdp, double* V, int32_t* pi, const ig_params* params,
                       ig_stats* stats, void* stream);

/* Measurement support (not part of the method): when bit k of `mask` is set,
 * every launch of kernel class k on this handle is bracketed by HIP events on
 * the launch stream.  Classes: 0 Bellman pass, 1 P^pi product (J-apply),
 * 2 Gram-Schmidt orthogonalisation + Givens update, 3 solution update,
 * 4 explicit residual, 5 value-iteration sweep, 6 other, 7 the single
 * persistent launch of a whole solve.  mask 0 disables. */
#define IG_PROFILE_CLASSES 8
ig_status ig_profile_enable(ig_mdp_t mdp, unsigned mask);
/* Sampling of the bracketed launches: with every = k only the first launch of
 * each enabled class and then one in every k are bracketed (default 1: all),
 * so that the events' own cost stays out of a timed run while every sampled
 * launch is still timed on its stream.  Restarts the per-class launch counts
 * (as do ig_profile_enable and a reset of ig_profile_read).  IG_E_INVALID for
 * every < 1. */
ig_status ig_profile_sample(ig_mdp_t mdp, int every);
/* Sum of event-timed milliseconds and counts of timed launches per class
 * since the last reset (synchronises on the recorded events).  ms and
 * launches have IG_PROFILE_CLASSES entries (host memory). */
ig_status ig_profile_read(ig_mdp_t mdp, double* ms, int64_t* launches, int reset);

/* ---- Continuous-batching serving ------------------------------------------
 * Many Algorithm 2 solves (igmres_pi_solve, persistent engine) in flight on
 * one GPU.  A server reserves one device arena of hbm_budget bytes, `slots`
 * HIP streams with pinned result buffers, `prep_threads` host threads that
 * convert requests to the device layout, and one scheduling thread.
 *   submit -> (prep thread) footprint; first-fit allocation in the arena, in
 *   submission order, waiting while it does not fit -> conversion and
 *   asynchronous upload -> (scheduler) launch of the request's persistent
 *   solve on a free slot once the workgroups of all running solves, spread
 *   over the 8 XCDs, stay co-resident -> completion -> results copied out,
 *   arena space and slot returned.
 * Admission and retirement happen while other solves run, so arriving
 * requests join the work on the device as slots and memory free up.  A
 * request's result depends only on the request (its workgroup count comes
 * from its shape, params->blocks and cfg.block_slices; every reduction is
 * per request): it is bitwise the same alone and in any mix.
 * Requests are sparse (IG_FMT_CSR) with host arrays; the server BORROWS
 * desc's arrays and V0 until srv_poll reports the ticket done (they are
 * read by the preparation, which runs after srv_submit returns).
 * The server's own calls are thread-safe. */
typedef struct ig_server_s* ig_server_t;
typedef struct {
  int32_t device;
  int32_t slots;          /* solves running at once, 1..16 (the device runs
                             kernels of at most GPU_MAX_HW_QUEUES streams at
                             once, 4 by default)                              */
  int32_t prep_threads;   /* host conversion/upload threads, 1..16            */
  int32_t block_slices;   /* params->blocks == 0: a solve gets
                             ceil(slices / block_slices) workgroups           */
  int64_t max_states;     /* largest n accepted (sizes pinned buffers)       */
  size_t hbm_budget;      /* device bytes reserved for resident requests     */
} ig_server_config;

typedef struct {
  int64_t submitted, completed, failed;
  int32_t queued, preparing, ready, running;
  int32_t peak_running;   /* most solves seen running at once                */
  int32_t xcd_units_cap;  /* co-residency budget (workgroups per XCD): one CU
                             per XCD less than the device has, so that the
                             preparation kernels of new requests find room;
                             a wider solve runs alone                         */
  size_t arena_bytes, arena_used, arena_peak;
} ig_server_info;

/* slots 4, prep_threads 4, block_slices 16, max_states 2^19,
 * hbm_budget 32 GiB, device 0. */
void ig_server_config_default(ig_server_config* cfg);

/* Reserve the arena and start the threads.  IG_E_INVALID (bad config),
 * IG_E_NOMEM (arena or pinned buffers), IG_E_DEVICE. */
ig_status srv_create(const ig_server_config* cfg, ig_server_t* out);

/* Queue one igmres_pi_solve request and return at once with its ticket.
 * desc: host CSR MDP (validated if desc->validate); V0: host n doubles or
 * NULL for V0 = 0; params: mode, restart <= 64, tol, ... as for
 * igmres_pi_solve (engine is ignored: the persistent engine is used).
 * IG_E_INVALID for a malformed request (checked here: shape, pointers,
 * params; the MDP data itself is checked by the preparation and reported by
 * srv_result), IG_E_TOO_LARGE if n > max_states or restart > 64. */
ig_status srv_submit(ig_server_t srv, const ig_mdp_desc* desc, const double* V0,
                     const ig_params* params, uint64_t* ticket);

/* *done = 1 once the ticket's result is ready (or failed), else 0.
 * IG_E_INVALID for an unknown ticket. */
ig_status srv_poll(ig_server_t srv, uint64_t ticket, int32_t* done);

/* Wait for the ticket, copy V (n doubles) and pi (n int32) to HOST memory
 * (either may be NULL), fill stats (may be NULL), and release the ticket.
 * Returns the request's status: IG_OK, IG_E_NOCONV (V, pi = last iterate),
 * IG_E_INVALID / IG_E_TOO_LARGE (found by the preparation, e.g. a footprint
 * above hbm_budget), IG_E_NUMERIC, IG_E_DEVICE. */
ig_status srv_result(ig_server_t srv, uint64_t ticket, double* V, int32_t* pi, ig_stats* stats);

ig_status srv_get_info(ig_server_t srv, ig_server_info* info);

/* Finish every submitted request, stop the threads and free everything
 * (results not collected are dropped).  NULL is ignored. */
void srv_destroy(ig_server_t srv);

/* Thread-local description of the last error (never NULL). */
const char* ig_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGMRES_H */
