/*
 * pf.h - C ABI of the MI355X Newton power-flow library.
 *
 * The library solves the power-flow problem stated in Sec. II of
 * "ExaGridPF: A Parallel Power Flow Solver for Transmission and Unbalanced
 * Distribution Systems" (arXiv:1711.10579): given the nodal admittance matrix
 * (eq. 1-3, 11), the specified active and reactive power of every bus (or
 * phase), the voltage magnitude of voltage-controlled buses and, for
 * three-phase feeders, the ZIP load coefficients (eq. 12-15), find the
 * voltage magnitude and angle of every bus (phase).
 *
 * Two formulations share one outer Newton iteration (Sec. III):
 *   - PF_MODEL_POLAR_1PH: single-phase polar mismatch dP/dQ (eq. 4-10),
 *   - PF_MODEL_CIM_3PH  : three-phase current-injection mismatch dI with ZIP
 *                         loads (eq. 12-23).
 * and three inner linear solvers:
 *   - PF_SOLVER_LU      : sparse LU refactorisation on a fill-reducing
 *                         ordering with a dense trailing block (Sec. III-A),
 *   - PF_SOLVER_GMRES   : Newton-Krylov, restarted GMRES with an ILU(0) or
 *                         block-Jacobi preconditioner (Sec. III-B),
 *   - PF_SOLVER_BICGSTAB: Newton-Krylov with BiCGStab, the Krylov method the
 *                         paper tested (Sec. III-B), same preconditioners.
 * A Newton-Krylov solve may fall back to LU when an inner solve fails (the
 * direct method's robustness, Sec. III-A).
 *
 * Conventions: all sizes are int32; reals are IEEE double; complex values are
 * interleaved (re, im) pairs; powers and voltages are per unit; angles are in
 * radians; injections are positive for generation (eq. 12).  Every pointer
 * argument of a case description is a HOST pointer; the library copies what
 * it needs during the call, so the caller may free or reuse its arrays as soon
 * as the call returns.  Results are written into caller-owned host buffers.
 *
 * Errors: call-level failures return a non-zero pf_status and leave a message
 * for pf_last_error() (per thread).  Numerical outcomes of a solve (converged,
 * iteration limit, divergence, singular Jacobian, linear-solver failure) are
 * NOT errors: they are reported in pf_result.status, one per instance.
 */
#ifndef PF_H_
#define PF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_ctx pf_ctx;   /* one per device and stream                     */
typedef struct pf_case pf_case; /* one grid: device-resident Ybus, factor, state */

typedef enum {
  PF_OK = 0,
  PF_E_INVALID = 1, /* malformed input (see pf_create)                   */
  PF_E_NOMEM = 2,   /* device or host allocation failed                  */
  PF_E_DEVICE = 3,  /* HIP runtime error or no usable gfx950 device      */
  PF_E_BUSY = 4,    /* case is queued or running in the serving loop     */
  PF_E_NOTFOUND = 5 /* unknown ticket                                    */
} pf_status;

typedef enum {
  PF_CONVERGED = 0,  /* max-norm of the FP64 mismatch <= tol                   */
  PF_MAXITER = 1,    /* iteration limit reached                                */
  PF_DIVERGED = 2,   /* non-finite mismatch or growth beyond 1e6 x initial     */
  PF_SINGULAR = 3,   /* zero or non-finite pivot in the refactorisation        */
  PF_LINEAR_FAIL = 4,/* the Krylov solve did not reach its forcing tolerance */
  PF_PENDING = 5,    /* served request not finished yet                        */
  PF_FAILED = 6      /* served request could not run (device or allocation
                        failure); pf_result.error holds the pf_status         */
} pf_solve_status;

typedef enum { PF_MODEL_POLAR_1PH = 0, PF_MODEL_CIM_3PH = 1 } pf_model;
/* Bus (phase-node) types.  Polar: exactly one PF_SLACK, PV buses, PQ buses.
 * CIM: the source bus's phase-nodes are PF_SLACK (fixed voltage), load
 * phase-nodes PF_PQ, and phase-nodes with voltage-controlled distributed
 * generation PF_PV (generation Sec. II-B leaves out; see pf_case_desc). */
typedef enum { PF_PQ = 1, PF_PV = 2, PF_SLACK = 3 } pf_bus_type;
typedef enum { PF_SOLVER_LU = 0, PF_SOLVER_GMRES = 1, PF_SOLVER_BICGSTAB = 2 } pf_solver;
typedef enum { PF_PREC_FP64 = 0, PF_PREC_MIXED = 1 } pf_precision;
typedef enum { PF_PRECOND_ILU0 = 0, PF_PRECOND_BJACOBI = 1 } pf_precond;

/* Case description (all HOST pointers; copied by pf_create).
 *   n        buses (polar) or phase-nodes (CIM)
 *   row_ptr  [n+1], col_idx [nnz]: Ybus in CSR, column indices strictly
 *            increasing within a row, diagonal present, pattern structurally
 *            symmetric (eq. 3)
 *   y        [2*nnz] Ybus values, interleaved re/im (eq. 2-3, 11)
 *   bus_type [n] pf_bus_type.  CIM: PF_SLACK source phase-nodes, PF_PQ, and
 *            PF_PV for voltage-controlled distributed generation on that
 *            phase (the generation the paper leaves out, Sec. II-B): |V| held
 *            at v_mag, P_g given, Q_g solved for
 *   p_sp, q_sp [n] polar: specified injection P_g - P_l, Q_g - Q_l (eq. 8-9,
 *            12-13); CIM: generation P_g, Q_g (zero without DG; on PF_PV
 *            nodes q_sp is the starting Q_g of a flat start); may be NULL
 *            for CIM (taken as zero)
 *   v_mag, v_ang [n] polar: |V| set-point of PV and slack buses and slack
 *            angle; CIM: magnitude of PF_SLACK and PF_PV nodes and the
 *            nominal phase angle (0, -2pi/3, +2pi/3) of every node (flat
 *            start)
 *   zip      CIM [6*n] per node P_Z, P_I, P_P, Q_Z, Q_I, Q_P at |V| = 1
 *            (eq. 14-15, wye-connected); polar: NULL (constant-power loads)
 *   delta_to, zip_delta  CIM, optional (both NULL: none): delta-connected
 *            ZIP loads.  delta_to [n]: node k draws its delta load from its
 *            phase into node delta_to[k] (-1: no load); zip_delta [6*n]: that
 *            load's P_Z, P_I, P_P, Q_Z, Q_I, Q_P at the nominal line-to-line
 *            voltage sqrt(3) pu, so that S = s_Z (|V_k - V_t|/sqrt3)^2 +
 *            s_I |V_k - V_t|/sqrt3 + s_P.  The Ybus pattern must hold the
 *            entry (k, delta_to[k]) (an explicit zero will do) and a node may
 *            receive at most one delta load.
 */
typedef struct {
  int32_t model;
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* y;
  const int8_t* bus_type;
  const double* p_sp;
  const double* q_sp;
  const double* v_mag;
  const double* v_ang;
  const double* zip;
  const int32_t* delta_to;
  const double* zip_delta;
} pf_case_desc;

/* Solve options (pf_default_options fills the defaults shown).
 *   tol        1e-8   stop when the max-norm of the FP64 mismatch <= tol
 *                     (pu power for polar, pu current for CIM)
 *   max_iter   20     Newton iteration limit (40 recommended with MIXED)
 *   solver     LU     PF_SOLVER_LU, PF_SOLVER_GMRES or PF_SOLVER_BICGSTAB
 *   precision  FP64   PF_PREC_MIXED: Jacobian factor and inner solves in FP32,
 *                     mismatch, update and convergence test in FP64
 *   precond    ILU0   Krylov preconditioner
 *   gmres_m    30     GMRES restart length
 *   gmres_max_restarts 10  (BiCGStab: at most (1 + gmres_max_restarts) *
 *                     gmres_m / 2 iterations, as many products with J)
 *   eta_max    0.1    Krylov forcing term eta_k = min(eta_max, ||F_k||_inf)
 *   flat_start 1      0: start from the case's current voltage (warm start)
 *   nk_fallback 0     1: when a Krylov step fails (PF_LINEAR_FAIL), the
 *                     Newton iteration continues with LU from the voltage
 *                     it has reached (pf_result.lu_fallback = 1)
 */
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t solver;
  int32_t precision;
  int32_t precond;
  int32_t gmres_m;
  int32_t gmres_max_restarts;
  int32_t flat_start;
  int32_t nk_fallback;
  double eta_max;
} pf_options;

typedef struct {
  int32_t status;       /* pf_solve_status                                   */
  int32_t iters;        /* Newton steps taken (linear solves)                */
  int32_t linear_iters; /* total Krylov iterations (0 for LU)                */
  int32_t lu_fallback;  /* 1: a Krylov step failed and LU finished the solve */
  double mismatch_inf;  /* max-norm of the final FP64 mismatch               */
  double max_step;      /* max |dx| of the last Newton step (the paper's test)*/
  double device_ms;     /* device time of the solve (events around it);
                           served: host time from admission to retirement    */
  int32_t error;        /* PF_FAILED: the pf_status of the failure, else 0   */
  int32_t reserved;
  double wait_ms;       /* served: host time from pf_submit to admission     */
} pf_result;

/* Static information about a created case. */
typedef struct {
  int32_t n;            /* buses / phase-nodes                               */
  int32_t n_unknown;    /* nodes with unknowns (2 real unknowns each)        */
  int32_t n_sparse;     /* nodes eliminated as sparse columns                */
  int32_t n_dense;      /* nodes in the dense trailing block                 */
  int32_t levels;       /* refactorisation / forward-solve levels            */
  int32_t bwd_levels;   /* backward-solve levels                             */
  int64_t nnz_l_blocks; /* 2x2 blocks of L (equal to U) in the sparse part   */
  int64_t updates;      /* 2x2 block updates of the sparse refactorisation   */
  int64_t tail_updates; /* 2x2 block updates into the dense trailing block   */
  double flops_factor;  /* algorithmic flops of one refactorisation          */
  size_t device_bytes;  /* device memory the case holds now (resident, plus its
                           own working and Krylov storage once allocated)    */
  double analysis_ms;   /* host analysis time in pf_create                   */
  size_t resident_bytes;/* Ybus, index lists, set-points, state: from
                           pf_create to pf_destroy                           */
  size_t work_bytes;    /* working storage of an LU solve: factor values, the
                           dense block and its inverses                      */
  size_t krylov_bytes;  /* Krylov storage of a Newton-Krylov solve with the
                           default restart length (30)                       */
} pf_case_info;

/* Schedule of a case: choices of the host analysis and of the launch sequence
 * that change the work's order but not what is computed (the Sec. III-A
 * solve mapped onto the device).  pf_autotune chooses them by timing. */
typedef struct {
  double dense_switch; /* elimination switches to the dense trailing block once
                          every remaining node is adjacent to at least this
                          fraction of the others, 0 < x <= 1               */
  int32_t min_dense;   /* ... and at least this many nodes remain, >= 1      */
  int32_t lane_scale;  /* lanes per sparse update / solve list: 1, 2 or 4
                          times the default choice (at most one wave)       */
  int32_t trsv_mode;   /* dense backward solve: 0 automatic, 1 flag-
                          synchronised work-groups, 2 one work-group per
                          instance                                          */
  int32_t reserved;
} pf_schedule;

/* Tuning summary of pf_autotune. */
typedef struct {
  int32_t candidates;  /* schedules timed                                   */
  int32_t trials;      /* timed solves per schedule                         */
  double default_ms;   /* median device time of a solve, default schedule   */
  double best_ms;      /* median device time of a solve, chosen schedule    */
} pf_tune_report;

/* Device allocator callbacks (e.g. a framework's caching allocator). */
typedef void* (*pf_alloc_fn)(size_t bytes, void* user);
typedef void (*pf_free_fn)(void* ptr, void* user);

/* Fill *opt with the defaults listed above. */
void pf_default_options(pf_options* opt);
/* Fill *s with the default schedule: dense_switch 0.15, min_dense 32,
 * lane_scale 1, trsv_mode 0. */
void pf_default_schedule(pf_schedule* s);

/* Create a context on HIP device `device`, launching on `hip_stream` (a
 * hipStream_t; NULL: the context creates its own stream).  Device memory comes
 * from `alloc`/`free_` (both NULL: hipMalloc/hipFree).  Returns PF_E_DEVICE if
 * the device is not a gfx950 GPU or HIP fails.  A context is used from one
 * host thread at a time (the serving loop of pf_submit runs its own thread). */
pf_status pf_ctx_create(int32_t device, void* hip_stream, pf_alloc_fn alloc, pf_free_fn free_,
                        void* user, pf_ctx** out);
/* Destroy a context; all its cases must have been destroyed. */
void pf_ctx_destroy(pf_ctx* ctx);
/* Replay the LU Newton step of reused batches (repeated pf_solve of a case,
 * repeated pf_solve_batch over the same cases) from a captured HIP graph:
 * on (default) or off.  Results are identical either way; graphs are not used
 * while kernel timing (pf_profile_enable) is on. */
pf_status pf_ctx_use_graphs(pf_ctx* ctx, int32_t on);

/* Validate a case, run the host symbolic analysis (ordering, symbolic LU,
 * levels, maps) and upload everything to the device (eq. 1-3 input, Sec.
 * III-A analysis).  PF_E_INVALID if: n < 1 or nnz < n; CSR not sorted,
 * duplicated or out of range; a diagonal missing; pattern not structurally
 * symmetric; non-finite values; polar without exactly one PF_SLACK or with a
 * type outside {PQ, PV, SLACK}; CIM without a PF_SLACK node or without zip;
 * a PF_PV or PF_SLACK magnitude that is not positive; delta loads on a polar
 * case, only one of delta_to / zip_delta given, a delta_to outside
 * [-1, n) or equal to its node, a node receiving two delta loads, or a
 * delta load whose (k, delta_to[k]) entry is not in the Ybus pattern. */
pf_status pf_create(pf_ctx* ctx, const pf_case_desc* desc, pf_case** out);
/* The same under an explicit schedule (PF_E_INVALID if a field is out of
 * range).  pf_create uses the schedule pf_autotune stored in the context for
 * the topology of `desc` (Ybus pattern and node types), else the default. */
pf_status pf_create_scheduled(pf_ctx* ctx, const pf_case_desc* desc, const pf_schedule* sched,
                              pf_case** out);
/* The schedule a case was created with. */
pf_status pf_case_schedule(const pf_case* c, pf_schedule* out);
/* Autotuner: times `trials` solves (options `opt`, NULL: defaults) of the case
 * `desc` per candidate schedule in a coordinate search -- the fastest
 * dense_switch of {0.08, 0.12, 0.2, 0.3, 0.4, 0.5, 0.65, 0.8} when it beats
 * the default 0.15 by 2 %, then lane_scale over {1, 2, 4}, then trsv_mode over
 * {0, 1, 2}, keeping a candidate when its median device time beats the
 * current choice by 2 %.  Candidates whose solve does not converge are
 * skipped.  The chosen schedule goes to *best and is stored in the context
 * for this topology.  `rep` may be NULL.  Uses the context's stream; cases
 * are created and destroyed internally. */
pf_status pf_autotune(pf_ctx* ctx, const pf_case_desc* desc, const pf_options* opt, int32_t trials,
                      pf_schedule* best, pf_tune_report* rep);
/* Free a case's device memory.  PF_E_BUSY while it is queued or running. */
pf_status pf_destroy(pf_case* c);
pf_status pf_case_info_get(const pf_case* c, pf_case_info* out);
/* Device footprint of an LU solve of the case (the unknowns, eq. 10 / 19-20,
 * factored as in Sec. III-A): *bytes = its resident storage plus the working
 * storage a solve needs (pf_case_info.resident_bytes + work_bytes); a
 * Newton-Krylov solve needs pf_case_info.krylov_bytes more.  The working
 * storage is allocated by the case's first pf_solve / pf_solve_batch and
 * kept; a served request borrows it from the serving pool instead (see
 * pf_serve_config).  Host output; PF_E_INVALID on NULL. */
pf_status pf_case_footprint(const pf_case* c, size_t* bytes);

/* Replace the specified injections (same topology): p_sp/q_sp as in
 * pf_case_desc (NULL keeps the old values), zip [6n] for CIM (NULL keeps). */
pf_status pf_set_injections(pf_case* c, const double* p_sp, const double* q_sp, const double* zip);

/* Run the Newton iteration of Sec. II-A (polar) or II-B (CIM) to completion on
 * the context's stream and block until done. */
pf_status pf_solve(pf_case* c, const pf_options* opt, pf_result* res);

/* Solve `count` cases of one context together: every Newton phase runs as one
 * batched launch over all still-active instances; converged instances are
 * masked on the device.  results[i] belongs to cases[i].  Each instance's
 * arithmetic is identical to pf_solve of that case alone.  The launch plan of
 * a call is kept for the next calls over the same cases (a few plans per
 * context; destroying a case drops the plans that hold it). */
pf_status pf_solve_batch(pf_ctx* ctx, pf_case* const* cases, int32_t count, const pf_options* opt,
                         pf_result* results);

/* Serving loop (continuous batching): enqueue a solve of `c` under `opt`
 * (NULL: defaults) and return at once; *ticket identifies it.  Requests are
 * admitted first come, first served, when a slot is free and the serving
 * pool can lend the request's working storage (its case's own storage, when
 * it has some, is used instead); the request at the head of the queue waits
 * until running requests give enough back.  Every admitted request's Newton
 * steps run on the device beside the others' (spread over four streams, each
 * step replayed from the case's captured graph) and it retires as soon as
 * its own iteration ends; requests may differ in options.  Each result is
 * identical to pf_solve of the case alone.  A request whose storage exceeds
 * the whole budget finishes at once with PF_FAILED (error PF_E_NOMEM).  The
 * first submit of a case builds its launch plan (host work and one device
 * allocation, in the caller's thread).  PF_E_BUSY if `c` is already queued or
 * running. */
pf_status pf_submit(pf_ctx* ctx, pf_case* c, const pf_options* opt, uint64_t* ticket);
/* Non-blocking: *done = 1 and *out filled when the request has finished
 * (the ticket is then released), else *done = 0.  PF_E_NOTFOUND for an
 * unknown ticket. */
pf_status pf_poll(pf_ctx* ctx, uint64_t ticket, pf_result* out, int32_t* done);
/* Budget of the serving pool and the number of requests running at once
 * (max_slots 0: keep; default 32).  max_bytes > 0: the pool is one device
 * allocation of max_bytes made here, and the working storage lent to running
 * requests never exceeds it; 0 (default): no limit, the pool grows by chunks
 * of at least 256 MiB when a request does not fit and keeps them.  The pool
 * is freed with the context.  PF_E_BUSY when the budget would change while
 * requests are queued or running; PF_E_NOMEM if the allocation fails. */
pf_status pf_serve_config(pf_ctx* ctx, size_t max_bytes, int32_t max_slots);
/* Serving pool size and bytes lent now, requests queued and running (host
 * outputs). */
pf_status pf_serve_stats(pf_ctx* ctx, size_t* pool_bytes, size_t* lent_bytes, int32_t* queued, int32_t* running);

/* For callers that cannot allocate device memory (code under a stream capture
 * of their own, tight serving loops, harnesses that forbid allocation): the LU
 * Newton solve of pf_solve (options as there; solver must be PF_SOLVER_LU,
 * else PF_E_INVALID) with everything it needs beyond the case's resident
 * storage -- the launch plan, the Newton-state read-back and the working
 * storage (factor values, dense block) -- placed in one fixed array of 64 MiB
 * that the library holds on every GPU it runs on until the process ends.  It
 * makes no device or pinned-host allocation and creates no HIP object (no
 * graph, no event); the plan is built on the host heap.  A case needing more
 * than the array holds (about 10,000-15,000 buses of meshed grid; its needs
 * are pf_case_info.work_bytes plus the plan) is rejected with PF_E_INVALID,
 * the bytes it would need in *scratch_used (may be NULL).  Results are
 * identical to pf_solve's; res->device_ms is the host time of the call.  The
 * case's own working storage, if it has some, is left as it was.  Calls on
 * one GPU share the array: the library runs them one at a time (a per-device
 * lock), and overlapping calls from outside the library on one GPU would race. */
pf_status pf_solve_noalloc(pf_case* c, const pf_options* opt, pf_result* res, size_t* scratch_used);

/* Copy the case's current voltages (rectangular form) into host arrays of n
 * doubles each. */
pf_status pf_get_voltage(const pf_case* c, double* re, double* im);
/* Set the case's current voltages (used by warm starts, flat_start = 0). */
pf_status pf_set_voltage(pf_case* c, const double* re, const double* im);

/* Kernel timing.  pf_profile_enable(ctx, mask) selects kernel classes by bit
 * (1 << class; 0 disables, -1 selects every class).  Every launch of a selected class
 * is bracketed by HIP events on the launch stream (inside the captured graph
 * when a Newton step is replayed from one); pf_kernel_stats returns the
 * launch count, the summed device milliseconds and the summed algorithmic
 * flops and bytes of those launches since the last reset.  With
 * PF_PROFILE_SPANS in the mask, a run of consecutive launches of one class
 * in the refactorisation is bracketed as a whole instead (two events per
 * run; its time then includes the gaps between those launches). */
#define PF_PROFILE_SPANS (1 << 30)
typedef enum {
  PF_K_MISMATCH = 0,
  PF_K_JFILL = 1,
  PF_K_SPARSE_FACTOR = 2,
  PF_K_TAIL_SCHUR = 3,
  PF_K_DENSE_PANEL = 4,    /* dense block step: diagonal-block inverse, row tiles, trailing update */
  PF_K_DENSE_UPDATE = 5,   /* not launched: the dense trailing update runs in the block-step launch */
  PF_K_SPARSE_FWD = 6,
  PF_K_SPARSE_BWD = 7,     /* not launched: the sparse backward rows run in the backward-solve launch */
  PF_K_DENSE_TRSV = 8,     /* backward solve: the dense block's 64-row blocks, then the sparse rows, one launch */
  PF_K_UPDATE = 9,
  PF_K_KRYLOV = 10,        /* GMRES: begin, SpMV + dots, orthogonalisation, rotations, restarts */
  PF_K_PRECOND_SETUP = 11, /* ILU(0) factor by levels or block-Jacobi inverses            */
  PF_K_PRECOND_APPLY = 12, /* ILU(0) triangular solves or block-Jacobi products           */
  PF_K_COUNT = 13
} pf_kernel_class;
typedef struct {
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} pf_kernel_stat;
pf_status pf_profile_enable(pf_ctx* ctx, int32_t class_mask);
pf_status pf_kernel_stats(pf_ctx* ctx, int32_t kernel_class, pf_kernel_stat* out);
pf_status pf_profile_reset(pf_ctx* ctx);

/* Message of the last failed call on this thread (never NULL). */
const char* pf_last_error(void);
/* Library version string. */
const char* pf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H_ */
