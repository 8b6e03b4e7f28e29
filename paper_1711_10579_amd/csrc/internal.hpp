// Internal objects behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pf.h"
#include "analysis.hpp"
#include "device.hpp"

namespace pfi {

void set_error(const std::string& msg);
// PF_OK, or PF_E_DEVICE with the last HIP error named (and cleared)
pf_status launch_status(const char* where);

struct Server;
struct Batch;

struct PendingEvent {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
  bool pooled;  // events return to the pool once read (else a graph owns them)
  int nl;       // launches between the two events
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // pf_solve, pf_solve_batch and set-up work
  bool own_stream = false;
  pf_alloc_fn alloc = nullptr;
  pf_free_fn freef = nullptr;
  void* user = nullptr;
  int profile_mask = 0;
  // set (under launch_mu) while the serving loop launches on its own
  // streams: no kernel timing there
  bool prof_off = false;
  int mask() const { return prof_off ? 0 : profile_mask; }
  pf_kernel_stat stats[PF_K_COUNT] = {};
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> evpool;
  // while a graph is captured: timing events come from cap_pool (made
  // before the capture) and are listed here instead of in `pending`;
  // capture_bad records a failed record or an empty pool
  std::vector<PendingEvent>* capture = nullptr;
  std::vector<hipEvent_t> cap_pool;
  bool capture_bad = false;
  std::atomic<int> ncases{0};
  std::shared_ptr<Server> server;  // created by serve.cpp (complete type there)
  std::mutex launch_mu;  // serialises launches of the serving thread and callers
  std::mutex tune_mu;
  std::map<uint64_t, pf_schedule> tuned;  // topology hash -> autotuned schedule
  bool use_graphs = true;                 // replay reused batches' Newton steps from HIP graphs
  std::vector<Batch*> bcache;             // batches of recent pf_solve_batch calls, newest first

  void* dalloc(size_t bytes);
  void dfree(void* p);
  void prof_begin(int cls, hipEvent_t* a);
  void prof_end(int cls, hipEvent_t a, double flops, double bytes, int nl = 1);
  void prof_flush();  // after a stream synchronisation
};

// One case: device-resident Ybus, set-points, factor storage and state.
struct Case {
  Ctx* ctx = nullptr;
  int model = 0;
  int n = 0, nnz = 0;
  pfh::Analysis an;
  int nlev = 0, nbl = 0;
  int64_t ntg = 0;
  int ntt = 0;
  int M = 0;  // order of the dense block (2 nt)
  double analysis_ms = 0;
  pf_schedule sched;
  std::atomic<int> busy{0};

  // host copies of set-points (for pf_set_injections and the case info)
  std::vector<int8_t> type;
  // lanes per list (power of two) of each level, and the per-level
  // algorithmic flops / bytes of the refactorisation (profiling)
  std::vector<int> fac_g, bwd_g;
  int tailfwd_g = 1;
  std::vector<double> fac_flops, fac_bytes;

  // one device allocation, carved into the arrays below (topology, index
  // lists, set-points and state: resident from pf_create to pf_destroy)
  char* base = nullptr;
  size_t bytes = 0;  // resident bytes, plus the Krylov storage the case owns
  // working storage of a solve (factor values, the dense block with its
  // inverses, and their flags): the case's own, allocated by its first
  // pf_solve / pf_solve_batch and kept, or lent by the serving loop for one
  // request (wbase null between requests)
  char* wbase = nullptr;
  bool wown = false;
  size_t wbytes = 0;

  int *row_ptr = nullptr, *col = nullptr, *yrow = nullptr, *jmap = nullptr;
  double* y = nullptr;
  int8_t* dtype = nullptr;
  double *psp = nullptr, *qsp = nullptr, *vmag = nullptr, *vang = nullptr, *zip = nullptr;
  // CIM: generator Q of PV nodes (Newton state), per node the delta-load
  // links (draws into, receives from; -1 none) and the delta ZIP coefficients
  double* qg = nullptr;
  int* dlink = nullptr;
  double* zipd = nullptr;
  bool has_delta = false;
  int nheavy = 0;  // Ybus rows of more than kHeavyRow entries
  int *pos = nullptr, *node = nullptr;
  double *vm = nullptr, *va = nullptr, *v = nullptr, *ibus = nullptr, *F = nullptr;
  void *x = nullptr, *lu = nullptr, *dinv = nullptr, *tail = nullptr, *dinvu = nullptr;
  void* xs = nullptr;     // the backward solve's published copy of the solution (2 nu values)
  unsigned long long* pflags = nullptr;  // per 64-row block: panel-tile flags
  int *colptr = nullptr, *rowidx = nullptr, *upd_l = nullptr, *upd_u = nullptr, *col_order = nullptr;
  int64_t* uptr = nullptr;
  int *tail_tgt = nullptr, *tail_l = nullptr, *tail_u = nullptr;
  int64_t* tail_uptr = nullptr;
  int *lrow_ptr = nullptr, *lrow_blk = nullptr, *lrow_col = nullptr, *bwd_rows = nullptr;
  pfd::Red* red = nullptr;
  pfd::Inst* d_inst = nullptr;  // device descriptor
  pfd::Inst hinst;              // host copy of the descriptor
  Batch* single = nullptr;      // cached batch of this case alone

  // Newton-Krylov storage, created by the first Krylov solve of the case
  std::unique_ptr<pfh::KAnalysis> ka;
  std::vector<int> kmap_host;  // Ybus entry -> Krylov block position
  char* kbase = nullptr;
  size_t kbytes = 0;
  bool kown = false;  // false: lent by the serving loop for one request
  int km = 0;         // restart length the storage holds
  std::vector<int4> k_linfo, k_uinfo;  // per level position {row, first, end, 0}

  int64_t lu_count() const { return 4LL * (an.ns + 2 * an.nnzl); }
  int64_t tail_count() const { return (int64_t)an.ldt * (M + 1); }
  int nblk() const { return (M + 63) / 64; }
  int64_t dinvu_count() const { return (int64_t)nblk() * 64 * 64; }
};

// One kernel launch of the linear-solve sequence of a batch.
struct Launch {
  int kind;        // Launch kinds below
  int G;           // lanes per list
  int k0;          // dense panel step
  int nflag;       // dense step: flagged update items listed first
  int cls;         // pf_kernel_class for profiling
  int64_t off;     // first work item
  int count;       // work items
  double flops, bytes;
};
enum { L_FACTOR = 0, L_FWD, L_SCHUR, L_PANEL, L_BWD };

// A batch of cases: device instance table, flattened work lists and the
// launch sequence of one Newton step's LU solve.  Each item's arithmetic
// depends only on its own instance.
struct Batch {
  Ctx* ctx = nullptr;
  hipStream_t stream = nullptr;  // where the batch's work is launched (set by build: the context's)
  std::vector<Case*> cases;
  int nslots = 0;
  char* dmem = nullptr;  // instance pointer table, work items
  const pfd::Inst* const* d_insts = nullptr;
  int2* d_work = nullptr;
  // pinned host memory that the state gathers write into directly: the
  // instances' Newton states, then their Krylov states and inner counts
  pfd::Red* h_reds = nullptr;
  int* h_kstate = nullptr;
  int lu_steps = 0;  // Newton steps of the batch's last LU solve (queued ahead of the first read-back)
  // iterations (BiCGStab) or Arnoldi steps (GMRES) the batch's inner solves
  // took at each Newton step of its last Newton-Krylov solve (queued ahead
  // of the first read at the same step)
  std::vector<int> k_inner;
  int nk_step_index = 0;  // Newton step of the current solve
  std::vector<Launch> seq;
  int64_t zero_off = 0;  // zeroing chunks of the factor storage: work items [zero_off, +nzero)
  int nzero = 0;
  int max_n = 0, max_nnz = 0, max_nu = 0, max_heavy = 0;
  int64_t max_lu = 0, max_tail = 0;
  int trsv_single = 0;

  // Krylov launch lists (built on the first Krylov step of the batch): rows
  // by ILU level (factor and forward solve), by backward level, and the
  // block-Jacobi blocks, as (offset, count) ranges of d_kwork
  // the Newton step of the LU inner solve captured as a HIP graph, per
  // precision, with the convergence-test options baked into it
  bool allow_graph = false;
  bool graph_failed = false;
  struct Graph {
    hipGraphExec_t exec = nullptr;
    double tol = 0;
    int max_iter = -1;
    int prof_mask = 0;                // kernel classes timed inside the graph
    std::vector<PendingEvent> prof;  // their event pairs, owned by the graph
    void reset();
  } graphs[2];

  bool kbuilt = false;
  char* kmem = nullptr;
  int2* d_kwork = nullptr;
  std::vector<std::pair<int64_t, int>> k_lev, k_ulev;
  std::pair<int64_t, int> k_blocks{0, 0};
  int k_blocks_big = 0;  // the first k_blocks_big groups of k_blocks are above the small size
  int max_kchunks = 0;
  int k_min_nu = 0, k_max_nu = 0;
  bool k_wide = false;    // some instance has an ILU(0) level wider than one work-group pass
  bool k_narrow = false;  // some instance runs its ILU(0) in one work-group

  ~Batch();
  // launch plan and device table in memory the batch allocates (and pinned
  // host memory for the state gathers)
  bool build(Ctx* ctx, const std::vector<Case*>& cs);
  // the parts: the host launch plan with its work items; the device bytes of
  // the instance table and work items; their upload into `mem` (the batch
  // frees nothing it did not allocate)
  void plan(Ctx* ctx, const std::vector<Case*>& cs, std::vector<int2>* work);
  size_t plan_bytes(size_t nwork) const;
  bool place(char* mem, const std::vector<int2>& work);
  bool build_krylov();
};

// Kernel-class timing of the launches issued while it lives.
struct Prof {
  Ctx* ctx;
  int cls;
  hipEvent_t a;
  double flops, bytes;
  Prof(Ctx* c, int k, double f, double b) : ctx(c), cls(k), a(nullptr), flops(f), bytes(b) {
    ctx->prof_begin(cls, &a);
  }
  ~Prof() { ctx->prof_end(cls, a, flops, bytes); }
};

// Krylov storage of a case for restart length m (allocates on first use or
// when m grows); false on failure with the error set.
bool ensure_krylov(Case* c, int m);
void free_krylov(Case* c);
// Bytes of the Krylov storage for restart length m, and its set-up in the
// given memory (own: the case frees it; else lent, and dropped by
// detach_krylov), launched on stream s (no synchronisation).
size_t krylov_bytes(const Case* c, int m);
bool krylov_wide(const pfh::KAnalysis& ka);
bool attach_krylov(Case* c, int m, char* base, bool own, hipStream_t s);
void detach_krylov(Case* c);
// Working storage of a solve: its size, its set-up in the given memory on
// stream s (pointers in the device descriptor, flags cleared; no
// synchronisation), the case's own allocation when it has none, and the
// release of lent storage.
size_t work_bytes(const Case* c);
void attach_work(Case* c, char* base, bool own, hipStream_t s);
bool ensure_work(Case* c);
void detach_work(Case* c);
// Case creation under a schedule (api.cpp), the schedule's validation and
// the topology hash that keys the autotuner's choices.
pf_status create_case(Ctx* ctx, const pf_case_desc* d, const pf_schedule& sched, Case** out);
bool valid_schedule(const pf_schedule& s);
uint64_t topology_hash(const pf_case_desc* d);
// Validation of solve options (PF_E_INVALID with the error set).
pf_status check_opts(const pf_options* opt);
// The Newton step's linear solve by GMRES and the voltage update.
pf_status nk_step(Batch* b, const pf_options* opt);

// Launch plan of the dense block's block LU (dense_plan.cpp), one launch per
// 64-wide block step.  Step k of an instance with dense order M has a
// kb-wide diagonal block, nrt row tiles below it and nct column tiles right
// of it (the last holding the right-hand side column M).  Per step k0 over
// instances of orders Ms, `items` lists first the *nflag update items of the
// next block column, then the *npanel panel items (slot, g) of step k0 (g = 0
// the diagonal block, g = 1..nrt its row tiles, each also applying step k0's
// update to its row's tile of the next block column), then the other update
// items.  An update item (slot, j | i << 12 | flag << 24) applies step
// k0 - 64's update to tile (i, j) in 64-blocks; a flagged one then sets its
// row block's flag, which the panel items of rows i and k0 / 64 wait for.
constexpr int kDenseNB = 64;
void dense_grid(int M, int k, int* kb, int* nrt, int* nct);
void dense_plan_step(const std::vector<int>& Ms, int k0, std::vector<int2>* items, int* nflag, int* npanel);
// The backward solve's work list (one launch): nd dense items, then nrw
// work-group descriptors (offset of the first row item, rows | G << 16),
// then the row items (slot, row).  Per instance: dense order M, backward
// level pointers and rows of the sparse part, lanes per row of each level.
struct BwdInput {
  int M = 0;
  const std::vector<int>* lev_ptr = nullptr;
  const std::vector<int>* rows = nullptr;
  const std::vector<int>* g = nullptr;
};
void bwd_plan(const std::vector<BwdInput>& in, bool single, std::vector<int2>* items, int* nd, int* nrw);

// Run the Newton iteration of every case of a built batch to completion.
pf_status run_batch(Batch* b, const pf_options* opt, pf_result* results);
// Device address of pf_solve_noalloc's scratch array on `device` (current),
// looked up once per device (noalloc.hip).
pf_status scratch_init(int device);
pf_status solve_case(Case* c, const pf_options* opt, pf_result* res);

}  // namespace pfi

struct pf_ctx : pfi::Ctx {};
struct pf_case : pfi::Case {};
