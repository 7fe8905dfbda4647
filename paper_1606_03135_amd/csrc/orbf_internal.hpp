// Internal declarations of liborbf (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "orbf.h"

namespace orbf {

// Device status word: [0] = first error code (0 = none), [1] = the node or
// stencil it concerns.  Written with atomicCAS so the first error wins.
struct DevStatus {
  int code;
  int where;
};

__device__ __forceinline__ void report(DevStatus* st, int code, int where) {
  if (atomicCAS(&st->code, 0, code) == 0) atomicExch(&st->where, where);
}

// Squared distance ((dx*dx)+(dy*dy))+(dz*dz), every operation rounded on its
// own: stencil order and retention-ball membership are integer decisions
// taken on these values, and they must be reproducible bit for bit.
__device__ __forceinline__ double exact_sqdist(double ax, double ay, double az,
                                               double bx, double by, double bz,
                                               int d) {
#pragma clang fp contract(off)
  double dx = ax - bx;
  double s = dx * dx;
  double dy = ay - by;
  s = s + dy * dy;
  if (d == 3) {
    double dz = az - bz;
    s = s + dz * dz;
  }
  return s;
}

// Uniform bucket grid over the node set (replaces the kd-tree of Sec. 2).
struct GridParams {
  double lo[3];
  double s;      // cell side
  double inv_s;  // 1/s
  double diag2;  // squared bounding-box diagonal, with slack
  int nc[3];     // cells per axis
  int ncell;     // product of nc
};

// Scratch buffers owned by a context; grow-only.
struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// The squared distances of the stencils of the context's last kNN call
// (B_KNN_D2, one row of n per node in cell order: row s belongs to node
// perm[s]) and the arrays they belong to.  The covering reuses them when it
// is handed the same xyz and knn arrays.
struct D2Cache {
  const double* xyz = nullptr;
  const int32_t* knn = nullptr;
  int64_t N = 0;
  int d = 0, n = 0;
  const double* d2 = nullptr;  // row i: squared distances of node i's stencil
  bool matches(const double* x, const int32_t* k, int64_t N_, int d_,
               int n_) const {
    return d2 && x == xyz && k == knn && N_ == N && d_ == d && n_ == n;
  }
};

// Retained-row count p of every center of the last covering without the
// Lebesgue test, in center order, kept in the context's own scratch
// (B_P_CACHE).  The weights entry point uses it, when handed the same
// centers and owner arrays, to choose each stencil's pass width; a stale
// count can only choose a slower width, never change a result.
// One node set of a covering: its stencils, its owner array, and the global
// number of its node 0 when several sets share the per-node arrays
struct CoverSet {
  const int32_t* knn;
  int32_t* owner;
  int64_t base;
  int n;
};

// Per-node arrays of a covering over many node sets (global numbering),
// the sets' table on the device, and the shared level queues
struct MultiCover {
  uint64_t* ball = nullptr;
  int32_t* cnt = nullptr;
  int32_t* state = nullptr;
  int32_t* flag = nullptr;
  int32_t* setid = nullptr;
  int32_t* q0 = nullptr;
  int32_t* q1 = nullptr;
  int32_t* qc = nullptr;
  const CoverSet* tab = nullptr;
  int64_t total = 0;
  const void* key = nullptr;  // identifies the batch for the recorded depth
};

struct PCache {
  const int32_t* centers = nullptr;
  const int32_t* owner = nullptr;
  int64_t N = 0;
  int n = 0;
  const int32_t* p = nullptr;
  bool matches(const int32_t* c, const int32_t* o, int64_t N_, int n_) const {
    return p && c == centers && o == owner && N_ == N && n_ == n;
  }
};

}  // namespace orbf

struct orbf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t held = 0;
  std::string err;
  orbf::DevStatus* status = nullptr;  // device
  orbf::DevStatus* status_host = nullptr;  // pinned mirror
  orbf::Buffer buf[32];  // indexed by BufId
  int num_cus = 256;
  hipEvent_t ev[10] = {};
  bool timing = true;  // record phase events (off on batch/serving workers)
  bool owns_stream = false;  // created by the library (workers, slots)
  bool is_worker = false;
  // batched builds: worker contexts, fork/join events, graph of the last
  // repeated batch (key = its descriptors and worker count)
  int n_workers = 4;
  std::vector<orbf_ctx*> workers;
  std::vector<hipEvent_t> join_ev;
  hipEvent_t fork_ev = nullptr;
  hipStream_t cap_stream = nullptr;  // origin of graph capture
  hipGraphExec_t graph_exec = nullptr;
  std::vector<unsigned char> graph_key;
  int graph_seen = 0;
  float phase_ms[5] = {0, 0, 0, 0, 0};
  bool phase_valid[5] = {false, false, false, false, false};
  int64_t* host_counter = nullptr;  // pinned, covering round control
  double* host_scalars = nullptr;  // pinned, inner products of a solve
  // rounds over the covering's straggler list that each (xyz, knn, N)
  // needed in an eager call; a captured call replays that many
  std::vector<std::pair<const void*, int64_t>> cover_keys;
  std::vector<int> cover_rounds;
  // an eager covering that replayed its recorded count without a read-back
  // leaves the number of levels its finishing workgroup still ran in
  // cover_extra_host (pinned) once cover_ev has completed; a later call
  // adds it to the count of cover_pending_key
  hipEvent_t cover_ev = nullptr;
  int32_t* cover_extra_host = nullptr;
  bool cover_pending = false;
  std::pair<const void*, int64_t> cover_pending_key{nullptr, 0};
  // propagation-only levels the Lebesgue covering of each (knn, N) needed;
  // a repeated call launches that many before its first read-back
  std::vector<std::pair<const void*, int64_t>> leb_keys;
  std::vector<int64_t> leb_levels;
  // weights kernel schedules: rows of (K, pclass, orbf_schedule)
  std::vector<int> schedules;
  int ir_max_corrections = 8;  // FP32 + refinement: cap before FP64 fallback
  void* csr_scratch = nullptr;  // device address of the CSR no-alloc array
  // batched builds: pinned staging of the node-set table of the shared
  // covering levels (kept while a captured graph may read it)
  void* cover_tab_host = nullptr;
  size_t cover_tab_cap = 0;
  orbf::D2Cache d2_cache;
  orbf::PCache p_cache;
};

namespace orbf {

enum BufId {
  B_GRID_PARAMS = 0,
  B_PARTIAL,
  B_CELL_OF,
  B_CELL_RANK,
  B_CELL_START,
  B_SCAN_TMP,
  B_PERM,
  B_XS,
  B_BALL,
  B_INDEG,
  B_PRED_START,
  B_PRED_FILL,
  B_PRED,
  B_STATE,
  B_FLAGS,
  B_COUNTER,
  B_CENTER_POS,
  B_ROWPTR_TMP,
  B_W_TMP,
  B_MISC,
  B_MISC2,
  B_IR_FALLBACK,
  B_IR_COUNT,
  B_KNN_D2,
  B_CSR_RANK,
  B_CLASS,
  B_CLASS_N,
  B_P_CACHE,
  B_GERSH,
  B_KRYLOV,
  B_ILU,
  B_NUM,
};
static_assert(B_NUM <= 32, "orbf_ctx::buf holds 32 scratch buffers");

// ctx helpers (api.hip)
orbf_status fail(orbf_ctx* ctx, orbf_status code, const std::string& msg);
void* scratch(orbf_ctx* ctx, int id, size_t bytes, orbf_status* st);
void release_scratch(orbf_ctx* ctx);
orbf_status hip_check(orbf_ctx* ctx, hipError_t e, const char* what);

// exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total),
// int64 output; temp from scratch (scan.hip)
orbf_status exclusive_scan_i32_to_i64(orbf_ctx* ctx, const int32_t* in,
                                      int64_t n, int64_t* out);
size_t scan_tmp_elems(int64_t n);  // int64 temporaries of a scan of n
// the same scan with caller-provided temporaries (scan_tmp_elems(n) int64)
orbf_status exclusive_scan_i32_to_i64_tmp(orbf_ctx* ctx, const int32_t* in,
                                          int64_t n, int64_t* out,
                                          int64_t* tmp);

// phase launchers
orbf_status launch_knn(orbf_ctx* ctx, const double* xyz, int64_t N, int d,
                       int n, int32_t* knn, double* rho2);
orbf_status launch_cover(orbf_ctx* ctx, const double* xyz, const int32_t* knn,
                         const double* rho2, int64_t N, int d, int n,
                         double t2, const uint8_t* eligible, int32_t* centers,
                         int64_t* n_centers, int32_t* owner, int32_t* p);
// covering of many node sets with shared levels (batched builds): per set
// on its worker, ball masks and seeds; then all levels at once; then per
// set its center list
orbf_status cover_multi_prologue(orbf_ctx* w, const double* xyz,
                                 const int32_t* knn, const double* rho2,
                                 int64_t N, int d, int n, double t2,
                                 const uint8_t* eligible, int32_t* owner,
                                 const MultiCover& mc, int64_t base,
                                 int32_t set_index);
// clears the shared queue counters (before any set's seeds), on stream s
void cover_multi_reset(const MultiCover& mc, hipStream_t s);
orbf_status cover_multi_levels(orbf_ctx* ctx, const MultiCover& mc,
                               hipStream_t s);
orbf_status cover_multi_epilogue(orbf_ctx* w, const int32_t* knn, int64_t N,
                                 int n, const int32_t* owner,
                                 int32_t* centers, int64_t* n_centers,
                                 const MultiCover& mc, int64_t base);
orbf_status launch_weights(orbf_ctx* ctx, orbf_op op, int m, int l, int n,
                           double t2, const orbf_weights_args* a);
orbf_status launch_spmv(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                        const int32_t* col, const double* val,
                        const double* x, double* y);
size_t gershgorin_scratch_bytes();
orbf_status launch_gershgorin(orbf_ctx* ctx, int64_t N,
                              const int64_t* row_ptr, const int32_t* col,
                              const double* val, double* diag, double* radius,
                              double* summary);
size_t krylov_scratch_bytes(int64_t N, int restart);
// ILU(0) of the implicit step matrix (ilu.hip)
size_t ilu_scratch_bytes(int64_t N);
orbf_status launch_ilu0(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                        const int32_t* col, const double* val,
                        const uint8_t* row_kind, double alpha, double beta,
                        double* lu);
orbf_status launch_ilu_prepare(orbf_ctx* ctx, int64_t N,
                               const int64_t* row_ptr, const int32_t* col);
orbf_status launch_ilu_apply(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                             const int32_t* col, const double* lu,
                             const double* in, double* out);
void bdf_coefficients(int k, double a[4], double* b);
orbf_status launch_bdf_rhs(orbf_ctx* ctx, int64_t N, int k,
                           const double* const u[4], const double* f,
                           double dt, const uint8_t* row_kind,
                           const double* bvals, double* rhs);
orbf_status launch_solve_implicit(orbf_ctx* ctx, int64_t N,
                                  const int64_t* row_ptr, const int32_t* col,
                                  const double* val, const uint8_t* row_kind,
                                  double alpha, double beta, const double* b,
                                  double* x, double tol, int max_iter,
                                  int precond, const double* lu, int method,
                                  int restart, int* iters, double* relres);
orbf_status launch_csr(orbf_ctx* ctx, int64_t N, int n, const int32_t* knn,
                       const int32_t* owner, const double* W,
                       int64_t* row_ptr, int32_t* col, double* val);
// allocation-free CSR assembly (csr.hip): device address of the file-scope
// scratch array on ctx's device, looked up once per device at orbf_create
orbf_status csr_noalloc_setup(orbf_ctx* ctx);
orbf_status launch_csr_noalloc(orbf_ctx* ctx, int64_t N, int n,
                               const int32_t* knn, const int32_t* owner,
                               const double* W, int64_t* row_ptr,
                               int32_t* col, double* val);

// retention-ball masks, in-degrees and initial states (cover.hip); uses the
// kNN's recorded squared distances when they belong to xyz and knn
void launch_ball(orbf_ctx* ctx, const double* xyz, const int32_t* knn,
                 const double* rho2, int64_t N, int d, int n, double t2,
                 const uint8_t* eligible, uint64_t* ball, int32_t* indeg,
                 int32_t* state, int32_t s_open, int32_t s_inel);

// schedule of (K, pclass), ORBF_SCHED_DEFAULT if none (api.hip)
int schedule_for(const orbf_ctx* ctx, int K, int pclass);

// batched builds and serving (batch.hip)
orbf_status build_set(orbf_ctx* c, const orbf_set_desc& s);
orbf_status ensure_workers(orbf_ctx* ctx, int want);
void drop_graph(orbf_ctx* ctx);

}  // namespace orbf
