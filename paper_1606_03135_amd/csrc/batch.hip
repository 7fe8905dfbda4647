// Many node sets per call, and a request engine with continuous admission.
//
// Both run the single-set path (stencils, covering, weights, boundary rows,
// CSR; Sec. 4.1) once per set on a worker context: a stream of its own with
// its own scratch.  A set's kernels read and write only that set's arrays
// and its worker's scratch, which every kernel writes before reading, so a
// result does not depend on what else runs beside it.
//
// Batched: sets are dealt to the workers largest estimated cost first, each
// to the currently least-loaded worker, between a fork event on the caller's
// stream and one join event per worker.  Identical batches are replayed from
// a HIP graph (captured from the caller's stream on the second occurrence).
//
// Serving: a fixed arena of device memory holds the outputs of admitted
// requests (first-fit free list with coalescing); waiting requests are
// admitted FIFO as slots and arena space free up, with bounded bypass of a
// head that does not fit yet.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "orbf_internal.hpp"

namespace orbf {

static int monomials(int d, int l) {
  long num = 1, den = 1;
  for (int i = 1; i <= d; ++i) {
    num *= (l + i);
    den *= i;
  }
  return (int)(num / den);
}

// The single-set path after the covering: weights, boundary rows, CSR.
static orbf_status build_after_cover(orbf_ctx* c, const orbf_set_desc& s) {
  orbf_weights_args a;
  memset(&a, 0, sizeof a);
  a.xyz = s.xyz;
  a.N = s.N;
  a.d = s.d;
  a.knn = s.knn;
  a.rho2 = s.rho2;
  a.centers = s.centers;
  a.n_centers = s.n_centers;
  a.owner = s.owner;
  a.eligible = s.eligible;
  a.tau = s.tau;
  a.prec = s.prec;
  a.W = s.W;
  a.lebesgue = s.lebesgue;
  a.ir_steps = s.ir_steps;
  orbf_status st =
      orbf_compute_weights(c, ORBF_OP_LAPLACIAN, s.m, s.l, s.n, s.delta, &a);
  if (st) return st;
  if (s.boundary && s.n_boundary > 0) {
    orbf_weights_args b = a;
    b.rows = s.boundary;
    b.n_rows = s.n_boundary;
    b.normals = s.normals;
    b.centers = nullptr;
    b.n_centers = nullptr;
    b.ir_steps = nullptr;
    b.tau = INFINITY;
    st = orbf_compute_weights(c, ORBF_OP_NEUMANN, s.m, s.l, s.n, 1.0, &b);
    if (st) return st;
  }
  return orbf_assemble_csr(c, s.N, s.n, s.knn, s.owner, s.W, s.row_ptr,
                           s.col, s.val);
}

// The whole single-set path on context c (asynchronous on c->stream).
orbf_status build_set(orbf_ctx* c, const orbf_set_desc& s) {
  orbf_status st =
      orbf_build_nodes_knn(c, s.xyz, s.N, s.d, s.n, s.knn, s.rho2);
  if (st) return st;
  if (isinf(s.tau)) {
    st = orbf_select_overlapped_stencils(c, s.xyz, s.knn, s.rho2, s.N, s.d,
                                         s.n, s.delta, s.eligible, s.centers,
                                         s.n_centers, s.owner, nullptr);
    if (st) return st;
  }
  return build_after_cover(c, s);
}

// Host-side checks of one set (the entry points check again).
static bool set_ok(const orbf_set_desc& s, std::string* why) {
  if (!s.xyz || !s.knn || !s.rho2 || !s.centers || !s.n_centers ||
      !s.owner || !s.W || !s.row_ptr || !s.col || !s.val) {
    *why = "NULL input or output pointer";
    return false;
  }
  if (s.d != 2 && s.d != 3) {
    *why = "d must be 2 or 3";
    return false;
  }
  if (s.N < 1 || s.n < 1 || s.n > s.N || s.n > 128) {
    *why = "need 1 <= n <= min(N, 128)";
    return false;
  }
  const int M = monomials(s.d, s.l);
  if (s.l < -1 || s.n < M || s.n + M > 160) {
    *why = "need C(l+d,d) <= n and n + C(l+d,d) <= 160";
    return false;
  }
  if (s.m < 3 || s.m % 2 == 0) {
    *why = "m must be odd and >= 3";
    return false;
  }
  if (!(s.delta >= 0.0 && s.delta <= 1.0) || !(s.tau >= 1.0)) {
    *why = "need 0 <= delta <= 1 and tau >= 1";
    return false;
  }
  if (s.boundary && s.n_boundary > 0 && !s.normals) {
    *why = "boundary rows need normals";
    return false;
  }
  return true;
}

// Relative cost of one set: stencils times one elimination, plus the
// per-node work of kNN and CSR.
static double set_cost(const orbf_set_desc& s) {
  const double K = s.n + monomials(s.d, s.l);
  const double keep = pow(1.0 - s.delta, s.d) * s.n;
  const double per_stencil = 2.0 / 3.0 * K * K * K;
  const double stencils = (double)s.N / (keep > 1.0 ? keep : 1.0);
  return stencils * per_stencil + (double)s.N * s.n * 200.0;
}

static orbf_status make_worker(orbf_ctx* parent, orbf_ctx** out) {
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_check(parent, e, "worker stream");
  const size_t share =
      parent->budget ? parent->budget / (size_t)parent->n_workers : 0;
  orbf_status st = orbf_create(parent->device, s, share, out);
  if (st) {
    hipStreamDestroy(s);
    return fail(parent, st, "worker context");
  }
  (*out)->owns_stream = true;
  (*out)->timing = false;
  (*out)->is_worker = true;
  return ORBF_OK;
}

orbf_status ensure_workers(orbf_ctx* ctx, int want) {
  while ((int)ctx->workers.size() < want) {
    orbf_ctx* w = nullptr;
    orbf_status st = make_worker(ctx, &w);
    if (st) return st;
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      orbf_destroy(w);
      return hip_check(ctx, e, "worker event");
    }
    ctx->workers.push_back(w);
    ctx->join_ev.push_back(ev);
  }
  if (!ctx->fork_ev) {
    hipError_t e =
        hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_check(ctx, e, "fork event");
  }
  return ORBF_OK;
}

// Enqueue a batch whose sets all have tau = INFINITY with the coverings'
// levels shared: (1) per worker, each set's kNN, ball masks and seeds,
// into per-node arrays numbered globally across the batch; (2) on `origin`,
// the covering levels of all sets at once, so the number of level launches
// is the deepest set's depth rather than the sum over sets; (3) per worker,
// each set's center list, weights, boundary rows and CSR.  Every step of a
// set reads and writes only that set's slice of the shared arrays, so its
// result is the same as alone.  Sets *no_room (with nothing enqueued) if
// the shared arrays do not fit the context's budget.
static orbf_status enqueue_batch_shared(
    orbf_ctx* ctx, const orbf_set_desc* sets, int nsets, int nw,
    hipStream_t origin, const std::vector<std::vector<int>>& plan,
    bool* no_room) {
  *no_room = false;
  // the shared arrays reuse this context's scratch (B_PERM among them), so
  // its caches of an earlier single-set call are no longer valid
  ctx->d2_cache = D2Cache();
  ctx->p_cache = PCache();
  std::vector<int64_t> base(nsets);
  int64_t total = 0;
  for (int i = 0; i < nsets; ++i) {
    base[i] = total;
    total += sets[i].N;
  }
  if (total >= INT32_MAX) {
    *no_room = true;
    return ORBF_OK;
  }
  orbf_status st = ORBF_OK;
  MultiCover mc;
  mc.ball = (uint64_t*)scratch(ctx, B_BALL, (size_t)total * 16, &st);
  mc.cnt = (int32_t*)scratch(ctx, B_INDEG, (size_t)(total + 1) * 4, &st);
  mc.state = (int32_t*)scratch(ctx, B_STATE, (size_t)(total + 1) * 4, &st);
  mc.flag = (int32_t*)scratch(ctx, B_FLAGS, (size_t)(total + 1) * 4, &st);
  mc.setid = (int32_t*)scratch(ctx, B_PERM, (size_t)(total + 1) * 4, &st);
  mc.q0 = (int32_t*)scratch(ctx, B_PRED_FILL, (size_t)(total + 1) * 4, &st);
  mc.q1 = (int32_t*)scratch(ctx, B_ROWPTR_TMP, (size_t)(total + 1) * 4, &st);
  mc.qc = (int32_t*)scratch(ctx, B_MISC2, 64, &st);
  auto* tab = (CoverSet*)scratch(ctx, B_CLASS,
                                 sizeof(CoverSet) * (size_t)nsets, &st);
  if (st == ORBF_EBUDGET) {
    *no_room = true;
    ctx->err.clear();
    return ORBF_OK;
  }
  if (st) return st;
  mc.tab = tab;
  mc.total = total;
  mc.key = sets[0].knn;
  const size_t tb = sizeof(CoverSet) * (size_t)nsets;
  if (ctx->cover_tab_cap < tb) {
    if (ctx->cover_tab_host) hipHostFree(ctx->cover_tab_host);
    ctx->cover_tab_host = nullptr;
    ctx->cover_tab_cap = 0;
    hipError_t e = hipHostMalloc(&ctx->cover_tab_host, tb,
                                 hipHostMallocDefault);
    if (e != hipSuccess) return hip_check(ctx, e, "batch set table");
    ctx->cover_tab_cap = tb;
  }
  auto* th = (CoverSet*)ctx->cover_tab_host;
  for (int i = 0; i < nsets; ++i)
    th[i] = CoverSet{sets[i].knn, sets[i].owner, base[i], sets[i].n};
  hipError_t e =
      hipMemcpyAsync(tab, th, tb, hipMemcpyHostToDevice, origin);
  if (e != hipSuccess) return hip_check(ctx, e, "batch set table copy");
  cover_multi_reset(mc, origin);

  auto fork = [&]() -> orbf_status {
    hipError_t e2 = hipEventRecord(ctx->fork_ev, origin);
    if (e2 != hipSuccess) return hip_check(ctx, e2, "batch fork");
    for (int w = 0; w < nw; ++w) {
      e2 = hipStreamWaitEvent(ctx->workers[w]->stream, ctx->fork_ev, 0);
      if (e2 != hipSuccess) return hip_check(ctx, e2, "batch fork wait");
    }
    return ORBF_OK;
  };
  auto join = [&]() -> orbf_status {
    for (int w = 0; w < nw; ++w) {
      hipError_t e2 = hipEventRecord(ctx->join_ev[w], ctx->workers[w]->stream);
      if (e2 != hipSuccess) return hip_check(ctx, e2, "batch join");
      e2 = hipStreamWaitEvent(origin, ctx->join_ev[w], 0);
      if (e2 != hipSuccess) return hip_check(ctx, e2, "batch join wait");
    }
    return ORBF_OK;
  };
  auto set_fail = [&](int i, orbf_ctx* wc, orbf_status code) {
    return fail(ctx, code, "set " + std::to_string(i) + ": " + wc->err);
  };
  if ((st = fork())) return st;
  for (int w = 0; w < nw; ++w) {
    orbf_ctx* wc = ctx->workers[w];
    for (int i : plan[w]) {
      const orbf_set_desc& s = sets[i];
      st = orbf_build_nodes_knn(wc, s.xyz, s.N, s.d, s.n, s.knn, s.rho2);
      if (st) return set_fail(i, wc, st);
      const double t = 1.0 - s.delta;
      st = cover_multi_prologue(wc, s.xyz, s.knn, s.rho2, s.N, s.d, s.n,
                                t * t, s.eligible, s.owner, mc, base[i], i);
      if (st) return set_fail(i, wc, st);
    }
  }
  if ((st = join())) return st;
  if ((st = cover_multi_levels(ctx, mc, origin))) return st;
  if ((st = fork())) return st;
  for (int w = 0; w < nw; ++w) {
    orbf_ctx* wc = ctx->workers[w];
    for (int i : plan[w]) {
      const orbf_set_desc& s = sets[i];
      st = cover_multi_epilogue(wc, s.knn, s.N, s.n, s.owner, s.centers,
                                s.n_centers, mc, base[i]);
      if (st) return set_fail(i, wc, st);
      st = build_after_cover(wc, s);
      if (st) return set_fail(i, wc, st);
    }
  }
  return join();
}

// Enqueue the batch on `origin`: fork, per-worker set lists, join.
static orbf_status enqueue_batch(orbf_ctx* ctx, const orbf_set_desc* sets,
                                 int nsets, int nw, hipStream_t origin,
                                 bool shared) {
  std::vector<int> order(nsets);
  std::vector<double> cost(nsets);
  for (int i = 0; i < nsets; ++i) {
    order[i] = i;
    cost[i] = set_cost(sets[i]);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(nw, 0.0);
  std::vector<std::vector<int>> plan(nw);
  for (int i : order) {
    int w = 0;
    for (int k = 1; k < nw; ++k)
      if (load[k] < load[w]) w = k;
    plan[w].push_back(i);
    load[w] += cost[i];
  }
  for (int w = 0; w < nw; ++w) {
    ctx->workers[w]->schedules = ctx->schedules;
    ctx->workers[w]->ir_max_corrections = ctx->ir_max_corrections;
  }
  if (shared) {
    bool no_room = false;
    const orbf_status st =
        enqueue_batch_shared(ctx, sets, nsets, nw, origin, plan, &no_room);
    // without room for the shared arrays, the sets go one by one
    if (st || !no_room) return st;
  }
  hipError_t e = hipEventRecord(ctx->fork_ev, origin);
  if (e != hipSuccess) return hip_check(ctx, e, "batch fork");
  for (int w = 0; w < nw; ++w) {
    orbf_ctx* wc = ctx->workers[w];
    e = hipStreamWaitEvent(wc->stream, ctx->fork_ev, 0);
    if (e != hipSuccess) return hip_check(ctx, e, "batch fork wait");
    for (int i : plan[w]) {
      orbf_status st = build_set(wc, sets[i]);
      if (st)
        return fail(ctx, st,
                    "set " + std::to_string(i) + ": " + wc->err);
    }
    e = hipEventRecord(ctx->join_ev[w], wc->stream);
    if (e != hipSuccess) return hip_check(ctx, e, "batch join");
    e = hipStreamWaitEvent(origin, ctx->join_ev[w], 0);
    if (e != hipSuccess) return hip_check(ctx, e, "batch join wait");
  }
  return ORBF_OK;
}

void drop_graph(orbf_ctx* ctx) {
  if (ctx->graph_exec) hipGraphExecDestroy(ctx->graph_exec);
  ctx->graph_exec = nullptr;
  ctx->graph_key.clear();
  ctx->graph_seen = 0;
}

}  // namespace orbf

using namespace orbf;

extern "C" {

orbf_status orbf_set_workers(orbf_ctx* ctx, int workers) {
  if (!ctx || workers < 1 || workers > 16) return ORBF_EINVAL;
  if (ctx->is_worker) return fail(ctx, ORBF_EINVAL, "worker context");
  ctx->n_workers = workers;
  drop_graph(ctx);
  return ORBF_OK;
}

orbf_status orbf_build_dm_batched(orbf_ctx* ctx, const orbf_set_desc* sets,
                                  int nsets) {
  if (!ctx) return ORBF_EINVAL;
  if (nsets < 0 || (nsets > 0 && !sets))
    return fail(ctx, ORBF_EINVAL, "bad set list");
  if (nsets == 0) return ORBF_OK;
  bool all_inf = true;
  for (int i = 0; i < nsets; ++i) {
    std::string why;
    if (!set_ok(sets[i], &why))
      return fail(ctx, ORBF_EINVAL, "set " + std::to_string(i) + ": " + why);
    all_inf = all_inf && isinf(sets[i].tau);
  }
  hipSetDevice(ctx->device);
  const int nw = std::min(ctx->n_workers, nsets);
  orbf_status st = ensure_workers(ctx, nw);
  if (st) return st;

  // graph replay of a repeated batch
  const size_t kbytes = sizeof(orbf_set_desc) * (size_t)nsets;
  const bool same = all_inf && ctx->graph_key.size() == kbytes + sizeof(int) &&
                    memcmp(ctx->graph_key.data(), sets, kbytes) == 0 &&
                    memcmp(ctx->graph_key.data() + kbytes, &nw,
                           sizeof(int)) == 0;
  if (same && ctx->graph_exec) {
    hipError_t e = hipGraphLaunch(ctx->graph_exec, ctx->stream);
    return hip_check(ctx, e, "batch graph launch");
  }
  if (same && ctx->graph_seen >= 1) {
    // second occurrence: scratch has its final size; capture on a stream of
    // the library's own (the caller's may be the legacy null stream), then
    // launch the graph on the caller's stream
    hipError_t e = hipSuccess;
    if (!ctx->cap_stream)
      e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_check(ctx, e, "capture stream");
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(ctx->cap_stream,
                              hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_check(ctx, e, "batch capture");
    st = enqueue_batch(ctx, sets, nsets, nw, ctx->cap_stream, all_inf);
    hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
    if (st || e2 != hipSuccess) {
      if (g) hipGraphDestroy(g);
      drop_graph(ctx);
      return st ? st : hip_check(ctx, e2, "batch capture end");
    }
    e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      ctx->graph_exec = nullptr;
      drop_graph(ctx);
      return hip_check(ctx, e, "batch graph instantiate");
    }
    e = hipGraphLaunch(ctx->graph_exec, ctx->stream);
    return hip_check(ctx, e, "batch graph launch");
  }
  drop_graph(ctx);
  if (all_inf) {
    ctx->graph_key.resize(kbytes + sizeof(int));
    memcpy(ctx->graph_key.data(), sets, kbytes);
    memcpy(ctx->graph_key.data() + kbytes, &nw, sizeof(int));
    ctx->graph_seen = 1;
  }
  return enqueue_batch(ctx, sets, nsets, nw, ctx->stream, all_inf);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving
// ---------------------------------------------------------------------------
namespace {

// First-fit allocator over [0, cap) with coalescing of free neighbours.
class Arena {
 public:
  void init(size_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t cap() const { return cap_; }

 private:
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct Layout {  // byte offsets of a request's outputs inside its block
  size_t knn, rho2, centers, n_centers, owner, W, lam, ir, row_ptr, col, val,
      total;
};

Layout layout(int64_t N, int n, orbf_prec prec) {
  Layout L;
  const size_t Nn = (size_t)N, nn = (size_t)N * n;
  size_t o = 0;
  L.knn = o; o += up(nn * 4);
  L.rho2 = o; o += up(Nn * 8);
  L.centers = o; o += up(Nn * 4);
  L.n_centers = o; o += up(8);
  L.owner = o; o += up(Nn * 4);
  L.W = o; o += up(nn * 8);
  L.lam = o; o += up(Nn * 8);
  L.ir = o; o += (prec == ORBF_PREC_FP32_IR) ? up(Nn * 4) : 0;
  L.row_ptr = o; o += up((Nn + 1) * 8);
  L.col = o; o += up(nn * 4);
  L.val = o; o += up(nn * 8);
  L.total = o;
  return L;
}

enum ReqState { WAITING = 0, RUNNING = 1, DONE = 2 };

struct Req {
  orbf_request r;
  ReqState state = WAITING;
  size_t off = 0, bytes = 0;
  int slot = -1;
  int bypassed = 0;
  int status = ORBF_OK;
  int64_t n_centers = 0;
  double t_admit = 0.0, t_done = 0.0;
};

struct Slot {
  orbf_ctx* ctx = nullptr;
  hipEvent_t done = nullptr;
  int64_t* nc_host = nullptr;  // pinned: number of stencils of the request
  uint64_t req = 0;
  bool busy = false;
};

double now_s() {
  return std::chrono::duration<double>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct orbf_server {
  int device = 0;
  char* base = nullptr;
  Arena arena;
  size_t slot_budget = 0;
  std::vector<Slot> slots;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<uint64_t> finished;
  uint64_t next = 1;
  int max_bypass = 8;
  std::string err;
};

namespace {

orbf_status sfail(orbf_server* s, orbf_status c, const std::string& m) {
  s->err = m;
  return c;
}

orbf_set_desc desc_of(orbf_server* s, const Req& q) {
  const Layout L = layout(q.r.N, q.r.n, q.r.prec);
  char* b = s->base + q.off;
  orbf_set_desc d;
  memset(&d, 0, sizeof d);
  d.xyz = q.r.xyz;
  d.N = q.r.N;
  d.d = q.r.d;
  d.n = q.r.n;
  d.m = q.r.m;
  d.l = q.r.l;
  d.delta = q.r.delta;
  d.tau = q.r.tau;
  d.prec = q.r.prec;
  d.knn = (int32_t*)(b + L.knn);
  d.rho2 = (double*)(b + L.rho2);
  d.centers = (int32_t*)(b + L.centers);
  d.n_centers = (int64_t*)(b + L.n_centers);
  d.owner = (int32_t*)(b + L.owner);
  d.W = (double*)(b + L.W);
  d.lebesgue = (double*)(b + L.lam);
  d.ir_steps =
      (q.r.prec == ORBF_PREC_FP32_IR) ? (int32_t*)(b + L.ir) : nullptr;
  d.row_ptr = (int64_t*)(b + L.row_ptr);
  d.col = (int32_t*)(b + L.col);
  d.val = (double*)(b + L.val);
  return d;
}

void start(orbf_server* s, int si, uint64_t id) {
  Req& q = s->reqs[id];
  Slot& sl = s->slots[si];
  q.state = RUNNING;
  q.slot = si;
  q.t_admit = now_s();
  // the slot's grow-only scratch holds the largest buffers of earlier
  // requests; start from nothing if keeping them could pass the cap
  const size_t need =
      orbf_workspace_size(q.r.N, q.r.d, q.r.n, q.r.l, q.r.prec);
  if (sl.ctx->held + need > s->slot_budget) release_scratch(sl.ctx);
  const orbf_set_desc d = desc_of(s, q);
  // the coordinates may still be in flight on the producer's stream
  if (q.r.ready)
    hipStreamWaitEvent(sl.ctx->stream, (hipEvent_t)q.r.ready, 0);
  orbf_status st = build_set(sl.ctx, d);
  if (st) {
    // failed on the host before its kernels were enqueued: the device word
    // was never written, so report no stencils
    q.status = st;
    *sl.nc_host = 0;
  } else {
    // the stencil count goes to the slot's pinned word when the build is
    // done
    hipMemcpyAsync(sl.nc_host, d.n_centers, sizeof(int64_t),
                   hipMemcpyDeviceToHost, sl.ctx->stream);
  }
  hipEventRecord(sl.done, sl.ctx->stream);
  sl.busy = true;
  sl.req = id;
}

void retire(orbf_server* s) {
  for (auto& sl : s->slots) {
    if (!sl.busy) continue;
    if (hipEventQuery(sl.done) != hipSuccess) continue;
    Req& q = s->reqs[sl.req];
    q.t_done = now_s();
    q.n_centers = *sl.nc_host;
    const orbf_status dev = orbf_sync(sl.ctx);
    if (q.status == ORBF_OK && dev != ORBF_OK) q.status = dev;
    q.state = DONE;
    sl.busy = false;
    s->finished.push_back(sl.req);
  }
}

void admit(orbf_server* s) {
  for (;;) {
    int free_slot = -1;
    for (size_t i = 0; i < s->slots.size(); ++i)
      if (!s->slots[i].busy) {
        free_slot = (int)i;
        break;
      }
    if (free_slot < 0 || s->queue.empty()) return;
    bool started = false;
    size_t pos = 0;
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it, ++pos) {
      Req& q = s->reqs[*it];
      size_t off;
      if (!s->arena.alloc(q.bytes, &off)) {
        // the head may be passed only a bounded number of times
        if (pos == 0 && q.bypassed >= s->max_bypass) return;
        continue;
      }
      q.off = off;
      const uint64_t id = *it;
      if (pos > 0) s->reqs[s->queue.front()].bypassed++;
      s->queue.erase(it);
      start(s, free_slot, id);
      started = true;
      break;
    }
    if (!started) return;
  }
}

}  // namespace

extern "C" {

double orbf_server_now(void) { return now_s(); }

size_t orbf_request_bytes(int64_t N, int d, int n, orbf_prec prec) {
  (void)d;
  if (N < 1 || n < 1) return 0;
  return layout(N, n, prec).total;
}

orbf_status orbf_server_create(int device, int slots, size_t arena_bytes,
                               size_t slot_scratch_bytes, orbf_server** out) {
  if (!out || slots < 1 || slots > 16 || arena_bytes < kAlign ||
      slot_scratch_bytes == 0)
    return ORBF_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return ORBF_EHIP;
  orbf_server* s = new (std::nothrow) orbf_server();
  if (!s) return ORBF_ENOMEM;
  s->device = device;
  const size_t arena = arena_bytes / kAlign * kAlign;
  s->slot_budget = slot_scratch_bytes;
  if (hipMalloc((void**)&s->base, arena) != hipSuccess) {
    delete s;
    return ORBF_ENOMEM;
  }
  s->arena.init(arena);
  s->slots.resize(slots);
  for (auto& sl : s->slots) {
    hipStream_t st = nullptr;
    orbf_status e = ORBF_OK;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      e = ORBF_EHIP;
    if (!e) e = orbf_create(device, st, s->slot_budget, &sl.ctx);
    if (!e) {
      sl.ctx->owns_stream = true;
      sl.ctx->timing = false;
      if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) !=
              hipSuccess ||
          hipHostMalloc((void**)&sl.nc_host, sizeof(int64_t),
                        hipHostMallocDefault) != hipSuccess)
        e = ORBF_EHIP;
    } else if (st) {
      hipStreamDestroy(st);
    }
    if (e) {
      orbf_server_destroy(s);
      return e;
    }
  }
  *out = s;
  return ORBF_OK;
}

void orbf_server_destroy(orbf_server* s) {
  if (!s) return;
  hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    if (sl.ctx) orbf_destroy(sl.ctx);  // waits for its stream
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.nc_host) hipHostFree(sl.nc_host);
  }
  if (s->base) hipFree(s->base);
  delete s;
}

const char* orbf_server_last_error(const orbf_server* s) {
  return s ? s->err.c_str() : "no server";
}

orbf_status orbf_server_submit(orbf_server* s, const orbf_request* r,
                               uint64_t* ticket) {
  if (!s || !r || !ticket) return ORBF_EINVAL;
  orbf_set_desc probe;
  memset(&probe, 0, sizeof probe);
  probe.xyz = r->xyz;
  probe.N = r->N;
  probe.d = r->d;
  probe.n = r->n;
  probe.m = r->m;
  probe.l = r->l;
  probe.delta = r->delta;
  probe.tau = r->tau;
  probe.prec = r->prec;
  // placeholders for the outputs the server will provide
  probe.knn = probe.col = probe.centers = probe.owner = (int32_t*)s->base;
  probe.rho2 = probe.W = probe.val = (double*)s->base;
  probe.n_centers = probe.row_ptr = (int64_t*)s->base;
  std::string why;
  if (!set_ok(probe, &why)) return sfail(s, ORBF_EINVAL, why);
  if (r->prec != ORBF_PREC_FP64 && r->prec != ORBF_PREC_FP32_IR)
    return sfail(s, ORBF_EINVAL, "unknown precision");
  const size_t bytes = layout(r->N, r->n, r->prec).total;
  if (bytes > s->arena.cap())
    return sfail(s, ORBF_EBUDGET, "outputs larger than the arena");
  if (orbf_workspace_size(r->N, r->d, r->n, r->l, r->prec) > s->slot_budget)
    return sfail(s, ORBF_EBUDGET, "scratch larger than a slot's share");
  const uint64_t id = s->next++;
  Req q;
  q.r = *r;
  q.bytes = bytes;
  s->reqs.emplace(id, q);
  s->queue.push_back(id);
  *ticket = id;
  return ORBF_OK;
}

orbf_status orbf_server_poll(orbf_server* s, uint64_t* done, int cap,
                             int* n_done) {
  if (!s) return ORBF_EINVAL;
  hipSetDevice(s->device);
  retire(s);
  admit(s);
  int k = 0;
  const int take = (int)std::min<size_t>(s->finished.size(),
                                         (size_t)std::max(cap, 0));
  for (; k < take; ++k) done[k] = s->finished[k];
  s->finished.erase(s->finished.begin(), s->finished.begin() + take);
  if (n_done) *n_done = k;
  return ORBF_OK;
}

orbf_status orbf_server_result(orbf_server* s, uint64_t ticket,
                               orbf_result* out) {
  if (!s || !out) return ORBF_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state != DONE)
    return sfail(s, ORBF_EINVAL, "unknown or unfinished ticket");
  const Req& q = it->second;
  out->status = q.status;
  out->N = q.r.N;
  out->n = q.r.n;
  out->n_centers = q.n_centers;
  out->t_arrival = q.r.t_arrival;
  out->t_admit = q.t_admit;
  out->t_done = q.t_done;
  return ORBF_OK;
}

orbf_status orbf_server_fetch(orbf_server* s, uint64_t ticket,
                              const orbf_set_desc* dst) {
  if (!s || !dst) return ORBF_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state != DONE)
    return sfail(s, ORBF_EINVAL, "unknown or unfinished ticket");
  const Req& q = it->second;
  const orbf_set_desc src = desc_of(s, q);
  const size_t Nn = (size_t)q.r.N, nn = Nn * q.r.n;
  struct C { void* d; const void* s; size_t b; } cp[] = {
      {dst->knn, src.knn, nn * 4},         {dst->rho2, src.rho2, Nn * 8},
      {dst->centers, src.centers, Nn * 4}, {dst->n_centers, src.n_centers, 8},
      {dst->owner, src.owner, Nn * 4},     {dst->W, src.W, nn * 8},
      {dst->lebesgue, src.lebesgue, Nn * 8},
      {dst->ir_steps, src.ir_steps, src.ir_steps ? Nn * 4 : 0},
      {dst->row_ptr, src.row_ptr, (Nn + 1) * 8},
      {dst->col, src.col, nn * 4},         {dst->val, src.val, nn * 8}};
  hipSetDevice(s->device);
  for (const C& c : cp) {
    if (!c.d || !c.b) continue;
    hipError_t e = hipMemcpy(c.d, c.s, c.b, hipMemcpyDeviceToDevice);
    if (e != hipSuccess)
      return sfail(s, ORBF_EHIP, std::string("fetch: ") + hipGetErrorString(e));
  }
  return ORBF_OK;
}

orbf_status orbf_server_release(orbf_server* s, uint64_t ticket) {
  if (!s) return ORBF_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state != DONE)
    return sfail(s, ORBF_EINVAL, "unknown or unfinished ticket");
  s->arena.release(it->second.off, it->second.bytes);
  s->reqs.erase(it);
  return ORBF_OK;
}

orbf_status orbf_server_stats(orbf_server* s, int64_t out5[5]) {
  if (!s || !out5) return ORBF_EINVAL;
  int64_t running = 0, done = 0;
  for (auto& kv : s->reqs) {
    running += kv.second.state == RUNNING;
    done += kv.second.state == DONE;
  }
  out5[0] = (int64_t)s->queue.size();
  out5[1] = running;
  out5[2] = done;
  out5[3] = (int64_t)s->arena.used();
  out5[4] = (int64_t)s->arena.cap();
  return ORBF_OK;
}

}  // extern "C"
