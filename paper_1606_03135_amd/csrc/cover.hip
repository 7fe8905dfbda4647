// Greedy overlapped covering (Sec. 4.1: retention ball of radius
// (1-delta) rho_k; a row computed by one stencil is never recomputed).
//
// The paper's rule is sequential: visit nodes in ascending index; an
// unclaimed eligible node becomes a center and claims the unclaimed eligible
// nodes of its ball.  Its result has a parallel characterisation: with edges
// c -> j for every eligible j > c inside ball(c), node j is a center iff no
// predecessor of j is a center, and its owner is the smallest center among
// its predecessors.  The device evaluates that DAG:
//   1. ball masks and in-degrees (one thread per node),
//   2. predecessor lists (scan + atomic fill),
//   3. a fixed number of parallel rounds (each undecided node is decided as
//      soon as one predecessor is a center, or all predecessors are
//      non-centers),
//   4. rounds over the compacted list of nodes still undecided, then a
//      single-workgroup finish over whatever remains, in ascending order,
//      so no host round trip is needed,
//   5. owners, the ascending center list and p per center.
#include <utility>

#include "orbf_internal.hpp"

namespace orbf {

namespace {

enum : int32_t { S_UNDECIDED = 0, S_CENTER = 1, S_COVERED = 2, S_INELIGIBLE = 3 };
constexpr int kRounds = 10;      // full rounds over all nodes
constexpr int kListRounds = 24;  // rounds over the remaining undecided
constexpr int kCheck = 64;       // further rounds between open-count checks
constexpr int kMaxCheck = 256;   // checks before the finish takes the rest
constexpr int64_t kFinishLeft = 256;  // open nodes left to the finish

// Retention balls from the coordinates: one thread per node, gathering the
// coordinates of its stencil.
__global__ __launch_bounds__(256) void ball_kernel(
    const double* __restrict__ x, const int32_t* __restrict__ knn,
    const double* __restrict__ rho2, int64_t N, int d, int n, double t2,
    const uint8_t* __restrict__ eligible, uint64_t* __restrict__ ball,
    int32_t* __restrict__ indeg, int32_t* __restrict__ state, int32_t s_open,
    int32_t s_inel) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  uint64_t b0 = 0, b1 = 0;
  const bool ec = eligible == nullptr || eligible[c] != 0;
  state[c] = ec ? s_open : s_inel;
  if (ec) {
    const double thr = t2 * rho2[c];
    const double cx = x[c * d], cy = x[c * d + 1];
    const double cz = (d == 3) ? x[c * d + 2] : 0.0;
    const int32_t* st = knn + c * n;
    for (int q = 1; q < n; ++q) {
      const int32_t j = st[q];
      if (j <= c || j >= N) continue;  // j >= N only after a failed kNN
      if (eligible != nullptr && eligible[j] == 0) continue;
      const double* p = x + (int64_t)j * d;
      const double d2 =
          exact_sqdist(cx, cy, cz, p[0], p[1], d == 3 ? p[2] : 0.0, d);
      if (d2 <= thr) {
        if (q < 64)
          b0 |= 1ull << q;
        else
          b1 |= 1ull << (q - 64);
        atomicAdd(&indeg[j], 1);
      }
    }
  }
  ball[2 * c] = b0;
  ball[2 * c + 1] = b1;
}

// Retention balls from the squared distances the kNN recorded for the same
// arrays (identical values: same formula, same operand order): one
// wavefront per node, taken in the kNN's cell order so the distance rows
// stream; lane q tests stencil position q and a ballot forms the mask.
__global__ __launch_bounds__(256) void ball_d2_kernel(
    const double* __restrict__ d2s, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ knn, const double* __restrict__ rho2,
    int64_t N, int n, double t2, const uint8_t* __restrict__ eligible,
    uint64_t* __restrict__ ball, int32_t* __restrict__ indeg,
    int32_t* __restrict__ state, int32_t s_open, int32_t s_inel) {
  const int64_t qs = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (qs >= N) return;  // whole wavefront
  const int64_t c = perm[qs];
  const double* d2 = d2s + qs * n;
  const bool ec = eligible == nullptr || eligible[c] != 0;
  const double thr = t2 * rho2[c];
  uint64_t b[2] = {0ull, 0ull};
  for (int h = 0; h < 2 && 64 * h < n; ++h) {
    const int q = lane + 64 * h;
    bool in = false;
    if (ec && q >= 1 && q < n) {
      const int32_t j = knn[c * n + q];
      if (j > c && j < N && (eligible == nullptr || eligible[j] != 0) &&
          d2[q] <= thr) {
        in = true;
        atomicAdd(&indeg[j], 1);
      }
    }
    b[h] = __ballot(in);
  }
  if (lane == 0) {
    state[c] = ec ? s_open : s_inel;
    ball[2 * c] = b[0];
    ball[2 * c + 1] = b[1];
  }
}

// The same for n <= 64 with four nodes per wavefront, sixteen lanes per
// node and four stencil positions per lane: each wavefront has four nodes'
// dependent loads and all their in-degree updates in flight at once.
__global__ __launch_bounds__(256) void ball_d2_quad_kernel(
    const double* __restrict__ d2s, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ knn, const double* __restrict__ rho2,
    int64_t N, int n, double t2, const uint8_t* __restrict__ eligible,
    uint64_t* __restrict__ ball, int32_t* __restrict__ indeg,
    int32_t* __restrict__ state, int32_t s_open, int32_t s_inel) {
  const int lane = threadIdx.x & 63, part = lane >> 4, pl = lane & 15;
  const int64_t qs = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6) * 4 + part;
  const bool valid = qs < N;  // no early return: the ballots need every lane
  int64_t c = 0;
  bool ec = false;
  double thr = 0.0;
  if (valid) {
    c = perm[qs];
    ec = eligible == nullptr || eligible[c] != 0;
    thr = t2 * rho2[c];
  }
  uint64_t bw[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = pl + 16 * i;
    bool in = false;
    if (ec && q >= 1 && q < n) {
      const double dq = d2s[qs * n + q];
      const int32_t j = knn[c * n + q];
      if (j > c && j < N && (eligible == nullptr || eligible[j] != 0) &&
          dq <= thr) {
        in = true;
        atomicAdd(&indeg[j], 1);
      }
    }
    bw[i] = __ballot(in);
  }
  if (valid && pl == 0) {
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) m |= ((bw[i] >> (16 * part)) & 0xFFFFull) << (16 * i);
    state[c] = ec ? s_open : s_inel;
    ball[2 * c] = m;
    ball[2 * c + 1] = 0ull;
  }
}

// Predecessor lists: sixteen lanes per node, eight stencil positions per
// lane (n <= 128), so all of a node's list insertions are in flight at once.
__global__ __launch_bounds__(256) void pred_fill_kernel(
    const int32_t* __restrict__ knn, int64_t N, int n,
    const uint64_t* __restrict__ ball, const int64_t* __restrict__ start,
    int32_t* __restrict__ fill, int32_t* __restrict__ pred) {
  const int64_t c = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
  const int pl = threadIdx.x & 15;
  if (c >= N) return;
  const uint64_t b0 = ball[2 * c], b1 = ball[2 * c + 1];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int q = pl + 16 * i;
    const uint64_t b = q < 64 ? b0 : b1;
    if (q < n && ((b >> (q & 63)) & 1ull)) {
      const int32_t j = knn[c * n + q];
      const int slot = atomicAdd(&fill[j], 1);
      pred[start[j] + slot] = (int32_t)c;
    }
  }
}

// Decide j from its predecessors' current states.  States only move from
// UNDECIDED to a final value, so reading a stale state can only delay a
// decision, never change it.
__device__ __forceinline__ int32_t decide(const int32_t* __restrict__ pred,
                                          int64_t p0, int64_t p1,
                                          const int32_t* state) {
  bool all = true;
  for (int64_t t = p0; t < p1; ++t) {
    const int32_t s = __atomic_load_n(&state[pred[t]], __ATOMIC_RELAXED);
    if (s == S_CENTER) return S_COVERED;
    if (s == S_UNDECIDED) all = false;
  }
  return all ? S_CENTER : S_UNDECIDED;
}

__global__ __launch_bounds__(256) void round_kernel(
    const int32_t* __restrict__ pred, const int64_t* __restrict__ start,
    int64_t N, int32_t* state) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  if (state[j] != S_UNDECIDED) return;
  const int32_t s = decide(pred, start[j], start[j + 1], state);
  if (s != S_UNDECIDED) __atomic_store_n(&state[j], s, __ATOMIC_RELAXED);
}

// A round over the compacted list of nodes still undecided after the full
// rounds (grid-stride; the list length is on the device).
__global__ __launch_bounds__(256) void round_list_kernel(
    const int32_t* __restrict__ pred, const int64_t* __restrict__ start,
    const int32_t* __restrict__ list, const int64_t* __restrict__ count,
    int32_t* state) {
  const int64_t cnt = *count;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < cnt;
       t += (int64_t)gridDim.x * 256) {
    const int32_t j = list[t];
    if (__atomic_load_n(&state[j], __ATOMIC_RELAXED) != S_UNDECIDED) continue;
    const int32_t s = decide(pred, start[j], start[j + 1], state);
    if (s != S_UNDECIDED) __atomic_store_n(&state[j], s, __ATOMIC_RELAXED);
  }
}

// Number of list entries still undecided (one atomic per block).
__global__ __launch_bounds__(256) void count_open_kernel(
    const int32_t* __restrict__ list, const int64_t* __restrict__ count,
    const int32_t* state, int64_t* __restrict__ open) {
  __shared__ int blk;
  if (threadIdx.x == 0) blk = 0;
  __syncthreads();
  const int64_t cnt = *count;
  int mine = 0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < cnt;
       t += (int64_t)gridDim.x * 256)
    mine += __atomic_load_n(&state[list[t]], __ATOMIC_RELAXED) == S_UNDECIDED;
  if (mine) atomicAdd(&blk, mine);
  __syncthreads();
  if (threadIdx.x == 0 && blk)
    atomicAdd((unsigned long long*)open, (unsigned long long)blk);
}

__global__ void zero_i64_kernel(int64_t* p) { *p = 0; }

__global__ __launch_bounds__(256) void undecided_flag_kernel(
    const int32_t* __restrict__ state, int64_t N, int32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < N) flag[j] = state[j] == S_UNDECIDED;
}

__global__ __launch_bounds__(256) void compact_kernel(
    const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
    int64_t N, int32_t* __restrict__ list) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < N && flag[j]) list[pos[j]] = (int32_t)j;
}

// One workgroup finishes the remaining undecided nodes.  Every pass
// decides at least the smallest undecided node (all its predecessors are
// smaller, hence decided), so the loop ends after at most |list| passes.
__global__ __launch_bounds__(1024) void finish_kernel(
    const int32_t* __restrict__ pred, const int64_t* __restrict__ start,
    const int32_t* __restrict__ list, const int64_t* __restrict__ count,
    int32_t* state) {
  __shared__ int left;
  const int64_t cnt = *count;
  for (int64_t pass = 0; pass <= cnt; ++pass) {
    if (threadIdx.x == 0) left = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < cnt; t += 1024) {
      const int32_t j = list[t];
      if (__atomic_load_n(&state[j], __ATOMIC_RELAXED) != S_UNDECIDED) continue;
      const int32_t s = decide(pred, start[j], start[j + 1], state);
      if (s != S_UNDECIDED)
        __atomic_store_n(&state[j], s, __ATOMIC_RELAXED);
      else
        atomicAdd(&left, 1);
    }
    __threadfence_block();
    __syncthreads();
    const int l = left;
    __syncthreads();
    if (l == 0) break;
  }
}

__global__ __launch_bounds__(256) void owner_kernel(
    const int32_t* __restrict__ pred, const int64_t* __restrict__ start,
    const int32_t* __restrict__ state, int64_t N, int32_t* __restrict__ owner,
    int32_t* __restrict__ is_center) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int32_t s = state[j];
  int32_t o = -1;
  if (s == S_CENTER) {
    o = (int32_t)j;
  } else if (s == S_COVERED) {
    o = INT32_MAX;
    for (int64_t t = start[j]; t < start[j + 1]; ++t) {
      const int32_t c = pred[t];
      if (state[c] == S_CENTER && c < o) o = c;
    }
  }
  owner[j] = o;
  is_center[j] = (s == S_CENTER);
}

__global__ __launch_bounds__(256) void centers_kernel(
    const int32_t* __restrict__ is_center, const int64_t* __restrict__ pos,
    const int32_t* __restrict__ knn, const uint64_t* __restrict__ ball,
    const int32_t* __restrict__ owner, int64_t N, int n,
    int32_t* __restrict__ centers, int32_t* __restrict__ p,
    int32_t* __restrict__ p_keep, int64_t* __restrict__ n_centers) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c == N) *n_centers = pos[N];
  if (c >= N || !is_center[c]) return;
  int cnt = 1;
  for (int h = 0; h < 2; ++h) {
    uint64_t b = ball[2 * c + h];
    while (b) {
      const int q = __ffsll((long long)b) - 1 + 64 * h;
      b &= b - 1;
      cnt += owner[knn[c * n + q]] == (int32_t)c;
    }
  }
  centers[pos[c]] = (int32_t)c;
  if (p) p[pos[c]] = cnt;
  p_keep[pos[c]] = cnt;
}

__global__ __launch_bounds__(256) void zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

}  // namespace

void launch_ball(orbf_ctx* ctx, const double* xyz, const int32_t* knn,
                 const double* rho2, int64_t N, int d, int n, double t2,
                 const uint8_t* eligible, uint64_t* ball, int32_t* indeg,
                 int32_t* state, int32_t s_open, int32_t s_inel) {
  hipStream_t s = ctx->stream;
  if (ctx->d2_cache.matches(xyz, knn, N, d, n) && n <= 64) {
    hipLaunchKernelGGL(ball_d2_quad_kernel, dim3((unsigned)((N + 15) / 16)),
                       dim3(256), 0, s, ctx->d2_cache.d2, ctx->d2_cache.perm,
                       knn, rho2, N, n, t2, eligible, ball, indeg, state,
                       s_open, s_inel);
  } else if (ctx->d2_cache.matches(xyz, knn, N, d, n)) {
    hipLaunchKernelGGL(ball_d2_kernel, dim3((unsigned)((N + 3) / 4)),
                       dim3(256), 0, s, ctx->d2_cache.d2, ctx->d2_cache.perm,
                       knn, rho2, N, n, t2, eligible, ball, indeg, state,
                       s_open, s_inel);
  } else {
    hipLaunchKernelGGL(ball_kernel, dim3((unsigned)((N + 255) / 256)),
                       dim3(256), 0, s, xyz, knn, rho2, N, d, n, t2, eligible,
                       ball, indeg, state, s_open, s_inel);
  }
}

orbf_status launch_cover(orbf_ctx* ctx, const double* xyz, const int32_t* knn,
                         const double* rho2, int64_t N, int d, int n,
                         double t2, const uint8_t* eligible, int32_t* centers,
                         int64_t* n_centers, int32_t* owner, int32_t* p) {
  orbf_status st = ORBF_OK;
  auto* ball = (uint64_t*)scratch(ctx, B_BALL, (size_t)N * 16, &st);
  auto* indeg = (int32_t*)scratch(ctx, B_INDEG, (size_t)(N + 1) * 4, &st);
  auto* pstart = (int64_t*)scratch(ctx, B_PRED_START, (size_t)(N + 2) * 8, &st);
  auto* fill = (int32_t*)scratch(ctx, B_PRED_FILL, (size_t)(N + 1) * 4, &st);
  auto* state = (int32_t*)scratch(ctx, B_STATE, (size_t)N * 4, &st);
  auto* flag = (int32_t*)scratch(ctx, B_FLAGS, (size_t)(N + 1) * 4, &st);
  auto* pos = (int64_t*)scratch(ctx, B_CENTER_POS, (size_t)(N + 2) * 8, &st);
  if (st) return st;
  hipStream_t s = ctx->stream;
  const unsigned g = (unsigned)((N + 255) / 256);
  const unsigned gz = (unsigned)((N + 256) / 256 < 65535 ? (N + 256) / 256 : 65535);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(gz), dim3(256), 0, s, indeg, N + 1);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(gz), dim3(256), 0, s, fill, N + 1);
  launch_ball(ctx, xyz, knn, rho2, N, d, n, t2, eligible, ball, indeg, state,
              S_UNDECIDED, S_INELIGIBLE);
  st = exclusive_scan_i32_to_i64(ctx, indeg, N, pstart);
  if (st) return st;
  // the predecessor array is sized from the edge count, known only on the
  // device; N * (n - 1) bounds it
  const size_t max_edges = (size_t)N * (size_t)(n > 1 ? n - 1 : 1);
  auto* pred = (int32_t*)scratch(ctx, B_PRED, max_edges * 4, &st);
  if (st) return st;
  hipLaunchKernelGGL(pred_fill_kernel, dim3((unsigned)((N + 15) / 16)),
                     dim3(256), 0, s, knn, N, n, ball, pstart, fill, pred);
  for (int r = 0; r < kRounds; ++r)
    hipLaunchKernelGGL(round_kernel, dim3(g), dim3(256), 0, s, pred, pstart, N,
                       state);
  // stragglers: ascending list of undecided nodes, finished by one workgroup
  auto* list = (int32_t*)scratch(ctx, B_ROWPTR_TMP, (size_t)(N + 1) * 4, &st);
  if (st) return st;
  hipLaunchKernelGGL(undecided_flag_kernel, dim3(g), dim3(256), 0, s, state, N,
                     flag);
  st = exclusive_scan_i32_to_i64(ctx, flag, N, pos);
  if (st) return st;
  hipLaunchKernelGGL(compact_kernel, dim3(g), dim3(256), 0, s, flag, pos, N,
                     list);
  // Rounds over the stragglers only.  An input order with long dependency
  // chains (a raster-ordered grid) needs as many rounds as the chains are
  // long: an eager call keeps launching rounds, checking the open count
  // every kCheck rounds, and records how many it used; a call under graph
  // capture cannot check and replays the recorded count.  One workgroup
  // finishes whatever is left either way.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipStreamIsCapturing(s, &cap);
  const std::pair<const void*, int64_t> key(knn, N);
  int recorded = -1;
  for (size_t i = 0; i < ctx->cover_keys.size(); ++i)
    if (ctx->cover_keys[i] == key) recorded = ctx->cover_rounds[i];
  auto rounds = [&](int k) {
    for (int r = 0; r < k; ++r)
      hipLaunchKernelGGL(round_list_kernel, dim3(256), dim3(256), 0, s, pred,
                         pstart, list, pos + N, state);
  };
  int used = kListRounds;
  if (cap != hipStreamCaptureStatusNone) {
    rounds(recorded > 0 ? recorded : kListRounds);
  } else {
    rounds(kListRounds);
    auto* open = (int64_t*)scratch(ctx, B_MISC, 8, &st);
    if (st) return st;
    for (int batch = 0; batch < kMaxCheck; ++batch) {
      hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(1), 0, s, open);
      hipLaunchKernelGGL(count_open_kernel, dim3(256), dim3(256), 0, s, list,
                         pos + N, state, open);
      hipError_t e = hipMemcpyAsync(ctx->host_counter, open, sizeof(int64_t),
                                    hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if ((st = hip_check(ctx, e, "cover: open count"))) return st;
      if (*ctx->host_counter <= kFinishLeft) break;
      rounds(kCheck);
      used += kCheck;
    }
    bool found = false;
    for (size_t i = 0; i < ctx->cover_keys.size(); ++i)
      if (ctx->cover_keys[i] == key) {
        ctx->cover_rounds[i] = used;
        found = true;
      }
    if (!found) {
      if (ctx->cover_keys.size() >= 4096) {
        ctx->cover_keys.clear();
        ctx->cover_rounds.clear();
      }
      ctx->cover_keys.push_back(key);
      ctx->cover_rounds.push_back(used);
    }
  }
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(1024), 0, s, pred, pstart,
                     list, pos + N, state);
  hipLaunchKernelGGL(owner_kernel, dim3(g), dim3(256), 0, s, pred, pstart,
                     state, N, owner, flag);
  st = exclusive_scan_i32_to_i64(ctx, flag, N, pos);
  if (st) return st;
  // the row counts are also kept in the context, for the weights entry
  // point's choice of pass width
  auto* p_keep = (int32_t*)scratch(ctx, B_P_CACHE, (size_t)N * 4, &st);
  if (st) return st;
  hipLaunchKernelGGL(centers_kernel, dim3((unsigned)((N + 256) / 256)),
                     dim3(256), 0, s, flag, pos, knn, ball, owner, N, n,
                     centers, p, p_keep, n_centers);
  ctx->p_cache = {centers, owner, N, n, p_keep};
  return hip_check(ctx, hipGetLastError(), "cover");
}

}  // namespace orbf
