// Greedy covering with the local L-Lebesgue test (Sec. 4.2.1, eq. calLstab
// with threshold tau): node j of stencil k is kept only if j is the center
// or Lambda(x_j) <= tau * Lambda(x_ref), x_ref the stencil node nearest the
// stencil centroid; a rejected node is left for a later stencil.
//
// Whether center c keeps j depends on c's stencil alone, so the sequential
// rule (ascending index) again has a parallel form.  With edges c -> j for
// eligible j > c in ball(c): j is a center iff every predecessor is a
// non-center or a center that rejects j; its owner is the smallest
// predecessor center that keeps it.
//
// The device settles that DAG with work proportional to its edges.  Every
// node j counts the predecessors that can no longer keep it: non-centers
// and centers that reject j.  A center that keeps j offers itself as j's
// owner (atomic min, the smallest offer winning; the first offer finds the
// owner unset and covers j) and never counts off, so a count that reaches
// zero proves that no predecessor keeps j: j is a center.  A node just
// covered counts itself off its own ball nodes.
// Every step is a relaxed atomic on one word; nothing needs ordering
// across words.
//
// A center's keep bits come from solving its stencil (the register kernel
// in acceptance mode), which needs the center decided first: level k
// solves the centers decided by level k - 1 and propagates them.  On a
// scattered numbering the DAG is shallow and a few levels settle it; on a
// spatially ordered one (a generation front, a raster) it is hundreds of
// levels deep, and one stencil solve per level would put hundreds of solve
// latencies on the critical path.  So after a few levels every node still
// undecided that has a ball is solved at once (its keep bits depend on its
// own stencil only, whatever it turns out to be), and the rest of the DAG
// settles by integer propagation alone, one launch per level, one group of
// sixteen lanes per decided node (a covered node's count-offs spread over
// its group rather than looped by one lane).  (One workgroup running all
// the remaining levels in a single launch measured slower: 10.7 against
// 4.9 ms on the 100k disk in generation order, since every level's chain
// of dependent atomics then funnels through one CU.)
#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

// accept-mode solve blocks per level (100k disk, whole build, shuffled /
// generation order: 1.480-1.489 / 4.11-4.15 ms at 4096, 1.50 / 4.06 at
// 16384, 1.50 / 4.05-4.07 at 65536)
constexpr int64_t kSolveGrid = 4096;
constexpr unsigned kPropBlocks = 256;   // propagation: 4 wavefronts a block
// levels solved one by one before the speculative solve (100k disk, whole
// build, shuffled / generation order: 1.52 / 4.08-4.14 ms at 3, 1.555 /
// 4.10 at 4, 1.474 / 4.09-4.16 at 6, 1.49 / 4.09-4.11 at 8)
constexpr int64_t kSolvedLevels = 6;
// propagation-only levels: 16 groups a block (100k disk in generation
// order, whole build: 4.02-4.06 ms at 128, 512 and 2048 blocks alike; the
// levels are launch bound)
constexpr unsigned kFollowBlocks = 512;
// decisions a group follows itself per entry in the propagation-only
// levels (100k disk in generation order, whole build: 4.75-4.96 ms at 1,
// 5.38 at 0, 5.30 at 2, 5.43 at 4, 5.80 at 16, 6.53 at 64: long follows
// serialise what the level spreads over the device)
constexpr int kFollow = 1;

// A covered node keeps L_UNDECIDED: its owner word (set by the first
// keeping center) is what marks it.
enum : int32_t {
  L_UNDECIDED = 0,
  L_CENTER = 1,   // center (its level solves it)
  L_INELIGIBLE = 3
};


__device__ __forceinline__ void push(int32_t* list, int64_t* count,
                                     int32_t j) {
  const int64_t slot = __hip_atomic_fetch_add(count, (int64_t)1,
                                              __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&list[slot], j, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// j loses one predecessor that cannot keep it; the last one makes j a
// center of the next level
__device__ __forceinline__ void count_off(int32_t* open, int32_t* state,
                                          int32_t j, int32_t* next,
                                          int64_t* next_count) {
  const int32_t left = __hip_atomic_fetch_add(&open[j], -1, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
  if (left == 1) {
    __hip_atomic_store(&state[j], L_CENTER, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    push(next, next_count, j);
  }
}

// center c keeps j: c offers itself as owner (the smallest offer wins); the
// first offer finds the owner unset, covers j, and j's ball nodes count it
// off (a center never has a keeping predecessor, so is never offered)
__device__ __forceinline__ void claim(int32_t c, int32_t j,
                                      const int32_t* __restrict__ knn, int n,
                                      const uint64_t* __restrict__ ball,
                                      int32_t* open, int32_t* state,
                                      int32_t* owner, int32_t* next,
                                      int64_t* next_count) {
  if (__hip_atomic_fetch_min(&owner[j], c, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) != INT32_MAX)
    return;
  for (int hj = 0; hj < 2 && 64 * hj < n; ++hj) {
    uint64_t b = ball[2 * (int64_t)j + hj];
    while (b) {
      const int qj = __ffsll((long long)b) - 1 + 64 * hj;
      b &= b - 1;
      count_off(open, state, knn[(int64_t)j * n + qj], next, next_count);
    }
  }
}

// owners start unset (eligible) or -1; nodes with no predecessor are the
// push j for every lane with `take`, one atomic per wavefront (one per
// node put up to N atomics on one counter); every lane of the wavefront
// calls it
__device__ __forceinline__ void push_wave(int32_t* list, int64_t* count,
                                          int32_t j, bool take) {
  const uint64_t m = __ballot(take);
  if (m == 0) return;
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((long long)m) - 1;
  int64_t base = 0;
  if (lane == leader)
    base = __hip_atomic_fetch_add(count, (int64_t)__popcll(m),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader, 64);
  if (take)
    __hip_atomic_store(&list[base + __popcll(m & ((1ull << lane) - 1ull))],
                       j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// first level's centers
__global__ __launch_bounds__(256) void lseed_kernel(
    const int32_t* __restrict__ open, int64_t N, int32_t* state,
    int32_t* __restrict__ owner, int32_t* __restrict__ list,
    int64_t* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool take = false;  // no early return: the push is per wavefront
  if (j < N) {
    const bool el = state[j] != L_INELIGIBLE;
    owner[j] = el ? INT32_MAX : -1;
    take = el && open[j] == 0;
    if (take) state[j] = L_CENTER;
  }
  push_wave(list, count, (int32_t)j, take);
}

// every undecided node with a nonempty ball, for the speculative solve
__global__ __launch_bounds__(256) void lspec_kernel(
    const int32_t* __restrict__ state, const int32_t* __restrict__ owner,
    const uint64_t* __restrict__ ball, int64_t N, int32_t* __restrict__ list,
    int64_t* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool take = j < N && state[j] == L_UNDECIDED &&
                    owner[j] == INT32_MAX && (ball[2 * j] | ball[2 * j + 1]);
  push_wave(list, count, (int32_t)j, take);
}

// one wavefront per center of the level; lane q takes stencil position q
// (and q + 64)
__global__ __launch_bounds__(256) void lprop_kernel(
    const int32_t* __restrict__ list, const int64_t* __restrict__ count,
    const int32_t* __restrict__ knn, int n, const uint64_t* __restrict__ ball,
    const uint64_t* __restrict__ acc, int32_t* open, int32_t* state,
    int32_t* owner, int32_t* next, int64_t* next_count, int64_t* zero) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *zero = 0;
  const int lane = threadIdx.x & 63;
  const int64_t cnt = *count;
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < cnt;
       w += (int64_t)gridDim.x * 4) {
    const int32_t c = list[w];
    for (int h = 0; h < 2 && 64 * h < n; ++h) {
      const int q = lane + 64 * h;
      const uint64_t bit = 1ull << lane;
      if (!(ball[2 * (int64_t)c + h] & bit)) continue;
      const int32_t j = knn[(int64_t)c * n + q];
      if (!(acc[2 * (int64_t)c + h] & bit)) {  // c rejects j
        count_off(open, state, j, next, next_count);
        continue;
      }
      claim(c, j, knn, n, ball, open, state, owner, next, next_count);
    }
  }
}

// After the speculative solve every node that can still become a center has
// its keep bits, so the rest of the DAG is integer propagation in any order.
// One group of sixteen lanes per entry (lane p takes stencil positions
// p + 16 i): an entry is a center (j >= 0: its rejected ball nodes count it
// off, its kept ones get its offer) or a node just covered (j | INT32_MIN:
// its ball nodes count it off).  The decisions a group makes are followed
// by the group itself through a small LDS stack, up to `follow` of them per
// entry; the rest go to the next level's list.  Every node is decided once,
// so it enters a list at most once.
constexpr int kLStack = 32;

__device__ __forceinline__ void lfollow_entry(
    int32_t entry, int32_t* stk, const int32_t* __restrict__ knn, int n,
    const uint64_t* __restrict__ ball, const uint64_t* __restrict__ acc,
    int32_t* open, int32_t* state, int32_t* owner, int32_t* next,
    int64_t* next_count, int follow) {
  const int lane = (int)(threadIdx.x & 63), pl = lane & 15;
  const int gshift = lane & 48;  // first lane of the group in the wave
  const uint32_t below = (1u << pl) - 1u;
  constexpr int32_t kNone = INT32_MAX;  // no decision (N < 2^25)
  int sp = 0;
  int32_t e = entry;
  for (;;) {
    const bool covered = e < 0;
    const int32_t c = e & INT32_MAX;
    const uint64_t b0 = ball[2 * (int64_t)c], b1 = ball[2 * (int64_t)c + 1];
    const uint64_t k0 = covered ? 0ull : acc[2 * (int64_t)c];
    const uint64_t k1 = covered ? 0ull : acc[2 * (int64_t)c + 1];
    int32_t dec[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = pl + 16 * i;
      dec[i] = kNone;
      const uint64_t bits = q < 64 ? b0 : b1;
      const uint64_t keep = q < 64 ? k0 : k1;
      if (q < n && ((bits >> (q & 63)) & 1ull)) {
        const int32_t j = knn[(int64_t)c * n + q];
        if (covered || !((keep >> (q & 63)) & 1ull)) {
          const int32_t left = __hip_atomic_fetch_add(
              &open[j], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (left == 1) {
            __hip_atomic_store(&state[j], L_CENTER, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            dec[i] = j;
          }
        } else if (__hip_atomic_fetch_min(&owner[j], c, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) ==
                   INT32_MAX) {
          dec[i] = j | INT32_MIN;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (16 * i >= n) break;
      const uint32_t m =
          (uint32_t)(__ballot(dec[i] != kNone) >> gshift) & 0xFFFFu;
      if (m == 0u) continue;
      const int k = __popc(m);
      int room = kLStack - sp;
      if (room > follow) room = follow;
      const int kept = k < room ? k : room;
      const int r = __popc(m & below);
      int64_t base = 0;
      if (k > kept) {
        if (pl == __ffs(m) - 1)
          base = __hip_atomic_fetch_add(next_count, (int64_t)(k - kept),
                                        __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, gshift + __ffs(m) - 1, 64);
      }
      if (dec[i] != kNone) {
        if (r < kept)
          stk[sp + r] = dec[i];
        else
          __hip_atomic_store(&next[base + r - kept], dec[i], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      sp += kept;
      follow -= kept;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (sp == 0) break;
    e = stk[--sp];
  }
}

// One propagation-only level, number `lvl`: the entries of `list` (count
// *count), one group of sixteen lanes each; *zero (the count the previous
// level read) is cleared for the next, and a level with entries records
// its number in *depth.
__global__ __launch_bounds__(256) void lfollow_kernel(
    const int32_t* __restrict__ list, const int64_t* __restrict__ count,
    const int32_t* __restrict__ knn, int n, const uint64_t* __restrict__ ball,
    const uint64_t* __restrict__ acc, int32_t* open, int32_t* state,
    int32_t* owner, int32_t* next, int64_t* next_count, int64_t* zero,
    int follow, int64_t lvl, int64_t* depth) {
  __shared__ int32_t stk[16 * kLStack];
  const int grp = threadIdx.x >> 4;
  const int64_t cnt = *count;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *zero = 0;
    if (cnt > 0) *depth = lvl;
  }
  for (int64_t t = (int64_t)blockIdx.x * 16 + grp; t < cnt;
       t += (int64_t)gridDim.x * 16)
    lfollow_entry(list[t], stk + grp * kLStack, knn, n, ball, acc, open,
                  state, owner, next, next_count, follow);
}

// centers own themselves; flags for the ascending center list
__global__ __launch_bounds__(256) void lfinal_kernel(
    const int32_t* __restrict__ state, int64_t N, int32_t* __restrict__ owner,
    int32_t* __restrict__ is_center, DevStatus* st) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int32_t s = state[j];
  if (s == L_CENTER) owner[j] = (int32_t)j;
  // neither a center nor covered: the levels ended before the DAG settled
  if (s == L_UNDECIDED && owner[j] == INT32_MAX) {
    report(st, ORBF_EINTERNAL, (int)j);
    owner[j] = -1;
  }
  is_center[j] = s == L_CENTER;
}

__global__ __launch_bounds__(256) void lcompact_kernel(
    const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
    int64_t N, int32_t* __restrict__ list, int64_t* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j == N) *count = pos[N];
  if (j < N && flag[j]) list[pos[j]] = (int32_t)j;
}

// the three list counts and the last propagation level with entries
__global__ void lzero4_kernel(int64_t* c) {
  if (threadIdx.x < 4) c[threadIdx.x] = 0;
}

__global__ void lzero1_kernel(int64_t* c) {
  if (threadIdx.x == 0) *c = 0;
}

__global__ __launch_bounds__(256) void lzero_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

}  // namespace

orbf_status launch_lebesgue_cover(orbf_ctx* ctx, const WeightsParams& P0,
                                  double t2, const uint8_t* eligible,
                                  int32_t* centers, int64_t* n_centers,
                                  int32_t* owner) {
  const int64_t N = P0.N;
  const int n = P0.n, d = P0.d;
  if (N >= (1 << 25) || n > 128)
    return fail(ctx, ORBF_EINVAL, "Lebesgue covering: N < 2^25, n <= 128");
  orbf_status st = ORBF_OK;
  auto* ball = (uint64_t*)scratch(ctx, B_BALL, (size_t)N * 16, &st);
  auto* open = (int32_t*)scratch(ctx, B_INDEG, (size_t)(N + 1) * 4, &st);
  auto* state = (int32_t*)scratch(ctx, B_STATE, (size_t)N * 4, &st);
  auto* flag = (int32_t*)scratch(ctx, B_FLAGS, (size_t)(N + 1) * 4, &st);
  auto* pos = (int64_t*)scratch(ctx, B_CENTER_POS, (size_t)(N + 2) * 8, &st);
  auto* lists = (int32_t*)scratch(ctx, B_PRED, (size_t)(N + 1) * 12, &st);
  auto* acc = (uint64_t*)scratch(ctx, B_W_TMP, (size_t)N * 16, &st);
  auto* cnt = (int64_t*)scratch(ctx, B_MISC2, 64, &st);
  if (st) return st;
  int32_t* list[3] = {lists, lists + (N + 1), lists + 2 * (N + 1)};
  hipStream_t s = ctx->stream;
  const unsigned g = (unsigned)((N + 255) / 256);
  const unsigned g1 = (unsigned)((N + 256) / 256);
  const unsigned gz = g1 < 65535 ? g1 : 65535;
  hipLaunchKernelGGL(lzero_kernel, dim3(gz), dim3(256), 0, s, open, N + 1);
  // acceptance words need no clearing: a center's are written by its solve
  // before its propagation reads them, and nothing else reads them
  hipLaunchKernelGGL(lzero4_kernel, dim3(1), dim3(64), 0, s, cnt);
  launch_ball(ctx, P0.xyz, P0.knn, P0.rho2, N, d, n, t2, eligible, ball, open,
              state, L_UNDECIDED, L_INELIGIBLE);
  hipLaunchKernelGGL(lseed_kernel, dim3(g), dim3(256), 0, s, open, N, state,
                     owner, list[0], cnt);

  WeightsParams P = P0;
  P.eligible = eligible;
  P.t2 = t2;
  P.ball = ball;
  P.accept = acc;
  P.owner = nullptr;
  P.W = nullptr;
  P.lebesgue = nullptr;
  // Level k propagates list k % 3 into list (k + 1) % 3 and clears the
  // count of list (k + 2) % 3, which level k - 1 has finished with and
  // level k + 1 fills.  Until the speculative solve, level k first solves
  // its list.  The kernels read the counts on the device, so levels run
  // back to back; the host reads the next level's count only after each
  // batch of levels, and levels past the last find nothing to do.
  const unsigned gs = (unsigned)(N < kSolveGrid ? N : kSolveGrid);
  const unsigned gp = (unsigned)((N + 3) / 4 < kPropBlocks ? (N + 3) / 4
                                                            : kPropBlocks);
  const unsigned gf = (unsigned)((N + 15) / 16 < kFollowBlocks
                                     ? (N + 15) / 16
                                     : kFollowBlocks);
  int64_t level = 0;
  bool solving = true;
  auto solve = [&](int32_t* l, int64_t* c) -> orbf_status {
    P.centers = l;
    P.n_centers = c;
    if (!launch_weights_reg(ctx, P, gs))
      return fail(ctx, ORBF_EINVAL,
                  "Lebesgue covering needs the register weights kernel "
                  "(n + M <= 72, M <= 35)");
    return ORBF_OK;
  };
  // The solved levels run back to back and the host checks once after
  // them; the propagation-only levels after batches of 1, 2, 4, ... 64, or
  // first after as many as the last call on the same arrays needed.
  const std::pair<const void*, int64_t> key(P0.knn, N);
  int64_t recorded = 0;
  for (size_t i = 0; i < ctx->leb_keys.size(); ++i)
    if (ctx->leb_keys[i] == key) recorded = ctx->leb_levels[i];
  int64_t first_prop = -1;  // number of the first propagation-only level
  bool from_record = false;  // the current batch is the recorded depth
  int batch = (int)kSolvedLevels;
  for (;;) {
    for (int r = 0; r < batch; ++r, ++level) {
      const int a = (int)(level % 3), b = (a + 1) % 3, z = (a + 2) % 3;
      if (solving) {
        if ((st = solve(list[a], cnt + a))) return st;
        hipLaunchKernelGGL(lprop_kernel, dim3(gp), dim3(256), 0, s, list[a],
                           cnt + a, P0.knn, n, ball, acc, open, state, owner,
                           list[b], cnt + b, cnt + z);
      } else {
        hipLaunchKernelGGL(lfollow_kernel, dim3(gf), dim3(256), 0, s, list[a],
                           cnt + a, P0.knn, n, ball, acc, open, state, owner,
                           list[b], cnt + b, cnt + z, kFollow, level, cnt + 3);
      }
    }
    int64_t counts[4] = {0, 0, 0, 0};  // list counts, last level with entries
    hipError_t e = hipMemcpyAsync(counts, cnt, sizeof counts,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((st = hip_check(ctx, e, "Lebesgue covering level"))) return st;
    if (counts[level % 3] == 0) {
      if (first_prop >= 0) {
        const int64_t need =
            counts[3] >= first_prop ? counts[3] - first_prop + 1 : 0;
        bool found = false;
        for (size_t i = 0; i < ctx->leb_keys.size(); ++i)
          if (ctx->leb_keys[i] == key) {
            ctx->leb_levels[i] = need;
            found = true;
          }
        if (!found) {
          if (ctx->leb_keys.size() >= 4096) {
            ctx->leb_keys.clear();
            ctx->leb_levels.clear();
          }
          ctx->leb_keys.push_back(key);
          ctx->leb_levels.push_back(need);
        }
      }
      break;
    }
    if (level > N + 2)
      return fail(ctx, ORBF_EINTERNAL, "Lebesgue covering did not settle");
    if (solving) {
      // the DAG is deep: solve the next level's centers and every node
      // still undecided now, then settle the rest without solves
      const int a = (int)(level % 3), z = (a + 2) % 3;
      if ((st = solve(list[a], cnt + a))) return st;
      hipLaunchKernelGGL(lzero1_kernel, dim3(1), dim3(64), 0, s, cnt + z);
      hipLaunchKernelGGL(lspec_kernel, dim3(g), dim3(256), 0, s, state,
                         owner, ball, N, list[z], cnt + z);
      if ((st = solve(list[z], cnt + z))) return st;
      hipLaunchKernelGGL(lzero1_kernel, dim3(1), dim3(64), 0, s, cnt + z);
      solving = false;
      first_prop = level;
      // the recorded depth plus two (a group that follows its own decisions
      // can move the depth by a level or so between calls); if that falls
      // short, the doubling starts again from one
      from_record = recorded > 0 && recorded < N;
      batch = from_record ? (int)recorded + 2 : 1;
      continue;
    }
    batch = from_record ? 1 : batch < 64 ? 2 * batch : 64;
    from_record = false;
  }
  hipLaunchKernelGGL(lfinal_kernel, dim3(g), dim3(256), 0, s, state, N, owner,
                     flag, ctx->status);
  if ((st = exclusive_scan_i32_to_i64(ctx, flag, N, pos))) return st;
  hipLaunchKernelGGL(lcompact_kernel, dim3(g1), dim3(256), 0, s, flag, pos, N,
                     centers, n_centers);
  return hip_check(ctx, hipGetLastError(), "Lebesgue covering");
}

}  // namespace orbf
