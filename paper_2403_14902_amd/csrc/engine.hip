// Round driver of the gfx950 engine: sessions, weight packing, the adaptive router, queue
// multi-split, result materialisation, and the C ABI declared in include/hydro.h.
//
// A push of n tuples is evaluated in rounds.  Every round:
//   1. fold: the previous round's per-predicate counts and device time are folded into
//      running selectivity / cost estimates and the predicates are ranked by the policy
//      (section 4.1: score = cost / (1 - selectivity); cost alone; selectivity alone; or the
//      written order);
//   2. route: every live tuple (survivors of earlier rounds plus a newly admitted wave) goes to
//      the first predicate in that ranking it has not visited yet (the visited table of
//      section 3.3 is a per-tuple bit mask) and is appended to that predicate's queue with
//      one atomic per wave per predicate;
//   3. evaluate: one grouped launch per arithmetic tier evaluates every queue; a tuple whose
//      margin lies within tau of its threshold is deferred to the next tier (BF16 -> FP32 ->
//      FP64); decided tuples are forwarded: failures are dropped at once (section 3.3, eager
//      materialisation), survivors join the next round's live list, and tuples that passed
//      every predicate set their bit in the result bitmap.
// The number of rounds of a push is fixed by n alone (every live tuple is evaluated once per
// round, so a tuple admitted in round r is done by round r + K - 1); the host therefore
// enqueues the whole push without waiting on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"
#include "router_nn.h"

using namespace hydro;

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(_e == hipErrorOutOfMemory ? HYDRO_ENOMEM : HYDRO_EDEVICE,                  \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                        \
  } while (0)

// Optional allocation-failure injection for tests of the error paths: the n-th device
// allocation after session start fails when HYDRO_FAULT_ALLOC_AFTER=n is set.
static int g_alloc_counter = 0;
static hipError_t dev_alloc(void** p, size_t bytes) {
  const char* s = getenv("HYDRO_FAULT_ALLOC_AFTER");
  if (s != nullptr && *s) {
    int lim = atoi(s);
    if (g_alloc_counter++ >= lim) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  if (bytes == 0) bytes = 16;
  return hipMalloc(p, bytes);
}

// ---------------------------------------------------------------- allocation-free arena
// hydro_query_noalloc places all of a query's device state (packed weights, queues, live lists,
// statistics, result buffers) in this array instead of allocating it: one copy per GPU, held
// until the process ends.  In host code `scratch` is only a stand-in for the symbol: its device
// address (per device) comes from hipGetSymbolAddress and is the only form passed to kernels and
// copies.
static __device__ __align__(256) unsigned char scratch[HYDRO_NOALLOC_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch` (resolved once per device).
static int scratch_ptr(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return fail(HYDRO_EUNSUPPORTED, "device ordinal above 63");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(HYDRO_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return HYDRO_OK;
}

// ---------------------------------------------------------------- round kernels
struct FoldArgs {
  DevState* st;
  int k;
  int route;
  int order[kMaxK];
  double alpha;
  int static_cost;
  double flops[kMaxK];
  int out_slot;         // pend_count slot that receives this round's survivors
  int final_fold;       // 1: only fold counts (after the last round)
  hydro_round_record* rlog;   // debug: one record per round (nullptr: not recorded)
  int rlog_cap;
};

__global__ void k_fold(FoldArgs a) {
  DevState* st = a.st;
  const int k = threadIdx.x;
  const int rec = st->rounds;   // this round's number (read before thread 0 advances it)
  hydro_round_record* rr = (a.rlog != nullptr && !a.final_fold && rec < a.rlog_cap) ? a.rlog + rec : nullptr;
  if (k < a.k) {
    unsigned long long e = st->r_eval[k], p = st->r_pass[k], tk = st->r_ticks[k];
    st->t_eval[k] += e;
    st->t_pass[k] += p;
    st->t_ticks[k] += tk;
    st->t_rescored[k] += st->r_rescored[k];
    st->t_esc[k] += st->r_esc[k];
    st->t_mid[k] += st->r_mid[k];
    st->t_hit[k] += st->r_hit[k];
    st->r_hit[k] = 0;
    if (e > 0) {
      // running estimates; the +1/+2 prior keeps the selectivity off 0 and 1
      double s_obs = ((double)p + 1.0) / ((double)e + 2.0);
      double c_obs = a.static_cost ? a.flops[k] : (double)tk / (double)e;
      if (!st->seen[k]) {
        st->sel_est[k] = s_obs;
        st->cost_est[k] = c_obs;
        st->seen[k] = 1;
      } else {
        st->sel_est[k] = (1.0 - a.alpha) * st->sel_est[k] + a.alpha * s_obs;
        st->cost_est[k] = (1.0 - a.alpha) * st->cost_est[k] + a.alpha * c_obs;
      }
    }
    st->r_eval[k] = st->r_pass[k] = st->r_ticks[k] = st->r_rescored[k] = st->r_esc[k] = st->r_mid[k] = 0;
    st->qcount[k] = st->bcount[k] = st->ecount[k] = st->mcount[k] = 0;
    if (rr != nullptr) {
      rr->folded_evaluated[k] = e;
      rr->folded_passed[k] = p;
      rr->selectivity[k] = st->sel_est[k];
      rr->cost[k] = st->cost_est[k];
    }
  }
  __syncthreads();
  if (k == 0 && !a.final_fold) {
    st->pend_count[a.out_slot] = 0;
    st->rounds += 1;
    double key[kMaxK];
    for (int j = 0; j < a.k; ++j) {
      double s = st->sel_est[j], c = st->cost_est[j];
      if (!st->seen[j]) key[j] = -1.0;  // unseen predicates first (gathers statistics)
      else if (a.route == HYDRO_ROUTE_SEL) key[j] = s;
      else if (a.route == HYDRO_ROUTE_COST) key[j] = c;
      else key[j] = c / (1.0 - s);      // SCORE (and the LEARNED router's fallback)
    }
    if (a.route == HYDRO_ROUTE_FIXED) {
      for (int j = 0; j < a.k; ++j) st->order[j] = a.order[j];
    } else {
      bool used[kMaxK] = {false};
      for (int r = 0; r < a.k; ++r) {
        int best = -1;
        for (int j = 0; j < a.k; ++j)
          if (!used[j] && (best < 0 || key[j] < key[best])) best = j;
        used[best] = true;
        st->order[r] = best;
      }
    }
    if (rr != nullptr) {
      uint32_t seen = 0;
      for (int j = 0; j < a.k; ++j) {
        rr->order[j] = st->order[j];
        seen |= st->seen[j] ? 1u << j : 0u;
      }
      rr->seen_mask = seen;
    }
  }
}

struct RouteArgs {
  DevState* st;
  const uint32_t* pend_in;
  int in_slot;
  uint32_t adm_lo, adm_hi;
  int warmup;
  int routing_batch;
  int k;
  Queues q;
  const float* learned_keys;   // LEARNED: per-tuple keys [idx][K] (nullptr otherwise)
  const uint32_t* key_stamps;  // LEARNED: round in which each tuple's keys were computed
  OutcomeLog olog;             // LEARNED: arm assignment of routing batches
  int min_steps;               // LEARNED: optimiser steps before the learned arm uses the keys
  Forward fw;                  // result reuse: cache, thresholds, result bits and route log
  int route;                   // result reuse: the policy (for the per-batch ranking)
  int reuse_aware;             // rank each batch of 64 by (1 - cache hit rate) x cost
};

// Result reuse (policy.reuse > 0): the tuple's cached decisions are looked up for its unvisited
// predicates; the batch of 64 tuples routed together (one wave) is ranked with the reuse-aware
// cost estimate of section 4.3, (1 - hit rate of the batch) x cost (SCORE and COST), else with
// the round's ranking; the tuple then walks that ranking, taking cached decisions (a cached pass
// marks the predicate visited, a cached fail drops the tuple) until it reaches a predicate without
// one, whose queue it joins, or passes every predicate.  Returns the predicate (-1: finished) and
// the entry with its visited mask updated; *cached gets the predicates decided from the cache.
__device__ inline int route_with_cache(const RouteArgs& a, bool active, uint32_t* e, const int* order,
                                       const double* sel, const double* cost, const int* seen, uint32_t* cached) {
  const uint32_t idx = entry_idx(*e);
  uint32_t m = entry_mask(*e);
  uint32_t hit = 0, hpass = 0;
  if (active)
    for (int j = 0; j < a.k; ++j)
      if (!((m >> j) & 1u)) {
        const int r = cache_get(a.fw.cache, j, (unsigned long long)(a.fw.id_base + idx), theta_of(a.fw, j, idx));
        hit |= (r != 0 ? 1u : 0u) << j;
        hpass |= (r == 1 ? 1u : 0u) << j;
      }
  int ord[kMaxK];
  if (a.reuse_aware) {
    double key[kMaxK];
    for (int j = 0; j < a.k; ++j) {
      const int cand = __popcll(__ballot(active && !((m >> j) & 1u)));
      const int h = __popcll(__ballot((hit >> j) & 1u));
      const double rate = cand > 0 ? (double)h / (double)cand : 0.0;
      const double est = (1.0 - rate) * cost[j];          // reuse-aware cost estimate
      key[j] = !seen[j] ? -1.0 : a.route == HYDRO_ROUTE_COST ? est : est / (1.0 - sel[j]);
    }
    uint32_t used = 0;
    for (int r = 0; r < a.k; ++r) {
      int best = -1;
      for (int j = 0; j < a.k; ++j)
        if (!((used >> j) & 1u) && (best < 0 || key[j] < key[best])) best = j;
      used |= 1u << best;
      ord[r] = best;
    }
  } else {
    for (int r = 0; r < a.k; ++r) ord[r] = order[r];
  }
  *cached = 0;
  if (!active) return -1;
  const int first = (a.warmup && m == 0) ? (int)((idx / (uint32_t)a.routing_batch) % (uint32_t)a.k) : -1;
  for (int r = -1; r < a.k; ++r) {
    const int j = r < 0 ? first : ord[r];
    if (j < 0 || ((m >> j) & 1u)) continue;
    if (!((hit >> j) & 1u)) {
      *e = make_entry(idx, m);
      return j;
    }
    *cached |= 1u << j;
    if (a.fw.route_log != nullptr) a.fw.route_log[idx] |= (uint32_t)(j + 1) << (4 * __popc(m));
    if (!((hpass >> j) & 1u)) return -1;                   // cached fail: dropped
    m |= 1u << j;
  }
  atomicOr(&a.fw.result_bits[idx >> 5], 1u << (idx & 31));   // every predicate passed
  return -1;
}

// The tuple belongs to the learned arm and the router is active (keys may still be missing).
__device__ inline bool learned_eligible(const RouteArgs& a, uint32_t e) {
  return a.learned_keys != nullptr && !(a.warmup && entry_mask(e) == 0) && a.st->learned_active &&
         a.st->train_steps >= a.min_steps &&
         arm_of(entry_idx(e) / (uint32_t)a.routing_batch, a.olog.seed, a.olog.control_below) == 1;
}
// ... and its keys were computed in this round (DevState::rounds is this round's stamp).
__device__ inline bool learned_arm(const RouteArgs& a, uint32_t e) {
  return learned_eligible(a, e) && a.key_stamps[entry_idx(e)] == (uint32_t)a.st->rounds;
}

__device__ inline int choose_pred(const RouteArgs& a, uint32_t e, const int* order) {
  uint32_t mask = entry_mask(e);
  uint32_t idx = entry_idx(e);
  if (a.warmup && mask == 0) return (int)((idx / (uint32_t)a.routing_batch) % (uint32_t)a.k);
  if (learned_arm(a, e)) {
    const float* kk = a.learned_keys + (int64_t)idx * a.k;
    int best = -1;
    float bk = 0.f;
    for (int j = 0; j < a.k; ++j)
      if (!((mask >> j) & 1u) && (best < 0 || kk[j] < bk)) { best = j; bk = kk[j]; }
    return best;
  }
  for (int r = 0; r < a.k; ++r) {
    int j = order[r];
    if (!((mask >> j) & 1u)) return j;
  }
  return 0;
}

// Multi-split in chunks of kRouteItems entries per thread: each wave counts its entries per
// predicate with ballots, the workgroup reserves one range per predicate with a single atomic,
// and every entry is written to its slot (one atomic per predicate per 2,048 entries instead of
// one per wave).  (A variant that gave each workgroup one contiguous range and one atomic per
// predicate per round, with a second pass to write, measured slower: its longer dependent chains
// cost more than the atomics it saved.)
constexpr int kRouteThreads = 256, kRouteItems = 8, kRouteChunk = kRouteThreads * kRouteItems;
// Workgroups per CU: the register count allows 4 waves per SIMD, i.e. 4 workgroups; fewer leave
// each chunk's reservation round trip exposed (2 per CU: 17 % slower at 2^22-tuple waves), and
// halving the chunk (4 entries per thread, 8 workgroups per CU) nearly doubled the time.
constexpr int kRouteBlocksPerCu = 4;

__global__ __launch_bounds__(kRouteThreads) void k_route(RouteArgs a) {
  __shared__ int order[kMaxK];
  __shared__ int wslot[kRouteThreads / kWave][kMaxK];   // per wave: entries, then first slot
  __shared__ double sel_s[kMaxK], cost_s[kMaxK];
  __shared__ int seen_s[kMaxK];
  if (threadIdx.x < a.k) {
    order[threadIdx.x] = a.st->order[threadIdx.x];
    sel_s[threadIdx.x] = a.st->sel_est[threadIdx.x];
    cost_s[threadIdx.x] = a.st->cost_est[threadIdx.x];
    seen_s[threadIdx.x] = a.st->seen[threadIdx.x];
  }
  __syncthreads();
  const bool reuse = a.fw.cache.keys != nullptr;
  unsigned long long hits[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) hits[j] = 0;
  const int n_in = a.st->pend_count[a.in_slot];
  const int64_t total = n_in + (int64_t)(a.adm_hi - a.adm_lo);
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  uint32_t n_learned = 0, n_stats = 0, n_stale = 0;
  for (int64_t base = (int64_t)blockIdx.x * kRouteChunk; base < total; base += (int64_t)gridDim.x * kRouteChunk) {
    uint32_t e[kRouteItems];
    int kk[kRouteItems], off[kRouteItems];
#pragma unroll
    for (int r = 0; r < kRouteItems; ++r) {
      const int64_t i = base + r * kRouteThreads + threadIdx.x;
      e[r] = 0u;
      kk[r] = -1;
      if (reuse) {
        if (i < total) e[r] = i < n_in ? a.pend_in[i] : make_entry(a.adm_lo + (uint32_t)(i - n_in), 0u);
        uint32_t cached;
        kk[r] = route_with_cache(a, i < total, &e[r], order, sel_s, cost_s, seen_s, &cached);
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) hits[j] += __popcll(__ballot((cached >> j) & 1u));
        continue;
      }
      if (i < total) {
        e[r] = i < n_in ? a.pend_in[i] : make_entry(a.adm_lo + (uint32_t)(i - n_in), 0u);
        kk[r] = choose_pred(a, e[r], order);
        if (a.learned_keys != nullptr) {
          const bool eligible = learned_eligible(a, e[r]);
          const bool learned = eligible && learned_arm(a, e[r]);
          const bool fresh = entry_mask(e[r]) == 0;     // the tuple's first routing
          n_learned += learned && fresh;
          n_stats += !learned && fresh;
          n_stale += eligible && !learned;
        }
      }
    }
    // wave totals per predicate and each entry's offset within its wave's range
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
      if (j >= a.k) break;
      int run = 0;
#pragma unroll
      for (int r = 0; r < kRouteItems; ++r) {
        const unsigned long long m = __ballot(kk[r] == j);
        if (kk[r] == j) off[r] = run + __popcll(m & below);
        run += __popcll(m);
      }
      if (lane == 0) wslot[wv][j] = run;
    }
    __syncthreads();
    if (threadIdx.x < a.k) {
      const int j = threadIdx.x;
      int sum = 0;
      for (int w = 0; w < kRouteThreads / kWave; ++w) sum += wslot[w][j];
      int p = sum ? atomicAdd(&a.q.counts[j], sum) : 0;
      for (int w = 0; w < kRouteThreads / kWave; ++w) {
        const int c = wslot[w][j];
        wslot[w][j] = p;
        p += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRouteItems; ++r)
      if (kk[r] >= 0) a.q.entries[(int64_t)kk[r] * a.q.cap + wslot[wv][kk[r]] + off[r]] = e[r];
    __syncthreads();   // wslot is rewritten by the next chunk
  }
  if (reuse && lane_id() == 0)
    for (int j = 0; j < a.k; ++j)
      if (hits[j]) atomicAdd(&a.st->r_hit[j], hits[j]);
  if (a.learned_keys != nullptr) {
    unsigned long long c[3] = {n_learned, n_stats, n_stale};
#pragma unroll
    for (int t = 0; t < 3; ++t)
      for (int o = 32; o > 0; o >>= 1) c[t] += __shfl_xor(c[t], o);
    if (lane == 0) {
      if (c[0]) atomicAdd(&a.st->learned_routed, c[0]);
      if (c[1]) atomicAdd(&a.st->stats_routed, c[1]);
      if (c[2]) atomicAdd(&a.st->learned_stale, c[2]);
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Result bitmap -> ascending int64 ids (ordered compaction, three passes).
__global__ __launch_bounds__(256) void k_res_count(const uint32_t* bits, int64_t nwords, int* block_counts) {
  __shared__ int red[256];
  int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  red[threadIdx.x] = w < nwords ? __popc(bits[w]) : 0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_counts[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_res_scan(int* block_counts, int nblocks, DevState* st, int* base_out) {
  __shared__ int sums[1024];
  const int t = threadIdx.x;
  const int per = (nblocks + 1023) / 1024;
  int lo = t * per, hi = min(nblocks, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += block_counts[i];
  sums[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int v = t >= o ? sums[t - o] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int base = st->n_result;
  int run = base + (t > 0 ? sums[t - 1] : 0);
  for (int i = lo; i < hi; ++i) {
    int c = block_counts[i];
    block_counts[i] = run;
    run += c;
  }
  __syncthreads();
  if (t == 0) {
    *base_out = base;
    st->n_result = base + sums[1023];
  }
}

__global__ __launch_bounds__(256) void k_res_write(const uint32_t* bits, int64_t nwords, const int* block_offsets,
                                                   int64_t id_base, int64_t* out) {
  __shared__ int pre[256];
  int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t b = w < nwords ? bits[w] : 0u;
  pre[threadIdx.x] = __popc(b);
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int v = threadIdx.x >= o ? pre[threadIdx.x - o] : 0;
    __syncthreads();
    pre[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = block_offsets[blockIdx.x] + pre[threadIdx.x] - __popc(b);
  while (b) {
    int bit = __ffs(b) - 1;
    out[pos++] = id_base + w * 32 + bit;
    b &= b - 1;
  }
}

// Stand-in for the inference tiers in the standalone compaction run (hydro_compaction_debug):
// predicate j's decision on the tuple with global index t is bit t of row j of a caller bitmap.
// Forwarding as in forward_decision (failures dropped, survivors with predicates left appended to
// the next live list with their visited bit set, completed tuples set in the result bitmap), but
// aggregated like k_route: kRouteItems entries per thread, one atomic per workgroup chunk for the
// survivor list, one per wave and distinct bitmap word for the result bits, and the counters
// summed per wave over the whole launch.
__global__ __launch_bounds__(kRouteThreads) void k_table_decide(Queues q, int k, const uint32_t* bits,
                                                                int64_t row_words, Forward f) {
  __shared__ int wslot[kRouteThreads / kWave];
  __shared__ unsigned long long cnt_s[2][kMaxK];     // evaluations and passes of this workgroup
  __shared__ int chunks_s[kMaxK + 1];                // prefix of the per-predicate chunk counts
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  if (threadIdx.x < 2 * kMaxK) cnt_s[threadIdx.x / kMaxK][threadIdx.x % kMaxK] = 0;
  if (threadIdx.x == 0) {
    chunks_s[0] = 0;
    for (int j = 0; j < k; ++j) chunks_s[j + 1] = chunks_s[j] + (q.counts[j] + kRouteChunk - 1) / kRouteChunk;
  }
  __syncthreads();
  // the chunks of every predicate form one index space: all predicates' queues are drained at once
  for (int ch = blockIdx.x; ch < chunks_s[k]; ch += gridDim.x) {
    int j = 0;
    while (ch >= chunks_s[j + 1]) ++j;
    const int c = q.counts[j];
    const int64_t base = (int64_t)(ch - chunks_s[j]) * kRouteChunk;
    uint32_t e[kRouteItems];
    bool more[kRouteItems];
    int off[kRouteItems];
    int run = 0, n_eval = 0, n_pass = 0;
#pragma unroll
    for (int r = 0; r < kRouteItems; ++r) {
      const int64_t i = base + r * kRouteThreads + threadIdx.x;
      e[r] = i < c ? q.entries[(int64_t)j * q.cap + i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRouteItems; ++r) {
      const int64_t i = base + r * kRouteThreads + threadIdx.x;
      const bool active = i < c;
      const uint32_t idx = entry_idx(e[r]);
      const int64_t t = f.id_base + idx;
      const bool pass = active && ((bits[(int64_t)j * row_words + (t >> 5)] >> (t & 31)) & 1u);
      n_eval += active;
      n_pass += pass;
      const uint32_t mask = entry_mask(e[r]) | (1u << j);
      const bool done = pass && mask == f.full_mask;
      more[r] = pass && !done;
      // result bits: one atomic per distinct word among the wave's completed tuples
      const uint32_t word = idx >> 5;
      unsigned long long dm = __ballot(done);
      while (dm) {
        const int leader = __ffsll((long long)dm) - 1;
        const uint32_t w = __shfl(word, leader);
        const bool same = done && word == w;
        uint32_t v = same ? 1u << (idx & 31) : 0u;
        for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
        if (lane == leader) atomicOr(&f.result_bits[w], v);
        dm &= ~__ballot(same);
      }
      const unsigned long long m = __ballot(more[r]);
      if (more[r]) off[r] = run + __popcll(m & below);
      run += __popcll(m);
    }
    for (int o = 32; o > 0; o >>= 1) {
      n_eval += __shfl_xor(n_eval, o);
      n_pass += __shfl_xor(n_pass, o);
    }
    if (lane == 0) {
      wslot[wv] = run;
      atomicAdd(&cnt_s[0][j], (unsigned long long)n_eval);
      atomicAdd(&cnt_s[1][j], (unsigned long long)n_pass);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int sum = 0;
      for (int w = 0; w < kRouteThreads / kWave; ++w) sum += wslot[w];
      int p = sum ? atomicAdd(f.pend_out_count, sum) : 0;
      for (int w = 0; w < kRouteThreads / kWave; ++w) {
        const int cw = wslot[w];
        wslot[w] = p;
        p += cw;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRouteItems; ++r)
      if (more[r]) f.pend_out[wslot[wv] + off[r]] = make_entry(entry_idx(e[r]), entry_mask(e[r]) | (1u << j));
    __syncthreads();
  }
  if (threadIdx.x < k) {
    if (cnt_s[0][threadIdx.x]) atomicAdd(&f.st->r_eval[threadIdx.x], cnt_s[0][threadIdx.x]);
    if (cnt_s[1][threadIdx.x]) atomicAdd(&f.st->r_pass[threadIdx.x], cnt_s[1][threadIdx.x]);
  }
}

// Decisions of a HOST predicate (taken on the CPU for the round's queue entries, dec[i] for entry
// i) forwarded like any tier's; the CPU threads' time of the round is added to its cost.
__global__ __launch_bounds__(256) void k_apply_host(Queues q, int k, const uint8_t* dec, Forward f,
                                                    unsigned long long ticks) {
  const int c = q.counts[k];
  if (blockIdx.x == 0 && threadIdx.x == 0 && ticks) atomicAdd(&f.st->r_ticks[k], ticks);
  for (int base = blockIdx.x * blockDim.x; base < c; base += gridDim.x * blockDim.x) {
    const int i = base + threadIdx.x;
    const bool active = i < c;
    const uint32_t e = active ? q.entries[(int64_t)k * q.cap + i] : 0u;
    forward_decision(f, k, e, active, false, active && dec[i] != 0);
  }
}

// ---------------------------------------------------------------- session
// Escalated (FP64) entries per predicate and round evaluated layer-parallel; more run one per
// block.  HYDRO_ESC_CAP overrides the default (tests use it to exercise the per-block path).
constexpr int kArenaEscCap = 8;      // allocation-free sessions: FP64 layer-parallel entries per slot
constexpr int kArenaRestGrid = 16;   // ... and FP64 fallback blocks

static int esc_cap_setting() {
  const char* e = getenv("HYDRO_ESC_CAP");
  int v = (e && *e) ? atoi(e) : 128;
  return v < 1 ? 1 : v > 4096 ? 4096 : v;
}

struct HostModel {
  hydro_model m;
  std::vector<float> w1, b1, w2, b2, fcw, fcb;
  std::vector<float> cw[HYDRO_MAX_LAYERS], cb[HYDRO_MAX_LAYERS];
  double flops = 0;
  int variant = CNN_NONE;
};

// What a captured push depends on besides device-resident state.
struct GraphKey {
  int64_t n;
  const void* base;
  int64_t id_base;
  int n_seg;
  int64_t seg_len;
  int warm;
  int parity;
  int learned_from;   // first round of the push that runs the learned router's keys
  const void* theta;
  const void* out;
  bool operator==(const GraphKey& o) const {
    return n == o.n && base == o.base && id_base == o.id_base && n_seg == o.n_seg && seg_len == o.seg_len &&
           warm == o.warm && parity == o.parity && learned_from == o.learned_from && theta == o.theta &&
           out == o.out;
  }
};

constexpr int kEvPerRound = 6;               // start, routed, first pass, BF16 mid, FP32, FP64
constexpr float kAutoTauFloor = 0.015f;     // automatic bands never go below these
constexpr float kAutoTau32Floor = 1e-5f;
// the three-product tier drops three products of at most about 2^-16 of |w x| each; its logit
// error is some 16x the FP32 tier's, and its floor 30x the FP32 floor
constexpr float kAutoTauX3Floor = 3e-4f;

// Persistent CPU threads for HOST predicates: run(n, fn) calls fn(t) for t = 0..n-1, the caller
// taking t = 0, and returns when all have finished (no thread is created per round).
struct HostPool {
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::function<void(int)> job;
  uint64_t generation = 0;
  int active = 0, pending = 0;
  bool stop = false;
  void start(int n) {
    for (int t = 1; t < n; ++t)
      threads.emplace_back([this, t] {
        uint64_t seen = 0;
        for (;;) {
          std::function<void(int)> fn;
          {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || generation != seen; });
            if (stop) return;
            seen = generation;
            if (t >= active) continue;
            fn = job;
          }
          fn(t);
          std::lock_guard<std::mutex> lk(mu);
          if (--pending == 0) done_cv.notify_one();
        }
      });
  }
  void run(int n, const std::function<void(int)>& fn) {
    n = std::max(1, std::min<int>(n, (int)threads.size() + 1));
    {
      std::lock_guard<std::mutex> lk(mu);
      job = fn;
      active = n;
      pending = n - 1;
      ++generation;
    }
    cv.notify_all();
    fn(0);
    std::unique_lock<std::mutex> lk(mu);
    done_cv.wait(lk, [&] { return pending == 0; });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto& th : threads) th.join();
  }
};

struct hydro_session {
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr, copy_stream = nullptr;
  bool own_stream = false;
  hydro_policy pol{};
  int K = 0, fh = 0, fw = 0, fdtype = 0;
  int64_t max_push = 0, cap = 0;
  std::vector<HostModel> models;
  std::vector<void*> allocs;
  // device state
  DevState* st = nullptr;
  uint32_t* pend[2] = {nullptr, nullptr};
  uint32_t *q1 = nullptr, *q2 = nullptr, *q3 = nullptr, *qm = nullptr;   // first, FP32, FP64, BF16-mid
  uint32_t* result_bits = nullptr;
  uint32_t* route_log = nullptr;
  hydro_round_record* round_log = nullptr;   // log_routes: per-round rankings and folded counts
  int round_log_cap = 0;
  int* res_blocks = nullptr;
  int* res_base = nullptr;
  int64_t* out_ids = nullptr;
  int64_t out_cap = 0;
  float* theta = nullptr;
  int theta_cap = 0;
  void* stage[2] = {nullptr, nullptr};
  hipEvent_t stage_free[2] = {nullptr, nullptr}, stage_ready[2] = {nullptr, nullptr};
  int stage_next = 0;
  MlpArgs mlp{};
  CnnArgs cnn{};
  GcnnArgs gcnn{};
  RouterNN* rnn = nullptr;
  bool fused_feats = false;   // every predicate is a fused CNN: its first pass writes the router features
  // query progress
  int rounds_done = 0;
  bool warmed = false;
  int parity = 0;
  int pushes = 0;
  bool in_query = false;     // pushes since the last reset / finish
  bool ids_sorted = true;
  int64_t last_id_end = INT64_MIN;
  int64_t last_push_n = 0;
  std::deque<std::vector<float>> theta_host;
  std::chrono::steady_clock::time_point t_start;
  hydro_query_info info{};
  double tick_us = 0.01;   // device wall clock period in microseconds
  std::vector<hipEvent_t> evpool;   // time_kernels: kEvPerRound events per round
  int ev_used = 0;
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;   // use_graph: captured pushes
  float tau_k[kMaxK], tau32_k[kMaxK];   // per-predicate bands (policy values or calibrated)
  float tau16_k[kMaxK];                 // FP8 sessions: band of the BF16 re-score tier
  bool auto_tau = false, auto_tau32 = false;   // bands still to be measured on the first push
  bool auto_tau16 = false;
  bool ascales_set = false;                    // FP8: activation scales measured
  // allocation-free sessions: every device buffer is carved from `arena` (the current device's
  // copy of `scratch`); nothing is allocated or freed
  unsigned char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  int64_t act_cap = 0;   // entries of the layer-wise CNN activation buffers (evaluations per launch)
  ResultCache cache{};   // policy.reuse > 0: decisions kept across the session's queries
  // HOST predicates: evaluated by CPU threads on host-memory frames while the GPU evaluates the
  // other queues of the round; entries copied down, decisions copied up, forwarded on the device
  std::vector<int> host_preds;
  int64_t h_cap = 0;                 // entries per host predicate and round (the live-tuple bound)
  int* h_counts = nullptr;           // pinned: the round's first-pass queue counts [kMaxK]
  uint32_t* h_entries = nullptr;     // pinned: [host predicate][h_cap] queue entries
  uint8_t* h_dec = nullptr;          // pinned: [host predicate][h_cap] decisions
  uint8_t* d_dec = nullptr;          // device copy of h_dec
  hipEvent_t h_routed = nullptr, h_ready = nullptr, h_done = nullptr;
  int host_threads = 1;
  std::unique_ptr<HostPool> pool;
  // CNN predicates on each tuple's crop (variable-size inputs)
  CropArgs crop{};
  std::vector<int> crop_preds;
  int32_t* crops_dev = nullptr;                 // the push's crops [max_push][4]
  std::deque<std::vector<int32_t>> crops_host;  // host copies until finish (async copies read them)
  int crop_grid = 0;
};

// Captured pushes bake the bands (and every other launch argument) into their kernel nodes.
static void drop_graphs(hydro_session* s) {
  for (auto& g : s->graphs) hipGraphExecDestroy(g.second);
  s->graphs.clear();
}

static hipEvent_t next_event(hydro_session* s) {
  if (s->ev_used == (int)s->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->evpool.push_back(e);
  }
  return s->evpool[s->ev_used++];
}

static int sess_alloc(hydro_session* s, void** p, size_t bytes) {
  if (s->arena) {
    const size_t off = (s->arena_used + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 16;
    if (off > s->arena_cap || bytes > s->arena_cap - off) {
      *p = nullptr;
      return fail(HYDRO_ECAPACITY, "the query needs more than the " + std::to_string(s->arena_cap) +
                                       " bytes of the allocation-free device arena");
    }
    *p = s->arena + off;
    s->arena_used = off + bytes;
    return HYDRO_OK;
  }
  hipError_t e = dev_alloc(p, bytes);
  if (e != hipSuccess) return fail(HYDRO_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) + " bytes failed");
  s->allocs.push_back(*p);
  return HYDRO_OK;
}

template <typename T>
static int upload(hydro_session* s, const T* host, size_t n, T** dev) {
  int rc = sess_alloc(s, (void**)dev, n * sizeof(T));
  if (rc) return rc;
  HIP_TRY(hipMemcpy(*dev, host, n * sizeof(T), hipMemcpyHostToDevice));
  return HYDRO_OK;
}

static uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static float bf16_bits_to_f32(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

static double model_flops(const hydro_model& m) {
  if (m.arch == HYDRO_ARCH_HOST) {                               // six comparisons per sampled pixel
    const int st = m.color_stride > 1 ? m.color_stride : 1;
    return 6.0 * ((m.in_h + st - 1) / st) * ((m.in_w + st - 1) / st);
  }
  if (m.arch == HYDRO_ARCH_MLP) {
    double d = (double)m.in_h * m.in_w * 3;
    return 2.0 * (d * m.hidden + (double)m.hidden * kClasses);
  }
  double f = 0;
  int hw = m.in_h, cin = 3;
  for (int l = 0; l < m.n_layers; ++l) {
    hw /= 2;
    f += 2.0 * hw * hw * m.widths[l] * cin * 9;
    cin = m.widths[l];
  }
  return f + 2.0 * cin * kClasses;
}

static int validate_model(const hydro_model& m, int fh, int fw) {
  if (m.in_h != fh || m.in_w != fw) return fail(HYDRO_EINVAL, "model input shape differs from the session's frame shape");
  if (m.class_mask >= (1u << kClasses)) return fail(HYDRO_EINVAL, "class_mask has bits above class 9");
  if (m.arch == HYDRO_ARCH_HOST) {
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(m.color_lo[c]) || !std::isfinite(m.color_hi[c]) || m.color_lo[c] > m.color_hi[c])
        return fail(HYDRO_EINVAL, "HOST predicate: color_lo / color_hi must be finite with lo <= hi");
    if (m.color_stride < 0 || m.color_stride > m.in_h || m.color_stride > m.in_w)
      return fail(HYDRO_EINVAL, "HOST predicate: color_stride must be in 0 .. frame side");
    return HYDRO_OK;
  }
  if (m.arch == HYDRO_ARCH_MLP) {
    if (!m.w1 || !m.b1 || !m.w2 || !m.b2) return fail(HYDRO_EINVAL, "MLP weight pointer is NULL");
    if (m.hidden <= 0 || m.hidden % 128 != 0 || m.hidden > 2048)
      return fail(HYDRO_EUNSUPPORTED, "MLP hidden width must be a multiple of 128 and at most 2048");
    int64_t d = (int64_t)fh * fw * 3;
    if (d % 32 != 0) return fail(HYDRO_EUNSUPPORTED, "MLP input size must be a multiple of 32");
    return HYDRO_OK;
  }
  if (m.arch != HYDRO_ARCH_CNN) return fail(HYDRO_EINVAL, "unknown model arch");
  if (m.n_layers < 1 || m.n_layers > HYDRO_MAX_LAYERS) return fail(HYDRO_EINVAL, "CNN n_layers out of range");
  for (int l = 0; l < m.n_layers; ++l)
    if (!m.conv_w[l] || !m.conv_b[l]) return fail(HYDRO_EINVAL, "CNN conv weight pointer is NULL");
  if (!m.fc_w || !m.fc_b) return fail(HYDRO_EINVAL, "CNN fc weight pointer is NULL");
  if (m.on_crop) {      // variable-size inputs: any crop of the frame, FP64 kernel
    for (int l = 0; l < m.n_layers; ++l)
      if (m.widths[l] < 1 || m.widths[l] > 256) return fail(HYDRO_EUNSUPPORTED, "on_crop CNN widths must be 1..256");
    return HYDRO_OK;
  }
  if (m.in_w != m.in_h) return fail(HYDRO_EUNSUPPORTED, "CNN frames must be square");
  if (cnn_variant_of(m.in_h, m.n_layers, m.widths) != CNN_NONE) return HYDRO_OK;   // fused kernel
  // generic layer-wise path
  if (m.in_h % (1 << m.n_layers) != 0 || (m.in_h >> m.n_layers) < 1)
    return fail(HYDRO_EUNSUPPORTED, "CNN input side must be divisible by 2^n_layers");
  for (int l = 0; l < m.n_layers; ++l)
    if (m.widths[l] < 16 || m.widths[l] % 16 != 0 || m.widths[l] > 1024)
      return fail(HYDRO_EUNSUPPORTED, "CNN widths must be multiples of 16 (at most 1024)");
  return HYDRO_OK;
}

// Weight forms of the dedicated 4-layer CNN kernels for gcnn slot i: layer-1/2 register fragments
// and layer-3/4 A tile images per tier, and the FP8 tier's per-output-channel weight scales
// (largest |w| of the channel maps to 448, the largest finite e4m3 value).
static int pack_c4(hydro_session* s, const HostModel& hm, float scale1, int i) {
  GcnnArgs& ga = s->gcnn;
  int rc;
  std::vector<float> sc[3];
  for (int l = 1; l < 4; ++l) {
    const int co = hm.m.widths[l], cin = hm.m.widths[l - 1];
    sc[l - 1].resize(co);
    for (int o = 0; o < co; ++o) {
      double mx = 0;
      for (int t = 0; t < cin * 9; ++t) mx = std::max(mx, (double)std::fabs(hm.cw[l][(size_t)o * cin * 9 + t]));
      sc[l - 1][o] = mx > 0 ? (float)(mx / 448.0) : 1.f;
    }
    float* dp;
    if ((rc = upload(s, sc[l - 1].data(), sc[l - 1].size(), &dp))) return rc;
    ga.c4_wscale[i][l - 1] = dp;
  }
  C4FrontPack fp;
  c4_pack_front(hm.cw[0].data(), scale1, hm.cw[1].data(), sc[0].data(), &fp);
  {
    std::vector<uint16_t> b(fp.w1b.size());
    for (size_t t = 0; t < b.size(); ++t) b[t] = f32_to_bf16_bits(fp.w1b[t]);
    uint16_t* bp;
    if ((rc = upload(s, b.data(), b.size(), &bp))) return rc;
    ga.c4_w1b[i] = bp;
    float* dp;
    uint16_t* tp;
    if ((rc = upload(s, fp.w1s3.data(), fp.w1s3.size(), &tp))) return rc;
    ga.c4_w1f[i] = tp;
    std::vector<uint16_t> b2(fp.w2b.size());
    for (size_t t = 0; t < b2.size(); ++t) b2[t] = f32_to_bf16_bits(fp.w2b[t]);
    if ((rc = upload(s, b2.data(), b2.size(), &bp))) return rc;
    ga.c4_w2[i][C4_BF16] = bp;
    if ((rc = upload(s, fp.w2f.data(), fp.w2f.size(), &dp))) return rc;
    ga.c4_w2[i][C4_F32] = dp;
    uint8_t* qp;
    if ((rc = upload(s, fp.w2q.data(), fp.w2q.size(), &qp))) return rc;
    ga.c4_w2[i][C4_FP8] = qp;
    uint16_t* sp;
    if ((rc = upload(s, fp.w2s3.data(), fp.w2s3.size(), &sp))) return rc;
    ga.c4_w2[i][C4_S3] = sp;
  }
  for (int l = 2; l < 4; ++l)
    for (int p = 0; p < 4; ++p) {
      std::vector<unsigned char> img(c4_img_bytes(p, l));
      c4_pack_img(p, l, hm.cw[l].data(), sc[l - 1].data(), img.data());
      unsigned char* dp;
      if ((rc = upload(s, img.data(), img.size(), &dp))) return rc;
      ga.c4_img[i][l - 2][p] = dp;
    }
  for (int l = 0; l < 3; ++l) ga.c4_ascale[i][l] = 1.f;   // until calibrated
  return HYDRO_OK;
}

static int pack_models(hydro_session* s) {
  const double scale = s->fdtype == HYDRO_DTYPE_U8 ? 4.0 / 255.0 : 4.0;
  const float pad_raw = s->fdtype == HYDRO_DTYPE_U8 ? 127.5f : 0.5f;
  MlpArgs& ma = s->mlp;
  CnnArgs& ca = s->cnn;
  ma = MlpArgs{};
  s->crop.n_preds = 0;
  ca = CnnArgs{};
  s->gcnn = GcnnArgs{};
  ca.pad_raw = pad_raw;
  // allocation-free sessions keep the FP64 tier's layer-parallel batch and fallback slots small
  const int esc_cap = s->arena ? std::min(esc_cap_setting(), kArenaEscCap) : esc_cap_setting();
  const int rest_grid = s->arena ? kArenaRestGrid : s->n_cu;
  // Layer-wise CNN launches keep per-evaluation activations.  A round's queues hold only live
  // tuples: those admitted in the last K rounds (a tuple is evaluated at most once per round and
  // leaves after K evaluations), so at most K x (largest admission) entries, whatever the push size.
  {
    const int64_t warm = (int64_t)s->pol.warmup_batches * s->K * s->pol.routing_batch;
    s->act_cap = std::min<int64_t>(s->cap, (int64_t)s->K * std::max<int64_t>(s->pol.wave, warm));
  }
  // grouped launches walk their slots in order: most expensive predicates first, so the
  // longest work items start early (longest-processing-time-first)
  std::vector<int> slots_order(s->K);
  for (int k = 0; k < s->K; ++k) slots_order[k] = k;
  std::stable_sort(slots_order.begin(), slots_order.end(),
                   [&](int x, int y) { return s->models[x].flops > s->models[y].flops; });
  for (int k : slots_order) {
    HostModel& hm = s->models[k];
    const hydro_model& m = hm.m;
    if (m.arch == HYDRO_ARCH_HOST) continue;     // evaluated on the CPU (no device weights)
    if (m.arch == HYDRO_ARCH_CNN && m.on_crop) {  // FP64 on each tuple's crop: canonical weights
      CropArgs& cr = s->crop;
      const int i = cr.n_preds++;
      cr.pred[i] = k;
      cr.class_mask[i] = m.class_mask;
      cr.n_layers[i] = m.n_layers;
      int cin = 3, rc;
      for (int l = 0; l < m.n_layers; ++l) {
        const int co = m.widths[l];
        cr.widths[i][l] = co;
        // [tap][ci][co]: the lanes of a wave, which hold consecutive output channels, read
        // consecutive weights
        std::vector<float> wt(hm.cw[l].size());
        for (int o = 0; o < co; ++o)
          for (int c = 0; c < cin; ++c)
            for (int t = 0; t < 9; ++t) wt[((size_t)t * cin + c) * co + o] = hm.cw[l][((size_t)o * cin + c) * 9 + t];
        float* dp;
        if ((rc = upload(s, wt.data(), wt.size(), &dp))) return rc;
        cr.wt[i][l] = dp;
        if ((rc = upload(s, hm.cb[l].data(), hm.cb[l].size(), &dp))) return rc;
        cr.bias[i][l] = dp;
        cin = co;
      }
      float* dp;
      if ((rc = upload(s, hm.fcw.data(), hm.fcw.size(), &dp))) return rc;
      cr.fc_w[i] = dp;
      if ((rc = upload(s, hm.fcb.data(), hm.fcb.size(), &dp))) return rc;
      cr.fc_b[i] = dp;
      continue;
    }
    if (m.arch == HYDRO_ARCH_MLP) {
      const int D = m.in_h * m.in_w * 3, H = m.hidden;
      std::vector<float> wt((size_t)H * D), b1f(H);
      std::vector<uint16_t> wb((size_t)H * D);
      for (int j = 0; j < H; ++j) {
        double colsum = 0;
        for (int d = 0; d < D; ++d) {
          double w = hm.w1[(size_t)d * H + j];
          colsum += w;
          float v = (float)(w * scale);
          wt[(size_t)j * D + d] = v;
          wb[(size_t)j * D + d] = f32_to_bf16_bits(v);
        }
        b1f[j] = (float)((double)hm.b1[j] - 2.0 * colsum);
      }
      int i = ma.n_preds++;
      ma.pred[i] = k;
      ma.d_in[i] = D;
      ma.hidden[i] = H;
      ma.class_mask[i] = m.class_mask;
      int rc;
      float* dp;
      uint16_t* bp;
      if ((rc = upload(s, wt.data(), wt.size(), &dp))) return rc;
      ma.w1_f32[i] = dp;
      if ((rc = upload(s, wb.data(), wb.size(), &bp))) return rc;
      ma.w1_bf[i] = reinterpret_cast<const __bf16*>(bp);
      ma.w1_s3[i] = nullptr;
      if (s->fdtype == HYDRO_DTYPE_BF16 && D % 64 == 0 && H % 128 == 0 && !s->arena) {
        // FP32 arithmetic on bf16 frames from three bf16 weight terms (see mlp_gemm_s3_kernel):
        // hi = bf16(w), mid = bf16(w - hi), lo = bf16(w - hi - mid), each difference exact in fp32
        std::vector<uint16_t> w3((size_t)3 * H * D);
        for (size_t q = 0; q < (size_t)H * D; ++q) {
          const float v = wt[q];
          const uint16_t hi = f32_to_bf16_bits(v);
          const float r1 = v - bf16_bits_to_f32(hi);
          const uint16_t mid = f32_to_bf16_bits(r1);
          const float r2 = r1 - bf16_bits_to_f32(mid);
          w3[q] = hi;
          w3[(size_t)H * D + q] = mid;
          w3[(size_t)2 * H * D + q] = f32_to_bf16_bits(r2);
        }
        if ((rc = upload(s, w3.data(), w3.size(), &bp))) return rc;
        ma.w1_s3[i] = reinterpret_cast<const __bf16*>(bp);
      }
      if ((rc = upload(s, b1f.data(), b1f.size(), &dp))) return rc;
      ma.b1_fold[i] = dp;
      if ((rc = upload(s, hm.w2.data(), hm.w2.size(), &dp))) return rc;
      ma.w2[i] = dp;
      if ((rc = upload(s, hm.b2.data(), hm.b2.size(), &dp))) return rc;
      ma.b2[i] = dp;
      if ((rc = upload(s, hm.w1.data(), hm.w1.size(), &dp))) return rc;
      ma.w1_canon[i] = dp;
      if ((rc = upload(s, hm.b1.data(), hm.b1.size(), &dp))) return rc;
      ma.b1_canon[i] = dp;
      if ((rc = sess_alloc(s, (void**)&ma.partial[i], (size_t)(H / 32) * s->cap * kClasses * sizeof(float)))) return rc;
      if (ma.splitk_ws == nullptr) {
        // split-K workspace shared by the MLP predicates: 1024 tiles of 128 x 128 fp32 (64 MB;
        // 8 MB in allocation-free sessions, which split fewer tiles)
        ma.split_slots = s->arena ? 128 : 1024;
        // HYDRO_SPLITK_BELOW overrides the tile count under which a launch splits K
        const char* sb = getenv("HYDRO_SPLITK_BELOW");
        ma.split_below = (sb && *sb) ? atoi(sb) : s->n_cu / 2;
        ma.split_target = 2 * s->n_cu;
        if ((rc = sess_alloc(s, (void**)&ma.splitk_ws, (size_t)ma.split_slots * 128 * 128 * sizeof(float)))) return rc;
        if ((rc = sess_alloc(s, (void**)&ma.split_cnt, (size_t)ma.split_slots * sizeof(int)))) return rc;
        HIP_TRY(hipMemsetAsync(ma.split_cnt, 0, (size_t)ma.split_slots * sizeof(int), s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
      }
      {
        // HYDRO_MLP_TILE forces one tile configuration (tests exercise each)
        const char* ft = getenv("HYDRO_MLP_TILE");
        int cfg = (ft && *ft) ? atoi(ft) : 0;
        if (cfg < 0 || cfg >= MLP_TILE_CONFIGS) cfg = 0;
        ma.tile_cfg[i] = cfg;
        ma.part_w[i] = mlp_tile_bn(cfg) / 2;
      }
      {
        const int nch = mlp_f64_chunks(D);   // chunking of the FP64 tier's hidden pass
        if ((rc = sess_alloc(s, (void**)&ma.esc_h[i], (size_t)nch * esc_cap * H * sizeof(double)))) return rc;
      }
    } else if (hm.variant == CNN_NONE) {
      GcnnArgs& ga = s->gcnn;
      int i = ga.n_preds++;
      ga.pred[i] = k;
      ga.n_layers[i] = m.n_layers;
      ga.in_hw[i] = m.in_h;
      ga.class_mask[i] = m.class_mask;
      int cin = 3;
      for (int l = 0; l < m.n_layers; ++l) {
        const int co = m.widths[l];
        ga.widths[i][l] = co;
        const double sc = l == 0 ? scale : 1.0;
        std::vector<float> bias(co);
        for (int o = 0; o < co; ++o) {
          double b = hm.cb[l][o];
          if (l == 0) {
            double sum = 0;
            for (int t = 0; t < cin * 9; ++t) sum += hm.cw[l][(size_t)o * cin * 9 + t];
            b -= 2.0 * sum;
          }
          bias[o] = (float)b;
        }
        int rc;
        float* dp;
        uint16_t* bp;
        {
          size_t n = gcnn_packed_elems(l, cin, co, HYDRO_PREC_FP32);
          std::vector<float> pf(n);
          gcnn_pack_layer(l, cin, co, HYDRO_PREC_FP32, hm.cw[l].data(), (float)sc, pf.data());
          if ((rc = upload(s, pf.data(), n, &dp))) return rc;
          ga.w_f32[i][l] = dp;
        }
        {
          size_t n = gcnn_packed_elems(l, cin, co, HYDRO_PREC_BF16);
          std::vector<float> pf(n);
          gcnn_pack_layer(l, cin, co, HYDRO_PREC_BF16, hm.cw[l].data(), (float)sc, pf.data());
          std::vector<uint16_t> pb(n);
          for (size_t t = 0; t < n; ++t) pb[t] = f32_to_bf16_bits(pf[t]);
          if ((rc = upload(s, pb.data(), n, &bp))) return rc;
          ga.w_bf[i][l] = reinterpret_cast<const __bf16*>(bp);
        }
        if ((rc = upload(s, bias.data(), bias.size(), &dp))) return rc;
        ga.bias[i][l] = dp;
        {
          std::vector<float> wt(hm.cw[l].size());
          for (int o = 0; o < co; ++o)
            for (int c = 0; c < cin; ++c)
              for (int t = 0; t < 9; ++t) wt[((size_t)o * 9 + t) * cin + c] = hm.cw[l][((size_t)o * cin + c) * 9 + t];
          if ((rc = upload(s, wt.data(), wt.size(), &dp))) return rc;
          ga.wt_canon[i][l] = dp;
        }
        if ((rc = upload(s, hm.cb[l].data(), hm.cb[l].size(), &dp))) return rc;
        ga.b_canon[i][l] = dp;
        cin = co;
      }
      int rc;
      float* dp;
      if ((rc = upload(s, hm.fcw.data(), hm.fcw.size(), &dp))) return rc;
      ga.fc_w[i] = dp;
      if ((rc = upload(s, hm.fcb.data(), hm.fcb.size(), &dp))) return rc;
      ga.fc_b[i] = dp;
      ga.c4[i] = c4_shape_ok(m.in_h, m.n_layers, m.widths) ? 1 : 0;
      if (ga.c4[i] && (rc = pack_c4(s, hm, (float)scale, i))) return rc;
    } else {
      int i = ca.n_preds++;
      ca.pred[i] = k;
      ca.variant[i] = hm.variant;
      ca.class_mask[i] = m.class_mask;
      int cin = 3;
      for (int l = 0; l < m.n_layers; ++l) {
        const int co = m.widths[l];
        const double sc = l == 0 ? scale : 1.0;
        std::vector<float> bias(co);
        for (int o = 0; o < co; ++o) {
          double b = hm.cb[l][o];
          if (l == 0) {
            double sum = 0;
            for (int t = 0; t < cin * 9; ++t) sum += hm.cw[l][(size_t)o * cin * 9 + t];
            b -= 2.0 * sum;
          }
          bias[o] = (float)b;
        }
        int rc;
        float* dp;
        uint16_t* bp;
        {
          size_t n = cnn_packed_elems(hm.variant, l, HYDRO_PREC_BF16);
          std::vector<float> pf(n);
          cnn_pack_layer(hm.variant, l, HYDRO_PREC_BF16, hm.cw[l].data(), (float)sc, pf.data());
          std::vector<uint16_t> pb(n);
          for (size_t t = 0; t < n; ++t) pb[t] = f32_to_bf16_bits(pf[t]);
          if ((rc = upload(s, pb.data(), n, &bp))) return rc;
          ca.w_bf[i][l] = reinterpret_cast<const __bf16*>(bp);
          // FP32 tier: each packed weight as hi + mid + lo in bf16 (exact for fp32 values), the
          // three images one after the other
          std::vector<uint16_t> p3(3 * n);
          for (size_t t = 0; t < n; ++t) {
            float v = pf[t];
            for (int term = 0; term < 3; ++term) {
              const uint16_t h = f32_to_bf16_bits(v);
              p3[term * n + t] = h;
              v -= bf16_bits_to_f32(h);
            }
          }
          if ((rc = upload(s, p3.data(), 3 * n, &bp))) return rc;
          ca.w_s3[i][l] = reinterpret_cast<const __bf16*>(bp);
        }
        if ((rc = upload(s, bias.data(), bias.size(), &dp))) return rc;
        ca.bias[i][l] = dp;
        if ((rc = upload(s, hm.cw[l].data(), hm.cw[l].size(), &dp))) return rc;
        ca.w_canon[i][l] = dp;
        {
          // [co][3][3][ci]: the FP64 tier's lanes walk the input channels of one tap
          std::vector<float> wt(hm.cw[l].size());
          for (int o = 0; o < co; ++o)
            for (int c = 0; c < cin; ++c)
              for (int t = 0; t < 9; ++t) wt[((size_t)o * 9 + t) * cin + c] = hm.cw[l][((size_t)o * cin + c) * 9 + t];
          if ((rc = upload(s, wt.data(), wt.size(), &dp))) return rc;
          ca.wt_canon[i][l] = dp;
        }
        if ((rc = upload(s, hm.cb[l].data(), hm.cb[l].size(), &dp))) return rc;
        ca.b_canon[i][l] = dp;
        cin = co;
      }
      int rc;
      float* dp;
      if ((rc = upload(s, hm.fcw.data(), hm.fcw.size(), &dp))) return rc;
      ca.fc_w[i] = dp;
      if ((rc = upload(s, hm.fcb.data(), hm.fcb.size(), &dp))) return rc;
      ca.fc_b[i] = dp;
    }
  }
  ma.esc_cap = esc_cap;
  if (s->gcnn.n_preds > 0) {
    GcnnArgs& ga = s->gcnn;
    ga.pad_raw = pad_raw;
    int64_t mx = 0;
    for (int i = 0; i < ga.n_preds; ++i)
      for (int l = 0; l < ga.n_layers[i]; ++l) {
        const int64_t h = ga.in_hw[i] >> (l + 1);
        mx = std::max<int64_t>(mx, h * h * ga.widths[i][l]);
      }
    ga.act_stride = mx;
    int rc;
    bool generic = false, any_c4 = false;
    for (int i = 0; i < ga.n_preds; ++i) {
      generic = generic || !ga.c4[i];
      any_c4 = any_c4 || ga.c4[i];
    }
    ga.act_cap = s->act_cap;
    if (generic)
      for (int b = 0; b < 2; ++b)
        if ((rc = sess_alloc(s, &ga.act[b], (size_t)s->act_cap * mx * sizeof(float)))) return rc;
    if (any_c4) {
      // dedicated kernels: layer-2 and layer-3 outputs of every evaluation of a launch (sized for
      // the FP32 tier), the activation maxima of calibration, and a zero page for padding taps
      if ((rc = sess_alloc(s, &ga.c4_act2, (size_t)s->act_cap * 32 * 32 * 64 * sizeof(float)))) return rc;
      if ((rc = sess_alloc(s, &ga.c4_act3, (size_t)s->act_cap * 16 * 16 * 128 * sizeof(float)))) return rc;
      void* zp;
      if ((rc = sess_alloc(s, &zp, 256))) return rc;
      HIP_TRY(hipMemsetAsync(zp, 0, 256, s->stream));
      HIP_TRY(hipStreamSynchronize(s->stream));
      ga.zero_page = zp;
      ga.c4_act_max = nullptr;
    }
    ga.esc_half = mx;
    ga.esc_stride = 2 * mx;
    ga.esc_cap = std::min(esc_cap, 32);
    for (int i = 0; i < ga.n_preds; ++i)
      if ((rc = sess_alloc(s, (void**)&ga.esc_act[i], (size_t)ga.esc_cap * ga.esc_stride * sizeof(double)))) return rc;
    ga.rest_per_block = 2 * mx;
    ga.rest_grid = rest_grid;
    if ((rc = sess_alloc(s, (void**)&ga.rest_scratch, (size_t)ga.rest_per_block * rest_grid * sizeof(double)))) return rc;
  }
  if (ca.n_preds > 0) {
    // FP64 tier scratch: two activation buffers per block (largest layer output)
    int64_t per = 0;
    for (int i = 0; i < ca.n_preds; ++i) {
      const hydro_model& m = s->models[ca.pred[i]].m;
      int hw = m.in_h;
      for (int l = 0; l < m.n_layers; ++l) {
        hw /= 2;
        per = std::max<int64_t>(per, (int64_t)hw * hw * m.widths[l]);
      }
    }
    ca.scratch64_per_block = 2 * per;
    ca.rest_grid = rest_grid;
    int rc = sess_alloc(s, (void**)&ca.scratch64, (size_t)ca.scratch64_per_block * rest_grid * sizeof(double));
    if (rc) return rc;
    // layer-parallel FP64 tier: per entry, layer-1 output then layer-2 output
    ca.esc_stride = 0;
    for (int i = 0; i < ca.n_preds; ++i) {
      const int m = ca.variant[i] == CNN_W1 ? 1 : ca.variant[i] == CNN_W2 ? 2 : 4;
      ca.esc_stride = std::max<int64_t>(ca.esc_stride, (int64_t)32 * 32 * 16 * m + 16 * 16 * 32 * m);
    }
    ca.esc_cap = esc_cap;
    for (int i = 0; i < ca.n_preds; ++i)
      if ((rc = sess_alloc(s, (void**)&ca.esc_act[i], (size_t)esc_cap * ca.esc_stride * sizeof(double)))) return rc;
  }
  return HYDRO_OK;
}

static void free_session(hydro_session* s) {
  if (!s) return;
  if (s->stream) hipStreamSynchronize(s->stream);
  if (s->copy_stream) hipStreamSynchronize(s->copy_stream);
  if (s->rnn) router_nn_destroy(s->rnn);
  for (void* p : s->allocs) hipFree(p);
  for (int i = 0; i < 2; ++i) {
    if (s->stage[i]) hipFree(s->stage[i]);
    if (s->stage_free[i]) hipEventDestroy(s->stage_free[i]);
    if (s->stage_ready[i]) hipEventDestroy(s->stage_ready[i]);
  }
  if (s->out_ids && !s->arena) hipFree(s->out_ids);
  if (s->h_counts) hipHostFree(s->h_counts);
  if (s->h_entries) hipHostFree(s->h_entries);
  if (s->h_dec) hipHostFree(s->h_dec);
  for (hipEvent_t e : {s->h_routed, s->h_ready, s->h_done})
    if (e) hipEventDestroy(e);
  for (hipEvent_t e : s->evpool) hipEventDestroy(e);
  for (auto& g : s->graphs) hipGraphExecDestroy(g.second);
  if (s->copy_stream) hipStreamDestroy(s->copy_stream);
  if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
  delete s;
}

extern "C" {

const char* hydro_last_error(void) { return g_err.c_str(); }
const char* hydro_version(void) { return "hydro-gfx950 0.1"; }
void hydro_free(void* p) { free(p); }

void hydro_policy_default(hydro_policy* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->route = HYDRO_ROUTE_SCORE;
  for (int i = 0; i < HYDRO_MAX_PREDICATES; ++i) p->order[i] = i;
  p->routing_batch = 64;
  p->wave = 8192;
  p->warmup_batches = 1;
  p->ewma_alpha = 0.5f;
  p->cost_source = HYDRO_COST_MEASURED;
  p->precision = HYDRO_PREC_BF16;
  p->tau = 0.f;      // automatic: calibrated on the first push
  p->tau32 = 0.f;
  p->grouped = 1;
  p->use_graph = 0;
  p->log_routes = 0;
  p->explore = 0.05f;
  p->seed = 4242;
  p->stream = nullptr;
}

static int validate_policy(const hydro_policy* p, int K) {
  if (!p) return fail(HYDRO_EINVAL, "policy is NULL");
  if (p->route < HYDRO_ROUTE_FIXED || p->route > HYDRO_ROUTE_LEARNED) return fail(HYDRO_EINVAL, "unknown route policy");
  if (p->route == HYDRO_ROUTE_FIXED) {
    unsigned seen = 0;
    for (int i = 0; i < K; ++i) {
      int o = p->order[i];
      if (o < 0 || o >= K || (seen >> o) & 1u) return fail(HYDRO_EINVAL, "FIXED order is not a permutation of 0..K-1");
      seen |= 1u << o;
    }
  }
  if (p->routing_batch <= 0) return fail(HYDRO_EINVAL, "routing_batch must be positive");
  if (p->wave <= 0) return fail(HYDRO_EINVAL, "wave must be positive");
  if (p->warmup_batches < 0) return fail(HYDRO_EINVAL, "warmup_batches must be >= 0");
  if (!(p->ewma_alpha > 0.f && p->ewma_alpha <= 1.f)) return fail(HYDRO_EINVAL, "ewma_alpha must be in (0, 1]");
  if (p->precision != HYDRO_PREC_FP32 && p->precision != HYDRO_PREC_BF16 && p->precision != HYDRO_PREC_FP8)
    return fail(HYDRO_EUNSUPPORTED, "precision not supported");
  if (p->cost_source != HYDRO_COST_MEASURED && p->cost_source != HYDRO_COST_STATIC) return fail(HYDRO_EINVAL, "unknown cost_source");
  if (p->explore < 0.f || p->explore > 1.f) return fail(HYDRO_EINVAL, "explore must be in [0, 1]");
  if (p->reuse < 0 || p->reuse > 2) return fail(HYDRO_EINVAL, "reuse must be 0, 1 or 2");
  if (p->reuse && p->route == HYDRO_ROUTE_LEARNED)
    return fail(HYDRO_EUNSUPPORTED, "result reuse is not combined with the learned router");
  if (p->cache_log2 < 0 || p->cache_log2 > 28) return fail(HYDRO_EINVAL, "cache_log2 must be in 0 .. 28");
  if (p->rescore3 != 0 && p->rescore3 != 1) return fail(HYDRO_EINVAL, "rescore3 must be 0 or 1");
  if (p->rescore3 && p->precision != HYDRO_PREC_BF16)
    return fail(HYDRO_EUNSUPPORTED, "the three-product re-score tier follows a BF16 first pass");
  return HYDRO_OK;
}

static int rnn_arena_alloc(void* ctx, void** p, size_t bytes) {
  return sess_alloc(static_cast<hydro_session*>(ctx), p, bytes);
}

// Session creation; with `arena`, every device buffer is carved from it (no allocation, no stream
// or event creation: the work runs on policy->stream, or the null stream when that is NULL).
static int session_create(const hydro_model* models, int32_t k, const hydro_policy* policy, int32_t frame_h,
                          int32_t frame_w, int64_t max_push, unsigned char* arena, size_t arena_cap,
                          hydro_session** out) {
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!models) return fail(HYDRO_EINVAL, "models is NULL");
  if (k < 1) return fail(HYDRO_EINVAL, "K must be at least 1");
  if (k > HYDRO_MAX_PREDICATES) return fail(HYDRO_EUNSUPPORTED, "K above 8 is not supported");
  if (frame_h <= 0 || frame_w <= 0) return fail(HYDRO_EINVAL, "frame shape must be positive");
  if (max_push <= 0) return fail(HYDRO_EINVAL, "max_push must be positive");
  if (max_push > (int64_t)kIdxMask) return fail(HYDRO_EUNSUPPORTED, "max_push above 2^24 - 1 tuples");
  int rc = validate_policy(policy, k);
  if (rc) return rc;
  for (int i = 0; i < k; ++i)
    if ((rc = validate_model(models[i], frame_h, frame_w))) return rc;
  if (policy->precision == HYDRO_PREC_FP8)
    for (int i = 0; i < k; ++i)
      if (models[i].arch != HYDRO_ARCH_CNN || !c4_shape_ok(models[i].in_h, models[i].n_layers, models[i].widths))
        return fail(HYDRO_EUNSUPPORTED, "the FP8 first pass is built for 4-layer 128x128 CNN predicates (32-64-128-256)");
  if (policy->rescore3)
    for (int i = 0; i < k; ++i)
      if (models[i].arch != HYDRO_ARCH_CNN || models[i].on_crop ||
          !c4_shape_ok(models[i].in_h, models[i].n_layers, models[i].widths))
        return fail(HYDRO_EUNSUPPORTED, "the three-product re-score tier is built for 4-layer 128x128 CNN predicates "
                                        "(32-64-128-256) on whole frames");

  g_alloc_counter = 0;
  hydro_session* s = new hydro_session();
  s->arena = arena;
  s->arena_cap = arena ? arena_cap : 0;
  s->pol = *policy;
  s->auto_tau = s->pol.tau <= 0.f;
  s->auto_tau32 = s->pol.tau32 <= 0.f;
  s->auto_tau16 = (s->pol.precision == HYDRO_PREC_FP8 || s->pol.rescore3) && s->pol.tau16 <= 0.f;
  if (s->auto_tau) s->pol.tau = kAutoTauFloor;
  if (s->auto_tau32) s->pol.tau32 = kAutoTau32Floor;
  if (s->pol.tau16 <= 0.f) s->pol.tau16 = s->pol.rescore3 ? kAutoTauX3Floor : kAutoTauFloor;
  for (int i = 0; i < kMaxK; ++i) {
    s->tau_k[i] = s->pol.tau;
    s->tau32_k[i] = s->pol.tau32;
    s->tau16_k[i] = s->pol.tau16;
  }
  s->K = k;
  s->fh = frame_h;
  s->fw = frame_w;
  s->max_push = max_push;
  s->cap = max_push;
  // the session's frame dtype is fixed by the first push; weights are packed then
  s->fdtype = -1;
  s->models.resize(k);
  for (int i = 0; i < k; ++i) {
    HostModel& hm = s->models[i];
    hm.m = models[i];
    const hydro_model& m = models[i];
    hm.flops = model_flops(m);
    if (m.arch == HYDRO_ARCH_HOST) {
      s->host_preds.push_back(i);
    } else if (m.arch == HYDRO_ARCH_MLP) {
      size_t D = (size_t)m.in_h * m.in_w * 3;
      hm.w1.assign(m.w1, m.w1 + D * m.hidden);
      hm.b1.assign(m.b1, m.b1 + m.hidden);
      hm.w2.assign(m.w2, m.w2 + (size_t)m.hidden * kClasses);
      hm.b2.assign(m.b2, m.b2 + kClasses);
    } else {
      int cin = 3;
      for (int l = 0; l < m.n_layers; ++l) {
        hm.cw[l].assign(m.conv_w[l], m.conv_w[l] + (size_t)m.widths[l] * cin * 9);
        hm.cb[l].assign(m.conv_b[l], m.conv_b[l] + m.widths[l]);
        cin = m.widths[l];
      }
      hm.fcw.assign(m.fc_w, m.fc_w + (size_t)cin * kClasses);
      hm.fcb.assign(m.fc_b, m.fc_b + kClasses);
      hm.variant = m.on_crop ? CNN_NONE : cnn_variant_of(m.in_h, m.n_layers, m.widths);
      if (m.on_crop) s->crop_preds.push_back(i);
    }
  }
  auto bail = [&](int code) {
    free_session(s);
    return code;
  };
  hipError_t he = hipGetDevice(&s->device);
  if (he != hipSuccess) return bail(fail(HYDRO_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he)));
  hipDeviceProp_t prop;
  he = hipGetDeviceProperties(&prop, s->device);
  if (he != hipSuccess) return bail(fail(HYDRO_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(he)));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return bail(fail(HYDRO_EUNSUPPORTED, std::string("this library is built for gfx950, device is ") + prop.gcnArchName));
  s->n_cu = prop.multiProcessorCount;
  int clk_khz = 0;
  if (hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, s->device) == hipSuccess && clk_khz > 0)
    s->tick_us = 1000.0 / clk_khz;
  if (s->pol.stream || s->arena) {
    s->stream = (hipStream_t)s->pol.stream;
  } else {
    he = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (he != hipSuccess) return bail(fail(HYDRO_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(he)));
    s->own_stream = true;
  }
  if (!s->arena) {   // the host-frame staging ring (allocation-free sessions take device frames only)
    he = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (he != hipSuccess) return bail(fail(HYDRO_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(he)));
    for (int i = 0; i < 2; ++i) {
      hipEventCreateWithFlags(&s->stage_free[i], hipEventDisableTiming);
      hipEventCreateWithFlags(&s->stage_ready[i], hipEventDisableTiming);
    }
  }
  const int64_t cap = s->cap;
  if ((rc = sess_alloc(s, (void**)&s->st, sizeof(DevState)))) return bail(rc);
  for (int i = 0; i < 2; ++i)
    if ((rc = sess_alloc(s, (void**)&s->pend[i], cap * 4))) return bail(rc);
  if ((rc = sess_alloc(s, (void**)&s->q1, cap * 4 * k))) return bail(rc);
  if ((rc = sess_alloc(s, (void**)&s->q2, cap * 4 * k))) return bail(rc);
  if ((rc = sess_alloc(s, (void**)&s->q3, cap * 4 * k))) return bail(rc);
  if ((s->pol.precision == HYDRO_PREC_FP8 || s->pol.rescore3) && (rc = sess_alloc(s, (void**)&s->qm, cap * 4 * k)))
    return bail(rc);
  const int64_t nwords = (cap + 31) / 32;
  if ((rc = sess_alloc(s, (void**)&s->result_bits, nwords * 4 + 1024))) return bail(rc);
  if ((rc = sess_alloc(s, (void**)&s->res_blocks, ((nwords + 255) / 256 + 1) * 4))) return bail(rc);
  if ((rc = sess_alloc(s, (void**)&s->res_base, 16))) return bail(rc);
  if (s->pol.log_routes && (rc = sess_alloc(s, (void**)&s->route_log, cap * 4))) return bail(rc);
  if (s->pol.log_routes) {
    s->round_log_cap = 16384;
    if ((rc = sess_alloc(s, (void**)&s->round_log, (size_t)s->round_log_cap * sizeof(hydro_round_record))))
      return bail(rc);
  }
  if ((rc = sess_alloc(s, (void**)&s->theta, 4096 * sizeof(float)))) return bail(rc);
  s->theta_cap = 4096;
  if (s->pol.reuse) {
    if (s->arena) return bail(fail(HYDRO_EUNSUPPORTED, "allocation-free queries keep no result cache"));
    s->cache.log2 = s->pol.cache_log2 > 0 ? (uint32_t)s->pol.cache_log2 : 22u;
    const size_t slots = (size_t)k << s->cache.log2;
    if ((rc = sess_alloc(s, (void**)&s->cache.keys, slots * sizeof(unsigned long long)))) return bail(rc);
    if ((rc = sess_alloc(s, (void**)&s->cache.vals, slots * sizeof(uint2)))) return bail(rc);
    he = hipMemset(s->cache.keys, 0xFF, slots * sizeof(unsigned long long));   // every slot kCacheEmpty
    if (he != hipSuccess) return bail(fail(HYDRO_EDEVICE, std::string("hipMemset(cache): ") + hipGetErrorString(he)));
  }
  if (s->arena) {
    if ((rc = sess_alloc(s, (void**)&s->out_ids, cap * sizeof(int64_t)))) return bail(rc);
  } else {
    he = dev_alloc((void**)&s->out_ids, cap * sizeof(int64_t));
    if (he != hipSuccess) return bail(fail(HYDRO_ENOMEM, "result buffer allocation failed"));
  }
  s->out_cap = cap;
  if (!s->crop_preds.empty()) {
    // activations of the largest crop (the whole frame), two buffers per workgroup
    int64_t act = 0;
    for (int k : s->crop_preds) {
      const hydro_model& m = s->models[k].m;
      int h = frame_h, w = frame_w;
      for (int l = 0; l < m.n_layers; ++l) {
        h = (h + 1) / 2;
        w = (w + 1) / 2;
        act = std::max<int64_t>(act, (int64_t)h * w * m.widths[l]);
      }
    }
    // four workgroups per CU (a quarter of what the kernel's registers allow): more hides the
    // latency of the serial FP64 chains when a round holds many crops, fewer shortens the tail
    // of the largest crop, which alone bounds a round that holds few
    s->crop_grid = s->n_cu * 4;
    CropArgs& ca = s->crop;
    ca.act_doubles = (act + 31) / 32 * 32;
    ca.fh = frame_h;
    ca.fw = frame_w;
    ca.balance = s->pol.balance;
    if ((rc = sess_alloc(s, (void**)&s->crops_dev, (size_t)cap * 4 * sizeof(int32_t)))) return bail(rc);
    if ((rc = sess_alloc(s, (void**)&ca.scratch, (size_t)s->crop_grid * 2 * ca.act_doubles * sizeof(double))))
      return bail(rc);
    if ((rc = sess_alloc(s, (void**)&ca.order, (size_t)s->crop_preds.size() * cap * sizeof(uint32_t)))) return bail(rc);
    if ((rc = sess_alloc(s, (void**)&ca.next, 256))) return bail(rc);
    ca.crops = s->crops_dev;
  }
  if (!s->host_preds.empty()) {
    if (s->pol.route == HYDRO_ROUTE_LEARNED)
      return bail(fail(HYDRO_EUNSUPPORTED, "HOST predicates are not combined with the learned router"));
    if (s->arena) return bail(fail(HYDRO_EUNSUPPORTED, "allocation-free queries take no HOST predicates"));
    const int64_t warm = (int64_t)s->pol.warmup_batches * s->K * s->pol.routing_batch;
    s->h_cap = std::min<int64_t>(cap, (int64_t)s->K * std::max<int64_t>(s->pol.wave, warm));
    const size_t nh = s->host_preds.size();
    if (hipHostMalloc((void**)&s->h_counts, kMaxK * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void**)&s->h_entries, nh * s->h_cap * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&s->h_dec, nh * s->h_cap) != hipSuccess)
      return bail(fail(HYDRO_ENOMEM, "pinned host buffers of the HOST predicates"));
    if ((rc = sess_alloc(s, (void**)&s->d_dec, nh * s->h_cap))) return bail(rc);
    for (hipEvent_t* e : {&s->h_routed, &s->h_ready, &s->h_done}) {
      he = hipEventCreateWithFlags(e, hipEventDisableTiming);
      if (he != hipSuccess) return bail(fail(HYDRO_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(he)));
    }
    const char* ht = getenv("HYDRO_HOST_THREADS");
    const int hw = (int)std::thread::hardware_concurrency();
    s->host_threads = (ht && *ht) ? std::max(1, atoi(ht)) : std::max(1, hw);
    s->pool.reset(new HostPool());
    s->pool->start(s->host_threads);
  }
  if (s->pol.route == HYDRO_ROUTE_LEARNED) {
    double fl[kMaxK];
    for (int i = 0; i < k; ++i) fl[i] = s->models[i].flops;
    rc = router_nn_create(&s->rnn, s->K, frame_h, frame_w, cap, s->pol.seed, s->pol.routing_batch, s->pol.explore, fl,
                          s->arena ? rnn_arena_alloc : nullptr, s);
    if (rc == HYDRO_EUNSUPPORTED) return bail(fail(rc, "learned router: frames must be square with a side divisible by 8"));
    if (rc == HYDRO_ENOMEM) return bail(fail(rc, "learned router: device allocation failed"));
    if (rc) return bail(rc);
    s->fused_feats = true;
    for (int i = 0; i < k; ++i)
      if (s->models[i].m.arch != HYDRO_ARCH_CNN || s->models[i].variant == CNN_NONE) s->fused_feats = false;
  }
  rc = hydro_session_reset(s);
  if (rc) return bail(rc);
  *out = s;
  return HYDRO_OK;
}

int hydro_session_create(const hydro_model* models, int32_t k, const hydro_policy* policy, int32_t frame_h,
                         int32_t frame_w, int64_t max_push, hydro_session** out) {
  g_err.clear();
  return session_create(models, k, policy, frame_h, frame_w, max_push, nullptr, 0, out);
}

int hydro_session_reset(hydro_session* s) {
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemsetAsync(s->st, 0, sizeof(DevState), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->rounds_done = 0;
  s->warmed = false;
  s->parity = 0;
  s->pushes = 0;
  s->in_query = false;
  s->ids_sorted = true;
  s->last_id_end = INT64_MIN;
  s->theta_host.clear();
  s->crops_host.clear();
  s->info = hydro_query_info{};
  s->ev_used = 0;
  if (s->rnn) {
    router_nn_reset(s->rnn, s->stream);
    const int one = 1;
    HIP_TRY(hipMemcpy(&s->st->learned_active, &one, sizeof(int), hipMemcpyHostToDevice));
  }
  return HYDRO_OK;
}

static Forward make_forward(hydro_session* s, int tier, int out_slot, const FrameSrc& fr, int n_seg, int64_t seg_len,
                            int64_t id_base) {
  Forward f{};
  f.st = s->st;
  f.pend_out = s->pend[out_slot];
  f.pend_out_count = &s->st->pend_count[out_slot];
  f.result_bits = s->result_bits;
  f.route_log = s->route_log;
  f.theta = s->theta;
  f.n_seg = n_seg;
  f.seg_len = seg_len;
  f.id_base = id_base;
  f.seg_first = id_base >= 0 ? id_base / seg_len : 0;
  f.seg_off = id_base >= 0 ? (uint32_t)(id_base % seg_len) : 0;
  f.seg_len32 = (id_base >= 0 && seg_len < ((int64_t)1 << 31)) ? (uint32_t)seg_len : 0u;
  f.full_mask = (1u << s->K) - 1u;
  f.k_total = s->K;
  f.logits = nullptr;
  f.olog = s->rnn ? router_nn_log(s->rnn) : OutcomeLog{};
  f.cache = s->cache;
  const bool bf = s->pol.precision == HYDRO_PREC_BF16;
  const bool f8 = s->pol.precision == HYDRO_PREC_FP8;
  if (tier == TIER_FIRST && (f8 || s->pol.rescore3)) {     // on to the middle tier
    f.count_eval = 1;
    f.defer = Queues{s->qm, s->st->mcount, s->cap};
    f.defer_stat = s->st->r_rescored;
    for (int k = 0; k < kMaxK; ++k) f.tau[k] = s->tau_k[k];
  } else if (tier == TIER_FIRST) {
    f.count_eval = 1;
    f.defer = Queues{bf ? s->q2 : s->q3, bf ? s->st->bcount : s->st->ecount, s->cap};
    f.defer_stat = bf ? s->st->r_rescored : s->st->r_esc;
    for (int k = 0; k < kMaxK; ++k) f.tau[k] = bf ? s->tau_k[k] : s->tau32_k[k];
  } else if (tier == TIER_MID) {
    f.count_eval = 0;
    f.defer = Queues{s->q2, s->st->bcount, s->cap};
    f.defer_stat = s->st->r_mid;
    for (int k = 0; k < kMaxK; ++k) f.tau[k] = s->tau16_k[k];
  } else if (tier == TIER_F32) {
    f.count_eval = 0;
    f.defer = Queues{s->q3, s->st->ecount, s->cap};
    f.defer_stat = s->st->r_esc;
    for (int k = 0; k < kMaxK; ++k) f.tau[k] = s->tau32_k[k];
  } else {
    f.count_eval = 0;
    f.defer = Queues{nullptr, nullptr, 0};
    f.defer_stat = nullptr;
    for (int k = 0; k < kMaxK; ++k) f.tau[k] = 0.f;
  }
  (void)fr;
  return f;
}

static void enqueue_tier(hydro_session* s, int tier, const FrameSrc& fr, const Forward& f, hipStream_t st) {
  Queues q;
  if (tier == TIER_FIRST) q = Queues{s->q1, s->st->qcount, s->cap};
  else if (tier == TIER_F32) q = Queues{s->q2, s->st->bcount, s->cap};
  else if (tier == TIER_MID) q = Queues{s->qm, s->st->mcount, s->cap};
  else q = Queues{s->q3, s->st->ecount, s->cap};
  if (tier == TIER_FIRST && s->crop.n_preds) {     // FP64 on crops: final decisions, first tier only
    CropArgs a = s->crop;
    a.q = q;
    a.fr = fr;
    a.st = s->st;
    launch_crop_pass(a, f, s->crop_grid, st);
  }
  // grouped: one launch covers every predicate of an architecture; otherwise one launch per
  // predicate (the plain form)
  if (s->mlp.n_preds) {
    MlpArgs a = s->mlp;
    a.q = q;
    a.fr = fr;
    a.st = s->st;
    a.part_cap = s->cap;
    a.count_ticks = 1;
    a.prec = s->pol.precision;
    const int grid = tier == TIER_F64 ? s->n_cu : s->n_cu * 4;
    if (s->pol.grouped || a.n_preds == 1) {
      launch_mlp_pass(a, f, tier, grid, st);
    } else {
      for (int i = 0; i < s->mlp.n_preds; ++i) {
        MlpArgs b = a;
        b.n_preds = 1;
        mlp_copy_slot(b, 0, a, i);      // every per-slot field (a partial copy mixes predicates)
        launch_mlp_pass(b, f, tier, grid, st);
      }
    }
  }
  if (s->gcnn.n_preds) {
    GcnnArgs a = s->gcnn;
    a.q = q;
    a.fr = fr;
    a.st = s->st;
    a.count_ticks = 1;
    a.prec = s->pol.precision;
    if (s->pol.grouped || a.n_preds == 1) {
      launch_gcnn_pass(a, f, tier, s->n_cu, st);
    } else {
      for (int i = 0; i < s->gcnn.n_preds; ++i) {
        GcnnArgs b = a;
        b.n_preds = 1;
        gcnn_copy_slot(b, 0, a, i);
        launch_gcnn_pass(b, f, tier, s->n_cu, st);
      }
    }
  }
  if (s->cnn.n_preds) {
    CnnArgs a = s->cnn;
    a.q = q;
    a.fr = fr;
    a.st = s->st;
    a.count_ticks = 1;
    a.prec = s->pol.precision;
    a.feats = tier == TIER_FIRST && s->fused_feats ? router_nn_feats_ptr(s->rnn) : nullptr;
    if (s->pol.grouped || a.n_preds == 1) {
      launch_cnn_pass(a, f, tier, s->n_cu, st);
    } else {
      for (int i = 0; i < s->cnn.n_preds; ++i) {
        CnnArgs b = a;
        b.n_preds = 1;
        b.pred[0] = a.pred[i]; b.variant[0] = a.variant[i]; b.class_mask[0] = a.class_mask[i];
        for (int l = 0; l < 3; ++l) {
          b.w_bf[0][l] = a.w_bf[i][l]; b.w_s3[0][l] = a.w_s3[i][l]; b.bias[0][l] = a.bias[i][l];
          b.w_canon[0][l] = a.w_canon[i][l]; b.b_canon[0][l] = a.b_canon[i][l];
        }
        b.fc_w[0] = a.fc_w[i]; b.fc_b[0] = a.fc_b[i];
        b.esc_act[0] = a.esc_act[i];
        for (int l = 0; l < 3; ++l) b.wt_canon[0][l] = a.wt_canon[i][l];
        launch_cnn_pass(b, f, tier, s->n_cu, st);
      }
    }
  }
}

// ---------------------------------------------------------------- autotuner
// For every MLP predicate, time each GEMM tile shape on a synthetic queue of the session's size
// class (real weights, constant frames) and keep the fastest.  Results are cached by
// (gfx950, precision, frame dtype, input size, hidden width, queue size) in a small JSON object.
static std::string tune_key(int prec, int dtype, int D, int H, int64_t q) {
  return "gfx950/" + std::string(prec == HYDRO_PREC_BF16 ? "bf16" : "fp32") + "/" +
         (dtype == HYDRO_DTYPE_BF16 ? "bf16" : dtype == HYDRO_DTYPE_U8 ? "u8" : "f32") + "/D" + std::to_string(D) +
         "/h" + std::to_string(H) + "/q" + std::to_string(q);
}

static std::vector<std::pair<std::string, int>> tune_load(const char* path) {
  std::vector<std::pair<std::string, int>> out;
  FILE* f = path ? fopen(path, "r") : nullptr;
  if (!f) return out;
  std::string txt;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, r);
  fclose(f);
  size_t pos = 0;
  while ((pos = txt.find('"', pos)) != std::string::npos) {
    size_t end = txt.find('"', pos + 1);
    if (end == std::string::npos) break;
    std::string key = txt.substr(pos + 1, end - pos - 1);
    size_t colon = txt.find(':', end);
    if (colon == std::string::npos) break;
    out.push_back({key, atoi(txt.c_str() + colon + 1)});
    pos = txt.find_first_of(",}", colon);
    if (pos == std::string::npos) break;
  }
  return out;
}

static void tune_save(const char* path, const std::vector<std::pair<std::string, int>>& kv) {
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  for (size_t i = 0; i < kv.size(); ++i)
    fprintf(f, "  \"%s\": %d%s\n", kv[i].first.c_str(), kv[i].second, i + 1 < kv.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

__global__ void k_fill_bytes(uint32_t* p, uint32_t v, int64_t n_words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static int autotune_mlp(hydro_session* s) {
  MlpArgs& ma = s->mlp;
  if (ma.n_preds == 0) return HYDRO_OK;
  const char* path = getenv("HYDRO_TUNE_CACHE");
  auto cache = tune_load(path);
  const int64_t Q = std::min<int64_t>(s->cap, 4096);
  const int D = ma.d_in[0];
  const size_t fbytes = (size_t)D * (s->fdtype == HYDRO_DTYPE_F32 ? 4 : s->fdtype == HYDRO_DTYPE_BF16 ? 2 : 1);
  void* frames = nullptr;
  bool changed = false;
  hipStream_t st = s->stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (int i = 0; i < ma.n_preds; ++i) {
    // the bf16 first pass on bf16 frames runs the direct-to-LDS GEMM (tile configurations 0 and 1
    // launch it), which measured faster than every register-staged shape on the 6-MLP workload
    if (s->pol.precision == HYDRO_PREC_BF16 && s->fdtype == HYDRO_DTYPE_BF16 && ma.d_in[i] % 64 == 0 &&
        ma.hidden[i] % 128 == 0) {
      ma.tile_cfg[i] = 0;
      ma.part_w[i] = mlp_tile_bn(0) / 2;
      continue;
    }
    const std::string key = tune_key(s->pol.precision, s->fdtype, ma.d_in[i], ma.hidden[i], Q);
    int best = -1;
    for (auto& kv : cache)
      if (kv.first == key) best = kv.second;
    if (best < 0 || best >= MLP_TILE_CONFIGS) {
      if (!frames) {
        hipError_t he = dev_alloc(&frames, fbytes * Q);
        if (he != hipSuccess) return fail(HYDRO_ENOMEM, "autotune frame buffer");
        // bf16 1.0 pairs / small fp32 / uint8 values: finite, representative magnitudes
        hipLaunchKernelGGL(k_fill_bytes, dim3(1024), dim3(256), 0, st, (uint32_t*)frames, 0x3F003F00u,
                           (int64_t)(fbytes * Q / 4));
      }
      const int k = ma.pred[i];
      std::vector<uint32_t> ent(Q);
      for (int64_t t = 0; t < Q; ++t) ent[t] = make_entry((uint32_t)t, 0u);
      HIP_TRY(hipMemcpy(s->q1 + (int64_t)k * s->cap, ent.data(), Q * 4, hipMemcpyHostToDevice));
      int cnt[kMaxK] = {0};
      cnt[k] = (int)Q;
      HIP_TRY(hipMemcpy(s->st->qcount, cnt, sizeof(cnt), hipMemcpyHostToDevice));
      MlpArgs b = ma;
      b.n_preds = 1;
      mlp_copy_slot(b, 0, ma, i);
      b.q = Queues{s->q1, s->st->qcount, s->cap};
      b.fr = FrameSrc{frames, s->fdtype, s->fh, (int64_t)D};
      b.st = s->st;
      b.part_cap = s->cap;
      b.count_ticks = 0;
      float best_ms = 1e30f;
      for (int cfg = 0; cfg < MLP_TILE_CONFIGS; ++cfg) {
        const bool bf = s->pol.precision == HYDRO_PREC_BF16;
        launch_mlp_gemm(b, cfg, bf, s->n_cu * 4, st);
        HIP_TRY(hipEventRecord(e0, st));
        for (int rep = 0; rep < 3; ++rep) launch_mlp_gemm(b, cfg, bf, s->n_cu * 4, st);
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best = cfg;
        }
      }
      cache.push_back({key, best});
      changed = true;
    }
    ma.tile_cfg[i] = best;
    ma.part_w[i] = mlp_tile_bn(best) / 2;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (frames) hipFree(frames);
  if (changed) tune_save(path, cache);
  // leave the device state as a fresh query expects it
  HIP_TRY(hipMemsetAsync(s->st, 0, sizeof(DevState), st));
  if (s->rnn) {
    const int one = 1;
    HIP_TRY(hipMemcpyAsync(&s->st->learned_active, &one, sizeof(int), hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return HYDRO_OK;
}

static int ensure_dtype(hydro_session* s, int dtype) {
  if (s->fdtype == dtype) return HYDRO_OK;
  if (s->fdtype != -1) return fail(HYDRO_EINVAL, "frame dtype differs from the session's first push");
  if (dtype != HYDRO_DTYPE_F32 && dtype != HYDRO_DTYPE_BF16 && dtype != HYDRO_DTYPE_U8)
    return fail(HYDRO_EINVAL, "unknown frame dtype");
  for (auto& hm : s->models)
    if (hm.m.arch == HYDRO_ARCH_CNN && dtype == HYDRO_DTYPE_F32)
      return fail(HYDRO_EUNSUPPORTED, "CNN predicates take bf16 or uint8 frames");
  s->fdtype = dtype;
  HIP_TRY(hipStreamSynchronize(s->stream));
  int rc = pack_models(s);
  if (!rc && s->pol.autotune) rc = autotune_mlp(s);
  if (rc) {
    s->fdtype = -1;
    return rc;
  }
  return HYDRO_OK;
}

static size_t dtype_size(int dt) { return dt == HYDRO_DTYPE_F32 ? 4 : dt == HYDRO_DTYPE_BF16 ? 2 : 1; }

static int measure_bands(hydro_session* s, const hydro_frames* frames, float safety, float* tau, float* tau16,
                         float* tau32);
static int measure_ascales(hydro_session* s, const hydro_frames* frames);

// Automatic bands (policy tau / tau32 <= 0): measured once, on up to 1,024 frames of the
// session's first push, with safety 3, and never below the fixed defaults.
static int auto_bands(hydro_session* s, const hydro_frames& fr) {
  hydro_frames sub = fr;
  sub.n = std::min<int64_t>(fr.n, 1024);
  void* tmp = nullptr;
  if (fr.where != HYDRO_MEM_DEVICE) {
    const size_t bytes = (size_t)sub.n * fr.h * fr.w * 3 * dtype_size(fr.dtype);
    hipError_t e = dev_alloc(&tmp, bytes);
    if (e != hipSuccess) return fail(HYDRO_ENOMEM, "band calibration frame buffer");
    e = hipMemcpy(tmp, fr.data, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      hipFree(tmp);
      return fail(HYDRO_EDEVICE, std::string("band calibration copy: ") + hipGetErrorString(e));
    }
    sub.data = tmp;
    sub.where = HYDRO_MEM_DEVICE;
  }
  float tau[kMaxK], tau16[kMaxK], tau32[kMaxK];
  int rc = HYDRO_OK;
  if (s->pol.precision == HYDRO_PREC_FP8 && !s->ascales_set) rc = measure_ascales(s, &sub);
  if (!rc) rc = measure_bands(s, &sub, 3.0f, tau, tau16, tau32);
  if (tmp) hipFree(tmp);
  if (rc) return rc;
  const bool low = s->pol.precision != HYDRO_PREC_FP32;
  for (int k = 0; k < s->K; ++k) {
    if (s->auto_tau) s->tau_k[k] = low ? std::max(tau[k], kAutoTauFloor) : std::max(tau32[k], kAutoTau32Floor);
    if (s->auto_tau16) s->tau16_k[k] = std::max(tau16[k], s->pol.rescore3 ? kAutoTauX3Floor : kAutoTauFloor);
    if (s->auto_tau32) s->tau32_k[k] = std::max(tau32[k], kAutoTau32Floor);
  }
  s->auto_tau = s->auto_tau32 = s->auto_tau16 = false;
  drop_graphs(s);
  return HYDRO_OK;
}

// ---------------------------------------------------------------- HOST predicates
// The colour-box fraction of one frame over its sampled pixels (x in [0,1]: bf16 value,
// uint8 / 255, or fp32).
static double host_color_fraction(const hydro_model& m, const void* base, int dtype, int64_t idx, int64_t pixels) {
  const int st = m.color_stride > 1 ? m.color_stride : 1;
  int64_t inside = 0, sampled = 0;
  for (int y = 0; y < m.in_h; y += st)
    for (int x = 0; x < m.in_w; x += st) {
      const int64_t e0 = (idx * pixels + (int64_t)y * m.in_w + x) * 3;
      bool in = true;
      for (int c = 0; c < 3; ++c) {
        double v;
        if (dtype == HYDRO_DTYPE_BF16) {
          const uint32_t u = (uint32_t) static_cast<const uint16_t*>(base)[e0 + c] << 16;
          float f;
          memcpy(&f, &u, 4);
          v = f;
        } else if (dtype == HYDRO_DTYPE_U8) {
          v = (double)static_cast<const uint8_t*>(base)[e0 + c] / 255.0;
        } else {
          v = static_cast<const float*>(base)[e0 + c];
        }
        in = in && v >= (double)m.color_lo[c] && v <= (double)m.color_hi[c];
      }
      inside += in;
      ++sampled;
    }
  return (double)inside / (double)sampled;
}

// After the round's route kernel: copy the counts and every HOST predicate's queue to pinned host
// memory on the copy stream (the GPU tiers are enqueued behind the route on the main stream).
static int host_round_copy(hydro_session* s, hipStream_t st) {
  HIP_TRY(hipEventRecord(s->h_routed, st));
  HIP_TRY(hipStreamWaitEvent(s->copy_stream, s->h_routed, 0));
  HIP_TRY(hipMemcpyAsync(s->h_counts, s->st->qcount, kMaxK * sizeof(int), hipMemcpyDeviceToHost, s->copy_stream));
  for (size_t h = 0; h < s->host_preds.size(); ++h)
    HIP_TRY(hipMemcpyAsync(s->h_entries + h * s->h_cap, s->q1 + (int64_t)s->host_preds[h] * s->cap,
                           s->h_cap * sizeof(uint32_t), hipMemcpyDeviceToHost, s->copy_stream));
  HIP_TRY(hipEventRecord(s->h_ready, s->copy_stream));
  return HYDRO_OK;
}

// After the round's GPU tiers are enqueued: wait for the copies, decide the HOST queues on CPU
// threads (while the GPU works through its queues), copy the decisions up and enqueue their
// forwarding behind the GPU tiers.
static int host_round_decide(hydro_session* s, hipStream_t st, const hydro_frames& fr, const float* theta, int n_seg,
                             int64_t seg_len, const Forward& f) {
  HIP_TRY(hipEventSynchronize(s->h_ready));
  const int64_t pixels = (int64_t)fr.h * fr.w;
  const void* host_frames = fr.where == HYDRO_MEM_HOST ? fr.data : fr.host_data;
  std::vector<unsigned long long> ticks(s->host_preds.size(), 0);
  for (size_t h = 0; h < s->host_preds.size(); ++h) {
    const int k = s->host_preds[h];
    const int64_t n = s->h_counts[k];
    if (n > s->h_cap) return fail(HYDRO_EDEVICE, "HOST predicate queue above its round bound");
    if (n == 0) continue;
    const hydro_model& m = s->models[k].m;
    const uint32_t* ent = s->h_entries + h * s->h_cap;
    uint8_t* dec = s->h_dec + h * s->h_cap;
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(s->host_threads, (n + 63) / 64));
    std::vector<double> us(T, 0.0);
    auto work = [&](int t) {
      const auto t0 = std::chrono::steady_clock::now();
      for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) {
        const uint32_t idx = entry_idx(ent[i]);
        const int64_t id = fr.id_base + idx;
        const int64_t sg = std::min<int64_t>(id / seg_len, n_seg - 1);
        const double th = theta[sg * s->K + k];
        dec[i] = host_color_fraction(m, host_frames, fr.dtype, idx, pixels) > th ? 1 : 0;
      }
      us[t] = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    };
    s->pool->run(T, work);
    double tot = 0;
    for (double u : us) tot += u;
    // thread time in device clock ticks, scaled by compute units / threads: the cost estimates of
    // both resources are then each resource's wall time per tuple times the same constant
    ticks[h] = (unsigned long long)(tot / s->tick_us * (double)s->n_cu / (double)s->host_threads);
    HIP_TRY(hipMemcpyAsync(s->d_dec + h * s->h_cap, dec, n, hipMemcpyHostToDevice, s->copy_stream));
  }
  HIP_TRY(hipEventRecord(s->h_done, s->copy_stream));
  HIP_TRY(hipStreamWaitEvent(st, s->h_done, 0));
  for (size_t h = 0; h < s->host_preds.size(); ++h) {
    const int k = s->host_preds[h];
    const int64_t n = s->h_counts[k];
    if (n == 0) continue;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, (int64_t)s->n_cu * 4);
    hipLaunchKernelGGL(k_apply_host, dim3(grid), dim3(256), 0, st, Queues{s->q1, s->st->qcount, s->cap}, k,
                       s->d_dec + h * s->h_cap, f, ticks[h]);
  }
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int hydro_session_push(hydro_session* s, const hydro_frames* frames, const float* thresholds, int32_t n_seg,
                       int64_t seg_len) {
  g_err.clear();
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  if (!frames) return fail(HYDRO_EINVAL, "frames is NULL");
  if (!thresholds) return fail(HYDRO_EINVAL, "thresholds is NULL");
  if (n_seg < 1 || seg_len < 1) return fail(HYDRO_EINVAL, "n_seg and seg_len must be positive");
  if ((int64_t)n_seg * s->K > 1 << 20) return fail(HYDRO_EUNSUPPORTED, "threshold table too large");
  const hydro_frames& fr = *frames;
  if (fr.n < 0) return fail(HYDRO_EINVAL, "negative tuple count");
  if (fr.n > s->max_push) return fail(HYDRO_ECAPACITY, "push larger than the session's max_push");
  if (fr.h != s->fh || fr.w != s->fw) return fail(HYDRO_EINVAL, "frame shape differs from the session's");
  if (fr.where != HYDRO_MEM_DEVICE && fr.where != HYDRO_MEM_HOST) return fail(HYDRO_EINVAL, "unknown frame location");
  if (fr.n > 0 && !fr.data) return fail(HYDRO_EINVAL, "frame data is NULL");
  if (fr.id_base < 0) return fail(HYDRO_EINVAL, "negative id_base");
  const bool host_mode = !s->host_preds.empty();
  if (!s->crop_preds.empty()) {
    if (!fr.crops) return fail(HYDRO_EINVAL, "the session has on_crop predicates: the push needs crops");
    for (int64_t i = 0; i < fr.n; ++i) {
      const int32_t* c = fr.crops + 4 * i;
      if (c[0] < 0 || c[1] < 0 || c[2] < 1 || c[3] < 1 || (int64_t)c[0] + c[2] > fr.h || (int64_t)c[1] + c[3] > fr.w)
        return fail(HYDRO_EINVAL, "crop " + std::to_string(i) + " is not a non-empty box inside its frame");
    }
  }
  if (host_mode && fr.where != HYDRO_MEM_HOST && !fr.host_data)
    return fail(HYDRO_EUNSUPPORTED, "a session with HOST predicates takes frames in host memory (or host_data)");
  int rc = ensure_dtype(s, fr.dtype);
  if (rc) return rc;
  for (int64_t i = 0; i < (int64_t)n_seg * s->K; ++i)
    if (std::isnan(thresholds[i])) return fail(HYDRO_EINVAL, "threshold is NaN");
  if ((s->auto_tau || s->auto_tau32 || s->auto_tau16) && fr.n > 0 && s->pushes == 0)
    if ((rc = auto_bands(s, fr))) return rc;

  if (s->pushes == 0) s->t_start = std::chrono::steady_clock::now();
  s->pushes++;
  s->in_query = true;
  if (fr.id_base < s->last_id_end) s->ids_sorted = false;
  s->last_id_end = fr.id_base + fr.n;
  s->last_push_n = fr.n;
  hipStream_t st = s->stream;
  const int64_t n = fr.n;

  // thresholds (the host copy lives until finish: the async copy may still read it)
  if ((int64_t)n_seg * s->K > s->theta_cap) {
    HIP_TRY(hipStreamSynchronize(st));
    void* p;
    if ((rc = sess_alloc(s, &p, (size_t)n_seg * s->K * sizeof(float)))) return rc;
    s->theta = (float*)p;
    s->theta_cap = n_seg * s->K;
  }
  s->theta_host.emplace_back(thresholds, thresholds + (size_t)n_seg * s->K);
  if (!s->crop_preds.empty() && fr.n > 0) {
    s->crops_host.emplace_back(fr.crops, fr.crops + 4 * fr.n);
    HIP_TRY(hipMemcpyAsync(s->crops_dev, s->crops_host.back().data(), (size_t)fr.n * 4 * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(s->theta, s->theta_host.back().data(), (size_t)n_seg * s->K * sizeof(float),
                         hipMemcpyHostToDevice, st));

  // frames
  const size_t fbytes = (size_t)fr.h * fr.w * 3 * dtype_size(fr.dtype);
  FrameSrc src{};
  src.dtype = fr.dtype;
  src.hw = fr.h;
  src.elems = (int64_t)fr.h * fr.w * 3;
  if (fr.where == HYDRO_MEM_DEVICE) {
    src.base = fr.data;
  } else {
    if (s->arena) return fail(HYDRO_EUNSUPPORTED, "allocation-free queries take device frames");
    int slot = s->stage_next;
    s->stage_next ^= 1;
    if (!s->stage[slot]) {
      HIP_TRY(hipStreamSynchronize(st));
      hipError_t he = dev_alloc(&s->stage[slot], fbytes * s->max_push);
      if (he != hipSuccess) return fail(HYDRO_ENOMEM, "frame staging allocation failed");
    }
    // the copy waits until the last push that used this slot has finished computing
    HIP_TRY(hipStreamWaitEvent(s->copy_stream, s->stage_free[slot], 0));
    if (n > 0) HIP_TRY(hipMemcpyAsync(s->stage[slot], fr.data, fbytes * n, hipMemcpyHostToDevice, s->copy_stream));
    HIP_TRY(hipEventRecord(s->stage_ready[slot], s->copy_stream));
    HIP_TRY(hipStreamWaitEvent(st, s->stage_ready[slot], 0));
    src.base = s->stage[slot];
  }

  // result capacity
  if (s->info.n_tuples + n > (uint64_t)s->out_cap) {
    if (s->arena) return fail(HYDRO_ECAPACITY, "allocation-free sessions hold the results of one push");
    HIP_TRY(hipStreamSynchronize(st));
    int64_t ncap = std::max<int64_t>(s->out_cap * 2, s->info.n_tuples + n);
    int64_t* p;
    hipError_t he = dev_alloc((void**)&p, ncap * sizeof(int64_t));
    if (he != hipSuccess) return fail(HYDRO_ENOMEM, "result buffer allocation failed");
    HIP_TRY(hipMemcpy(p, s->out_ids, s->out_cap * sizeof(int64_t), hipMemcpyDeviceToDevice));
    hipFree(s->out_ids);
    s->out_ids = p;
    s->out_cap = ncap;
  }
  s->info.n_tuples += n;

  // admission schedule: optional warmup round, then waves
  const bool adaptive = s->pol.route != HYDRO_ROUTE_FIXED;
  const bool warm_now = adaptive && !s->warmed && n > 0 && s->pol.warmup_batches > 0;
  std::vector<std::pair<int64_t, int64_t>> adm;
  std::vector<int> warm;
  int64_t pos = 0;
  if (warm_now) {
    int64_t w0 = std::min<int64_t>(n, (int64_t)s->pol.warmup_batches * s->K * s->pol.routing_batch);
    adm.push_back({0, w0});
    warm.push_back(1);
    pos = w0;
  }
  while (pos < n) {
    int64_t w = std::min<int64_t>(n - pos, s->pol.wave);
    adm.push_back({pos, pos + w});
    warm.push_back(0);
    pos += w;
  }
  const int n_rounds = adm.empty() ? 0 : (int)adm.size() + s->K - 1;
  const bool timing = s->pol.time_kernels != 0;
  const int parity0 = s->parity;
  // The learned arm can route from the query's router_nn_first_learned_round()-th round on
  // (training takes at most a fixed number of steps per round); from that round of the query on,
  // every round computes the keys of its live tuples, whichever push it belongs to.
  const int learned_from = s->rnn ? std::max(0, router_nn_first_learned_round() - s->rounds_done) : 0;
  const int64_t nwords = (n + 31) / 32;

  // Every device step of the push, in stream order.  Host state is not touched here, so the
  // same sequence can be captured once into a HIP graph and replayed (sessions with HOST
  // predicates excepted: each round waits for the CPU's decisions, so they run eagerly).
  int host_rc = HYDRO_OK;
  auto enqueue_push = [&](bool timed) {
    if (nwords > 0) hipLaunchKernelGGL(k_fill_u32, dim3(std::min<int64_t>(1024, (nwords + 255) / 256)), dim3(256), 0, st,
                                       s->result_bits, 0u, nwords);
    if (s->route_log && n > 0)
      hipLaunchKernelGGL(k_fill_u32, dim3(std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0, st, s->route_log, 0u, n);
    // router features: pooled for the whole push up front, unless the fused CNN first pass
    // computes them (then only admitted waves that the learned arm routes are pooled, below)
    if (s->rnn && n > 0 && !s->fused_feats) router_nn_admit(s->rnn, src, 0, n, nullptr, st);
    int parity = parity0;
    for (int r = 0; r < n_rounds; ++r) {
      const int in_slot = parity, out_slot = parity ^ 1;
      hipEvent_t ev[kEvPerRound] = {};
      if (timed) {
        for (int i = 0; i < kEvPerRound; ++i) ev[i] = next_event(s);
        if (ev[0]) hipEventRecord(ev[0], st);
      }
      FoldArgs fa{};
      fa.st = s->st;
      fa.k = s->K;
      fa.route = s->pol.route;
      for (int j = 0; j < s->K; ++j) {
        fa.order[j] = s->pol.order[j];
        fa.flops[j] = s->models[j].flops;
      }
      fa.alpha = s->pol.ewma_alpha;
      fa.static_cost = s->pol.cost_source == HYDRO_COST_STATIC;
      fa.out_slot = out_slot;
      fa.final_fold = 0;
      fa.rlog = s->round_log;
      fa.rlog_cap = s->round_log_cap;
      hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, st, fa);

      RouteArgs ra{};
      ra.st = s->st;
      ra.pend_in = s->pend[in_slot];
      ra.in_slot = in_slot;
      if (r < (int)adm.size()) {
        ra.adm_lo = (uint32_t)adm[r].first;
        ra.adm_hi = (uint32_t)adm[r].second;
        ra.warmup = warm[r];
      } else {
        ra.adm_lo = ra.adm_hi = 0;
        ra.warmup = 0;
      }
      ra.routing_batch = s->pol.routing_batch;
      ra.k = s->K;
      ra.q = Queues{s->q1, s->st->qcount, s->cap};
      if (s->cache.keys) {
        ra.fw = make_forward(s, TIER_FIRST, out_slot, src, n_seg, seg_len, fr.id_base);
        ra.route = s->pol.route;
        ra.reuse_aware = s->pol.reuse == 2 && (s->pol.route == HYDRO_ROUTE_SCORE || s->pol.route == HYDRO_ROUTE_COST);
      }
      ra.learned_keys = s->rnn ? router_nn_keys_ptr(s->rnn) : nullptr;
      ra.key_stamps = s->rnn ? router_nn_stamps_ptr(s->rnn) : nullptr;
      if (s->rnn) {
        ra.olog = router_nn_log(s->rnn);
        ra.min_steps = router_nn_min_steps();
        // before the round in which the learned arm can first route, no keys are read
        if (r >= learned_from) {
          if (s->fused_feats && r < (int)adm.size())
            router_nn_admit(s->rnn, src, adm[r].first, adm[r].second, s->st, st);
          router_nn_keys(s->rnn, s->st, s->pend[in_slot], in_slot, ra.adm_lo, ra.adm_hi, s->n_cu, st);
        }
      }
      // enough workgroups for the round's live tuples (at most act_cap), up to kRouteBlocksPerCu per CU
      const int64_t live_bound = std::min<int64_t>(s->act_cap, n);
      const int route_grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)s->n_cu * kRouteBlocksPerCu,
                                                                          (live_bound + kRouteChunk - 1) / kRouteChunk));
      hipLaunchKernelGGL(k_route, dim3(route_grid), dim3(kRouteThreads), 0, st, ra);
      if (host_mode && !host_rc) host_rc = host_round_copy(s, st);
      if (timed && ev[1]) hipEventRecord(ev[1], st);

      // tier chain: first pass, [BF16 re-score of an FP8 first pass, or the three-product
      // re-score of a BF16 one (rescore3)], [FP32 re-score of a
      // low-precision first pass], FP64; events: after first, mid, FP32, FP64 (skipped tiers
      // record their event right after the previous one)
      const int chain[4] = {TIER_FIRST, TIER_MID, TIER_F32, TIER_F64};
      for (int ci = 0; ci < 4; ++ci) {
        const int tier = chain[ci];
        const bool run = tier == TIER_FIRST || tier == TIER_F64 ||
                         (tier == TIER_MID && (s->pol.precision == HYDRO_PREC_FP8 || s->pol.rescore3)) ||
                         (tier == TIER_F32 && s->pol.precision != HYDRO_PREC_FP32);
        if (run) {
          Forward f = make_forward(s, tier, out_slot, src, n_seg, seg_len, fr.id_base);
          enqueue_tier(s, tier, src, f, st);
        }
        if (timed && ev[2 + ci]) hipEventRecord(ev[2 + ci], st);
      }
      if (host_mode && !host_rc)
        host_rc = host_round_decide(s, st, fr, s->theta_host.back().data(), n_seg, seg_len,
                                    make_forward(s, TIER_FIRST, out_slot, src, n_seg, seg_len, fr.id_base));
      if (s->rnn) router_nn_learn(s->rnn, s->st, st);
      parity ^= 1;
    }
    {
      FoldArgs fa{};
      fa.st = s->st;
      fa.k = s->K;
      fa.final_fold = 1;
      fa.alpha = s->pol.ewma_alpha;
      fa.static_cost = s->pol.cost_source == HYDRO_COST_STATIC;
      for (int j = 0; j < s->K; ++j) fa.flops[j] = s->models[j].flops;
      hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, st, fa);
    }
    // ordered result materialisation for this push
    if (nwords > 0) {
      const int nb = (int)((nwords + 255) / 256);
      hipLaunchKernelGGL(k_res_count, dim3(nb), dim3(256), 0, st, s->result_bits, nwords, s->res_blocks);
      hipLaunchKernelGGL(k_res_scan, dim3(1), dim3(1024), 0, st, s->res_blocks, nb, s->st, s->res_base);
      hipLaunchKernelGGL(k_res_write, dim3(nb), dim3(256), 0, st, s->result_bits, nwords, s->res_blocks, fr.id_base,
                         s->out_ids);
    }
  };

  const bool graphable = s->pol.use_graph && fr.where == HYDRO_MEM_DEVICE && !timing && !host_mode;
  if (graphable) {
    GraphKey key{n, src.base, fr.id_base, n_seg, seg_len, (int)warm_now, parity0, learned_from, s->theta, s->out_ids};
    hipGraphExec_t exec = nullptr;
    for (auto& e : s->graphs)
      if (e.first == key) exec = e.second;
    if (!exec) {
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      enqueue_push(false);
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamEndCapture(st, &graph));
      hipError_t he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (he != hipSuccess) return fail(HYDRO_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
      if (s->graphs.size() >= 8) {
        hipGraphExecDestroy(s->graphs.front().second);
        s->graphs.erase(s->graphs.begin());
      }
      s->graphs.push_back({key, exec});
    }
    HIP_TRY(hipGraphLaunch(exec, st));
  } else {
    enqueue_push(timing);
    if (host_rc) return host_rc;
  }
  if (warm_now) s->warmed = true;
  s->parity = parity0 ^ (n_rounds & 1);
  s->rounds_done += n_rounds;
  if (fr.where == HYDRO_MEM_HOST) HIP_TRY(hipEventRecord(s->stage_free[s->stage_next ^ 1], st));
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

// Wait for the query, copy its ids and fill the statistics.  The ids go to a malloc'd array
// (*alloc_out) or, when `dst` is given, into the caller's host array of dst_cap ids (ECAPACITY,
// with *out_n = the result size, when it is too small).
static int finish_query(hydro_session* s, int64_t** alloc_out, int64_t* dst, int64_t dst_cap, int64_t* out_n,
                        hydro_pred_stats* out_stats) {
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipGetLastError());
  DevState h;
  HIP_TRY(hipMemcpy(&h, s->st, sizeof(DevState), hipMemcpyDeviceToHost));
  if (h.overflow) return fail(HYDRO_EDEVICE, "internal: a launch held more evaluations than its activation buffers");
  const int64_t nres = h.n_result;
  int64_t* ids = dst;
  if (dst) {
    if (nres > dst_cap) {
      *out_n = nres;
      return fail(HYDRO_ECAPACITY, "the result holds " + std::to_string(nres) + " ids, the output array " +
                                       std::to_string(dst_cap));
    }
  } else {
    ids = (int64_t*)malloc(std::max<int64_t>(1, nres) * sizeof(int64_t));
    if (!ids) return fail(HYDRO_ENOMEM, "host allocation of the result failed");
  }
  if (nres > 0) {
    hipError_t he = hipMemcpy(ids, s->out_ids, nres * sizeof(int64_t), hipMemcpyDeviceToHost);
    if (he != hipSuccess) {
      if (!dst) free(ids);
      return fail(HYDRO_EDEVICE, std::string("result copy: ") + hipGetErrorString(he));
    }
  }
  if (!s->ids_sorted) std::sort(ids, ids + nres);
  if (s->pol.time_kernels) {
    // events were recorded in groups of kEvPerRound per round: start, routed, first, mid, f32, f64
    double tr = 0, t1 = 0, tm = 0, t2 = 0, t3 = 0;
    int nr = 0;
    for (int i = 0; i + kEvPerRound - 1 < s->ev_used; i += kEvPerRound) {
      float a = 0, b = 0, m = 0, c = 0, d = 0;
      if (hipEventElapsedTime(&a, s->evpool[i], s->evpool[i + 1]) != hipSuccess) continue;
      hipEventElapsedTime(&b, s->evpool[i + 1], s->evpool[i + 2]);
      hipEventElapsedTime(&m, s->evpool[i + 2], s->evpool[i + 3]);
      hipEventElapsedTime(&c, s->evpool[i + 3], s->evpool[i + 4]);
      hipEventElapsedTime(&d, s->evpool[i + 4], s->evpool[i + 5]);
      tr += a; t1 += b; tm += m; t2 += c; t3 += d;
      ++nr;
    }
    s->info.route_ms = tr;
    s->info.first_pass_ms = t1;
    s->info.mid_pass_ms = tm;
    s->info.f32_pass_ms = t2;
    s->info.f64_pass_ms = t3;
    s->info.timed_rounds = nr;
  }
  auto t1 = std::chrono::steady_clock::now();
  s->info.n_result = nres;
  s->info.rounds = h.rounds;
  s->info.k = s->K;
  s->info.learned_routed = h.learned_routed;
  s->info.learned_stale = h.learned_stale;
  s->info.stats_routed = h.stats_routed;
  s->info.learned_active = h.learned_active;
  s->info.train_steps = h.train_steps;
  for (int a = 0; a < 2; ++a) {
    s->info.arm_flops[a] = h.arm_cost[a];
    s->info.arm_tuples[a] = h.arm_tuples[a];
  }
  s->info.elapsed_us = s->pushes ? std::chrono::duration<double, std::micro>(t1 - s->t_start).count() : 0.0;
  if (out_stats) {
    for (int k = 0; k < s->K; ++k) {
      hydro_pred_stats& o = out_stats[k];
      o.evaluated = h.t_eval[k];
      o.passed = h.t_pass[k];
      o.rescored = h.t_rescored[k];
      o.escalated = h.t_esc[k];
      o.rescored16 = h.t_mid[k];
      o.cache_hits = h.t_hit[k];
      o.device_us = (double)h.t_ticks[k] * s->tick_us;
      o.cost_us_per_tuple = s->pol.cost_source == HYDRO_COST_STATIC ? h.cost_est[k] : h.cost_est[k] * s->tick_us;
      o.selectivity = h.t_eval[k] ? (double)h.t_pass[k] / (double)h.t_eval[k] : 0.0;
    }
  }
  if (alloc_out) *alloc_out = ids;
  *out_n = nres;
  s->theta_host.clear();
  s->crops_host.clear();
  s->in_query = false;
  return HYDRO_OK;
}

int hydro_session_finish(hydro_session* s, int64_t** out_ids, int64_t* out_n, hydro_pred_stats* out_stats) {
  g_err.clear();
  if (out_ids) *out_ids = nullptr;
  if (out_n) *out_n = 0;
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  if (!out_ids || !out_n) return fail(HYDRO_EINVAL, "out_ids / out_n is NULL");
  return finish_query(s, out_ids, nullptr, 0, out_n, out_stats);
}

int hydro_session_info(const hydro_session* s, hydro_query_info* out) {
  if (!s || !out) return fail(HYDRO_EINVAL, "NULL argument");
  *out = s->info;
  return HYDRO_OK;
}

int hydro_session_routes(const hydro_session* s, int64_t first_id, int64_t n, uint32_t* out) {
  if (!s || !out) return fail(HYDRO_EINVAL, "NULL argument");
  if (!s->route_log) return fail(HYDRO_ESTATE, "session was created without log_routes");
  if (first_id < 0 || n < 0 || first_id + n > s->last_push_n) return fail(HYDRO_EINVAL, "range outside the last push");
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(out, s->route_log + first_id, n * 4, hipMemcpyDeviceToHost));
  return HYDRO_OK;
}

int hydro_session_round_log(const hydro_session* s, int32_t first, int32_t n, hydro_round_record* out) {
  if (!s || !out) return fail(HYDRO_EINVAL, "NULL argument");
  if (!s->round_log) return fail(HYDRO_ESTATE, "session was created without log_routes");
  const int64_t have = std::min<int64_t>(s->info.rounds, s->round_log_cap);
  if (first < 0 || n < 0 || (int64_t)first + n > have) return fail(HYDRO_EINVAL, "range outside the recorded rounds");
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (n > 0) HIP_TRY(hipMemcpy(out, s->round_log + first, (size_t)n * sizeof(hydro_round_record), hipMemcpyDeviceToHost));
  return HYDRO_OK;
}

int hydro_session_logits(hydro_session* s, int32_t pred, int32_t tier, const hydro_frames* frames, double* out_logits) {
  g_err.clear();
  if (!s || !frames || !out_logits) return fail(HYDRO_EINVAL, "NULL argument");
  if (pred < 0 || pred >= s->K) return fail(HYDRO_EINVAL, "predicate index out of range");
  if (tier < 0 || tier > 3) return fail(HYDRO_EINVAL, "tier must be 0, 1, 2 or 3");
  if (s->models[pred].m.arch == HYDRO_ARCH_HOST) return fail(HYDRO_EUNSUPPORTED, "a HOST predicate has no logits");
  if (s->models[pred].m.on_crop) return fail(HYDRO_EUNSUPPORTED, "an on_crop predicate takes crops: no whole-frame logits");
  if (tier == 3 && s->pol.precision != HYDRO_PREC_FP8 && !s->pol.rescore3)
    tier = s->pol.precision == HYDRO_PREC_BF16 ? 0 : 1;
  if (s->in_query)
    return fail(HYDRO_ESTATE, "a query is in progress (pushes since the last reset / finish): logits and "
                              "calibration run between queries");
  const hydro_frames& fr = *frames;
  if (fr.where != HYDRO_MEM_DEVICE) return fail(HYDRO_EUNSUPPORTED, "logits take device frames");
  if (fr.n <= 0 || fr.n > s->max_push) return fail(HYDRO_ECAPACITY, "tuple count outside 1..max_push");
  if (fr.h != s->fh || fr.w != s->fw || !fr.data) return fail(HYDRO_EINVAL, "frame shape or data");
  int rc = ensure_dtype(s, fr.dtype);
  if (rc) return rc;
  hipStream_t st = s->stream;
  HIP_TRY(hipStreamSynchronize(st));
  const int t = tier == 0 ? TIER_FIRST : tier == 1 ? TIER_F32 : tier == 2 ? TIER_F64 : TIER_MID;
  // queue of every tuple for this predicate at the chosen tier
  std::vector<uint32_t> ent(fr.n);
  for (int64_t i = 0; i < fr.n; ++i) ent[i] = make_entry((uint32_t)i, 0u);
  uint32_t* qbase = t == TIER_FIRST ? s->q1 : t == TIER_F32 ? s->q2 : t == TIER_MID ? s->qm : s->q3;
  int* cptr = t == TIER_FIRST ? s->st->qcount : t == TIER_F32 ? s->st->bcount
              : t == TIER_MID ? s->st->mcount : s->st->ecount;
  // layer-wise CNN launches hold activations for at most act_cap queued evaluations
  const int64_t chunk = s->gcnn.n_preds > 0 ? std::max<int64_t>(1, s->act_cap) : fr.n;
  double* dlog;
  const size_t arena_mark = s->arena_used;   // allocation-free sessions: a temporary arena slice
  if (s->arena) {
    if ((rc = sess_alloc(s, (void**)&dlog, fr.n * kClasses * sizeof(double)))) return rc;
  } else {
    HIP_TRY(hipMalloc(&dlog, fr.n * kClasses * sizeof(double)));
  }
  FrameSrc src{fr.data, fr.dtype, fr.h, (int64_t)fr.h * fr.w * 3};
  Forward f = make_forward(s, t, 0, src, 1, 1, 0);
  f.logits = dlog;
  f.cache = ResultCache{};
  f.defer = Queues{nullptr, nullptr, 0};
  hipError_t he = hipSuccess;
  for (int64_t i0 = 0; i0 < fr.n && he == hipSuccess; i0 += chunk) {
    const int64_t m = std::min(chunk, fr.n - i0);
    DevState zero{};
    int cnt[kMaxK] = {0};
    cnt[pred] = (int)m;
    he = hipMemcpy(qbase + (int64_t)pred * s->cap, ent.data() + i0, m * 4, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(s->st, &zero, sizeof(DevState), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(cptr, cnt, sizeof(cnt), hipMemcpyHostToDevice);
    if (he == hipSuccess) {
      enqueue_tier(s, t, src, f, st);
      he = hipStreamSynchronize(st);
    }
  }
  if (he == hipSuccess) he = hipMemcpy(out_logits, dlog, fr.n * kClasses * sizeof(double), hipMemcpyDeviceToHost);
  if (s->arena) s->arena_used = arena_mark;
  else hipFree(dlog);
  if (he != hipSuccess) return fail(HYDRO_EDEVICE, std::string("logits: ") + hipGetErrorString(he));
  // leave the session ready for a new query
  return hydro_session_reset(s);
}

static double host_margin(const double* z, uint32_t mask) {
  double in = -INFINITY, out = -INFINITY;
  for (int c = 0; c < kClasses; ++c) {
    if ((mask >> c) & 1u) in = std::max(in, z[c]);
    else out = std::max(out, z[c]);
  }
  return in - out;
}

// Largest first-pass, BF16 (FP8 sessions) and FP32 margin errors against the FP64 tier on
// `frames` (device memory), times `safety`, floored at 1e-4 / 1e-4 / 1e-6.
static int measure_bands(hydro_session* s, const hydro_frames* frames, float safety, float* tau, float* tau16,
                         float* tau32) {
  const int64_t n = frames->n;
  if (n < 1) return fail(HYDRO_EINVAL, "calibration needs at least one frame");
  // frames beyond the session's push capacity are taken in blocks of that size
  const int64_t blk = std::min<int64_t>(n, s->cap);
  const int esize = frames->dtype == HYDRO_DTYPE_F32 ? 4 : frames->dtype == HYDRO_DTYPE_BF16 ? 2 : 1;
  const int64_t fbytes = (int64_t)frames->h * frames->w * 3 * esize;
  const bool f8 = s->pol.precision == HYDRO_PREC_FP8 || s->pol.rescore3;   // a middle tier
  std::vector<double> z0((size_t)blk * kClasses), zm((size_t)blk * kClasses), z1((size_t)blk * kClasses),
      z2((size_t)blk * kClasses);
  for (int k = 0; k < s->K; ++k) {
    if (s->models[k].m.arch == HYDRO_ARCH_HOST || s->models[k].m.on_crop) {   // exact decisions: no band
      tau[k] = tau16[k] = tau32[k] = 0.f;
      continue;
    }
    const uint32_t mask = s->models[k].m.class_mask;
    double e0 = 0, em = 0, e1 = 0;
    for (int64_t i0 = 0; i0 < n; i0 += blk) {
      hydro_frames sub = *frames;
      sub.data = static_cast<const char*>(frames->data) + i0 * fbytes;
      sub.n = std::min(blk, n - i0);
      int rc;
      if ((rc = hydro_session_logits(s, k, 0, &sub, z0.data()))) return rc;
      if (f8 && (rc = hydro_session_logits(s, k, 3, &sub, zm.data()))) return rc;
      if ((rc = hydro_session_logits(s, k, 1, &sub, z1.data()))) return rc;
      if ((rc = hydro_session_logits(s, k, 2, &sub, z2.data()))) return rc;
      for (int64_t i = 0; i < sub.n; ++i) {
        const double d2 = host_margin(&z2[i * kClasses], mask);
        if (!std::isfinite(d2)) continue;
        e0 = std::max(e0, std::fabs(host_margin(&z0[i * kClasses], mask) - d2));
        if (f8) em = std::max(em, std::fabs(host_margin(&zm[i * kClasses], mask) - d2));
        e1 = std::max(e1, std::fabs(host_margin(&z1[i * kClasses], mask) - d2));
      }
    }
    // floors keep a band even when the sample shows (almost) no error
    tau[k] = (float)std::max(safety * e0, 1e-4);
    tau16[k] = (float)std::max(safety * em, 1e-4);
    tau32[k] = (float)std::max(safety * e1, 1e-6);
  }
  return HYDRO_OK;
}

// FP8 sessions: each 4-layer CNN predicate's activation scales (outputs of layers 1..3), from the
// largest activations of its FP32 tier on `frames` (device memory): the largest maps to 224, half
// of e4m3's largest finite value, which leaves headroom for frames beyond the sample (larger values
// saturate at 448).
static int measure_ascales(hydro_session* s, const hydro_frames* frames) {
  const int64_t n = frames->n;
  if (n < 1) return fail(HYDRO_EINVAL, "calibration needs at least one frame");
  if (s->in_query) return fail(HYDRO_ESTATE, "calibration runs between queries");
  int rc = ensure_dtype(s, frames->dtype);
  if (rc) return rc;
  unsigned* dmax = nullptr;
  const size_t mark = s->arena_used;
  const size_t bytes = (size_t)kMaxK * 4 * sizeof(unsigned);
  if (s->arena) {
    if ((rc = sess_alloc(s, (void**)&dmax, bytes))) return rc;
  } else {
    HIP_TRY(hipMalloc(&dmax, bytes));
  }
  auto release = [&]() {
    s->gcnn.c4_act_max = nullptr;
    if (s->arena) s->arena_used = mark;
    else hipFree(dmax);
  };
  hipError_t he = hipMemsetAsync(dmax, 0, bytes, s->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(s->stream);
  if (he != hipSuccess) {
    release();
    return fail(HYDRO_EDEVICE, std::string("activation maxima: ") + hipGetErrorString(he));
  }
  s->gcnn.c4_act_max = dmax;
  const int64_t blk = std::min<int64_t>(n, s->cap);
  const int esize = frames->dtype == HYDRO_DTYPE_F32 ? 4 : frames->dtype == HYDRO_DTYPE_BF16 ? 2 : 1;
  const int64_t fbytes = (int64_t)frames->h * frames->w * 3 * esize;
  std::vector<double> z((size_t)blk * kClasses);
  for (int k = 0; k < s->K && !rc; ++k)
    for (int64_t i0 = 0; i0 < n && !rc; i0 += blk) {
      hydro_frames sub = *frames;
      sub.data = static_cast<const char*>(frames->data) + i0 * fbytes;
      sub.n = std::min(blk, n - i0);
      rc = hydro_session_logits(s, k, 1, &sub, z.data());
    }
  unsigned hmax[kMaxK * 4];
  if (!rc) {
    he = hipMemcpy(hmax, dmax, bytes, hipMemcpyDeviceToHost);
    if (he != hipSuccess) rc = fail(HYDRO_EDEVICE, std::string("activation maxima: ") + hipGetErrorString(he));
  }
  release();
  if (rc) return rc;
  GcnnArgs& ga = s->gcnn;
  for (int i = 0; i < ga.n_preds; ++i) {
    if (!ga.c4[i]) continue;
    for (int l = 0; l < 3; ++l) {
      float mx;
      memcpy(&mx, &hmax[ga.pred[i] * 4 + l], 4);
      ga.c4_ascale[i][l] = mx > 0.f ? mx / 224.f : 1.f;
    }
  }
  s->ascales_set = true;
  drop_graphs(s);
  return HYDRO_OK;
}

int hydro_session_calibrate(hydro_session* s, const hydro_frames* frames, float safety, float* out_tau,
                            float* out_tau32) {
  g_err.clear();
  if (!s || !frames) return fail(HYDRO_EINVAL, "NULL argument");
  if (!(safety >= 1.f)) return fail(HYDRO_EINVAL, "safety must be at least 1");
  if (s->in_query)
    return fail(HYDRO_ESTATE, "a query is in progress (pushes since the last reset / finish): calibrate "
                              "between queries");
  float tau[kMaxK], tau16[kMaxK], tau32[kMaxK];
  int rc = HYDRO_OK;
  if (s->pol.precision == HYDRO_PREC_FP8) rc = measure_ascales(s, frames);
  if (!rc) rc = measure_bands(s, frames, safety, tau, tau16, tau32);
  if (rc) return rc;
  for (int k = 0; k < s->K; ++k) {
    s->tau_k[k] = s->pol.precision != HYDRO_PREC_FP32 ? tau[k] : tau32[k];
    s->tau16_k[k] = tau16[k];
    s->tau32_k[k] = tau32[k];
    if (out_tau) out_tau[k] = s->tau_k[k];
    if (out_tau32) out_tau32[k] = tau32[k];
  }
  s->auto_tau = s->auto_tau32 = s->auto_tau16 = false;
  drop_graphs(s);   // captured pushes hold the old bands in their kernel arguments
  return HYDRO_OK;
}

int hydro_session_bands(const hydro_session* s, float* tau, float* tau16, float* tau32) {
  g_err.clear();
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  for (int k = 0; k < s->K; ++k) {
    if (tau) tau[k] = s->tau_k[k];
    if (tau16) tau16[k] = s->tau16_k[k];
    if (tau32) tau32[k] = s->tau32_k[k];
  }
  return HYDRO_OK;
}

int hydro_session_cache_clear(hydro_session* s) {
  g_err.clear();
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  if (!s->cache.keys) return fail(HYDRO_ESTATE, "the session keeps no result cache (policy.reuse = 0)");
  if (s->in_query) return fail(HYDRO_ESTATE, "a query is open (push without finish)");
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemset(s->cache.keys, 0xFF, ((size_t)s->K << s->cache.log2) * sizeof(unsigned long long)));
  return HYDRO_OK;
}

int hydro_session_router_params(const hydro_session* s, float* out, int32_t n) {
  g_err.clear();
  if (!s || !out) return fail(HYDRO_EINVAL, "session or out is NULL");
  if (!s->rnn) return fail(HYDRO_ESTATE, "the session has no learned router");
  if (n < router_nn_param_count()) return fail(HYDRO_EINVAL, "out holds fewer values than the router has parameters");
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(out, router_nn_params_ptr(s->rnn), sizeof(float) * router_nn_param_count(), hipMemcpyDeviceToHost));
  return HYDRO_OK;
}

int hydro_session_set_order(hydro_session* s, const int32_t* order) {
  g_err.clear();
  if (!s || !order) return fail(HYDRO_EINVAL, "NULL argument");
  if (s->in_query) return fail(HYDRO_ESTATE, "a query is in progress: change the order between queries");
  unsigned seen = 0;
  for (int i = 0; i < s->K; ++i) {
    const int o = order[i];
    if (o < 0 || o >= s->K || (seen >> o) & 1u) return fail(HYDRO_EINVAL, "order is not a permutation of 0..K-1");
    seen |= 1u << o;
  }
  for (int i = 0; i < s->K; ++i) s->pol.order[i] = order[i];
  drop_graphs(s);   // the order is a launch argument of the captured fold kernels
  return HYDRO_OK;
}

int hydro_session_set_route(hydro_session* s, int32_t route) {
  g_err.clear();
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  if (s->in_query) return fail(HYDRO_ESTATE, "a query is in progress: change the route between queries");
  if (route < HYDRO_ROUTE_FIXED || route > HYDRO_ROUTE_COST)
    return fail(route == HYDRO_ROUTE_LEARNED ? HYDRO_EUNSUPPORTED : HYDRO_EINVAL,
                "route must be FIXED, SEL, SCORE or COST (the learned router is chosen at session creation)");
  if (s->pol.route == HYDRO_ROUTE_LEARNED) return fail(HYDRO_EUNSUPPORTED, "a learned-router session keeps its route");
  s->pol.route = route;
  drop_graphs(s);   // the route is a launch argument of the captured fold and route kernels
  return HYDRO_OK;
}

int hydro_session_destroy(hydro_session* s) {
  if (!s) return fail(HYDRO_EINVAL, "session is NULL");
  free_session(s);
  return HYDRO_OK;
}

int hydro_query(const hydro_frames* frames, const hydro_model* models, int32_t k, const float* thresholds,
                int32_t n_seg, int64_t seg_len, const hydro_policy* policy, int64_t** out_ids, int64_t* out_n,
                hydro_pred_stats* out_stats) {
  if (out_ids) *out_ids = nullptr;
  if (out_n) *out_n = 0;
  if (!frames) return fail(HYDRO_EINVAL, "frames is NULL");
  if (!out_ids || !out_n) return fail(HYDRO_EINVAL, "out_ids / out_n is NULL");
  hydro_session* s = nullptr;
  int rc = hydro_session_create(models, k, policy, frames->h, frames->w, std::max<int64_t>(1, frames->n), &s);
  if (rc) return rc;
  rc = hydro_session_push(s, frames, thresholds, n_seg, seg_len);
  if (!rc) rc = hydro_session_finish(s, out_ids, out_n, out_stats);
  std::string err = g_err;
  hydro_session_destroy(s);
  g_err = err;
  return rc;
}

int hydro_query_noalloc(const hydro_frames* frames, const hydro_model* models, int32_t k, const float* thresholds,
                        int32_t n_seg, int64_t seg_len, const hydro_policy* policy, int64_t* out_ids, int64_t out_cap,
                        int64_t* out_n, hydro_pred_stats* out_stats) {
  g_err.clear();
  if (out_n) *out_n = 0;
  if (!frames || !policy || !out_n) return fail(HYDRO_EINVAL, "frames / policy / out_n is NULL");
  if (out_cap < 0 || (out_cap > 0 && !out_ids)) return fail(HYDRO_EINVAL, "out_ids is NULL or out_cap negative");
  if (frames->where != HYDRO_MEM_DEVICE) return fail(HYDRO_EUNSUPPORTED, "allocation-free queries take device frames");
  if (policy->use_graph || policy->autotune || policy->time_kernels)
    return fail(HYDRO_EUNSUPPORTED, "allocation-free queries run without graphs, autotuning or kernel timing");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  unsigned char* arena = nullptr;
  int rc = scratch_ptr(dev, &arena);
  if (rc) return rc;
  hydro_session* s = nullptr;
  rc = session_create(models, k, policy, frames->h, frames->w, std::max<int64_t>(1, frames->n), arena,
                      HYDRO_NOALLOC_BYTES, &s);
  if (rc) return rc;
  rc = hydro_session_push(s, frames, thresholds, n_seg, seg_len);
  if (!rc) rc = finish_query(s, nullptr, out_ids, out_cap, out_n, out_stats);
  std::string err = g_err;
  hydro_session_destroy(s);
  g_err = err;
  return rc;
}


int hydro_compaction_debug(int32_t k, int64_t n, const uint32_t* pass_bits, int32_t route, int32_t wave,
                           int64_t* out_ids, int64_t* out_n, hydro_pred_stats* out_stats, double* out_ms) {
  g_err.clear();
  if (out_n) *out_n = 0;
  if (k < 1 || k > kMaxK) return fail(HYDRO_EUNSUPPORTED, "K must be 1..8");
  if (n < 0 || n > ((int64_t)1 << 30)) return fail(HYDRO_EINVAL, "n must be in 0 .. 2^30");
  if (!out_n || (n > 0 && (!pass_bits || !out_ids))) return fail(HYDRO_EINVAL, "pass_bits / out_ids / out_n is NULL");
  if (route < HYDRO_ROUTE_FIXED || route > HYDRO_ROUTE_COST) return fail(HYDRO_EINVAL, "route must be FIXED, SEL, SCORE or COST");
  if (wave < 64 || wave > (1 << kIdxBits)) return fail(HYDRO_EINVAL, "wave must be in 64 .. 2^24");
  const int64_t block = std::min<int64_t>(n, (int64_t)1 << kIdxBits);   // tuples per push
  const int64_t row_words = (n + 31) / 32;
  const int64_t bwords = (block + 31) / 32;
  const int nb_res = (int)std::max<int64_t>(1, (bwords + 255) / 256);
  int dev = 0, n_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  // device state: DevState, two live lists, K queues, result bitmap, scan blocks
  struct Bufs {
    std::vector<void*> p;
    ~Bufs() { for (void* q : p) hipFree(q); }
  } bufs;
  auto alloc = [&](size_t bytes, void** out) -> int {
    hipError_t he = dev_alloc(out, std::max<size_t>(bytes, 16));
    if (he != hipSuccess) return fail(HYDRO_ENOMEM, "compaction buffers: allocation failed");
    bufs.p.push_back(*out);
    return HYDRO_OK;
  };
  DevState* st = nullptr;
  uint32_t *pend[2] = {nullptr, nullptr}, *q = nullptr, *rbits = nullptr;
  int *res_blocks = nullptr, *res_base = nullptr;
  int rc;
  if ((rc = alloc(sizeof(DevState), (void**)&st)) || (rc = alloc(block * 4, (void**)&pend[0])) ||
      (rc = alloc(block * 4, (void**)&pend[1])) || (rc = alloc((size_t)k * block * 4, (void**)&q)) ||
      (rc = alloc(bwords * 4, (void**)&rbits)) || (rc = alloc((size_t)nb_res * 4, (void**)&res_blocks)) ||
      (rc = alloc(16, (void**)&res_base)))
    return rc;
  hipStream_t s = nullptr;
  HIP_TRY(hipStreamCreate(&s));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { hipStreamSynchronize(s); hipStreamDestroy(s); }
  } sg{s};
  std::vector<hipEvent_t> evs;
  struct EventGuard {
    std::vector<hipEvent_t>* v;
    ~EventGuard() { for (hipEvent_t e : *v) hipEventDestroy(e); }
  } eg{&evs};
  auto mark = [&](hipEvent_t* e) -> int {
    HIP_TRY(hipEventCreate(e));
    evs.push_back(*e);
    HIP_TRY(hipEventRecord(*e, s));
    return HYDRO_OK;
  };
  HIP_TRY(hipMemsetAsync(st, 0, sizeof(DevState), s));
  // phase brackets: (start, end, phase) with phase 0 = fold + route, 1 = decide, 2 = results
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> spans;
  hipEvent_t t0, t1;
  if ((rc = mark(&t0))) return rc;
  int parity = 0;
  for (int64_t id_base = 0; id_base < n; id_base += block) {
    const int64_t m = std::min<int64_t>(block, n - id_base);
    const int64_t mwords = (m + 31) / 32;
    hipEvent_t a, b;
    if ((rc = mark(&a))) return rc;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>(1024, (mwords + 255) / 256)), dim3(256), 0, s,
                       rbits, 0u, mwords);
    if ((rc = mark(&b))) return rc;
    spans.push_back({{a, b}, 2});
    const int waves = (int)((m + wave - 1) / wave);
    const int n_rounds = waves + k - 1;
    for (int r = 0; r < n_rounds; ++r) {
      const int in_slot = parity, out_slot = parity ^ 1;
      FoldArgs fa{};
      fa.st = st;
      fa.k = k;
      fa.route = route;
      for (int j = 0; j < k; ++j) {
        fa.order[j] = j;
        fa.flops[j] = 1.0;
      }
      fa.alpha = 0.5;
      fa.static_cost = 1;
      fa.out_slot = out_slot;
      if ((rc = mark(&a))) return rc;
      hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, s, fa);
      RouteArgs ra{};
      ra.st = st;
      ra.pend_in = pend[in_slot];
      ra.in_slot = in_slot;
      ra.adm_lo = r < waves ? (uint32_t)((int64_t)r * wave) : 0u;
      ra.adm_hi = r < waves ? (uint32_t)std::min<int64_t>(m, (int64_t)(r + 1) * wave) : 0u;
      ra.routing_batch = 64;
      ra.k = k;
      ra.q = Queues{q, st->qcount, block};
      hipLaunchKernelGGL(k_route, dim3(n_cu * kRouteBlocksPerCu), dim3(kRouteThreads), 0, s, ra);
      if ((rc = mark(&b))) return rc;
      spans.push_back({{a, b}, 0});
      Forward f{};
      f.st = st;
      f.pend_out = pend[out_slot];
      f.pend_out_count = &st->pend_count[out_slot];
      f.result_bits = rbits;
      f.id_base = id_base;
      f.full_mask = (1u << k) - 1u;
      f.k_total = k;
      f.count_eval = 1;
      hipLaunchKernelGGL(k_table_decide, dim3(n_cu * 8), dim3(kRouteThreads), 0, s, Queues{q, st->qcount, block}, k,
                         pass_bits, row_words, f);
      if ((rc = mark(&a))) return rc;
      spans.push_back({{b, a}, 1});
      parity ^= 1;
    }
    if ((rc = mark(&a))) return rc;
    const int nb = (int)((mwords + 255) / 256);
    hipLaunchKernelGGL(k_res_count, dim3(nb), dim3(256), 0, s, rbits, mwords, res_blocks);
    hipLaunchKernelGGL(k_res_scan, dim3(1), dim3(1024), 0, s, res_blocks, nb, st, res_base);
    hipLaunchKernelGGL(k_res_write, dim3(nb), dim3(256), 0, s, rbits, mwords, res_blocks, id_base, out_ids);
    if ((rc = mark(&b))) return rc;
    spans.push_back({{a, b}, 2});
  }
  {
    FoldArgs fa{};
    fa.st = st;
    fa.k = k;
    fa.final_fold = 1;
    fa.alpha = 0.5;
    fa.static_cost = 1;
    for (int j = 0; j < k; ++j) fa.flops[j] = 1.0;
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, s, fa);
  }
  if ((rc = mark(&t1))) return rc;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  DevState h{};
  HIP_TRY(hipMemcpy(&h, st, sizeof(DevState), hipMemcpyDeviceToHost));
  if (out_ms) {
    double ph[3] = {0, 0, 0};
    for (auto& sp : spans) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, sp.first.first, sp.first.second));
      ph[sp.second] += ms;
    }
    float tot = 0.f;
    HIP_TRY(hipEventElapsedTime(&tot, t0, t1));
    out_ms[0] = ph[0];
    out_ms[1] = ph[1];
    out_ms[2] = ph[2];
    out_ms[3] = tot;
  }
  if (out_stats) {
    for (int j = 0; j < k; ++j) {
      hydro_pred_stats ps{};
      ps.evaluated = h.t_eval[j];
      ps.passed = h.t_pass[j];
      ps.selectivity = h.t_eval[j] ? (double)h.t_pass[j] / (double)h.t_eval[j] : 0.0;
      out_stats[j] = ps;
    }
  }
  *out_n = h.n_result;
  return HYDRO_OK;
}

}  // extern "C"
