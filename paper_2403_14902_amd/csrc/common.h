// Shared device/host definitions of the gfx950 engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hydro.h"

namespace hydro {

constexpr int kMaxK = HYDRO_MAX_PREDICATES;
constexpr int kClasses = HYDRO_N_CLASSES;
constexpr int kWave = 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A queue entry packs a tuple's local index (within its push) and the set of predicates
// already evaluated on it (the per-tuple analogue of the visited table of section 3.3).
constexpr int kIdxBits = 24;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1;
__host__ __device__ inline uint32_t entry_idx(uint32_t e) { return e & kIdxMask; }
__host__ __device__ inline uint32_t entry_mask(uint32_t e) { return e >> kIdxBits; }
__host__ __device__ inline uint32_t make_entry(uint32_t idx, uint32_t mask) { return (mask << kIdxBits) | idx; }

// Kernel variants of the fused CNN (widths (16m, 32m, 64m) on 64x64x3 frames).
enum CnnVariant { CNN_W1 = 0, CNN_W2 = 1, CNN_W4 = 2, CNN_NONE = -1 };

// Per-predicate device descriptor (lives in device memory, built at session creation).
struct PredDesc {
  int arch;            // HYDRO_ARCH_*
  int variant;         // CnnVariant for CNNs
  int d_in, hidden;    // MLP
  int n_layers;
  int widths[HYDRO_MAX_LAYERS];
  int in_hw;
  uint32_t class_mask;
  float flops;
  // first-pass / FP32 weights, normalisation folded into layer 1 (see the packing code)
  const __bf16* w1_bf;     // MLP: [hidden][d_in] (n-major, k contiguous), bf16
  const float* w1_f32;     // MLP: [hidden][d_in], fp32
  const float* b1_fold;    // MLP: folded layer-1 bias, fp32
  const float* w2;         // MLP: [hidden][10] fp32 (canonical)
  const float* b2;         // MLP: [10]
  // CNN packed weights: per layer, MFMA-fragment order (see cnn.hip)
  const __bf16* cw_bf[HYDRO_MAX_LAYERS];
  const float* cw_f32[HYDRO_MAX_LAYERS];
  const float* cb_fold[HYDRO_MAX_LAYERS];   // bias (layer 1 folded), fp32
  const float* fc_w;       // [c_last][10] canonical fp32
  const float* fc_b;       // [10]
  // canonical fp32 weights for the FP64 tier (unfolded)
  const float* w1_canon;   // MLP [d_in][hidden]
  const float* b1_canon;
  const float* cw_canon[HYDRO_MAX_LAYERS];  // [co][ci][3][3]
  const float* cb_canon[HYDRO_MAX_LAYERS];
};

// Device-resident routing state and statistics (one per session).
struct DevState {
  // per-round accumulators (cleared by the fold kernel at the start of every round)
  unsigned long long r_eval[kMaxK], r_pass[kMaxK], r_ticks[kMaxK], r_rescored[kMaxK], r_esc[kMaxK], r_mid[kMaxK];
  // query totals
  unsigned long long t_eval[kMaxK], t_pass[kMaxK], t_ticks[kMaxK], t_rescored[kMaxK], t_esc[kMaxK], t_mid[kMaxK];
  double sel_est[kMaxK], cost_est[kMaxK];
  int seen[kMaxK];
  int order[kMaxK];            // predicate ranking used by this round's router
  int rounds;
  // queue counters
  int pend_count[2];
  int qcount[kMaxK];           // first-pass queues
  int bcount[kMaxK];           // FP32 re-score queues
  int ecount[kMaxK];           // FP64 escalation queues
  int mcount[kMaxK];           // BF16 re-score queues of an FP8 first pass
  int n_result;
  // learned router
  unsigned long long learned_routed, stats_routed;
  unsigned long long learned_stale;    // learned-arm decisions whose keys were not computed this
                                       // round (routed by the ranking instead)
  double arm_cost[2], arm_tuples[2];   // judge: realised UDF FLOPs and finished tuples per arm
  int learned_active;                  // 0 once the judge has fallen back to score routing
  int train_steps;
  unsigned long long ring_head;        // outcomes logged so far (ring index = head mod size)
  unsigned long long ring_trained;     // ring position the trainer has consumed up to
  int overflow;                        // set if a launch saw more evaluations than its buffers hold
  unsigned long long r_hit[kMaxK], t_hit[kMaxK];   // decisions taken from the result cache
};

// Which arm a routing batch belongs to: 1 = learned router, 0 = score routing (control).
__host__ __device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
  return x;
}
__host__ __device__ inline int arm_of(uint32_t batch, uint32_t seed, uint32_t control_below) {
  return mix32(batch ^ seed) >= control_below ? 1 : 0;
}

// Outcome log of the learned router: idx | k << 24 | rejected << 31.
struct OutcomeLog {
  uint32_t* ring;            // nullptr: no learned router
  uint32_t ring_mask;        // size - 1 (power of two)
  const float* flops;        // per predicate, for the judge's cost accounting
  uint32_t seed, control_below;
  int routing_batch;
};

// Where the frames of the current push live.
struct FrameSrc {
  const void* base;     // device pointer to tuple 0 of the push
  int dtype;            // hydro_dtype
  int hw;               // frame side
  int64_t elems;        // elements per frame (hw*hw*3)
};

// Device result cache (section 4.3, "Reuse-aware Routing": results of earlier queries reused
// instead of running the UDF).  One open-addressing table per predicate: keys[k << log2 | slot]
// is a global tuple id (kCacheEmpty when free), vals the decision taken on it: the threshold it
// was decided against (fp32 bits) and 1 for pass.  A decision "d > theta0 holds" also decides
// d > theta for every theta <= theta0, and "fails" for every theta >= theta0, so an entry answers
// exactly whenever the new threshold lies on the decided side; otherwise the tuple is evaluated.
constexpr unsigned long long kCacheEmpty = ~0ull;
constexpr int kCacheProbes = 16;
struct ResultCache {
  unsigned long long* keys;   // nullptr: no cache
  uint2* vals;
  uint32_t log2;
};

__device__ inline uint32_t cache_home(const ResultCache& c, unsigned long long id) {
  return (uint32_t)((id * 0x9E3779B97F4A7C15ull) >> (64 - c.log2));
}

// 0: no decisive entry; 1: cached pass; 2: cached fail (at threshold theta).
__device__ inline int cache_get(const ResultCache& c, int k, unsigned long long id, float theta) {
  const uint32_t mask = (1u << c.log2) - 1u;
  const uint32_t h = cache_home(c, id);
  const size_t row = (size_t)k << c.log2;
  for (int p = 0; p < kCacheProbes; ++p) {
    const size_t s = row + ((h + p) & mask);
    const unsigned long long key = c.keys[s];
    if (key == kCacheEmpty) return 0;
    if (key == id) {
      const uint2 v = c.vals[s];
      const float th = __uint_as_float(v.x);
      if (v.y && theta <= th) return 1;
      if (!v.y && theta >= th) return 2;
      return 0;
    }
  }
  return 0;
}

__device__ inline void cache_put(const ResultCache& c, int k, unsigned long long id, float theta, bool pass) {
  const uint32_t mask = (1u << c.log2) - 1u;
  const uint32_t h = cache_home(c, id);
  const size_t row = (size_t)k << c.log2;
  for (int p = 0; p < kCacheProbes; ++p) {
    const size_t s = row + ((h + p) & mask);
    const unsigned long long prev = atomicCAS(&c.keys[s], kCacheEmpty, id);
    if (prev == kCacheEmpty || prev == id) {
      c.vals[s] = make_uint2(__float_as_uint(theta), pass ? 1u : 0u);
      return;
    }
  }
}

// Queues of one tier: entries[k * cap + i], i < counts[k].
struct Queues {
  uint32_t* entries;
  int* counts;
  int64_t cap;
};

// Where deciding kernels send their decisions.
struct Forward {
  DevState* st;
  uint32_t* pend_out;        // survivors with predicates left
  int* pend_out_count;
  uint32_t* result_bits;     // completed tuples (bit per local index)
  uint32_t* route_log;       // optional
  Queues defer;              // next tier (band) queues; entries == nullptr for the last tier
  unsigned long long* defer_stat;   // per-predicate counter of deferred decisions
  float tau[kMaxK];          // per predicate: |d - theta| < tau defers to the next tier
  const float* theta;        // [n_seg][K]
  int n_seg;
  int64_t seg_len;
  int64_t id_base;
  int64_t seg_first;         // segment of local index 0 (id_base / seg_len)
  uint32_t seg_off;          // id_base mod seg_len
  uint32_t seg_len32;        // seg_len when below 2^31 (32-bit segment arithmetic), else 0
  uint32_t full_mask;        // (1 << K) - 1
  int k_total;
  int count_eval;            // 1 in the first pass (counts evaluated tuples)
  double* logits;            // if set: write fp64 logits [idx][10] instead of deciding
  OutcomeLog olog;
  ResultCache cache;         // decisions are recorded here when cache.keys is set
};

__device__ inline float theta_of(const Forward& f, int k, uint32_t idx) {
  int64_t s;
  if (f.seg_len32 != 0) s = f.seg_first + (int64_t)((f.seg_off + idx) / f.seg_len32);  // idx < 2^24
  else s = (f.id_base + (int64_t)idx) / f.seg_len;
  if (s >= f.n_seg) s = f.n_seg - 1;
  return f.theta[s * f.k_total + k];
}

// Cross-lane sums.  row_sum16: over the 16 lanes of each DPP row (lanes 16r..16r+15), by
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and row_mirror (each step adds a lane
// whose partial covers the complementary lanes, so every lane ends with the row total).
// wave_sum_n: all 64 lanes: the four row totals are read out of lanes 0, 16, 32, 48 (no LDS
// round trip) and added as (r0 + r1) + (r2 + r3); every lane ends with the same total.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ inline float row_sum16(float v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  return v;
}
__device__ inline float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <int N>
__device__ inline void wave_sum_n(float (&v)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] = row_sum16(v[c]);
#pragma unroll
  for (int c = 0; c < N; ++c)
    v[c] = (lane_value(v[c], 0) + lane_value(v[c], 16)) + (lane_value(v[c], 32) + lane_value(v[c], 48));
}

__device__ inline int lane_id() { return __lane_id(); }

// 16 bytes per lane from global memory straight into LDS (lane i at lds_off + 16 i), issued as
// one instruction per wave.  The asynchronous write is tracked by vmcnt; the caller waits for it
// explicitly with wait_vmcnt (the compiler does not see this LDS write, so it adds no waits of
// its own).  lds_off must be wave-uniform.
__device__ inline void lds_dma16(const void* src, uint32_t lds_off) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(lds_off)
               : "memory", "m0");
}
// s_waitcnt vmcnt(N) (other counters not waited for)
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Wave-aggregated append: every active lane with `want` set gets a unique slot in *counter.
__device__ inline int wave_append(int* counter, bool want) {
  unsigned long long m = __ballot(want);
  if (m == 0) return -1;
  int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader);
  unsigned long long below = m & ((1ull << lane_id()) - 1ull);
  return want ? base + __popcll(below) : -1;
}

__device__ inline void wave_add_u64(unsigned long long* counter, bool pred) {
  unsigned long long m = __ballot(pred);
  if (m != 0 && lane_id() == __ffsll((long long)m) - 1) atomicAdd(counter, (unsigned long long)__popcll(m));
}

// Margin d = max_{c in S} z_c - max_{c not in S} z_c (a max over no classes is -inf).
template <typename T>
__device__ inline T class_margin(const T* z, uint32_t mask) {
  T in = -__builtin_inf(), out = -__builtin_inf();
  for (int c = 0; c < kClasses; ++c) {
    if ((mask >> c) & 1u) in = z[c] > in ? z[c] : in;
    else out = z[c] > out ? z[c] : out;
  }
  return in - out;
}

// Record the decision on one (tuple, predicate) evaluation.  Called by every lane of a wave
// (lanes with active == false take part in the ballots only).
//   decided: pass / fail known at this tier;  pass: the decision;  defer: send to next tier.
__device__ inline void forward_decision(const Forward& f, int k, uint32_t e, bool active, bool defer, bool pass) {
  bool decided = active && !defer;
  if (f.count_eval) wave_add_u64(&f.st->r_eval[k], active);
  // next tier
  if (f.defer.entries != nullptr) {
    wave_add_u64(&f.defer_stat[k], active && defer);
    int slot = wave_append(&f.defer.counts[k], active && defer);
    if (active && defer) f.defer.entries[(int64_t)k * f.defer.cap + slot] = e;
  }
  bool ok = decided && pass;
  wave_add_u64(&f.st->r_pass[k], ok);
  uint32_t idx = entry_idx(e);
  if (f.cache.keys != nullptr && decided) cache_put(f.cache, k, (unsigned long long)(f.id_base + idx), theta_of(f, k, idx), pass);
  uint32_t mask = entry_mask(e) | (1u << k);
  if (decided && f.route_log != nullptr) {
    int step = __popc(entry_mask(e));
    f.route_log[idx] |= (uint32_t)(k + 1) << (4 * step);
  }
  bool done = ok && mask == f.full_mask;
  bool more = ok && mask != f.full_mask;
  if (f.olog.ring != nullptr) {
    // learned router: log the outcome; judge: UDF FLOPs spent and tuples finished per arm
    unsigned long long m = __ballot(decided);
    if (m != 0) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long base = 0;
      if (lane_id() == leader) base = atomicAdd(&f.st->ring_head, (unsigned long long)__popcll(m));
      base = __shfl(base, leader);
      if (decided) {
        unsigned long long pos = base + __popcll(m & ((1ull << lane_id()) - 1ull));
        f.olog.ring[pos & f.olog.ring_mask] = idx | ((uint32_t)k << 24) | (pass ? 0u : 0x80000000u);
      }
      const int arm = arm_of(idx / (uint32_t)f.olog.routing_batch, f.olog.seed, f.olog.control_below);
      const bool finished = decided && (!pass || done);
      for (int a = 0; a < 2; ++a) {
        const int ne = __popcll(__ballot(decided && arm == a));
        const int nf = __popcll(__ballot(finished && arm == a));
        if (lane_id() == leader) {
          if (ne) atomicAdd(&f.st->arm_cost[a], (double)ne * (double)f.olog.flops[k]);
          if (nf) atomicAdd(&f.st->arm_tuples[a], (double)nf);
        }
      }
    }
  }
  if (done) atomicOr(&f.result_bits[idx >> 5], 1u << (idx & 31));
  int slot = wave_append(f.pend_out_count, more);
  if (more) f.pend_out[slot] = make_entry(idx, mask);
}

}  // namespace hydro
