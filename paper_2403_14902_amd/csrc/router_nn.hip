// Learned content-based router (the idea of content-based routing, section 2.2 of the paper:
// route each tuple on attributes that correlate with predicate selectivity; the paper notes the
// per-tuple decision is too costly on CPUs, which a GPU kernel does not suffer).
//
// Features: the frame mean-pooled to 8x8x3 (192 values, normalised as the predicates normalise
// their input), computed once per tuple at admission.
// Model: MLP 192-64-K; output k estimates P(predicate k rejects the tuple).
// Inference (every round, on the live tuples): bf16 weights on MFMA, fp32 accumulation; the key
// of predicate k is cost_k / max(P(reject_k), 0.02), the per-tuple analogue of the score
// cost / (1 - selectivity); a tuple goes to its unvisited predicate with the smallest key.
// Training (every round): the outcomes the query itself logs (tuple, predicate, rejected), masked
// binary cross-entropy on the evaluated predicate only, fp32 forward/backward, Adam.
// Judge: routing batches are split by a hash into a control arm (score routing, a fraction
// `explore`) and the learned arm; both arms' realised UDF FLOPs per finished tuple are compared and
// the router falls back to score routing for good if it loses.
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "router_nn.h"

namespace hydro {

constexpr int RF = 192;           // features
constexpr int RH = 64;            // hidden units
constexpr int RK = 8;             // output slots (K <= 8)
constexpr int RING = 1 << 16;     // outcome log entries
constexpr int TB = 64;            // training minibatch
constexpr int TSTEPS = 2;         // optimiser steps per round (successive windows of the log)
constexpr int MIN_STEPS = 8;      // steps before the learned arm uses the router
constexpr int NPARAM = RF * RH + RH + RH * RK + RK;

struct RouterNN {
  int k, fh, fw, routing_batch;
  int64_t cap;
  uint64_t seed;
  float explore;
  bool external = false;          // buffers owned by the caller's allocator (not freed here)
  __bf16* feats = nullptr;        // [cap][192]
  float* keys = nullptr;          // [cap][K]
  uint32_t* stamps = nullptr;     // [cap]: round whose keys kernel wrote the tuple's keys
  uint32_t* ring = nullptr;
  float* params = nullptr;        // W1 [192][64] | b1 [64] | W2 [64][8] | b2 [8]
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  __bf16* w1_frag = nullptr;      // W1^T as MFMA A fragments [6 ksteps][4 ntiles][64][8]
  float* flops = nullptr;         // [K]
  std::vector<float> init;
};

// With `guard` set, a pooling launch does nothing unless the learned arm is routing (the keys
// of newly admitted tuples need their features before any predicate has seen the frame).
__device__ inline bool pool_skipped(const DevState* guard) {
  return guard != nullptr && (!guard->learned_active || guard->train_steps < MIN_STEPS);
}

// Any frame side divisible by 8: one thread per output feature (scalar loads).  Frames lo..lo+n-1.
__global__ void rnn_pool_kernel(FrameSrc fr, int64_t lo, int64_t n, __bf16* feats, const DevState* guard) {
  if (pool_skipped(guard)) return;
  const int64_t total = n * RF;
  const int blk = fr.hw / 8;
  const float inv = 1.0f / (float)(blk * blk);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = lo + q / RF;
    const int o = (int)(q % RF);
    const int by = o / 24, bx = (o / 3) % 8, c = o % 3;
    float s = 0.f;
    const int64_t base = t * fr.elems;
    for (int y = 0; y < blk; ++y)
      for (int x = 0; x < blk; ++x) {
        const int64_t e = base + ((int64_t)(by * blk + y) * fr.hw + bx * blk + x) * 3 + c;
        float v;
        if (fr.dtype == HYDRO_DTYPE_BF16) v = (float)static_cast<const __bf16*>(fr.base)[e];
        else if (fr.dtype == HYDRO_DTYPE_U8) v = (float)static_cast<const uint8_t*>(fr.base)[e] * (1.0f / 255.0f);
        else v = static_cast<const float*>(fr.base)[e];
        s += v;
      }
    feats[t * RF + o] = static_cast<__bf16>((s * inv - 0.5f) * 4.0f);
  }
}

template <typename T, int CH>
__device__ inline void load_chunk(const T* p, float (&v)[CH]) {
  if constexpr (sizeof(T) == 2) {
    static_assert(CH % 8 == 0 || CH == 4, "chunk");
    if constexpr (CH == 4) {
      const uint2 u = *reinterpret_cast<const uint2*>(p);
      const __bf16* h = reinterpret_cast<const __bf16*>(&u);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (float)h[e];
    } else {
      const uint4 u = *reinterpret_cast<const uint4*>(p);
      const __bf16* h = reinterpret_cast<const __bf16*>(&u);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (float)h[e];
    }
  } else if constexpr (sizeof(T) == 1) {
    if constexpr (CH == 4) {
      const uint32_t u = *reinterpret_cast<const uint32_t*>(p);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (float)((u >> (8 * e)) & 0xffu);
    } else {
      const uint2 u = *reinterpret_cast<const uint2*>(p);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (float)((u.x >> (8 * e)) & 0xffu);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 + e] = (float)((u.y >> (8 * e)) & 0xffu);
    }
  } else {
#pragma unroll
    for (int q = 0; q < CH / 4; ++q) {
      const float4 u = *reinterpret_cast<const float4*>(p + 4 * q);
      v[4 * q] = u.x;
      v[4 * q + 1] = u.y;
      v[4 * q + 2] = u.z;
      v[4 * q + 3] = u.w;
    }
  }
}

// One thread per (frame, 8x8 cell): the cell's rows are read as NCH vector chunks of CH elements
// (a cell row holds 3*hw/8 = NCH*CH values); per-position sums over the rows are folded into the
// three channel means at the end.  64 consecutive threads cover one frame, so each wave's loads
// walk whole frame rows.
template <typename T, int CH, int NCH>
__global__ __launch_bounds__(256) void rnn_pool_vec_kernel(FrameSrc fr, int64_t lo, int64_t n, __bf16* feats,
                                                           const DevState* guard) {
  if (pool_skipped(guard)) return;
  const int blk = fr.hw / 8;
  const int row_elems = fr.hw * 3;
  const float scale = (sizeof(T) == 1 ? 1.0f / 255.0f : 1.0f) / (float)(blk * blk);
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; (gid >> 6) < n;
       gid += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = lo + (gid >> 6);
    const int cell = (int)(gid & 63), by = cell >> 3, bx = cell & 7;
    const T* p = static_cast<const T*>(fr.base) + t * fr.elems + (int64_t)(by * blk) * row_elems + bx * (NCH * CH);
    float acc[NCH][CH];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int e = 0; e < CH; ++e) acc[c][e] = 0.f;
#pragma unroll 4
    for (int y = 0; y < blk; ++y) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        float v[CH];
        load_chunk<T, CH>(p + (int64_t)y * row_elems + c * CH, v);
#pragma unroll
        for (int e = 0; e < CH; ++e) acc[c][e] += v[e];
      }
    }
    float ch[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int e = 0; e < CH; ++e) ch[(c * CH + e) % 3] += acc[c][e];
    __bf16* o = feats + t * RF + by * 24 + bx * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = static_cast<__bf16>((ch[c] * scale - 0.5f) * 4.0f);
  }
}

template <typename T>
static bool launch_pool_vec(const FrameSrc& fr, int64_t lo, int64_t n, __bf16* feats, const DevState* guard,
                            hipStream_t s) {
  // guarded launches (most of which return at once) take a small grid and stride over the frames
  const int64_t blocks = std::min<int64_t>((n * 64 + 255) / 256, guard != nullptr ? 2048 : INT32_MAX);
  if (fr.hw == 32) {
    hipLaunchKernelGGL((rnn_pool_vec_kernel<T, 4, 3>), dim3((unsigned)blocks), dim3(256), 0, s, fr, lo, n, feats, guard);
  } else if (fr.hw == 64) {
    hipLaunchKernelGGL((rnn_pool_vec_kernel<T, 8, 3>), dim3((unsigned)blocks), dim3(256), 0, s, fr, lo, n, feats, guard);
  } else if (fr.hw == 128) {
    hipLaunchKernelGGL((rnn_pool_vec_kernel<T, 8, 6>), dim3((unsigned)blocks), dim3(256), 0, s, fr, lo, n, feats, guard);
  } else {
    return false;
  }
  return true;
}

struct KeyArgs {
  DevState* st;
  const uint32_t* pend_in;
  int in_slot;
  uint32_t adm_lo, adm_hi;
  const __bf16* feats;
  const __bf16* w1_frag;
  const float* params;
  float* keys;
  uint32_t* stamps;
  int k;
};

// One wave per 16 live tuples: h = ReLU(W1^T f + b1) on MFMA (rows = hidden units, columns =
// tuples), then the K outputs from lane-local partial sums and a reduction over lane groups.
__global__ __launch_bounds__(256) void rnn_keys_kernel(KeyArgs a) {
  const DevState* st = a.st;
  if (!st->learned_active || st->train_steps < MIN_STEPS) return;
  const int n_in = st->pend_count[a.in_slot];
  const int total = n_in + (int)(a.adm_hi - a.adm_lo);
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const float* b1 = a.params + RF * RH;
  const float* W2 = b1 + RH;
  const float* b2 = W2 + RH * RK;
  double cost[RK];
  for (int j = 0; j < a.k; ++j) cost[j] = st->cost_est[j];
  const int nw = gridDim.x * 4;
  for (int tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile * 16 < total; tile += nw) {
    const int i = tile * 16 + l16;
    const bool valid = i < total;
    uint32_t idx = 0;
    if (valid) idx = i < n_in ? entry_idx(a.pend_in[i]) : a.adm_lo + (uint32_t)(i - n_in);
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = (floatx4){0.f, 0.f, 0.f, 0.f};
    const bf16x8* fw = reinterpret_cast<const bf16x8*>(a.w1_frag);
#pragma unroll
    for (int ks = 0; ks < RF / 32; ++ks) {
      bf16x8 bv = *reinterpret_cast<const bf16x8*>(a.feats + (int64_t)idx * RF + ks * 32 + 8 * g);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[(ks * 4 + nt) * 64 + lane], bv, acc[nt], 0, 0, 0);
    }
    float o[RK];
#pragma unroll
    for (int j = 0; j < RK; ++j) o[j] = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int hu = nt * 16 + 4 * g + r;
        const float h = fmaxf(acc[nt][r] + b1[hu], 0.f);
#pragma unroll
        for (int j = 0; j < RK; ++j) o[j] += h * W2[hu * RK + j];
      }
#pragma unroll
    for (int j = 0; j < RK; ++j) {
      o[j] += __shfl_xor(o[j], 16);
      o[j] += __shfl_xor(o[j], 32);
    }
    if (valid && g == 0) {
      for (int j = 0; j < a.k; ++j) {
        const float p = 1.0f / (1.0f + __expf(-(o[j] + b2[j])));
        a.keys[(int64_t)idx * a.k + j] = (float)(cost[j] / fmaxf(p, 0.02f));
      }
      a.stamps[idx] = (uint32_t)st->rounds;
    }
  }
}

// Online training, one workgroup of four waves: TSTEPS Adam steps per round on successive windows
// of TB logged outcomes (newest first), masked binary cross-entropy on the evaluated predicate.
// Both contractions run on fp32 MFMA (16x16x4): the forward pass H = F W1 (64 x 192 x 64; wave w
// owns samples 16w..16w+15) and the W1 gradient F^T dH (192 x 64 x 64; wave w owns feature rows
// 48w..48w+47).  Every global read the launch needs (parameters, Adam moments, the windows'
// features, the judge's counters) is issued up front; parameters live in LDS across the steps and
// each thread keeps the Adam moments of the parameters it updates in registers, writing
// everything back once at the end.
constexpr int FSB = RF + 2;  // LDS row stride (bf16) of the sample features
constexpr int HS = RH + 4;   // LDS row stride of H and dH
constexpr int NREST = RH + RH * RK + RK;   // b1, W2, b2
constexpr int REST_PER = (NREST + 255) / 256;

__global__ __launch_bounds__(256) void rnn_train_kernel(DevState* st, const uint32_t* __restrict__ ring,
                                                        const __bf16* __restrict__ feats, float* __restrict__ params,
                                                        float* __restrict__ am, float* __restrict__ av,
                                                        __bf16* __restrict__ w1_frag, float lr) {
  __shared__ __attribute__((aligned(16))) float W1s[RF * RH];     // 48 KB, [i][j]
  __shared__ __attribute__((aligned(16))) __bf16 Fb[TSTEPS * TB * FSB];   // both windows, [b][i]
  __shared__ float Hr[TB * HS];    // ReLU(h), [b][j]
  __shared__ float dHs[TB * HS];   // dL/dh, [b][j]
  __shared__ float rest[NREST];    // b1 | W2 | b2
  __shared__ float part[4 * NREST];  // per-wave partial gradients of b1 | W2 | b2
  __shared__ float dO[TB], yv[TSTEPS * TB];
  __shared__ int kk[TSTEPS * TB];
  __shared__ int s_go;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const unsigned long long head = st->ring_head;
  const int steps0 = st->train_steps;
  if (!st->learned_active || (long long)head < (long long)TB) return;  // uniform across the workgroup
  const int n_steps = (long long)head >= (long long)TSTEPS * TB ? TSTEPS : (int)(head / TB);

  // ---- all global reads up front
  {
    const float4* p4 = reinterpret_cast<const float4*>(params);
    float4 wv[RF * RH / 4 / 256];
#pragma unroll
    for (int r = 0; r < RF * RH / 4 / 256; ++r) wv[r] = p4[tid + 256 * r];
#pragma unroll
    for (int r = 0; r < RF * RH / 4 / 256; ++r) reinterpret_cast<float4*>(W1s)[tid + 256 * r] = wv[r];
  }
  for (int q = tid; q < NREST; q += 256) rest[q] = params[RF * RH + q];
  float m1[3][4][4], v1[3][4][4];
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = (48 * w + 16 * mt + 4 * g + r) * RH + 16 * nt + l16;
        m1[mt][nt][r] = am[q];
        v1[mt][nt][r] = av[q];
      }
  float mr[REST_PER], vr[REST_PER];
#pragma unroll
  for (int c = 0; c < REST_PER; ++c) {
    const int q = tid + 256 * c;
    mr[c] = q < NREST ? am[RF * RH + q] : 0.f;
    vr[c] = q < NREST ? av[RF * RH + q] : 0.f;
  }
  // window `back` covers ring positions [head - (back+1) TB, head - back TB); sample sb = back TB + b
  if (tid < n_steps * TB) {
    const int back = tid / TB, b = tid % TB;
    const uint32_t e = ring[(uint64_t)((long long)head - (long long)(back + 1) * TB + b) & (RING - 1)];
    kk[tid] = (e >> 24) & 7;
    yv[tid] = (e >> 31) ? 1.f : 0.f;
  }
  {
    constexpr int CH = TSTEPS * TB * (RF / 8);    // 16-byte chunks of features
    uint4 fv[(CH + 255) / 256];
    int dsto[(CH + 255) / 256];
#pragma unroll
    for (int r = 0; r < (CH + 255) / 256; ++r) {
      const int q = tid + 256 * r;
      dsto[r] = -1;
      if (q < CH) {
        const int sb = q / (RF / 8), f8 = q % (RF / 8), back = sb / TB, b = sb % TB;
        if (back < n_steps) {
          const uint32_t e = ring[(uint64_t)((long long)head - (long long)(back + 1) * TB + b) & (RING - 1)];
          fv[r] = *reinterpret_cast<const uint4*>(feats + (int64_t)(e & kIdxMask) * RF + f8 * 8);
          dsto[r] = sb * FSB + f8 * 8;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < (CH + 255) / 256; ++r)
      if (dsto[r] >= 0) {
        // FSB is even, so each chunk lands 4-byte aligned
        uint32_t* d = reinterpret_cast<uint32_t*>(&Fb[dsto[r]]);
        d[0] = fv[r].x; d[1] = fv[r].y; d[2] = fv[r].z; d[3] = fv[r].w;
      }
  }
  // judge state (thread 0)
  int active = 1;
  double arm_c0 = 0.0, arm_c1 = 0.0, arm_t0 = 0.0, arm_t1 = 0.0;
  if (tid == 0) {
    arm_c0 = st->arm_cost[0]; arm_c1 = st->arm_cost[1];
    arm_t0 = st->arm_tuples[0]; arm_t1 = st->arm_tuples[1];
  }
  bool reset_arms = false;
  int steps = steps0;

  for (int back = 0; back < n_steps; ++back) {
    __syncthreads();  // staging done / previous step's LDS updates settled
    if (tid == 0) s_go = active;
    __syncthreads();
    if (!s_go) break;
    const __bf16* F = Fb + back * TB * FSB;
    const float* b1s = rest;
    const float* W2s = rest + RH;
    const float* b2s = rest + RH + RH * RK;

    // forward on MFMA: lane holds h[s = 16w + 4g + r][j = 16nt + l16]
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int ks = 0; ks < RF / 4; ++ks) {
      const float a_ = (float)F[(16 * w + l16) * FSB + 4 * ks + g];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_, W1s[(4 * ks + g) * RH + 16 * nt + l16], acc[nt], 0, 0, 0);
    }
    float po[4] = {0.f, 0.f, 0.f, 0.f};
    int ksl[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ksl[r] = kk[back * TB + 16 * w + 4 * g + r];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[nt][r] += b1s[j];
        const float h = fmaxf(acc[nt][r], 0.f);
        Hr[(16 * w + 4 * g + r) * HS + j] = h;
        po[r] += h * W2s[j * RK + ksl[r]];
      }
    }
    // logit of the evaluated slot: reduce over the 16 lanes of the group
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      po[r] = row_sum16(po[r]);
    }
    float d[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int sidx = 16 * w + 4 * g + r;
      const float o = po[r] + b2s[ksl[r]];
      d[r] = (1.0f / (1.0f + __expf(-o)) - yv[back * TB + sidx]) * (1.0f / TB);
      if (l16 == 0) dO[sidx] = d[r];
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dHs[(16 * w + 4 * g + r) * HS + j] = acc[nt][r] > 0.f ? d[r] * W2s[j * RK + ksl[r]] : 0.f;
    }
    __syncthreads();

    const int t_adam = steps + 1;
    const float c1 = 1.f / (1.f - powf(0.9f, (float)t_adam)), c2 = 1.f / (1.f - powf(0.999f, (float)t_adam));
    // W1 gradient on MFMA: lane holds g[i = 48w + 16mt + 4g + r][j = 16nt + l16]
    floatx4 gacc[3][4];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gacc[mt][nt] = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < TB / 4; ++ks) {
      const int b = 4 * ks + g;
      float a3[3], b4[4];
#pragma unroll
      for (int mt = 0; mt < 3; ++mt) a3[mt] = (float)F[b * FSB + 48 * w + 16 * mt + l16];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) b4[nt] = dHs[b * HS + 16 * nt + l16];
#pragma unroll
      for (int mt = 0; mt < 3; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
          gacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[mt], b4[nt], gacc[mt][nt], 0, 0, 0);
    }
    // b1, W2, b2 gradients: wave w sums its own 16 samples (lane j = hidden unit) into part[w],
    // the owners add the four partials below
    {
      float gb1 = 0.f, gb2 = 0.f, gw2[RK];
#pragma unroll
      for (int kc = 0; kc < RK; ++kc) gw2[kc] = 0.f;
#pragma unroll 4
      for (int bi = 0; bi < 16; ++bi) {
        const int b = 16 * w + bi;
        const int kb = kk[back * TB + b];
        const float o = dO[b];
        const float ho = Hr[b * HS + lane] * o;
        gb1 += dHs[b * HS + lane];
#pragma unroll
        for (int kc = 0; kc < RK; ++kc) gw2[kc] += kb == kc ? ho : 0.f;
        gb2 += kb == lane ? o : 0.f;
      }
      float* pw = part + w * NREST;
      pw[lane] = gb1;
#pragma unroll
      for (int kc = 0; kc < RK; ++kc) pw[RH + lane * RK + kc] = gw2[kc];
      if (lane < RK) pw[RH + RH * RK + lane] = gb2;
    }
    // Adam on the owned entries (moments in registers, parameters in LDS)
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = (48 * w + 16 * mt + 4 * g + r) * RH + 16 * nt + l16;
          const float gq = gacc[mt][nt][r];
          const float m = 0.9f * m1[mt][nt][r] + 0.1f * gq;
          const float v = 0.999f * v1[mt][nt][r] + 0.001f * gq * gq;
          m1[mt][nt][r] = m;
          v1[mt][nt][r] = v;
          W1s[q] -= lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
        }
    __syncthreads();  // partials complete
#pragma unroll
    for (int c = 0; c < REST_PER; ++c) {
      const int q = tid + 256 * c;
      if (q < NREST) {
        const float gq = part[q] + part[NREST + q] + part[2 * NREST + q] + part[3 * NREST + q];
        const float m = 0.9f * mr[c] + 0.1f * gq;
        const float v = 0.999f * vr[c] + 0.001f * gq * gq;
        mr[c] = m;
        vr[c] = v;
        rest[q] -= lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
      }
    }
    steps += 1;
    if (tid == 0) {
      if (steps == MIN_STEPS) {
        // the learned arm starts routing now: judge only what follows
        reset_arms = true;
        arm_c0 = arm_c1 = arm_t0 = arm_t1 = 0.0;
      }
      // judge: learned arm's UDF FLOPs per finished tuple against the control arm's
      if (steps >= MIN_STEPS && arm_t0 >= 2048.0 && arm_t1 >= 2048.0 && arm_c1 / arm_t1 > 1.02 * (arm_c0 / arm_t0))
        active = 0;
    }
  }
  __syncthreads();
  // ---- write back: parameters, inference fragments, moments, counters
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 48 * w + 16 * mt + 4 * g + r, j = 16 * nt + l16, q = i * RH + j;
        const float np = W1s[q];
        am[q] = m1[mt][nt][r];
        av[q] = v1[mt][nt][r];
        params[q] = np;
        // lane l of fragment (ks, nt) holds hidden unit nt*16 + l%16, features ks*32 + 8(l/16) + e
        const int ksi = i / 32, gg = (i % 32) / 8, e = i % 8, ntf = j / 16, ln = gg * 16 + j % 16;
        w1_frag[(((ksi * 4 + ntf) * 64) + ln) * 8 + e] = static_cast<__bf16>(np);
      }
#pragma unroll
  for (int c = 0; c < REST_PER; ++c) {
    const int q = tid + 256 * c;
    if (q < NREST) {
      am[RF * RH + q] = mr[c];
      av[RF * RH + q] = vr[c];
      params[RF * RH + q] = rest[q];
    }
  }
  if (tid == 0) {
    st->train_steps = steps;
    st->ring_trained = head;
    if (reset_arms) {
      st->arm_cost[0] = st->arm_cost[1] = 0.0;
      st->arm_tuples[0] = st->arm_tuples[1] = 0.0;
    }
    if (!active) st->learned_active = 0;
  }
}

int router_nn_create(RouterNN** out, int k, int fh, int fw, int64_t cap, uint64_t seed, int routing_batch,
                     float explore, const double* flops, RouterAllocFn alloc, void* alloc_ctx) {
  *out = nullptr;
  if (fh != fw || fh % 8 != 0) return HYDRO_EUNSUPPORTED;
  RouterNN* r = new RouterNN();
  r->k = k;
  r->fh = fh;
  r->fw = fw;
  r->cap = cap;
  r->seed = seed;
  r->routing_batch = routing_batch;
  r->explore = explore;
  r->external = alloc != nullptr;
  int fail_rc = HYDRO_ENOMEM;
  auto get = [&](void** p, size_t bytes) {
    if (alloc) {
      const int rc = alloc(alloc_ctx, p, bytes);
      if (rc) fail_rc = rc;
      return rc == 0;
    }
    return hipMalloc(p, bytes) == hipSuccess;
  };
  bool ok = get((void**)&r->feats, (size_t)cap * RF * sizeof(__bf16)) &&
            get((void**)&r->keys, (size_t)cap * k * sizeof(float)) &&
            get((void**)&r->stamps, (size_t)cap * sizeof(uint32_t)) &&
            get((void**)&r->ring, (size_t)RING * sizeof(uint32_t)) &&
            get((void**)&r->params, NPARAM * sizeof(float)) &&
            get((void**)&r->adam_m, NPARAM * sizeof(float)) &&
            get((void**)&r->adam_v, NPARAM * sizeof(float)) &&
            get((void**)&r->w1_frag, (size_t)(RF / 32) * 4 * 64 * 8 * sizeof(__bf16)) &&
            get((void**)&r->flops, RK * sizeof(float));
  if (!ok) {
    router_nn_destroy(r);
    return fail_rc;
  }
  // He-normal init of W1 and W2 (fp32), zero biases
  std::mt19937_64 rng(seed);
  std::normal_distribution<float> nd(0.f, 1.f);
  r->init.assign(NPARAM, 0.f);
  for (int q = 0; q < RF * RH; ++q) r->init[q] = nd(rng) * std::sqrt(2.f / RF);
  for (int q = 0; q < RH * RK; ++q) r->init[RF * RH + RH + q] = nd(rng) * std::sqrt(2.f / RH) * 0.1f;
  float fl[RK] = {0};
  for (int j = 0; j < k; ++j) fl[j] = (float)flops[j];
  hipMemcpy(r->flops, fl, sizeof(fl), hipMemcpyHostToDevice);
  *out = r;
  return HYDRO_OK;
}

void router_nn_destroy(RouterNN* r) {
  if (!r) return;
  if (r->external) {
    delete r;
    return;
  }
  hipFree(r->feats);
  hipFree(r->keys);
  hipFree(r->stamps);
  hipFree(r->ring);
  hipFree(r->params);
  hipFree(r->adam_m);
  hipFree(r->adam_v);
  hipFree(r->w1_frag);
  hipFree(r->flops);
  delete r;
}

void router_nn_reset(RouterNN* r, hipStream_t s) {
  hipMemcpyAsync(r->params, r->init.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, s);
  hipMemsetAsync(r->adam_m, 0, NPARAM * sizeof(float), s);
  hipMemsetAsync(r->adam_v, 0, NPARAM * sizeof(float), s);
  // no tuple has keys of this query yet (round numbers restart at every reset)
  hipMemsetAsync(r->stamps, 0xFF, (size_t)r->cap * sizeof(uint32_t), s);
  hipStreamSynchronize(s);
}

int router_nn_admit(RouterNN* r, const FrameSrc& fr, int64_t lo, int64_t hi, const DevState* guard, hipStream_t s) {
  const int64_t n = hi - lo;
  if (n <= 0) return HYDRO_OK;
  if (fr.hw != r->fh) return HYDRO_EUNSUPPORTED;
  // vector path: frame sides 32, 64 and 128 (the cell row is a whole number of aligned chunks)
  bool done = false;
  if (reinterpret_cast<uintptr_t>(fr.base) % 16 != 0) {
  } else if (fr.dtype == HYDRO_DTYPE_BF16) done = launch_pool_vec<__bf16>(fr, lo, n, r->feats, guard, s);
  else if (fr.dtype == HYDRO_DTYPE_U8) done = launch_pool_vec<uint8_t>(fr, lo, n, r->feats, guard, s);
  else done = launch_pool_vec<float>(fr, lo, n, r->feats, guard, s);
  if (!done) {
    const int64_t work = n * RF;
    const int grid = (int)std::min<int64_t>(4096, (work + 255) / 256);
    hipLaunchKernelGGL(rnn_pool_kernel, dim3(grid), dim3(256), 0, s, fr, lo, n, r->feats, guard);
  }
  return HYDRO_OK;
}

__bf16* router_nn_feats_ptr(RouterNN* r) { return r->feats; }

void router_nn_keys(RouterNN* r, DevState* st, const uint32_t* pend_in, int in_slot, uint32_t adm_lo,
                    uint32_t adm_hi, int grid, hipStream_t s) {
  KeyArgs a{st, pend_in, in_slot, adm_lo, adm_hi, r->feats, r->w1_frag, r->params, r->keys, r->stamps, r->k};
  hipLaunchKernelGGL(rnn_keys_kernel, dim3(grid), dim3(256), 0, s, a);
}

void router_nn_learn(RouterNN* r, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(rnn_train_kernel, dim3(1), dim3(256), 0, s, st, r->ring, r->feats, r->params, r->adam_m,
                     r->adam_v, r->w1_frag, 3e-3f);
}

const float* router_nn_keys_ptr(RouterNN* r) { return r->keys; }
const uint32_t* router_nn_stamps_ptr(RouterNN* r) { return r->stamps; }

OutcomeLog router_nn_log(RouterNN* r) {
  OutcomeLog o{};
  o.ring = r->ring;
  o.ring_mask = RING - 1;
  o.flops = r->flops;
  o.seed = (uint32_t)(r->seed * 0x9E3779B97F4A7C15ull >> 32);
  o.control_below = (uint32_t)std::min(4294967295.0, (double)r->explore * 4294967296.0);
  o.routing_batch = r->routing_batch;
  return o;
}

const float* router_nn_params_ptr(RouterNN* r) { return r->params; }
int router_nn_param_count() { return NPARAM; }
int router_nn_min_steps() { return MIN_STEPS; }

}  // namespace hydro

// Debug entry (declared in include/hydro.h): one launch of the training kernel on caller data.
extern "C" int hydro_router_train_debug(int32_t k, const uint16_t* feats, const int32_t* pred, const uint8_t* rejected,
                                        int32_t n, float* params, float* adam_m, float* adam_v, int32_t steps_done,
                                        float lr) {
  using namespace hydro;
  if (!feats || !pred || !rejected || !params || !adam_m || !adam_v) return HYDRO_EINVAL;
  if (k < 1 || k > RK || n != TSTEPS * TB || steps_done < 0) return HYDRO_EINVAL;
  for (int i = 0; i < n; ++i)
    if (pred[i] < 0 || pred[i] >= k) return HYDRO_EINVAL;
  DevState* st = nullptr;
  uint32_t* ring = nullptr;
  __bf16* f = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr;
  __bf16* frag = nullptr;
  int rc = HYDRO_OK;
  bool ok = hipMalloc(&st, sizeof(DevState)) == hipSuccess && hipMalloc(&ring, RING * sizeof(uint32_t)) == hipSuccess &&
            hipMalloc(&f, (size_t)n * RF * sizeof(__bf16)) == hipSuccess &&
            hipMalloc(&p, NPARAM * sizeof(float)) == hipSuccess && hipMalloc(&m, NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&v, NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&frag, (size_t)(RF / 32) * 4 * 64 * 8 * sizeof(__bf16)) == hipSuccess;
  if (!ok) rc = HYDRO_ENOMEM;
  if (rc == HYDRO_OK) {
    DevState h{};
    h.learned_active = 1;
    h.train_steps = steps_done;
    h.ring_head = (unsigned long long)n;     // the samples occupy ring positions 0 .. n-1, oldest first
    std::vector<uint32_t> r(RING, 0u);
    for (int i = 0; i < n; ++i) r[i] = (uint32_t)i | ((uint32_t)pred[i] << 24) | (rejected[i] ? 0x80000000u : 0u);
    ok = hipMemcpy(st, &h, sizeof(h), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(ring, r.data(), RING * sizeof(uint32_t), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(f, feats, (size_t)n * RF * sizeof(__bf16), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(p, params, NPARAM * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m, adam_m, NPARAM * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(v, adam_v, NPARAM * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
    if (ok) {
      hipLaunchKernelGGL(rnn_train_kernel, dim3(1), dim3(256), 0, nullptr, st, ring, f, p, m, v, frag, lr);
      ok = hipDeviceSynchronize() == hipSuccess &&
           hipMemcpy(params, p, NPARAM * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(adam_m, m, NPARAM * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(adam_v, v, NPARAM * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
    }
    if (!ok) rc = HYDRO_EDEVICE;
  }
  hipFree(st); hipFree(ring); hipFree(f); hipFree(p); hipFree(m); hipFree(v); hipFree(frag);
  return rc;
}

namespace hydro {
// Training takes at most TSTEPS steps a round, after the round's passes: keys can first be
// learned in this round (0-based).
int router_nn_first_learned_round() { return (MIN_STEPS + TSTEPS - 1) / TSTEPS; }

}  // namespace hydro
