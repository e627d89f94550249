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
constexpr int TSTEPS = 2;         // optimiser steps per round
constexpr int MIN_STEPS = 8;      // steps before the learned arm uses the router
constexpr int NPARAM = RF * RH + RH + RH * RK + RK;

struct RouterNN {
  int k, fh, fw, routing_batch;
  int64_t cap;
  uint64_t seed;
  float explore;
  __bf16* feats = nullptr;        // [cap][192]
  float* keys = nullptr;          // [cap][K]
  uint32_t* ring = nullptr;
  float* params = nullptr;        // W1 [192][64] | b1 [64] | W2 [64][8] | b2 [8]
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  __bf16* w1_frag = nullptr;      // W1^T as MFMA A fragments [6 ksteps][4 ntiles][64][8]
  float* flops = nullptr;         // [K]
  std::vector<float> init;
};

__global__ void rnn_pool_kernel(FrameSrc fr, int64_t n, __bf16* feats) {
  const int64_t total = n * RF;
  const int blk = fr.hw / 8;
  const float inv = 1.0f / (float)(blk * blk);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / RF;
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
    feats[q] = static_cast<__bf16>((s * inv - 0.5f) * 4.0f);
  }
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
    }
  }
}

// Adam on the router parameters from the newest logged outcomes.  One workgroup.
__global__ __launch_bounds__(256) void rnn_train_kernel(DevState* st, const uint32_t* ring, const __bf16* feats,
                                                        float* params, float* am, float* av, __bf16* w1_frag, int k,
                                                        float lr, int n_seen_min) {
  __shared__ float W1s[RF * RH];        // 48 KB
  __shared__ float F[TB][RF];           // 48 KB
  __shared__ float Hr[TB][RH];          // ReLU(h)
  __shared__ float dH[TB][RH];
  __shared__ float dO[TB];
  __shared__ int kk[TB];
  __shared__ float part[TB][4];
  const int tid = threadIdx.x;
  const unsigned long long head = st->ring_head;
  float* b1 = params + RF * RH;
  float* W2 = b1 + RH;
  float* b2 = W2 + RH * RK;
  int steps = 0;
  for (int s = 0; s < TSTEPS; ++s) {
    // step s trains on the TB outcomes logged just before position hi
    const long long hi = (long long)head - (long long)s * TB;
    if (hi < (long long)n_seen_min || hi - TB < 0) break;
    // stage weights and samples
    for (int q = tid; q < RF * RH; q += 256) W1s[q] = params[q];
    for (int q = tid; q < TB * RF; q += 256) {
      const int si = q / RF, fi = q % RF;
      const uint32_t e = ring[(uint64_t)(hi - TB + si) & (RING - 1)];
      F[si][fi] = (float)feats[(int64_t)(e & kIdxMask) * RF + fi];
    }
    if (tid < TB) {
      const uint32_t e = ring[(uint64_t)(hi - TB + tid) & (RING - 1)];
      kk[tid] = (e >> 24) & 7;
    }
    __syncthreads();
    // forward: 4 threads per sample, 16 hidden units each
    const int si = tid >> 2, hq = (tid & 3) * 16;
    float hv[16];
    const int ks = kk[si];
    float po = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      float h = b1[hq + j];
      for (int i = 0; i < RF; ++i) h += W1s[i * RH + hq + j] * F[si][i];
      hv[j] = h;
      const float r = fmaxf(h, 0.f);
      Hr[si][hq + j] = r;
      po += r * W2[(hq + j) * RK + ks];
    }
    part[si][tid & 3] = po;
    __syncthreads();
    if (tid < TB) {
      const float o = part[tid][0] + part[tid][1] + part[tid][2] + part[tid][3] + b2[kk[tid]];
      const uint32_t e = ring[(uint64_t)(hi - TB + tid) & (RING - 1)];
      const float y = (e >> 31) ? 1.f : 0.f;
      dO[tid] = (1.0f / (1.0f + __expf(-o)) - y) * (1.0f / TB);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) dH[si][hq + j] = hv[j] > 0.f ? dO[si] * W2[(hq + j) * RK + ks] : 0.f;
    __syncthreads();
    // gradients and Adam (bias-corrected), parameter by parameter
    const int t_adam = st->train_steps + steps + 1;
    const float c1 = 1.f / (1.f - powf(0.9f, (float)t_adam)), c2 = 1.f / (1.f - powf(0.999f, (float)t_adam));
    for (int q = tid; q < NPARAM; q += 256) {
      float gsum = 0.f;
      if (q < RF * RH) {
        const int i = q / RH, j = q % RH;
        for (int b = 0; b < TB; ++b) gsum += F[b][i] * dH[b][j];
      } else if (q < RF * RH + RH) {
        const int j = q - RF * RH;
        for (int b = 0; b < TB; ++b) gsum += dH[b][j];
      } else if (q < RF * RH + RH + RH * RK) {
        const int r = q - RF * RH - RH, j = r / RK, kc = r % RK;
        for (int b = 0; b < TB; ++b) gsum += kk[b] == kc ? Hr[b][j] * dO[b] : 0.f;
      } else {
        const int kc = q - RF * RH - RH - RH * RK;
        for (int b = 0; b < TB; ++b) gsum += kk[b] == kc ? dO[b] : 0.f;
      }
      const float m = 0.9f * am[q] + 0.1f * gsum;
      const float v = 0.999f * av[q] + 0.001f * gsum * gsum;
      am[q] = m;
      av[q] = v;
      params[q] -= lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
    }
    __syncthreads();
    ++steps;
  }
  // bf16 fragments of W1^T for inference: lane l holds rows (hidden) nt*16 + l%16, k = ks*32 + 8(l/16) + e
  if (steps > 0) {
    for (int q = tid; q < (RF / 32) * 4 * 64 * 8; q += 256) {
      const int e = q & 7, lane = (q >> 3) & 63, nt = (q >> 9) & 3, ksi = q >> 11;
      const int hu = nt * 16 + (lane & 15), fi = ksi * 32 + 8 * (lane >> 4) + e;
      w1_frag[q] = static_cast<__bf16>(params[fi * RH + hu]);
    }
  }
  if (tid == 0) {
    const int before = st->train_steps;
    st->train_steps = before + steps;
    st->ring_trained = head;
    if (before < MIN_STEPS && before + steps >= MIN_STEPS) {
      // the learned arm starts routing now: judge only what follows
      st->arm_cost[0] = st->arm_cost[1] = 0.0;
      st->arm_tuples[0] = st->arm_tuples[1] = 0.0;
    }
    // judge: learned arm's UDF FLOPs per finished tuple against the control arm's
    if (st->learned_active && st->train_steps >= MIN_STEPS && st->arm_tuples[0] >= 2048.0 &&
        st->arm_tuples[1] >= 2048.0) {
      const double cl = st->arm_cost[1] / st->arm_tuples[1];
      const double cc = st->arm_cost[0] / st->arm_tuples[0];
      if (cl > 1.02 * cc) st->learned_active = 0;
    }
  }
}

int router_nn_create(RouterNN** out, int k, int fh, int fw, int64_t cap, uint64_t seed, int routing_batch,
                     float explore, const double* flops) {
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
  bool ok = hipMalloc(&r->feats, (size_t)cap * RF * sizeof(__bf16)) == hipSuccess &&
            hipMalloc(&r->keys, (size_t)cap * k * sizeof(float)) == hipSuccess &&
            hipMalloc(&r->ring, (size_t)RING * sizeof(uint32_t)) == hipSuccess &&
            hipMalloc(&r->params, NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&r->adam_m, NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&r->adam_v, NPARAM * sizeof(float)) == hipSuccess &&
            hipMalloc(&r->w1_frag, (size_t)(RF / 32) * 4 * 64 * 8 * sizeof(__bf16)) == hipSuccess &&
            hipMalloc(&r->flops, RK * sizeof(float)) == hipSuccess;
  if (!ok) {
    router_nn_destroy(r);
    return HYDRO_ENOMEM;
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
  hipFree(r->feats);
  hipFree(r->keys);
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
  hipStreamSynchronize(s);
}

int router_nn_admit(RouterNN* r, const FrameSrc& fr, int64_t n, hipStream_t s) {
  if (n <= 0) return HYDRO_OK;
  if (fr.hw != r->fh) return HYDRO_EUNSUPPORTED;
  const int64_t work = n * RF;
  const int grid = (int)std::min<int64_t>(4096, (work + 255) / 256);
  hipLaunchKernelGGL(rnn_pool_kernel, dim3(grid), dim3(256), 0, s, fr, n, r->feats);
  return HYDRO_OK;
}

void router_nn_keys(RouterNN* r, DevState* st, const uint32_t* pend_in, int in_slot, uint32_t adm_lo,
                    uint32_t adm_hi, int grid, hipStream_t s) {
  KeyArgs a{st, pend_in, in_slot, adm_lo, adm_hi, r->feats, r->w1_frag, r->params, r->keys, r->k};
  hipLaunchKernelGGL(rnn_keys_kernel, dim3(grid), dim3(256), 0, s, a);
}

void router_nn_learn(RouterNN* r, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(rnn_train_kernel, dim3(1), dim3(256), 0, s, st, r->ring, r->feats, r->params, r->adam_m,
                     r->adam_v, r->w1_frag, r->k, 3e-3f, TB);
}

const float* router_nn_keys_ptr(RouterNN* r) { return r->keys; }

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

int router_nn_min_steps() { return MIN_STEPS; }

}  // namespace hydro
