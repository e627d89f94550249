// Four-layer CNN predicates on 128x128x3 frames (conv3x3/s2/p1 widths 32-64-128-256, ReLU, mean
// pool, FC 10) on gfx950, in three launches per tier and round:
//
//   front   one frame per workgroup pass: layer 1 (K = 27 on one bf16 MFMA k-step) and layer 2,
//           streamed in eight bands of four layer-2 output rows.  Layer 1's output never leaves
//           LDS: a ring of nine layer-1 rows (the eight of the band plus the one above it) feeds
//           layer 2, whose weights stay in registers for the whole launch.  Layer 2's output
//           (32x32x64) goes to an activation buffer.
//   gemm3   layer 3 as an implicit GEMM over every queued frame of the launch: rows = output
//           positions, columns = the 128 output channels, K = (tap, input channel) = 576.
//   gemm4   layer 4 the same way (K = 1152, 256 channels), with the epilogue pooling each
//           frame's 64 positions, applying FC, the class-subset margin and the decision.
//
// Arithmetic tiers (template P): FP32 (fp32 MFMA 16x16x4), BF16 (bf16 MFMA 16x16x32) and FP8
// (OCP e4m3 operands on the scaled 16x16x128 MFMA with unit block scales; per-output-channel
// weight scales and per-layer activation scales applied in fp32 in the epilogues).  Layer 1 runs
// bf16 in the BF16 and FP8 tiers: raw uint8 / bf16 frame values are exact in bf16, and the
// normalisation is folded into its weights.  Accumulation is fp32 throughout.
//
// The GEMM tiles stage A (weights, pre-packed per k-block in the LDS image order) and B (the
// im2col rows of the activations, gathered per 16-byte chunk) in a double-buffered LDS ring from
// register stages.  LDS rows are XOR-swizzled by 16-byte chunk so that the sixteen rows an MFMA
// fragment reads fall on distinct banks.
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

namespace hydro {

template <int P> struct C4T;
template <> struct C4T<C4_F32> { typedef float T; static constexpr int ES = 4; };
template <> struct C4T<C4_BF16> { typedef __bf16 T; static constexpr int ES = 2; };
template <> struct C4T<C4_FP8> { typedef uint8_t T; static constexpr int ES = 1; };

typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ inline floatx4 c4_mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 c4_mfma(float a, float b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
// e4m3 x e4m3, K = 128, block scales 2^0 (E8M0 127)
__device__ inline floatx4 c4_mfma(i32x8 a, i32x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// Round to e4m3 (RNE) with saturation at the largest finite value (the conversion itself does
// not saturate: values above 448 would become NaN).
__device__ inline uint32_t c4_pack_fp8x4(float v0, float v1, float v2, float v3) {
  v0 = fminf(v0, 448.f); v1 = fminf(v1, 448.f); v2 = fminf(v2, 448.f); v3 = fminf(v3, 448.f);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(v0, v1, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(v2, v3, w, true);
  return (uint32_t)w;
}

// Stores 4 consecutive activations (already >= 0) in the tier's element type.
template <int P>
__device__ inline void c4_store4(void* dst, float v0, float v1, float v2, float v3) {
  if constexpr (P == C4_F32) {
    *reinterpret_cast<float4*>(dst) = make_float4(v0, v1, v2, v3);
  } else if constexpr (P == C4_BF16) {
    alignas(8) __bf16 h[4] = {static_cast<__bf16>(v0), static_cast<__bf16>(v1), static_cast<__bf16>(v2),
                              static_cast<__bf16>(v3)};
    *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(h);
  } else {
    *reinterpret_cast<uint32_t*>(dst) = c4_pack_fp8x4(v0, v1, v2, v3);
  }
}

// Calibration (FP32 tier): running maximum of a layer's activations, as float bits (values >= 0
// order like their bit patterns).
__device__ inline void c4_track_max(unsigned* slot, float v) {
  if (slot == nullptr) return;
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if (lane_id() == 0 && v > 0.f) atomicMax(slot, __float_as_uint(v));
}

// ---------------------------------------------------------------- front: layers 1 and 2
constexpr int F_NB = 8;            // bands per frame (four layer-2 rows each)
constexpr int F_RING = 9;          // layer-1 rows held: the band's eight and the one above
constexpr int F_SLOTS = 65;        // layer-1 columns of a row: even 0..62, then odd -1..63
constexpr int F_FROWS = 17;        // frame rows a band reads
constexpr int F_FPITCH = 388;      // bf16 elements per staged frame row: [0] unused, [1..3] the left
                                   // pad column, [4 + 3x + c] column x channel c
template <int P> struct FrontCfg;
// bytes per layer-1 column slot (32 channels + padding: the slot pitch in 16-byte units is odd so
// that eight consecutive slots fall on distinct bank groups)
template <> struct FrontCfg<C4_F32> { static constexpr int PITCH = 144; };
template <> struct FrontCfg<C4_BF16> { static constexpr int PITCH = 80; };
template <> struct FrontCfg<C4_FP8> { static constexpr int PITCH = 48; };

constexpr int F_FRAME_B = (F_FROWS * F_FPITCH * 2 + 15) / 16 * 16;   // staged frame band, bytes
__host__ __device__ constexpr int front_lds_bytes(int pitch) { return F_FRAME_B + F_RING * F_SLOTS * pitch; }

// Layer-1 column j -> its slot in a ring row.
__device__ inline int f_slot(int j) { return (j & 1) ? 32 + ((j + 1) >> 1) : (j >> 1); }

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == C4_F32 ? 1 : 2)))
void c4_front_kernel(GcnnArgs a) {
  typedef typename C4T<P>::T T;
  constexpr int ES = C4T<P>::ES;
  constexpr int PITCH = FrontCfg<P>::PITCH;
  __shared__ __attribute__((aligned(16))) unsigned char lds[front_lds_bytes(PITCH)];
  __shared__ unsigned long long ticks_s[kMaxK];
  __bf16* fb = reinterpret_cast<__bf16*>(lds);          // staged frame band (raw values, bf16)
  unsigned char* ring = lds + F_FRAME_B;                   // layer-1 output rows
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  if (tid < kMaxK) ticks_s[tid] = 0;
  // the left pad column (slot 32) of every ring row is a zero activation
  for (int q = tid; q < F_RING * (PITCH / 4); q += 256)
    reinterpret_cast<uint32_t*>(ring + (q / (PITCH / 4)) * F_SLOTS * PITCH + 32 * PITCH)[q % (PITCH / 4)] = 0u;
  // frame band pad column: elements 1..3 of every row
  for (int q = tid; q < F_FROWS * 4; q += 256) fb[(q >> 2) * F_FPITCH + (q & 3)] = static_cast<__bf16>(a.pad_raw);

  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += a.c4[i] ? a.q.counts[a.pred[i]] : 0;
  const bool u8 = a.fr.dtype == HYDRO_DTYPE_U8;
  // frame staging: chunk q (16 bytes) of band row r; u8: 24 chunks a row, bf16: 48
  const int cpr = u8 ? 24 : 48;
  const int nchunks = F_FROWS * cpr;

  // per-slot state (reloaded when the slot changes)
  int cur = -1;
  bf16x8 w1b[2];                      // layer-1 weights, bf16 tiers
  float w1f[7][2];                    // layer-1 weights, FP32 tier
  bf16x8 w2b[P == C4_BF16 ? 9 : 1][P == C4_BF16 ? 4 : 1];
  i32x8 w2q[P == C4_FP8 ? 3 : 1][P == C4_FP8 ? 4 : 1];
  float inv_s1 = 1.f, inv_s2 = 1.f, asc1 = 1.f;

  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t, ebase = 0;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = a.c4[i] ? a.q.counts[a.pred[i]] : 0;
      if (off < c) { slot = i; break; }
      off -= c;
      ebase += a.q.counts[a.pred[i]];
    }
    const int k = a.pred[slot];
    const int64_t ent = (int64_t)ebase + off;
    if (ent >= a.act_cap) {   // cannot happen: a round holds at most act_cap evaluations
      if (tid == 0) atomicOr(&a.st->overflow, 1);
      continue;
    }
    const uint32_t idx = entry_idx(a.q.entries[(int64_t)k * a.q.cap + off]);
    if (slot != cur) {
      cur = slot;
      if constexpr (P == C4_F32) {
        const float* w1 = static_cast<const float*>(a.c4_w1f[slot]);
#pragma unroll
        for (int s = 0; s < 7; ++s)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) w1f[s][ct] = w1[(s * 2 + ct) * 64 + lane];
      } else {
        const bf16x8* w1 = static_cast<const bf16x8*>(a.c4_w1b[slot]);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) w1b[ct] = w1[ct * 64 + lane];
      }
      if constexpr (P == C4_BF16) {
        const bf16x8* w2 = static_cast<const bf16x8*>(a.c4_w2[slot][C4_BF16]);
#pragma unroll
        for (int tp = 0; tp < 9; ++tp)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) w2b[tp][ct] = w2[(tp * 4 + ct) * 64 + lane];
      }
      if constexpr (P == C4_FP8) {
        const i32x8* w2 = static_cast<const i32x8*>(a.c4_w2[slot][C4_FP8]);
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) w2q[s][ct] = w2[(s * 4 + ct) * 64 + lane];
        asc1 = a.c4_ascale[slot][0];
        inv_s1 = 1.f / a.c4_ascale[slot][0];
        inv_s2 = 1.f / a.c4_ascale[slot][1];
      }
    }
    const unsigned long long t0 = wall_clock64();
    const unsigned char* frame = static_cast<const unsigned char*>(a.fr.base) + (int64_t)idx * a.fr.elems * (u8 ? 1 : 2);
    T* out2 = reinterpret_cast<T*>(a.c4_act2) + ent * (32 * 32 * 64);
    unsigned* amax1 = a.c4_act_max ? a.c4_act_max + k * 4 + 0 : nullptr;
    unsigned* amax2 = a.c4_act_max ? a.c4_act_max + k * 4 + 1 : nullptr;

    for (int b = 0; b < F_NB; ++b) {
      // ---- stage frame rows 16b-1 .. 16b+15 (raw values as bf16); row -1 is the pad value
      for (int q = tid; q < nchunks; q += 256) {
        const int r = q / cpr, j = q % cpr, y = 16 * b - 1 + r;
        __bf16* dst = fb + r * F_FPITCH + 4 + (u8 ? 16 : 8) * j;
        if (y < 0) {
          for (int e = 0; e < (u8 ? 16 : 8); ++e) dst[e] = static_cast<__bf16>(a.pad_raw);
          continue;
        }
        const uint4 v = reinterpret_cast<const uint4*>(frame + (int64_t)y * 128 * 3 * (u8 ? 1 : 2))[j];
        if (u8) {
          const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            alignas(8) __bf16 e4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) e4[e] = static_cast<__bf16>((float)((wv[h] >> (8 * e)) & 0xFFu));
            *reinterpret_cast<uint2*>(dst + 4 * h) = *reinterpret_cast<const uint2*>(e4);
          }
        } else {
          *reinterpret_cast<uint2*>(dst) = make_uint2(v.x, v.y);
          *reinterpret_cast<uint2*>(dst + 4) = make_uint2(v.z, v.w);
        }
      }
      // the ring slot of layer-1 row -1 is zero for the first band
      const int base_slot = (8 * b) % F_RING;   // ring index of layer-1 row 8b - 1
      if (b == 0)
        for (int q = tid; q < F_SLOTS * PITCH / 4; q += 256) reinterpret_cast<uint32_t*>(ring)[q] = 0u;
      __syncthreads();

      // ---- layer 1: rows 8b + 2w, 8b + 2w + 1 (local i = 2w, 2w+1), 64 columns each
#pragma unroll 2
      for (int pt = 0; pt < 8; ++pt) {
        const int il = 2 * wave + (pt >> 2), j = (pt & 3) * 16 + l16;
        floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        const __bf16* fr = fb + (2 * il) * F_FPITCH + 1 + 6 * j;
        if constexpr (P == C4_F32) {
#pragma unroll
          for (int s = 0; s < 7; ++s) {
            int kk = 4 * s + g;
            kk = kk > 26 ? 26 : kk;
            const int u = kk / 9, tt = kk % 9;
            const float x = static_cast<float>(fr[u * F_FPITCH + tt]);
            acc[0] = c4_mfma(w1f[s][0], x, acc[0]);
            acc[1] = c4_mfma(w1f[s][1], x, acc[1]);
          }
        } else {
          bf16x8 xb;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            int kk = 8 * g + e;
            kk = kk > 26 ? 26 : kk;   // k = 27..31: zero weights (any finite element)
            const int u = kk / 9, tt = kk % 9;
            xb[e] = fr[u * F_FPITCH + tt];
          }
          acc[0] = c4_mfma(w1b[0], xb, acc[0]);
          acc[1] = c4_mfma(w1b[1], xb, acc[1]);
        }
        const int ridx = (base_slot + 1 + il) % F_RING;
        unsigned char* dst = ring + (ridx * F_SLOTS + f_slot(j)) * PITCH;
        float m = 0.f;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const float4 bb = *reinterpret_cast<const float4*>(a.bias[slot][0] + ct * 16 + 4 * g);
          const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
          float v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            v[r] = fmaxf(acc[ct][r] + bv[r], 0.f);
            m = fmaxf(m, v[r]);
            v[r] *= inv_s1;
          }
          c4_store4<P>(dst + (ct * 16 + 4 * g) * ES, v[0], v[1], v[2], v[3]);
        }
        if constexpr (P == C4_F32) c4_track_max(amax1, m);
      }
      __syncthreads();

      // ---- layer 2: output row 4b + w, columns 0..31 (two position tiles).  The FP8 and FP32
      // tiers split the k-steps over two accumulation chains (the BF16 tier has no registers
      // left for a second chain: its layer-2 weights take 144)
      floatx4 acc[2][4][2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) acc[h][ct][mt] = (floatx4){0.f, 0.f, 0.f, 0.f};
      // ring row of layer-1 row 8b + 2w + u - 1 is (base_slot + 2w + u) mod 9
      if constexpr (P == C4_FP8) {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
          int tp = 4 * s + g;
          tp = tp > 8 ? 8 : tp;       // taps 9..11: zero weights
          const int u = tp / 3, v = tp % 3;
          const int rr = (base_slot + 2 * wave + u) % F_RING;
          i32x8 xb[2];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const int j = mt * 16 + l16;
            const int sl = v == 1 ? j : v == 0 ? 32 + j : 33 + j;
            const uint4* src = reinterpret_cast<const uint4*>(ring + (rr * F_SLOTS + sl) * PITCH);
            const uint4 lo = src[0], hi = src[1];
            xb[mt] = (i32x8){(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
          }
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[s & 1][ct][mt] = c4_mfma(w2q[s][ct], xb[mt], acc[s & 1][ct][mt]);
        }
      } else if constexpr (P == C4_BF16) {
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
          const int u = tp / 3, v = tp % 3;
          const int rr = (base_slot + 2 * wave + u) % F_RING;
          bf16x8 xb[2];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const int j = mt * 16 + l16;
            const int sl = v == 1 ? j : v == 0 ? 32 + j : 33 + j;
            xb[mt] = *reinterpret_cast<const bf16x8*>(ring + (rr * F_SLOTS + sl) * PITCH + 16 * g);
          }
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[0][ct][mt] = c4_mfma(w2b[tp][ct], xb[mt], acc[0][ct][mt]);
        }
      } else {
        // FP32: weights from global (L2-resident) per tap; lane group g holds channels 8g..8g+7,
        // k-step e of a tap uses channel 8g + e
        const float4* w2 = static_cast<const float4*>(a.c4_w2[slot][C4_F32]);
#pragma unroll 1
        for (int tp = 0; tp < 9; ++tp) {
          const int u = tp / 3, v = tp % 3;
          const int rr = (base_slot + 2 * wave + u) % F_RING;
          float xf[2][8];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const int j = mt * 16 + l16;
            const int sl = v == 1 ? j : v == 0 ? 32 + j : 33 + j;
            const float4* src = reinterpret_cast<const float4*>(ring + (rr * F_SLOTS + sl) * PITCH + 32 * g);
            const float4 p0 = src[0], p1 = src[1];
            xf[mt][0] = p0.x; xf[mt][1] = p0.y; xf[mt][2] = p0.z; xf[mt][3] = p0.w;
            xf[mt][4] = p1.x; xf[mt][5] = p1.y; xf[mt][6] = p1.z; xf[mt][7] = p1.w;
          }
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const float4 q0 = w2[((tp * 4 + ct) * 64 + lane) * 2], q1 = w2[((tp * 4 + ct) * 64 + lane) * 2 + 1];
            const float wf[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
              for (int mt = 0; mt < 2; ++mt) acc[e & 1][ct][mt] = c4_mfma(wf[e], xf[mt][e], acc[e & 1][ct][mt]);
          }
        }
      }
      // bias + ReLU -> layer-2 activations of row 4b + w
      {
        const int orow = 4 * b + wave;
        float m = 0.f;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const int j = mt * 16 + l16;
          T* o = out2 + (orow * 32 + j) * 64;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const float4 bb = *reinterpret_cast<const float4*>(a.bias[slot][1] + ct * 16 + 4 * g);
            const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
            float sv[4] = {1.f, 1.f, 1.f, 1.f};
            if constexpr (P == C4_FP8) {
              const float4 ss = *reinterpret_cast<const float4*>(a.c4_wscale[slot][0] + ct * 16 + 4 * g);
              sv[0] = ss.x * asc1; sv[1] = ss.y * asc1; sv[2] = ss.z * asc1; sv[3] = ss.w * asc1;
            }
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              float x = acc[0][ct][mt][r] + acc[1][ct][mt][r];
              if constexpr (P == C4_FP8) x *= sv[r];
              v[r] = fmaxf(x + bv[r], 0.f);
              m = fmaxf(m, v[r]);
              v[r] *= inv_s2;
            }
            c4_store4<P>(o + ct * 16 + 4 * g, v[0], v[1], v[2], v[3]);
          }
        }
        if constexpr (P == C4_F32) c4_track_max(amax2, m);
      }
      __syncthreads();   // the next band restages the frame rows and overwrites ring rows
    }
    if (tid == 0) ticks_s[k] += wall_clock64() - t0;
  }
  __syncthreads();
  if (tid < kMaxK && ticks_s[tid] && a.count_ticks) atomicAdd(&a.st->r_ticks[tid], ticks_s[tid]);
}

// ---------------------------------------------------------------- layers 3 and 4: implicit GEMM
template <int P> struct GemmCfg;
// ROWB: bytes of one LDS tile row per k-block; UPR: 16-byte units per row; CE: elements per unit
template <> struct GemmCfg<C4_F32> { static constexpr int ROWB = 64, UPR = 4, CE = 4, KSUB = 4; };
template <> struct GemmCfg<C4_BF16> { static constexpr int ROWB = 64, UPR = 4, CE = 8, KSUB = 1; };
template <> struct GemmCfg<C4_FP8> { static constexpr int ROWB = 128, UPR = 8, CE = 16, KSUB = 1; };

// chunk swizzle of tile row r: rows of 4 units xor (r/2) mod 4, rows of 8 units xor r mod 8
template <int UPR>
__host__ __device__ inline int c4_swz(int r) { return UPR == 4 ? ((r >> 1) & 3) : (r & 7); }

template <int P, int LAYER> struct GemmShape;
// LAYER 2 = the third conv (32x32x64 -> 16x16x128), LAYER 3 = the fourth (16x16x128 -> 8x8x256)
template <int P> struct GemmShape<P, 2> {
  static constexpr int CIN = 64, COUT = 128, HIN = 32, HOUT = 16;
  static constexpr int BM = P == C4_BF16 ? 256 : 128, BN = 128;
  static constexpr int WM = 64, WN = P == C4_BF16 ? 128 : 64;
};
template <int P> struct GemmShape<P, 3> {
  static constexpr int CIN = 128, COUT = 256, HIN = 16, HOUT = 8;
  static constexpr int BM = P == C4_BF16 ? 128 : 64, BN = 256;
  static constexpr int WM = 64, WN = P == C4_BF16 ? 128 : 64;
};

__host__ __device__ inline int c4_nkb(int prec, int layer) {
  const int cin = layer == 2 ? 64 : 128;
  const int bke = prec == C4_FP8 ? 128 : prec == C4_BF16 ? 32 : 16;
  return (9 * cin + bke - 1) / bke;
}

template <int P, int LAYER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == C4_FP8 && LAYER == 3 ? 1 : 2)))
void c4_gemm_kernel(GcnnArgs a, Forward f) {
  typedef typename C4T<P>::T T;
  typedef GemmCfg<P> G;
  typedef GemmShape<P, LAYER> S;
  constexpr int ES = C4T<P>::ES, UPR = G::UPR, CE = G::CE, BKE = G::ROWB / ES;
  constexpr int CIN = S::CIN, COUT = S::COUT, HIN = S::HIN, HOUT = S::HOUT, PP = HOUT * HOUT;
  constexpr int BM = S::BM, BN = S::BN, WM = S::WM, WN = S::WN;
  constexpr int MT = WM / 16, NT = WN / 16;
  constexpr int WGM = BM / WM;                       // waves along M
  constexpr int NKB = (9 * CIN + BKE - 1) / BKE;
  constexpr int UNITS = (BN + BM) * UPR, NU = UNITS / 256, NA = BN * UPR / 256;
  constexpr int STAGE = UNITS * 16;
  constexpr bool HEAD = LAYER == 3;
  static_assert(UNITS % 256 == 0 && (BN * UPR) % 256 == 0, "tile rows must fill the thread units");
  static_assert(WGM * (BN / WN) == 4, "four waves per tile");
  static_assert(!HEAD || (BN == COUT && WM == PP), "the head needs whole frames per wave and all channels");
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  __shared__ float zpart[4][kClasses];
  __shared__ unsigned long long ticks_s[kMaxK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave % WGM, wn = wave / WGM;
  if (tid < kMaxK) ticks_s[tid] = 0;
  const T* act_in = reinterpret_cast<const T*>(LAYER == 2 ? a.c4_act2 : a.c4_act3);
  // tiles: per slot ceil(count * PP / BM) x COUT / BN
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i)
    if (a.c4[i]) total += (int)(((int64_t)a.q.counts[a.pred[i]] * PP + BM - 1) / BM) * (COUT / BN);
  const int u_slot = tid % UPR;     // the LDS slot of every unit this thread stages

  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t, ebase = 0;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = a.c4[i] ? (int)(((int64_t)a.q.counts[a.pred[i]] * PP + BM - 1) / BM) * (COUT / BN) : 0;
      if (off < c) { slot = i; break; }
      off -= c;
      ebase += a.q.counts[a.pred[i]];
    }
    const int k = a.pred[slot];
    const int cnt = a.q.counts[k];
    const int mt0 = off / (COUT / BN), cb = off % (COUT / BN);
    const int64_t row0 = (int64_t)mt0 * BM;           // first position row of the tile (slot-local)
    const int64_t rows = (int64_t)cnt * PP;
    const unsigned long long t0 = wall_clock64();
    const unsigned char* img = static_cast<const unsigned char*>(a.c4_img[slot][LAYER - 2][P]) + (size_t)cb * BN * G::ROWB;

    // B rows this thread stages: precomputed frame pointer, output position and chunk
    const T* bsrc[NU - NA];
    int boi[NU - NA], boj[NU - NA], bch[NU - NA];
#pragma unroll
    for (int v = NA; v < NU; ++v) {
      const int U = tid + 256 * v - BN * UPR;
      const int rb = U / UPR;
      const int64_t row = row0 + rb;
      const bool valid = row < rows && ebase + row / PP < a.act_cap;
      const int64_t e = valid ? row / PP : 0;
      const int p = valid ? (int)(row % PP) : 0;
      bsrc[v - NA] = act_in + ((int64_t)ebase + e) * (HIN * HIN * CIN);
      boi[v - NA] = valid ? p / HOUT : -1000;        // invalid rows read the zero page
      boj[v - NA] = p % HOUT;
      bch[v - NA] = (u_slot ^ c4_swz<UPR>(rb)) * CE;  // element offset of the chunk in the k-block
    }
    u32x4 stg[NU];
    // stage k-block kb of A (the packed image) and B (im2col gathers) into registers
#define C4_GLOAD(kb_)                                                                              \
  do {                                                                                             \
    const int kbv = (kb_);                                                                         \
    _Pragma("unroll") for (int v = 0; v < NA; ++v)                                                 \
      stg[v] = reinterpret_cast<const u32x4*>(img + (size_t)kbv * COUT * G::ROWB)[tid + 256 * v];  \
    _Pragma("unroll") for (int v = NA; v < NU; ++v) {                                              \
      const int ke = kbv * BKE + bch[v - NA];                                                      \
      const int tap = ke / CIN, ch = ke % CIN;                                                     \
      const int y = 2 * boi[v - NA] + tap / 3 - 1, x = 2 * boj[v - NA] + tap % 3 - 1;              \
      const bool ok = tap < 9 && y >= 0 && x >= 0 && y < HIN && x < HIN;                           \
      const u32x4* src = ok ? reinterpret_cast<const u32x4*>(bsrc[v - NA] + (y * HIN + x) * CIN + ch) \
                            : static_cast<const u32x4*>(a.zero_page);                              \
      stg[v] = *src;                                                                               \
    }                                                                                              \
  } while (0)
#define C4_LSTORE(buf_)                                                                            \
  do {                                                                                             \
    _Pragma("unroll") for (int v = 0; v < NU; ++v)                                                 \
      reinterpret_cast<u32x4*>(lds + (buf_) * STAGE)[tid + 256 * v] = stg[v];                      \
  } while (0)

    floatx4 acc[NT][MT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (floatx4){0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int buf) {
      const unsigned char* A = lds + buf * STAGE;
      const unsigned char* B = A + BN * G::ROWB;
      if constexpr (P == C4_FP8) {
        i32x8 af[NT], bfr[MT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int r = wn * WN + nt * 16 + l16;
          const uint4 lo = *reinterpret_cast<const uint4*>(A + (r * UPR + ((2 * g) ^ c4_swz<UPR>(r))) * 16);
          const uint4 hi = *reinterpret_cast<const uint4*>(A + (r * UPR + ((2 * g + 1) ^ c4_swz<UPR>(r))) * 16);
          af[nt] = (i32x8){(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int r = wm * WM + mt * 16 + l16;
          const uint4 lo = *reinterpret_cast<const uint4*>(B + (r * UPR + ((2 * g) ^ c4_swz<UPR>(r))) * 16);
          const uint4 hi = *reinterpret_cast<const uint4*>(B + (r * UPR + ((2 * g + 1) ^ c4_swz<UPR>(r))) * 16);
          bfr[mt] = (i32x8){(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = c4_mfma(af[nt], bfr[mt], acc[nt][mt]);
      } else if constexpr (P == C4_BF16) {
        bf16x8 af[NT], bfr[MT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int r = wn * WN + nt * 16 + l16;
          af[nt] = *reinterpret_cast<const bf16x8*>(A + (r * UPR + (g ^ c4_swz<UPR>(r))) * 16);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int r = wm * WM + mt * 16 + l16;
          bfr[mt] = *reinterpret_cast<const bf16x8*>(B + (r * UPR + (g ^ c4_swz<UPR>(r))) * 16);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = c4_mfma(af[nt], bfr[mt], acc[nt][mt]);
      } else {
        floatx4 af[NT], bfr[MT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int r = wn * WN + nt * 16 + l16;
          af[nt] = *reinterpret_cast<const floatx4*>(A + (r * UPR + (g ^ c4_swz<UPR>(r))) * 16);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int r = wm * WM + mt * 16 + l16;
          bfr[mt] = *reinterpret_cast<const floatx4*>(B + (r * UPR + (g ^ c4_swz<UPR>(r))) * 16);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = c4_mfma(af[nt][j], bfr[mt][j], acc[nt][mt]);
      }
    };

    // double-buffered k loop, one barrier per k-block: block kb+1 is stored while block kb is
    // read; block kb+2 is in flight meanwhile
    C4_GLOAD(0);
    C4_LSTORE(0);
    if (NKB > 1) C4_GLOAD(1);
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < NKB; ++kb) {
      if (kb + 1 < NKB) {
        C4_LSTORE((kb + 1) & 1);
        if (kb + 2 < NKB) C4_GLOAD(kb + 2);
      }
      compute(kb & 1);
      __syncthreads();
    }
#undef C4_GLOAD
#undef C4_LSTORE

    // ---- epilogue
    const float* bias = a.bias[slot][LAYER];
    const float* wsc = a.c4_wscale[slot][LAYER - 1];
    const float asc = P == C4_FP8 ? a.c4_ascale[slot][LAYER - 1] : 1.f;
    if constexpr (!HEAD) {
      T* out = reinterpret_cast<T*>(a.c4_act3);
      const float inv_out = P == C4_FP8 ? 1.f / a.c4_ascale[slot][2] : 1.f;
      unsigned* amax = a.c4_act_max ? a.c4_act_max + k * 4 + 2 : nullptr;
      float m = 0.f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int64_t row = row0 + wm * WM + mt * 16 + l16;
        const bool valid = row < rows && ebase + row / PP < a.act_cap;
        const int64_t e = valid ? row / PP : 0;
        const int p = (int)(row % PP);
        T* o = out + ((int64_t)ebase + e) * (PP * COUT) + (int64_t)p * COUT;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int ch = cb * BN + wn * WN + nt * 16 + 4 * g;
          float v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float x = acc[nt][mt][r];
            if constexpr (P == C4_FP8) x *= wsc[ch + r] * asc;
            v[r] = fmaxf(x + bias[ch + r], 0.f);
            m = fmaxf(m, valid ? v[r] : 0.f);
            v[r] *= inv_out;
          }
          if (valid) c4_store4<P>(o + ch, v[0], v[1], v[2], v[3]);
        }
      }
      if constexpr (P == C4_F32) c4_track_max(amax, m);
    } else {
      // wave (wm, wn): frame wm of the tile, channels wn*WN .. +WN-1.  Pool over the frame's 64
      // positions, then this wave's share of FC.
      const int64_t frow = row0 + wm * WM;             // first row of the frame
      const bool fvalid = frow < rows;
      const float* fw = a.fc_w[slot];
      float zc = 0.f;                                   // lane l16 < 10: class l16
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int chb = wn * WN + nt * 16 + 4 * g;
        float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float x = acc[nt][mt][r];
            if constexpr (P == C4_FP8) x *= wsc[chb + r] * asc;
            s[r] += fmaxf(x + bias[chb + r], 0.f);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float gch = row_sum16(s[r]) * (1.f / PP);
          if (l16 < kClasses) zc += gch * fw[(chb + r) * kClasses + l16];
        }
      }
      // rows g = 0..3 hold different channel groups: add them
      zc = (__shfl(zc, l16) + __shfl(zc, 16 + l16)) + (__shfl(zc, 32 + l16) + __shfl(zc, 48 + l16));
      if (lane < kClasses) zpart[wave][lane] = zc;
      __syncthreads();
      if (wn == 0) {
        bool pass = false, defer = false, active = false;
        uint32_t e = 0;
        if (fvalid) {
          const int64_t ei = frow / PP;
          e = a.q.entries[(int64_t)k * a.q.cap + ei];
          if (lane == 0) {
            active = true;
            float z[kClasses];
#pragma unroll
            for (int c = 0; c < kClasses; ++c) {
              float s = 0.f;
              for (int w2 = 0; w2 < BN / WN; ++w2) s += zpart[wm + WGM * w2][c];
              z[c] = s + a.fc_b[slot][c];
            }
            const uint32_t idx = entry_idx(e);
            if (f.logits != nullptr)
              for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = (double)z[c];
            const float d = class_margin(z, a.class_mask[slot]);
            const float th = theta_of(f, k, idx);
            pass = d > th;
            defer = f.defer.entries != nullptr && fabsf(d - th) < f.tau[k];
          }
        }
        if (f.logits == nullptr) forward_decision(f, k, e, active, defer, pass);
      }
    }
    if (tid == 0) ticks_s[k] += wall_clock64() - t0;
    __syncthreads();   // the next tile's prologue rewrites LDS (and zpart)
  }
  if (tid < kMaxK && ticks_s[tid] && a.count_ticks) atomicAdd(&a.st->r_ticks[tid], ticks_s[tid]);
}

// ---------------------------------------------------------------- launch
void launch_c4_pass(const GcnnArgs& a, const Forward& f, int prec, int grid, hipStream_t s) {
  const int g1 = grid * (prec == C4_F32 ? 1 : 2);
  if (prec == C4_FP8) {
    hipLaunchKernelGGL(c4_front_kernel<C4_FP8>, dim3(g1), dim3(256), 0, s, a);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_FP8, 2>), dim3(grid * 2), dim3(256), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_FP8, 3>), dim3(grid * 2), dim3(256), 0, s, a, f);
  } else if (prec == C4_BF16) {
    hipLaunchKernelGGL(c4_front_kernel<C4_BF16>, dim3(g1), dim3(256), 0, s, a);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_BF16, 2>), dim3(grid * 2), dim3(256), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_BF16, 3>), dim3(grid * 2), dim3(256), 0, s, a, f);
  } else {
    hipLaunchKernelGGL(c4_front_kernel<C4_F32>, dim3(g1), dim3(256), 0, s, a);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_F32, 2>), dim3(grid * 2), dim3(256), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_F32, 3>), dim3(grid * 2), dim3(256), 0, s, a, f);
  }
}

// ---------------------------------------------------------------- host-side packing
bool c4_shape_ok(int in_hw, int n_layers, const int* widths) {
  return in_hw == 128 && n_layers == 4 && widths[0] == 32 && widths[1] == 64 && widths[2] == 128 && widths[3] == 256;
}

// OCP e4m3 (bias 7, largest finite 448, no infinities), round to nearest even, saturating.
uint8_t c4_fp8_e4m3(float x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
  float a = std::fabs(x);
  if (!(a == a)) return 0x7F;
  if (a >= 448.f) return sign | 0x7E;
  if (a < std::ldexp(1.f, -10)) return sign;            // below half the smallest subnormal
  int e;
  std::frexp(a, &e);                                     // a = m * 2^e, m in [0.5, 1)
  int ex = e - 1;                                        // a in [2^ex, 2^(ex+1))
  if (ex < -6) ex = -6;                                  // subnormal range: spacing 2^-9
  const float q = std::ldexp(1.f, ex - 3);               // spacing of the binade
  float r = std::nearbyint(a / q);                       // round half even (default mode)
  float v = r * q;
  if (v >= 448.f) return sign | 0x7E;
  // encode v
  if (v < std::ldexp(1.f, -6)) return sign | (uint8_t)(int)std::nearbyint(v / std::ldexp(1.f, -9));
  int ev;
  const float mv = std::frexp(v, &ev);                   // v = mv * 2^ev
  const int E = ev - 1 + 7;
  const int M = (int)std::nearbyint((mv * 2.f - 1.f) * 8.f);
  return sign | (uint8_t)((E << 3) | M);
}

float c4_fp8_value(uint8_t b) {
  const int s = b >> 7, E = (b >> 3) & 15, M = b & 7;
  float v = E == 0 ? std::ldexp((float)M, -9) : std::ldexp(1.f + M / 8.f, E - 7);
  if (E == 15 && M == 7) v = NAN;
  return s ? -v : v;
}

// conv weights w: [cout][cin][3][3] canonical fp32.  Element (oc, k) of the GEMM with
// k = tap * cin + ch, tap = 3u + v.
static inline float c4_w(const float* w, int cin, int oc, int k) {
  const int tap = k / cin, ch = k % cin;
  return w[((size_t)(oc * cin + ch) * 3 + tap / 3) * 3 + tap % 3];
}

void c4_pack_front(const float* w1, float scale1, const float* w2, const float* s2, C4FrontPack* out) {
  // layer 1: k = 9u + 3v + c (27 real)
  auto w1k = [&](int oc, int kk) -> float {
    if (kk >= 27) return 0.f;
    const int u = kk / 9, t = kk % 9, v = t / 3, c = t % 3;
    return scale1 * w1[((size_t)(oc * 3 + c) * 3 + u) * 3 + v];
  };
  out->w1b.assign(2 * 64 * 8, 0.f);
  for (int ct = 0; ct < 2; ++ct)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 8; ++e) out->w1b[(ct * 64 + l) * 8 + e] = w1k(ct * 16 + (l & 15), 8 * (l >> 4) + e);
  out->w1f.assign(7 * 2 * 64, 0.f);
  for (int s = 0; s < 7; ++s)
    for (int ct = 0; ct < 2; ++ct)
      for (int l = 0; l < 64; ++l) out->w1f[(s * 2 + ct) * 64 + l] = w1k(ct * 16 + (l & 15), 4 * s + (l >> 4));
  // layer 2 (cin 32): bf16 [tap][ct][lane][8]: channels 8g + e; fp32 the same order
  out->w2b.assign(9 * 4 * 64 * 8, 0.f);
  for (int tp = 0; tp < 9; ++tp)
    for (int ct = 0; ct < 4; ++ct)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e)
          out->w2b[((tp * 4 + ct) * 64 + l) * 8 + e] = c4_w(w2, 32, ct * 16 + (l & 15), tp * 32 + 8 * (l >> 4) + e);
  // fp8 [s][ct][lane][32 bytes]: tap 4s + g, channels 0..31
  out->w2q.assign(3 * 4 * 64 * 32, 0);
  for (int s = 0; s < 3; ++s)
    for (int ct = 0; ct < 4; ++ct)
      for (int l = 0; l < 64; ++l) {
        const int tp = 4 * s + (l >> 4), oc = ct * 16 + (l & 15);
        for (int c = 0; c < 32; ++c)
          out->w2q[((s * 4 + ct) * 64 + l) * 32 + c] = tp < 9 ? c4_fp8_e4m3(c4_w(w2, 32, oc, tp * 32 + c) / s2[oc]) : 0;
      }
}

size_t c4_img_bytes(int prec, int layer) {
  const int cout = layer == 2 ? 128 : 256;
  const int rowb = prec == C4_FP8 ? 128 : 64;
  return (size_t)c4_nkb(prec, layer) * cout * rowb;
}

// A image of a GEMM layer: [kb][oc][UPR units of 16 bytes], unit s holding chunk s ^ swz(oc);
// chunk c of k-block kb holds k = kb * BKE + c * CE + e.
void c4_pack_img(int prec, int layer, const float* w, const float* scale, unsigned char* out) {
  const int cin = layer == 2 ? 64 : 128, cout = layer == 2 ? 128 : 256;
  const int es = prec == C4_FP8 ? 1 : prec == C4_BF16 ? 2 : 4;
  const int rowb = prec == C4_FP8 ? 128 : 64, upr = rowb / 16, ce = 16 / es, bke = rowb / es;
  const int nkb = c4_nkb(prec, layer);
  for (int kb = 0; kb < nkb; ++kb)
    for (int oc = 0; oc < cout; ++oc)
      for (int s = 0; s < upr; ++s) {
        const int c = s ^ (upr == 4 ? c4_swz<4>(oc) : c4_swz<8>(oc));
        unsigned char* dst = out + (((size_t)kb * cout + oc) * upr + s) * 16;
        for (int e = 0; e < ce; ++e) {
          const int kk = kb * bke + c * ce + e;
          const float v = kk < 9 * cin ? c4_w(w, cin, oc, kk) : 0.f;
          if (prec == C4_FP8) {
            dst[e] = c4_fp8_e4m3(v / scale[oc]);
          } else if (prec == C4_BF16) {
            uint32_t u;
            memcpy(&u, &v, 4);
            u += 0x7FFFu + ((u >> 16) & 1u);
            const uint16_t h = (uint16_t)(u >> 16);
            memcpy(dst + 2 * e, &h, 2);
          } else {
            memcpy(dst + 4 * e, &v, 4);
          }
        }
      }
}

}  // namespace hydro
