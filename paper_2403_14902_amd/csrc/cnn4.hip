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
template <> struct C4T<C4_S3> { typedef float T; static constexpr int ES = 4; };

typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ inline floatx4 c4_mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 c4_mfma(float a, float b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
// BF16 contractions use the 32x32x16 MFMA, which keeps the matrix pipe busy with few independent
// accumulators.  Lane l supplies A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32]; output
// element (i, j) sits in lane j + 32 ((i / 4) % 2), value (i % 4) + 4 (i / 8).
typedef float floatx16 __attribute__((ext_vector_type(16)));
__device__ inline floatx16 c4_mfma32(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
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
  if constexpr (P == C4_F32 || P == C4_S3) {
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
// Layer 1's K slot (lane group g, element e of a 16x16x32 fragment) -> k = 9u + 3v + c: lane
// groups 0..2 hold the first 8 of the 9 (pixel, channel) values of input row g, lane group 3 the
// ninth of rows 0..2; slots 27.. (k >= 27) have zero weights.  Each lane then reads five aligned
// dwords of one staged row (or the ninth element of each row) instead of eight 2-byte elements.
__host__ __device__ inline int c4_l1_k(int g, int e) { return g < 3 ? 9 * g + e : e < 3 ? 9 * e + 8 : 27; }

template <int P> struct FrontCfg;
// bytes per layer-1 column slot (32 channels + padding: the slot pitch in 16-byte units is odd so
// that eight consecutive slots fall on distinct bank groups)
template <> struct FrontCfg<C4_F32> { static constexpr int PITCH = 144; };
template <> struct FrontCfg<C4_BF16> { static constexpr int PITCH = 80; };
template <> struct FrontCfg<C4_FP8> { static constexpr int PITCH = 48; };

// bytes per position row of the layer-2 output staging (64 channels + 16 bytes of padding)
template <int P> constexpr int F_TPITCH = 64 * C4T<P>::ES + 16;
// the frame band area, which also stages the layer-2 output (4 waves x 32 positions) after
// layer 1 has read the band
template <int P>
constexpr int F_FRAME_B = ((F_FROWS * F_FPITCH * 2 > 4 * 32 * F_TPITCH<P> ? F_FROWS * F_FPITCH * 2 : 4 * 32 * F_TPITCH<P>) + 15) / 16 * 16;
template <int P> constexpr int front_lds_bytes() { return F_FRAME_B<P> + F_RING * F_SLOTS * FrontCfg<P>::PITCH; }

// Layer-1 column j -> its slot in a ring row.
__device__ inline int f_slot(int j) { return (j & 1) ? 32 + ((j + 1) >> 1) : (j >> 1); }

// X3 (with P = C4_F32 only): the three-product arithmetic of the C4_X3 tier
template <int P, bool U8, bool X3 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == C4_F32 ? 1 : 2)))
void c4_front_kernel(GcnnArgs a) {
  typedef typename C4T<P>::T T;
  constexpr int ES = C4T<P>::ES;
  constexpr int PITCH = FrontCfg<P>::PITCH;
  __shared__ __attribute__((aligned(16))) unsigned char lds[front_lds_bytes<P>()];
  __shared__ unsigned long long ticks_s[kMaxK];
  // per-slot epilogue constants: layer-1 bias [32], layer-2 bias [64], FP8 layer-2 scales [64]
  __shared__ __attribute__((aligned(16))) float consts_s[160];
  __shared__ __attribute__((aligned(16))) bf16x8 w1_s[2][64];   // layer-1 fragments (bf16 tiers)
  __bf16* fb = reinterpret_cast<__bf16*>(lds);          // staged frame band (raw values, bf16)
  unsigned char* ring = lds + F_FRAME_B<P>;                // layer-1 output rows
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, l16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < kMaxK) ticks_s[tid] = 0;
  // the left pad column (slot 32) of every ring row is a zero activation
  for (int q = tid; q < F_RING * (PITCH / 4); q += 256)
    reinterpret_cast<uint32_t*>(ring + (q / (PITCH / 4)) * F_SLOTS * PITCH + 32 * PITCH)[q % (PITCH / 4)] = 0u;

  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += a.c4[i] ? a.q.counts[a.pred[i]] : 0;
  // frame staging: chunk q (16 bytes) of band row r; uint8 frames: 24 chunks a row, bf16: 48.
  // The next band's chunks are loaded into registers while the current band's layer 2 runs (the
  // next frame's first band during the last band), and converted into LDS after it.
  constexpr int CPR = U8 ? 24 : 48;
  constexpr int NCHUNK = F_FROWS * CPR;
  constexpr int NPF = (NCHUNK + 255) / 256;
  constexpr int FROWB = 128 * 3 * (U8 ? 1 : 2);
  u32x4 pf[NPF];
  // the loads are unconditional (indices clamped; a clamped chunk is never committed), so that the
  // registers are not merged across branches and the wait for them falls at the commit
#define C4_FISSUE(frm_, band_)                                                                     \
  do {                                                                                             \
    _Pragma("unroll") for (int c = 0; c < NPF; ++c) {                                              \
      const int q = min(tid + 256 * c, NCHUNK - 1);                                                \
      const int y = max(16 * (band_) - 1 + q / CPR, 0);                                            \
      pf[c] = reinterpret_cast<const u32x4*>((frm_) + (int64_t)y * FROWB)[q % CPR];                \
    }                                                                                              \
  } while (0)
#define C4_FCOMMIT(band_)                                                                          \
  do {                                                                                             \
    /* the pad column (elements 1..3 of each row; the area also stages layer-2 output) */           \
    if (tid < F_FROWS * 4) fb[(tid >> 2) * F_FPITCH + (tid & 3)] = static_cast<__bf16>(a.pad_raw); \
    _Pragma("unroll") for (int c = 0; c < NPF; ++c) {                                              \
      const int q = tid + 256 * c;                                                                 \
      if (q < NCHUNK) {                                                                            \
        const int r = q / CPR, j = q % CPR, y = 16 * (band_) - 1 + r;                              \
        __bf16* dst = fb + r * F_FPITCH + 4 + (U8 ? 16 : 8) * j;                                   \
        if (y < 0) {                                                                               \
          _Pragma("unroll") for (int e = 0; e < (U8 ? 16 : 8); ++e) dst[e] = static_cast<__bf16>(a.pad_raw); \
        } else if (U8) {                                                                           \
          _Pragma("unroll") for (int h = 0; h < 4; ++h) {                                          \
            alignas(8) __bf16 e4[4];                                                               \
            _Pragma("unroll") for (int e = 0; e < 4; ++e)                                          \
              e4[e] = static_cast<__bf16>((float)((pf[c][h] >> (8 * e)) & 0xFFu));                 \
            *reinterpret_cast<uint2*>(dst + 4 * h) = *reinterpret_cast<const uint2*>(e4);           \
          }                                                                                        \
        } else {                                                                                   \
          *reinterpret_cast<uint2*>(dst) = make_uint2(pf[c][0], pf[c][1]);                         \
          *reinterpret_cast<uint2*>(dst + 4) = make_uint2(pf[c][2], pf[c][3]);                     \
        }                                                                                          \
      }                                                                                            \
    }                                                                                              \
  } while (0)
  bool pf_valid = false;      // pf holds the first band of frame pf_idx
  uint32_t pf_idx = 0;

  // per-slot state (reloaded when the slot changes)
  int cur = -1;
  bf16x8 w1t[P == C4_F32 ? 3 : 1][2];   // layer-1 weights, FP32 arithmetic: [term][channel tile]
  bf16x8 w2b[P == C4_BF16 ? 9 : 1][2][2];            // [tap][channel half of the tap][32-channel tile]
  i32x8 w2q[P == C4_FP8 ? 3 : 1][P == C4_FP8 ? 4 : 1];
  float inv_s1 = 1.f, inv_s2 = 1.f;

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
      // (the previous frame's last barrier ordered every read of the previous slot's constants)
      if (tid < 32) consts_s[tid] = a.bias[slot][0][tid];
      else if (tid < 96) consts_s[tid] = a.bias[slot][1][tid - 32];
      else if (tid < 160)
        consts_s[tid] = P == C4_FP8 ? a.c4_wscale[slot][0][tid - 96] * a.c4_ascale[slot][0] : 1.f;
      if constexpr (P == C4_F32) {
        const bf16x8* w1 = static_cast<const bf16x8*>(a.c4_w1f[slot]);
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) w1t[t][ct] = w1[(t * 2 + ct) * 64 + lane];
      } else {
        if (tid < 128) w1_s[tid >> 6][tid & 63] = static_cast<const bf16x8*>(a.c4_w1b[slot])[tid];
      }
      if constexpr (P == C4_BF16) {
        const bf16x8* w2 = static_cast<const bf16x8*>(a.c4_w2[slot][C4_BF16]);
#pragma unroll
        for (int tp = 0; tp < 9; ++tp)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) w2b[tp][h][c2] = w2[((tp * 2 + h) * 2 + c2) * 64 + lane];
      }
      if constexpr (P == C4_FP8) {
        const i32x8* w2 = static_cast<const i32x8*>(a.c4_w2[slot][C4_FP8]);
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) w2q[s][ct] = w2[(s * 4 + ct) * 64 + lane];
        inv_s1 = 1.f / a.c4_ascale[slot][0];
        inv_s2 = 1.f / a.c4_ascale[slot][1];
      }
    }
    const unsigned long long t0 = wall_clock64();
    const unsigned char* frame = static_cast<const unsigned char*>(a.fr.base) + (int64_t)idx * a.fr.elems * (U8 ? 1 : 2);
    // the work item after this one (its first band is prefetched during this frame's last band)
    const unsigned char* next_frame = nullptr;
    uint32_t nidx = 0;
    {
      const int t2 = t + gridDim.x;
      if (t2 < total) {
        int off2 = t2, eb2 = 0, s2 = -1;
        for (int i = 0; i < a.n_preds; ++i) {
          const int c = a.c4[i] ? a.q.counts[a.pred[i]] : 0;
          if (off2 < c) { s2 = i; break; }
          off2 -= c;
          eb2 += a.q.counts[a.pred[i]];
        }
        if (s2 >= 0 && (int64_t)eb2 + off2 < a.act_cap) {
          nidx = entry_idx(a.q.entries[(int64_t)a.pred[s2] * a.q.cap + off2]);
          next_frame = static_cast<const unsigned char*>(a.fr.base) + (int64_t)nidx * a.fr.elems * (U8 ? 1 : 2);
        }
      }
    }
    if (!(pf_valid && pf_idx == idx)) C4_FISSUE(frame, 0);
    C4_FCOMMIT(0);
    pf_valid = false;
    T* out2 = reinterpret_cast<T*>(a.c4_act2) + ent * (32 * 32 * 64);
    unsigned* amax1 = a.c4_act_max ? a.c4_act_max + k * 4 + 0 : nullptr;
    unsigned* amax2 = a.c4_act_max ? a.c4_act_max + k * 4 + 1 : nullptr;

    for (int b = 0; b < F_NB; ++b) {
      {
        // next band of this frame, or the first band of the next work item (this frame again when
        // there is none: a load whose data is not used); in flight over this band's layers 1 and 2
        const unsigned char* src = b + 1 < F_NB ? frame : next_frame != nullptr ? next_frame : frame;
        C4_FISSUE(src, b + 1 < F_NB ? b + 1 : 0);
        if (b + 1 == F_NB && next_frame != nullptr) {
          pf_valid = true;
          pf_idx = nidx;
        }
      }
      // the ring slot of layer-1 row -1 is zero for the first band
      const int base_slot = (8 * b) % F_RING;   // ring index of layer-1 row 8b - 1
      if (b == 0)
        for (int q = tid; q < F_SLOTS * PITCH / 4; q += 256) reinterpret_cast<uint32_t*>(ring)[q] = 0u;
      __syncthreads();

      // ---- layer 1: rows 8b + 2w, 8b + 2w + 1 (local i = 2w, 2w+1), 64 columns each
#pragma unroll 1
      for (int pt = 0; pt < 8; ++pt) {
        const int il = 2 * wave + (pt >> 2), j = (pt & 3) * 16 + l16;
        floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        // the 9 values of input row u for output column j (pixels 2j-1 .. 2j+1) are elements
        // 6j+1 .. 6j+9 of the staged row; dwords from element 6j hold them in pairs
        const uint32_t* rw = reinterpret_cast<const uint32_t*>(fb + (2 * il) * F_FPITCH + 6 * j);
        constexpr int RP = F_FPITCH / 2;      // dwords per staged row
        uint32_t d[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) d[i] = rw[g < 3 ? g * RP + i : (i < 3 ? i * RP + 4 : 4)];
        uint32_t xw[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t row = __builtin_amdgcn_alignbit(d[i + 1], d[i], 16);   // elements 2i+1, 2i+2
          const uint32_t ninth = i == 0 ? (d[0] >> 16) | (d[1] & 0xFFFF0000u) : i == 1 ? d[2] >> 16 : 0u;
          xw[i] = g < 3 ? row : ninth;
        }
        bf16x8 xb;
        __builtin_memcpy(&xb, xw, sizeof(xb));
        if constexpr (P == C4_F32) {
          // raw frame values are exact in bf16 and the weights are the sum of their three terms:
          // every product exact, fp32 sums (smallest term first); X3 drops the lowest term
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            if constexpr (!X3) acc[ct] = c4_mfma(w1t[2][ct], xb, acc[ct]);
            acc[ct] = c4_mfma(w1t[1][ct], xb, acc[ct]);
            acc[ct] = c4_mfma(w1t[0][ct], xb, acc[ct]);
          }
        } else {
          acc[0] = c4_mfma(w1_s[0][lane], xb, acc[0]);
          acc[1] = c4_mfma(w1_s[1][lane], xb, acc[1]);
        }
        const int ridx = (base_slot + 1 + il) % F_RING;
        unsigned char* dst = ring + (ridx * F_SLOTS + f_slot(j)) * PITCH;
        float m = 0.f;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const float4 bb = *reinterpret_cast<const float4*>(consts_s + ct * 16 + 4 * g);
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
      floatx4 acc[P == C4_BF16 ? 1 : 2][4][2];
      floatx16 acc32[P == C4_BF16 ? 2 : 1];
      if constexpr (P == C4_BF16) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
          for (int e = 0; e < 16; ++e) acc32[c2][e] = 0.f;
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[h][ct][mt] = (floatx4){0.f, 0.f, 0.f, 0.f};
      }
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
        // the wave's 32 positions (lane % 32) x two 32-channel tiles; k-step (tap, h): channels
        // 16h .. 16h + 15 of the tap, lane half lane / 32 taking 8 of them
        const int j = lane & 31, hg = lane >> 5;
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
          const int u = tp / 3, v = tp % 3;
          const int rr = (base_slot + 2 * wave + u) % F_RING;
          const int sl = v == 1 ? j : v == 0 ? 32 + j : 33 + j;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bf16x8 xb = *reinterpret_cast<const bf16x8*>(ring + (rr * F_SLOTS + sl) * PITCH + (16 * h + 8 * hg) * 2);
            acc32[0] = c4_mfma32(w2b[tp][h][0], xb, acc32[0]);
            acc32[1] = c4_mfma32(w2b[tp][h][1], xb, acc32[1]);
          }
          // keep each tap's fragment reads next to its MFMAs (hoisting them all spills registers)
          if (tp & 1) __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // FP32 arithmetic from bf16 MFMAs: per tap, lane group g takes input channels 8g..8g+7
        // (one 16x16x32 k-step); the fp32 layer-1 activations are split into three bf16 terms
        // and multiplied with the three-term weights (L2-resident, [tap][ct][term][lane]); the
        // six products down to 2^-24 relative are summed, smallest first
        const bf16x8* w2 = static_cast<const bf16x8*>(a.c4_w2[slot][C4_S3]);
#pragma unroll 1
        for (int tp = 0; tp < 9; ++tp) {
          const int u = tp / 3, v = tp % 3;
          const int rr = (base_slot + 2 * wave + u) % F_RING;
          bf16x8 xs[2][3];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const int j = mt * 16 + l16;
            const int sl = v == 1 ? j : v == 0 ? 32 + j : 33 + j;
            const float4* src = reinterpret_cast<const float4*>(ring + (rr * F_SLOTS + sl) * PITCH + 32 * g);
            const float4 p0 = src[0], p1 = src[1];
            const float xv[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const __bf16 h = static_cast<__bf16>(xv[e]);
              const float r1 = xv[e] - static_cast<float>(h);
              const __bf16 m = static_cast<__bf16>(r1);
              xs[mt][0][e] = h;
              xs[mt][1][e] = m;
              xs[mt][2][e] = static_cast<__bf16>(r1 - static_cast<float>(m));
            }
          }
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const bf16x8 wh = w2[((tp * 4 + ct) * 3 + 0) * 64 + lane];
            const bf16x8 wm = w2[((tp * 4 + ct) * 3 + 1) * 64 + lane];
            const bf16x8 wl = w2[((tp * 4 + ct) * 3 + 2) * 64 + lane];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
              floatx4 c = acc[0][ct][mt];
              if constexpr (X3) {       // hi x hi + hi x mid + mid x hi (about 2^-16 relative)
                c = c4_mfma(wh, xs[mt][1], c);
                c = c4_mfma(wm, xs[mt][0], c);
              } else {
                c = c4_mfma(wh, xs[mt][2], c);
                c = c4_mfma(wm, xs[mt][1], c);
                c = c4_mfma(wh, xs[mt][1], c);
                c = c4_mfma(wl, xs[mt][0], c);
                c = c4_mfma(wm, xs[mt][0], c);
              }
              acc[0][ct][mt] = c4_mfma(wh, xs[mt][0], c);
            }
          }
        }
      }
      // bias + ReLU -> layer-2 activations of row 4b + w, staged through this wave's slice of the
      // (now free) frame band area so that the global stores are whole contiguous lines
      {
        const int orow = 4 * b + wave;
        unsigned char* tw = lds + wave * 32 * F_TPITCH<P>;
        float m = 0.f;
        // 8 quads of 4 consecutive channels per lane: (position j, first channel c0, values)
#pragma unroll
        for (int qd = 0; qd < 8; ++qd) {
          int j, c0;
          float x[4];
          if constexpr (P == C4_BF16) {
            const int c2 = qd >> 2, vq = qd & 3;
            j = lane & 31;
            c0 = c2 * 32 + 8 * vq + 4 * (lane >> 5);
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = acc32[c2][4 * vq + r];
          } else {
            const int mt = qd >> 2, ct = qd & 3;
            j = mt * 16 + l16;
            c0 = ct * 16 + 4 * g;
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = acc[0][ct][mt][r] + acc[1][ct][mt][r];
          }
          const float4 bb = *reinterpret_cast<const float4*>(consts_s + 32 + c0);
          const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
          float sv[4] = {1.f, 1.f, 1.f, 1.f};
          if constexpr (P == C4_FP8) {
            const float4 ss = *reinterpret_cast<const float4*>(consts_s + 96 + c0);
            sv[0] = ss.x; sv[1] = ss.y; sv[2] = ss.z; sv[3] = ss.w;
          }
          float v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float xr = x[r];
            if constexpr (P == C4_FP8) xr *= sv[r];
            v[r] = fmaxf(xr + bv[r], 0.f);
            m = fmaxf(m, v[r]);
            v[r] *= inv_s2;
          }
          c4_store4<P>(tw + j * F_TPITCH<P> + c0 * ES, v[0], v[1], v[2], v[3]);
        }
        if constexpr (P == C4_F32) c4_track_max(amax2, m);
        // the wave's 32 positions x 64 channels are contiguous in the output: 16 bytes a lane
        constexpr int RB = 64 * ES;                      // bytes of one position
        u32x4* dst = reinterpret_cast<u32x4*>(reinterpret_cast<unsigned char*>(out2) + (int64_t)orow * 32 * RB);
#pragma unroll
        for (int i = 0; i < RB / 32; ++i) {
          const int off = i * 1024 + lane * 16;
          dst[off / 16] = *reinterpret_cast<const u32x4*>(tw + (off / RB) * F_TPITCH<P> + off % RB);
        }
      }
      __syncthreads();   // the next band restages the frame rows and overwrites ring rows
      if (b + 1 < F_NB) C4_FCOMMIT(b + 1);
    }
    if (tid == 0) ticks_s[k] += wall_clock64() - t0;
  }
  __syncthreads();
  if (tid < kMaxK && ticks_s[tid] && a.count_ticks) atomicAdd(&a.st->r_ticks[tid], ticks_s[tid]);
#undef C4_FISSUE
#undef C4_FCOMMIT
}

// ---------------------------------------------------------------- layers 3 and 4: implicit GEMM
template <int P> struct GemmCfg;
// ROWB: bytes of one LDS tile row per k-block; UPR: 16-byte units per row; CE: elements per unit;
// KSUB: MFMA k-steps per k-block
// (128-byte rows: 2 bf16 / 8 fp32 / 1 fp8 MFMA k-steps per k-block and barrier)
template <> struct GemmCfg<C4_F32> { static constexpr int ROWB = 128, UPR = 8, CE = 4, KSUB = 8; };
template <> struct GemmCfg<C4_BF16> { static constexpr int ROWB = 128, UPR = 8, CE = 8, KSUB = 2; };
template <> struct GemmCfg<C4_FP8> { static constexpr int ROWB = 128, UPR = 8, CE = 16, KSUB = 1; };
// S3: B rows (fp32 activations) as FP32; A rows are three 64-byte bf16 rows (hi, mid, lo)
template <> struct GemmCfg<C4_S3> { static constexpr int ROWB = 128, UPR = 8, CE = 4, KSUB = 1; };

// chunk swizzle of tile row r: rows of 4 units xor (r/2) mod 4, rows of 8 units xor r mod 8
template <int UPR>
__host__ __device__ inline int c4_swz(int r) { return UPR == 4 ? ((r >> 1) & 3) : (r & 7); }

template <int P, int LAYER> struct GemmShape;
// LAYER 2 = the third conv (32x32x64 -> 16x16x128), LAYER 3 = the fourth (16x16x128 -> 8x8x256).
// Eight waves, each a 64 x 64 tile (4 x 4 MFMA tiles): layer 3 tiles one frame (256 positions) x
// all 128 channels, layer 4 two frames (128 positions) x all 256 channels (the head needs every
// channel of a frame in one workgroup).
template <int P> struct GemmShape<P, 2> {
  static constexpr int CIN = 64, COUT = 128, HIN = 32, HOUT = 16, BM = 256, BN = 128;
};
template <int P> struct GemmShape<P, 3> {
  static constexpr int CIN = 128, COUT = 256, HIN = 16, HOUT = 8, BM = 128, BN = 256;
};

// Output channel held by row R of the BF16 third-convolution weight image.  In a 16x16 MFMA
// tile, lane group g holds rows 4 g .. 4 g + 3 of the tile; with this order the four tiles of a
// wave's 64 channels give lane group g channels 8 g .. 8 g + 7 (tiles 0, 1) and 32 + 8 g .. + 7
// (tiles 2, 3), so each lane stores 16 contiguous bytes and a position's 64 channels are two
// 64-byte runs per store instruction.
__host__ __device__ inline int c4_l3_channel(int row) {
  const int blk = row / 64, w = row % 64, nt = w / 16, i = w % 16;
  return 64 * blk + (nt / 2) * 32 + 8 * (i / 4) + (nt % 2) * 4 + i % 4;
}

__host__ __device__ inline int c4_nkb(int prec, int layer) {
  const int cin = layer == 2 ? 64 : 128;
  const int bke = prec == C4_FP8 ? 128 : prec == C4_BF16 ? 64 : 32;   // FP32 and S3: 32
  return (9 * cin + bke - 1) / bke;
}


// Epilogue of one GEMM tile (acc: the 64 x 64 block of wave (wm, wn) of the tile).  Layer 3: bias +
// ReLU, stored as the next layer's activations.  Layer 4: bias + ReLU, mean over each frame's 64
// positions, this wave's share of the FC, then the margin and decision (or the logits).
// PERM: the tile's channels follow c4_l3_channel (BF16 third convolution).
template <int P, int LAYER, bool PERM = false>
__device__ inline void c4_gemm_epilogue(const GcnnArgs& a, const Forward& f, const floatx4 (&acc)[4][4], int slot,
                                        int k, int cb, int ebase, int64_t row0, int64_t rows, const float* ep_bias,
                                        const float* ep_scale, const float* fcw_s, float (*zpart)[kClasses]) {
  typedef typename C4T<P>::T T;
  typedef GemmShape<P, LAYER> S;
  constexpr int COUT = S::COUT, HOUT = S::HOUT, PP = HOUT * HOUT, BM = S::BM, BN = S::BN, WM = 64, WN = 64;
  constexpr int MT = WM / 16, NT = WN / 16, WGM = BM / WM;
  constexpr bool HEAD = LAYER == 3;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave % WGM, wn = wave / WGM;
  if constexpr (PERM) {
    static_assert(P == C4_BF16 && !HEAD, "permuted channels: BF16 third convolution");
    __bf16* out = reinterpret_cast<__bf16*>(a.c4_act3);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int64_t row = row0 + wm * WM + mt * 16 + l16;
      const bool valid = row < rows && ebase + row / PP < a.act_cap;
      const int64_t e = valid ? row / PP : 0;
      const int p = (int)(row % PP);
      __bf16* o = out + ((int64_t)ebase + e) * (PP * COUT) + (int64_t)p * COUT + cb * BN;
#pragma unroll
      for (int h = 0; h < 2; ++h) {              // tiles 2h, 2h + 1: channels 32 h + 8 g .. + 7
        const int cl = wn * WN + 32 * h + 8 * g;
        const floatx4 b0 = *reinterpret_cast<const floatx4*>(ep_bias + cl);
        const floatx4 b1 = *reinterpret_cast<const floatx4*>(ep_bias + cl + 4);
        alignas(16) __bf16 v[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v[r] = static_cast<__bf16>(fmaxf(acc[2 * h][mt][r] + b0[r], 0.f));
          v[4 + r] = static_cast<__bf16>(fmaxf(acc[2 * h + 1][mt][r] + b1[r], 0.f));
        }
        if (valid) *reinterpret_cast<uint4*>(o + cl) = *reinterpret_cast<const uint4*>(v);
      }
    }
  } else if constexpr (!HEAD) {
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
        const int cl = wn * WN + nt * 16 + 4 * g;    // channel within the tile
        const int ch = cb * BN + cl;
        const floatx4 bb = *reinterpret_cast<const floatx4*>(ep_bias + cl);
        floatx4 sc = {1.f, 1.f, 1.f, 1.f};
        if constexpr (P == C4_FP8) sc = *reinterpret_cast<const floatx4*>(ep_scale + cl);
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float x = acc[nt][mt][r];
          if constexpr (P == C4_FP8) x *= sc[r];
          v[r] = fmaxf(x + bb[r], 0.f);
          m = fmaxf(m, valid ? v[r] : 0.f);
          v[r] *= inv_out;
        }
        if (valid) c4_store4<P>(o + ch, v[0], v[1], v[2], v[3]);
      }
    }
    if constexpr (P == C4_F32 || P == C4_S3) c4_track_max(amax, m);
  } else {
    // wave (wm, wn): frame wm of the tile, channels wn*WN .. +WN-1.  Pool over the frame's 64
    // positions, then this wave's share of FC.
    const int64_t frow = row0 + wm * WM;             // first row of the frame
    const bool fvalid = frow < rows;
    float zc = 0.f;                                   // lane l16 < 10: class l16
    const int cls = l16 < kClasses ? l16 : 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int chb = wn * WN + nt * 16 + 4 * g;
      const floatx4 bb = *reinterpret_cast<const floatx4*>(ep_bias + chb);
      floatx4 sc = {1.f, 1.f, 1.f, 1.f};
      if constexpr (P == C4_FP8) sc = *reinterpret_cast<const floatx4*>(ep_scale + chb);
      float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float x = acc[nt][mt][r];
          if constexpr (P == C4_FP8) x *= sc[r];
          s[r] += fmaxf(x + bb[r], 0.f);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float gch = row_sum16(s[r]) * (1.f / PP);
        zc += gch * fcw_s[(chb + r) * kClasses + cls];
      }
    }
    if (l16 >= kClasses) zc = 0.f;
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
            float sum = 0.f;
            for (int w2 = 0; w2 < BN / WN; ++w2) sum += zpart[wm + WGM * w2][c];
            z[c] = sum + a.fc_b[slot][c];
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
}

// X3 (with P = C4_S3 only): the three-product arithmetic of the C4_X3 tier
template <int P, int LAYER, bool X3 = false>
__global__ __launch_bounds__(512) void c4_gemm_kernel(GcnnArgs a, Forward f) {
  typedef typename C4T<P>::T T;
  typedef GemmCfg<P> G;
  typedef GemmShape<P, LAYER> S;
  constexpr int ES = C4T<P>::ES, UPR = G::UPR, CE = G::CE, BKE = G::ROWB / ES;
  constexpr int CIN = S::CIN, COUT = S::COUT, HIN = S::HIN, HOUT = S::HOUT, PP = HOUT * HOUT;
  constexpr int BM = S::BM, BN = S::BN, WM = 64, WN = 64;
  constexpr int MT = WM / 16, NT = WN / 16;
  constexpr int WGM = BM / WM;                        // waves along M (8 waves in all)
  constexpr int NKB = (9 * CIN + BKE - 1) / BKE;
  constexpr bool S3 = P == C4_S3;
  constexpr int ATERMS = X3 ? 2 : 3;                  // weight terms staged (X3 reads hi and mid)
  constexpr int AUNITS = S3 ? ATERMS * BN * 4 : BN * UPR;   // A: S3 holds a 64-byte row per channel and term
  constexpr int UNITS = AUNITS + BM * UPR;            // 16-byte units of one stage
  constexpr int NI = UNITS / 64 / 8;                  // load instructions per wave and stage
  constexpr int NIA = AUNITS / 64 / 8;                // ... of them for A (the rest gather B)
  constexpr int STAGE = UNITS * 16;
  constexpr int NS = S3 && !X3 ? 2 : 3;               // stages in flight (what LDS holds)
  constexpr bool HEAD = LAYER == 3;
  static_assert(UNITS % 512 == 0 && AUNITS % 512 == 0, "stage rows must fill the waves' load units");
  static_assert(WGM * (BN / WN) == 8, "eight waves per tile");
  static_assert(!HEAD || (BN == COUT && WM == PP), "the head needs whole frames per wave and all channels");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[NS * STAGE];
  __shared__ float zpart[8][kClasses];
  // epilogue constants of the tile, staged before its k loop: bias and (FP8) weight scale x input
  // activation scale of its channels, and (last layer) the FC weights
  __shared__ __attribute__((aligned(16))) float ep_bias[BN];
  __shared__ __attribute__((aligned(16))) float ep_scale[P == C4_FP8 ? BN : 1];
  __shared__ float fcw_s[HEAD ? COUT * kClasses : 1];
  __shared__ unsigned long long ticks_s[kMaxK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave % WGM, wn = wave / WGM;
  if (tid < kMaxK) ticks_s[tid] = 0;
  const T* act_in = reinterpret_cast<const T*>(LAYER == 2 ? a.c4_act2 : a.c4_act3);
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)lds);
  // tiles: per slot ceil(count * PP / BM) x COUT / BN
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i)
    if (a.c4[i]) total += (int)(((int64_t)a.q.counts[a.pred[i]] * PP + BM - 1) / BM) * (COUT / BN);
  const int u_slot = lane % UPR;     // the LDS slot of every unit this lane loads

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
    const unsigned char* img = static_cast<const unsigned char*>(a.c4_img[slot][LAYER - 2][P]) +
                               (size_t)cb * BN * (S3 ? 64 : G::ROWB);
    // (the previous tile's closing barrier ordered every read of these)
    for (int i = tid; i < BN; i += 512) {
      ep_bias[i] = a.bias[slot][LAYER][cb * BN + i];
      if constexpr (P == C4_FP8) ep_scale[i] = a.c4_wscale[slot][LAYER - 1][cb * BN + i] * a.c4_ascale[slot][LAYER - 1];
    }
    if constexpr (HEAD)
      for (int i = tid; i < COUT * kClasses; i += 512) fcw_s[i] = a.fc_w[slot][i];

    // B rows this lane gathers: frame pointer, output position and chunk, per load instruction
    const T* bsrc[NI - NIA];
    int boi[NI - NIA], boj[NI - NIA], bch[NI - NIA];
#pragma unroll
    for (int i = NIA; i < NI; ++i) {
      const int U = (wave + 8 * i) * 64 + lane - AUNITS;
      const int rb = U / UPR;
      const int64_t row = row0 + rb;
      const bool valid = row < rows && ebase + row / PP < a.act_cap;
      const int64_t e = valid ? row / PP : 0;
      const int p = valid ? (int)(row % PP) : 0;
      bsrc[i - NIA] = act_in + ((int64_t)ebase + e) * (HIN * HIN * CIN);
      boi[i - NIA] = valid ? p / HOUT : -1000;        // invalid rows read the zero page
      boj[i - NIA] = p % HOUT;
      bch[i - NIA] = (u_slot ^ c4_swz<UPR>(rb)) * CE;  // element offset of the chunk in the k-block
    }
    // stage kb of A (packed image, a straight copy) and B (im2col gathers) into LDS buffer buf
    auto issue = [&](int kb, int buf) {
      const uint32_t base = lds0 + buf * STAGE;
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int q = wave + 8 * i;
        const void* src;
        if (i < NIA) {
          // S3 image: [kb][term][oc][64 bytes], the tile's channels of each term contiguous
          if constexpr (S3) {
            const int U = q * 64 + lane, term = U / (BN * 4), r = (U / 4) % BN;
            src = img + (size_t)kb * 3 * COUT * 64 + ((size_t)term * COUT + r) * 64 + (U % 4) * 16;
          } else {
            src = img + (size_t)kb * COUT * G::ROWB + (size_t)(q * 64 + lane) * 16;
          }
        } else {
          const int ke = kb * BKE + bch[i - NIA];
          const int tap = ke / CIN, ch = ke % CIN;
          const int y = 2 * boi[i - NIA] + tap / 3 - 1, x = 2 * boj[i - NIA] + tap % 3 - 1;
          const bool ok = tap < 9 && y >= 0 && x >= 0 && y < HIN && x < HIN;
          src = ok ? static_cast<const void*>(bsrc[i - NIA] + (y * HIN + x) * CIN + ch) : a.zero_page;
        }
        lds_dma16(src, __builtin_amdgcn_readfirstlane(base + q * 1024));
      }
    };

    floatx4 acc[NT][MT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (floatx4){0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int buf) {
      const unsigned char* A = lds + buf * STAGE;
      const unsigned char* B = A + AUNITS * 16;
      if constexpr (S3) {
        // one 32-deep k-step: lane group g takes k = 8 g .. 8 g + 7 (A chunk g of each 64-byte
        // row, B chunks 2 g and 2 g + 1 of each 128-byte fp32 row); the fp32 activations are
        // split a = hi + mid + lo in bf16 and the six products down to 2^-24 relative are summed,
        // smallest first
        bf16x8 aw[3][NT];
#pragma unroll
        for (int term = 0; term < ATERMS; ++term)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int r = wn * WN + nt * 16 + l16;
            aw[term][nt] = *reinterpret_cast<const bf16x8*>(A + ((term * BN + r) * 4 + (g ^ c4_swz<4>(r))) * 16);
          }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int r = wm * WM + mt * 16 + l16;
          const floatx4 x0 = *reinterpret_cast<const floatx4*>(B + (r * UPR + ((2 * g) ^ c4_swz<UPR>(r))) * 16);
          const floatx4 x1 = *reinterpret_cast<const floatx4*>(B + (r * UPR + ((2 * g + 1) ^ c4_swz<UPR>(r))) * 16);
          bf16x8 xh, xm, xl;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float v = e < 4 ? x0[e] : x1[e - 4];
            const __bf16 h = static_cast<__bf16>(v);
            const float r1 = v - static_cast<float>(h);
            const __bf16 m = static_cast<__bf16>(r1);
            xh[e] = h;
            xm[e] = m;
            xl[e] = static_cast<__bf16>(r1 - static_cast<float>(m));
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            floatx4 c = acc[nt][mt];
            if constexpr (X3) {         // hi x hi + hi x mid + mid x hi (about 2^-16 relative)
              c = c4_mfma(aw[0][nt], xm, c);
              c = c4_mfma(aw[1][nt], xh, c);
            } else {
              c = c4_mfma(aw[0][nt], xl, c);
              c = c4_mfma(aw[1][nt], xm, c);
              c = c4_mfma(aw[0][nt], xm, c);
              c = c4_mfma(aw[2][nt], xh, c);
              c = c4_mfma(aw[1][nt], xh, c);
            }
            acc[nt][mt] = c4_mfma(aw[0][nt], xh, c);
          }
        }
      } else if constexpr (P == C4_FP8) {
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
        // k-step ks reads chunk 4 ks + g of each row
#pragma unroll
        for (int ks = 0; ks < G::KSUB; ++ks) {
          bf16x8 af[NT], bfr[MT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int r = wn * WN + nt * 16 + l16;
            af[nt] = *reinterpret_cast<const bf16x8*>(A + (r * UPR + ((4 * ks + g) ^ c4_swz<UPR>(r))) * 16);
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int r = wm * WM + mt * 16 + l16;
            bfr[mt] = *reinterpret_cast<const bf16x8*>(B + (r * UPR + ((4 * ks + g) ^ c4_swz<UPR>(r))) * 16);
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = c4_mfma(af[nt], bfr[mt], acc[nt][mt]);
        }
      } else {
        // lane group g reads chunks 2g and 2g + 1 (8 values); k-step j uses value j
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          floatx4 af[NT], bfr[MT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int r = wn * WN + nt * 16 + l16;
            af[nt] = *reinterpret_cast<const floatx4*>(A + (r * UPR + ((2 * g + h) ^ c4_swz<UPR>(r))) * 16);
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int r = wm * WM + mt * 16 + l16;
            bfr[mt] = *reinterpret_cast<const floatx4*>(B + (r * UPR + ((2 * g + h) ^ c4_swz<UPR>(r))) * 16);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = c4_mfma(af[nt][j], bfr[mt][j], acc[nt][mt]);
        }
      }
    };

    // NS-stage ring, one barrier per k-block: block kb + NS - 1 is loaded while block kb is read.
    // The wait before the barrier covers this wave's loads of block kb (the blocks issued after
    // it may stay in flight); the barrier then covers every wave's.
#pragma unroll
    for (int s0 = 0; s0 < NS - 1; ++s0)
      if (s0 < NKB) issue(s0, s0);
#pragma unroll 1
    for (int kb = 0; kb < NKB; ++kb) {
      const int ahead = min(NS - 2, NKB - 1 - kb);
      if (NS >= 4 && ahead >= 2) wait_vmcnt<2 * NI>();
      else if (NS >= 3 && ahead >= 1) wait_vmcnt<NI>();
      else wait_vmcnt<0>();
      __syncthreads();
      if (kb + NS - 1 < NKB) issue(kb + NS - 1, (kb + NS - 1) % NS);
      compute(kb % NS);
    }

    c4_gemm_epilogue<P, LAYER>(a, f, acc, slot, k, cb, ebase, row0, rows, ep_bias, ep_scale, fcw_s, zpart);
    if (tid == 0) ticks_s[k] += wall_clock64() - t0;
    __syncthreads();   // the next tile's prologue rewrites LDS (stages, constants, zpart)
  }
  if (tid < kMaxK && ticks_s[tid] && a.count_ticks) atomicAdd(&a.st->r_ticks[tid], ticks_s[tid]);
}

// BF16 layers 3 and 4 (the first pass): the implicit GEMM of c4_gemm_kernel with its pipeline
// restructured so that the matrix cores are not left waiting on LDS or memory latency:
//  - one stream of k-blocks over all of a workgroup's tiles: the first stages of the next tile are
//    loaded during the current tile's last k-blocks and its epilogue;
//  - each k-block's fragments are read into registers one MFMA step ahead (two register sets), and
//    the barrier that publishes the next k-block and frees the oldest buffer sits between the two
//    MFMA steps of a k-block, so that every wave arrives at it with MFMAs in its pipe and issues
//    its next fragment reads before the MFMAs that follow.
// The arithmetic (operands, products and the order in which they are added) is the generic
// kernel's.
// Epilogue of a four-frame layer-4 tile: wave (wm, wn) holds frames 2 wm and 2 wm + 1 of the tile
// (rows 64 h .. 64 h + 63 of its 128, h = 0, 1) x channels 64 wn .. 64 wn + 63.  Bias + ReLU, mean
// over each frame's 64 positions, this wave's share of the FC; then per frame the sum over the
// four channel quarters, margin and decision (or the logits).  Same arithmetic, in the same
// order, as the two-frame epilogue of c4_gemm_epilogue.
__device__ inline void c4_head4_epilogue(const GcnnArgs& a, const Forward& f, const floatx4 (&acc)[4][8], int slot,
                                         int k, int64_t row0, int64_t rows, const float* ep_bias, const float* fcw_s,
                                         float (*zp)[2][kClasses]) {
  constexpr int PP = 64, WN = 64, NT = 4, WGM = 2, NWN = 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave % WGM, wn = wave / WGM;
  const int cls = l16 < kClasses ? l16 : 0;
  float zc[2] = {0.f, 0.f};                         // lane l16 < 10: class l16 of frame h
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int chb = wn * WN + nt * 16 + 4 * g;
    const floatx4 bb = *reinterpret_cast<const floatx4*>(ep_bias + chb);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float s4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int mt = 4 * h; mt < 4 * h + 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) s4[r] += fmaxf(acc[nt][mt][r] + bb[r], 0.f);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float gch = row_sum16(s4[r]) * (1.f / PP);
        zc[h] += gch * fcw_s[(chb + r) * kClasses + cls];
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float z = l16 < kClasses ? zc[h] : 0.f;
    // rows g = 0..3 hold different channel groups: add them
    z = (__shfl(z, l16) + __shfl(z, 16 + l16)) + (__shfl(z, 32 + l16) + __shfl(z, 48 + l16));
    if (lane < kClasses) zp[wave][h][lane] = z;
  }
  __syncthreads();
  if (wn == 0) {
    // lane h < 2: frame 2 wm + h of the tile
    const int h = lane & 1;
    const int64_t frow = row0 + (int64_t)(2 * wm + h) * PP;
    bool pass = false, defer = false, active = false;
    uint32_t e = 0;
    if (lane < 2 && frow < rows) {
      e = a.q.entries[(int64_t)k * a.q.cap + frow / PP];
      active = true;
      float z[kClasses];
#pragma unroll
      for (int c = 0; c < kClasses; ++c) {
        float sum = 0.f;
        for (int w2 = 0; w2 < NWN; ++w2) sum += zp[wm + WGM * w2][h][c];
        z[c] = sum + a.fc_b[slot][c];
      }
      const uint32_t idx = entry_idx(e);
      if (f.logits != nullptr)
        for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = (double)z[c];
      const float d = class_margin(z, a.class_mask[slot]);
      const float th = theta_of(f, k, idx);
      pass = d > th;
      defer = f.defer.entries != nullptr && fabsf(d - th) < f.tau[k];
    }
    if (f.logits == nullptr) forward_decision(f, k, e, active, defer, pass);
  }
}

struct C4Tile {
  int slot, k, cb, ebase;
  int64_t row0, rows;
  bool valid;
};

template <int LAYER>
__global__ __launch_bounds__(512) void c4_gemm_bf16_kernel(GcnnArgs a, Forward f) {
  constexpr int P = C4_BF16;
  typedef __bf16 T;
  typedef GemmCfg<P> G;
  typedef GemmShape<P, LAYER> S;
  constexpr int UPR = G::UPR, CE = G::CE, BKE = G::ROWB / 2;
  constexpr int CIN = S::CIN, COUT = S::COUT, HIN = S::HIN, HOUT = S::HOUT, PP = HOUT * HOUT;
  // layer 3: one frame per tile (a wave: 64 positions x 64 channels), three 48 KB stages; layer 4:
  // four frames per tile (a wave: two frames x 64 channels), two 64 KB stages, so the weight image
  // is read once per four frames
  constexpr bool HEAD = LAYER == 3;
  constexpr int BM = HEAD ? 4 * PP : S::BM, BN = S::BN, WM = HEAD ? 2 * PP : 64, WN = 64;
  constexpr int MT = WM / 16, NT = WN / 16, WGM = BM / WM;
  constexpr int NKB = 9 * CIN / BKE;
  constexpr int AUNITS = BN * UPR, UNITS = AUNITS + BM * UPR, NI = UNITS / 512, NIA = AUNITS / 512, NB = NI - NIA;
  constexpr int STAGE = UNITS * 16, NS = HEAD ? 2 : 3;
  static_assert(9 * CIN % BKE == 0 && NKB >= NS, "whole k-blocks, at least one per stage");
  static_assert(UNITS % 512 == 0 && AUNITS % 512 == 0 && WGM * (BN / WN) == 8, "tile layout");
  static_assert(!HEAD || (BN == COUT && MT == 8 && NT == 4), "layer 4: whole frames, all channels");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[NS * STAGE];
  __shared__ float zpart[8][2][kClasses];
  __shared__ __attribute__((aligned(16))) float ep_bias[BN];
  __shared__ float fcw_s[HEAD ? COUT * kClasses : 1];
  __shared__ unsigned long long ticks_s[kMaxK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave % WGM, wn = wave / WGM;
  if (tid < kMaxK) ticks_s[tid] = 0;
  const T* act_in = reinterpret_cast<const T*>(LAYER == 2 ? a.c4_act2 : a.c4_act3);
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)lds);
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i)
    if (a.c4[i]) total += (int)(((int64_t)a.q.counts[a.pred[i]] * PP + BM - 1) / BM) * (COUT / BN);
  const int u_slot = lane % UPR;

  // past the last tile: no rows (the B loads read the zero page) and the weight image of the
  // launch's first 4-layer slot (a valid image whatever the other slots hold; nothing uses them)
  int first_c4 = 0;
  for (int i = a.n_preds - 1; i >= 0; --i)
    if (a.c4[i]) first_c4 = i;
  auto decode = [&](int t) {
    C4Tile r{};
    r.slot = first_c4;
    r.valid = t < total;
    if (!r.valid) return r;
    r.slot = 0;
    int off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = a.c4[i] ? (int)(((int64_t)a.q.counts[a.pred[i]] * PP + BM - 1) / BM) * (COUT / BN) : 0;
      if (off < c) { r.slot = i; break; }
      off -= c;
      r.ebase += a.q.counts[a.pred[i]];
    }
    r.k = a.pred[r.slot];
    r.cb = off % (COUT / BN);
    r.row0 = (int64_t)(off / (COUT / BN)) * BM;
    r.rows = (int64_t)a.q.counts[r.k] * PP;
    return r;
  };
  // B rows this lane gathers for a tile, per load: the element offset of its chunk at tap (0, 0)
  // (input position (2i - 1, 2j - 1) of output (i, j)) and 3 flag bits: output row 0 (tap row 0
  // reads padding), output column 0 (tap column 0 reads padding), no row (past the queue).  A
  // stride-2 3x3 convolution with HIN = 2 HOUT reads padding nowhere else.
  struct Gather { int64_t off[NB]; uint32_t flags; };
  auto gather = [&](const C4Tile& tl, Gather& q) {
    q.flags = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int U = (wave + 8 * (NIA + i)) * 64 + lane - AUNITS;
      const int rb = U / UPR;
      const int64_t row = tl.row0 + rb;
      const bool valid = tl.valid && row < tl.rows && tl.ebase + row / PP < a.act_cap;
      const int64_t e = valid ? row / PP : 0;
      const int p = valid ? (int)(row % PP) : 0;
      const int oi = p / HOUT, oj = p % HOUT;
      q.off[i] = ((int64_t)(valid ? tl.ebase : 0) + e) * (HIN * HIN * CIN) +
                 ((int64_t)(2 * oi - 1) * HIN + (2 * oj - 1)) * CIN + (u_slot ^ c4_swz<UPR>(rb)) * CE;
      q.flags |= ((oi == 0 ? 1u : 0u) | (oj == 0 ? 2u : 0u) | (valid ? 0u : 4u)) << (3 * i);
    }
  };
  // source addresses of k-block kb of a tile: A (packed weight image, a straight copy), B (im2col:
  // k-block kb is tap kb * BKE / CIN, channels from kb * BKE % CIN)
  // (img: the tile's weight image, from tile_img)
  auto tile_img = [&](const C4Tile& tl) {
    return static_cast<const unsigned char*>(a.c4_img[tl.slot][LAYER - 2][P]) + (size_t)tl.cb * BN * G::ROWB;
  };
  auto addrs = [&](const unsigned char* img0, const Gather& q, int kb, const void* (&src)[NI]) {
    const unsigned char* img = img0 + (size_t)kb * COUT * G::ROWB;
    const int tap = kb * BKE / CIN, dy = tap / 3, dx = tap % 3;
    const int64_t toff = (int64_t)(dy * HIN + dx) * CIN + kb * BKE % CIN;
    const uint32_t bad = 4u | (dy == 0 ? 1u : 0u) | (dx == 0 ? 2u : 0u);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      if (i < NIA) {
        src[i] = img + (size_t)((wave + 8 * i) * 64 + lane) * 16;
      } else {
        const bool ok = ((q.flags >> (3 * (i - NIA))) & bad) == 0;
        src[i] = ok ? static_cast<const void*>(act_in + q.off[i - NIA] + toff) : a.zero_page;
      }
    }
  };
  auto dma = [&](const void* const (&src)[NI], int buf) {
    const uint32_t base = lds0 + buf * STAGE;
#pragma unroll
    for (int i = 0; i < NI; ++i) lds_dma16(src[i], __builtin_amdgcn_readfirstlane(base + (wave + 8 * i) * 1024));
  };
  struct Frag { bf16x8 a[NT], b[MT]; };
  // MFMA step ks (k = 32 ks .. 32 ks + 31 of the k-block) of buffer buf: lane group g reads chunk
  // 4 ks + g of each row
  auto frags = [&](int buf, int ks, Frag& F) {
    const unsigned char* A = lds + buf * STAGE;
    const unsigned char* B = A + AUNITS * 16;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int r = wn * WN + nt * 16 + l16;
      F.a[nt] = *reinterpret_cast<const bf16x8*>(A + (r * UPR + ((4 * ks + g) ^ c4_swz<UPR>(r))) * 16);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int r = wm * WM + mt * 16 + l16;
      F.b[mt] = *reinterpret_cast<const bf16x8*>(B + (r * UPR + ((4 * ks + g) ^ c4_swz<UPR>(r))) * 16);
    }
  };
  floatx4 acc[NT][MT];
  auto mma = [&](const Frag& F) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = c4_mfma(F.a[nt], F.b[mt], acc[nt][mt]);
  };

  // The compute side walks this workgroup's tiles; the issue side walks the same stream of
  // k-blocks NS k-blocks ahead (its tile changes once per tile, after a k-block's MFMAs).
  int t = blockIdx.x;
  C4Tile cur = decode(t);
  if (cur.valid) {
    int it = t, ikb = 0;
    C4Tile itl = cur;
    Gather ig;
    gather(itl, ig);
    const unsigned char* iimg = tile_img(itl);
    auto advance = [&]() {
      if (++ikb == NKB) {
        ikb = 0;
        it += gridDim.x;
        itl = decode(it);
        gather(itl, ig);
        iimg = tile_img(itl);
      }
    };
    // prologue: the stream's first NS k-blocks
#pragma unroll
    for (int s0 = 0; s0 < NS; ++s0) {
      const void* src[NI];
      addrs(iimg, ig, ikb, src);
      dma(src, s0);
      advance();
    }
    wait_vmcnt<(NS - 1) * NI>();
    __syncthreads();
    Frag F0, F1;
    frags(0, 0, F0);
    int buf = 0;                      // buffer of the current k-block
    for (;;) {
      const unsigned long long t0 = wall_clock64();
      // epilogue constants of this tile (the previous tile's closing barrier ordered every read)
      for (int i = tid; i < BN; i += 512) ep_bias[i] = a.bias[cur.slot][LAYER][cur.cb * BN + i];
      if constexpr (HEAD)
        for (int i = tid; i < COUT * kClasses; i += 512) fcw_s[i] = a.fc_w[cur.slot][i];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
      for (int kb = 0; kb < NKB; ++kb) {
        // the next k-block of the issue stream goes into this buffer once every wave has read
        // it; its addresses are formed while the MFMAs run (no branch in the loop body, so the
        // compiler can interleave them)
        const void* src[NI];
        addrs(iimg, ig, ikb, src);
        frags(buf, 1, F1);
        mma(F0);
        // publish k-block kb + 1 (issued NS - 1 k-blocks ago; the NS - 2 after it may stay in
        // flight) and free this buffer
        wait_vmcnt<(NS - 2) * NI>();
        __syncthreads();
        dma(src, buf);
        buf = buf + 1 == NS ? 0 : buf + 1;
        frags(buf, 0, F0);            // the next k-block's first step (unused after the last)
        mma(F1);
        advance();
      }
      if constexpr (HEAD)
        c4_head4_epilogue(a, f, acc, cur.slot, cur.k, cur.row0, cur.rows, ep_bias, fcw_s, zpart);
      else
        c4_gemm_epilogue<P, LAYER, true>(a, f, acc, cur.slot, cur.k, cur.cb, cur.ebase, cur.row0, cur.rows, ep_bias,
                                         nullptr, fcw_s, zpart[0]);
      if (tid == 0) ticks_s[cur.k] += wall_clock64() - t0;
      __syncthreads();                // epilogue constants and zpart are rewritten next
      t += gridDim.x;
      cur = decode(t);
      if (!cur.valid) break;
    }
    wait_vmcnt<0>();                  // the loads issued past the last tile
  }
  __syncthreads();
  if (tid < kMaxK && ticks_s[tid] && a.count_ticks) atomicAdd(&a.st->r_ticks[tid], ticks_s[tid]);
}

// ---------------------------------------------------------------- launch
template <int P, bool X3 = false>
static void launch_front(const GcnnArgs& a, int grid, hipStream_t s) {
  if (a.fr.dtype == HYDRO_DTYPE_U8) hipLaunchKernelGGL((c4_front_kernel<P, true, X3>), dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((c4_front_kernel<P, false, X3>), dim3(grid), dim3(256), 0, s, a);
}

void launch_c4_pass(const GcnnArgs& a, const Forward& f, int prec, int grid, hipStream_t s) {
  const int g1 = grid * (prec == C4_F32 || prec == C4_X3 ? 1 : 2);
  if (prec == C4_FP8) {
    launch_front<C4_FP8>(a, g1, s);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_FP8, 2>), dim3(grid), dim3(512), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_FP8, 3>), dim3(grid), dim3(512), 0, s, a, f);
  } else if (prec == C4_BF16) {
    launch_front<C4_BF16>(a, g1, s);
    hipLaunchKernelGGL((c4_gemm_bf16_kernel<2>), dim3(grid), dim3(512), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_bf16_kernel<3>), dim3(grid), dim3(512), 0, s, a, f);
  } else if (prec == C4_X3) {
    // the FP32 tier's kernels and images with the three leading products only
    launch_front<C4_F32, true>(a, g1, s);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_S3, 2, true>), dim3(grid), dim3(512), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_S3, 3, true>), dim3(grid), dim3(512), 0, s, a, f);
  } else {
    // FP32 arithmetic: the front in fp32, layers 3 and 4 as three-term bf16 products
    launch_front<C4_F32>(a, g1, s);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_S3, 2>), dim3(grid), dim3(512), 0, s, a, f);
    hipLaunchKernelGGL((c4_gemm_kernel<C4_S3, 3>), dim3(grid), dim3(512), 0, s, a, f);
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

static uint16_t c4_bf16_bits(float v) {
  uint32_t u;
  memcpy(&u, &v, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float c4_bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float v;
  memcpy(&v, &u, 4);
  return v;
}

// conv weights w: [cout][cin][3][3] canonical fp32.  Element (oc, k) of the GEMM with
// k = tap * cin + ch, tap = 3u + v.
static inline float c4_w(const float* w, int cin, int oc, int k) {
  const int tap = k / cin, ch = k % cin;
  return w[((size_t)(oc * cin + ch) * 3 + tap / 3) * 3 + tap % 3];
}

void c4_pack_front(const float* w1, float scale1, const float* w2, const float* s2, C4FrontPack* out) {
  // layer 1: k = 9u + 3v + c (27 real), K slots per c4_l1_k
  auto w1k = [&](int oc, int kk) -> float {
    if (kk >= 27) return 0.f;
    const int u = kk / 9, t = kk % 9, v = t / 3, c = t % 3;
    return scale1 * w1[((size_t)(oc * 3 + c) * 3 + u) * 3 + v];
  };
  out->w1b.assign(2 * 64 * 8, 0.f);
  for (int ct = 0; ct < 2; ++ct)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 8; ++e) out->w1b[(ct * 64 + l) * 8 + e] = w1k(ct * 16 + (l & 15), c4_l1_k(l >> 4, e));
  // FP32 arithmetic: the bf16 fragments' values split into three bf16 terms [term][ct][lane][8]
  out->w1s3.assign(3 * 2 * 64 * 8, 0);
  for (int ct = 0; ct < 2; ++ct)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 8; ++e) {
        float v = w1k(ct * 16 + (l & 15), c4_l1_k(l >> 4, e));
        for (int t = 0; t < 3; ++t) {
          const uint16_t h = c4_bf16_bits(v);
          out->w1s3[(((size_t)t * 2 + ct) * 64 + l) * 8 + e] = h;
          v -= c4_bf16_value(h);
        }
      }
  // layer 2 (cin 32), bf16 32x32x16 fragments [tap][h][c2][lane][8]: output channel
  // 32 c2 + lane % 32, input channel 16 h + 8 (lane / 32) + e
  out->w2b.assign(9 * 2 * 2 * 64 * 8, 0.f);
  for (int tp = 0; tp < 9; ++tp)
    for (int h = 0; h < 2; ++h)
      for (int c2 = 0; c2 < 2; ++c2)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e)
            out->w2b[(((tp * 2 + h) * 2 + c2) * 64 + l) * 8 + e] =
                c4_w(w2, 32, c2 * 32 + (l & 31), tp * 32 + 16 * h + 8 * (l >> 5) + e);
  // fp32 [tap][ct][lane][8]: output channel 16 ct + lane % 16, input channels 8 (lane / 16) + e
  out->w2f.assign(9 * 4 * 64 * 8, 0.f);
  for (int tp = 0; tp < 9; ++tp)
    for (int ct = 0; ct < 4; ++ct)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e)
          out->w2f[((tp * 4 + ct) * 64 + l) * 8 + e] = c4_w(w2, 32, ct * 16 + (l & 15), tp * 32 + 8 * (l >> 4) + e);
  // FP32 arithmetic from bf16 terms, [tap][ct][term][lane][8]: the fp32 fragment's eight values
  // (output channel 16 ct + lane % 16, input channels 8 (lane / 16) + e) split hi, mid, lo
  out->w2s3.assign(9 * 4 * 3 * 64 * 8, 0);
  for (int tp = 0; tp < 9; ++tp)
    for (int ct = 0; ct < 4; ++ct)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          float v = c4_w(w2, 32, ct * 16 + (l & 15), tp * 32 + 8 * (l >> 4) + e);
          for (int t = 0; t < 3; ++t) {
            const uint16_t h = c4_bf16_bits(v);
            out->w2s3[((((size_t)tp * 4 + ct) * 3 + t) * 64 + l) * 8 + e] = h;
            v -= c4_bf16_value(h);
          }
        }
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
  return (size_t)c4_nkb(prec, layer) * cout * (prec == C4_S3 ? 3 * 64 : 128);
}


// A image of a GEMM layer: [kb][oc][UPR units of 16 bytes], unit s holding chunk s ^ swz(oc);
// chunk c of k-block kb holds k = kb * BKE + c * CE + e.
void c4_pack_img(int prec, int layer, const float* w, const float* scale, unsigned char* out) {
  const int cin = layer == 2 ? 64 : 128, cout = layer == 2 ? 128 : 256;
  if (prec == C4_S3) {
    // [kb][term][oc][4 units]: unit s of a row holds chunk s ^ swz4(oc), chunk c holds
    // k = 32 kb + 8 c + e; term t of w is the bf16 rounding of w minus the earlier terms
    const int nkb = c4_nkb(prec, layer);
    for (int kb = 0; kb < nkb; ++kb)
      for (int oc = 0; oc < cout; ++oc)
        for (int s = 0; s < 4; ++s) {
          const int c = s ^ c4_swz<4>(oc);
          for (int e = 0; e < 8; ++e) {
            const int kk = kb * 32 + c * 8 + e;
            float v = kk < 9 * cin ? c4_w(w, cin, oc, kk) : 0.f;
            for (int t = 0; t < 3; ++t) {
              const uint16_t h = c4_bf16_bits(v);
              memcpy(out + ((((size_t)kb * 3 + t) * cout + oc) * 4 + s) * 16 + 2 * e, &h, 2);
              v -= c4_bf16_value(h);
            }
          }
        }
    return;
  }
  const int es = prec == C4_FP8 ? 1 : prec == C4_BF16 ? 2 : 4;
  const int rowb = 128, upr = rowb / 16, ce = 16 / es, bke = rowb / es;
  const int nkb = c4_nkb(prec, layer);
  for (int kb = 0; kb < nkb; ++kb)
    for (int row = 0; row < cout; ++row)
      for (int s = 0; s < upr; ++s) {
        // BF16 layer 3 (the third convolution): image row R holds channel c4_l3_channel(R)
        const int oc = prec == C4_BF16 && layer == 2 ? c4_l3_channel(row) : row;
        const int c = s ^ (upr == 4 ? c4_swz<4>(row) : c4_swz<8>(row));
        unsigned char* dst = out + (((size_t)kb * cout + row) * upr + s) * 16;
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
