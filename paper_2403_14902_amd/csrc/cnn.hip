// CNN predicates on gfx950: one fused kernel evaluates conv3x3/s2 x3 + ReLU, global average
// pooling, FC and the class-subset decision for a frame entirely in LDS and registers.
//
// Model (synthetic UDF): 64x64x3 frame -> conv(16m) -> conv(32m) -> conv(64m) -> mean over 8x8 ->
// FC 10, m in {1, 2, 4}; every conv has stride 2, zero padding 1 (in normalised space), ReLU.
//
// Per frame, one workgroup (8 wave64s for the widest class; 4 for the two narrower ones in the
// bf16 first pass, two workgroups per CU):
//   FR   the raw frame in LDS as bf16 (exact for bf16 and uint8 inputs): rows of 64 pixels x 3
//        channels (row stride 200 elements), with a one-pixel top/left border holding the raw
//        value that normalises to zero.
//        Layer 1 uses the folded form sW * raw + (b - 2 sum W), so no normalisation pass runs.
//   S1   one 16-channel slab of layer-1 output (all 32x32 positions);
//   ACC2 layer-2 accumulators for all 16x16 positions and all 32m channels stay in registers while
//        the m slabs of layer 1 stream through S1 (layer 2's K loop runs slab by slab), so
//        layer 1's full output never needs to fit in LDS and every layer-2 weight is read once
//        per frame;
//   L2   layer-2 output (bias + ReLU) written over FR/S1 once all slabs are consumed;
//   ACC3 layer-3 accumulators (64 positions x 64m channels) in registers; their ReLU is summed
//        straight into the pooled vector, then FC, margin and decision.
// Convolutions are implicit GEMMs on MFMA: M = output positions, N = output channels,
// K = (tap, input channel).  Weights are pre-packed in MFMA-fragment order so each lane reads
// one contiguous run per fragment.
#include "engine.h"

namespace hydro {

template <typename T> struct Mf;
template <> struct Mf<__bf16> {
  static constexpr int KSTEP = 32, KPL = 8;
  typedef bf16x8 frag;
};
template <> struct Mf<float> {
  static constexpr int KSTEP = 4, KPL = 1;
  typedef float frag;
};

__device__ inline floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ inline typename Mf<T>::frag ld_frag(const T* p) {
  if constexpr (sizeof(T) == 2) return *reinterpret_cast<const bf16x8*>(p);
  else return *p;
}

// FP32 arithmetic from bf16 MFMAs: fp32 activations split into three bf16 terms (x = h + m + l
// exactly), weights held as three terms likewise; the six products down to 2^-24 relative, summed
// smallest first.
__device__ inline void split3(const float4& p0, const float4& p1, bf16x8 (&x)[3]) {
  const float xv[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = static_cast<__bf16>(xv[e]);
    const float r1 = xv[e] - static_cast<float>(h);
    const __bf16 m = static_cast<__bf16>(r1);
    x[0][e] = h;
    x[1][e] = m;
    x[2][e] = static_cast<__bf16>(r1 - static_cast<float>(m));
  }
}
__device__ inline floatx4 mfma_s3(const bf16x8 (&w)[3], const bf16x8 (&x)[3], floatx4 c) {
  c = mfma(w[0], x[2], c);
  c = mfma(w[1], x[1], c);
  c = mfma(w[0], x[1], c);
  c = mfma(w[2], x[0], c);
  c = mfma(w[1], x[0], c);
  return mfma(w[0], x[0], c);
}

// geometry
constexpr int H0 = 64, H1 = 32, H2 = 16, H3 = 8;
constexpr int NTHR = 512;           // 8 wave64s per workgroup (the narrowest class: 4, two per CU)
constexpr int FRS = 200;            // FR row stride (bf16 elements): 5 unused, border pixel, 64 pixels
constexpr int FR_X0 = 8;            // element offset of pixel 0 in an FR row (16-byte aligned)
constexpr int S1_W = H1 + 1;        // layer-1 slab row stride in pixels (top/left border)
constexpr int L2_W = H2 + 1;
constexpr int CB1 = 16;             // layer-1 channels per slab

// Pixel strides (elements) of the layer-1 slab and the layer-2 output are padded so that the 16
// lanes of an MFMA row group, which read 16 different pixels, spread over the LDS banks.
template <typename T> struct Pad {
  static constexpr int S1P = CB1 + (sizeof(T) == 4 ? 4 : 0);   // fp32: 16-byte aligned pixels
  static constexpr int L2E = 16 / (int)sizeof(T);      // extra elements per layer-2 pixel
};

template <typename T, int MMAX = 4> struct CnnLds {
  static constexpr int FR_BYTES = (H0 + 1) * FRS * 2;
  static constexpr int S1_OFF = (FR_BYTES + 15) / 16 * 16;
  static constexpr int S1_BYTES = S1_W * S1_W * Pad<T>::S1P * (int)sizeof(T);
  static constexpr int L2_BYTES_MAX = L2_W * L2_W * (32 * MMAX + Pad<T>::L2E) * (int)sizeof(T);
  static constexpr int REGION = (S1_OFF + S1_BYTES) > L2_BYTES_MAX ? (S1_OFF + S1_BYTES) : L2_BYTES_MAX;
};

constexpr int DBUF = 64;
// First pass, the two narrower classes: workgroups of four waves (with the LDS of their own
// width), two per CU, so one frame's barriers and per-frame work overlap another frame's MFMAs.

// packed-layer geometry: [slab][kstep][ntile][64][KPL]
// layer 1: K = 27 in (row u, column v, channel c) order, k = 9u + 3v + c, padded to KSTEP
template <typename T>
__host__ __device__ constexpr int cnn_ksteps(int layer, int m) {
  return layer == 0 ? (27 + Mf<T>::KSTEP - 1) / Mf<T>::KSTEP
       : layer == 1 ? (9 * CB1 + Mf<T>::KSTEP - 1) / Mf<T>::KSTEP
                    : 9 * 32 * m / Mf<T>::KSTEP;
}
__host__ __device__ constexpr int cnn_slabs(int layer, int m) { return layer == 2 ? 1 : m; }
__host__ __device__ constexpr int cnn_ntiles(int layer, int m) { return layer == 0 ? 1 : layer == 1 ? 2 * m : 4 * m; }

// Per-slot constants staged in LDS when a workgroup's slot changes: biases of the three layers
// (offsets 0, 64, 192) and, in the bf16 kernels, the FC weights and bias.
constexpr int CB_L2 = 64, CB_L3 = 192, CB_N = 448;
constexpr int FCW_MAX = 256 * kClasses;

struct CnnShared {
  float cb[CB_N];
  float fcb[kClasses];
  float gpart[2][256];
  float z[kClasses];
  uint32_t d_e[DBUF];
  uint8_t d_k[DBUF];
  uint8_t d_f[DBUF];
  int d_n;
  unsigned long long ticks[kMaxK];
  __attribute__((aligned(16))) __bf16 feat[192];   // router features of the current frame
};

__device__ void flush_decisions(const Forward& f, CnnShared& sh, int n_slots, const int* pred) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int n = sh.d_n;
    bool active = lane < n;
    uint32_t e = active ? sh.d_e[lane] : 0u;
    int k = active ? (int)sh.d_k[lane] : -1;
    uint8_t fl = active ? sh.d_f[lane] : 0;
    for (int i = 0; i < n_slots; ++i) {
      int kk = pred[i];
      if (__ballot(active && k == kk) == 0) continue;
      forward_decision(f, kk, e, active && k == kk, (fl & 2) != 0, (fl & 1) != 0);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sh.d_n = 0;
  __syncthreads();
}

// Raw frame bytes held in registers between the issue of their loads and their LDS store
// (the next frame is fetched while the current one is in layer 3).
template <int NT>
struct FramePrefetch {
  uint4 v[1536 / NT];
};

// bf16 frames: 1536 chunks of 8 elements; uint8 frames: 768 chunks of 16 elements.  One
// unconditional load sequence serves both (uint8 chunk indices past the frame are clamped to its
// last chunk and the values ignored), so the loads are never skipped and no register is the
// target of two alternative loads: the compiler can count outstanding loads exactly.
template <int NT>
__device__ inline void frame_issue(const CnnArgs& a, uint32_t idx, FramePrefetch<NT>& pf) {
  const int tid = threadIdx.x;
  const bool bf = a.fr.dtype == HYDRO_DTYPE_BF16;
  const int last = bf ? 1535 : 767;
  const uint4* src = reinterpret_cast<const uint4*>(static_cast<const unsigned char*>(a.fr.base) +
                                                    (int64_t)idx * a.fr.elems * (bf ? 2 : 1));
#pragma unroll
  for (int r = 0; r < 1536 / NT; ++r) pf.v[r] = src[min(tid + r * NT, last)];
}

// The loaded registers pass through an empty asm statement at the point of use, so no
// computation on them (the uint8 unpacking, which the compiler otherwise evaluates speculatively
// for every frame type) can be scheduled next to the loads: the wave does not wait for the frame
// until it stores it.
__device__ inline uint4 frame_regs_ready(uint4 v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
  return v;
}

// Store a prefetched frame into FR and (re)write the borders of FR and the layer-1 slab.
template <typename T, int NT>
__device__ inline void frame_store(const CnnArgs& a, const FramePrefetch<NT>& pf, unsigned char* region) {
  const int tid = threadIdx.x;
  __bf16* FR = reinterpret_cast<__bf16*>(region);
  if (a.fr.dtype == HYDRO_DTYPE_BF16) {
#pragma unroll
    for (int r = 0; r < 1536 / NT; ++r) {
      const int q = tid + r * NT, y = q / 24, c = q % 24;
      *reinterpret_cast<uint4*>(FR + (y + 1) * FRS + FR_X0 + c * 8) = frame_regs_ready(pf.v[r]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < (768 + NT - 1) / NT; ++r) {
      const int q = tid + r * NT;
      if (q < 768) {
        const int y = q / 12, c = q % 12;
        const uint4 raw = frame_regs_ready(pf.v[r]);
        const uint8_t* b = reinterpret_cast<const uint8_t*>(&raw);
        alignas(16) __bf16 o[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) o[j] = static_cast<__bf16>((float)b[j]);
        uint4* d = reinterpret_cast<uint4*>(FR + (y + 1) * FRS + FR_X0 + c * 16);
        d[0] = reinterpret_cast<const uint4*>(o)[0];
        d[1] = reinterpret_cast<const uint4*>(o)[1];
      }
    }
  }
  const __bf16 padv = static_cast<__bf16>(a.pad_raw);
  for (int e = tid; e < FRS; e += NT) FR[e] = padv;                                // top border row
  for (int e = tid; e < H0 * 3; e += NT) FR[(e / 3 + 1) * FRS + FR_X0 - 3 + e % 3] = padv;  // left border
  T* S1 = reinterpret_cast<T*>(region + CnnLds<T>::S1_OFF);
  for (int p = tid; p < (2 * S1_W - 1) * CB1; p += NT) {
    const int q = p / CB1, c = p % CB1;
    const int y = q < S1_W ? 0 : q - S1_W + 1, x = q < S1_W ? q : 0;
    S1[(y * S1_W + x) * Pad<T>::S1P + c] = static_cast<T>(0.f);
  }
}

// 4 consecutive channels of one position, stored with one LDS write.
template <typename T>
__device__ inline void store4(T* dst, float v0, float v1, float v2, float v3) {
  if constexpr (sizeof(T) == 2) {
    alignas(8) __bf16 h[4] = {static_cast<__bf16>(v0), static_cast<__bf16>(v1), static_cast<__bf16>(v2),
                              static_cast<__bf16>(v3)};
    *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(h);
  } else {
    *reinterpret_cast<float4*>(dst) = make_float4(v0, v1, v2, v3);
  }
}

// One frame through the network (FR already holds it).  The MFMAs compute the transposed
// products (rows = output channels from the packed weights, columns = positions from LDS), so
// each lane ends with 4 consecutive channels of one position.  Wave 0 finishes with FC, margin
// and the decision record; if next_valid, the next frame is stored into FR meanwhile.  Returns
// the logits in z (wave 0, lane 0 holds all 10).
// Router features of the frame in FR: the 8x8-pixel cell means per channel (8 x 8 cells x 3),
// normalised as the predicates normalise their input.  Each (cell, row) segment is 8 pixels x 3
// channels = 24 contiguous elements (three aligned 16-byte reads); lanes 8m..8m+7 hold the eight
// rows of one cell and add them with three DPP steps.  Pass it (0 .. 512/NT - 1) covers segments
// tid + it * NT; lanes with row 0 hold their cell's three values.
template <int NT>
struct FrameFeat {
  float v[512 / NT][3];
};
template <int NT>
__device__ inline void frame_features(const __bf16* FR, float scale, FrameFeat<NT>& ff) {
#pragma unroll
  for (int it = 0; it < 512 / NT; ++it) {
    const int sg = threadIdx.x + it * NT;
    const int cell = sg >> 3, r = sg & 7, by = cell >> 3, bx = cell & 7;
    const uint4* p = reinterpret_cast<const uint4*>(FR + (8 * by + r + 1) * FRS + FR_X0 + 24 * bx);
    float c3[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint4 u = p[q];
      const __bf16* h = reinterpret_cast<const __bf16*>(&u);
#pragma unroll
      for (int e = 0; e < 8; ++e) c3[(8 * q + e) % 3] += (float)h[e];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      c3[c] += dpp_mov<0xB1>(c3[c]);    // quad_perm [1,0,3,2]
      c3[c] += dpp_mov<0x4E>(c3[c]);    // quad_perm [2,3,0,1]
      c3[c] += dpp_mov<0x141>(c3[c]);   // row_half_mirror: the other quad of the 8 lanes
      ff.v[it][c] = (c3[c] * scale - 0.5f) * 4.0f;
    }
  }
}
// Each thread with row 0 writes its cells' values (to HBM, or to sh.feat).
template <int NT>
__device__ inline void frame_features_put(const FrameFeat<NT>& ff, __bf16* dst) {
#pragma unroll
  for (int it = 0; it < 512 / NT; ++it) {
    const int sg = threadIdx.x + it * NT;
    if ((sg & 7) == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) dst[(sg >> 3) * 3 + c] = static_cast<__bf16>(ff.v[it][c]);
    }
  }
}

template <typename T, int M, int NWV>
__device__ void cnn_frame(const CnnArgs& a, int slot, unsigned char* region, CnnShared& sh, const float* fcw,
                          bool next_valid, uint32_t next_idx, __bf16* feat_dst, float* z_out) {
  constexpr int NT = NWV * 64;                       // threads
  constexpr int C2 = 32 * M, C3 = 64 * M;
  constexpr int S1P = Pad<T>::S1P, C2P = C2 + Pad<T>::L2E;
  // FP32 tier (T = float): fp32 activations, bf16 MFMAs on three-term operands, in the bf16
  // fragment layout (k-steps of 32, 8 per lane)
  constexpr bool S3 = sizeof(T) == 4;
  typedef typename std::conditional<S3, __bf16, T>::type KT;
  constexpr int KSTEP = Mf<KT>::KSTEP, KPL = Mf<KT>::KPL;
  typedef typename Mf<T>::frag frag;
  // term t of the FP32 tier's packed layer l: fragments [slab][k-step][n-tile][lane]
  auto s3w = [&](int l, int t) {
    const size_t per_term = (size_t)cnn_slabs(l, M) * cnn_ksteps<__bf16>(l, M) * cnn_ntiles(l, M) * 64;
    return reinterpret_cast<const bf16x8*>(a.w_s3[slot][l]) + t * per_term;
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;

  const __bf16* FR = reinterpret_cast<const __bf16*>(region);
  T* S1 = reinterpret_cast<T*>(region + CnnLds<T>::S1_OFF);
  T* L2 = reinterpret_cast<T*>(region);

  const T* const* wpk = reinterpret_cast<const T* const*>(a.w_bf[slot]);   // (bf16 tier)
  const float* b1 = sh.cb;
  const float* b2 = sh.cb + CB_L2;
  const float* b3 = sh.cb + CB_L3;
  // The narrow classes fetch the next frame now: their layer 3 is too short to cover the HBM
  // latency before the frame is stored (not the four-wave m = 2 form: no registers to spare).
  constexpr bool kEarlyFetch = M == 1 || (M == 2 && NWV == 8);
  constexpr int KS1 = cnn_ksteps<KT>(0, M), KS2 = cnn_ksteps<KT>(1, M);
  constexpr int NT2 = 2 * M;
  // layer-2 wave tile: MT2 position tiles x NW2 channel tiles (the waves cover 16 x NT2)
  constexpr int MT2 = (M == 1 && NWV == 8) ? 2 : (M == 4 && sizeof(T) == 2) ? 8 : 4, NW2 = NT2 * (16 / MT2) / NWV;
  constexpr int NG2 = NT2 / NW2;                       // channel groups
  // weight prefetch depth (k-steps); the widest bf16 class has no registers to spare in layer 2
  constexpr int PD2 = S3 ? 1 : ((M == 4 || (M == 2 && NWV == 4)) ? 2 : 3);
  const int mg2 = wave / NG2, ng2 = wave % NG2;
  static_assert((16 / MT2) * NG2 == NWV, "layer-2 wave tiling must cover the waves");
  // With the early fetch, slab 0's layer-1 weights and its first PD2 layer-2 weight k-steps are
  // requested before the frame: a wave's vector loads complete in issue order, so a weight load
  // issued after the frame's would wait for the frame's HBM latency.  (Not in the FP32 kernel:
  // it has no registers to spare.)
  constexpr bool kPreW = kEarlyFetch && sizeof(T) == 2;
  frag w1_0[kPreW ? KS1 : 1];
  frag bw2_0[kPreW ? PD2 : 1][NW2];
  if constexpr (kPreW) {
    const frag* w1p0 = reinterpret_cast<const frag*>(wpk[0]);
#pragma unroll
    for (int ks = 0; ks < KS1; ++ks) w1_0[ks] = w1p0[ks * 64 + lane];
    const frag* w2p0 = reinterpret_cast<const frag*>(wpk[1]) + ng2 * NW2 * 64 + lane;
#pragma unroll
    for (int d = 0; d < PD2; ++d)
#pragma unroll
      for (int n = 0; n < NW2; ++n)
        if (d < KS2) bw2_0[d][n] = w2p0[(d * NT2 + n) * 64];
  }
  // First evaluation of a tuple in the first pass: its router features, from the frame in LDS.
  // Early fetch: computed now and stored by every wave right after the frame loads are issued
  // (everything waited on later already waits for those loads, which complete in issue order).
  // Late fetch: staged in LDS at slab 0 and stored by wave 0 after the late frame issue.
  const float fscale = (a.fr.dtype == HYDRO_DTYPE_U8 ? 1.0f / 255.0f : 1.0f) * (1.0f / 64.0f);
  FrameFeat<NT> ff;
  if (kEarlyFetch && feat_dst != nullptr) frame_features<NT>(FR, fscale, ff);
  // The frame loads are issued whether or not a next frame exists (next_idx is then the current
  // frame and nothing is stored): a conditional issue would leave the compiler unsure how many
  // loads are outstanding, and every later weight wait would then also wait for the frame.
  FramePrefetch<NT> pf;
  if (kEarlyFetch) frame_issue<NT>(a, next_idx, pf);
  if (kEarlyFetch && feat_dst != nullptr) frame_features_put<NT>(ff, feat_dst);

  // ---- layer-1 im2col fragments of this wave's MPW m-tiles (cached when several slabs reuse them)
  constexpr int MPW = 64 / NWV;                      // layer-1 m-tiles per wave
  constexpr bool kCacheA1 = sizeof(T) == 2 && M > 1 && NWV == 8;
  frag a1[kCacheA1 ? MPW : 1][KS1];
  auto gather1b = [&](int mt) -> bf16x8 {
    const int px = mt * 16 + l16, i = px >> 5, j = px & 31;
    const __bf16* rowp = FR + 2 * i * FRS + 5 + 6 * j;
    alignas(16) __bf16 t8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = min(8 * g + e, 26);
      t8[e] = rowp[(k / 9) * FRS + k % 9];
    }
    return *reinterpret_cast<const bf16x8*>(t8);
  };
  auto gather1 = [&](int mt, int ks) -> frag {
    const int px = mt * 16 + l16, i = px >> 5, j = px & 31;
    // im2col row of output (i, j): FR row 2i+u, elements 5 + 6j + (3v + c), k = 9u + 3v + c
    const __bf16* rowp = FR + 2 * i * FRS + 5 + 6 * j;
    // padded k (27..31, zero weights) reads element 26, a finite value: the reads need no
    // per-lane predication, so the tiles' reads can be scheduled ahead of the MFMAs
    if constexpr (sizeof(T) == 2) {
      alignas(16) __bf16 t8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = min(ks * 32 + 8 * g + e, 26);
        t8[e] = rowp[(k / 9) * FRS + k % 9];
      }
      return *reinterpret_cast<const bf16x8*>(t8);
    } else {
      const int k = min(ks * 4 + g, 26);
      return (float)rowp[(k / 9) * FRS + k % 9];
    }
  };
  if constexpr (kCacheA1) {
#pragma unroll
    for (int q = 0; q < MPW; ++q)
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) a1[q][ks] = gather1(wave * MPW + q, ks);
  }

  floatx4 acc2[MT2][NW2];
#pragma unroll
  for (int q = 0; q < MT2; ++q)
#pragma unroll
    for (int j = 0; j < NW2; ++j) acc2[q][j] = (floatx4){0.f, 0.f, 0.f, 0.f};

  for (int slab = 0; slab < M; ++slab) {
    // layer 1: 64 m-tiles (16 positions each) x 16 channels; wave w owns m-tiles 8w..8w+7
    const frag* w1p = reinterpret_cast<const frag*>(wpk[0]) + (size_t)slab * KS1 * 64;
    frag w1f[S3 ? 1 : KS1];
    bf16x8 w1t[3];
    if constexpr (S3) {
#pragma unroll
      for (int t = 0; t < 3; ++t) w1t[t] = s3w(0, t)[slab * 64 + lane];
    } else if (kPreW && slab == 0) {
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) w1f[ks] = w1_0[ks];
    } else {
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) w1f[ks] = w1p[ks * 64 + lane];
    }
    (void)w1t;
    float bb1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bb1[r] = b1[slab * CB1 + 4 * g + r];
    if (!kEarlyFetch && slab == 0 && feat_dst != nullptr) {
      frame_features<NT>(FR, fscale, ff);
      frame_features_put<NT>(ff, sh.feat);
    }
    auto l1_store = [&](int mt, const floatx4& acc) {
      const int px = mt * 16 + l16, i = px >> 5, j = px & 31;
      store4<T>(S1 + ((i + 1) * S1_W + (j + 1)) * S1P + 4 * g, fmaxf(acc[0] + bb1[0], 0.f),
                fmaxf(acc[1] + bb1[1], 0.f), fmaxf(acc[2] + bb1[2], 0.f), fmaxf(acc[3] + bb1[3], 0.f));
    };
    if constexpr (sizeof(T) == 2 && !kCacheA1 && KS1 == 1) {
      // tiles in pairs: both gathers, both MFMAs, then both epilogues, so one tile's LDS and
      // MFMA latencies overlap the other's
      const floatx4 zero = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int q = 0; q < MPW; q += 2) {
        const int mt = wave * MPW + q;
        const frag av0 = gather1(mt, 0), av1 = gather1(mt + 1, 0);
        const floatx4 acc0 = mfma(w1f[0], av0, zero), acc1 = mfma(w1f[0], av1, zero);
        l1_store(mt, acc0);
        l1_store(mt + 1, acc1);
      }
    } else if constexpr (S3) {
      // FP32 tier: the raw frame values are exact in bf16, so the three weight terms give every
      // product exactly (smallest term first); tiles in pairs
#pragma unroll 2
      for (int q = 0; q < MPW; q += 2) {
        const int mt = wave * MPW + q;
        const bf16x8 av0 = gather1b(mt), av1 = gather1b(mt + 1);
        floatx4 acc0 = (floatx4){0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
        for (int t = 2; t >= 0; --t) {
          acc0 = mfma(w1t[t], av0, acc0);
          acc1 = mfma(w1t[t], av1, acc1);
        }
        l1_store(mt, acc0);
        l1_store(mt + 1, acc1);
      }
    } else {
#pragma unroll 8
      for (int q = 0; q < MPW; ++q) {
        const int mt = wave * MPW + q;
        floatx4 acc = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) {
          frag av;
          if constexpr (kCacheA1) av = a1[q][ks];
          else av = gather1(mt, ks);
          acc = mfma(w1f[ks], av, acc);
        }
        l1_store(mt, acc);
      }
    }
    __syncthreads();
    if constexpr (S3) {
      // FP32 tier, layer 2 partial of this slab: K = 9 taps x 16 channels in k-steps of 32 (lane
      // group g: tap (32 ks + 8 g) / 16, channels from 8 (g % 2)); a k-step's weights are
      // requested before its activation reads and splits
      const bf16x8* w2t[3] = {s3w(1, 0), s3w(1, 1), s3w(1, 2)};
#pragma unroll 1
      for (int ks = 0; ks < KS2; ++ks) {
        bf16x8 w[NW2][3];
#pragma unroll
        for (int n = 0; n < NW2; ++n)
#pragma unroll
          for (int t = 0; t < 3; ++t) w[n][t] = w2t[t][((slab * KS2 + ks) * NT2 + ng2 * NW2 + n) * 64 + lane];
        const int k0 = ks * 32 + 8 * g;
        const int tp = min(k0 / CB1, 8);        // padded k (zero weights) reads a valid tap
        const int c0 = k0 % CB1;
        const int u = tp / 3, v = tp % 3;
#pragma unroll
        for (int q = 0; q < MT2; ++q) {
          const int px = (mg2 * MT2 + q) * 16 + l16, i = px >> 4, j = px & 15;
          const float4* src = reinterpret_cast<const float4*>(S1 + ((2 * i + u) * S1_W + 2 * j + v) * S1P + c0);
          bf16x8 x[3];
          split3(src[0], src[1], x);
#pragma unroll
          for (int n = 0; n < NW2; ++n) acc2[q][n] = mfma_s3(w[n], x, acc2[q][n]);
          __builtin_amdgcn_sched_barrier(0);    // one position tile's operands live at a time
        }
      }
    } else {
      // layer 2 partial: K = 9 taps x 16 channels of this slab.  The weight fragments run PD2
      // k-steps ahead of the MFMAs (they come from L2 cache; one k-step of MFMAs is far shorter
      // than that latency).
      const frag* w2p = reinterpret_cast<const frag*>(wpk[1]) + (size_t)slab * KS2 * NT2 * 64 + ng2 * NW2 * 64 + lane;
      frag bw2[PD2][NW2];
      if (kPreW && slab == 0) {
  #pragma unroll
        for (int d = 0; d < PD2; ++d)
  #pragma unroll
          for (int n = 0; n < NW2; ++n)
            if (d < KS2) bw2[d][n] = bw2_0[d][n];
      } else {
  #pragma unroll
        for (int d = 0; d < PD2; ++d)
  #pragma unroll
          for (int n = 0; n < NW2; ++n)
            if (d < KS2) bw2[d][n] = w2p[(d * NT2 + n) * 64];
      }
  #pragma unroll (kPreW && M == 1 ? 4 : 1)
      for (int ks0 = 0; ks0 < KS2; ks0 += PD2) {
  #pragma unroll
        for (int d = 0; d < PD2; ++d) {
          const int ks = ks0 + d;
          // (when PD2 divides KS2 the guard folds away and the loop body has no branches)
          if (KS2 % PD2 == 0 || ks < KS2) {
            const int k0 = ks * KSTEP + KPL * g;
            int t = k0 / CB1;
            const int c0 = k0 % CB1;
            if (t > 8) t = 8;                       // padded k (zero weights) reads a valid tap
            const int u = t / 3, v = t % 3;
            frag av[MT2];
  #pragma unroll
            for (int q = 0; q < MT2; ++q) {
              const int px = (mg2 * MT2 + q) * 16 + l16, i = px >> 4, j = px & 15;
              av[q] = ld_frag<T>(S1 + ((2 * i + u) * S1_W + 2 * j + v) * S1P + c0);
            }
  #pragma unroll
            for (int n = 0; n < NW2; ++n)
  #pragma unroll
              for (int q = 0; q < MT2; ++q) acc2[q][n] = mfma(bw2[d][n], av[q], acc2[q][n]);
            if constexpr (KS2 % PD2 == 0) {
              // unconditional refill; the last PD2 k-steps re-read the last fragment (unused).  The
              // scheduling barrier keeps the loads here: sunk to the end of the iteration (to
              // shorten register lifetimes) they would be waited on right after being issued.
  #pragma unroll
              for (int n = 0; n < NW2; ++n) bw2[d][n] = w2p[(min(ks + PD2, KS2 - 1) * NT2 + n) * 64];
              __builtin_amdgcn_sched_barrier(0);
            } else if (ks + PD2 < KS2) {
  #pragma unroll
              for (int n = 0; n < NW2; ++n) bw2[d][n] = w2p[((ks + PD2) * NT2 + n) * 64];
            }
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- layer-2 epilogue into L2 (overwrites FR / S1)
#pragma unroll
  for (int n = 0; n < NW2; ++n) {
    const int ch = (ng2 * NW2 + n) * 16 + 4 * g;
    const float bb0 = b2[ch], bb1v = b2[ch + 1], bb2 = b2[ch + 2], bb3 = b2[ch + 3];
#pragma unroll
    for (int q = 0; q < MT2; ++q) {
      const int px = (mg2 * MT2 + q) * 16 + l16, i = px >> 4, j = px & 15;
      store4<T>(L2 + ((i + 1) * L2_W + (j + 1)) * C2P + ch, fmaxf(acc2[q][n][0] + bb0, 0.f),
                fmaxf(acc2[q][n][1] + bb1v, 0.f), fmaxf(acc2[q][n][2] + bb2, 0.f), fmaxf(acc2[q][n][3] + bb3, 0.f));
    }
  }
  for (int p = tid; p < (2 * L2_W - 1) * (C2 / 4); p += NT) {
    const int qq = p / (C2 / 4), c = (p % (C2 / 4)) * 4;
    const int y = qq < L2_W ? 0 : qq - L2_W + 1, x = qq < L2_W ? qq : 0;
    store4<T>(L2 + (y * L2_W + x) * C2P + c, 0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();

  // ---- layer 3: 4 position tiles (64 positions) x 4M channel tiles; wave tile MT3 x NW3
  constexpr int KS3 = cnn_ksteps<KT>(2, M), NT3 = 4 * M;
  constexpr int MT3 = (M == 1 && NWV == 8) ? 2 : 4, NW3 = NT3 * (4 / MT3) / NWV;
  constexpr int MG3 = 4 / MT3;                         // position groups (1 or 2)
  constexpr int PD3 = S3 ? 1 : ((M == 2 && NWV == 4) ? 2 : 3);
  static_assert(MG3 * (NT3 / NW3) == NWV, "layer-3 wave tiling must cover the waves");
  const int mh = wave % MG3, ng = wave / MG3;
  floatx4 acc3[MT3][NW3];
#pragma unroll
  for (int q = 0; q < MT3; ++q)
#pragma unroll
    for (int j = 0; j < NW3; ++j) acc3[q][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
  const frag* w3p = reinterpret_cast<const frag*>(wpk[2]) + (size_t)(ng * NW3) * 64 + lane;
  static_assert(KS3 % PD3 == 0, "layer-3 k-steps must be a multiple of the prefetch depth");
  frag bw3[PD3][NW3];
  if constexpr (!S3) {
#pragma unroll
    for (int d = 0; d < PD3; ++d)
#pragma unroll
      for (int n = 0; n < NW3; ++n) bw3[d][n] = w3p[(d * NT3 + n) * 64];
  }
  auto l3_step = [&](int ks, const frag (&b)[NW3]) {
    const int k0 = ks * KSTEP + KPL * g;
    const int t = k0 / C2, c0 = k0 % C2;
    const int u = t / 3, v = t % 3;
    frag av[MT3];
#pragma unroll
    for (int q = 0; q < MT3; ++q) {
      const int px = (mh * MT3 + q) * 16 + l16, i = px >> 3, j = px & 7;
      av[q] = ld_frag<T>(L2 + ((2 * i + u) * L2_W + 2 * j + v) * C2P + c0);
    }
#pragma unroll
    for (int n = 0; n < NW3; ++n)
#pragma unroll
      for (int q = 0; q < MT3; ++q) acc3[q][n] = mfma(b[n], av[q], acc3[q][n]);
  };
  if constexpr (sizeof(T) == 2) {
    // every k-step but the last PD3 refills its buffer PD3 k-steps ahead
#pragma unroll 1
    for (int ks0 = 0; ks0 < KS3 - PD3; ks0 += PD3) {
#pragma unroll
      for (int d = 0; d < PD3; ++d) {
        const int ks = ks0 + d;
        l3_step(ks, bw3[d]);
#pragma unroll
        for (int n = 0; n < NW3; ++n) bw3[d][n] = w3p[((ks + PD3) * NT3 + n) * 64];
      }
    }
    // The late fetch goes after the last weight request: loads complete in issue order, so any
    // weight requested after the frame would wait for it.
    if (!kEarlyFetch) frame_issue<NT>(a, next_idx, pf);
    if (!kEarlyFetch && feat_dst != nullptr && wave == 0 && lane < 24)
      reinterpret_cast<uint4*>(feat_dst)[lane] = reinterpret_cast<const uint4*>(sh.feat)[lane];
#pragma unroll
    for (int d = 0; d < PD3; ++d) l3_step(KS3 - PD3 + d, bw3[d]);
  } else {
    // FP32 tier: the frame is requested before layer 3 (its wait falls on the first k-step only);
    // per k-step the weight terms are requested before the activation reads and splits
    if (!kEarlyFetch) frame_issue<NT>(a, next_idx, pf);
    if (!kEarlyFetch && feat_dst != nullptr && wave == 0 && lane < 24)
      reinterpret_cast<uint4*>(feat_dst)[lane] = reinterpret_cast<const uint4*>(sh.feat)[lane];
    (void)bw3;
    const bf16x8* w3t[3] = {s3w(2, 0), s3w(2, 1), s3w(2, 2)};
#pragma unroll 1
    for (int ks = 0; ks < KS3; ++ks) {
      bf16x8 w[NW3][3];
#pragma unroll
      for (int n = 0; n < NW3; ++n)
#pragma unroll
        for (int t = 0; t < 3; ++t) w[n][t] = w3t[t][(ks * NT3 + ng * NW3 + n) * 64 + lane];
      const int k0 = ks * 32 + 8 * g;
      const int tp = k0 / C2, c0 = k0 % C2;
      const int u = tp / 3, v = tp % 3;
#pragma unroll
      for (int q = 0; q < MT3; ++q) {
        const int px = (mh * MT3 + q) * 16 + l16, i = px >> 3, j = px & 7;
        const float4* src = reinterpret_cast<const float4*>(L2 + ((2 * i + u) * L2_W + 2 * j + v) * C2P + c0);
        bf16x8 x[3];
        split3(src[0], src[1], x);
#pragma unroll
        for (int n = 0; n < NW3; ++n) acc3[q][n] = mfma_s3(w[n], x, acc3[q][n]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // ReLU + pooled partial sums over this wave's positions
#pragma unroll
  for (int n = 0; n < NW3; ++n) {
    const int ch0 = (ng * NW3 + n) * 16 + 4 * g;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float bb = b3[ch0 + r];
      float s = 0.f;
#pragma unroll
      for (int q = 0; q < MT3; ++q) s += fmaxf(acc3[q][n][r] + bb, 0.f);
      s = row_sum16(s);
      if (l16 == 0) sh.gpart[mh][ch0 + r] = s;
    }
  }
  if (MG3 == 1) {
    for (int c = tid; c < C3; c += NT) sh.gpart[1][c] = 0.f;
  }
  __syncthreads();
  // wave 0: FC (lanes over channels) -> z; the other waves store the next frame meanwhile
  if (wave == 0) {
    const float* fw = fcw;
    float zp[kClasses];
#pragma unroll
    for (int c = 0; c < kClasses; ++c) zp[c] = 0.f;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int ch = lane + 64 * q;
      const float gch = (sh.gpart[0][ch] + sh.gpart[1][ch]) * (1.0f / 64.0f);
#pragma unroll
      for (int c = 0; c < kClasses; ++c) zp[c] += gch * fw[ch * kClasses + c];
    }
    wave_sum_n(zp);
#pragma unroll
    for (int c = 0; c < kClasses; ++c) z_out[c] = zp[c] + sh.fcb[c];
  }
  if (next_valid) frame_store<T, NT>(a, pf, region);
}

// Persistent over every queue of the launch: entry t of the concatenated queues goes to workgroup
// t mod grid; slots are ordered by cost, so the widest frames come first.  VSET is the set of width
// classes the instantiation holds code for (bit m for width multiplier m); one register
// allocation covers them all, so classes whose union would spill get launches of their own.
template <typename T, int VSET, int NWV = 8>
__global__ __launch_bounds__(NWV * 64) __attribute__((amdgpu_waves_per_eu(NWV == 4 ? 2 : 1)))
void cnn_fused_kernel(CnnArgs a, Forward f) {
  constexpr int NT = NWV * 64;
  constexpr int MMAX = (VSET & 4) ? 4 : (VSET & 2) ? 2 : 1;   // widest class of the launch
  __shared__ __attribute__((aligned(16))) unsigned char region[CnnLds<T, MMAX>::REGION];
  __shared__ CnnShared sh;
  // FC weights of the current slot (bf16 kernels; the FP32 kernel has no LDS left and reads them
  // from global memory)
  __shared__ float fcw_s[sizeof(T) == 2 ? 64 * MMAX * kClasses : 1];
  const int tid = threadIdx.x;
  if (tid == 0) sh.d_n = 0;
  if (tid < kMaxK) sh.ticks[tid] = 0;
  // queue prefix offsets, kept in LDS (read when entries are staged)
  __shared__ int cum_s[kMaxK + 1];
  if (tid == 0) {
    int c = 0;
    cum_s[0] = 0;
    for (int i = 0; i < kMaxK; ++i) {
      c += i < a.n_preds ? a.q.counts[a.pred[i]] : 0;
      cum_s[i + 1] = c;
    }
  }
  __syncthreads();
  const int total = cum_s[kMaxK];
  const int G = gridDim.x;
  // This workgroup's queue entries, their slots and decision thresholds are staged in LDS, ECH
  // frames per chunk, double-buffered: wave 0 requests chunk c + 1 when chunk c starts.  The
  // per-frame path then issues no dependent global load (a wave's vector loads complete in issue
  // order, so a per-frame entry or threshold load would hold up the next weight wait).
  constexpr int ECH = 64;
  __shared__ uint32_t ring_e[2 * ECH];
  __shared__ float ring_th[2 * ECH];
  __shared__ uint8_t ring_s[2 * ECH];
  auto fill = [&](int c, int lo) {
    const int i = tid - lo;
    if (i >= 0 && i < ECH) {
      const int t = (int)blockIdx.x + (c * ECH + i) * G;
      if (t < total) {
        int slot = 0, base = 0;
        for (int j = 1; j < a.n_preds; ++j)
          if (t >= cum_s[j]) { slot = j; base = cum_s[j]; }
        const uint32_t e = a.q.entries[(int64_t)a.pred[slot] * a.q.cap + (t - base)];
        ring_e[(c & 1) * ECH + i] = e;
        ring_s[(c & 1) * ECH + i] = (uint8_t)slot;
        ring_th[(c & 1) * ECH + i] = f.logits == nullptr ? theta_of(f, a.pred[slot], entry_idx(e)) : 0.f;
      }
    }
  };
  fill(0, 0);
  fill(1, 64);
  __syncthreads();
  if ((int)blockIdx.x < total) {
    FramePrefetch<NT> pf;
    frame_issue<NT>(a, entry_idx(ring_e[0]), pf);
    frame_store<T, NT>(a, pf, region);
  }
  __syncthreads();
  int loaded = -1;
  int nf = 0;   // frames of this workgroup so far
  for (int t = blockIdx.x; t < total; t += G, ++nf) {
    if (nf % ECH == 0 && nf > 0) fill(nf / ECH + 1, 0);   // read after this frame's barriers
    const int slot = ring_s[nf % (2 * ECH)];
    const int k = a.pred[slot];
    const int v = a.variant[slot];
    if (slot != loaded) {
      const int m = v == CNN_W4 ? 4 : v == CNN_W2 ? 2 : 1;
      for (int q = tid; q < 16 * m; q += NT) sh.cb[q] = a.bias[slot][0][q];
      for (int q = tid; q < 32 * m; q += NT) sh.cb[CB_L2 + q] = a.bias[slot][1][q];
      for (int q = tid; q < 64 * m; q += NT) sh.cb[CB_L3 + q] = a.bias[slot][2][q];
      if (tid < kClasses) sh.fcb[tid] = a.fc_b[slot][tid];
      if constexpr (sizeof(T) == 2) {
        for (int q = tid; q < 64 * m * kClasses; q += NT) fcw_s[q] = a.fc_w[slot][q];
      }
      __syncthreads();
      loaded = slot;
    }
    const float* fcw = sizeof(T) == 2 ? fcw_s : a.fc_w[slot];
    const uint32_t e = ring_e[nf % (2 * ECH)];
    const uint32_t idx = entry_idx(e);
    const float th = ring_th[nf % (2 * ECH)];
    const bool next_valid = t + G < total;
    // with no next frame, the loads re-read this one (cached) unused
    const uint32_t next_idx = next_valid ? entry_idx(ring_e[(nf + 1) % (2 * ECH)]) : idx;
    __bf16* feat_dst = a.feats != nullptr && f.logits == nullptr && entry_mask(e) == 0
                           ? a.feats + (int64_t)idx * 192 : nullptr;
    unsigned long long t0 = wall_clock64();
    float z[kClasses];
    if constexpr ((VSET & 4) != 0) {
      if (v == CNN_W4) cnn_frame<T, 4, NWV>(a, slot, region, sh, fcw, next_valid, next_idx, feat_dst, z);
    }
    if constexpr ((VSET & 2) != 0) {
      if (v == CNN_W2) cnn_frame<T, 2, NWV>(a, slot, region, sh, fcw, next_valid, next_idx, feat_dst, z);
    }
    if constexpr ((VSET & 1) != 0) {
      if (v == CNN_W1) cnn_frame<T, 1, NWV>(a, slot, region, sh, fcw, next_valid, next_idx, feat_dst, z);
    }
    if (tid == 0) {
      if (f.logits != nullptr) {
        for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = (double)z[c];
      } else {
        float d = class_margin(z, a.class_mask[slot]);
        bool defer = f.defer.entries != nullptr && fabsf(d - th) < f.tau[k];
        int n = sh.d_n;
        sh.d_e[n] = e;
        sh.d_k[n] = (uint8_t)k;
        sh.d_f[n] = (uint8_t)((d > th ? 1 : 0) | (defer ? 2 : 0));
        sh.d_n = n + 1;
      }
      sh.ticks[k] += wall_clock64() - t0;
    }
    __syncthreads();
    if (sh.d_n == DBUF) flush_decisions(f, sh, a.n_preds, a.pred);
  }
  if (f.logits == nullptr) flush_decisions(f, sh, a.n_preds, a.pred);
  __syncthreads();
  if (tid < kMaxK && sh.ticks[tid] && a.count_ticks) atomicAdd(&a.st->r_ticks[tid], sh.ticks[tid]);
}

// ---------------------------------------------------------------- FP64 tier
// The frame normalised in fp64 exactly as defined, the canonical (unfolded) fp32 weights
// widened to fp64, fp64 accumulation.  The first esc_cap escalated entries of each predicate are
// evaluated layer-parallel across the whole GPU: layer 1 with one thread per output activation,
// layers 2 and 3 with one wave per output activation whose lanes split the (tap, channel) sum
// (weights laid out [co][3][3][ci] so the lanes read consecutive weights and activations) and
// reduce it with cross-lane adds; any entries beyond that run one per workgroup.
__device__ inline double frame_norm64(const FrameSrc& fr, uint32_t idx, int y, int x, int c) {
  const int64_t o = (int64_t)idx * fr.elems + ((int64_t)y * fr.hw + x) * 3 + c;
  double v;
  if (fr.dtype == HYDRO_DTYPE_BF16) v = (double)(float)static_cast<const __bf16*>(fr.base)[o];
  else v = (double)static_cast<const uint8_t*>(fr.base)[o] / 255.0;
  return (v - 0.5) * 4.0;
}

__device__ inline int mult_dev(int variant) { return variant == CNN_W1 ? 1 : variant == CNN_W2 ? 2 : 4; }

// Activation (after ReLU) of output (p, o) of `layer` for one entry.  `in` is the previous layer's
// output ([H][H][Cin] fp64) for layers 1 and 2.
__device__ inline double conv64_at(const CnnArgs& a, int slot, int layer, uint32_t idx, const double* in, int p, int o) {
  const int m = mult_dev(a.variant[slot]);
  const int cin = layer == 0 ? 3 : layer == 1 ? 16 * m : 32 * m;
  const int hin = layer == 0 ? H0 : layer == 1 ? H1 : H2;
  const int hout = hin / 2;
  const int i = p / hout, j = p % hout;
  const float* W = a.wt_canon[slot][layer];
  double s = (double)a.b_canon[slot][layer][o];
  for (int u = 0; u < 3; ++u) {
    const int y = 2 * i + u - 1;
    if (y < 0 || y >= hin) continue;
    for (int v = 0; v < 3; ++v) {
      const int x = 2 * j + v - 1;
      if (x < 0 || x >= hin) continue;
      const float* w = W + ((o * 3 + u) * 3 + v) * cin;
      if (layer == 0) {
        for (int c = 0; c < 3; ++c) s = fma((double)w[c], frame_norm64(a.fr, idx, y, x, c), s);
      } else {
        const double* xin = in + (y * hin + x) * cin;
        for (int c = 0; c < cin; ++c) s = fma((double)w[c], xin[c], s);
      }
    }
  }
  return s > 0.0 ? s : 0.0;
}

__device__ inline int64_t act_off(int layer, int m) {
  // per entry: [layer-1 output | layer-2 output]; layer 3 reuses the layer-1 region
  return layer == 1 ? (int64_t)H1 * H1 * 16 * m : 0;
}

__device__ inline void f64_decode(const CnnArgs& a, int layer, int64_t gi, const int* ne, const int64_t* outs,
                                  int& slot, int& e, int& p, int& o) {
  slot = 0;
  int64_t rem = gi;
  for (int i = 0; i < a.n_preds; ++i) {
    const int64_t c = ne[i] * outs[i];
    if (rem < c) { slot = i; break; }
    rem -= c;
  }
  e = (int)(rem / outs[slot]);
  const int oi = (int)(rem % outs[slot]);
  const int m = mult_dev(a.variant[slot]);
  const int cout = layer == 0 ? 16 * m : layer == 1 ? 32 * m : 64 * m;
  p = oi / cout;
  o = oi % cout;
}

__global__ __launch_bounds__(256) void cnn_f64_layer_kernel(CnnArgs a, int layer) {
  int64_t total = 0;
  int64_t outs[kMaxK];
  int ne[kMaxK];
  for (int i = 0; i < a.n_preds; ++i) {
    const int m = mult_dev(a.variant[i]);
    const int hout = layer == 0 ? H1 : layer == 1 ? H2 : H3;
    const int cout = layer == 0 ? 16 * m : layer == 1 ? 32 * m : 64 * m;
    ne[i] = min(a.q.counts[a.pred[i]], a.esc_cap);
    outs[i] = (int64_t)hout * hout * cout;
    total += ne[i] * outs[i];
  }
  if (layer == 0) {
    // layer 1 (27 products per output): one thread per output
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < total; gi += stride) {
      int slot, e, p, o;
      f64_decode(a, 0, gi, ne, outs, slot, e, p, o);
      const int m = mult_dev(a.variant[slot]);
      const uint32_t idx = entry_idx(a.q.entries[(int64_t)a.pred[slot] * a.q.cap + e]);
      double* act = a.esc_act[slot] + (int64_t)e * a.esc_stride;
      act[p * 16 * m + o] = conv64_at(a, slot, 0, idx, nullptr, p, o);
    }
    return;
  }
  // layers 2 and 3: one wave per output, lanes over (tap, input channel)
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t gi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); gi < total; gi += nwaves) {
    int slot, e, p, o;
    f64_decode(a, layer, gi, ne, outs, slot, e, p, o);
    const int m = mult_dev(a.variant[slot]);
    const int cin = layer == 1 ? 16 * m : 32 * m;
    const int cout = layer == 1 ? 32 * m : 64 * m;
    const int hin = layer == 1 ? H1 : H2, hout = hin / 2;
    const int i = p / hout, j = p % hout;
    double* act = a.esc_act[slot] + (int64_t)e * a.esc_stride;
    const double* in = layer == 1 ? act + act_off(0, m) : act + act_off(1, m);
    const float* W = a.wt_canon[slot][layer] + (int64_t)o * 9 * cin;
    double s = 0.0;
    for (int kk = lane; kk < 9 * cin; kk += 64) {
      const int t = kk / cin, c = kk % cin;
      const int y = 2 * i + t / 3 - 1, x = 2 * j + t % 3 - 1;
      if (y >= 0 && x >= 0 && y < hin && x < hin) s = fma((double)W[kk], in[(y * hin + x) * cin + c], s);
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
      s += (double)a.b_canon[slot][layer][o];
      double* out = layer == 1 ? act + act_off(1, m) : act;   // layers 1 and 3 share a region
      out[p * cout + o] = s > 0.0 ? s : 0.0;
    }
  }
}

// Pool, FC, margin and decision: one wave per escalated entry.
__device__ inline void cnn_head64(const CnnArgs& a, const Forward& f, int slot, uint32_t e, const double* act3,
                                  bool active) {
  const int lane = threadIdx.x & 63;
  const int m = mult_dev(a.variant[slot]);
  const int C3 = 64 * m;
  double zp[kClasses];
#pragma unroll
  for (int c = 0; c < kClasses; ++c) zp[c] = 0.0;
  if (active) {
    const float* fw = a.fc_w[slot];
    for (int ch = lane; ch < C3; ch += 64) {
      double sum = 0.0;
      for (int p = 0; p < H3 * H3; ++p) sum += act3[p * C3 + ch];
      const double gch = sum / 64.0;
#pragma unroll
      for (int c = 0; c < kClasses; ++c) zp[c] = fma(gch, (double)fw[ch * kClasses + c], zp[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < kClasses; ++c)
    for (int o = 32; o >= 1; o >>= 1) zp[c] += __shfl_xor(zp[c], o);
  const int k = a.pred[slot];
  const uint32_t idx = entry_idx(e);
  bool lead = active && lane == 0;
  bool pass = false;
  if (lead) {
    double z[kClasses];
    for (int c = 0; c < kClasses; ++c) z[c] = (double)a.fc_b[slot][c] + zp[c];
    if (f.logits != nullptr)
      for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = z[c];
    pass = class_margin(z, a.class_mask[slot]) > (double)theta_of(f, k, idx);
  }
  if (f.logits == nullptr) forward_decision(f, k, e, lead, false, pass);
}

__global__ __launch_bounds__(256) void cnn_f64_head_kernel(CnnArgs a, Forward f) {
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += min(a.q.counts[a.pred[i]], a.esc_cap);
  const int wave = threadIdx.x >> 6;
  const int nw = gridDim.x * 4;
  for (int base = blockIdx.x * 4; base < total; base += nw) {
    const int t = base + wave;
    const bool active = t < total;
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = min(a.q.counts[a.pred[i]], a.esc_cap);
      if (off < c) { slot = i; break; }
      off -= c;
    }
    if (!active) { slot = 0; off = 0; }
    const uint32_t e = active ? a.q.entries[(int64_t)a.pred[slot] * a.q.cap + off] : 0u;
    const double* act3 = a.esc_act[slot] + (int64_t)off * a.esc_stride;
    cnn_head64(a, f, slot, e, act3, active);
  }
}

// Entries beyond esc_cap: one workgroup per entry, per-block scratch.
__global__ __launch_bounds__(256) void cnn_f64_rest_kernel(CnnArgs a, Forward f) {
  const int tid = threadIdx.x;
  double* A = a.scratch64 + (int64_t)blockIdx.x * a.scratch64_per_block;
  double* B = A + a.scratch64_per_block / 2;
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += max(0, a.q.counts[a.pred[i]] - a.esc_cap);
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = max(0, a.q.counts[a.pred[i]] - a.esc_cap);
      if (off < c) { slot = i; break; }
      off -= c;
    }
    off += a.esc_cap;
    const int k = a.pred[slot];
    const uint32_t e = a.q.entries[(int64_t)k * a.q.cap + off];
    const uint32_t idx = entry_idx(e);
    const int m = mult_dev(a.variant[slot]);
    for (int q = tid; q < H1 * H1 * 16 * m; q += 256) A[q] = conv64_at(a, slot, 0, idx, nullptr, q / (16 * m), q % (16 * m));
    __syncthreads();
    for (int q = tid; q < H2 * H2 * 32 * m; q += 256) B[q] = conv64_at(a, slot, 1, idx, A, q / (32 * m), q % (32 * m));
    __syncthreads();
    for (int q = tid; q < H3 * H3 * 64 * m; q += 256) A[q] = conv64_at(a, slot, 2, idx, B, q / (64 * m), q % (64 * m));
    __syncthreads();
    if (tid < 64) cnn_head64(a, f, slot, e, A, true);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host helpers
int cnn_variant_of(int in_hw, int n_layers, const int* widths) {
  if (in_hw != 64 || n_layers != 3) return CNN_NONE;
  for (int v = 0, m = 1; v < 3; ++v, m *= 2)
    if (widths[0] == 16 * m && widths[1] == 32 * m && widths[2] == 64 * m) return v;
  return CNN_NONE;
}

static int mult_of(int variant) { return variant == CNN_W1 ? 1 : variant == CNN_W2 ? 2 : 4; }

template <typename T>
static size_t packed_elems_t(int variant, int layer) {
  const int m = mult_of(variant);
  return (size_t)cnn_slabs(layer, m) * cnn_ksteps<T>(layer, m) * cnn_ntiles(layer, m) * 64 * Mf<T>::KPL;
}

size_t cnn_packed_elems(int variant, int layer, int prec) {
  return prec == HYDRO_PREC_BF16 ? packed_elems_t<__bf16>(variant, layer) : packed_elems_t<float>(variant, layer);
}

// Pack one conv layer ([co][ci][3][3] fp32, scaled by `scale`) into fragment order.
template <typename T>
static void pack_t(int variant, int layer, const float* w, float scale, float* out) {
  const int m = mult_of(variant);
  const int KSTEP = Mf<T>::KSTEP, KPL = Mf<T>::KPL;
  const int slabs = cnn_slabs(layer, m), ks_n = cnn_ksteps<T>(layer, m), nt_n = cnn_ntiles(layer, m);
  const int C2 = 32 * m;
  const int cin = layer == 0 ? 3 : layer == 1 ? 16 * m : C2;
  size_t o = 0;
  for (int sl = 0; sl < slabs; ++sl)
    for (int ks = 0; ks < ks_n; ++ks)
      for (int nt = 0; nt < nt_n; ++nt)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < KPL; ++e) {
            const int k = ks * KSTEP + KPL * (lane >> 4) + e;
            const int n = nt * 16 + (lane & 15);
            int oc, ic, tap;
            bool valid;
            if (layer == 0) {
              // k = 9u + 3v + c
              tap = (k / 9) * 3 + (k % 9) / 3;
              ic = k % 3;
              oc = sl * CB1 + n;
              valid = k < 27;
            } else if (layer == 1) {
              tap = k / CB1;
              ic = sl * CB1 + k % CB1;
              oc = n;
              valid = tap < 9;
            } else {
              tap = k / C2;
              ic = k % C2;
              oc = n;
              valid = tap < 9;
            }
            out[o++] = valid ? scale * w[((size_t)(oc * cin + ic) * 3 + tap / 3) * 3 + tap % 3] : 0.f;
          }
}

void cnn_pack_layer(int variant, int layer, int prec, const float* w_canon, float scale, float* out) {
  if (prec == HYDRO_PREC_BF16) pack_t<__bf16>(variant, layer, w_canon, scale, out);
  else pack_t<float>(variant, layer, w_canon, scale, out);
}

void launch_cnn_pass(const CnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s) {
  if (a.n_preds == 0) return;
  if (tier == TIER_F64) {
    for (int layer = 0; layer < 3; ++layer)
      hipLaunchKernelGGL(cnn_f64_layer_kernel, dim3(grid * 4), dim3(256), 0, s, a, layer);
    hipLaunchKernelGGL(cnn_f64_head_kernel, dim3(grid), dim3(256), 0, s, a, f);
    hipLaunchKernelGGL(cnn_f64_rest_kernel, dim3(a.rest_grid), dim3(256), 0, s, a, f);
    return;
  }
  // FP32: one persistent launch over every queue of the pass.  BF16: one launch per width class
  // (a shared launch would give the narrow classes the widest one's register allocation and code
  // footprint, measured slower): the widest class runs 8-wave workgroups, one per CU; the two
  // narrower classes run 4-wave workgroups, two per CU, so one workgroup's LDS phases overlap the
  // other's matrix phases.
  if (!(a.prec == HYDRO_PREC_BF16 && tier == TIER_FIRST)) {
    hipLaunchKernelGGL((cnn_fused_kernel<float, 7>), dim3(grid), dim3(NTHR), 0, s, a, f);
    return;
  }
  for (int v = CNN_W4; v >= CNN_W1; --v) {
    CnnArgs b = a;
    b.n_preds = 0;
    for (int i = 0; i < a.n_preds; ++i) {
      if (a.variant[i] != v) continue;
      const int j = b.n_preds++;
      b.pred[j] = a.pred[i]; b.variant[j] = a.variant[i]; b.class_mask[j] = a.class_mask[i];
      for (int l = 0; l < 3; ++l) {
        b.w_bf[j][l] = a.w_bf[i][l]; b.w_s3[j][l] = a.w_s3[i][l]; b.bias[j][l] = a.bias[i][l];
        b.w_canon[j][l] = a.w_canon[i][l]; b.b_canon[j][l] = a.b_canon[i][l]; b.wt_canon[j][l] = a.wt_canon[i][l];
      }
      b.fc_w[j] = a.fc_w[i]; b.fc_b[j] = a.fc_b[i]; b.esc_act[j] = a.esc_act[i];
    }
    if (b.n_preds == 0) continue;
    if (v == CNN_W4) hipLaunchKernelGGL((cnn_fused_kernel<__bf16, 4>), dim3(grid), dim3(NTHR), 0, s, b, f);
    else if (v == CNN_W2) hipLaunchKernelGGL((cnn_fused_kernel<__bf16, 2, 4>), dim3(grid * 2), dim3(256), 0, s, b, f);
    else hipLaunchKernelGGL((cnn_fused_kernel<__bf16, 1, 4>), dim3(grid * 2), dim3(256), 0, s, b, f);
  }
}

}  // namespace hydro
