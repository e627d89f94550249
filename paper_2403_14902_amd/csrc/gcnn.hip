// Generic CNN predicates on gfx950 (any square input divisible by 2^L, up to 4 conv3x3/s2
// layers with widths that are multiples of 16): used when a model's activations do not fit the
// fused per-frame kernel (e.g. 128x128 frames with 4 layers).
//
// Each layer is one implicit-GEMM launch over every queued frame of the tier: rows = output
// positions of all frames (a 64-row tile may span frames, so each weight fragment serves
// 64 positions), columns = output channels, K = (tap, input channel).  Activations live in a
// per-tier scratch (bf16 or fp32, NHWC per frame).  Layer 1 reads the raw frame (bf16 or uint8,
// exact in bf16) with the normalisation folded into its weights and border taps set to the raw
// value that normalises to zero.  A head launch pools, applies FC and decides.  The FP64 tier
// evaluates the same layers with one wave per output activation.
#include "engine.h"

namespace hydro {

typedef float floatx4_g __attribute__((ext_vector_type(4)));

template <typename T> struct GMf;
template <> struct GMf<__bf16> { static constexpr int KSTEP = 32, KPL = 8; typedef bf16x8 frag; };
template <> struct GMf<float> { static constexpr int KSTEP = 4, KPL = 1; typedef float frag; };

__device__ inline floatx4 gmfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 gmfma(float a, float b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// K of a layer, padded: layer 1 uses k = (u*3 + v)*3 + c (27 real values); later layers
// k = (u*3 + v)*Cin + c.
__host__ __device__ inline int g_kreal(int layer, int cin) { return layer == 0 ? 27 : 9 * cin; }
template <typename T>
__host__ __device__ inline int g_ksteps(int layer, int cin) {
  return (g_kreal(layer, cin) + GMf<T>::KSTEP - 1) / GMf<T>::KSTEP;
}

constexpr int GT_M = 64;     // positions per tile
constexpr int GT_N = 64;     // channels per tile

// One layer over all frames of all generic-CNN predicates in this launch.
template <typename T>
__global__ __launch_bounds__(256) void gconv_layer_kernel(GcnnArgs a, int layer) {
  typedef typename GMf<T>::frag frag;
  constexpr int KSTEP = GMf<T>::KSTEP, KPL = GMf<T>::KPL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  // tiles per predicate slot: ceil(count * P / 64) position tiles x Cout / 64 channel tiles
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) {
    if (layer >= a.n_layers[i]) continue;
    const int hout = a.in_hw[i] >> (layer + 1);
    const int64_t rows = (int64_t)a.q.counts[a.pred[i]] * hout * hout;
    total += (int)((rows + GT_M - 1) / GT_M) * (a.widths[i][layer] / GT_N > 0 ? a.widths[i][layer] / GT_N : 1);
  }
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      if (layer >= a.n_layers[i]) continue;
      const int hout = a.in_hw[i] >> (layer + 1);
      const int64_t rows = (int64_t)a.q.counts[a.pred[i]] * hout * hout;
      const int c = (int)((rows + GT_M - 1) / GT_M) * (a.widths[i][layer] / GT_N > 0 ? a.widths[i][layer] / GT_N : 1);
      if (off < c) { slot = i; break; }
      off -= c;
    }
    const int k = a.pred[slot];
    const int cnt = a.q.counts[k];
    const int hin = a.in_hw[slot] >> layer, hout = hin >> 1, P = hout * hout;
    const int cin = layer == 0 ? 3 : a.widths[slot][layer - 1];
    const int cout = a.widths[slot][layer];
    const int nct = cout / GT_N > 0 ? cout / GT_N : 1;
    const int ncw = cout < GT_N ? cout / 16 : 4;        // channel tiles of 16 per wave group
    const int mt = off / nct, ct = off % nct;
    const int KS = g_ksteps<T>(layer, cin);
    const frag* wp = reinterpret_cast<const frag*>(sizeof(T) == 2 ? (const void*)a.w_bf[slot][layer]
                                                                  : (const void*)a.w_f32[slot][layer]);
    // this wave's 16 positions
    const int64_t row = (int64_t)mt * GT_M + wave * 16 + l16;
    const bool rvalid = row < (int64_t)cnt * P;
    const int e = rvalid ? (int)(row / P) : 0;
    const int p = rvalid ? (int)(row % P) : 0;
    const int oi = p / hout, oj = p % hout;
    const uint32_t idx = entry_idx(a.q.entries[(int64_t)k * a.q.cap + e]);
    int ebase = 0;
    for (int i = 0; i < slot; ++i) ebase += a.q.counts[a.pred[i]];
    const int64_t ent = (int64_t)ebase + e;
    const T* in = layer == 0 ? nullptr : reinterpret_cast<const T*>(a.act[(layer - 1) & 1]) + ent * a.act_stride;
    floatx4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (floatx4){0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < KS; ++ks) {
      frag av;
      if (layer == 0) {
        // raw frame gather, k = (u*3 + v)*3 + c
        if constexpr (sizeof(T) == 2) {
          alignas(16) __bf16 t8[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int kk = ks * 32 + 8 * g + q;
            float v = 0.f;
            if (kk < 27 && rvalid) {
              const int tap = kk / 3, c = kk % 3, y = 2 * oi + tap / 3 - 1, x = 2 * oj + tap % 3 - 1;
              if (y < 0 || x < 0 || y >= hin || x >= hin) v = a.pad_raw;
              else {
                const int64_t o = (int64_t)idx * a.fr.elems + ((int64_t)y * hin + x) * 3 + c;
                v = a.fr.dtype == HYDRO_DTYPE_BF16 ? (float)static_cast<const __bf16*>(a.fr.base)[o]
                                                  : (float)static_cast<const uint8_t*>(a.fr.base)[o];
              }
            }
            t8[q] = static_cast<__bf16>(v);
          }
          av = *reinterpret_cast<const bf16x8*>(t8);
        } else {
          const int kk = ks * 4 + g;
          float v = 0.f;
          if (kk < 27 && rvalid) {
            const int tap = kk / 3, c = kk % 3, y = 2 * oi + tap / 3 - 1, x = 2 * oj + tap % 3 - 1;
            if (y < 0 || x < 0 || y >= hin || x >= hin) v = a.pad_raw;
            else {
              const int64_t o = (int64_t)idx * a.fr.elems + ((int64_t)y * hin + x) * 3 + c;
              v = a.fr.dtype == HYDRO_DTYPE_BF16 ? (float)static_cast<const __bf16*>(a.fr.base)[o]
                                                : (float)static_cast<const uint8_t*>(a.fr.base)[o];
            }
          }
          av = v;
        }
      } else {
        const int k0 = ks * KSTEP + KPL * g;
        const int tap = k0 / cin, c0 = k0 % cin;
        const int y = 2 * oi + tap / 3 - 1, x = 2 * oj + tap % 3 - 1;
        if (rvalid && tap < 9 && y >= 0 && x >= 0 && y < hin && x < hin) {
          const T* src = in + ((int64_t)y * hin + x) * cin + c0;
          if constexpr (sizeof(T) == 2) av = *reinterpret_cast<const bf16x8*>(src);
          else av = *src;
        } else {
          if constexpr (sizeof(T) == 2) av = bf16x8{};
          else av = 0.f;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < ncw) acc[j] = gmfma(wp[((int64_t)ks * (cout / 16) + ct * 4 + j) * 64 + lane], av, acc[j]);
    }
    // bias + ReLU -> activations (rows = channels 4g.., column = this lane's position)
    if (rvalid) {
      const float* bias = a.bias[slot][layer];
      T* out = reinterpret_cast<T*>(a.act[layer & 1]) + ent * a.act_stride + (int64_t)p * cout;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j >= ncw) continue;
        const int ch = ct * GT_N + j * 16 + 4 * g;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[ch + r] = static_cast<T>(fmaxf(acc[j][r] + bias[ch + r], 0.f));
      }
    }
  }
}

// Layers after the first when Cin is a multiple of the k-block and Cout of 64: an LDS-tiled
// implicit GEMM.  Tile = 128 output positions (any frames of one slot) x BN output channels
// (128 when Cout allows, else 64);
// k-block = 32 (bf16) or 16 (fp32) consecutive input channels of one tap, so each position's
// slice of the block is one contiguous run of its NHWC input.  Activations and the packed
// weight fragments of a block are staged in LDS (double buffer) from NS register stages of
// global loads; wave w multiplies channels 0..BN-1 (MFMA A, from the weights) by positions
// 32w..32w+31 (MFMA B), so each lane ends with 4 consecutive channels of one position.
template <typename T> struct GTile;
template <> struct GTile<__bf16> { static constexpr int BK = 32, LD = 40; };
template <> struct GTile<float> { static constexpr int BK = 16, LD = 20; };
constexpr int GB_M = 128;

__host__ __device__ inline bool gconv_tiled_ok(int layer, int cin, int cout, int bk, int bn) {
  return layer > 0 && cin % bk == 0 && cout % bn == 0;
}

template <typename T, int GB_N>
__global__ __launch_bounds__(256) void gconv_tile_kernel(GcnnArgs a, int layer) {
  typedef typename GMf<T>::frag frag;
  constexpr int BK = GTile<T>::BK, LD = GTile<T>::LD, KSTEP = GMf<T>::KSTEP, KPL = GMf<T>::KPL;
  constexpr int KSUB = BK / KSTEP;                 // MFMA k-steps per block (1 bf16, 4 fp32)
  constexpr int NS = 4;
  constexpr int NCT = GB_N / 16;                   // 16-channel MFMA tiles per block
  constexpr int WV = NCT / 4;                      // 16-byte weight chunks per thread and block
  __shared__ __attribute__((aligned(16))) T Xs[2][GB_M * LD];
  __shared__ __attribute__((aligned(16))) uint4 Ws[2][256 * WV];   // KSUB x NCT tiles x 64 lanes
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;

  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) {
    if (layer >= a.n_layers[i]) continue;
    const int hout = a.in_hw[i] >> (layer + 1);
    const int64_t rows = (int64_t)a.q.counts[a.pred[i]] * hout * hout;
    total += (int)((rows + GB_M - 1) / GB_M) * (a.widths[i][layer] / GB_N);
  }
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t, ebase = 0;
    for (int i = 0; i < a.n_preds; ++i) {
      if (layer >= a.n_layers[i]) { ebase += a.q.counts[a.pred[i]]; continue; }
      const int hout = a.in_hw[i] >> (layer + 1);
      const int64_t rows = (int64_t)a.q.counts[a.pred[i]] * hout * hout;
      const int c = (int)((rows + GB_M - 1) / GB_M) * (a.widths[i][layer] / GB_N);
      if (off < c) { slot = i; break; }
      off -= c;
      ebase += a.q.counts[a.pred[i]];
    }
    const int cnt = a.q.counts[a.pred[slot]];
    const int hin = a.in_hw[slot] >> layer, hout = hin >> 1, P = hout * hout;
    const int cin = a.widths[slot][layer - 1], cout = a.widths[slot][layer];
    const int nct = cout / GB_N;
    const int mt = off / nct, cb = off % nct;   // cb: block of GB_N channels
    const int nkb = 9 * cin / BK;
    const int ctile16 = cout / 16;
    const frag* wp = reinterpret_cast<const frag*>(sizeof(T) == 2 ? (const void*)a.w_bf[slot][layer]
                                                                  : (const void*)a.w_f32[slot][layer]);
    const T* act_in = reinterpret_cast<const T*>(a.act[(layer - 1) & 1]);
    // staging row of this thread (two threads per row, BK / 2 elements each)
    const int srow = tid >> 1, shalf = tid & 1;
    const int64_t R = (int64_t)mt * GB_M + srow;
    const bool svalid = R < (int64_t)cnt * P;
    const int se = svalid ? (int)(R / P) : 0, sp = svalid ? (int)(R % P) : 0;
    const int soi = sp / hout, soj = sp % hout;
    const T* sin = act_in + ((int64_t)ebase + se) * a.act_stride;

    uint4 rx[NS][BK * (int)sizeof(T) / 32];   // 32 bytes of activations per stage
    uint4 rw[NS][WV];
    auto gload = [&](int kb, int st) {
      const int k0 = kb * BK, tap = k0 / cin, c0 = k0 % cin;
      const int y = 2 * soi + tap / 3 - 1, x = 2 * soj + tap % 3 - 1;
      if (svalid && y >= 0 && x >= 0 && y < hin && x < hin) {
        const uint4* src = reinterpret_cast<const uint4*>(sin + ((int64_t)y * hin + x) * cin + c0 + shalf * (BK / 2));
#pragma unroll
        for (int v = 0; v < BK * (int)sizeof(T) / 32; ++v) rx[st][v] = src[v];
      } else {
#pragma unroll
        for (int v = 0; v < BK * (int)sizeof(T) / 32; ++v) rx[st][v] = make_uint4(0u, 0u, 0u, 0u);
      }
      // weights, chunk q = tid + 256 v: bf16 fragment (ks = kb, tile cb*NCT + q/64, lane q%64);
      // fp32: 4 consecutive lanes of (ks = kb*4 + kss, tile) with q = (kss*NCT + tile)*16 + lane/4
#pragma unroll
      for (int v = 0; v < WV; ++v) {
        const int q = tid + 256 * v;
        if constexpr (sizeof(T) == 2) {
          rw[st][v] = *reinterpret_cast<const uint4*>(&wp[((int64_t)kb * ctile16 + cb * NCT + (q >> 6)) * 64 + (q & 63)]);
        } else {
          const int kss = q / (NCT * 16), tl = (q >> 4) % NCT, l4 = (q & 15) * 4;
          rw[st][v] = *reinterpret_cast<const uint4*>(&wp[((int64_t)(kb * 4 + kss) * ctile16 + cb * NCT + tl) * 64 + l4]);
        }
      }
    };
    auto lstore = [&](int st, int buf) {
#pragma unroll
      for (int v = 0; v < BK * (int)sizeof(T) / 32; ++v)
        reinterpret_cast<uint4*>(&Xs[buf][srow * LD + shalf * (BK / 2)])[v] = rx[st][v];
#pragma unroll
      for (int v = 0; v < WV; ++v) Ws[buf][tid + 256 * v] = rw[st][v];
    };

    floatx4 acc[NCT][2];
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[c][q] = (floatx4){0.f, 0.f, 0.f, 0.f};
    auto compute = [&](int buf) {
#pragma unroll
      for (int kss = 0; kss < KSUB; ++kss) {
        frag xf[2], wf[NCT];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const T* xp = &Xs[buf][(wave * 32 + q * 16 + l16) * LD + kss * KSTEP + KPL * g];
          if constexpr (sizeof(T) == 2) xf[q] = *reinterpret_cast<const bf16x8*>(xp);
          else xf[q] = *xp;
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          if constexpr (sizeof(T) == 2) wf[c] = *reinterpret_cast<const bf16x8*>(&Ws[buf][c * 64 + lane]);
          else wf[c] = reinterpret_cast<const float*>(&Ws[buf][0])[(kss * NCT + c) * 64 + lane];
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c)
#pragma unroll
          for (int q = 0; q < 2; ++q) acc[c][q] = gmfma(wf[c], xf[q], acc[c][q]);
      }
    };

#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
      if (u < nkb) gload(u, u);
    lstore(0, 0);
    __syncthreads();
    for (int kb0 = 0; kb0 < nkb; kb0 += NS) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int kb = kb0 + u;
        if (kb < nkb) {
          const int buf = kb & 1;
          if (kb + NS - 1 < nkb) gload(kb + NS - 1, (u + NS - 1) % NS);
          compute(buf);
          if (kb + 1 < nkb) {
            __syncthreads();
            lstore((u + 1) % NS, buf ^ 1);
            __syncthreads();
          }
        }
      }
    }
    // bias + ReLU; lane holds channels 4g..4g+3 of tile c for position 16q + l16 of its wave
    const float* bias = a.bias[slot][layer] + cb * GB_N;
    T* out = reinterpret_cast<T*>(a.act[layer & 1]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t Ro = (int64_t)mt * GB_M + wave * 32 + q * 16 + l16;
      if (Ro >= (int64_t)cnt * P) continue;
      const int e = (int)(Ro / P), p = (int)(Ro % P);
      T* o = out + ((int64_t)ebase + e) * a.act_stride + (int64_t)p * cout + cb * GB_N;
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int ch = c * 16 + 4 * g;
        const float v0 = fmaxf(acc[c][q][0] + bias[ch], 0.f), v1 = fmaxf(acc[c][q][1] + bias[ch + 1], 0.f);
        const float v2 = fmaxf(acc[c][q][2] + bias[ch + 2], 0.f), v3 = fmaxf(acc[c][q][3] + bias[ch + 3], 0.f);
        if constexpr (sizeof(T) == 2) {
          alignas(8) __bf16 h[4] = {static_cast<__bf16>(v0), static_cast<__bf16>(v1), static_cast<__bf16>(v2),
                                    static_cast<__bf16>(v3)};
          *reinterpret_cast<uint2*>(o + ch) = *reinterpret_cast<const uint2*>(h);
        } else {
          *reinterpret_cast<float4*>(o + ch) = make_float4(v0, v1, v2, v3);
        }
      }
    }
    __syncthreads();   // the next tile's prologue rewrites the LDS buffers
  }
}

// First layer (Cin = 3, K = 27) when 128 output positions are whole output rows of one frame
// (hout divides 128, P a multiple of 128) and Cout <= 64: a tile stages the 2*(128/hout) + 1
// input rows it reads (raw values, top border = the pad value) in LDS once, builds the im2col
// fragments from there and writes 128 positions x Cout channels.
__host__ __device__ inline bool gconv_first_ok(int hout, int cout) {
  return hout >= 16 && 128 % hout == 0 && cout % 16 == 0 && cout <= 64;
}

template <typename T>
__global__ __launch_bounds__(256) void gconv_first_kernel(GcnnArgs a) {
  typedef typename GMf<T>::frag frag;
  constexpr int KSTEP = GMf<T>::KSTEP, KPL = GMf<T>::KPL, KS = (27 + KSTEP - 1) / KSTEP;
  constexpr int MAXV = 17 * 33 * 3 > 5 * 129 * 3 ? (17 * 33 * 3 > 3 * 257 * 3 ? 17 * 33 * 3 : 3 * 257 * 3) : 5 * 129 * 3;
  __shared__ float xin[MAXV + 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) {
    const int hout = a.in_hw[i] >> 1;
    total += (int)((int64_t)a.q.counts[a.pred[i]] * hout * hout / 128);
  }
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t, ebase = 0;
    for (int i = 0; i < a.n_preds; ++i) {
      const int hout = a.in_hw[i] >> 1;
      const int c = (int)((int64_t)a.q.counts[a.pred[i]] * hout * hout / 128);
      if (off < c) { slot = i; break; }
      off -= c;
      ebase += a.q.counts[a.pred[i]];
    }
    const int hin = a.in_hw[slot], hout = hin >> 1, P = hout * hout;
    const int cout = a.widths[slot][0], nct = cout / 16;
    const int tiles_per_frame = P / 128, rows_out = 128 / hout, rows_in = 2 * rows_out + 1, W = hin + 1;
    const int e = off / tiles_per_frame, oi0 = (off % tiles_per_frame) * rows_out;
    const uint32_t idx = entry_idx(a.q.entries[(int64_t)a.pred[slot] * a.q.cap + e]);
    // stage input rows y = 2*oi0 - 1 + r, columns x = c - 1 (c = 0 is the left border)
    const int nvals = rows_in * W * 3;
    for (int q = tid; q < nvals; q += 256) {
      const int r = q / (W * 3), rem = q % (W * 3), c = rem / 3, ch = rem % 3;
      const int y = 2 * oi0 - 1 + r, x = c - 1;
      float v = a.pad_raw;
      if (y >= 0 && x >= 0) {
        const int64_t o = (int64_t)idx * a.fr.elems + ((int64_t)y * hin + x) * 3 + ch;
        v = a.fr.dtype == HYDRO_DTYPE_BF16 ? (float)static_cast<const __bf16*>(a.fr.base)[o]
                                          : (float)static_cast<const uint8_t*>(a.fr.base)[o];
      }
      xin[q] = v;
    }
    __syncthreads();
    const frag* wp = reinterpret_cast<const frag*>(sizeof(T) == 2 ? (const void*)a.w_bf[slot][0]
                                                                  : (const void*)a.w_f32[slot][0]);
    floatx4 acc[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[c][q] = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      frag xf[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int pl = wave * 32 + q * 16 + l16, oi = pl / hout, oj = pl % hout;
        const float* base = xin + ((2 * oi) * W + 2 * oj) * 3;
        if constexpr (sizeof(T) == 2) {
          alignas(16) __bf16 t8[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int k = ks * KSTEP + KPL * g + j, tap = k / 3, ch = k % 3;
            t8[j] = static_cast<__bf16>(k < 27 ? base[((tap / 3) * W + tap % 3) * 3 + ch] : 0.f);
          }
          xf[q] = *reinterpret_cast<const bf16x8*>(t8);
        } else {
          const int k = ks * KSTEP + g, tap = k / 3, ch = k % 3;
          xf[q] = k < 27 ? base[((tap / 3) * W + tap % 3) * 3 + ch] : 0.f;
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= nct) continue;
        const frag wf = wp[((int64_t)ks * nct + c) * 64 + lane];
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[c][q] = gmfma(wf, xf[q], acc[c][q]);
      }
    }
    const float* bias = a.bias[slot][0];
    T* o0 = reinterpret_cast<T*>(a.act[0]) + ((int64_t)ebase + e) * a.act_stride + (int64_t)oi0 * hout * cout;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int pl = wave * 32 + q * 16 + l16;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= nct) continue;
        const int ch = c * 16 + 4 * g;
        const float v0 = fmaxf(acc[c][q][0] + bias[ch], 0.f), v1 = fmaxf(acc[c][q][1] + bias[ch + 1], 0.f);
        const float v2 = fmaxf(acc[c][q][2] + bias[ch + 2], 0.f), v3 = fmaxf(acc[c][q][3] + bias[ch + 3], 0.f);
        T* o = o0 + (int64_t)pl * cout + ch;
        if constexpr (sizeof(T) == 2) {
          alignas(8) __bf16 h[4] = {static_cast<__bf16>(v0), static_cast<__bf16>(v1), static_cast<__bf16>(v2),
                                    static_cast<__bf16>(v3)};
          *reinterpret_cast<uint2*>(o) = *reinterpret_cast<const uint2*>(h);
        } else {
          *reinterpret_cast<float4*>(o) = make_float4(v0, v1, v2, v3);
        }
      }
    }
    __syncthreads();   // the next tile restages xin
  }
}

// Pool + FC + margin + decision: one wave per frame.
template <typename T>
__global__ __launch_bounds__(256) void gcnn_head_kernel(GcnnArgs a, Forward f) {
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += a.q.counts[a.pred[i]];
  const int lane = threadIdx.x & 63;
  for (int base = blockIdx.x * 4; base < total; base += gridDim.x * 4) {
    const int t = base + (threadIdx.x >> 6);
    const bool active = t < total;
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = a.q.counts[a.pred[i]];
      if (off < c) { slot = i; break; }
      off -= c;
    }
    if (!active) { slot = 0; off = 0; }
    const int k = a.pred[slot];
    const uint32_t e = active ? a.q.entries[(int64_t)k * a.q.cap + off] : 0u;
    const int L = a.n_layers[slot];
    const int hl = a.in_hw[slot] >> L, P = hl * hl;
    const int cl = a.widths[slot][L - 1];
    float zp[kClasses];
#pragma unroll
    for (int c = 0; c < kClasses; ++c) zp[c] = 0.f;
    if (active) {
      int ebase = 0;
      for (int i = 0; i < slot; ++i) ebase += a.q.counts[a.pred[i]];
      const T* act = reinterpret_cast<const T*>(a.act[(L - 1) & 1]) + ((int64_t)ebase + off) * a.act_stride;
      const float* fw = a.fc_w[slot];
      for (int ch = lane; ch < cl; ch += 64) {
        float s = 0.f;
#pragma unroll 8
        for (int p = 0; p < P; ++p) s += (float)act[(int64_t)p * cl + ch];
        const float gch = s / (float)P;
#pragma unroll
        for (int c = 0; c < kClasses; ++c) zp[c] += gch * fw[ch * kClasses + c];
      }
    }
    wave_sum_n(zp);
    bool pass = false, defer = false;
    if (active) {
      float z[kClasses];
      for (int c = 0; c < kClasses; ++c) z[c] = zp[c] + a.fc_b[slot][c];
      const uint32_t idx = entry_idx(e);
      if (f.logits != nullptr && lane == 0)
        for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = (double)z[c];
      const float d = class_margin(z, a.class_mask[slot]);
      const float th = theta_of(f, k, idx);
      pass = d > th;
      defer = f.defer.entries != nullptr && fabsf(d - th) < f.tau[k];
    }
    if (f.logits == nullptr) forward_decision(f, k, e, active && lane == 0, defer, pass);
  }
}

// ---------------------------------------------------------------- FP64 tier
__device__ inline double g_frame64(const FrameSrc& fr, uint32_t idx, int hw, int y, int x, int c) {
  const int64_t o = (int64_t)idx * fr.elems + ((int64_t)y * hw + x) * 3 + c;
  double v;
  if (fr.dtype == HYDRO_DTYPE_BF16) v = (double)(float)static_cast<const __bf16*>(fr.base)[o];
  else v = (double)static_cast<const uint8_t*>(fr.base)[o] / 255.0;
  return (v - 0.5) * 4.0;
}

// One wave per output activation of every escalated frame (up to esc_cap per predicate).
__global__ __launch_bounds__(256) void gconv64_layer_kernel(GcnnArgs a, int layer) {
  int64_t total = 0;
  int64_t outs[kMaxK];
  int ne[kMaxK];
  for (int i = 0; i < a.n_preds; ++i) {
    ne[i] = layer < a.n_layers[i] ? min(a.q.counts[a.pred[i]], a.esc_cap) : 0;
    const int hout = a.in_hw[i] >> (layer + 1);
    outs[i] = layer < a.n_layers[i] ? (int64_t)hout * hout * a.widths[i][layer] : 0;
    total += ne[i] * outs[i];
  }
  const int lane = threadIdx.x & 63;
  for (int64_t gi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); gi < total; gi += (int64_t)gridDim.x * 4) {
    int slot = 0;
    int64_t rem = gi;
    for (int i = 0; i < a.n_preds; ++i) {
      const int64_t c = ne[i] * outs[i];
      if (rem < c) { slot = i; break; }
      rem -= c;
    }
    const int e = (int)(rem / outs[slot]);
    const int oi_all = (int)(rem % outs[slot]);
    const int cout = a.widths[slot][layer];
    const int cin = layer == 0 ? 3 : a.widths[slot][layer - 1];
    const int hin = a.in_hw[slot] >> layer, hout = hin >> 1;
    const int p = oi_all / cout, o = oi_all % cout, i = p / hout, j = p % hout;
    const uint32_t idx = entry_idx(a.q.entries[(int64_t)a.pred[slot] * a.q.cap + e]);
    double* act = a.esc_act[slot] + (int64_t)e * a.esc_stride;
    const double* in = layer == 0 ? nullptr : act + ((layer - 1) & 1) * a.esc_half;
    const float* W = a.wt_canon[slot][layer] + (int64_t)o * 9 * cin;   // [co][3][3][ci]
    double s = 0.0;
    for (int kk = lane; kk < 9 * cin; kk += 64) {
      const int t = kk / cin, c = kk % cin;
      const int y = 2 * i + t / 3 - 1, x = 2 * j + t % 3 - 1;
      if (y < 0 || x < 0 || y >= hin || x >= hin) continue;
      const double xv = layer == 0 ? g_frame64(a.fr, idx, hin, y, x, c) : in[((int64_t)y * hin + x) * cin + c];
      s = fma((double)W[kk], xv, s);
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
      s += (double)a.b_canon[slot][layer][o];
      act[(layer & 1) * a.esc_half + (int64_t)p * cout + o] = s > 0.0 ? s : 0.0;
    }
  }
}

__global__ __launch_bounds__(256) void gcnn64_head_kernel(GcnnArgs a, Forward f) {
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += min(a.q.counts[a.pred[i]], a.esc_cap);
  const int lane = threadIdx.x & 63;
  for (int base = blockIdx.x * 4; base < total; base += gridDim.x * 4) {
    const int t = base + (threadIdx.x >> 6);
    const bool active = t < total;
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = min(a.q.counts[a.pred[i]], a.esc_cap);
      if (off < c) { slot = i; break; }
      off -= c;
    }
    if (!active) { slot = 0; off = 0; }
    const int k = a.pred[slot];
    const uint32_t e = active ? a.q.entries[(int64_t)k * a.q.cap + off] : 0u;
    const int L = a.n_layers[slot];
    const int hl = a.in_hw[slot] >> L, P = hl * hl;
    const int cl = a.widths[slot][L - 1];
    double zp[kClasses];
#pragma unroll
    for (int c = 0; c < kClasses; ++c) zp[c] = 0.0;
    if (active) {
      const double* act = a.esc_act[slot] + (int64_t)off * a.esc_stride + ((L - 1) & 1) * a.esc_half;
      const float* fw = a.fc_w[slot];
      for (int ch = lane; ch < cl; ch += 64) {
        double s = 0.0;
        for (int p = 0; p < P; ++p) s += act[(int64_t)p * cl + ch];
        const double gch = s / (double)P;
#pragma unroll
        for (int c = 0; c < kClasses; ++c) zp[c] = fma(gch, (double)fw[ch * kClasses + c], zp[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < kClasses; ++c)
      for (int o = 32; o >= 1; o >>= 1) zp[c] += __shfl_xor(zp[c], o);
    bool pass = false;
    const bool lead = active && lane == 0;
    if (lead) {
      double z[kClasses];
      for (int c = 0; c < kClasses; ++c) z[c] = zp[c] + (double)a.fc_b[slot][c];
      const uint32_t idx = entry_idx(e);
      if (f.logits != nullptr)
        for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = z[c];
      pass = class_margin(z, a.class_mask[slot]) > (double)theta_of(f, k, idx);
    }
    if (f.logits == nullptr) forward_decision(f, k, e, lead, false, pass);
  }
}

// Escalated entries beyond esc_cap: one workgroup per entry, per-block scratch.
__global__ __launch_bounds__(256) void gcnn64_rest_kernel(GcnnArgs a, Forward f, double* scratch, int64_t per_block) {
  const int tid = threadIdx.x;
  double* buf[2] = {scratch + (int64_t)blockIdx.x * per_block, scratch + (int64_t)blockIdx.x * per_block + per_block / 2};
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
    const int L = a.n_layers[slot];
    for (int layer = 0; layer < L; ++layer) {
      const int cout = a.widths[slot][layer];
      const int cin = layer == 0 ? 3 : a.widths[slot][layer - 1];
      const int hin = a.in_hw[slot] >> layer, hout = hin >> 1;
      const double* in = buf[(layer + 1) & 1];
      double* out = buf[layer & 1];
      for (int q = tid; q < hout * hout * cout; q += 256) {
        const int p = q / cout, o = q % cout, i = p / hout, j = p % hout;
        const float* W = a.wt_canon[slot][layer] + (int64_t)o * 9 * cin;
        double s = (double)a.b_canon[slot][layer][o];
        for (int t9 = 0; t9 < 9; ++t9) {
          const int y = 2 * i + t9 / 3 - 1, x = 2 * j + t9 % 3 - 1;
          if (y < 0 || x < 0 || y >= hin || x >= hin) continue;
          for (int c = 0; c < cin; ++c) {
            const double xv = layer == 0 ? g_frame64(a.fr, idx, hin, y, x, c) : in[((int64_t)y * hin + x) * cin + c];
            s = fma((double)W[t9 * cin + c], xv, s);
          }
        }
        out[q] = s > 0.0 ? s : 0.0;
      }
      __syncthreads();
    }
    if (tid < 64) {
      const int lane = tid;
      const int hl = a.in_hw[slot] >> L, P = hl * hl, cl = a.widths[slot][L - 1];
      const double* act = buf[(L - 1) & 1];
      double zp[kClasses];
      for (int c = 0; c < kClasses; ++c) zp[c] = 0.0;
      for (int ch = lane; ch < cl; ch += 64) {
        double s = 0.0;
        for (int p = 0; p < P; ++p) s += act[(int64_t)p * cl + ch];
        const double gch = s / (double)P;
        for (int c = 0; c < kClasses; ++c) zp[c] = fma(gch, (double)a.fc_w[slot][ch * kClasses + c], zp[c]);
      }
      for (int c = 0; c < kClasses; ++c)
        for (int o = 32; o >= 1; o >>= 1) zp[c] += __shfl_xor(zp[c], o);
      bool pass = false;
      if (lane == 0) {
        double z[kClasses];
        for (int c = 0; c < kClasses; ++c) z[c] = zp[c] + (double)a.fc_b[slot][c];
        if (f.logits != nullptr)
          for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = z[c];
        pass = class_margin(z, a.class_mask[slot]) > (double)theta_of(f, k, idx);
      }
      if (f.logits == nullptr) forward_decision(f, k, e, lane == 0, false, pass);
    }
    __syncthreads();
  }
}

void launch_gcnn_layerwise(const GcnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s);

// ---------------------------------------------------------------- host side
size_t gcnn_packed_elems(int layer, int cin, int cout, int prec) {
  const int ks = prec == HYDRO_PREC_BF16 ? g_ksteps<__bf16>(layer, cin) : g_ksteps<float>(layer, cin);
  const int kpl = prec == HYDRO_PREC_BF16 ? 8 : 1;
  return (size_t)ks * (cout / 16) * 64 * kpl;
}

// [kstep][channel tile of 16][64 lanes][KPL]; lane l: output channel tile*16 + l%16,
// k = kstep*KSTEP + KPL*(l/16) + e.
void gcnn_pack_layer(int layer, int cin, int cout, int prec, const float* w, float scale, float* out) {
  const int KSTEP = prec == HYDRO_PREC_BF16 ? 32 : 4, KPL = prec == HYDRO_PREC_BF16 ? 8 : 1;
  const int ks_n = prec == HYDRO_PREC_BF16 ? g_ksteps<__bf16>(layer, cin) : g_ksteps<float>(layer, cin);
  const int kreal = g_kreal(layer, cin);
  size_t o = 0;
  for (int ks = 0; ks < ks_n; ++ks)
    for (int ct = 0; ct < cout / 16; ++ct)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < KPL; ++e) {
          const int k = ks * KSTEP + KPL * (lane >> 4) + e;
          const int oc = ct * 16 + (lane & 15);
          float v = 0.f;
          if (k < kreal) {
            int tap, ic;
            if (layer == 0) { tap = k / 3; ic = k % 3; }
            else { tap = k / cin; ic = k % cin; }
            v = scale * w[((size_t)(oc * cin + ic) * 3 + tap / 3) * 3 + tap % 3];
          }
          out[o++] = v;
        }
}

// Slot i of src becomes slot j of dst.
void gcnn_copy_slot(GcnnArgs& dst, int j, const GcnnArgs& src, int i) {
  dst.pred[j] = src.pred[i]; dst.n_layers[j] = src.n_layers[i]; dst.in_hw[j] = src.in_hw[i];
  dst.class_mask[j] = src.class_mask[i]; dst.fc_w[j] = src.fc_w[i]; dst.fc_b[j] = src.fc_b[i];
  dst.esc_act[j] = src.esc_act[i]; dst.c4[j] = src.c4[i];
  dst.c4_w1b[j] = src.c4_w1b[i]; dst.c4_w1f[j] = src.c4_w1f[i];
  for (int l = 0; l < HYDRO_MAX_LAYERS; ++l) {
    dst.widths[j][l] = src.widths[i][l]; dst.w_bf[j][l] = src.w_bf[i][l]; dst.w_f32[j][l] = src.w_f32[i][l];
    dst.bias[j][l] = src.bias[i][l]; dst.wt_canon[j][l] = src.wt_canon[i][l]; dst.b_canon[j][l] = src.b_canon[i][l];
  }
  // (array extents, so that a new entry is never left behind)
  for (size_t p = 0; p < sizeof(src.c4_w2[0]) / sizeof(src.c4_w2[0][0]); ++p) dst.c4_w2[j][p] = src.c4_w2[i][p];
  for (size_t p = 0; p < sizeof(src.c4_wscale[0]) / sizeof(src.c4_wscale[0][0]); ++p) dst.c4_wscale[j][p] = src.c4_wscale[i][p];
  for (size_t p = 0; p < sizeof(src.c4_ascale[0]) / sizeof(src.c4_ascale[0][0]); ++p) dst.c4_ascale[j][p] = src.c4_ascale[i][p];
  for (int l = 0; l < 2; ++l)
    for (size_t p = 0; p < sizeof(src.c4_img[0][0]) / sizeof(src.c4_img[0][0][0]); ++p) dst.c4_img[j][l][p] = src.c4_img[i][l][p];
}

void launch_gcnn_pass(const GcnnArgs& a0, const Forward& f, int tier, int grid, hipStream_t s) {
  if (a0.n_preds == 0) return;
  if (tier != TIER_F64) {
    // slots of the 4-layer 128x128 shape take the dedicated kernels; the rest the layer-wise ones
    GcnnArgs c4a = a0, gen = a0;
    c4a.n_preds = gen.n_preds = 0;
    for (int i = 0; i < a0.n_preds; ++i) {
      if (a0.c4[i]) gcnn_copy_slot(c4a, c4a.n_preds++, a0, i);
      else gcnn_copy_slot(gen, gen.n_preds++, a0, i);
    }
    if (c4a.n_preds > 0) {
      const int p = tier == TIER_MID ? (a0.prec == HYDRO_PREC_FP8 ? C4_BF16 : C4_X3)
                    : tier != TIER_FIRST ? C4_F32
                    : a0.prec == HYDRO_PREC_FP8 ? C4_FP8 : a0.prec == HYDRO_PREC_BF16 ? C4_BF16 : C4_F32;
      launch_c4_pass(c4a, f, p, grid, s);
    }
    if (gen.n_preds == 0) return;
    launch_gcnn_layerwise(gen, f, tier, grid, s);
    return;
  }
  launch_gcnn_layerwise(a0, f, tier, grid, s);
}

void launch_gcnn_layerwise(const GcnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s) {
  int maxl = 0;
  for (int i = 0; i < a.n_preds; ++i) maxl = a.n_layers[i] > maxl ? a.n_layers[i] : maxl;
  if (tier == TIER_F64) {
    for (int l = 0; l < maxl; ++l) hipLaunchKernelGGL(gconv64_layer_kernel, dim3(grid * 8), dim3(256), 0, s, a, l);
    hipLaunchKernelGGL(gcnn64_head_kernel, dim3(grid), dim3(256), 0, s, a, f);
    hipLaunchKernelGGL(gcnn64_rest_kernel, dim3(a.rest_grid), dim3(256), 0, s, a, f, a.rest_scratch, a.rest_per_block);
    return;
  }
  const bool bf = a.prec == HYDRO_PREC_BF16 && tier == TIER_FIRST;
  for (int l = 0; l < maxl; ++l) {
    // the tiled kernel when every slot that has this layer fits its shape constraints
    if (l == 0) {
      bool first_ok = true;
      for (int i = 0; i < a.n_preds; ++i) first_ok = first_ok && gconv_first_ok(a.in_hw[i] >> 1, a.widths[i][0]);
      if (first_ok) {
        if (bf) hipLaunchKernelGGL(gconv_first_kernel<__bf16>, dim3(grid * 4), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(gconv_first_kernel<float>, dim3(grid * 4), dim3(256), 0, s, a);
        continue;
      }
    }
    bool tiled = true, wide = true;
    for (int i = 0; i < a.n_preds; ++i) {
      if (l >= a.n_layers[i]) continue;
      const int cin = l == 0 ? 3 : a.widths[i][l - 1], cout = a.widths[i][l];
      tiled = tiled && gconv_tiled_ok(l, cin, cout, bf ? 32 : 16, 64);
      wide = wide && gconv_tiled_ok(l, cin, cout, bf ? 32 : 16, 128);
    }
    if (tiled && wide) {
      if (bf) hipLaunchKernelGGL((gconv_tile_kernel<__bf16, 128>), dim3(grid * 4), dim3(256), 0, s, a, l);
      else hipLaunchKernelGGL((gconv_tile_kernel<float, 128>), dim3(grid * 4), dim3(256), 0, s, a, l);
    } else if (tiled) {
      if (bf) hipLaunchKernelGGL((gconv_tile_kernel<__bf16, 64>), dim3(grid * 4), dim3(256), 0, s, a, l);
      else hipLaunchKernelGGL((gconv_tile_kernel<float, 64>), dim3(grid * 4), dim3(256), 0, s, a, l);
    } else {
      if (bf) hipLaunchKernelGGL(gconv_layer_kernel<__bf16>, dim3(grid * 4), dim3(256), 0, s, a, l);
      else hipLaunchKernelGGL(gconv_layer_kernel<float>, dim3(grid * 4), dim3(256), 0, s, a, l);
    }
  }
  if (bf) hipLaunchKernelGGL(gcnn_head_kernel<__bf16>, dim3(grid), dim3(256), 0, s, a, f);
  else hipLaunchKernelGGL(gcnn_head_kernel<float>, dim3(grid), dim3(256), 0, s, a, f);
}

}  // namespace hydro
