// MLP predicates on gfx950: gathered-row GEMM1 on MFMA (bf16 or fp32 operands, fp32
// accumulation) with ReLU and a partial GEMM2 in the epilogue; a head kernel that finishes the
// logits, takes the class-subset margin and forwards the decision; and an FP64 tier.
//
// The model (one synthetic UDF predicate): h = ReLU(x' W1 + b1), z = h W2 + b2 with
// x' = (x - 0.5) * 4 flattened NHWC.  The first two passes use the folded form
// h = ReLU((s W1)^T raw + (b1 - 2 colsum(W1))) with s = 4 (or 4/255 for uint8 frames), which is
// the same function of the stored frame without a separate normalisation step.
#include "engine.h"

namespace hydro {

template <typename T> struct MlpTile;
template <> struct MlpTile<__bf16> { static constexpr int BK = 32, LD = 40; };   // LDS row stride (elements)
template <> struct MlpTile<float> { static constexpr int BK = 16, LD = 20; };

// Load `N` consecutive frame elements of type In starting at element `off` of frame `idx`,
// converted to T.  The element type is a template parameter, so the loads are straight-line code
// and the compiler can count the ones in flight precisely.
template <typename T, typename In, int N>
__device__ inline void load_frame_run(const FrameSrc& fr, uint32_t idx, int64_t off, T* out) {
  constexpr int BYTES = N * (int)sizeof(In);
  static_assert(BYTES == 4 || BYTES == 8 || BYTES % 16 == 0, "frame run size");
  const In* p = static_cast<const In*>(fr.base) + (int64_t)idx * fr.elems + off;
  alignas(16) In buf[N];
  if constexpr (BYTES % 16 == 0) {
#pragma unroll
    for (int v = 0; v < BYTES / 16; ++v) reinterpret_cast<uint4*>(buf)[v] = reinterpret_cast<const uint4*>(p)[v];
  } else if constexpr (BYTES == 8) {
    *reinterpret_cast<uint2*>(buf) = *reinterpret_cast<const uint2*>(p);
  } else {
    *reinterpret_cast<uint32_t*>(buf) = *reinterpret_cast<const uint32_t*>(p);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) out[j] = static_cast<T>((float)buf[j]);
}

// Split-K: when a launch has fewer (rows x hidden) tiles than split_below (small queues, e.g.
// the re-score bands), every tile's K range is divided into S parts computed by different
// workgroups, S ~ split_target / tiles.  Each part stores its raw sums in the workspace and
// counts itself in the tile's counter; the part that arrives last adds the S sums in split order
// (deterministic whichever part is last), resets the counter and runs the usual epilogue.  S is
// a pure function of the queue counts.
constexpr int SPLIT_MAX = 8;
__device__ inline int mlp_splits(int base_total, int nk_min, const MlpArgs& a) {
  if (a.splitk_ws == nullptr || base_total <= 0 || base_total >= a.split_below) return 1;
  int sp = (a.split_target + base_total - 1) / base_total;
  sp = min(sp, SPLIT_MAX);
  sp = min(sp, a.split_slots / base_total);
  sp = min(sp, nk_min / 4);
  return max(sp, 1);
}

// Tile shapes (rows of queued tuples x hidden units) an autotuner may pick per predicate.
// Every launch covers the predicates of one tile shape.
template <typename T, typename In, int BM, int BN>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(MlpArgs a) {
  constexpr int BK = MlpTile<T>::BK, LD = MlpTile<T>::LD;
  // every thread loads one run of each k-tile: 256 / BM threads per gathered frame row (PA
  // elements each) and 256 / BN per weight row (PB elements each)
  constexpr int TPA = 256 / BM, PA = BK / TPA, TPB = 256 / BN, PB = BK / TPB;
  constexpr int WM = BM / 2, WN = BN / 2;         // 2 x 2 waves
  constexpr int FM = WM / 16, FN = WN / 16;       // MFMA tiles per wave
  __shared__ __attribute__((aligned(16))) T As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN * LD];
  __shared__ int s_last;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int ar = tid / TPA, ak = (tid % TPA) * PA;   // this thread's frame row in the tile, k offset
  const int br = tid / TPB, bk = (tid % TPB) * PB;   // this thread's weight row in the tile, k offset

  int base_total = 0, nk_min = 1 << 30;
  for (int i = 0; i < a.n_preds; ++i) {
    const int cnt = a.q.counts[a.pred[i]];
    base_total += ((cnt + BM - 1) / BM) * (a.hidden[i] / BN);
    nk_min = min(nk_min, a.d_in[i] / BK);
  }
  const int S = mlp_splits(base_total, nk_min, a);
  const int total = base_total * S;

  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int tb = t / S, sp = t % S;
    int slot = 0, mt = 0, nt = 0;
    {
      int acc0 = 0;
      for (int i = 0; i < a.n_preds; ++i) {
        const int cnt = a.q.counts[a.pred[i]];
        const int n_nt = a.hidden[i] / BN;
        const int tiles = ((cnt + BM - 1) / BM) * n_nt;
        if (tb < acc0 + tiles) {
          slot = i;
          mt = (tb - acc0) / n_nt;
          nt = (tb - acc0) % n_nt;
          break;
        }
        acc0 += tiles;
      }
    }
    const int k = a.pred[slot];
    const int cnt = a.q.counts[k];
    const int D = a.d_in[slot];
    const uint32_t* qe = a.q.entries + (int64_t)k * a.q.cap;
    unsigned long long t0 = wall_clock64();

    const int row = mt * BM + ar;
    const uint32_t idx = entry_idx(qe[row < cnt ? row : cnt - 1]);
    const T* wrow;
    if constexpr (sizeof(T) == 2) wrow = reinterpret_cast<const T*>(a.w1_bf[slot]) + (int64_t)(nt * BN + br) * D;
    else wrow = reinterpret_cast<const T*>(a.w1_f32[slot]) + (int64_t)(nt * BN + br) * D;

    floatx4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};

    // NS register stages: the global loads of k-tile kt + NS - 1 are issued while tile kt is
    // computed (two stages measured fastest: deeper staging costs more than it hides here).
    constexpr int NS = 2;
    alignas(16) T ra[NS][PA];
    alignas(16) T rb[NS][PB];
    auto gload = [&](int kt, int st) {
      load_frame_run<T, In, PA>(a.fr, idx, (int64_t)kt * BK + ak, ra[st]);
      const uint4* pb = reinterpret_cast<const uint4*>(wrow + (int64_t)kt * BK + bk);
#pragma unroll
      for (int v = 0; v < PB * (int)sizeof(T) / 16; ++v) reinterpret_cast<uint4*>(rb[st])[v] = pb[v];
    };
    auto lstore = [&](int st, int buf) {
#pragma unroll
      for (int v = 0; v < PA * (int)sizeof(T) / 16; ++v)
        reinterpret_cast<uint4*>(&As[buf][ar * LD + ak])[v] = reinterpret_cast<uint4*>(ra[st])[v];
#pragma unroll
      for (int v = 0; v < PB * (int)sizeof(T) / 16; ++v)
        reinterpret_cast<uint4*>(&Bs[buf][br * LD + bk])[v] = reinterpret_cast<uint4*>(rb[st])[v];
    };
    auto compute = [&](int buf) {
      if constexpr (sizeof(T) == 2) {
        bf16x8 af[FM], bfr[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          af[i] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm * WM + i * 16 + (lane & 15)) * LD + 8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn * WN + j * 16 + (lane & 15)) * LD + 8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      } else {
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
          float af[FM], bfr[FN];
#pragma unroll
          for (int i = 0; i < FM; ++i) af[i] = As[buf][(wm * WM + i * 16 + (lane & 15)) * LD + ks * 4 + (lane >> 4)];
#pragma unroll
          for (int j = 0; j < FN; ++j) bfr[j] = Bs[buf][(wn * WN + j * 16 + (lane & 15)) * LD + ks * 4 + (lane >> 4)];
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
      }
    };

    const int nk_all = D / BK;
    const int kt0 = (int)((int64_t)nk_all * sp / S), nk = (int)((int64_t)nk_all * (sp + 1) / S);
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
      if (kt0 + u < nk) gload(kt0 + u, u);
    lstore(0, kt0 & 1);
    __syncthreads();
    // k-tile kt = kb + u lives in register stage u (kb - kt0 is a multiple of NS)
    for (int kb = kt0; kb < nk; kb += NS) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int kt = kb + u;
        if (kt < nk) {
          const int buf = kt & 1;
          if (kt + NS - 1 < nk) gload(kt + NS - 1, (u + NS - 1) % NS);
          compute(buf);
          if (kt + 1 < nk) {
            __syncthreads();
            lstore((u + 1) % NS, buf ^ 1);
            __syncthreads();
          }
        }
      }
    }

    if (S > 1) {
      // raw sums of this K range: ws[tb][sp][column in tile][row in tile], each lane's four
      // consecutive rows in one 16-byte store
      float* wt = a.splitk_ws + (int64_t)tb * S * (BM * BN);
      auto at = [&](int q, int i, int j) -> float4* {
        return reinterpret_cast<float4*>(
            &wt[(int64_t)q * (BM * BN) + (wn * WN + j * 16 + (lane & 15)) * BM + wm * WM + i * 16 + 4 * (lane >> 4)]);
      };
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) *at(sp, i, j) = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
      __threadfence();
      __syncthreads();
      if (tid == 0) s_last = atomicAdd(&a.split_cnt[tb], 1) == S - 1;
      __syncthreads();
      if (!s_last) {
        if (tid == 0 && a.count_ticks) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - t0));
        continue;
      }
      __threadfence();
      if (tid == 0) a.split_cnt[tb] = 0;      // ready for the next launch
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          floatx4 sum = (floatx4){0.f, 0.f, 0.f, 0.f};
          for (int q = 0; q < S; ++q) {
            float4 v;
            if (q == sp) v = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
            else v = *at(q, i, j);
            sum[0] += v.x; sum[1] += v.y; sum[2] += v.z; sum[3] += v.w;
          }
          acc[i][j] = sum;
        }
    }
    // epilogue: H = ReLU(acc + b1'), partial logits over this wave's WN hidden columns
    const float* b1 = a.b1_fold[slot];
    const float* w2 = a.w2[slot];
    const int col0 = nt * BN + wn * WN + (lane & 15);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const float bb = b1[col0 + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = fmaxf(acc[i][j][r] + bb, 0.f);
    }
    float* part = a.partial[slot] + ((int64_t)(nt * 2 + wn) * a.part_cap) * kClasses;
    for (int c = 0; c < kClasses; ++c) {
      float w2v[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) w2v[j] = w2[(col0 + j * 16) * kClasses + c];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < FN; ++j) s += acc[i][j][r] * w2v[j];
          s = row_sum16(s);
          const int rr = mt * BM + wm * WM + i * 16 + 4 * (lane >> 4) + r;
          if ((lane & 15) == 0 && rr < cnt) part[(int64_t)rr * kClasses + c] = s;
        }
    }
    __syncthreads();
    if (tid == 0 && a.count_ticks) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - t0));
  }
}

// Head: z = b2 + sum of partial logits; margin; decision / deferral; forwarding.
__global__ __launch_bounds__(256) void mlp_head_kernel(MlpArgs a, Forward f) {
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += a.q.counts[a.pred[i]];
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < total; base += stride) {
    int g = base + threadIdx.x;
    bool active = g < total;
    // find predicate slot (uniform work per lane; K <= 8)
    int slot = 0, off = g;
    for (int i = 0; i < a.n_preds; ++i) {
      int c = a.q.counts[a.pred[i]];
      if (off < c || i == a.n_preds - 1) { slot = i; break; }
      off -= c;
    }
    int k = a.pred[slot];
    uint32_t e = 0;
    bool pass = false, defer = false;
    if (active) {
      e = a.q.entries[(int64_t)k * a.q.cap + off];
      float z[kClasses];
      const float* b2 = a.b2[slot];
#pragma unroll
      for (int c = 0; c < kClasses; ++c) z[c] = b2[c];
      const int parts = a.hidden[slot] / a.part_w[slot];
      const float* part = a.partial[slot];
      for (int p = 0; p < parts; ++p) {
        const float* pp = part + ((int64_t)p * a.part_cap + off) * kClasses;
#pragma unroll
        for (int c = 0; c < kClasses; ++c) z[c] += pp[c];
      }
      if (f.logits != nullptr) {
        for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)entry_idx(e) * kClasses + c] = (double)z[c];
        continue;
      }
      float d = class_margin(z, a.class_mask[slot]);
      float th = theta_of(f, k, entry_idx(e));
      float gap = d - th;
      defer = f.defer.entries != nullptr && fabsf(gap) < f.tau[k];
      pass = d > th;
    }
    if (f.logits != nullptr) continue;
    // all lanes of every wave reach this point; k differs per lane only at predicate seams,
    // so forward per distinct k present in the wave
    for (int i = 0; i < a.n_preds; ++i) {
      int kk = a.pred[i];
      if (__ballot(active && k == kk) == 0) continue;
      forward_decision(f, kk, e, active && k == kk, defer, pass);
    }
  }
}

// FP64 tier: frames normalised in fp64 exactly as defined; canonical fp32 weights widened to
// fp64.  The first esc_cap escalated entries of each predicate are evaluated across many
// workgroups: work item = (predicate, group of 8 entries, 256 hidden units, 256-long chunk of
// the input) -> partial hidden sums; a head (one wave per entry) adds the chunks, applies
// ReLU, GEMM2, the margin and the decision.  Entries beyond esc_cap run one group per block.
constexpr int F64_B = 8;
constexpr int F64_DCH = 256;
int mlp_f64_chunks(int d_in) { return (d_in + F64_DCH - 1) / F64_DCH; }

__device__ inline double frame_norm64_flat(const FrameSrc& fr, uint32_t idx, int64_t d) {
  const int64_t o = (int64_t)idx * fr.elems + d;
  double x;
  if (fr.dtype == HYDRO_DTYPE_BF16) x = (double)(float)static_cast<const __bf16*>(fr.base)[o];
  else if (fr.dtype == HYDRO_DTYPE_U8) x = (double)static_cast<const uint8_t*>(fr.base)[o] / 255.0;
  else x = (double)static_cast<const float*>(fr.base)[o];
  return (x - 0.5) * 4.0;
}

__global__ __launch_bounds__(256) void mlp_f64_hidden_kernel(MlpArgs a) {
  __shared__ double xs[F64_B][256];
  __shared__ uint32_t ents[F64_B];
  const int tid = threadIdx.x;
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) {
    const int ne = min(a.q.counts[a.pred[i]], a.esc_cap);
    total += (ne + F64_B - 1) / F64_B * (a.hidden[i] / 256 + (a.hidden[i] % 256 ? 1 : 0)) *
             ((a.d_in[i] + F64_DCH - 1) / F64_DCH);
  }
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int ne = min(a.q.counts[a.pred[i]], a.esc_cap);
      const int c = (ne + F64_B - 1) / F64_B * (a.hidden[i] / 256 + (a.hidden[i] % 256 ? 1 : 0)) *
                    ((a.d_in[i] + F64_DCH - 1) / F64_DCH);
      if (off < c) { slot = i; break; }
      off -= c;
    }
    const int k = a.pred[slot];
    const int D = a.d_in[slot], H = a.hidden[slot];
    const int ne = min(a.q.counts[k], a.esc_cap);
    const int nch = (D + F64_DCH - 1) / F64_DCH;
    const int nhb = H / 256 + (H % 256 ? 1 : 0);
    const int ch = off % nch;
    const int hb = (off / nch) % nhb;
    const int grp = off / (nch * nhb);
    const int nb = min(F64_B, ne - grp * F64_B);
    if (tid < F64_B) ents[tid] = tid < nb ? a.q.entries[(int64_t)k * a.q.cap + grp * F64_B + tid] : 0u;
    __syncthreads();
    const int j = hb * 256 + tid;
    double s[F64_B];
#pragma unroll
    for (int b = 0; b < F64_B; ++b) s[b] = 0.0;
    const float* W1 = a.w1_canon[slot];
    const int d_lo = ch * F64_DCH, d_hi = min(D, d_lo + F64_DCH);
    for (int d0 = d_lo; d0 < d_hi; d0 += 256) {
      const int dl = min(256, d_hi - d0);
      for (int q = tid; q < F64_B * 256; q += 256) {
        const int b = q >> 8, dd = q & 255;
        xs[b][dd] = (b < nb && dd < dl) ? frame_norm64_flat(a.fr, entry_idx(ents[b]), d0 + dd) : 0.0;
      }
      __syncthreads();
      if (j < H) {
#pragma unroll 16
        for (int dd = 0; dd < dl; ++dd) {
          const double w = (double)W1[(int64_t)(d0 + dd) * H + j];
#pragma unroll
          for (int b = 0; b < F64_B; ++b) s[b] = fma(w, xs[b][dd], s[b]);
        }
      }
      __syncthreads();
    }
    if (j < H) {
      double* hp = a.esc_h[slot] + ((int64_t)ch * a.esc_cap) * H;
      for (int b = 0; b < nb; ++b) hp[(int64_t)(grp * F64_B + b) * H + j] = s[b];
    }
    __syncthreads();
  }
}

__device__ inline void mlp_head64(const MlpArgs& a, const Forward& f, int slot, uint32_t e, int ei, bool active) {
  const int lane = threadIdx.x & 63;
  const int k = a.pred[slot];
  const int D = a.d_in[slot], H = a.hidden[slot];
  const int nch = (D + F64_DCH - 1) / F64_DCH;
  double zp[kClasses];
#pragma unroll
  for (int c = 0; c < kClasses; ++c) zp[c] = 0.0;
  if (active) {
    const float* b1 = a.b1_canon[slot];
    const float* w2 = a.w2[slot];
    for (int j = lane; j < H; j += 64) {
      double h = (double)b1[j];
      for (int c = 0; c < nch; ++c) h += a.esc_h[slot][((int64_t)c * a.esc_cap + ei) * H + j];
      h = h > 0.0 ? h : 0.0;
#pragma unroll
      for (int c = 0; c < kClasses; ++c) zp[c] = fma(h, (double)w2[j * kClasses + c], zp[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < kClasses; ++c)
    for (int o = 32; o >= 1; o >>= 1) zp[c] += __shfl_xor(zp[c], o);
  const uint32_t idx = entry_idx(e);
  const bool lead = active && lane == 0;
  bool pass = false;
  if (lead) {
    double z[kClasses];
    for (int c = 0; c < kClasses; ++c) z[c] = (double)a.b2[slot][c] + zp[c];
    if (f.logits != nullptr)
      for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)idx * kClasses + c] = z[c];
    pass = class_margin(z, a.class_mask[slot]) > (double)theta_of(f, k, idx);
  }
  if (f.logits == nullptr) forward_decision(f, k, e, lead, false, pass);
}

__global__ __launch_bounds__(256) void mlp_f64_head_kernel(MlpArgs a, Forward f) {
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += min(a.q.counts[a.pred[i]], a.esc_cap);
  const int wave = threadIdx.x >> 6;
  for (int base = blockIdx.x * 4; base < total; base += gridDim.x * 4) {
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
    mlp_head64(a, f, slot, e, off, active);
  }
}

// Entries beyond esc_cap: groups of 4 per block, the whole input and hidden width in one block.
constexpr int R64_B = 4;
constexpr int R64_DCH = 256;

__global__ __launch_bounds__(256) void mlp_f64_rest_kernel(MlpArgs a, Forward f) {
  __shared__ double xs[R64_B][R64_DCH];
  __shared__ double zred[4][R64_B][kClasses];
  __shared__ uint32_t ents[R64_B];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += (max(0, a.q.counts[a.pred[i]] - a.esc_cap) + R64_B - 1) / R64_B;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = (max(0, a.q.counts[a.pred[i]] - a.esc_cap) + R64_B - 1) / R64_B;
      if (off < c) { slot = i; break; }
      off -= c;
    }
    const int k = a.pred[slot];
    const int rest = a.q.counts[k] - a.esc_cap;
    const int D = a.d_in[slot], H = a.hidden[slot];
    const int nb = min(R64_B, rest - off * R64_B);
    if (tid < R64_B) ents[tid] = tid < nb ? a.q.entries[(int64_t)k * a.q.cap + a.esc_cap + off * R64_B + tid] : 0u;
    __syncthreads();
    constexpr int JMAX = 8;            // hidden units per thread (H <= 2048)
    double s[JMAX][R64_B];
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
#pragma unroll
      for (int b = 0; b < R64_B; ++b) s[j][b] = 0.0;
    const float* W1 = a.w1_canon[slot];
    for (int d0 = 0; d0 < D; d0 += R64_DCH) {
      for (int q = tid; q < R64_B * R64_DCH; q += blockDim.x) {
        const int b = q / R64_DCH, dd = q % R64_DCH;
        xs[b][dd] = (b < nb && d0 + dd < D) ? frame_norm64_flat(a.fr, entry_idx(ents[b]), d0 + dd) : 0.0;
      }
      __syncthreads();
      const int dlim = min(R64_DCH, D - d0);
      for (int dd = 0; dd < dlim; ++dd) {
        const float* wr = W1 + (int64_t)(d0 + dd) * H;
#pragma unroll
        for (int j = 0; j < JMAX; ++j) {
          const int col = tid + j * 256;
          if (col < H) {
            const double w = (double)wr[col];
#pragma unroll
            for (int b = 0; b < R64_B; ++b) s[j][b] = fma(w, xs[b][dd], s[j][b]);
          }
        }
      }
      __syncthreads();
    }
    double zp[R64_B][kClasses];
#pragma unroll
    for (int b = 0; b < R64_B; ++b)
#pragma unroll
      for (int c = 0; c < kClasses; ++c) zp[b][c] = 0.0;
    const float* b1 = a.b1_canon[slot];
    const float* w2 = a.w2[slot];
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      const int col = tid + j * 256;
      if (col < H) {
        const double bb = (double)b1[col];
#pragma unroll
        for (int b = 0; b < R64_B; ++b) {
          double h = s[j][b] + bb;
          h = h > 0.0 ? h : 0.0;
#pragma unroll
          for (int c = 0; c < kClasses; ++c) zp[b][c] = fma(h, (double)w2[col * kClasses + c], zp[b][c]);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < R64_B; ++b)
#pragma unroll
      for (int c = 0; c < kClasses; ++c) {
        double v = zp[b][c];
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) zred[wave][b][c] = v;
      }
    __syncthreads();
    if (wave == 0) {
      const bool active = lane < nb;
      bool pass = false;
      const uint32_t e = active ? ents[lane] : 0u;
      if (active) {
        double z[kClasses];
        const float* b2 = a.b2[slot];
        for (int c = 0; c < kClasses; ++c)
          z[c] = (double)b2[c] + ((zred[0][lane][c] + zred[1][lane][c]) + (zred[2][lane][c] + zred[3][lane][c]));
        if (f.logits != nullptr)
          for (int c = 0; c < kClasses; ++c) f.logits[(int64_t)entry_idx(e) * kClasses + c] = z[c];
        pass = class_margin(z, a.class_mask[slot]) > (double)theta_of(f, k, entry_idx(e));
      }
      if (f.logits == nullptr) forward_decision(f, k, e, active, false, pass);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers
// Tile configurations: 0 = 128x128, 1 = 64x128, 2 = 128x64, 3 = 64x64 (rows x hidden units).
int mlp_tile_bn(int cfg) { return cfg == 0 || cfg == 1 ? 128 : 64; }

// BF16 first pass on bf16 frames (d_in a multiple of 64): 256 queued rows x 128 hidden units per
// tile, eight waves of 64 x 64.  Each k-block (64 elements: 128 bytes of every frame row and
// weight row) is copied global -> LDS with global_load_lds_dwordx4 into a three-stage ring, one
// barrier per k-block; the 16-byte chunks of row r sit at slot chunk ^ (r mod 8), so the MFMA
// operand reads of 16 rows spread over the banks.  Split-K and the epilogue as in
// mlp_gemm_kernel (workspace tiles of 256 x 128: the launch passes half the 128 x 128 slots).
constexpr int MD_BM = 256, MD_BN = 128, MD_NS = 3;
__global__ __launch_bounds__(512) void mlp_gemm_dma_kernel(MlpArgs a) {
  constexpr int UPR = 8, ROWB = 128, BKE = 64;             // 16-byte units per row, bytes, elements
  constexpr int UNITS = (MD_BM + MD_BN) * UPR;
  constexpr int NI = UNITS / 512, NIF = MD_BM * UPR / 512; // loads per wave and stage (frames first)
  constexpr int STAGE = UNITS * 16;
  constexpr int WM = 64, WN = 64, MT = WM / 16, NT = WN / 16;
  static_assert(UNITS % 512 == 0 && (MD_BM * UPR) % 512 == 0, "stage rows fill the waves' loads");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[MD_NS * STAGE];
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave & 3, wn = wave >> 2;
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)lds);
  const int u_slot = lane % UPR;

  int base_total = 0, nk_min = 1 << 30;
  for (int i = 0; i < a.n_preds; ++i) {
    const int cnt = a.q.counts[a.pred[i]];
    base_total += ((cnt + MD_BM - 1) / MD_BM) * (a.hidden[i] / MD_BN);
    nk_min = min(nk_min, a.d_in[i] / BKE);
  }
  const int S = mlp_splits(base_total, nk_min, a);
  const int total = base_total * S;

  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int tb = t / S, sp = t % S;
    int slot = 0, mt = 0, nt = 0;
    {
      int acc0 = 0;
      for (int i = 0; i < a.n_preds; ++i) {
        const int cnt = a.q.counts[a.pred[i]];
        const int n_nt = a.hidden[i] / MD_BN;
        const int tiles = ((cnt + MD_BM - 1) / MD_BM) * n_nt;
        if (tb < acc0 + tiles) {
          slot = i;
          mt = (tb - acc0) / n_nt;
          nt = (tb - acc0) % n_nt;
          break;
        }
        acc0 += tiles;
      }
    }
    const int k = a.pred[slot];
    const int cnt = a.q.counts[k];
    const int D = a.d_in[slot];
    const uint32_t* qe = a.q.entries + (int64_t)k * a.q.cap;
    const unsigned long long t0 = wall_clock64();

    // the rows this lane copies: gathered frame rows (rows past the queue re-read its last entry;
    // their results are never stored), then weight rows; element offset of the lane's chunk
    const __bf16* src[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int U = (wave + 8 * i) * 64 + lane;
      if (i < NIF) {
        const int r = U / UPR;
        const int row = mt * MD_BM + r;
        const uint32_t idx = entry_idx(qe[row < cnt ? row : cnt - 1]);
        src[i] = static_cast<const __bf16*>(a.fr.base) + (int64_t)idx * a.fr.elems + (u_slot ^ (r & 7)) * 8;
      } else {
        const int r = U / UPR - MD_BM;
        src[i] = a.w1_bf[slot] + (int64_t)(nt * MD_BN + r) * D + (u_slot ^ (r & 7)) * 8;
      }
    }
    auto issue = [&](int kb, int buf) {
      const uint32_t base = lds0 + buf * STAGE;
#pragma unroll
      for (int i = 0; i < NI; ++i)
        lds_dma16(src[i] + (int64_t)kb * BKE, __builtin_amdgcn_readfirstlane(base + (wave + 8 * i) * 1024));
    };

    floatx4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
    // k-step ks (chunk 4 ks + g of each row) of buffer buf, read into registers
    struct Frag { bf16x8 a[MT], b[NT]; };
    auto frags = [&](int buf, int ks, Frag& fr) {
      const unsigned char* F = lds + buf * STAGE;
      const unsigned char* W = F + MD_BM * ROWB;
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const int r = wm * WM + i * 16 + l16;
        fr.a[i] = *reinterpret_cast<const bf16x8*>(F + (r * UPR + ((4 * ks + g) ^ (r & 7))) * 16);
      }
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int r = wn * WN + j * 16 + l16;
        fr.b[j] = *reinterpret_cast<const bf16x8*>(W + (r * UPR + ((4 * ks + g) ^ (r & 7))) * 16);
      }
    };
    auto mma = [&](const Frag& fr) {
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.a[i], fr.b[j], acc[i][j], 0, 0, 0);
    };

    const int nk_all = D / BKE;
    const int kt0 = (int)((int64_t)nk_all * sp / S), kt1 = (int)((int64_t)nk_all * (sp + 1) / S);
    const int nkb = kt1 - kt0;
    // Ring of MD_NS k-blocks (k-block kb in buffer kb % MD_NS).  Fragments are read one MFMA step
    // ahead, and the barrier that publishes k-block kb + 1 and frees buffer kb sits between a
    // k-block's two steps: every wave reaches it with MFMAs in its pipe.  (The previous tile's last
    // barrier ordered every read of the ring.)
#pragma unroll
    for (int s0 = 0; s0 < MD_NS; ++s0)
      if (s0 < nkb) issue(kt0 + s0, s0);
    if (nkb >= 3) wait_vmcnt<2 * NI>();
    else if (nkb == 2) wait_vmcnt<NI>();
    else wait_vmcnt<0>();
    __syncthreads();
    Frag F0, F1;
    frags(0, 0, F0);
    int buf = 0;
#pragma unroll 1
    for (int kb = 0; kb < nkb; ++kb) {
      frags(buf, 1, F1);
      mma(F0);
      if (kb + 2 < nkb) wait_vmcnt<NI>();   // k-block kb + 1 landed; kb + 2 may stay in flight
      else wait_vmcnt<0>();
      __syncthreads();
      if (kb + MD_NS < nkb) issue(kt0 + kb + MD_NS, buf);
      buf = buf + 1 == MD_NS ? 0 : buf + 1;
      frags(buf, 0, F0);                     // the next k-block's first step (unused after the last)
      mma(F1);
    }

    if (S > 1) {
      // raw sums of this K range: ws[tb][sp][column in tile][row in tile]
      float* wt = a.splitk_ws + (int64_t)tb * S * (MD_BM * MD_BN);
      auto at = [&](int q, int i, int j) -> float4* {
        return reinterpret_cast<float4*>(
            &wt[(int64_t)q * (MD_BM * MD_BN) + (wn * WN + j * 16 + l16) * MD_BM + wm * WM + i * 16 + 4 * g]);
      };
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) *at(sp, i, j) = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
      __threadfence();
      __syncthreads();
      if (tid == 0) s_last = atomicAdd(&a.split_cnt[tb], 1) == S - 1;
      __syncthreads();
      if (!s_last) {
        if (tid == 0 && a.count_ticks) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - t0));
        continue;
      }
      __threadfence();
      if (tid == 0) a.split_cnt[tb] = 0;      // ready for the next launch
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          floatx4 sum = (floatx4){0.f, 0.f, 0.f, 0.f};
          for (int q = 0; q < S; ++q) {
            float4 v;
            if (q == sp) v = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
            else v = *at(q, i, j);
            sum[0] += v.x; sum[1] += v.y; sum[2] += v.z; sum[3] += v.w;
          }
          acc[i][j] = sum;
        }
    }
    // epilogue: H = ReLU(acc + b1'), partial logits over this wave's 64 hidden columns
    const float* b1 = a.b1_fold[slot];
    const float* w2 = a.w2[slot];
    const int col0 = nt * MD_BN + wn * WN + l16;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const float bb = b1[col0 + j * 16];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = fmaxf(acc[i][j][r] + bb, 0.f);
    }
    float* part = a.partial[slot] + ((int64_t)(nt * 2 + wn) * a.part_cap) * kClasses;
    for (int c = 0; c < kClasses; ++c) {
      float w2v[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) w2v[j] = w2[(col0 + j * 16) * kClasses + c];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float sacc = 0.f;
#pragma unroll
          for (int j = 0; j < NT; ++j) sacc += acc[i][j][r] * w2v[j];
          sacc = row_sum16(sacc);
          const int rr = mt * MD_BM + wm * WM + i * 16 + 4 * g + r;
          if (l16 == 0 && rr < cnt) part[(int64_t)rr * kClasses + c] = sacc;
        }
    }
    __syncthreads();
    if (tid == 0 && a.count_ticks) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - t0));
  }
}

// FP32 arithmetic on bf16 frames (the FP32 tier, and an FP32 first pass): every fp32 weight w is
// split into three bf16 terms w = hi + mid + lo (each the bf16 rounding of what is left; three
// terms carry all 24 bits of the fp32 significand), so x * w = x * hi + x * mid + x * lo with
// every product exact (a bf16 x bf16 product fits fp32) and fp32 accumulation: the fp32 GEMM's
// result up to summation order, from three bf16 MFMAs instead of eight fp32 ones (16x16x32 bf16
// against 16x16x4 fp32).  128 x 128 tiles, four waves of 64 x 64, k-blocks of 64 elements (the
// frame rows, then the hi, mid and lo weight rows) in a two-stage direct-to-LDS ring.
constexpr int M3_BM = 128, M3_BN = 128, M3_NS = 2;
__global__ __launch_bounds__(256) void mlp_gemm_s3_kernel(MlpArgs a) {
  constexpr int UPR = 8, ROWB = 128, BKE = 64;
  constexpr int UNITS = (M3_BM + 3 * M3_BN) * UPR;
  constexpr int NI = UNITS / 256, NIF = M3_BM * UPR / 256;   // loads per wave and stage (frames first)
  constexpr int STAGE = UNITS * 16;
  constexpr int WM = 64, WN = 64, MT = WM / 16, NT = WN / 16;
  static_assert(UNITS % 256 == 0 && (M3_BM * UPR) % 256 == 0, "stage rows fill the waves' loads");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[M3_NS * STAGE];
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)lds);
  const int u_slot = lane % UPR;

  int base_total = 0, nk_min = 1 << 30;
  for (int i = 0; i < a.n_preds; ++i) {
    const int cnt = a.q.counts[a.pred[i]];
    base_total += ((cnt + M3_BM - 1) / M3_BM) * (a.hidden[i] / M3_BN);
    nk_min = min(nk_min, a.d_in[i] / BKE);
  }
  const int S = mlp_splits(base_total, nk_min, a);
  const int total = base_total * S;

  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int tb = t / S, sp = t % S;
    int slot = 0, mt = 0, nt = 0;
    {
      int acc0 = 0;
      for (int i = 0; i < a.n_preds; ++i) {
        const int cnt = a.q.counts[a.pred[i]];
        const int n_nt = a.hidden[i] / M3_BN;
        const int tiles = ((cnt + M3_BM - 1) / M3_BM) * n_nt;
        if (tb < acc0 + tiles) {
          slot = i;
          mt = (tb - acc0) / n_nt;
          nt = (tb - acc0) % n_nt;
          break;
        }
        acc0 += tiles;
      }
    }
    const int k = a.pred[slot];
    const int cnt = a.q.counts[k];
    const int D = a.d_in[slot], H = a.hidden[slot];
    const uint32_t* qe = a.q.entries + (int64_t)k * a.q.cap;
    const unsigned long long t0 = wall_clock64();

    const __bf16* src[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int U = (wave + 4 * i) * 64 + lane;
      if (i < NIF) {
        const int r = U / UPR;
        const int row = mt * M3_BM + r;
        const uint32_t idx = entry_idx(qe[row < cnt ? row : cnt - 1]);
        src[i] = static_cast<const __bf16*>(a.fr.base) + (int64_t)idx * a.fr.elems + (u_slot ^ (r & 7)) * 8;
      } else {
        const int r = U / UPR - M3_BM;                   // 0 .. 3 * BN - 1: term r / BN, row r % BN
        const int term = r / M3_BN, rr = r % M3_BN;
        src[i] = a.w1_s3[slot] + ((int64_t)term * H + nt * M3_BN + rr) * D + (u_slot ^ (rr & 7)) * 8;
      }
    }
    auto issue = [&](int kb, int buf) {
      const uint32_t base = lds0 + buf * STAGE;
#pragma unroll
      for (int i = 0; i < NI; ++i)
        lds_dma16(src[i] + (int64_t)kb * BKE, __builtin_amdgcn_readfirstlane(base + (wave + 4 * i) * 1024));
    };

    floatx4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
    auto compute = [&](int buf) {
      const unsigned char* F = lds + buf * STAGE;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        bf16x8 af[MT];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          const int r = wm * WM + i * 16 + l16;
          af[i] = *reinterpret_cast<const bf16x8*>(F + (r * UPR + ((4 * ks + g) ^ (r & 7))) * 16);
        }
        // smallest terms first: the three partial products enter each sum in the order lo, mid, hi
#pragma unroll
        for (int term = 2; term >= 0; --term) {
          const unsigned char* W = F + (M3_BM + term * M3_BN) * ROWB;
          bf16x8 bfr[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int r = wn * WN + j * 16 + l16;
            bfr[j] = *reinterpret_cast<const bf16x8*>(W + (r * UPR + ((4 * ks + g) ^ (r & 7))) * 16);
          }
#pragma unroll
          for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
      }
    };

    const int nk_all = D / BKE;
    const int kt0 = (int)((int64_t)nk_all * sp / S), kt1 = (int)((int64_t)nk_all * (sp + 1) / S);
    const int nkb = kt1 - kt0;
    // two stages: block kb + 1 is copied while block kb is read; the barrier at the top of each
    // iteration also retires every wave's reads of the buffer the next copy overwrites
    if (nkb > 0) issue(kt0, 0);
#pragma unroll 1
    for (int kb = 0; kb < nkb; ++kb) {
      wait_vmcnt<0>();
      __syncthreads();
      if (kb + 1 < nkb) issue(kt0 + kb + 1, (kb + 1) & 1);
      compute(kb & 1);
    }

    if (S > 1) {
      float* wt = a.splitk_ws + (int64_t)tb * S * (M3_BM * M3_BN);
      auto at = [&](int q, int i, int j) -> float4* {
        return reinterpret_cast<float4*>(
            &wt[(int64_t)q * (M3_BM * M3_BN) + (wn * WN + j * 16 + l16) * M3_BM + wm * WM + i * 16 + 4 * g]);
      };
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) *at(sp, i, j) = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
      __threadfence();
      __syncthreads();
      if (tid == 0) s_last = atomicAdd(&a.split_cnt[tb], 1) == S - 1;
      __syncthreads();
      if (!s_last) {
        if (tid == 0 && a.count_ticks) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - t0));
        continue;
      }
      __threadfence();
      if (tid == 0) a.split_cnt[tb] = 0;
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          floatx4 sum = (floatx4){0.f, 0.f, 0.f, 0.f};
          for (int q = 0; q < S; ++q) {
            float4 v;
            if (q == sp) v = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
            else v = *at(q, i, j);
            sum[0] += v.x; sum[1] += v.y; sum[2] += v.z; sum[3] += v.w;
          }
          acc[i][j] = sum;
        }
    }
    const float* b1 = a.b1_fold[slot];
    const float* w2 = a.w2[slot];
    const int col0 = nt * M3_BN + wn * WN + l16;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const float bb = b1[col0 + j * 16];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = fmaxf(acc[i][j][r] + bb, 0.f);
    }
    float* part = a.partial[slot] + ((int64_t)(nt * 2 + wn) * a.part_cap) * kClasses;
    for (int c = 0; c < kClasses; ++c) {
      float w2v[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) w2v[j] = w2[(col0 + j * 16) * kClasses + c];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float sacc = 0.f;
#pragma unroll
          for (int j = 0; j < NT; ++j) sacc += acc[i][j][r] * w2v[j];
          sacc = row_sum16(sacc);
          const int rr = mt * M3_BM + wm * WM + i * 16 + 4 * g + r;
          if (l16 == 0 && rr < cnt) part[(int64_t)rr * kClasses + c] = sacc;
        }
    }
    __syncthreads();
    if (tid == 0 && a.count_ticks) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - t0));
  }
}

template <typename T, int BM, int BN>
static void launch_gemm_t(const MlpArgs& b, int grid, hipStream_t s) {
  if (b.fr.dtype == HYDRO_DTYPE_BF16)
    hipLaunchKernelGGL((mlp_gemm_kernel<T, __bf16, BM, BN>), dim3(grid), dim3(256), 0, s, b);
  else if (b.fr.dtype == HYDRO_DTYPE_U8)
    hipLaunchKernelGGL((mlp_gemm_kernel<T, uint8_t, BM, BN>), dim3(grid), dim3(256), 0, s, b);
  else
    hipLaunchKernelGGL((mlp_gemm_kernel<T, float, BM, BN>), dim3(grid), dim3(256), 0, s, b);
}

void launch_mlp_gemm(const MlpArgs& b, int cfg, bool bf, int grid, hipStream_t s) {
  bool dma = bf && b.fr.dtype == HYDRO_DTYPE_BF16 && (cfg == 0 || cfg == 1);
  for (int i = 0; i < b.n_preds && dma; ++i) dma = b.d_in[i] % 64 == 0 && b.hidden[i] % MD_BN == 0;
  bool s3 = !bf && b.fr.dtype == HYDRO_DTYPE_BF16 && (cfg == 0 || cfg == 1);
  for (int i = 0; i < b.n_preds && s3; ++i) s3 = b.w1_s3[i] != nullptr;
  if (s3) {
    hipLaunchKernelGGL(mlp_gemm_s3_kernel, dim3(grid), dim3(256), 0, s, b);
  } else if (dma) {
    MlpArgs c = b;
    c.split_slots = b.split_slots / 2;     // workspace tiles of 256 x 128
    hipLaunchKernelGGL(mlp_gemm_dma_kernel, dim3(grid), dim3(512), 0, s, c);
  } else if (bf) {
    if (cfg == 0) launch_gemm_t<__bf16, 128, 128>(b, grid, s);
    else if (cfg == 1) launch_gemm_t<__bf16, 64, 128>(b, grid, s);
    else if (cfg == 2) launch_gemm_t<__bf16, 128, 64>(b, grid, s);
    else launch_gemm_t<__bf16, 64, 64>(b, grid, s);
  } else {
    if (cfg == 0) launch_gemm_t<float, 128, 128>(b, grid, s);
    else if (cfg == 1) launch_gemm_t<float, 64, 128>(b, grid, s);
    else if (cfg == 2) launch_gemm_t<float, 128, 64>(b, grid, s);
    else launch_gemm_t<float, 64, 64>(b, grid, s);
  }
}

void mlp_copy_slot(MlpArgs& dst, int j, const MlpArgs& src, int i) {
  dst.pred[j] = src.pred[i];
  dst.d_in[j] = src.d_in[i];
  dst.hidden[j] = src.hidden[i];
  dst.class_mask[j] = src.class_mask[i];
  dst.w1_bf[j] = src.w1_bf[i];
  dst.w1_f32[j] = src.w1_f32[i];
  dst.w1_s3[j] = src.w1_s3[i];
  dst.b1_fold[j] = src.b1_fold[i];
  dst.w2[j] = src.w2[i];
  dst.b2[j] = src.b2[i];
  dst.w1_canon[j] = src.w1_canon[i];
  dst.b1_canon[j] = src.b1_canon[i];
  dst.partial[j] = src.partial[i];
  dst.part_w[j] = src.part_w[i];
  dst.tile_cfg[j] = src.tile_cfg[i];
  dst.esc_h[j] = src.esc_h[i];
}

void launch_mlp_pass(const MlpArgs& a, const Forward& f, int tier, int grid, hipStream_t s) {
  if (a.n_preds == 0) return;
  if (tier == TIER_F64) {
    hipLaunchKernelGGL(mlp_f64_hidden_kernel, dim3(grid * 2), dim3(256), 0, s, a);
    hipLaunchKernelGGL(mlp_f64_head_kernel, dim3(grid), dim3(256), 0, s, a, f);
    hipLaunchKernelGGL(mlp_f64_rest_kernel, dim3(grid), dim3(256), 0, s, a, f);
    return;
  }
  // one GEMM launch per tile shape present among the predicates
  const bool bf = a.prec == HYDRO_PREC_BF16 && tier == TIER_FIRST;
  for (int cfg = 0; cfg < MLP_TILE_CONFIGS; ++cfg) {
    MlpArgs b = a;
    b.n_preds = 0;
    for (int i = 0; i < a.n_preds; ++i) {
      if (a.tile_cfg[i] != cfg) continue;
      mlp_copy_slot(b, b.n_preds++, a, i);
    }
    if (b.n_preds == 0) continue;
    launch_mlp_gemm(b, cfg, bf, grid, s);
  }
  hipLaunchKernelGGL(mlp_head_kernel, dim3(grid), dim3(256), 0, s, a, f);
}

}  // namespace hydro
