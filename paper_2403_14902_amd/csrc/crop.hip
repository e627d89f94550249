// CNN predicates on variable-size inputs: each tuple's crop (y0, x0, h, w) of its frame (the UDF
// composition of section 5.3, a classifier applied to Crop(frame, bbox)).  Evaluated in FP64 (the
// decisions are final), one workgroup per tuple, so the work of a tuple follows its crop's area.
// How a round's tuples are dealt to the workgroups is the data-aware load balancing of section
// 5.3: in queue order (each workgroup takes every gridDim-th tuple), or largest estimated work
// first (the crop's area, the paper's input-size heuristic) from a shared counter, so that no
// workgroup is left with a long tail of large crops.
#include "engine.h"

namespace hydro {

constexpr int kCropThreads = 256;
constexpr int kCropBuckets = 256;

// One workgroup per crop predicate slot: queue positions in decreasing order of crop area
// (bucketed: area * 255 / frame area), and the work counter of the following launch reset.
__global__ __launch_bounds__(kCropThreads) void k_crop_order(CropArgs a) {
  __shared__ int hist[kCropBuckets];
  const int slot = blockIdx.x;
  const int k = a.pred[slot];
  const int c = a.q.counts[k];
  const int64_t full = (int64_t)a.fh * a.fw;
  for (int b = threadIdx.x; b < kCropBuckets; b += kCropThreads) hist[b] = 0;
  if (slot == 0 && threadIdx.x == 0) *a.next = 0;
  __syncthreads();
  auto bucket = [&](int i) {
    const uint32_t idx = entry_idx(a.q.entries[(int64_t)k * a.q.cap + i]);
    const int64_t area = (int64_t)a.crops[idx * 4 + 2] * a.crops[idx * 4 + 3];
    return (kCropBuckets - 1) - (int)(area * (kCropBuckets - 1) / full);   // larger area, smaller bucket
  };
  for (int i = threadIdx.x; i < c; i += kCropThreads) atomicAdd(&hist[bucket(i)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int b = 0; b < kCropBuckets; ++b) {
      const int n = hist[b];
      hist[b] = run;
      run += n;
    }
  }
  __syncthreads();
  uint32_t* ord = a.order + (int64_t)slot * a.q.cap;
  for (int i = threadIdx.x; i < c; i += kCropThreads) ord[atomicAdd(&hist[bucket(i)], 1)] = (uint32_t)i;
}

// Normalised input value of the crop at (y, x) (zero padding outside the crop).
__device__ inline double crop_in(const CropArgs& a, uint32_t idx, int y0, int x0, int h, int w, int y, int x, int ch) {
  if (y < 0 || x < 0 || y >= h || x >= w) return 0.0;
  const int64_t o = (int64_t)idx * a.fr.elems + ((int64_t)(y0 + y) * a.fw + (x0 + x)) * 3 + ch;
  double v;
  if (a.fr.dtype == HYDRO_DTYPE_BF16) v = (double)(float)static_cast<const __bf16*>(a.fr.base)[o];
  else if (a.fr.dtype == HYDRO_DTYPE_U8) v = (double)static_cast<const uint8_t*>(a.fr.base)[o] / 255.0;
  else v = (double)static_cast<const float*>(a.fr.base)[o];
  return (v - 0.5) * 4.0;
}

__global__ __launch_bounds__(kCropThreads) void k_crop_cnn(CropArgs a, Forward f) {
  __shared__ double g_s[256];
  __shared__ double z_s[kClasses];
  __shared__ int item_s;
  const int tid = threadIdx.x;
  int total = 0;
  for (int i = 0; i < a.n_preds; ++i) total += a.q.counts[a.pred[i]];
  double* buf0 = a.scratch + (int64_t)blockIdx.x * 2 * a.act_doubles;
  double* buf1 = buf0 + a.act_doubles;
  for (int t0 = blockIdx.x;; t0 += gridDim.x) {
    // the next work item: the queue's t0-th (queue order) or the counter's (largest first)
    if (a.balance) {
      if (tid == 0) item_s = atomicAdd(a.next, 1);
      __syncthreads();
    }
    const int t = a.balance ? item_s : t0;
    if (a.balance) __syncthreads();          // everyone has read item_s before it changes
    if (t >= total) break;
    int slot = 0, off = t;
    for (int i = 0; i < a.n_preds; ++i) {
      const int c = a.q.counts[a.pred[i]];
      if (off < c) { slot = i; break; }
      off -= c;
    }
    const int k = a.pred[slot];
    const int pos = a.balance ? (int)a.order[(int64_t)slot * a.q.cap + off] : off;
    const uint32_t e = a.q.entries[(int64_t)k * a.q.cap + pos];
    const uint32_t idx = entry_idx(e);
    const unsigned long long c0 = wall_clock64();
    const int y0 = a.crops[idx * 4], x0 = a.crops[idx * 4 + 1];
    int hin = a.crops[idx * 4 + 2], win = a.crops[idx * 4 + 3], cin = 3;
    double* in = nullptr;
    double* out = buf0;
    for (int l = 0; l < a.n_layers[slot]; ++l) {
      const int ho = (hin + 1) / 2, wo = (win + 1) / 2, co = a.widths[slot][l];
      const float* W = a.wt[slot][l];
      const float* B = a.bias[slot][l];
      for (int o = tid; o < ho * wo * co; o += kCropThreads) {
        const int oc = o % co, p = o / co, i = p / wo, j = p % wo;
        double s = 0.0;
        for (int u = 0; u < 3; ++u)
          for (int v = 0; v < 3; ++v) {
            const int y = 2 * i + u - 1, x = 2 * j + v - 1;
            if (y < 0 || x < 0 || y >= hin || x >= win) continue;
            const float* wr = W + (int64_t)(u * 3 + v) * cin * co + oc;
            for (int ch = 0; ch < cin; ++ch) {
              const double xv = l == 0 ? crop_in(a, idx, y0, x0, hin, win, y, x, ch)
                                       : in[((int64_t)y * win + x) * cin + ch];
              s = fma((double)wr[(int64_t)ch * co], xv, s);
            }
          }
        s += (double)B[oc];
        out[o] = s > 0.0 ? s : 0.0;
      }
      __syncthreads();
      in = out;
      out = out == buf0 ? buf1 : buf0;
      hin = ho;
      win = wo;
      cin = co;
    }
    // mean over the final positions, FC, margin, decision
    for (int ch = tid; ch < cin; ch += kCropThreads) {
      double s = 0.0;
      for (int p = 0; p < hin * win; ++p) s += in[(int64_t)p * cin + ch];
      g_s[ch] = s / (double)(hin * win);
    }
    __syncthreads();
    if (tid < kClasses) {
      double z = (double)a.fc_b[slot][tid];
      for (int ch = 0; ch < cin; ++ch) z = fma(g_s[ch], (double)a.fc_w[slot][ch * kClasses + tid], z);
      z_s[tid] = z;
    }
    __syncthreads();
    if (tid < kWave) {
      const double d = class_margin(z_s, a.class_mask[slot]);
      const bool pass = d > (double)theta_of(f, k, idx);
      forward_decision(f, k, e, tid == 0, false, pass);
      if (tid == 0 && f.count_eval) atomicAdd(&a.st->r_ticks[k], (unsigned long long)(wall_clock64() - c0));
    }
    __syncthreads();          // g_s, z_s and the buffers are reused by the next item
  }
}

void launch_crop_pass(const CropArgs& a, const Forward& f, int grid, hipStream_t s) {
  if (a.n_preds == 0) return;
  if (a.balance) hipLaunchKernelGGL(k_crop_order, dim3(a.n_preds), dim3(kCropThreads), 0, s, a);
  hipLaunchKernelGGL(k_crop_cnn, dim3(grid), dim3(kCropThreads), 0, s, a, f);
}

}  // namespace hydro
