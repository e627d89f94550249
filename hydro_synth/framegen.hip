// Device generator of the structured synthetic frames (inputs only: no part of the query's
// arithmetic lives here).
//
// It reproduces, bit for bit, the numpy recipe of hydro_synth.make_frames for the structured
// workloads: per chunk of frames a PCG64 stream (seeded on the host through numpy's
// SeedSequence) first yields the 8x8x3 low-frequency field z per frame (drawn on the host, where
// numpy's normal sampler runs), then one uniform double per frame value for the noise e.  The
// device takes over the second part: it advances each chunk's PCG64 state to the first value a
// thread produces (LCG jump-ahead, Brown 1994, "Random number generation with arbitrary
// strides"), steps it with the PCG XSL-RR 128/64 output function (O'Neill 2014, the generator
// numpy calls PCG64), maps each output to a double as numpy does ((x >> 11) * 2^-53, scaled to
// [-1, 1)), and evaluates the same fp64 expressions in the same order as the numpy code:
//   t  = w_lo[x] * z[lo[x]] + w_hi[x] * z[hi[x]]        (columns)
//   up = w_lo[y] * t[lo[y]] + w_hi[y] * t[hi[y]]        (rows)
//   v  = clip((0.5 + 0.25 * up) + 0.10 * e, 0, 1)
// then quantises v to uint8 (round-half-even of 255 v) or bf16 (fp32 RNE, then bf16 RNE).
// The file is compiled with -ffp-contract=off so that no multiply-add is fused.
//
// The same functions run on the host (hs_frames_host) so that the CPU tests can pin the
// arithmetic against numpy without a GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <string>

namespace {

typedef unsigned __int128 u128;

constexpr int kSrc = 8;          // side of the low-frequency field
constexpr int kMaxHw = 256;
constexpr int kDtypeBf16 = 1;
constexpr int kDtypeU8 = 2;

__host__ __device__ inline u128 pcg_mult() {
  return ((u128)0x2360ED051FC65DA4ull << 64) | (u128)0x4385DF649FCCF645ull;
}

// state advanced by delta LCG steps: s -> s * M + inc, delta times
__host__ __device__ inline u128 pcg_advance(u128 s, u128 inc, uint64_t delta) {
  u128 acc_mult = 1, acc_plus = 0, cur_mult = pcg_mult(), cur_plus = inc;
  while (delta > 0) {
    if (delta & 1) {
      acc_mult *= cur_mult;
      acc_plus = acc_plus * cur_mult + cur_plus;
    }
    cur_plus = (cur_mult + 1) * cur_plus;
    cur_mult *= cur_mult;
    delta >>= 1;
  }
  return acc_mult * s + acc_plus;
}

__host__ __device__ inline uint64_t pcg_output(u128 s) {
  const uint64_t x = (uint64_t)(s >> 64) ^ (uint64_t)s;
  const unsigned r = (unsigned)(s >> 122);
  return (x >> r) | (x << ((64u - r) & 63u));
}

__host__ __device__ inline double noise_of(uint64_t bits) {
  const double u = (double)(bits >> 11) * (1.0 / 9007199254740992.0);
  return -1.0 + 2.0 * u;
}

struct GenArgs {
  int dtype;
  int hw;
  int frames_per_chunk;      // frames of every chunk (the chunk's draw stride)
  int n_chunks;              // chunks in this call
  int first_frame;           // frame of chunk 0 to start at (later chunks start at frame 0)
  int64_t n_frames;          // frames written in total
  const double* z;           // [n_chunks][frames_per_chunk][3][8][8]
  const uint64_t* state;     // [n_chunks][4]: state lo, state hi, inc lo, inc hi (after z)
  const double* w_lo;        // [hw]
  const double* w_hi;        // [hw]
  const int* lo;             // [hw]
  const int* hi;             // [hw]
  void* out;                 // [n_frames][hw][hw][3]
};

// Quantise one value into the output.
__host__ __device__ inline void store_value(const GenArgs& a, int64_t o, double v) {
  if (a.dtype == kDtypeU8) {
    static_cast<uint8_t*>(a.out)[o] = (uint8_t)__builtin_rint(255.0 * v);
  } else {
    const float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    const uint64_t w = (uint64_t)u;
    static_cast<uint16_t*>(a.out)[o] = (uint16_t)((w + 0x7FFFull + ((w >> 16) & 1ull)) >> 16);
  }
}

// One frame row: hw pixels x 3 values, drawn in the chunk's C order (frame, y, x, c).
__host__ __device__ inline void gen_row(const GenArgs& a, int64_t out_frame, int chunk, int f, int y) {
  const int hw = a.hw;
  const double* zf = a.z + ((int64_t)chunk * a.frames_per_chunk + f) * 3 * kSrc * kSrc;
  const uint64_t* st = a.state + 4 * chunk;
  const u128 s0 = ((u128)st[1] << 64) | st[0];
  const u128 inc = ((u128)st[3] << 64) | st[2];
  const uint64_t first = (((uint64_t)f * hw + y) * hw) * 3;   // draws before this row
  u128 s = pcg_advance(s0, inc, first);
  const u128 M = pcg_mult();
  const int ly = a.lo[y], hy = a.hi[y];
  const double wly = a.w_lo[y], why = a.w_hi[y];
  const int64_t base = ((out_frame * hw) + y) * (int64_t)hw * 3;
  for (int x = 0; x < hw; ++x) {
    const int lx = a.lo[x], hx = a.hi[x];
    const double wlx = a.w_lo[x], whx = a.w_hi[x];
    for (int c = 0; c < 3; ++c) {
      const double* zc = zf + c * kSrc * kSrc;   // z[c][i][j]
      const double t_lo = wlx * zc[ly * kSrc + lx] + whx * zc[ly * kSrc + hx];
      const double t_hi = wlx * zc[hy * kSrc + lx] + whx * zc[hy * kSrc + hx];
      const double up = wly * t_lo + why * t_hi;
      s = s * M + inc;
      const double e = noise_of(pcg_output(s));
      double v = (0.5 + 0.25 * up) + 0.10 * e;
      v = v < 0.0 ? 0.0 : v;
      v = v > 1.0 ? 1.0 : v;
      store_value(a, base + x * 3 + c, v);
    }
  }
}

// (chunk, frame) of output frame j of the call
__host__ __device__ inline void locate(const GenArgs& a, int64_t j, int* chunk, int* f) {
  const int64_t g = j + a.first_frame;
  *chunk = (int)(g / a.frames_per_chunk);
  *f = (int)(g % a.frames_per_chunk);
}

__global__ __launch_bounds__(256) void gen_rows_kernel(GenArgs a) {
  const int64_t rows = a.n_frames * a.hw;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = r / a.hw;
    const int y = (int)(r % a.hw);
    int chunk, f;
    locate(a, j, &chunk, &f);
    gen_row(a, j, chunk, f, y);
  }
}

thread_local std::string g_err;

int check_args(const GenArgs& a) {
  if (a.dtype != kDtypeU8 && a.dtype != kDtypeBf16) { g_err = "dtype must be bf16 (1) or u8 (2)"; return -1; }
  if (a.hw < 1 || a.hw > kMaxHw) { g_err = "frame side out of range"; return -1; }
  if (a.frames_per_chunk < 1 || a.n_chunks < 1 || a.first_frame < 0 || a.first_frame >= a.frames_per_chunk) {
    g_err = "bad chunk layout";
    return -1;
  }
  if (a.n_frames < 0 || a.first_frame + a.n_frames > (int64_t)a.n_chunks * a.frames_per_chunk) {
    g_err = "more frames than the chunks hold";
    return -1;
  }
  if (!a.z || !a.state || !a.w_lo || !a.w_hi || !a.lo || !a.hi || !a.out) { g_err = "null pointer"; return -1; }
  return 0;
}

GenArgs make_args(int dtype, int hw, int fpc, int n_chunks, int first_frame, int64_t n_frames, const double* z,
                  const uint64_t* state, const double* w_lo, const double* w_hi, const int* lo, const int* hi,
                  void* out) {
  GenArgs a;
  a.dtype = dtype; a.hw = hw; a.frames_per_chunk = fpc; a.n_chunks = n_chunks; a.first_frame = first_frame;
  a.n_frames = n_frames; a.z = z; a.state = state; a.w_lo = w_lo; a.w_hi = w_hi; a.lo = lo; a.hi = hi; a.out = out;
  return a;
}

}  // namespace

extern "C" {

// Host evaluation of the recipe (every pointer in host memory).  Returns 0, or -1 with a message.
int hs_frames_host(int dtype, int hw, int frames_per_chunk, int n_chunks, int first_frame, int64_t n_frames,
                   const double* z, const uint64_t* state, const double* w_lo, const double* w_hi, const int* lo,
                   const int* hi, void* out) {
  GenArgs a = make_args(dtype, hw, frames_per_chunk, n_chunks, first_frame, n_frames, z, state, w_lo, w_hi, lo, hi, out);
  if (check_args(a)) return -1;
  for (int64_t j = 0; j < n_frames; ++j) {
    int chunk, f;
    locate(a, j, &chunk, &f);
    for (int y = 0; y < hw; ++y) gen_row(a, j, chunk, f, y);
  }
  return 0;
}

// Device evaluation: the same arguments as device pointers, enqueued on `stream` (a
// hipStream_t, or NULL for the default stream).  Returns 0, -1 (arguments) or -3 (HIP error).
int hs_frames_device(int dtype, int hw, int frames_per_chunk, int n_chunks, int first_frame, int64_t n_frames,
                     const double* z, const uint64_t* state, const double* w_lo, const double* w_hi, const int* lo,
                     const int* hi, void* out, void* stream) {
  GenArgs a = make_args(dtype, hw, frames_per_chunk, n_chunks, first_frame, n_frames, z, state, w_lo, w_hi, lo, hi, out);
  if (check_args(a)) return -1;
  if (n_frames == 0) return 0;
  const int64_t rows = n_frames * hw;
  int64_t blocks = (rows + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gen_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_err = std::string("frame generator launch: ") + hipGetErrorString(e);
    return -3;
  }
  return 0;
}

const char* hs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
