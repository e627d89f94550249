// Internal interfaces between the round driver (engine.hip) and the predicate kernels.
#pragma once

#include <vector>

#include "common.h"

namespace hydro {

// TIER_MID: the BF16 re-score tier between an FP8 first pass and the FP32 tier.
enum Tier { TIER_FIRST = 0, TIER_F32 = 1, TIER_F64 = 2, TIER_MID = 3 };

// Grouped launch over the MLP predicates of one tier.
struct MlpArgs {
  int n_preds;
  int pred[kMaxK];                  // predicate index of each slot
  int d_in[kMaxK], hidden[kMaxK];
  uint32_t class_mask[kMaxK];
  const __bf16* w1_bf[kMaxK];       // [hidden][d_in], folded
  const float* w1_f32[kMaxK];       // [hidden][d_in], folded
  const __bf16* w1_s3[kMaxK];       // bf16 frames: w1_f32 as three bf16 terms [3][hidden][d_in]
                                    // (hi, mid, lo; nullptr where not built)
  const float* b1_fold[kMaxK];
  const float* w2[kMaxK];           // [hidden][10]
  const float* b2[kMaxK];
  const float* w1_canon[kMaxK];     // [d_in][hidden]
  const float* b1_canon[kMaxK];
  float* partial[kMaxK];            // [hidden / part_w][part_cap][10]
  int part_w[kMaxK];                // hidden units per partial-logit part (half the tile width)
  int tile_cfg[kMaxK];              // GEMM tile configuration (see mlp_tile_bn)
  int64_t part_cap;
  double* esc_h[kMaxK];             // FP64 tier: partial hidden sums [chunk][esc_cap][hidden]
  int esc_cap;
  float* splitk_ws;                 // split-K partial sums, split_slots tiles of 128 x 128
  int* split_cnt;                   // per base tile: parts finished (zero between launches)
  int split_below;                  // launches with fewer (rows x hidden) tiles than this split K
  int split_target;                 // ... into about this many tiles
  int split_slots;
  Queues q;
  FrameSrc fr;
  DevState* st;
  int count_ticks;
  int prec;
};

// Grouped launch over the CNN predicates of one tier.
struct CnnArgs {
  int n_preds;
  int pred[kMaxK];
  int variant[kMaxK];
  uint32_t class_mask[kMaxK];
  const __bf16* w_bf[kMaxK][3];     // packed per layer (bf16 fragments)
  const __bf16* w_s3[kMaxK][3];     // FP32 tier: the same fragments as three bf16 terms (hi, mid,
                                    // lo; w = hi + mid + lo exactly), [term][fragment image]
  const float* bias[kMaxK][3];      // fp32, layer 1 folded
  const float* fc_w[kMaxK];         // [c_last][10]
  const float* fc_b[kMaxK];
  const float* w_canon[kMaxK][3];   // [co][ci][3][3]
  const float* b_canon[kMaxK][3];
  float pad_raw;                    // raw frame value that normalises to 0
  const float* wt_canon[kMaxK][3];  // FP64 tier: canonical weights as [co][3][3][ci]
  double* esc_act[kMaxK];           // FP64 tier: per-entry activations (esc_cap entries per slot)
  int64_t esc_stride;               // doubles per entry
  int esc_cap;                      // entries handled layer-parallel; the rest run one per block
  double* scratch64;                // FP64 tier fallback: per-block activation scratch
  int64_t scratch64_per_block;      // doubles
  int rest_grid;                    // blocks of the FP64 fallback launch (one scratch slot each)
  Queues q;
  FrameSrc fr;
  DevState* st;
  int count_ticks;
  int prec;
  __bf16* feats;                    // first pass: router features of each tuple's first evaluation
                                    // ([n][192] bf16), or nullptr
};

// Grouped launch over the generic (layer-wise) CNN predicates of one tier.
struct GcnnArgs {
  int n_preds;
  int pred[kMaxK];
  int n_layers[kMaxK];
  int in_hw[kMaxK];
  int widths[kMaxK][HYDRO_MAX_LAYERS];
  uint32_t class_mask[kMaxK];
  const __bf16* w_bf[kMaxK][HYDRO_MAX_LAYERS];    // packed fragments, layer 1 folded
  const float* w_f32[kMaxK][HYDRO_MAX_LAYERS];
  const float* bias[kMaxK][HYDRO_MAX_LAYERS];
  const float* fc_w[kMaxK];
  const float* fc_b[kMaxK];
  const float* wt_canon[kMaxK][HYDRO_MAX_LAYERS]; // FP64 tier: [co][3][3][ci]
  const float* b_canon[kMaxK][HYDRO_MAX_LAYERS];
  float pad_raw;
  void* act[2];                     // activations of every queued frame (all slots, in order)
  int64_t act_stride;               // elements per frame
  double* esc_act[kMaxK];           // FP64 tier: [esc_cap][2][esc_half]
  int64_t esc_stride, esc_half;
  int esc_cap;
  double* rest_scratch;             // FP64 tier beyond esc_cap: per block, two activation buffers
  int64_t rest_per_block;
  int rest_grid;                    // blocks of that launch (one scratch slot each)
  Queues q;
  FrameSrc fr;
  DevState* st;
  int count_ticks;
  int prec;
  // 4-layer 128x128 CNNs (conv 32-64-128-256): dedicated kernels (cnn4.hip); per slot
  int c4[kMaxK];                               // 1: the slot takes the dedicated kernels
  const void* c4_w1b[kMaxK];                   // layer 1, bf16 MFMA fragments [2][64][8]
  const void* c4_w1f[kMaxK];                   // layer 1, FP32 arithmetic: three-term bf16 fragments [3][2][64][8]
  const void* c4_w2[kMaxK][4];                 // layer 2 fragments per arithmetic (C4_*)
  const void* c4_img[kMaxK][2][4];             // layers 3, 4: A tile images per arithmetic (C4_*)
  const float* c4_wscale[kMaxK][3];            // FP8 tier: per-channel weight scales, layers 2..4
  float c4_ascale[kMaxK][3];                   // FP8 tier: activation scales, outputs of layers 1..3
  void* c4_act2;                               // layer-2 outputs [act_cap][32][32][64]
  void* c4_act3;                               // layer-3 outputs [act_cap][16][16][128]
  int64_t act_cap;                             // evaluations one launch may hold
  unsigned* c4_act_max;                        // calibration: [predicate][4] activation maxima (bits)
  const void* zero_page;                       // 256 zero bytes (padding taps of the GEMM gathers)
};

// Grouped launch over the CNN predicates that take each tuple's crop (variable-size inputs).
struct CropArgs {
  int n_preds;
  int pred[kMaxK];
  uint32_t class_mask[kMaxK];
  int n_layers[kMaxK];
  int widths[kMaxK][HYDRO_MAX_LAYERS];
  const float* wt[kMaxK][HYDRO_MAX_LAYERS];   // [3][3][ci][co] (output channels last), fp32
  const float* bias[kMaxK][HYDRO_MAX_LAYERS];
  const float* fc_w[kMaxK];                    // [c_last][10]
  const float* fc_b[kMaxK];
  const int32_t* crops;        // device copy of the push's crops [n][4]: y0, x0, h, w
  Queues q;
  FrameSrc fr;
  int fh, fw;                  // frame side lengths
  DevState* st;
  double* scratch;             // per workgroup: two activation buffers of act_doubles each
  int64_t act_doubles;
  int balance;                 // 1: data-aware order (largest crop first, shared counter)
  uint32_t* order;             // balance: queue positions by decreasing area, [kMaxK][cap]
  int* next;                   // balance: the launch's work counter (set to 0 by the order kernel)
};
void launch_crop_pass(const CropArgs& a, const Forward& f, int grid, hipStream_t s);

// Arithmetic tiers of the dedicated 4-layer CNN kernels.
// C4_S3: FP32 arithmetic of the layer-3/4 GEMMs from bf16 MFMAs (fp32 activations split into
// three bf16 terms on the fly, weights packed as three bf16 terms; see cnn4.hip).
// C4_X3: the C4_S3 kernels and images with the three leading products only (hi x hi, hi x mid,
// mid x hi; layer 1 the two leading weight terms): about 2^-16 relative, the re-score tier between
// a BF16 first pass and the FP32 tier (policy rescore3).
enum { C4_F32 = 0, C4_BF16 = 1, C4_FP8 = 2, C4_S3 = 3, C4_X3 = 4 };
struct C4FrontPack {
  std::vector<float> w1b;             // layer 1 (bf16 fragment order)
  std::vector<float> w2b, w2f;        // layer 2 (bf16 / fp32 fragment order, fp32 values)
  std::vector<uint16_t> w1s3, w2s3;   // layers 1 and 2 for FP32 arithmetic from three bf16 terms
  std::vector<uint8_t> w2q;           // layer 2 e4m3
};
bool c4_shape_ok(int in_hw, int n_layers, const int* widths);
void c4_pack_front(const float* w1, float scale1, const float* w2, const float* s2, C4FrontPack* out);
size_t c4_img_bytes(int prec, int layer);
void c4_pack_img(int prec, int layer, const float* w, const float* scale, unsigned char* out);
uint8_t c4_fp8_e4m3(float x);
float c4_fp8_value(uint8_t b);
void launch_c4_pass(const GcnnArgs& a, const Forward& f, int prec, int grid, hipStream_t s);

void launch_gcnn_pass(const GcnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s);
// Slot i of src becomes slot j of dst (every per-slot field).
void gcnn_copy_slot(GcnnArgs& dst, int j, const GcnnArgs& src, int i);
size_t gcnn_packed_elems(int layer, int cin, int cout, int prec);
void gcnn_pack_layer(int layer, int cin, int cout, int prec, const float* w, float scale, float* out);

constexpr int MLP_TILE_CONFIGS = 4;
int mlp_f64_chunks(int d_in);    // input chunks of the FP64 MLP hidden pass
void launch_mlp_pass(const MlpArgs& a, const Forward& f, int tier, int grid, hipStream_t s);
void launch_mlp_gemm(const MlpArgs& b, int cfg, bool bf, int grid, hipStream_t s);
int mlp_tile_bn(int cfg);
// Copy every per-predicate field of slot i of src into slot j of dst.
void mlp_copy_slot(MlpArgs& dst, int j, const MlpArgs& src, int i);
void launch_cnn_pass(const CnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s);
size_t cnn_packed_elems(int variant, int layer, int prec);
void cnn_pack_layer(int variant, int layer, int prec, const float* w_canon, float scale, float* out);
int cnn_variant_of(int in_hw, int n_layers, const int* widths);
int cnn_grid_hint(int variant, int tier);

}  // namespace hydro
