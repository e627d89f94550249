// Internal interfaces between the round driver (engine.hip) and the predicate kernels.
#pragma once

#include "common.h"

namespace hydro {

enum Tier { TIER_FIRST = 0, TIER_F32 = 1, TIER_F64 = 2 };

// Grouped launch over the MLP predicates of one tier.
struct MlpArgs {
  int n_preds;
  int pred[kMaxK];                  // predicate index of each slot
  int d_in[kMaxK], hidden[kMaxK];
  uint32_t class_mask[kMaxK];
  const __bf16* w1_bf[kMaxK];       // [hidden][d_in], folded
  const float* w1_f32[kMaxK];       // [hidden][d_in], folded
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
  const float* w_f32[kMaxK][3];     // packed per layer (fp32 fragments)
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
};

void launch_gcnn_pass(const GcnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s);
size_t gcnn_packed_elems(int layer, int cin, int cout, int prec);
void gcnn_pack_layer(int layer, int cin, int cout, int prec, const float* w, float scale, float* out);

constexpr int MLP_TILE_CONFIGS = 4;
int mlp_f64_chunks(int d_in);    // input chunks of the FP64 MLP hidden pass
void launch_mlp_pass(const MlpArgs& a, const Forward& f, int tier, int grid, hipStream_t s);
void launch_mlp_gemm(const MlpArgs& b, int cfg, bool bf, int grid, hipStream_t s);
int mlp_tile_bn(int cfg);
void launch_cnn_pass(const CnnArgs& a, const Forward& f, int tier, int grid, hipStream_t s);
size_t cnn_packed_elems(int variant, int layer, int prec);
void cnn_pack_layer(int variant, int layer, int prec, const float* w_canon, float scale, float* out);
int cnn_variant_of(int in_hw, int n_layers, const int* widths);
int cnn_grid_hint(int variant, int tier);

}  // namespace hydro
