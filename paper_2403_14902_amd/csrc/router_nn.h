// Learned content-based router: interface used by the round driver.
#pragma once

#include "common.h"

namespace hydro {

struct RouterNN;

// Device buffers come from `alloc(ctx, &p, bytes)` when it is given (and are then not freed by
// router_nn_destroy), else from hipMalloc.
typedef int (*RouterAllocFn)(void* ctx, void** p, size_t bytes);
int router_nn_create(RouterNN** out, int k, int fh, int fw, int64_t cap, uint64_t seed, int routing_batch,
                     float explore, const double* flops, RouterAllocFn alloc, void* alloc_ctx);
void router_nn_destroy(RouterNN* r);
// New query: initial weights, cleared optimiser state.
void router_nn_reset(RouterNN* r, hipStream_t s);
// Pooled features of the push's tuples lo..hi-1.  With `guard`, the launch does nothing unless the
// learned arm is routing (the fused CNN first pass computes every tuple's features on its first
// evaluation; only tuples admitted while the learned arm routes need them earlier).
int router_nn_admit(RouterNN* r, const FrameSrc& fr, int64_t lo, int64_t hi, const DevState* guard, hipStream_t s);
// Feature rows [cap][192] bf16 (written by the pooling kernels or by the fused CNN first pass).
__bf16* router_nn_feats_ptr(RouterNN* r);
// Keys of this round's live tuples (survivors in pend_in plus the admitted range).
void router_nn_keys(RouterNN* r, DevState* st, const uint32_t* pend_in, int in_slot, uint32_t adm_lo,
                    uint32_t adm_hi, int grid, hipStream_t s);
// Optimiser steps on the newest logged outcomes, then the judge.
void router_nn_learn(RouterNN* r, DevState* st, hipStream_t s);
const float* router_nn_keys_ptr(RouterNN* r);
// Per tuple: the round (DevState::rounds) in which its keys were last computed.
const uint32_t* router_nn_stamps_ptr(RouterNN* r);
OutcomeLog router_nn_log(RouterNN* r);
int router_nn_min_steps();
// Parameters (device, fp32: W1 | b1 | W2 | b2) and their number.
const float* router_nn_params_ptr(RouterNN* r);
int router_nn_param_count();
// First round (0-based) in which the learned arm can route.
int router_nn_first_learned_round();

}  // namespace hydro
