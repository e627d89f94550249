// Learned content-based router: interface used by the round driver.
#pragma once

#include "common.h"

namespace hydro {

struct RouterNN;

int router_nn_create(RouterNN** out, int k, int fh, int fw, int64_t cap, uint64_t seed, int routing_batch,
                     float explore, const double* flops);
void router_nn_destroy(RouterNN* r);
// New query: initial weights, cleared optimiser state.
void router_nn_reset(RouterNN* r, hipStream_t s);
// Pooled features of every tuple of a push.
int router_nn_admit(RouterNN* r, const FrameSrc& fr, int64_t n, hipStream_t s);
// Keys of this round's live tuples (survivors in pend_in plus the admitted range).
void router_nn_keys(RouterNN* r, DevState* st, const uint32_t* pend_in, int in_slot, uint32_t adm_lo,
                    uint32_t adm_hi, int grid, hipStream_t s);
// Optimiser steps on the newest logged outcomes, then the judge.
void router_nn_learn(RouterNN* r, DevState* st, hipStream_t s);
const float* router_nn_keys_ptr(RouterNN* r);
OutcomeLog router_nn_log(RouterNN* r);
int router_nn_min_steps();

}  // namespace hydro
