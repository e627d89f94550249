// Learned content-based router: interface used by the round driver.
#pragma once

#include "common.h"

namespace hydro {

struct RouterNN;

int router_nn_create(RouterNN** out, int k, int fh, int fw, int64_t cap, uint64_t seed, int routing_batch);
void router_nn_destroy(RouterNN* r);
void router_nn_reset(RouterNN* r, hipStream_t s);
int router_nn_admit(RouterNN* r, const FrameSrc& fr, int64_t n, hipStream_t s);
void router_nn_round(RouterNN* r, DevState* st, hipStream_t s);
void router_nn_learn(RouterNN* r, DevState* st, const FrameSrc& fr, const uint32_t* route_log, hipStream_t s);
const float* router_nn_keys(RouterNN* r);
const uint8_t* router_nn_arms(RouterNN* r);

}  // namespace hydro
