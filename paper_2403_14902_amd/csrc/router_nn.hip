// Learned content-based router (not yet available in this build).
#include <string>

#include "router_nn.h"

namespace hydro {

struct RouterNN {};

int router_nn_create(RouterNN** out, int, int, int, int64_t, uint64_t, int) {
  *out = nullptr;
  return HYDRO_EUNSUPPORTED;
}
void router_nn_destroy(RouterNN*) {}
void router_nn_reset(RouterNN*, hipStream_t) {}
int router_nn_admit(RouterNN*, const FrameSrc&, int64_t, hipStream_t) { return HYDRO_EUNSUPPORTED; }
void router_nn_round(RouterNN*, DevState*, hipStream_t) {}
void router_nn_learn(RouterNN*, DevState*, const FrameSrc&, const uint32_t*, hipStream_t) {}
const float* router_nn_keys(RouterNN*) { return nullptr; }
const uint8_t* router_nn_arms(RouterNN*) { return nullptr; }

}  // namespace hydro
