// Serving entry points (continuous batching); filled in by the scheduler.
#include "../../include/slh.h"

extern "C" slh_status slh_server_create(const slh_server_cfg*, slh_server** out) {
  if (out) *out = nullptr;
  return SLH_E_STATE;
}
extern "C" slh_status slh_server_submit(slh_server*, const slh_problem*, int32_t, uint64_t*) {
  return SLH_E_STATE;
}
extern "C" slh_status slh_server_poll(slh_server*, uint64_t, int32_t*) { return SLH_E_STATE; }
extern "C" slh_status slh_server_result(slh_server*, uint64_t, double*, slh_balance*,
                                        slh_latency*) {
  return SLH_E_STATE;
}
extern "C" void slh_server_destroy(slh_server*) {}
