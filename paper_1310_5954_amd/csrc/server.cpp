// Serving scheduler (placeholder until the batched scheduler lands).
#include "internal.hpp"

using namespace letkf;

extern "C" {
int letkf_server_create(void*, size_t, int32_t, uint32_t, letkf_server** out) {
  if (out) *out = nullptr;
  return fail(LETKF_ESTATE, "serving scheduler not built");
}
int letkf_server_add(letkf_server*, const letkf_dims*, const letkf_model*, const letkf_domain_map*, int,
                     uint32_t, const double*, letkf_handle**) { return fail(LETKF_ESTATE, "serving scheduler not built"); }
int letkf_server_remove(letkf_server*, letkf_handle*) { return fail(LETKF_ESTATE, "serving scheduler not built"); }
int letkf_submit_frame(letkf_handle*, const double*, uint64_t, double*, letkf_done_fn, void*) {
  return fail(LETKF_ESTATE, "serving scheduler not built");
}
int letkf_server_drain(letkf_server*) { return fail(LETKF_ESTATE, "serving scheduler not built"); }
int letkf_server_stats(letkf_server*, uint64_t*, uint64_t*, uint64_t*) { return fail(LETKF_ESTATE, "serving scheduler not built"); }
int letkf_server_destroy(letkf_server*) { return LETKF_OK; }
}
