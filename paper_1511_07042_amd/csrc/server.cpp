// Continuous-batching server (placeholder until the grouped launcher lands).
#include "bmg_internal.h"

extern "C" {

int bmg_server_create(int64_t, int32_t, bmg_server** out) {
  if (out) *out = nullptr;
  bmg::set_error("serving is not available in this build");
  return BMG_EINVAL;
}
int bmg_server_submit(bmg_server*, const bmg_surface_desc*, int32_t, int32_t, double, double,
                      const bmg_solve_opts*, uint64_t*) {
  bmg::set_error("serving is not available in this build");
  return BMG_EINVAL;
}
int bmg_server_poll(bmg_server*, uint64_t, double*, double*, int64_t, bmg_solve_stats*, double*) {
  bmg::set_error("serving is not available in this build");
  return BMG_EINVAL;
}
int bmg_server_cancel(bmg_server*, uint64_t) {
  bmg::set_error("serving is not available in this build");
  return BMG_EINVAL;
}
void bmg_server_destroy(bmg_server*) {}

}
