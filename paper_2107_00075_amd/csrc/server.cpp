// Served form (placeholder; replaced by the continuous-batching server).
#include "api_internal.hpp"

struct color_server {
  int dummy;
};

extern "C" {
color_server* color_server_create(size_t, int32_t, int* err) {
  if (err) *err = COLOR_EINVAL;
  return nullptr;
}
int color_server_submit(color_server*, const color_host_job*, uint64_t*) { return COLOR_EINVAL; }
int color_server_poll(color_server*, uint64_t, int32_t*, color_stats*) { return COLOR_EINVAL; }
int color_server_drain(color_server*) { return COLOR_EINVAL; }
int color_server_destroy(color_server*) { return COLOR_OK; }
}
