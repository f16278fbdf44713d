// Batched form (placeholder: sequential per-graph calls; replaced by the
// persistent multi-graph kernel).
#include "api_internal.hpp"

extern "C" int color_batch(int32_t num_jobs, const color_job* jobs, color_stats* per_job,
                           const color_params* params, void* stream) {
  if (num_jobs < 0 || (num_jobs > 0 && !jobs)) return COLOR_EINVAL;
  for (int i = 0; i < num_jobs; ++i) {
    const color_job& j = jobs[i];
    color_stats* st = per_job ? &per_job[i] : nullptr;
    int rc;
    if (j.kind == COLOR_KIND_D1)
      rc = color_d1(j.n, j.row_ptr, j.col_idx, j.seed, nullptr, nullptr, j.colors, st, params, stream);
    else if (j.kind == COLOR_KIND_D2)
      rc = color_d2(j.n, j.row_ptr, j.col_idx, j.seed, nullptr, nullptr, j.colors, st, params, stream);
    else if (j.kind == COLOR_KIND_PD2)
      rc = color_pd2(j.n_rows, j.n, j.row_ptr, j.col_idx, j.col_ptr, j.row_idx, j.seed, nullptr, nullptr,
                     j.colors, st, params, stream);
    else
      rc = COLOR_EINVAL;
    if (rc) return rc;
  }
  return COLOR_OK;
}
