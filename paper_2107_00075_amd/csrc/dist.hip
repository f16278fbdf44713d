// Algorithm 2 (Section 3) over several ranks whose local graphs all sit on
// this GPU: the ranks' steps (color_d1_ghost_step) run one after another on
// one stream, and the boundary exchange that MPI messages would carry is one
// gather kernel over every rank's ghost copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "graphcolor.h"

namespace gcol {
namespace {

constexpr int kDistBlock = 256;

// New ghost colors: copy i of a ghost takes its owner's current color.
// Counts the copies whose color changed (the copies a rank would send).
__global__ __launch_bounds__(kDistBlock) void exchange_kernel(int32_t total, const int32_t* owner,
                                                              const int32_t* index, int32_t* const* owned_colors,
                                                              int32_t* gc, unsigned long long* changed) {
  const int32_t i = blockIdx.x * kDistBlock + threadIdx.x;
  uint32_t ch = 0;
  if (i < total) {
    const int32_t c = owned_colors[owner[i]][index[i]];
    if (c != gc[i]) {
      gc[i] = c;
      ch = 1;
    }
  }
  uint64_t t = __popcll(__ballot(ch != 0));
  if (lane_id() == 0 && t) atomicAdd(changed, static_cast<unsigned long long>(t));
}

// COLOR_FLAG_VALIDATE: every ghost's owner and index in range.
__global__ __launch_bounds__(kDistBlock) void check_map_kernel(int32_t total, const int32_t* owner,
                                                               const int32_t* index, int32_t parts,
                                                               const int32_t* n_owned, int32_t* err) {
  const int32_t i = blockIdx.x * kDistBlock + threadIdx.x;
  if (i >= total) return;
  const int32_t q = owner[i];
  if (q < 0 || q >= parts || index[i] < 0 || index[i] >= n_owned[q]) atomicOr(err, 1);
}

__global__ __launch_bounds__(kDistBlock) void fill_zero_kernel(int32_t n, int32_t* a) {
  const int32_t i = blockIdx.x * kDistBlock + threadIdx.x;
  if (i < n) a[i] = 0;
}

inline dim3 grid_of(int64_t n) { return dim3(static_cast<unsigned>((n + kDistBlock - 1) / kDistBlock)); }

// Device memory of one call, freed on every return path.
struct DistMem {
  void* p = nullptr;
  ~DistMem() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace
}  // namespace gcol

using namespace gcol;

extern "C" int color_d1_distributed(int32_t num_parts, const color_part* parts, uint32_t seed, int32_t max_detects,
                                    color_dist_stats* stats, const color_params* params, void* stream) {
  if (num_parts < 1 || !parts || max_detects < 0) return COLOR_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const bool degrees = params && (params->flags & COLOR_FLAG_RECOLOR_DEGREES);
  const bool validate = params && (params->flags & COLOR_FLAG_VALIDATE);
  std::vector<int64_t> off(num_parts + 1, 0);
  for (int32_t p = 0; p < num_parts; ++p) {
    const color_part& q = parts[p];
    if (q.n_owned < 0 || q.n_ghost < 0) return COLOR_EINVAL;
    if (q.n_owned > 0 && !q.owned_colors) return COLOR_EINVAL;
    if (q.n_ghost > 0 && (!q.ghost_owner || !q.ghost_index)) return COLOR_EINVAL;
    if (degrees && q.n_ghost > 0 && !q.ghost_degree) return COLOR_EINVAL;
    off[p + 1] = off[p] + q.n_ghost;
  }
  const int64_t total = off[num_parts];
  if (total >= INT_MAX) return COLOR_EOVERFLOW;
  // one allocation: ghost owners, indices and colors of every copy, the
  // ranks' owned-color pointers and sizes, the change counter, an error word
  const size_t t = static_cast<size_t>(std::max<int64_t>(total, 1));
  const size_t b_owner = 0, b_index = b_owner + 4 * t, b_gc = b_index + 4 * t;
  const size_t b_ptrs = (b_gc + 4 * t + 255) / 256 * 256;
  const size_t b_nown = b_ptrs + sizeof(int32_t*) * static_cast<size_t>(num_parts);
  const size_t b_ctr = (b_nown + 4 * static_cast<size_t>(num_parts) + 255) / 256 * 256;
  const size_t bytes = b_ctr + 256;
  DistMem mem;
  if (hipMalloc(&mem.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    mem.p = nullptr;
    return COLOR_ENOMEM;
  }
  char* base = static_cast<char*>(mem.p);
  int32_t* g_owner = reinterpret_cast<int32_t*>(base + b_owner);
  int32_t* g_index = reinterpret_cast<int32_t*>(base + b_index);
  int32_t* gc = reinterpret_cast<int32_t*>(base + b_gc);
  int32_t** d_ptrs = reinterpret_cast<int32_t**>(base + b_ptrs);
  int32_t* d_nown = reinterpret_cast<int32_t*>(base + b_nown);
  unsigned long long* d_changed = reinterpret_cast<unsigned long long*>(base + b_ctr);
  int32_t* d_err = reinterpret_cast<int32_t*>(base + b_ctr + 8);
  std::vector<int32_t*> ptrs(num_parts);
  std::vector<int32_t> nown(num_parts);
  for (int32_t p = 0; p < num_parts; ++p) {
    const color_part& q = parts[p];
    ptrs[p] = q.owned_colors;
    nown[p] = q.n_owned;
    const size_t nb = sizeof(int32_t) * static_cast<size_t>(q.n_ghost);
    if (nb && (hipMemcpyAsync(g_owner + off[p], q.ghost_owner, nb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
               hipMemcpyAsync(g_index + off[p], q.ghost_index, nb, hipMemcpyDeviceToDevice, st) != hipSuccess))
      return COLOR_EHIP;
  }
  if (hipMemcpyAsync(d_ptrs, ptrs.data(), sizeof(int32_t*) * ptrs.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_nown, nown.data(), sizeof(int32_t) * nown.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return COLOR_EHIP;
  hipLaunchKernelGGL(fill_zero_kernel, grid_of(static_cast<int64_t>(t)), dim3(kDistBlock), 0, st,
                     static_cast<int32_t>(t), gc);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(kDistBlock), 0, st, 4, reinterpret_cast<int32_t*>(d_changed));
  if (validate && total > 0) {
    int32_t err = 0;
    hipLaunchKernelGGL(check_map_kernel, grid_of(total), dim3(kDistBlock), 0, st, static_cast<int32_t>(total),
                       g_owner, g_index, num_parts, d_nown, d_err);
    if (hipMemcpyAsync(&err, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return COLOR_EHIP;
    if (err) return COLOR_EINVAL;
  }
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;

  const int32_t cap = stats && stats->trace_cap > 0 ? stats->trace_cap : 0;
  int32_t detects = 0, max_color = 0;
  int64_t rounds = 0, exchanged_total = 0;
  int n_exchanges = 0;
  auto exchange = [&]() -> int {
    unsigned long long changed = 0;
    if (total > 0) {
      hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(kDistBlock), 0, st, 2,
                         reinterpret_cast<int32_t*>(d_changed));
      hipLaunchKernelGGL(exchange_kernel, grid_of(total), dim3(kDistBlock), 0, st, static_cast<int32_t>(total),
                         g_owner, g_index, d_ptrs, gc, d_changed);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(&changed, d_changed, sizeof(changed), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return COLOR_EHIP;
    }
    if (stats && stats->exchanged_trace && n_exchanges < cap)
      stats->exchanged_trace[n_exchanges] = static_cast<int64_t>(changed);
    ++n_exchanges;
    exchanged_total += static_cast<int64_t>(changed);
    return COLOR_OK;
  };
  // one step of every rank; init: start from the rank's committed colors
  auto step_all = [&](bool init, int64_t* conflicts) -> int {
    *conflicts = 0;
    max_color = 0;
    for (int32_t p = 0; p < num_parts; ++p) {
      const color_part& q = parts[p];
      color_stats s{};
      const int rc = color_d1_ghost_step(q.n_owned, q.n_ghost, q.layers, q.n_g1, q.row_ptr, q.col_idx, q.gid,
                                         q.n_ghost > 0 ? gc + off[p] : nullptr, q.ghost_degree, seed,
                                         init ? q.owned_colors : nullptr, q.owned_colors, nullptr, &s, params,
                                         stream);
      if (rc != COLOR_OK) return rc;
      *conflicts += s.boundary_conflicts;
      rounds += s.rounds;
      max_color = std::max(max_color, s.num_colors);
    }
    return COLOR_OK;
  };

  int64_t conflicts = 0;
  int e;
  // the ranks' ghost-blind colorings (their ghosts' colors are not known yet:
  // the received colors are all 0, which constrain nothing)
  if ((e = step_all(false, &conflicts))) return e;
  int rc = COLOR_OK;
  while (true) {
    if ((e = exchange())) return e;
    if ((e = step_all(true, &conflicts))) return e;
    if (stats && stats->conflicts_trace && detects < cap) stats->conflicts_trace[detects] = conflicts;
    ++detects;
    if (conflicts == 0) break;
    if (max_detects > 0 && detects >= max_detects) {
      rc = COLOR_ENOCONVERGE;
      break;
    }
  }
  if (stats) {
    stats->detects = detects;
    stats->iterations = detects - 1;
    stats->num_colors = max_color;
    stats->exchanged_total = exchanged_total;
    stats->rounds_total = rounds;
  }
  return rc;
}
