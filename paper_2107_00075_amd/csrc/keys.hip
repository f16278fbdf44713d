// The recolorDegrees key as a per-vertex rank (Section 3.3; Algorithm 4 with
// recolorDegrees set).  See keys.hpp.
//
// Two ways to the (deg, p, gid) order, both by stable radix sorts:
//  * p is the hash of gid (no explicit priorities): p is a bijection of the
//    distinct gids, so p alone orders vertices of equal degree and one sort of
//    the 64-bit words (deg << 32) | p gives the order;
//  * explicit priorities may tie: sort by (p << 32) | gid first, then stably
//    by deg.
#include <hipcub/hipcub.hpp>

#include "device_common.hpp"
#include "keys.hpp"

namespace gcol {

namespace {

constexpr int kKeyBlock = 256;

__device__ __forceinline__ uint32_t degree_of(int32_t v, const int32_t* deg_ptr, int32_t n_rows,
                                              const int32_t* extra_deg) {
  if (v < n_rows) return static_cast<uint32_t>(deg_ptr[v + 1] - deg_ptr[v]);
  return static_cast<uint32_t>(extra_deg[v - n_rows]);
}

// Sort words of the first (or only) sort, and the identity permutation.
__global__ __launch_bounds__(kKeyBlock) void rank_words_kernel(int32_t m, const int32_t* deg_ptr, int32_t n_rows,
                                                               const int32_t* extra_deg, const int32_t* gid,
                                                               const uint32_t* prio, uint32_t hs, uint64_t* key,
                                                               int32_t* val) {
  const int32_t v = blockIdx.x * kKeyBlock + threadIdx.x;
  if (v >= m) return;
  const uint32_t g = gid ? static_cast<uint32_t>(gid[v]) : static_cast<uint32_t>(v);
  uint64_t w;
  if (prio) {
    w = (static_cast<uint64_t>(prio[v]) << 32) | g;
  } else {
    w = (static_cast<uint64_t>(degree_of(v, deg_ptr, n_rows, extra_deg)) << 32) | fmix32(g ^ hs);
  }
  key[v] = w;
  val[v] = v;
}

// Degrees in the order of the first sort (keys of the second, stable sort).
__global__ __launch_bounds__(kKeyBlock) void rank_degrees_kernel(int32_t m, const int32_t* order,
                                                                 const int32_t* deg_ptr, int32_t n_rows,
                                                                 const int32_t* extra_deg, uint32_t* deg) {
  const int32_t i = blockIdx.x * kKeyBlock + threadIdx.x;
  if (i < m) deg[i] = degree_of(order[i], deg_ptr, n_rows, extra_deg);
}

// rank[order[i]] = i.  The round kernels of later launches read the ranks
// with device-scope loads, so they are stored at device scope.
__global__ __launch_bounds__(kKeyBlock) void rank_scatter_kernel(int32_t m, const int32_t* order, uint32_t* rank) {
  const int32_t i = blockIdx.x * kKeyBlock + threadIdx.x;
  if (i < m) st_dev(&rank[order[i]], static_cast<uint32_t>(i));
}

inline dim3 grid_of(int32_t m) { return dim3(static_cast<unsigned>((m + kKeyBlock - 1) / kKeyBlock)); }

}  // namespace

size_t rank_tmp_bytes(int32_t m) {
  size_t a = 0, b = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, a, static_cast<const uint64_t*>(nullptr),
                                         static_cast<uint64_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                         static_cast<int32_t*>(nullptr), m) != hipSuccess)
    return 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, b, static_cast<const uint32_t*>(nullptr),
                                         static_cast<uint32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                         static_cast<int32_t*>(nullptr), m) != hipSuccess)
    return 0;
  return std::max<size_t>(std::max(a, b), 1);
}

int build_degree_rank(int32_t m, const int32_t* deg_ptr, int32_t n_rows, const int32_t* extra_deg,
                      const int32_t* gid, const uint32_t* prio, uint32_t hs, const RankBufs& b, uint32_t* rank,
                      hipStream_t st) {
  if (m <= 0) return 0;
  size_t tb = b.tmp_bytes;
  hipLaunchKernelGGL(rank_words_kernel, grid_of(m), dim3(kKeyBlock), 0, st, m, deg_ptr, n_rows, extra_deg, gid,
                     prio, hs, b.key0, b.val0);
  if (hipcub::DeviceRadixSort::SortPairs(b.tmp, tb, b.key0, b.key1, b.val0, b.val1, m, 0, 64, st) != hipSuccess)
    return -1;
  const int32_t* order = b.val1;
  if (prio) {
    hipLaunchKernelGGL(rank_degrees_kernel, grid_of(m), dim3(kKeyBlock), 0, st, m, b.val1, deg_ptr, n_rows,
                       extra_deg, b.deg0);
    tb = b.tmp_bytes;
    if (hipcub::DeviceRadixSort::SortPairs(b.tmp, tb, b.deg0, b.deg1, b.val1, b.val0, m, 0, 32, st) !=
        hipSuccess)
      return -1;
    order = b.val0;
  }
  hipLaunchKernelGGL(rank_scatter_kernel, grid_of(m), dim3(kKeyBlock), 0, st, m, order, rank);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gcol
