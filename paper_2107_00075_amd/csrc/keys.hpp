// The recolorDegrees key (Section 3.3; Algorithm 4 with recolorDegrees set).
//
// key(v) = (deg(v), p(v), gid(v)) compared lexicographically: of two
// conflicting vertices the one with the lower degree is uncolored, and the
// random number p (ties by gid) only decides between equal degrees.  Degrees
// are computed once, before the rounds (Section 3.3).
//
// The kernels do not compare three fields.  The library sorts the vertices by
// that key once per call and hands the kernels each vertex's rank in the
// order (KeySource::rank): one 32-bit value per vertex whose order is the
// key's order, and which never ties.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gcol {

// Device buffers of the sort (all owned by the caller, sized for m vertices;
// tmp is hipcub's temporary storage of tmp_bytes, see rank_tmp_bytes).
struct RankBufs {
  uint64_t* key0;
  uint64_t* key1;
  int32_t* val0;
  int32_t* val1;
  uint32_t* deg0;
  uint32_t* deg1;
  void* tmp;
  size_t tmp_bytes;
};

// Bytes of hipcub temporary storage the sorts of m vertices need (0 on error).
size_t rank_tmp_bytes(int32_t m);

// rank[v] for v < m: the position of v in ascending (deg, p, gid) order.
//   deg(v) = deg_ptr[v+1] - deg_ptr[v] for v < n_rows, extra_deg[v - n_rows]
//            for the others (a ghost's degree, reported by its owner)
//   gid    nullable (gid(v) = v); prio nullable (p = the hash of gid)
// Returns 0, or -1 when a HIP call failed.
int build_degree_rank(int32_t m, const int32_t* deg_ptr, int32_t n_rows, const int32_t* extra_deg,
                      const int32_t* gid, const uint32_t* prio, uint32_t hs, const RankBufs& b, uint32_t* rank,
                      hipStream_t st);

}  // namespace gcol
