// Device helpers shared by the round kernels: the priority key and the
// 64-lane wavefront primitives of CDNA4 (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcol {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // workgroup of the round kernels: 4 wavefronts
constexpr int kWavesPerBlock = kBlock / kWave;

// Problem kinds (the coloring variants of Section 2.1).
enum Mode : int { kD1 = 1, kD2 = 2, kPD2 = 3 };

// MurmurHash3 32-bit finalizer.  With h = seed-derived constant, the
// priority p(v) = fmix32(gid ^ h) stands for rand(GID) of Algorithm 4: a
// bijection of uint32, so two vertices never draw the same number.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

inline uint32_t host_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

inline uint32_t hash_seed(uint32_t seed) { return host_fmix32(seed ^ 0x9E3779B9u); }

// Device-coherent accesses.  Arrays that the library's kernels write and
// later kernels read (colors, tentative colors, worklists, per-call setup
// arrays) are written and read with device-scope (sc1) loads and stores.
// Measured on MI355X: plain loads of such data written by an earlier kernel on
// another XCD could return stale values (agent- or system-scope fences issued
// by every wavefront at kernel start and end did not prevent it), while
// device-scope accesses gave bit-exact results in every run.
template <typename X>
__device__ __forceinline__ X ld_dev(const X* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename X>
__device__ __forceinline__ void st_dev(X* p, X v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads of a round kernel's bulk arrays (worklists, lists, offsets, colors,
// bitsets).  The per-round kernels read them with plain, L2-cacheable loads
// (MUT = 0): the data was written by earlier launches, whose writes every
// later launch on the stream sees (measured on MI355X: 3.8e9 reads of lines
// that another XCD rewrote in the previous launch, none stale), or it is
// written concurrently in ways whose late visibility cannot change a
// result (a compaction that keeps a neighbour committed in the same round, a
// bitset pre-read that only skips an atomic).  Kernels whose phases hand
// data to each other inside one launch (the tail kernel across its grid
// barriers, the persistent batched kernel) read them at device scope
// (MUT = 1).
template <int MUT, typename X>
__device__ __forceinline__ X ld_mut(const X* p) {
  if constexpr (MUT != 0) return ld_dev(p);
  else return *p;
}
template <int MUT, typename X>
__device__ __forceinline__ void st_mut(X* p, X v) {
  if constexpr (MUT != 0) st_dev(p, v);
  else *p = v;
}

// The row of CSR entry e (0 <= e < rp[n]): the last row whose start is <= e,
// by binary search over the n row offsets (empty rows are skipped).
__device__ __forceinline__ int32_t row_of(const int32_t* rp, int32_t n, int32_t e) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Where a vertex's key comes from.  key(v) = (p(v), gid(v)) packed into 64
// bits so that one unsigned compare is the lexicographic compare; the lower
// key loses a conflict.  With recolorDegrees (Section 3.3) the key is
// (deg(v), p(v), gid(v)); the library then passes each vertex's rank in that
// order, which compares the same way and never ties.
struct KeySource {
  const uint32_t* prio;  // nullable: explicit p(v)
  const int32_t* gid;    // nullable: gid(v) = v
  uint32_t hs;           // hash_seed(seed)
  const uint32_t* rank;  // nullable: recolorDegrees rank (written by an earlier kernel of the call)
};

__device__ __forceinline__ uint64_t key_of(const KeySource& k, int32_t v) {
  if (k.rank) return ld_dev(&k.rank[v]);
  const uint32_t g = k.gid ? static_cast<uint32_t>(k.gid[v]) : static_cast<uint32_t>(v);
  const uint32_t p = k.prio ? k.prio[v] : fmix32(g ^ k.hs);
  return (static_cast<uint64_t>(p) << 32) | g;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups are dispatched round-robin over the 8 XCDs; this renumbering
// gives every XCD a contiguous range of logical ids (grids that are a
// multiple of 8), so each XCD's L2 sees a contiguous range of the work.
__device__ __forceinline__ int32_t xcd_logical_block_of(int32_t nb, int32_t i) {
  const int32_t per = nb / 8;
  if (per == 0 || (nb & 7) != 0) return i;
  return (i & 7) * per + (i >> 3);
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// OR of a 64-bit value over aligned groups of G lanes (all lanes of a group
// must be active).
template <int G>
__device__ __forceinline__ uint64_t group_or(uint64_t x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x |= __shfl_xor(x, off, kWave);
  return x;
}

// 1 if any lane of the calling lane's aligned G-lane group has pred set.
template <int G>
__device__ __forceinline__ bool group_any(bool pred) {
  const uint64_t b = __ballot(pred);
  if (G == kWave) return b != 0;
  const int first = lane_id() & ~(G - 1);
  const uint64_t gm = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  return ((b >> first) & gm) != 0;
}

__device__ __forceinline__ uint64_t atomic_load_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t atomic_load_i32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Resets of words that other workgroups update with atomics in the same
// kernel use an atomic read-modify-write too, so that every access to such a
// word (and to its cache line) is performed at the same coherence point;
// a plain store there could leave a dirty partial line in one XCD's L2.
__device__ __forceinline__ void atomic_reset_u32(uint32_t* p) { (void)atomicExch(p, 0u); }
__device__ __forceinline__ void atomic_reset_i32(int32_t* p) { (void)atomicExch(p, 0); }

}  // namespace gcol
