// Round kernels of synchronous speculative coloring for CDNA4 (gfx950).
//
// One round (Section 3, Algorithm 2's loop; the local speculative rounds of
// Section 3.2) is two launches:
//   color  : every vertex v of the worklist W_r takes T[v] = the smallest
//            color >= 1 that its neighbourhood does not hold in the committed
//            array C (first-fit, Section 2.2, Algorithm 1).  Only C is read.
//   detect : v loses when a neighbour u holds T[u] == T[v] with key(u) >
//            key(v) (Section 3.2, Algorithms 3 and 4, with the lower key
//            uncolored).  Only T is read.  Winners commit C[v] = T[v] in
//            place; losers are appended to W_{r+1} by ballot/prefix
//            compaction.
// Committed neighbours never tie: T[u] == C[u] for them and T[v] avoids every
// committed neighbour color, so reading T of all neighbours equals reading T
// of the worklist neighbours only.  Neither kernel reads what it writes, so
// the round is exactly the synchronous (snapshot) round.
//
// Neighbourhoods: D1 = N(v); D2 = N(v) u N(N(v)) minus v (Section 2.1,
// Algorithm 5 with doPartialColoring false); PD2 = columns sharing a row
// with column v (Section 3.6, doPartialColoring true: no one-hop term).
//
// Mapping: each worklist is split into five static degree bins.  Bins 0..2
// give a vertex an aligned group of G lanes (G = 1..64) that stride over its
// adjacency, so a group reads contiguous col_idx entries and OR-reduces a
// 64-bit forbidden-color window with cross-lane shuffles.  Bin 3 gives a
// vertex a workgroup (register window for colors 1..64 plus an LDS bitset for
// the next 32768 colors).  Bin 4 splits a vertex over several workgroups that
// merge their windows into a global per-vertex bitset; the last workgroup to
// arrive picks the color or commits (the edge-split parallelism that the
// paper's edge-based kernel provides for very high degrees, Section 3.2).
// Light bins are cut into chunks of 256 worklist entries that workgroups take
// by a static XCD-aware partition (no device atomics on the hot path; one
// atomic per chunk appends the chunk's losers); heavy units are taken
// dynamically from a device counter afterwards.
#include <algorithm>
#include <climits>

#include "round_steps.hpp"

namespace gcol {

// Per-round work map, built once per workgroup in LDS.  Light bins (0..2) are
// cut into chunks of kBlock worklist entries that workgroups take by a static,
// XCD-aware partition; heavy units (one per bin-3 vertex, split_chunks per
// bin-4 vertex) are taken dynamically from a device counter afterwards.
struct RoundMap {
  int32_t cnt[kBins];
  int32_t chunks[3];
  int32_t light_total;
  int32_t heavy_block;   // units of bin 3
  int32_t heavy_total;   // units of bins 3 and 4
};

__device__ __forceinline__ void make_round_map(const RoundBufs& b, const BinLayout& L, RoundMap& m) {
  int32_t lt = 0;
  for (int i = 0; i < kBins; ++i) m.cnt[i] = atomic_load_i32(&b.cnt_in[i]);
  for (int i = 0; i < 3; ++i) {
    m.chunks[i] = (m.cnt[i] + kBlock - 1) / kBlock;
    lt += m.chunks[i];
  }
  m.light_total = lt;
  m.heavy_block = m.cnt[kBlockBin];
  m.heavy_total = m.cnt[kBlockBin] + m.cnt[kSplitBin] * L.split_chunks;
}

__device__ __forceinline__ int32_t xcd_logical_block() { return xcd_logical_block_of(gridDim.x, blockIdx.x); }

// Chunk c of the light bins -> (bin, first entry, entries).
__device__ __forceinline__ void light_chunk(const RoundMap& m, int32_t c, int& bin, int32_t& first,
                                            int32_t& count) {
  bin = 0;
  while (bin < 2 && c >= m.chunks[bin]) {
    c -= m.chunks[bin];
    ++bin;
  }
  first = c * kBlock;
  count = min(kBlock, m.cnt[bin] - first);
}

// ---------------------------------------------------------------------------
// color: one chunk of a split vertex
// ---------------------------------------------------------------------------
template <int MODE>
__device__ void color_split_chunk(const GraphView& g, const RoundBufs& b, const BinLayout& L,
                                  int32_t si, int chunk, uint32_t* ovf, uint64_t* red,
                                  int32_t* s_misc, uint64_t& work_acc) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int nch = L.split_chunks;
  const int32_t v = ld_dev(&b.split_vertex[si]);
  const int32_t rb = g.rp[v], re = g.rp[v + 1];
  const int64_t len = re - rb;
  const int32_t cb = rb + static_cast<int32_t>(len * chunk / nch);
  const int32_t ce = rb + static_cast<int32_t>(len * (chunk + 1) / nch);
  uint32_t* gm = b.split_mask + static_cast<size_t>(si) * b.capw;
  const uint32_t capbits = static_cast<uint32_t>(b.capw) * 32u;
  const int32_t* __restrict__ C = b.C;

  for (int w = tid; w < kOvfWords; w += kBlock) ovf[w] = 0u;
  __syncthreads();
  uint64_t m = 0;
  scan_nbhd<MODE>(g, v, cb, ce, tid, kBlock, [&](int32_t u) {
    const int32_t c = ld_dev(&C[u]);
    if (c <= 0) return false;
    uint32_t d = static_cast<uint32_t>(c - 1);  // bit c-1 stands for color c
    if (d < 64u) {
      m |= 1ull << d;
    } else if (d - 64u < static_cast<uint32_t>(kOvfWords * 32)) {
      d -= 64u;
      atomicOr(&ovf[d >> 5], 1u << (d & 31u));
    } else if (d < capbits) {
      atomicOr(&gm[d >> 5], 1u << (d & 31u));
    }
    return false;
  });
  m = group_or<kWave>(m);
  if (lane_id() == 0) red[wave] = m;
  __syncthreads();
  if (tid == 0) {
    m = red[0] | red[1] | red[2] | red[3];
    if (static_cast<uint32_t>(m)) atomicOr(&gm[0], static_cast<uint32_t>(m));
    if (m >> 32) atomicOr(&gm[1], static_cast<uint32_t>(m >> 32));
    if (chunk == 0) work_acc += static_cast<uint64_t>(ld_dev(&b.work[v]));
  }
  for (int w = tid; w < kOvfWords && 2 + w < b.capw; w += kBlock) {
    const uint32_t x = ovf[w];
    if (x) atomicOr(&gm[2 + w], x);
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) s_misc[1] = (atomicAdd(&b.split_ctr[si], 1u) == static_cast<uint32_t>(nch - 1));
  __syncthreads();
  if (s_misc[1]) {  // last chunk to arrive: pick the color
    __threadfence();
    const int32_t mc = atomic_load_i32(b.maxc);
    const int32_t nwords = min(b.capw, mc / 32 + 1);
    if (tid == 0) s_misc[0] = INT_MAX;
    __syncthreads();
    for (int w = tid; w < nwords; w += kBlock) {
      const uint32_t x = atomic_load_u32(&gm[w]);
      if (x != ~0u) {
        atomicMin(&s_misc[0], w * 32 + __builtin_ctz(~x));
        break;
      }
    }
    __syncthreads();
    const int32_t bit = s_misc[0];
    for (int w = tid; w < nwords; w += kBlock) atomic_reset_u32(&gm[w]);
    if (tid == 0) {
      st_dev(&b.T[v], (bit == INT_MAX ? nwords * 32 : bit) + 1);
      atomic_reset_u32(&b.split_ctr[si]);
    }
  }
  __syncthreads();
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void color_round_kernel(GraphView g, KeySource k, RoundBufs b,
                                                             BinLayout L, int round) {
  __shared__ uint32_t ovf[kOvfWords];
  __shared__ uint64_t red[kWavesPerBlock];
  __shared__ int32_t s_misc[4];
  __shared__ int32_t s_unit;
  __shared__ unsigned long long s_work;
  __shared__ RoundMap M;
  (void)k;
  if (threadIdx.x == 0) {
    make_round_map(b, L, M);
    s_work = 0ull;
    if (blockIdx.x == 0) {
      int64_t total = 0;
      for (int i = 0; i < kBins; ++i) {
        atomic_reset_i32(&b.cnt_out[i]);
        total += M.cnt[i];
      }
      atomic_reset_i32(&b.tile_ctr[1]);
      if (total > 0) {
        atomicMax(b.rounds_done, round);
        if (b.trace && round <= b.trace_cap) st_dev(&b.trace[round - 1], static_cast<int32_t>(total));
        atomicAdd(&b.visits[0], static_cast<unsigned long long>(total));
      }
    }
  }
  __syncthreads();
  uint64_t work_acc = 0;
  // light bins: a static, contiguous share of chunks per workgroup
  const int32_t lb = xcd_logical_block();
  const int32_t c0 = static_cast<int32_t>(static_cast<int64_t>(lb) * M.light_total / gridDim.x);
  const int32_t c1 = static_cast<int32_t>(static_cast<int64_t>(lb + 1) * M.light_total / gridDim.x);
  for (int32_t c = c0; c < c1; ++c) {
    int bin;
    int32_t first, count;
    light_chunk(M, c, bin, first, count);
    const int32_t* wl = b.wl_in + L.off[bin] + first;
    switch (L.lanes[bin]) {
      case 1: color_chunk_group<MODE, 1>(g, b, wl, count, work_acc); break;
      case 2: color_chunk_group<MODE, 2>(g, b, wl, count, work_acc); break;
      case 4: color_chunk_group<MODE, 4>(g, b, wl, count, work_acc); break;
      case 8: color_chunk_group<MODE, 8>(g, b, wl, count, work_acc); break;
      case 16: color_chunk_group<MODE, 16>(g, b, wl, count, work_acc); break;
      case 32: color_chunk_group<MODE, 32>(g, b, wl, count, work_acc); break;
      default: color_chunk_group<MODE, 64>(g, b, wl, count, work_acc); break;
    }
  }
  // heavy bins: units taken dynamically
  if (M.heavy_total > 0) {
    while (true) {
      if (threadIdx.x == 0) s_unit = atomicAdd(&b.tile_ctr[0], 1);
      __syncthreads();
      const int32_t u = s_unit;
      __syncthreads();
      if (u >= M.heavy_total) break;
      if (u < M.heavy_block) {
        const int32_t v = ld_dev(&b.wl_in[L.off[kBlockBin] + u]);
        color_vertex_block<MODE>(g, b, v, ovf, red, &s_misc[0]);
        if (threadIdx.x == 0) work_acc += static_cast<uint64_t>(ld_dev(&b.work[v]));
      } else {
        const int32_t us = u - M.heavy_block;
        const int32_t si = ld_dev(&b.wl_in[L.off[kSplitBin] + us / L.split_chunks]);
        color_split_chunk<MODE>(g, b, L, si, us % L.split_chunks, ovf, red, s_misc, work_acc);
      }
    }
  }
  work_acc = wave_sum_u64(work_acc);
  if (lane_id() == 0 && work_acc) atomicAdd(&s_work, static_cast<unsigned long long>(work_acc));
  __syncthreads();
  if (threadIdx.x == 0 && s_work) atomicAdd(&b.visits[1], s_work);
}

template <int MODE>
__device__ void detect_split_chunk(const GraphView& g, const KeySource& k, const RoundBufs& b,
                                   const BinLayout& L, int32_t si, int chunk, int32_t* s_misc,
                                   int32_t& maxc_acc) {
  const int tid = threadIdx.x;
  const int nch = L.split_chunks;
  const int32_t v = ld_dev(&b.split_vertex[si]);
  const int32_t rb = g.rp[v], re = g.rp[v + 1];
  const int64_t len = re - rb;
  const int32_t cb = rb + static_cast<int32_t>(len * chunk / nch);
  const int32_t ce = rb + static_cast<int32_t>(len * (chunk + 1) / nch);
  const int32_t* __restrict__ T = b.T;
  const int32_t tv = ld_dev(&T[v]);
  const uint64_t kv = key_of(k, v);
  bool lose = false;
  if (atomic_load_u32(&b.split_flag[si]) == 0u) {  // another chunk may already have decided
    scan_nbhd<MODE>(g, v, cb, ce, tid, kBlock, [&](int32_t u) {
      if (key_of(k, u) > kv && ld_dev(&T[u]) == tv) {
        lose = true;
        return true;
      }
      return false;
    });
  }
  lose = __syncthreads_or(lose);
  if (tid == 0 && lose) atomicOr(&b.split_flag[si], 1u);
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const bool last = atomicAdd(&b.split_ctr[si], 1u) == static_cast<uint32_t>(nch - 1);
    if (last) {
      __threadfence();
      const uint32_t f = atomic_load_u32(&b.split_flag[si]);
      if (!f) {
        st_dev(&b.C[v], tv);
        maxc_acc = max(maxc_acc, tv);
      } else {
        const int32_t pos = atomicAdd(&b.cnt_out[kSplitBin], 1);
        st_dev(&b.wl_out[L.off[kSplitBin] + pos], si);
      }
      atomic_reset_u32(&b.split_flag[si]);
      atomic_reset_u32(&b.split_ctr[si]);
    }
  }
  __syncthreads();
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void detect_round_kernel(GraphView g, KeySource k, RoundBufs b,
                                                              BinLayout L, int round) {
  __shared__ int32_t s_misc[4];
  __shared__ int32_t s_unit;
  __shared__ int32_t s_max;
  __shared__ int32_t s_ent[kBlock];
  __shared__ int32_t s_wc[kWavesPerBlock + 1];
  __shared__ RoundMap M;
  (void)round;
  if (threadIdx.x == 0) {
    make_round_map(b, L, M);
    s_max = 0;
    if (blockIdx.x == 0) atomic_reset_i32(&b.tile_ctr[0]);
  }
  __syncthreads();
  int32_t maxc_acc = 0;
  const int32_t lb = xcd_logical_block();
  const int32_t c0 = static_cast<int32_t>(static_cast<int64_t>(lb) * M.light_total / gridDim.x);
  const int32_t c1 = static_cast<int32_t>(static_cast<int64_t>(lb + 1) * M.light_total / gridDim.x);
  for (int32_t c = c0; c < c1; ++c) {
    int bin;
    int32_t first, count;
    light_chunk(M, c, bin, first, count);
    const int32_t* wl = b.wl_in + L.off[bin] + first;
    const int32_t oo = L.off[bin];
    switch (L.lanes[bin]) {
      case 1: detect_chunk_group<MODE, 1>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
      case 2: detect_chunk_group<MODE, 2>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
      case 4: detect_chunk_group<MODE, 4>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
      case 8: detect_chunk_group<MODE, 8>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
      case 16: detect_chunk_group<MODE, 16>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
      case 32: detect_chunk_group<MODE, 32>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
      default: detect_chunk_group<MODE, 64>(g, k, b, bin, wl, count, oo, s_ent, s_wc, maxc_acc); break;
    }
  }
  if (M.heavy_total > 0) {
    while (true) {
      if (threadIdx.x == 0) s_unit = atomicAdd(&b.tile_ctr[1], 1);
      __syncthreads();
      const int32_t u = s_unit;
      __syncthreads();
      if (u >= M.heavy_total) break;
      if (u < M.heavy_block) {
        const int32_t v = ld_dev(&b.wl_in[L.off[kBlockBin] + u]);
        detect_vertex_block<MODE>(g, k, b, v, L.off[kBlockBin], maxc_acc);
      } else {
        const int32_t us = u - M.heavy_block;
        const int32_t si = ld_dev(&b.wl_in[L.off[kSplitBin] + us / L.split_chunks]);
        detect_split_chunk<MODE>(g, k, b, L, si, us % L.split_chunks, s_misc, maxc_acc);
      }
    }
  }
  maxc_acc = wave_max_i32(maxc_acc);
  if (lane_id() == 0 && maxc_acc > 0) atomicMax(&s_max, maxc_acc);
  __syncthreads();
  if (threadIdx.x == 0 && s_max > 0) atomicMax(b.maxc, s_max);
}

template <int MODE>
static int resident_blocks_of() {
  int dev = 0, cus = 0, a = 0, d = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2048;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2048;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, color_round_kernel<MODE>, kBlock, 0) != hipSuccess)
    return 2048;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&d, detect_round_kernel<MODE>, kBlock, 0) != hipSuccess)
    return 2048;
  const int per_cu = std::max(1, std::min(a, d));
  return std::max(8, (per_cu * cus) / 8 * 8);
}

int resident_round_blocks(int mode) {
  static int cache[4] = {0, 0, 0, 0};
  if (mode < 1 || mode > 3) return 2048;
  if (cache[mode] == 0) {
    cache[mode] = mode == kD1 ? resident_blocks_of<kD1>()
                  : mode == kD2 ? resident_blocks_of<kD2>()
                                : resident_blocks_of<kPD2>();
  }
  return cache[mode];
}

template <int MODE>
void launch_color_round(const GraphView& g, const KeySource& k, const RoundBufs& b,
                        const BinLayout& L, int round, int grid, hipStream_t st) {
  hipLaunchKernelGGL(color_round_kernel<MODE>, dim3(grid), dim3(kBlock), 0, st, g, k, b, L, round);
}

template <int MODE>
void launch_detect_round(const GraphView& g, const KeySource& k, const RoundBufs& b,
                         const BinLayout& L, int round, int grid, hipStream_t st) {
  hipLaunchKernelGGL(detect_round_kernel<MODE>, dim3(grid), dim3(kBlock), 0, st, g, k, b, L, round);
}

template void launch_color_round<kD1>(const GraphView&, const KeySource&, const RoundBufs&,
                                      const BinLayout&, int, int, hipStream_t);
template void launch_color_round<kD2>(const GraphView&, const KeySource&, const RoundBufs&,
                                      const BinLayout&, int, int, hipStream_t);
template void launch_color_round<kPD2>(const GraphView&, const KeySource&, const RoundBufs&,
                                       const BinLayout&, int, int, hipStream_t);
template void launch_detect_round<kD1>(const GraphView&, const KeySource&, const RoundBufs&,
                                       const BinLayout&, int, int, hipStream_t);
template void launch_detect_round<kD2>(const GraphView&, const KeySource&, const RoundBufs&,
                                       const BinLayout&, int, int, hipStream_t);
template void launch_detect_round<kPD2>(const GraphView&, const KeySource&, const RoundBufs&,
                                        const BinLayout&, int, int, hipStream_t);

}  // namespace gcol
