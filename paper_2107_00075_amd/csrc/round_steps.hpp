// Per-vertex steps of one round, shared by the per-graph round kernels and
// the batched persistent kernel: the neighbourhood walk, the first-fit color
// step for a group of G lanes or a whole workgroup, and the detect + commit +
// compact step (Section 3.2, Algorithms 2-4; Section 2.1 and Algorithm 5
// for the distance-2 and partial distance-2 neighbourhoods).
#pragma once

#include <climits>

#include "rounds.hpp"

namespace gcol {

// Loads of the graph arrays.  LD = 0: plain loads (arrays written before the
// call and never rewritten during it).  LD = 1: device-scope loads, for
// graphs whose memory is rewritten by copies between launches of the same
// library instance (the served form's arena), where an XCD's L2 could still
// hold lines of the previous contents.
template <int LD, typename X>
__device__ __forceinline__ X gld(const X* p) {
  if constexpr (LD != 0) return ld_dev(p);
  else return *p;
}

// Visits the neighbourhood entries of v reachable from hop-1 positions
// [beg, end) with lane stride (sub, stride).  f(u) returns true to stop.
template <int MODE, int LD = 0, typename F>
__device__ __forceinline__ void scan_nbhd(const GraphView& g, int32_t v, int32_t beg, int32_t end,
                                          int sub, int stride, F&& f) {
  for (int32_t e = beg + sub; e < end; e += stride) {
    const int32_t u = gld<LD>(&g.ci[e]);
    if (MODE == kD1) {
      if (u < g.limit && f(u)) return;
    } else {
      if (MODE == kD2) {
        if (f(u)) return;
      }
      const int32_t b2 = gld<LD>(&g.rp2[u]), e2 = gld<LD>(&g.rp2[u + 1]);
      for (int32_t q = b2; q < e2; ++q) {
        const int32_t x = gld<LD>(&g.ci2[q]);
        if (x != v && f(x)) return;
      }
    }
  }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t x) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) x = max(x, __shfl_xor(x, off, kWave));
  return x;
}

// ---------------------------------------------------------------------------
// color: group of G lanes per vertex, one chunk of kBlock worklist entries
// ---------------------------------------------------------------------------
template <int MODE, int G, int LD = 0>
__device__ __forceinline__ void color_chunk_group(const GraphView& g, const RoundBufs& b, const int32_t* wl, int32_t count,
                                  uint64_t& work_acc) {
  constexpr int per_pass = kBlock / G;
  const int gi = threadIdx.x / G;
  const int sub = threadIdx.x % G;
  const int32_t* __restrict__ C = b.C;
  for (int32_t idx = gi; idx < count; idx += per_pass) {  // whole groups stay together
    const int32_t v = ld_dev(&wl[idx]);
    const int32_t beg = gld<LD>(&g.rp[v]), end = gld<LD>(&g.rp[v + 1]);
    int32_t base = 1;
    while (true) {
      uint64_t m = 0;
      scan_nbhd<MODE, LD>(g, v, beg, end, sub, G, [&](int32_t u) {
        const uint32_t d = static_cast<uint32_t>(ld_dev(&C[u]) - base);
        if (d < 64u) m |= 1ull << d;
        return false;
      });
      m = group_or<G>(m);
      if (m != ~0ull) {
        if (sub == 0) st_dev(&b.T[v], base + static_cast<int32_t>(__builtin_ctzll(~m)));
        break;
      }
      base += 64;
    }
    if (sub == 0) work_acc += static_cast<uint64_t>(ld_dev(&b.work[v]));
  }
}

// ---------------------------------------------------------------------------
// color: one workgroup per vertex
// ---------------------------------------------------------------------------
template <int MODE, int LD = 0>
__device__ __forceinline__ void color_vertex_block(const GraphView& g, const RoundBufs& b, int32_t v,
                                   uint32_t* ovf, uint64_t* red, int32_t* s_min) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int32_t beg = gld<LD>(&g.rp[v]), end = gld<LD>(&g.rp[v + 1]);
  const int32_t* __restrict__ C = b.C;
  int32_t base = 1;
  while (true) {
    for (int w = tid; w < kOvfWords; w += kBlock) ovf[w] = 0u;
    if (tid == 0) *s_min = INT_MAX;
    __syncthreads();
    uint64_t m = 0;
    scan_nbhd<MODE, LD>(g, v, beg, end, tid, kBlock, [&](int32_t u) {
      uint32_t d = static_cast<uint32_t>(ld_dev(&C[u]) - base);
      if (d < 64u) {
        m |= 1ull << d;
      } else {
        d -= 64u;
        if (d < static_cast<uint32_t>(kOvfWords * 32)) atomicOr(&ovf[d >> 5], 1u << (d & 31u));
      }
      return false;
    });
    m = group_or<kWave>(m);
    if (lane_id() == 0) red[wave] = m;
    __syncthreads();
    m = red[0] | red[1] | red[2] | red[3];
    int32_t mex = -1;
    if (m != ~0ull) {
      mex = base + __builtin_ctzll(~m);
    } else {
      for (int w = tid; w < kOvfWords; w += kBlock) {
        const uint32_t x = ovf[w];
        if (x != ~0u) {
          atomicMin(s_min, w * 32 + __builtin_ctz(~x));
          break;
        }
      }
      __syncthreads();
      if (*s_min != INT_MAX) mex = base + 64 + *s_min;
    }
    __syncthreads();
    if (mex > 0) {
      if (tid == 0) st_dev(&b.T[v], mex);
      return;
    }
    base += 64 + kOvfWords * 32;
  }
}

// ---------------------------------------------------------------------------
// detect + commit + compact: group of G lanes per vertex, one chunk
// ---------------------------------------------------------------------------
// Losers of the chunk are collected in LDS and appended to W_{r+1} with one
// device atomic per chunk (workgroup prefix over the wavefront ballots).
template <int MODE, int G, int LD = 0>
__device__ __forceinline__ void detect_chunk_group(const GraphView& g, const KeySource& k, const RoundBufs& b, int bin,
                                   const int32_t* wl, int32_t count, int32_t off_out, int32_t* s_ent,
                                   int32_t* s_wc, int32_t& maxc_acc) {
  constexpr int per_pass = kBlock / G;
  const int gi = threadIdx.x / G;
  const int sub = threadIdx.x % G;
  const int32_t* __restrict__ T = b.T;
  for (int32_t idx = gi; idx < count; idx += per_pass) {
    const int32_t v = ld_dev(&wl[idx]);
    const int32_t tv = ld_dev(&T[v]);
    const uint64_t kv = key_of(k, v);
    bool lose = false;
    scan_nbhd<MODE, LD>(g, v, gld<LD>(&g.rp[v]), gld<LD>(&g.rp[v + 1]), sub, G, [&](int32_t u) {
      if (key_of(k, u) > kv && ld_dev(&T[u]) == tv) {  // keys first: only higher keys can win
        lose = true;
        return true;
      }
      return false;
    });
    lose = group_any<G>(lose);
    if (sub == 0) {
      if (lose) {
        s_ent[idx] = v;
      } else {
        s_ent[idx] = -1;
        st_dev(&b.C[v], tv);
        maxc_acc = max(maxc_acc, tv);
      }
    }
  }
  __syncthreads();
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int32_t x = tid < count ? s_ent[tid] : -1;
  const uint64_t bal = __ballot(x >= 0);
  if (lane_id() == 0) s_wc[wave] = static_cast<int32_t>(__popcll(bal));
  __syncthreads();
  if (tid == 0) {
    int32_t tot = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      const int32_t c = s_wc[w];
      s_wc[w] = tot;
      tot += c;
    }
    s_wc[kWavesPerBlock] = tot ? atomicAdd(&b.cnt_out[bin], tot) : 0;
  }
  __syncthreads();
  if (x >= 0) st_dev(&b.wl_out[off_out + s_wc[kWavesPerBlock] + s_wc[wave] + static_cast<int32_t>(lanes_below(bal))], x);
  __syncthreads();
}

template <int MODE, int LD = 0>
__device__ __forceinline__ void detect_vertex_block(const GraphView& g, const KeySource& k, const RoundBufs& b,
                                    int32_t v, int32_t off, int32_t& maxc_acc) {
  const int tid = threadIdx.x;
  const int32_t* __restrict__ T = b.T;
  const int32_t tv = ld_dev(&T[v]);
  const uint64_t kv = key_of(k, v);
  bool lose = false;
  scan_nbhd<MODE, LD>(g, v, gld<LD>(&g.rp[v]), gld<LD>(&g.rp[v + 1]), tid, kBlock, [&](int32_t u) {
    if (key_of(k, u) > kv && ld_dev(&T[u]) == tv) {  // keys first: only higher keys can win
      lose = true;
      return true;
    }
    return false;
  });
  lose = __syncthreads_or(lose);
  if (tid == 0) {
    if (!lose) {
      st_dev(&b.C[v], tv);
      maxc_acc = max(maxc_acc, tv);
    } else {
      const int32_t pos = atomicAdd(&b.cnt_out[kBlockBin], 1);
      st_dev(&b.wl_out[off + pos], v);
    }
  }
}

}  // namespace gcol
