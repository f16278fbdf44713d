// Per-call setup kernels: static work and degree bins, initial worklists,
// input-contract validation, the priority hash, and the boundary phase of the
// ghost-layer variant.
#include <algorithm>
#include <climits>

#include "inc.hpp"
#include "setup.hpp"

namespace gcol {

// Adjacency entries one visit of v reads: D1 deg(v); D2 sum over u in N(v)
// of 1 + deg(u); PD2 sum over the rows r of column v of 1 + deg(r) (the
// row entry of the CSC, then the row's columns in the CSR).
template <int MODE>
__device__ __forceinline__ int64_t vertex_work(const GraphView& g, int32_t v) {
  const int32_t b = g.rp[v], e = g.rp[v + 1];
  if (MODE == kD1) return e - b;
  int64_t w = 0;
  for (int32_t q = b; q < e; ++q) {
    const int32_t u = g.ci[q];
    w += 1 + (g.rp2[u + 1] - g.rp2[u]);
  }
  return w;
}

// Bookkeeping of one vertex once its work is known: work, bin, initial colors,
// per-bin counts and the maxima the driver needs.  Called by whole wavefronts
// (wavefront reductions, one atomic per wavefront and quantity).
__device__ void account_vertex(const BinSetup& s, int32_t v, int64_t w, bool active) {
  int bin = -1;
  int32_t c = 0;
  if (active) {
    const int32_t wc = static_cast<int32_t>(w > INT_MAX ? INT_MAX : w);
    st_dev(&s.work[v], wc);
    bin = kBins - 1;
    for (int i = 0; i < kBins - 1; ++i) {
      if (wc <= s.bin_hi[i]) {
        bin = i;
        break;
      }
    }
    st_dev(&s.bin[v], static_cast<int8_t>(bin));
    c = s.init ? ld_dev(&s.init[v]) : 0;
    st_dev(&s.C[v], c);
    st_dev(&s.T[v], c);
  }
  int32_t cmax = c;
  int32_t smax = (active && bin == kSplitBin && c == 0) ? static_cast<int32_t>(w > INT_MAX ? INT_MAX : w) : 0;
  int32_t wmax = (active && c == 0) ? static_cast<int32_t>(w > INT_MAX ? INT_MAX : w) : 0;
  uint64_t wsum = (active && c == 0) ? static_cast<uint64_t>(w) : 0ull;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    cmax = max(cmax, __shfl_xor(cmax, off, kWave));
    smax = max(smax, __shfl_xor(smax, off, kWave));
    wmax = max(wmax, __shfl_xor(wmax, off, kWave));
    wsum += __shfl_xor(wsum, off, kWave);
  }
  if (lane_id() == 0) {
    if (cmax > 0) atomicMax(s.maxc, cmax);
    if (smax > 0) atomicMax(s.max_split_work, smax);
    if (wmax > 0) atomicMax(s.max_work, wmax);
    if (wsum) atomicAdd(s.total_work, static_cast<unsigned long long>(wsum));
  }
  for (int i = 0; i < kBins; ++i) {
    const uint64_t all = __ballot(active && bin == i);
    const uint64_t unc = __ballot(active && bin == i && c == 0);
    if (lane_id() == 0) {
      if (all) atomicAdd(&s.count_all[i], static_cast<int32_t>(__popcll(all)));
      if (unc) atomicAdd(&s.count_unc[i], static_cast<int32_t>(__popcll(unc)));
    }
  }
}

// Per-call totals of the vertices one thread records, flushed once per
// workgroup (a handful of device atomics per workgroup instead of per
// wavefront).
struct BinAcc {
  int32_t cmax = 0, smax = 0, wmax = 0;
  uint64_t wsum = 0;
  int32_t all[kBins] = {0, 0, 0, 0, 0};
  int32_t unc[kBins] = {0, 0, 0, 0, 0};
};

__device__ __forceinline__ void record_vertex(const BinSetup& s, int32_t v, int64_t w, BinAcc& a) {
  const int32_t wc = static_cast<int32_t>(w > INT_MAX ? INT_MAX : w);
  st_dev(&s.work[v], wc);
  int bin = kBins - 1;
  for (int i = 0; i < kBins - 1; ++i) {
    if (wc <= s.bin_hi[i]) {
      bin = i;
      break;
    }
  }
  st_dev(&s.bin[v], static_cast<int8_t>(bin));
  const int32_t c = s.init ? ld_dev(&s.init[v]) : 0;
  st_dev(&s.C[v], c);
  st_dev(&s.T[v], c);
  a.cmax = max(a.cmax, c);
  if (c == 0) {
    if (bin == kSplitBin) a.smax = max(a.smax, wc);
    a.wmax = max(a.wmax, wc);
    a.wsum += static_cast<uint64_t>(w);
  }
#pragma unroll
  for (int i = 0; i < kBins; ++i) {
    a.all[i] += bin == i ? 1 : 0;
    a.unc[i] += (bin == i && c == 0) ? 1 : 0;
  }
}

__device__ void flush_acc(const BinSetup& s, BinAcc& a) {
  __shared__ int32_t s_i[3 + 2 * kBins];
  __shared__ unsigned long long s_sum;
  const int tid = threadIdx.x;
  if (tid < 3 + 2 * kBins) s_i[tid] = 0;
  if (tid == 0) s_sum = 0ull;
  __syncthreads();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    a.cmax = max(a.cmax, __shfl_xor(a.cmax, off, kWave));
    a.smax = max(a.smax, __shfl_xor(a.smax, off, kWave));
    a.wmax = max(a.wmax, __shfl_xor(a.wmax, off, kWave));
    a.wsum += __shfl_xor(a.wsum, off, kWave);
#pragma unroll
    for (int i = 0; i < kBins; ++i) {
      a.all[i] += __shfl_xor(a.all[i], off, kWave);
      a.unc[i] += __shfl_xor(a.unc[i], off, kWave);
    }
  }
  if (lane_id() == 0) {
    atomicMax(&s_i[0], a.cmax);
    atomicMax(&s_i[1], a.smax);
    atomicMax(&s_i[2], a.wmax);
    for (int i = 0; i < kBins; ++i) {
      atomicAdd(&s_i[3 + i], a.all[i]);
      atomicAdd(&s_i[3 + kBins + i], a.unc[i]);
    }
    if (a.wsum) atomicAdd(&s_sum, static_cast<unsigned long long>(a.wsum));
  }
  __syncthreads();
  if (tid == 0) {
    if (s_i[0] > 0) atomicMax(s.maxc, s_i[0]);
    if (s_i[1] > 0) atomicMax(s.max_split_work, s_i[1]);
    if (s_i[2] > 0) atomicMax(s.max_work, s_i[2]);
    if (s_sum) atomicAdd(s.total_work, s_sum);
  } else if (tid <= kBins) {
    const int i = tid - 1;
    if (s_i[3 + i]) atomicAdd(&s.count_all[i], s_i[3 + i]);
    if (s_i[3 + kBins + i]) atomicAdd(&s.count_unc[i], s_i[3 + kBins + i]);
  }
}

// A grid-stride loop, one thread per vertex.  D2/PD2 vertices whose first
// hop is longer than kSetupHeavy entries are deferred to heavy_work_kernel
// (a workgroup each).
template <int MODE>
__global__ __launch_bounds__(kBlock) void bin_kernel(GraphView g, BinSetup s) {
  BinAcc acc;
  const int32_t stride = gridDim.x * kBlock;
  for (int32_t base = blockIdx.x * kBlock; base < g.n; base += stride) {
    const int32_t v = base + threadIdx.x;
    bool active = v < g.n;
    bool defer = false;
    if (MODE != kD1 && active) defer = g.rp[v + 1] - g.rp[v] > kSetupHeavy;
    const uint64_t dbal = __ballot(defer);
    if (dbal) {
      const int first = __builtin_ctzll(dbal);
      int32_t b0 = 0;
      if (lane_id() == first) b0 = atomicAdd(s.deferred_cnt, static_cast<int32_t>(__popcll(dbal)));
      b0 = __shfl(b0, first, kWave);
      if (defer) {
        const int32_t di = b0 + static_cast<int32_t>(lanes_below(dbal));
        st_dev(&s.deferred[di], v);
        st_dev(&s.deferred_work[di], 0ull);
        st_dev(&s.deferred_done[di], 0);
      }
    }
    active = active && !defer;
    if (active) record_vertex(s, v, vertex_work<MODE>(g, v), acc);
  }
  flush_acc(s, acc);
}

// Deferred heavy vertices: each is cut into kHeavySlices equal ranges of its
// first hop, handed out as units; a unit's workgroup adds its range's
// contributions to the vertex's sum, and the workgroup that completes the
// last range records the vertex.  (One workgroup per vertex left the
// longest first hop on one workgroup: 2.6 ms on the 4M x 1M PD2 pattern.)
constexpr int kHeavySlices = 16;

template <int MODE>
__global__ __launch_bounds__(kBlock) void heavy_work_kernel(GraphView g, BinSetup s) {
  __shared__ int32_t s_u, s_last;
  __shared__ unsigned long long s_sum;
  const int32_t nd = ld_dev(s.deferred_cnt);
  const int64_t units = static_cast<int64_t>(nd) * kHeavySlices;
  while (true) {
    if (threadIdx.x == 0) {
      s_u = atomicAdd(s.deferred_grab, 1);
      s_sum = 0ull;
    }
    __syncthreads();
    const int32_t u = s_u;
    if (u >= units) break;
    const int32_t i = u / kHeavySlices, j = u % kHeavySlices;
    const int32_t v = ld_dev(&s.deferred[i]);
    const int32_t q0 = g.rp[v], len = g.rp[v + 1] - q0;
    const int32_t a = q0 + static_cast<int32_t>(static_cast<int64_t>(len) * j / kHeavySlices);
    const int32_t z = q0 + static_cast<int32_t>(static_cast<int64_t>(len) * (j + 1) / kHeavySlices);
    uint64_t w = 0;
    for (int32_t q = a + static_cast<int32_t>(threadIdx.x); q < z; q += kBlock) {
      const int32_t x = g.ci[q];
      w += 1 + static_cast<uint64_t>(g.rp2[x + 1] - g.rp2[x]);
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) w += __shfl_xor(w, off, kWave);
    if (lane_id() == 0 && w) atomicAdd(&s_sum, static_cast<unsigned long long>(w));
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_sum) atomicAdd(&s.deferred_work[i], s_sum);
      __threadfence();
      s_last = atomicAdd(&s.deferred_done[i], 1) == kHeavySlices - 1 ? 1 : 0;
      __threadfence();
    }
    __syncthreads();
    if (s_last && threadIdx.x < kWave)
      account_vertex(s, v, static_cast<int64_t>(ld_dev(&s.deferred_work[i])), threadIdx.x == 0);
    __syncthreads();
  }
}

// Appends every uncolored vertex (C[v] == 0) to its bin's region of the
// worklist; split vertices get a split index (their position in the split
// region) and the region holds indices.  Each workgroup owns a contiguous
// range of per_block vertices: it counts its vertices per bin, reserves its
// slots with one device atomic per bin, then writes them.
__global__ __launch_bounds__(kBlock) void scatter_kernel(int32_t n, const int32_t* C, const int8_t* binv,
                                                         BinLayout L, int32_t* wl, int32_t* cnt,
                                                         int32_t* split_vertex, int32_t per_block) {
  __shared__ int32_t s_cnt[kBins][kWavesPerBlock];
  __shared__ int32_t s_next[kBins];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int32_t lo = blockIdx.x * per_block;
  const int32_t hi = min(n, lo + per_block);
  int32_t my[kBins] = {0, 0, 0, 0, 0};
  for (int32_t v = lo + tid; v < hi; v += kBlock) {
    const bool active = ld_dev(&C[v]) == 0;
    const int bin = active ? static_cast<int>(ld_dev(&binv[v])) : -1;
#pragma unroll
    for (int i = 0; i < kBins; ++i) my[i] += bin == i ? 1 : 0;
  }
#pragma unroll
  for (int i = 0; i < kBins; ++i) {
    int32_t x = my[i];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) x += __shfl_xor(x, off, kWave);
    if (lane_id() == 0) s_cnt[i][wave] = x;
  }
  __syncthreads();
  if (tid < kBins) {
    int32_t tot = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) tot += s_cnt[tid][w];
    s_next[tid] = tot ? atomicAdd(&cnt[tid], tot) : 0;
  }
  __syncthreads();
  for (int32_t base = lo; base < hi; base += kBlock) {
    const int32_t v = base + tid;
    const bool active = v < hi && ld_dev(&C[v]) == 0;
    const int bin = active ? static_cast<int>(ld_dev(&binv[v])) : -1;
    int32_t rank = 0;
#pragma unroll
    for (int i = 0; i < kBins; ++i) {
      const uint64_t bal = __ballot(bin == i);
      if (bin == i) rank = static_cast<int32_t>(lanes_below(bal));
      if (lane_id() == 0) s_cnt[i][wave] = static_cast<int32_t>(__popcll(bal));
    }
    __syncthreads();
    if (active) {
      int32_t pos = s_next[bin] + rank;
      for (int w = 0; w < wave; ++w) pos += s_cnt[bin][w];
      if (bin == kSplitBin) {
        st_dev(&split_vertex[pos], v);
        st_dev(&wl[L.off[bin] + pos], pos);
      } else {
        st_dev(&wl[L.off[bin] + pos], v);
      }
    }
    __syncthreads();
    if (tid < kBins) {
      int32_t tot = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) tot += s_cnt[tid][w];
      s_next[tid] += tot;
    }
    __syncthreads();
  }
}

__device__ void validate_row(int32_t v, int32_t n_cols, const int32_t* rp, const int32_t* ci,
                             const int32_t* rpT, const int32_t* ciT, int32_t n_trows, int square,
                             int32_t* err);

// Input contract (COLOR_FLAG_VALIDATE).  Rows strictly increasing, ids in
// range, no self-loops when `square`, and every entry (v, u) mirrored as
// (u, v) in the transpose arrays (rpT, ciT) — for D1/D2 the adjacency itself,
// for PD2 the CSC of the same pattern.
__global__ __launch_bounds__(kBlock) void validate_kernel(int32_t n_rows, int32_t n_cols, const int32_t* rp,
                                                          const int32_t* ci, const int32_t* rpT,
                                                          const int32_t* ciT, int32_t n_trows, int square,
                                                          int32_t* err) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n_rows) validate_row(v, n_cols, rp, ci, rpT, ciT, n_trows, square, err);
}

__device__ void validate_row(int32_t v, int32_t n_cols, const int32_t* rp, const int32_t* ci,
                             const int32_t* rpT, const int32_t* ciT, int32_t n_trows, int square,
                             int32_t* err) {
  const int32_t b = rp[v], e = rp[v + 1];
  if (b > e) {
    atomicOr(err, 1);
    return;
  }
  int32_t prev = -1;
  for (int32_t q = b; q < e; ++q) {
    const int32_t u = ci[q];
    if (u < 0 || u >= n_cols) {
      atomicOr(err, 2);
      return;
    }
    if (u <= prev) atomicOr(err, 4);
    if (square && u == v) atomicOr(err, 8);
    prev = u;
    if (u >= n_trows) continue;  // no transpose row for u (e.g. a ghost without a row)
    // binary search v in the transpose row of u
    int32_t lo = rpT[u], hi = rpT[u + 1] - 1;
    bool found = false;
    while (lo <= hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      const int32_t x = ciT[mid];
      if (x == v) {
        found = true;
        break;
      }
      if (x < v) lo = mid + 1;
      else hi = mid - 1;
    }
    if (!found) atomicOr(err, 16);
  }
}

__global__ __launch_bounds__(kBlock) void check_rowptr_kernel(int32_t n, const int32_t* rp, int32_t* err) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v == 0 && rp[0] != 0) atomicOr(err, 1);
  if (v < n && rp[v] > rp[v + 1]) atomicOr(err, 1);
}

__global__ __launch_bounds__(kBlock) void priority_kernel(int32_t n, const int32_t* gid, uint32_t hs,
                                                          uint32_t* out) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const uint32_t g = gid ? static_cast<uint32_t>(gid[i]) : static_cast<uint32_t>(i);
    st_dev(&out[i], fmix32(g ^ hs));
  }
}

// Ghost phase 2 (Algorithm 3 with Algorithm 4 on the ghosts' fixed colors):
// every owned-ghost edge with equal colors is a conflict; the owned endpoint
// loses when the ghost's key is greater, otherwise the ghost is flagged.  All
// pairs are judged on the phase-1 colors (a thread per owned-row entry, so a
// hub's row spreads over many threads); losers are uncolored afterwards by
// boundary_uncolor_kernel.  loser must be zeroed first.

__global__ __launch_bounds__(kBlock) void boundary_kernel(int32_t n_owned, const int32_t* rp,
                                                          const int32_t* ci, const int32_t* C,
                                                          const int32_t* ghost_colors, KeySource k,
                                                          int32_t* loser, int32_t* gflag,
                                                          unsigned long long* conflicts) {
  const int32_t e = blockIdx.x * kBlock + threadIdx.x;
  uint32_t found = 0;
  if (e < rp[n_owned]) {
    const int32_t u = ci[e];
    if (u >= n_owned) {
      const int32_t v = row_of(rp, n_owned, e);
      if (ghost_colors[u - n_owned] == ld_dev(&C[v])) {
        found = 1;
        if (key_of(k, u) > key_of(k, v)) st_dev(&loser[v], 1);
        else st_dev(&gflag[u - n_owned], 1);
      }
    }
  }
  const uint64_t tot = __popcll(__ballot(found != 0));
  if (lane_id() == 0 && tot) atomicAdd(conflicts, static_cast<unsigned long long>(tot));
}

// Distance-2 / partial distance-2 ghost phase 2 (Algorithm 5 over the owned
// vertices): every owned vertex's two-hop walk is compared with the ghosts'
// fixed colors, a thread per hop-1 entry (u) walking u itself (D2) and u's
// hop-2 row, so heavy vertices spread over many threads.  A conflicting
// ghost x of v makes v lose (key(x) > key(v)) or flags x; both are
// idempotent, so the walk's repeated entries do not matter to them.  The
// count is of distinct (v, x) pairs: pass 1 counts the conflicting entries,
// pass 2 inserts them into an open-addressing set of (v, x) keys sized for
// them and counts the insertions that found an empty slot.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void boundary2_kernel(GraphView g, int32_t n_owned, const int32_t* C,
                                                           const int32_t* ghost_colors, KeySource k, int32_t* loser,
                                                           int32_t* gflag, unsigned long long* hits,
                                                           unsigned long long* set, uint64_t set_mask,
                                                           unsigned long long* conflicts) {
  const int32_t e = blockIdx.x * kBlock + threadIdx.x;
  const int32_t nnz1 = g.rp[n_owned];
  uint64_t n_hit = 0, n_new = 0;
  if (e < nnz1) {
    const int32_t v = row_of(g.rp, n_owned, e);
    const int32_t cv = ld_dev(&C[v]);
    const int32_t u = g.ci[e];
    auto visit = [&](int32_t x) {
      if (x < n_owned || x == v || ghost_colors[x - n_owned] != cv) return;
      ++n_hit;
      if (key_of(k, x) > key_of(k, v)) st_dev(&loser[v], 1);
      else st_dev(&gflag[x - n_owned], 1);
      if (set) {
        const unsigned long long pair = (static_cast<unsigned long long>(v) << 32) | static_cast<uint32_t>(x);
        for (uint64_t h = mix64(pair) & set_mask;; h = (h + 1) & set_mask) {
          const unsigned long long was = atomicCAS(&set[h], ~0ull, pair);
          if (was == ~0ull) {
            ++n_new;
            break;
          }
          if (was == pair) break;
        }
      }
    };
    if (MODE == kD2) visit(u);
    for (int32_t q = g.rp2[u]; q < g.rp2[u + 1]; ++q) visit(g.ci2[q]);
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    n_hit += __shfl_xor(n_hit, off, kWave);
    n_new += __shfl_xor(n_new, off, kWave);
  }
  if (lane_id() == 0) {
    if (n_hit) atomicAdd(hits, static_cast<unsigned long long>(n_hit));
    if (n_new) atomicAdd(conflicts, static_cast<unsigned long long>(n_new));
  }
}

__global__ __launch_bounds__(kBlock) void fill_u64_kernel(unsigned long long* p, uint64_t n, unsigned long long x) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = x;
}

__global__ __launch_bounds__(kBlock) void boundary_uncolor_kernel(int32_t n_owned, const int32_t* loser,
                                                                  int32_t* C) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n_owned && ld_dev(&loser[v])) st_dev(&C[v], 0);
}

// Ghost colors become fixed committed colors for phase 3.
__global__ __launch_bounds__(kBlock) void ghost_fill_kernel(int32_t n_owned, int32_t n_ghost,
                                                            const int32_t* ghost_colors, int32_t* C,
                                                            int32_t* T, int32_t* maxc) {
  const int32_t j = blockIdx.x * kBlock + threadIdx.x;
  int32_t c = 0;
  if (j < n_ghost) {
    c = ghost_colors[j];
    st_dev(&C[n_owned + j], c);
    st_dev(&T[n_owned + j], c);
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) c = max(c, __shfl_xor(c, off, kWave));
  if (lane_id() == 0 && c > 0) atomicMax(maxc, c);
}

// Largest value of an int32 array (wave-reduced, one atomic per wavefront).
__global__ __launch_bounds__(kBlock) void max_i32_kernel(int32_t n, const int32_t* a, int32_t* out) {
  int32_t x = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    x = max(x, ld_dev(&a[i]));
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) x = max(x, __shfl_xor(x, off, kWave));
  if (lane_id() == 0 && x > 0) atomicMax(out, x);
}

__global__ __launch_bounds__(kBlock) void flags_out_kernel(int32_t n, const int32_t* gflag, uint8_t* out,
                                                           unsigned long long* count) {
  const int32_t j = blockIdx.x * kBlock + threadIdx.x;
  const bool f = j < n && ld_dev(&gflag[j]) != 0;
  if (j < n && out) out[j] = f ? 1 : 0;
  const uint64_t bal = __ballot(f);
  if (lane_id() == 0 && bal) atomicAdd(count, static_cast<unsigned long long>(__popcll(bal)));
}

__global__ __launch_bounds__(kBlock) void copy_i32_kernel(int32_t n, const int32_t* src, int32_t* dst) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) st_dev(&dst[i], ld_dev(&src[i]));
}

static inline int blocks_for(int64_t n) { return static_cast<int>((n + kBlock - 1) / kBlock); }

// Grid cap of the grid-stride setup kernels (their per-workgroup totals
// become device atomics).
constexpr int kSetupGrid = 2048;

template <int MODE>
void launch_bin(const GraphView& g, const BinSetup& s, hipStream_t st) {
  if (g.n <= 0) return;
  hipLaunchKernelGGL(bin_kernel<MODE>, dim3(std::min(blocks_for(g.n), kSetupGrid)), dim3(kBlock), 0, st, g, s);
  if (MODE != kD1)
    hipLaunchKernelGGL(heavy_work_kernel<MODE>, dim3(std::min(blocks_for(g.n), 512)), dim3(kBlock), 0, st, g, s);
}
template void launch_bin<kD1>(const GraphView&, const BinSetup&, hipStream_t);
template void launch_bin<kD2>(const GraphView&, const BinSetup&, hipStream_t);
template void launch_bin<kPD2>(const GraphView&, const BinSetup&, hipStream_t);

void launch_scatter(int32_t n, const int32_t* C, const int8_t* bin, const BinLayout& L, int32_t* wl,
                    int32_t* cnt, int32_t* split_vertex, hipStream_t st) {
  if (n <= 0) return;
  const int blocks = std::min(blocks_for(n), kSetupGrid);
  const int64_t per = (static_cast<int64_t>(n) + blocks - 1) / blocks;
  const int32_t per_block = static_cast<int32_t>((per + kBlock - 1) / kBlock * kBlock);
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(kBlock), 0, st, n, C, bin, L, wl, cnt, split_vertex,
                     per_block);
}

void launch_validate(int32_t n_rows, int32_t n_cols, const int32_t* rp, const int32_t* ci,
                     const int32_t* rpT, const int32_t* ciT, int32_t n_trows, int square, int32_t* err,
                     hipStream_t st) {
  hipLaunchKernelGGL(check_rowptr_kernel, dim3(blocks_for(static_cast<int64_t>(n_rows) + 1)), dim3(kBlock),
                     0, st, n_rows, rp, err);
  if (n_rows > 0)
    hipLaunchKernelGGL(validate_kernel, dim3(blocks_for(n_rows)), dim3(kBlock), 0, st, n_rows, n_cols, rp,
                       ci, rpT, ciT, n_trows, square, err);
}

void launch_priority(int32_t n, const int32_t* gid, uint32_t hs, uint32_t* out, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(priority_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, gid, hs, out);
}

void launch_boundary(int32_t n_owned, int32_t owned_nnz, const int32_t* rp, const int32_t* ci, const int32_t* C,
                     const int32_t* ghost_colors, const KeySource& k, int32_t* loser, int32_t* gflag,
                     unsigned long long* conflicts, hipStream_t st) {
  if (n_owned > 0 && owned_nnz > 0)
    hipLaunchKernelGGL(boundary_kernel, dim3(blocks_for(owned_nnz)), dim3(kBlock), 0, st, n_owned, rp, ci, C,
                       ghost_colors, k, loser, gflag, conflicts);
}

void launch_boundary_uncolor(int32_t n_owned, const int32_t* loser, int32_t* C, hipStream_t st) {
  if (n_owned > 0)
    hipLaunchKernelGGL(boundary_uncolor_kernel, dim3(blocks_for(n_owned)), dim3(kBlock), 0, st, n_owned,
                       loser, C);
}

// Ghost phase 1 reads the owned-induced subgraph: the owned rows without
// their ghost entries (ids >= n_owned).  A flag per owned-row entry (1: kept),
// an exclusive scan of the flags, then every kept entry moves to its scanned
// position and every row starts at the scan of its first entry.
__global__ __launch_bounds__(kBlock) void owned_flags_kernel(int32_t n_owned, const int32_t* rp, const int32_t* ci,
                                                             int32_t* flag) {
  const int32_t e = blockIdx.x * kBlock + threadIdx.x;
  const int32_t nnz = rp[n_owned];
  if (e < nnz) st_dev(&flag[e], ci[e] < n_owned ? 1 : 0);
  else if (e == nnz) st_dev(&flag[e], 0);
}

__global__ __launch_bounds__(kBlock) void owned_compact_kernel(int32_t n_owned, const int32_t* rp, const int32_t* ci,
                                                               const int32_t* pos, int32_t* rp1, int32_t* ci1) {
  const int32_t e = blockIdx.x * kBlock + threadIdx.x;
  if (e <= n_owned) st_dev(&rp1[e], pos[rp[e]]);
  if (e < rp[n_owned] && ci[e] < n_owned) st_dev(&ci1[pos[e]], ci[e]);
}

// Tentative ghost recoloring, one layer: a ghost's row in the local graph is
// the owned vertices adjacent to it (the local graph's undirected
// owned-ghost edges).  Counts them per ghost ...
__global__ __launch_bounds__(kBlock) void ghost_row_count_kernel(int32_t n_owned, const int32_t* rp,
                                                                 const int32_t* ci, int32_t* cnt) {
  const int32_t e = blockIdx.x * kBlock + threadIdx.x;  // a thread per owned-row entry
  if (e >= rp[n_owned]) return;
  const int32_t u = ci[e];
  if (u >= n_owned) atomicAdd(&cnt[u - n_owned], 1);
}

// ... and, with the per-ghost offsets goff (exclusive scan of the counts,
// n_ghost + 1 entries), writes the local CSR over all owned + ghost ids:
// owned rows as given, then the ghosts' rows.
__global__ __launch_bounds__(kBlock) void ghost_rows_kernel(int32_t n_owned, int32_t n_ghost, const int32_t* rp,
                                                            const int32_t* ci, const int32_t* goff, int32_t* fill,
                                                            int32_t* rp3, int32_t* ci3) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;  // offsets by id, entries by position
  const int32_t owned_nnz = rp[n_owned];
  if (i <= n_owned) st_dev(&rp3[i], rp[i]);
  if (i > 0 && i <= n_ghost) st_dev(&rp3[n_owned + i], owned_nnz + goff[i]);
  if (i >= owned_nnz) return;
  const int32_t u = ci[i];
  st_dev(&ci3[i], u);
  if (u >= n_owned) {
    const int32_t j = u - n_owned;
    st_dev(&ci3[owned_nnz + goff[j] + atomicAdd(&fill[j], 1)], row_of(rp, n_owned, i));
  }
}

// Colors the recoloring phase starts from, for the rows-carrying ids
// [0, n3): owned vertices as committed (losers already 0), ghosts as
// received except the losing ones (0: recolored tentatively); a ghost whose
// color is not known yet (0 received) gets kGhostUnknown, which keeps it out
// of the worklist and out of every first fit.
__global__ __launch_bounds__(kBlock) void ghost_recolor_init_kernel(int32_t n_owned, int32_t n3, const int32_t* C,
                                                                    const int32_t* gc, const int32_t* gflag,
                                                                    int32_t* init) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n3) return;
  int32_t c;
  if (v < n_owned) {
    c = ld_dev(&C[v]);
  } else {
    const int32_t j = v - n_owned;
    c = ld_dev(&gflag[j]) ? 0 : (gc[j] == 0 ? kGhostUnknown : gc[j]);
  }
  st_dev(&init[v], c);
}

void launch_ghost_rows(int32_t n_owned, int32_t n_ghost, int32_t owned_nnz, const int32_t* rp, const int32_t* ci,
                       int32_t* cnt, int32_t* goff, int32_t* fill, int32_t* rp3, int32_t* ci3, void* scan_tmp,
                       size_t scan_bytes, hipStream_t st, int* err) {
  *err = 0;
  if (n_ghost > 0) {
    hipLaunchKernelGGL(ghost_row_count_kernel, dim3(blocks_for(std::max(owned_nnz, 1))), dim3(kBlock), 0, st,
                       n_owned, rp, ci, cnt);
    if (exclusive_scan_i32(cnt, goff, n_ghost + 1, scan_tmp, &scan_bytes, st)) *err = 1;
  }
  const int32_t items = std::max(std::max(n_owned + 1, n_ghost + 1), owned_nnz);
  hipLaunchKernelGGL(ghost_rows_kernel, dim3(blocks_for(items)), dim3(kBlock), 0, st, n_owned, n_ghost, rp, ci,
                     goff, fill, rp3, ci3);
}

int launch_owned_subgraph(int32_t n_owned, int32_t owned_nnz, const int32_t* rp, const int32_t* ci, int32_t* flag,
                          int32_t* pos, int32_t* rp1, int32_t* ci1_or_null, void* scan_tmp, size_t scan_bytes,
                          hipStream_t st) {
  const int32_t items = std::max(owned_nnz + 1, n_owned + 1);
  if (ci1_or_null == nullptr) {
    hipLaunchKernelGGL(owned_flags_kernel, dim3(blocks_for(owned_nnz + 1)), dim3(kBlock), 0, st, n_owned, rp, ci, flag);
    return exclusive_scan_i32(flag, pos, owned_nnz + 1, scan_tmp, &scan_bytes, st);
  }
  hipLaunchKernelGGL(owned_compact_kernel, dim3(blocks_for(items)), dim3(kBlock), 0, st, n_owned, rp, ci, pos, rp1,
                     ci1_or_null);
  return 0;
}

void launch_ghost_recolor_init(int32_t n_owned, int32_t n3, const int32_t* C, const int32_t* gc, const int32_t* gflag,
                               int32_t* init, hipStream_t st) {
  if (n3 > 0)
    hipLaunchKernelGGL(ghost_recolor_init_kernel, dim3(blocks_for(n3)), dim3(kBlock), 0, st, n_owned, n3, C, gc,
                       gflag, init);
}

void launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long x, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(fill_u64_kernel, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p,
                       n, x);
}

template <int MODE>
void launch_boundary2(const GraphView& g, int32_t n_owned, int32_t nnz1, const int32_t* C, const int32_t* ghost_colors,
                      const KeySource& k, int32_t* loser, int32_t* gflag, unsigned long long* hits,
                      unsigned long long* set, uint64_t set_mask, unsigned long long* conflicts, hipStream_t st) {
  if (nnz1 > 0)
    hipLaunchKernelGGL(boundary2_kernel<MODE>, dim3(blocks_for(nnz1)), dim3(kBlock), 0, st, g, n_owned, C,
                       ghost_colors, k, loser, gflag, hits, set, set_mask, conflicts);
}
template void launch_boundary2<kD2>(const GraphView&, int32_t, int32_t, const int32_t*, const int32_t*,
                                    const KeySource&, int32_t*, int32_t*, unsigned long long*, unsigned long long*,
                                    uint64_t, unsigned long long*, hipStream_t);
template void launch_boundary2<kPD2>(const GraphView&, int32_t, int32_t, const int32_t*, const int32_t*,
                                     const KeySource&, int32_t*, int32_t*, unsigned long long*, unsigned long long*,
                                     uint64_t, unsigned long long*, hipStream_t);

void launch_ghost_fill(int32_t n_owned, int32_t n_ghost, const int32_t* gc, int32_t* C, int32_t* T,
                       int32_t* maxc, hipStream_t st) {
  if (n_ghost > 0)
    hipLaunchKernelGGL(ghost_fill_kernel, dim3(blocks_for(n_ghost)), dim3(kBlock), 0, st, n_owned, n_ghost,
                       gc, C, T, maxc);
}

void launch_max_i32(int32_t n, const int32_t* a, int32_t* out, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(max_i32_kernel, dim3(std::min(blocks_for(n), 1024)), dim3(kBlock), 0, st, n, a, out);
}

void launch_flags_out(int32_t n, const int32_t* gflag, uint8_t* out, unsigned long long* count,
                      hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(flags_out_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, gflag, out, count);
}

void launch_copy_i32(int32_t n, const int32_t* src, int32_t* dst, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(copy_i32_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, src, dst);
}

}  // namespace gcol
