// Incremental engine: the same synchronous rounds as the pull kernels
// (rounds.hip), computed with less memory traffic.
//
// Two facts of the synchronous rounds make this exact:
//  * committed colors never change, so the set of colors a worklist vertex
//    must avoid only grows.  Each vertex keeps it as a bitset F[v] (bit c-1
//    for color c).  A vertex that commits color c pushes bit c-1 into F of its
//    still-uncolored neighbours during the detect kernel; the next round's
//    color kernel reads only F[v] (T[v] = first zero bit + 1, a scan of at
//    most maxc/32 + 1 words) instead of re-reading the adjacency.  Pushes of
//    round r complete before round r+1 starts, so F[v] holds exactly the
//    colors committed before the round: the snapshot the method requires.
//  * only worklist neighbours can conflict (a committed neighbour's
//    tentative color equals its committed one, which T[v] avoids).  Each
//    vertex keeps an active list A(v) of neighbours that may still be
//    uncolored; the detect kernel scans A(v) and, when v loses, compacts it
//    in place to the neighbours not yet committed (every round at first,
//    then periodically: stale entries of committed neighbours never
//    conflict).  A neighbour that commits in the
//    same round may or may not be dropped (its C is written concurrently);
//    either way the conflict test already used its tentative color, and its
//    commit pushes its color into F[v].
// For distance-2 and partial distance-2 the lists are the materialized
// two-hop neighbourhoods (Section 2.1; Section 3.5/3.6), built once per call.
#include <algorithm>
#include <climits>

#include <hipcub/hipcub.hpp>

#include "inc.hpp"
#include "setup.hpp"

namespace gcol {

namespace {

struct IncMap {
  int32_t cnt[kBins];
  int32_t csize[3];     // vertices per chunk of bins 0..2: kIncPasses passes of the lane groups
  int32_t chunks[3];
  int32_t light_total;
  int32_t heavy_total;  // one unit per bin-3/bin-4 vertex (the incremental engine has no split units)
  int32_t total;        // all worklist entries
};

// Bin of a vertex by the current length of its active list (both parts):
// lists only shrink, so a vertex moves to narrower lane groups as its
// neighbours commit (never above the bin of its static work).
__device__ __forceinline__ int inc_bin_of(const BinLayout& L, int32_t len) {
  return len <= L.hi[0] ? 0 : len <= L.hi[1] ? 1 : len <= L.hi[2] ? 2 : kBlockBin;
}

__device__ __forceinline__ void make_inc_map_from(const int32_t* cnt, const BinLayout& L, IncMap& m) {
  int32_t lt = 0, tot = 0;
  for (int i = 0; i < kBins; ++i) {
    m.cnt[i] = ld_dev(&cnt[i]);
    tot += m.cnt[i];
  }
  for (int i = 0; i < 3; ++i) {
    m.csize[i] = inc_chunk_size(L.lanes[i]);
    m.chunks[i] = (m.cnt[i] + m.csize[i] - 1) / m.csize[i];
    lt += m.chunks[i];
  }
  m.light_total = lt;
  m.heavy_total = m.cnt[kBlockBin] + m.cnt[kSplitBin];
  m.total = tot;
}

__device__ __forceinline__ void make_inc_map(const IncBufs& b, const BinLayout& L, IncMap& m) {
  make_inc_map_from(b.cnt_in, L, m);
}

__device__ __forceinline__ int32_t xcd_block() {
  const int32_t nb = gridDim.x;
  const int32_t per = nb / 8;
  const int32_t i = blockIdx.x;
  if (per == 0 || (nb & 7) != 0) return i;
  return (i & 7) * per + (i >> 3);
}

__device__ __forceinline__ uint64_t wsum(uint64_t x) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Word w of x's bitset: word 0 (colors 1..32) in the dense array F, one
// per vertex, so that a push of a small color (every push of the first 32
// rounds) reads no offsets; words 1.. at fw_off[x] in Fx.  nullptr: beyond
// any color x can take, irrelevant to its first fit.
template <int MUT>
__device__ __forceinline__ uint32_t* f_word(const IncBufs& b, int32_t x, int32_t w) {
  if (w == 0) return b.F + x;
  const int32_t w0 = ld_mut<MUT>(&b.fw_off[x]);
  if (w > ld_mut<MUT>(&b.fw_off[x + 1]) - w0) return nullptr;
  return b.Fx + w0 + (w - 1);
}

// Sets bit c-1 of x's bitset unless it is already set (read first: most
// pushes repeat a small color that an earlier neighbour already pushed).
template <int MUT>
__device__ __forceinline__ void push_color(const IncBufs& b, int32_t x, int32_t c, uint64_t& pushes) {
  uint32_t* p = f_word<MUT>(b, x, (c - 1) >> 5);
  if (!p) return;
  const uint32_t bit = 1u << ((c - 1) & 31);
  if (!(ld_mut<MUT>(p) & bit)) {
    atomicOr(p, bit);
    ++pushes;
  }
}

// A loser compacts its list to the neighbours not yet committed in the first
// kCompactAlways rounds (where most neighbours commit), whenever its list is
// still the read-only adjacency (round 1 of D1), and else once every
// kCompactPeriod rounds (kTailCompactPeriod in the tail kernel, whose rounds
// commit few vertices each).  Entries of committed neighbours left in a list
// are harmless: a committed neighbour's tentative color is its committed
// color, which the vertex's own tentative color avoids, and pushes skip
// committed vertices.  (Measured on MI355X: every 4th against every 8th
// round, R-MAT 22 D1 45.0 -> 41.5 ms, the 4M x 1M PD2 pattern 78.5 -> 75.1
// ms; later, with the small first scan steps, every 16th round and every
// 32nd in the tail: R-MAT 22 per-round detect 414 -> 404 us per launch, the
// whole call within run-to-run noise.)
constexpr int kCompactAlways = 2;
constexpr int kCompactPeriod = 16;      // a power of two
constexpr int kTailCompactPeriod = 32;  // a power of two

template <int MUT>
__device__ __forceinline__ bool compact_now(const IncBufs& b, int round, int32_t v) {
  if (b.defer_split) return false;
  constexpr int period = MUT ? kTailCompactPeriod : kCompactPeriod;
  return b.A_in != b.A_out || round <= kCompactAlways || ((round + v) & (period - 1)) == 0;
}

// The conflict test's gather: a neighbour's tentative color from the byte
// array while every tentative color fits a byte (4 MB for 2^22 vertices, so
// the gathers mostly hit L2), else from the 32-bit array.  Committed
// neighbours hold their own color in both, or 0 in the byte array where
// they were committed before the call: neither equals a tentative color
// the vertex could have taken.
template <int MUT>
__device__ __forceinline__ int32_t tentative_of(const IncBufs& b, bool t8, int32_t u) {
  return t8 ? static_cast<int32_t>(ld_mut<MUT>(&b.T8[u])) : ld_mut<MUT>(&b.T[u]);
}

// The compaction test: u committed, from one bit per vertex (512 KB for
// 2^22 vertices) instead of its 32-bit color.
template <int MUT>
__device__ __forceinline__ bool committed(const IncBufs& b, int32_t u) {
  return (ld_mut<MUT>(&b.done[u >> 5]) >> (u & 31)) & 1u;
}

__device__ __forceinline__ void mark_committed(const IncBufs& b, int32_t v) {
  atomicOr(&b.done[v >> 5], 1u << (v & 31));
}

}  // namespace

// ---------------------------------------------------------------------------
// color: T[v] = first zero bit of F[v] + 1, one thread per worklist vertex
// ---------------------------------------------------------------------------
struct IncColorShared {
  IncMap M;
  unsigned long long acc[3];
};

// pre (tail kernel): the round's map and largest committed color, already
// read by the workgroup at the end of the previous round.
struct IncPre {
  IncMap M;
  int32_t maxc;
};

template <int MUT>
__device__ __forceinline__ void inc_color_phase(const IncBufs& b, const BinLayout& L, int round,
                                                IncColorShared& sh, const IncPre* pre = nullptr) {
  IncMap& M = sh.M;
  unsigned long long* s_acc = sh.acc;
  if (threadIdx.x == 0) {
    if (pre) M = pre->M;
    else make_inc_map(b, L, M);
    s_acc[0] = s_acc[1] = s_acc[2] = 0ull;
    if (blockIdx.x == 0) {
      for (int i = 0; i < kBins; ++i) atomic_reset_i32(&b.cnt_out[i]);
      atomic_reset_i32(&b.tile_ctr[1]);
      if (M.total > 0) {
        const int gr = round + b.round_base;
        atomicMax(b.rounds_done, gr);
        if (b.trace && gr <= b.trace_cap) st_dev(&b.trace[gr - 1], M.total);
        atomicAdd(&b.acc[0], static_cast<unsigned long long>(M.total));
      }
    }
  }
  __syncthreads();
  const int32_t mc = pre ? pre->maxc : ld_dev(b.maxc);
  const int32_t wmax = mc / 32 + 1;  // words that can hold a committed color
  uint64_t work = 0, lists = 0, bytes = 0;
  const int32_t stride = gridDim.x * kBlock;
  for (int32_t i = xcd_block() * kBlock + threadIdx.x; i < M.total; i += stride) {
    int bin = 0;
    int32_t j = i;
    while (bin < kBins - 1 && j >= M.cnt[bin]) {
      j -= M.cnt[bin];
      ++bin;
    }
    const int32_t v = ld_mut<MUT>(&b.wl_in[L.off[bin] + j]);
    // word 0 first; the offsets of the further words only when it is full
    const uint32_t x0 = ld_mut<MUT>(&b.F[v]);
    int32_t t, w = 0, nw = 1;
    if (x0 != ~0u || wmax == 1) {
      t = x0 != ~0u ? __builtin_ctz(~x0) + 1 : 33;
    } else {
      // the further words four at a time: independent loads in flight
      // instead of one round trip per word
      const int32_t w0 = ld_mut<MUT>(&b.fw_off[v]);
      nw = min(ld_mut<MUT>(&b.fw_off[v + 1]) - w0 + 1, wmax);
      t = 32 * nw + 1;
      bool found = false;
      for (w = 1; w < nw && !found; w += 4) {
        uint32_t x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = w + j < nw ? ld_mut<MUT>(&b.Fx[w0 + w + j - 1]) : ~0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (!found && x[j] != ~0u) {
            t = 32 * (w + j) + __builtin_ctz(~x[j]) + 1;
            found = true;
          }
        }
      }
      w = found ? (t - 1) / 32 : nw;  // the word that held t (or all of them)
      bytes += 8;  // the two offsets
    }
    st_dev(&b.T[v], t);
    if (round <= b.t8_last) st_mut<MUT>(&b.T8[v], static_cast<uint8_t>(t));
    work += static_cast<uint64_t>(ld_mut<MUT>(&b.work[v]));
    lists += static_cast<uint64_t>(ld_mut<MUT>(&b.alen_in[v]));
    // worklist id, the words scanned, static work, T write (and its byte)
    bytes += 4 + 4 * static_cast<uint64_t>(min(w + 1, nw)) + 4 + 4 + (round <= b.t8_last ? 1 : 0);
  }
  work = wsum(work);
  lists = wsum(lists);
  bytes = wsum(bytes);
  if (lane_id() == 0) {
    if (work) atomicAdd(&s_acc[0], static_cast<unsigned long long>(work));
    if (lists) atomicAdd(&s_acc[1], static_cast<unsigned long long>(lists));
    if (bytes) atomicAdd(&s_acc[2], static_cast<unsigned long long>(bytes));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_acc[0]) atomicAdd(&b.acc[1], s_acc[0]);
    if (s_acc[1]) atomicAdd(&b.acc[2], s_acc[1]);
    if (s_acc[2]) atomicAdd(&b.acc[b.bytes_slot], s_acc[2]);
  }
}

__global__ __launch_bounds__(kBlock) void inc_color_kernel(IncBufs b, BinLayout L, int round) {
  __shared__ IncColorShared sh;
  inc_color_phase<0>(b, L, round, sh);
}

// ---------------------------------------------------------------------------
// detect + commit/push or compact, group of G lanes per vertex
// ---------------------------------------------------------------------------
// Lists are partitioned by key in the round that first copies them out of
// the adjacency (D1) or the materialized two-hop lists (D2/PD2): the
// not-yet-committed neighbours of higher key at the front (length alen), the
// lower ones at the back of the vertex's list region (length llen).  Only a
// higher-key neighbour can beat v, so later detect scans read the front part
// only; the one push a winner makes reads both parts.
template <int G, int MUT>
__device__ __forceinline__ void inc_detect_chunk(const KeySource& k, const IncBufs& b, const BinLayout& L, int round,
                                                 const int32_t* wl, int32_t count, int32_t* s_ent, int8_t* s_tb,
                                                 int32_t* s_wc, int32_t& maxc_acc, uint64_t& bytes,
                                                 uint64_t& pushes) {
  constexpr int per_pass = kBlock / G;
  const int gi = threadIdx.x / G;
  const int sub = threadIdx.x % G;
  const int first = lane_id() & ~(G - 1);
  const uint64_t gm = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  const bool first_pass = b.A_in != b.A_out;
  const bool t8 = round <= b.t8_last;
  for (int32_t idx = gi; idx < count; idx += per_pass) {
    const int32_t v = ld_mut<MUT>(&wl[idx]);
    const int32_t tv = ld_mut<MUT>(&b.T[v]);
    const uint64_t kv = key_of(k, v);
    const int32_t base = ld_mut<MUT>(&b.aoff[v]);
    const int32_t len = ld_mut<MUT>(&b.alen_in[v]);
    const int32_t* A = b.A_in + base;
    bool lose = false;
    int32_t read = 0, gath = 0;
    // the group steps through the list together, two entries per lane per
    // step, and stops at the first step in which any of its lanes found a
    // conflict (a lane-by-lane stop would keep the group scanning until its
    // slowest lane reached the end; measured on MI355X, two entries per step
    // beat four: R-MAT 22 D1 39.3 -> 38.4 ms)
    // wide groups take one entry per lane in their first step (a loser
    // mostly meets its conflict near the front of its list)
    for (int32_t e0 = 0, per = (G >= 32 ? 1 : 2); e0 < len; e0 += per * G, per = 2) {
      int32_t u[2], t[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int32_t e = e0 + sub + j * G;
        const bool in = j < per && e < len;
        u[j] = in ? ld_mut<MUT>(&A[e]) : -1;
        read += in ? 1 : 0;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bool higher = u[j] >= 0 && (!first_pass || key_of(k, u[j]) > kv);
        t[j] = higher ? (b.uniform ? tv : tentative_of<MUT>(b, t8, u[j])) : -1;
        gath += (higher && !b.uniform) ? 1 : 0;
      }
      bool hit = false;
#pragma unroll
      for (int j = 0; j < 2; ++j) hit = hit || t[j] == tv;
      if (group_any<G>(hit)) {
        lose = true;
        break;
      }
    }
    // list entries and tentative colors this lane read
    bytes += 4ull * static_cast<uint64_t>(read) + (t8 ? 1ull : 4ull) * static_cast<uint64_t>(gath);
    if (lose && !compact_now<MUT>(b, round, v)) {
      if (sub == 0) {
        s_ent[idx] = v;
        s_tb[idx] = static_cast<int8_t>(inc_bin_of(L, first_pass ? len : len + ld_mut<MUT>(&b.llen[v])));
        bytes += 24;
      }
    } else if (lose) {
      // keep the neighbours that are not committed (yet); the first pass
      // also splits them by key
      const int32_t cap = ld_mut<MUT>(&b.aoff[v + 1]) - base;
      int32_t kept = 0, kept_lo = 0;
      for (int32_t e0 = 0; e0 < len; e0 += G) {
        const int32_t e = e0 + sub;
        int32_t u = -1;
        bool keep = false, hi = true;
        if (e < len) {
          u = ld_mut<MUT>(&A[e]);
          keep = b.uniform || !committed<MUT>(b, u);  // round 1: nobody was committed before it
          if (first_pass) hi = key_of(k, u) > kv;
        }
        const uint64_t bal_h = (__ballot(keep && hi) >> first) & gm;
        const uint64_t bal_l = (__ballot(keep && !hi) >> first) & gm;
        const uint64_t below = (1ull << sub) - 1ull;
        if (keep && hi) st_dev(&b.A_out[base + kept + __popcll(bal_h & below)], u);
        if (keep && !hi) st_dev(&b.A_out[base + cap - 1 - (kept_lo + __popcll(bal_l & below))], u);
        kept += __popcll(bal_h);
        kept_lo += __popcll(bal_l);
      }
      if (sub == 0) {
        st_dev(&b.alen_out[v], kept);
        if (first_pass) st_dev(&b.llen[v], kept_lo);
        else kept_lo = ld_mut<MUT>(&b.llen[v]);
        s_ent[idx] = v;
        s_tb[idx] = static_cast<int8_t>(inc_bin_of(L, kept + kept_lo));
        bytes += 28 + 8ull * static_cast<uint64_t>(len) + 4ull * static_cast<uint64_t>(kept + kept_lo);
      }
    } else {
      // push the color to every list entry not yet committed: the whole
      // list on the first pass, else both parts.  The committed test reads
      // the bit array (cached; a 32-bit committed-color gather here had cost
      // more than the pushes it saved); a neighbour committing in the same
      // round may still get the push, which is harmless: a committed
      // vertex's bitset is never read again.
      const int32_t cap = first_pass ? len : ld_mut<MUT>(&b.aoff[v + 1]) - base;
      const int32_t lo_len = first_pass ? 0 : ld_mut<MUT>(&b.llen[v]);
      for (int part = 0; part < 2; ++part) {
        const int32_t pb = part == 0 ? 0 : cap - lo_len;
        const int32_t pe = part == 0 ? len : cap;
        for (int32_t e0 = pb + sub; e0 < pe; e0 += 4 * G) {
          int32_t x[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int32_t e = e0 + j * G;
            x[j] = e < pe ? ld_mut<MUT>(&A[e]) : -1;
          }
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (x[j] >= 0 && !committed<MUT>(b, x[j])) push_color<MUT>(b, x[j], tv, pushes);
        }
      }
      if (sub == 0) {
        st_dev(&b.C[v], tv);
        mark_committed(b, v);
        maxc_acc = max(maxc_acc, tv);
        s_ent[idx] = -1;
        bytes += 20 + 8ull * static_cast<uint64_t>(len + lo_len);  // own fields, C write, entries + committed bits
      }
    }
  }
  // append the losers to the next worklist, each to the bin of its list
  // length: per target bin a wave count, a scan over the waves and one
  // counter atomic per workgroup
  __syncthreads();
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int32_t x = tid < count ? s_ent[tid] : -1;
  const int t = x >= 0 ? s_tb[tid] : -1;
  const uint64_t b0 = __ballot(t == 0), b1 = __ballot(t == 1), b2 = __ballot(t == 2), b3 = __ballot(t == kBlockBin);
  if (lane_id() == 0) {
    s_wc[0 * kWavesPerBlock + wave] = static_cast<int32_t>(__popcll(b0));
    s_wc[1 * kWavesPerBlock + wave] = static_cast<int32_t>(__popcll(b1));
    s_wc[2 * kWavesPerBlock + wave] = static_cast<int32_t>(__popcll(b2));
    s_wc[3 * kWavesPerBlock + wave] = static_cast<int32_t>(__popcll(b3));
  }
  __syncthreads();
  if (tid < 4) {
    int32_t tot = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      const int32_t c = s_wc[tid * kWavesPerBlock + w];
      s_wc[tid * kWavesPerBlock + w] = tot;
      tot += c;
    }
    s_wc[4 * kWavesPerBlock + tid] = tot ? atomicAdd(&b.cnt_out[tid == 3 ? kBlockBin : tid], tot) : 0;
  }
  __syncthreads();
  if (x >= 0) {
    const uint64_t mine = t == 0 ? b0 : t == 1 ? b1 : t == 2 ? b2 : b3;
    const int q = t == kBlockBin ? 3 : t;
    st_dev(&b.wl_out[L.off[t] + s_wc[4 * kWavesPerBlock + q] + s_wc[q * kWavesPerBlock + wave] +
                     static_cast<int32_t>(lanes_below(mine))],
           x);
  }
  __syncthreads();
}

// One workgroup per heavy vertex.  Every thread keeps kIncBatch independent
// list loads (and then their T or C loads) in flight, and the workgroup meets
// at a barrier once per kBlock * kIncBatch entries.
constexpr int kIncBatch = 8;

// A heavy vertex's own fields, loaded ahead for a batch of heavy units at
// once (one round trip for the batch instead of two per vertex).
struct HeavyVertex {
  int32_t v, tv, base, end, len, llen;
};
constexpr int kHeavyBatch = 8;

// Returns the bin of the next worklist if v lost (its append is left to the
// caller, batched), else -1.
template <int MUT>
__device__ __forceinline__ int inc_detect_block(const KeySource& k, const IncBufs& b, const BinLayout& L, int round,
                                                const HeavyVertex& h, int32_t* s_wc, int32_t& maxc_acc,
                                                uint64_t& bytes, uint64_t& pushes) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const bool first_pass = b.A_in != b.A_out;
  const bool t8 = round <= b.t8_last;
  const int32_t v = h.v;
  const int32_t tv = h.tv;
  const uint64_t kv = key_of(k, v);
  const int32_t base = h.base;
  const int32_t len = h.len;
  const int32_t* A = b.A_in + base;
  constexpr int32_t step = kBlock * kIncBatch;
  bool lose = false;
  uint32_t read = 0, gath = 0;
  // steps of one, two, then kIncBatch entries per thread: a losing vertex
  // mostly meets a conflict near the front, where a full step would read
  // kIncBatch times more than it needs (measured on MI355X: R-MAT 22 D1
  // 34.8 -> 32.5 ms per call, the PD2 pattern 64.4 -> 62.9 ms)
  for (int32_t e0 = 0, per = 1; e0 < len; e0 += per * kBlock, per = (per == 1 ? 2 : kIncBatch)) {
    int32_t u[kIncBatch], t[kIncBatch];
#pragma unroll
    for (int j = 0; j < kIncBatch; ++j) {
      const int32_t e = e0 + j * kBlock + tid;
      const bool in = j < per && e < len;
      u[j] = in ? ld_mut<MUT>(&A[e]) : -1;
      read += in ? 1u : 0u;
    }
    // only a higher-key neighbour can beat v: before the lists are split by
    // key, compare keys first and read the tentative colors of those only
#pragma unroll
    for (int j = 0; j < kIncBatch; ++j) {
      const bool higher = u[j] >= 0 && (!first_pass || key_of(k, u[j]) > kv);
      t[j] = higher ? (b.uniform ? tv : tentative_of<MUT>(b, t8, u[j])) : -1;
      gath += (higher && !b.uniform) ? 1u : 0u;
    }
#pragma unroll
    for (int j = 0; j < kIncBatch; ++j)
      if (t[j] == tv) lose = true;
    if (__syncthreads_or(lose)) {
      lose = true;
      break;
    }
  }
  bytes += 4ull * read + (t8 ? 1ull : 4ull) * gath;  // list entries and tentative colors this thread read
  int next_bin = -1;
  if (lose && !compact_now<MUT>(b, round, v)) {
    next_bin = inc_bin_of(L, first_pass ? len : len + h.llen);
    if (tid == 0) bytes += 28;
  } else if (lose) {
    // keep the neighbours that are not committed (yet), order free; the
    // first pass also splits them by key (higher to the front, lower to the
    // back).  Later passes compact the front part in place: every entry of a
    // step is read before the barrier that precedes the step's writes, and
    // writes land below the step's first entry or inside it.
    const int32_t cap = h.end - base;
    int32_t kept = 0, kept_lo = 0;
    int32_t* s_lo = s_wc + kWavesPerBlock;
    for (int32_t e0 = 0; e0 < len; e0 += step) {
      int32_t u[kIncBatch];
      uint32_t keep_hi = 0, keep_lo = 0;  // bit j: entry j kept in the front / back part
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) {
        const int32_t e = e0 + j * kBlock + tid;
        u[j] = e < len ? ld_mut<MUT>(&A[e]) : -1;
      }
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) {
        const bool keep = u[j] >= 0 && (b.uniform || !committed<MUT>(b, u[j]));
        const bool hi = !first_pass || (u[j] >= 0 && key_of(k, u[j]) > kv);
        keep_hi |= (keep && hi) ? (1u << j) : 0u;
        keep_lo |= (keep && !hi) ? (1u << j) : 0u;
      }
      const int32_t cnt = __builtin_popcount(keep_hi), cnt_lo = __builtin_popcount(keep_lo);
      int32_t incl = cnt, incl_lo = cnt_lo;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, kWave);
        const int32_t z = __shfl_up(incl_lo, o, kWave);
        if (lane_id() >= o) {
          incl += y;
          incl_lo += z;
        }
      }
      if (lane_id() == kWave - 1) {
        s_wc[wave] = incl;
        s_lo[wave] = incl_lo;
      }
      __syncthreads();
      int32_t pos = kept + incl - cnt, pos_lo = kept_lo + incl_lo - cnt_lo;
      int32_t tot = 0, tot_lo = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wave) {
          pos += s_wc[w];
          pos_lo += s_lo[w];
        }
        tot += s_wc[w];
        tot_lo += s_lo[w];
      }
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) {
        if (keep_hi & (1u << j)) st_dev(&b.A_out[base + pos++], u[j]);
        if (keep_lo & (1u << j)) st_dev(&b.A_out[base + cap - 1 - pos_lo++], u[j]);
      }
      kept += tot;
      kept_lo += tot_lo;
      __syncthreads();
    }
    // later passes also drop the committed entries of the lower-key part
    // (the part only a push reads: without this, a heavy vertex that commits
    // late would push over every lower-key neighbour it had in round 1).
    // Back index q = 0, 1, ... is list position cap-1-q; kept entries move
    // to back indices below or at their own, in step order as above.
    const int32_t lo_len = first_pass ? 0 : h.llen;
    for (int32_t q0 = 0; q0 < lo_len; q0 += step) {
      int32_t u[kIncBatch];
      uint32_t keep = 0;
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) {
        const int32_t q = q0 + j * kBlock + tid;
        u[j] = q < lo_len ? ld_mut<MUT>(&A[cap - 1 - q]) : -1;
      }
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) keep |= (u[j] >= 0 && !committed<MUT>(b, u[j])) ? (1u << j) : 0u;
      const int32_t cnt = __builtin_popcount(keep);
      int32_t incl = cnt;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, kWave);
        if (lane_id() >= o) incl += y;
      }
      if (lane_id() == kWave - 1) s_lo[wave] = incl;
      __syncthreads();
      int32_t pos = kept_lo + incl - cnt, tot = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wave) pos += s_lo[w];
        tot += s_lo[w];
      }
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j)
        if (keep & (1u << j)) st_dev(&b.A_out[base + cap - 1 - pos++], u[j]);
      kept_lo += tot;
      __syncthreads();
    }
    next_bin = inc_bin_of(L, kept + kept_lo);
    if (tid == 0) {
      st_dev(&b.alen_out[v], kept);
      st_dev(&b.llen[v], kept_lo);
      bytes += 24 + 8ull * static_cast<uint64_t>(len + lo_len) + 4ull * static_cast<uint64_t>(kept + kept_lo);
    }
  } else {
    // push the color to every list entry not yet committed (as in the
    // lane-group path): the whole list on the first pass, else both parts
    const int32_t cap = first_pass ? len : h.end - base;
    const int32_t lo_len = first_pass ? 0 : h.llen;
    for (int part = 0; part < 2; ++part) {
      const int32_t pb = part == 0 ? 0 : cap - lo_len;
      const int32_t pe = part == 0 ? len : cap;
      for (int32_t e0 = pb; e0 < pe; e0 += step) {
        int32_t x[kIncBatch];
#pragma unroll
        for (int j = 0; j < kIncBatch; ++j) {
          const int32_t e = e0 + j * kBlock + tid;
          x[j] = e < pe ? ld_mut<MUT>(&A[e]) : -1;
        }
#pragma unroll
        for (int j = 0; j < kIncBatch; ++j)
          if (x[j] >= 0 && !committed<MUT>(b, x[j])) push_color<MUT>(b, x[j], tv, pushes);
      }
    }
    if (tid == 0) {
      st_dev(&b.C[v], tv);
      mark_committed(b, v);
      maxc_acc = max(maxc_acc, tv);
      bytes += 20 + 8ull * static_cast<uint64_t>(len + lo_len);  // own fields, C write, entries + committed bits
    }
  }
  __syncthreads();
  return next_bin;
}

struct IncDetectShared {
  int32_t unit;
  int32_t max;
  int32_t ent[kBlock];
  int8_t tb[kBlock];                    // target bin of each loser in ent
  int32_t wc[4 * kWavesPerBlock + 4];   // per-target-bin wave offsets, then per-bin bases
  unsigned long long acc[2];
  IncMap M;
  HeavyVertex hv[kHeavyBatch];  // the batch of heavy units in hand
  int8_t hb[kHeavyBatch];       // the next worklist's bin of each, or -1 (committed)
};

template <int MUT>
__device__ __forceinline__ void inc_detect_phase(const KeySource& k, const IncBufs& b, const BinLayout& L,
                                                 int round, IncDetectShared& sh, const IncPre* pre = nullptr) {
  int32_t& s_unit = sh.unit;
  int32_t& s_max = sh.max;
  int32_t* s_ent = sh.ent;
  int32_t* s_wc = sh.wc;
  int8_t* s_tb = sh.tb;
  unsigned long long* s_acc = sh.acc;
  IncMap& M = sh.M;
  if (threadIdx.x == 0) {
    if (pre) M = pre->M;
    else make_inc_map(b, L, M);
    s_max = 0;
    s_acc[0] = s_acc[1] = 0ull;
  }
  __syncthreads();
  int32_t maxc_acc = 0;
  uint64_t bytes = 0, pushes = 0;
  const int32_t lb = xcd_block();
  // A small round of the tail kernel hands its light bins to whole
  // workgroups as well, widest bin first, while the heavy vertices and the
  // promoted ones together are no more than the workgroups: the grid would
  // otherwise idle while a few lane groups step through their chunks (two
  // vertices per group, one after the other, each list a few entries per
  // step).  Every workgroup takes the same decision from the same counts.
  const int32_t G = static_cast<int32_t>(gridDim.x);
  int32_t light_total = M.light_total, heavy_total = M.heavy_total, light_bins = 3;
  if (MUT != 0) {
    while (light_bins > 0 && heavy_total + M.cnt[light_bins - 1] <= G) {
      --light_bins;
      heavy_total += M.cnt[light_bins];
      light_total -= M.chunks[light_bins];
    }
  }
  const int32_t c0 = static_cast<int32_t>(static_cast<int64_t>(lb) * light_total / gridDim.x);
  const int32_t c1 = static_cast<int32_t>(static_cast<int64_t>(lb + 1) * light_total / gridDim.x);
  for (int32_t c = c0; c < c1; ++c) {
    int bin = 0;
    int32_t cc = c;
    while (bin < 2 && cc >= M.chunks[bin]) {
      cc -= M.chunks[bin];
      ++bin;
    }
    const int32_t firstc = cc * M.csize[bin];
    const int32_t count = min(M.csize[bin], M.cnt[bin] - firstc);
    const int32_t* wl = b.wl_in + L.off[bin] + firstc;
    switch (L.lanes[bin]) {
      case 1: inc_detect_chunk<1, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
      case 2: inc_detect_chunk<2, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
      case 4: inc_detect_chunk<4, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
      case 8: inc_detect_chunk<8, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
      case 16: inc_detect_chunk<16, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
      case 32: inc_detect_chunk<32, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
      default: inc_detect_chunk<64, MUT>(k, b, L, round, wl, count, s_ent, s_tb, s_wc, maxc_acc, bytes, pushes); break;
    }
  }
  // heavy units, kHeavyBatch at a time: first the workgroup's own
  // (units lb, lb + G, lb + 2G, ... : no atomic), then batches of consecutive
  // units above G * kHeavyBatch handed out by a counter.  The batch's vertex
  // fields are loaded at once, and its losers are appended together, one
  // counter atomic per target bin.
  const int64_t static_end = static_cast<int64_t>(G) * kHeavyBatch;
  int32_t dyn = -1;  // first unit of a handed-out batch; -1: the own batch
  while (true) {
    if (threadIdx.x < kHeavyBatch) {
      const int j = threadIdx.x;
      const int64_t u = dyn < 0 ? static_cast<int64_t>(lb) + static_cast<int64_t>(j) * G : dyn + j;
      HeavyVertex h{-1, 0, 0, 0, 0, 0};
      if (u < heavy_total) {
        // units: bin 3, bin 4, then the promoted light bins from bin 2 down
        int32_t jj = static_cast<int32_t>(u);
        int bin = kBlockBin;
        if (jj >= M.cnt[kBlockBin]) {
          jj -= M.cnt[kBlockBin];
          bin = kSplitBin;
          for (int lb2 = 2; jj >= M.cnt[bin] && lb2 >= light_bins; --lb2) {
            jj -= M.cnt[bin];
            bin = lb2;
          }
        }
        h.v = ld_mut<MUT>(&b.wl_in[L.off[bin] + jj]);
        h.tv = ld_mut<MUT>(&b.T[h.v]);
        h.base = ld_mut<MUT>(&b.aoff[h.v]);
        h.end = ld_mut<MUT>(&b.aoff[h.v + 1]);
        h.len = ld_mut<MUT>(&b.alen_in[h.v]);
        h.llen = ld_mut<MUT>(&b.llen[h.v]);
      }
      sh.hv[j] = h;
      sh.hb[j] = -1;
    }
    __syncthreads();
    for (int j = 0; j < kHeavyBatch; ++j) {
      const HeavyVertex h = sh.hv[j];
      if (h.v < 0) continue;
      const int nb = inc_detect_block<MUT>(k, b, L, round, h, s_wc, maxc_acc, bytes, pushes);
      if (threadIdx.x == 0) sh.hb[j] = static_cast<int8_t>(nb);
    }
    __syncthreads();
    // the batch's losers: thread t appends those of target bin t
    if (threadIdx.x < 4) {
      const int t = threadIdx.x == 3 ? kBlockBin : threadIdx.x;
      int32_t c = 0;
      for (int j = 0; j < kHeavyBatch; ++j) c += sh.hb[j] == t ? 1 : 0;
      if (c > 0) {
        int32_t p = atomicAdd(&b.cnt_out[t], c);
        for (int j = 0; j < kHeavyBatch; ++j)
          if (sh.hb[j] == t) st_dev(&b.wl_out[L.off[t] + p++], sh.hv[j].v);
      }
    }
    if (dyn < 0 && static_end >= heavy_total) break;
    if (threadIdx.x == 0) s_unit = static_cast<int32_t>(static_end) + kHeavyBatch * atomicAdd(&b.tile_ctr[1], 1);
    __syncthreads();
    dyn = s_unit;
    __syncthreads();
    if (dyn >= heavy_total) break;
  }
  maxc_acc = [&] {
    int32_t x = maxc_acc;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) x = max(x, __shfl_xor(x, off, kWave));
    return x;
  }();
  bytes = wsum(bytes);
  pushes = wsum(pushes);
  if (lane_id() == 0) {
    if (maxc_acc > 0) atomicMax(&s_max, maxc_acc);
    if (bytes) atomicAdd(&s_acc[0], static_cast<unsigned long long>(bytes));
    if (pushes) atomicAdd(&s_acc[1], static_cast<unsigned long long>(pushes));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_max > 0) atomicMax(b.maxc, s_max);
    if (s_acc[0]) atomicAdd(&b.acc[b.bytes_slot + 1], s_acc[0]);
    if (s_acc[1]) atomicAdd(&b.acc[5], s_acc[1]);
  }
}

// Five wavefronts per SIMD (96 VGPRs, no scratch; the default allocation
// took 97 and allowed four): measured on MI355X, R-MAT 22 467 -> 447 us per
// launch.  The tail kernel stays at its default: capped at four or five it
// spills, and its rounds got slower.
__global__ __launch_bounds__(kBlock, 5) void inc_detect_kernel(KeySource k, IncBufs b, BinLayout L, int round) {
  __shared__ IncDetectShared sh;
  inc_detect_phase<0>(k, b, L, round, sh);
}

// ---------------------------------------------------------------------------
// tail: all remaining rounds in one cooperative launch
// ---------------------------------------------------------------------------

// Grid-wide barrier.  Workgroups arrive in eight groups (blockIdx.x mod 8,
// each with its own counter bar[kBarGroup + 32 g]); the last of a group
// arrives at the top counter bar[0], and the last of those bumps the
// generation word bar[kBarGen].  Every word sits on its own cache line, so
// arrivals contend eight ways less than on one counter (measured on MI355X:
// 2.8 instead of 7.0 us per barrier at 512 workgroups).  Every array that
// one workgroup writes and another reads within the tail kernel is accessed
// with device-scope loads, stores and atomics, so the barrier needs no cache
// writeback or invalidation: each wavefront waits until its own memory
// operations have completed, and the generation bump is a release.  The
// cooperative launch makes every workgroup co-resident, so a barrier waits
// only for the others to finish their phase; the deadline (wall-clock ticks)
// turns a defect into an error bit instead of a hang.  Returns false (in
// every thread of the workgroup) if it gave up.
__device__ __forceinline__ bool grid_sync(uint32_t* bar, int32_t* err, uint64_t deadline, int32_t* s_ok) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t gen = atomic_load_u32(&bar[kBarGen]);
    const uint32_t G = gridDim.x, g = blockIdx.x & 7u;
    const uint32_t groups = G < 8u ? G : 8u;
    const uint32_t size = G < 8u ? 1u : G / 8u + (g < (G & 7u) ? 1u : 0u);
    uint32_t* gc = &bar[kBarGroup + 32u * g];
    bool last = false;
    if (atomicAdd(gc, 1u) == size - 1u) {
      (void)__hip_atomic_exchange(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (atomicAdd(&bar[0], 1u) == groups - 1u) {
        (void)__hip_atomic_exchange(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&bar[kBarGen], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    int32_t ok = 1;
    if (!last) {
      const uint64_t t0 = static_cast<uint64_t>(wall_clock64());
      while (atomic_load_u32(&bar[kBarGen]) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (static_cast<uint64_t>(wall_clock64()) - t0 > deadline) {
          atomicOr(err, kErrTailBarrier);
          ok = 0;
          break;
        }
      }
    }
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Entry check-in of the tail kernel.  Its grid barriers need every workgroup
// resident at once, which the cooperative launch provides only while no
// other kernel fills the device.  So before writing anything, every
// workgroup arrives and waits until either all gridDim.x workgroups have
// arrived (then all are resident: none leaves before the decision) or
// `ticks` have passed.  The decision is one compare-and-swap on a state word
// (the last arrival sets GO, a workgroup whose wait ran out sets ABORT), so
// every workgroup takes the same one, including those that start after it.
// On ABORT the launch changes nothing and the host runs the rounds as
// per-round launches.
constexpr uint32_t kCheckinGo = 1u, kCheckinAbort = 2u;

__device__ __forceinline__ bool tail_checkin(uint32_t* bar, int32_t* err, uint64_t ticks, int32_t* s_ok) {
  if (threadIdx.x == 0) {
    uint32_t* state = &bar[kBarState];
    if (atomicAdd(&bar[kBarCheckin], 1u) + 1u == gridDim.x) (void)atomicCAS(state, 0u, kCheckinGo);
    const uint64_t t0 = static_cast<uint64_t>(wall_clock64());
    uint32_t s;
    while ((s = atomic_load_u32(state)) == 0u) {
      if (static_cast<uint64_t>(wall_clock64()) - t0 >= ticks) {
        if (atomicCAS(state, 0u, kCheckinAbort) == 0u) atomicOr(err, kErrTailCheckin);
      } else {
        __builtin_amdgcn_s_sleep(1);
      }
    }
    *s_ok = s == kCheckinGo ? 1 : 0;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Rounds round0 .. round_cap of one call: color phase, barrier, detect phase,
// barrier, stop when the next worklist is empty.
// *left receives 1 if the cap was reached with vertices left.
__global__ __launch_bounds__(kBlock) void inc_tail_kernel(KeySource k, IncRoundSet set, BinLayout L, int round0,
                                                          int round_cap, uint32_t* bar, int32_t* err,
                                                          int32_t* left, uint64_t deadline,
                                                          uint64_t checkin_ticks) {
  __shared__ union {
    IncColorShared c;
    IncDetectShared d;
  } sh;
  __shared__ int32_t s_ok;
  __shared__ IncPre s_pre;  // next round's map and largest color, read once per round
  if (!tail_checkin(bar, err, checkin_ticks, &s_ok)) return;
  for (int r = round0; r <= round_cap; ++r) {
    IncBufs b = set.base;
    const bool odd = (r & 1) != 0;
    b.wl_in = odd ? set.wl0 : set.wl1;
    b.wl_out = odd ? set.wl1 : set.wl0;
    b.cnt_in = odd ? set.cnt0 : set.cnt1;
    b.cnt_out = odd ? set.cnt1 : set.cnt0;
    b.A_in = (r == 1 || (r == 2 && set.defer1)) ? set.A0 : set.base.A_out;
    b.uniform = r == 1 ? set.uniform1 : 0;
    b.defer_split = r == 1 ? set.defer1 : 0;
    const bool first = r == round0;
    inc_color_phase<1>(b, L, r, sh.c, first ? nullptr : &s_pre);
    if (!grid_sync(bar, err, deadline, &s_ok)) return;
    inc_detect_phase<1>(k, b, L, r, sh.d, first ? nullptr : &s_pre);
    if (!grid_sync(bar, err, deadline, &s_ok)) return;
    if (threadIdx.x == 0) {
      make_inc_map_from(b.cnt_out, L, s_pre.M);  // the next round's worklist counts
      s_pre.maxc = ld_dev(b.maxc);
    }
    __syncthreads();
    const bool done = s_pre.M.total == 0;
    if (done) return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st_dev(left, 1);
}

int tail_blocks_resident() {
  static int cache = 0;
  if (cache == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, inc_tail_kernel, kBlock, 0) != hipSuccess)
      cache = -1;
    else
      cache = std::max(0, per * cus);
  }
  return cache;
}

bool launch_inc_tail(const KeySource& k, const IncRoundSet& set, const BinLayout& L, int round0, int round_cap,
                    uint32_t* bar, int32_t* err, int32_t* left, int grid, int32_t checkin_us, hipStream_t st) {
  static uint64_t khz = 0;
  if (khz == 0) {
    int dev = 0, rate = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate <= 0)
      rate = 100000;
    khz = static_cast<uint64_t>(rate);
  }
  KeySource kk = k;
  IncRoundSet ss = set;
  BinLayout ll = L;
  int r0 = round0, rc = round_cap;
  uint64_t dl = khz * 1000ull * kTailBarrierSeconds;
  uint64_t ci = checkin_us < 0 ? 0ull : khz * static_cast<uint64_t>(checkin_us) / 1000ull;
  void* args[] = {&kk, &ss, &ll, &r0, &rc, &bar, &err, &left, &dl, &ci};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(inc_tail_kernel), dim3(grid), dim3(kBlock), args, 0,
                                    st) == hipSuccess;
}

// ---------------------------------------------------------------------------
// setup: list lengths, bitset sizes, list materialization, initial pushes
// ---------------------------------------------------------------------------

// len(v): entries of v's list.  D1: deg(v).  D2: the two-hop walk without v
// itself, sum over u in N(v) of deg(u) = work(v) - deg(v) (v appears once in
// each neighbour's row).  PD2: sum over the rows of column v of deg(row) - 1
// = work(v) - 2 (rows of v), work counting each row entry and the row's
// columns.  words(v): the bitset words beyond word 0 (which every vertex has
// in the dense array) that cover colors 1..min(len, ids)+1, the largest
// first fit v can ever take (ids: the vertices a walk can reach, g.ids or
// else n).
template <int MODE>
__global__ __launch_bounds__(kBlock) void inc_sizes_kernel(GraphView g, const int32_t* work, int32_t* len,
                                                           int32_t* words, int32_t* alen0,
                                                           unsigned long long* total) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  int64_t l = 0;
  if (v < g.n) {
    const int64_t d1 = g.rp[v + 1] - g.rp[v];
    l = MODE == kD1 ? d1 : static_cast<int64_t>(ld_dev(&work[v])) - (MODE == kPD2 ? 2 : 1) * d1;
    if (l < 0) l = 0;
  }
  __shared__ unsigned long long s_t;
  if (threadIdx.x == 0) s_t = 0ull;
  __syncthreads();
  uint64_t t = wsum(static_cast<uint64_t>(l));
  if (lane_id() == 0 && t) atomicAdd(&s_t, static_cast<unsigned long long>(t));
  __syncthreads();
  if (threadIdx.x == 0 && s_t) atomicAdd(total, s_t);
  if (v >= g.n) return;
  const int32_t lc = static_cast<int32_t>(l > INT_MAX ? INT_MAX : l);
  st_dev(&len[v], lc);
  st_dev(&alen0[v], lc);
  st_dev(&words[v], static_cast<int32_t>(min<int64_t>(l, max(g.n, g.ids)) / 32));
}

// Materializes the two-hop list of a vertex with a short first hop (one
// thread).  At most len(v) entries are written.  Every fill keeps only
// members below g.limit: the colorable vertices, or (a rank's ghost step,
// whose walks pass through ghosts) the owned ones.
template <int MODE>
// Every fill stores the number of entries it wrote as the list length
// (alen), so that a list never exposes an unwritten slot, even where the
// graph breaks the input contract and the walk is shorter than its bound.
__global__ __launch_bounds__(kBlock) void inc_fill_kernel(GraphView g, const int32_t* aoff, const int32_t* len,
                                                          int32_t* A, int32_t* alen) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= g.n || g.rp[v + 1] - g.rp[v] > kFillThread) return;
  const int32_t base = ld_dev(&aoff[v]);
  const int32_t end = base + ld_dev(&len[v]);
  int32_t o = base;
  for (int32_t q = g.rp[v]; q < g.rp[v + 1]; ++q) {
    const int32_t u = g.ci[q];
    if (MODE == kD2 && u < g.limit && o < end) st_dev(&A[o++], u);
    for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
      const int32_t x = g.ci2[p];
      if (x != v && x < g.limit && o < end) st_dev(&A[o++], x);
    }
  }
  st_dev(&alen[v], o - base);
}

// Two-hop lists of vertices with kFillThread < first-hop length <= kSetupHeavy:
// a wavefront per vertex; each pass takes 64 first-hop entries, scans their
// entry counts across the wavefront and writes them in first-hop order.
template <int MODE>
__global__ __launch_bounds__(kBlock) void inc_fill_wave_kernel(GraphView g, const int32_t* aoff,
                                                               const int32_t* len, int32_t* A, int32_t* alen) {
  const int32_t v = static_cast<int32_t>((blockIdx.x * kBlock + threadIdx.x) / kWave);
  if (v >= g.n) return;
  const int32_t q0 = g.rp[v], q1 = g.rp[v + 1];
  if (q1 - q0 <= kFillThread || q1 - q0 > kSetupHeavy) return;
  const int32_t end = ld_dev(&aoff[v]) + ld_dev(&len[v]);
  int32_t out = ld_dev(&aoff[v]);
  for (int32_t qb = q0; qb < q1; qb += kWave) {
    const int32_t q = qb + lane_id();
    int32_t u = -1, cnt = 0;
    if (q < q1) {
      u = g.ci[q];
      cnt = (MODE == kD2 && u < g.limit) ? 1 : 0;
      for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
        const int32_t x = g.ci2[p];
        cnt += x != v && x < g.limit;
      }
    }
    int32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int32_t y = __shfl_up(incl, off, kWave);
      if (lane_id() >= off) incl += y;
    }
    int32_t o = out + incl - cnt;
    if (u >= 0) {
      if (MODE == kD2 && u < g.limit && o < end) st_dev(&A[o++], u);
      for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
        const int32_t x = g.ci2[p];
        if (x != v && x < g.limit && o < end) st_dev(&A[o++], x);
      }
    }
    out += __shfl(incl, kWave - 1, kWave);
  }
  if (lane_id() == 0) st_dev(&alen[v], min(out, end) - ld_dev(&aoff[v]));
}

// Two-hop lists of the heavy (deferred) vertices: a workgroup per vertex;
// each pass takes kBlock first-hop entries, scans their entry counts across
// the workgroup and writes them in first-hop order.
template <int MODE>
__global__ __launch_bounds__(kBlock) void inc_fill_heavy_kernel(GraphView g, const int32_t* aoff,
                                                                const int32_t* len, int32_t* A,
                                                                const int32_t* deferred, const int32_t* nd_ptr,
                                                                int32_t* grab, int32_t* alen) {
  __shared__ int32_t s_i;
  __shared__ int32_t s_wt[kWavesPerBlock];
  const int32_t nd = ld_dev(nd_ptr);
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  while (true) {
    if (tid == 0) s_i = atomicAdd(grab, 1);
    __syncthreads();
    const int32_t i = s_i;
    __syncthreads();
    if (i >= nd) break;
    const int32_t v = ld_dev(&deferred[i]);
    const int32_t base = ld_dev(&aoff[v]);
    const int32_t end = base + ld_dev(&len[v]);
    int32_t out = base;
    for (int32_t q0 = g.rp[v]; q0 < g.rp[v + 1]; q0 += kBlock) {
      const int32_t q = q0 + tid;
      int32_t u = -1, cnt = 0;
      if (q < g.rp[v + 1]) {
        u = g.ci[q];
        cnt = (MODE == kD2 && u < g.limit) ? 1 : 0;
        for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
          const int32_t x = g.ci2[p];
          cnt += x != v && x < g.limit;
        }
      }
      // inclusive scan of cnt within the wavefront, then across wavefronts
      int32_t incl = cnt;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, kWave);
        if (lane_id() >= off) incl += y;
      }
      if (lane_id() == kWave - 1) s_wt[wave] = incl;
      __syncthreads();
      int32_t wbase = 0, tot = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wave) wbase += s_wt[w];
        tot += s_wt[w];
      }
      int32_t o = out + wbase + incl - cnt;
      if (u >= 0) {
        if (MODE == kD2 && u < g.limit && o < end) st_dev(&A[o++], u);
        for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
          const int32_t x = g.ci2[p];
          if (x != v && x < g.limit && o < end) st_dev(&A[o++], x);
        }
      }
      out += tot;
      __syncthreads();
    }
    if (tid == 0) st_dev(&alen[v], min(out, end) - base);
  }
}

// Committed initial colors enter the bitsets of their uncolored neighbours.
__global__ __launch_bounds__(kBlock) void inc_init_push_kernel(IncBufs b, int32_t n, const int32_t* A0) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const int32_t c = ld_dev(&b.C[v]);
  if (c == 0) return;
  uint64_t pushes = 0;
  const int32_t base = ld_dev(&b.aoff[v]);
  const int32_t len = ld_dev(&b.alen_in[v]);
  for (int32_t e = 0; e < len; ++e) {
    const int32_t x = ld_dev(&A0[base + e]);
    if (ld_dev(&b.C[x]) == 0) push_color<1>(b, x, c, pushes);
  }
}

// Committed colors of every walk member, list member or not (a rank's
// ghosts above g.limit), enter the bitset of each uncolored vertex: one
// thread per first-hop entry, which walks its second-hop row.
template <int MODE>
__global__ __launch_bounds__(kBlock) void inc_init_pull_kernel(GraphView g, int32_t nnz1, IncBufs b) {
  const int32_t q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nnz1) return;
  const int32_t v = row_of(g.rp, g.n, q);
  if (ld_dev(&b.C[v]) != 0) return;
  auto take = [&](int32_t x) {
    const int32_t c = ld_dev(&b.C[x]);
    if (c == 0) return;
    uint32_t* p = f_word<0>(b, v, (c - 1) >> 5);
    const uint32_t bit = 1u << ((c - 1) & 31);
    if (p && !(*p & bit)) atomicOr(p, bit);
  };
  const int32_t u = g.ci[q];
  if (MODE == kD2) take(u);
  for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
    const int32_t x = g.ci2[p];
    if (x != v) take(x);
  }
}

static inline int blocks_for(int64_t n) { return static_cast<int>((n + kBlock - 1) / kBlock); }

// Per-call state of the byte and bit arrays: T8 cleared (0 is no tentative
// color), the committed bit of every vertex with an initial color set.  One
// thread per bitmap word.
__global__ __launch_bounds__(kBlock) void inc_state_init_kernel(int32_t n, const int32_t* C, uint8_t* T8,
                                                                uint32_t* done) {
  const int32_t w = blockIdx.x * kBlock + threadIdx.x;
  if (w > n / 32) return;
  uint32_t bits = 0;
  for (int i = 0; i < 32; ++i) {
    const int32_t v = 32 * w + i;
    if (v < n) {
      bits |= (ld_dev(&C[v]) != 0 ? 1u : 0u) << i;
      T8[v] = 0;
    }
  }
  done[w] = bits;
}

void launch_inc_state_init(int32_t n, const int32_t* C, uint8_t* T8, uint32_t* done, hipStream_t st) {
  hipLaunchKernelGGL(inc_state_init_kernel, dim3(blocks_for(n / 32 + 1)), dim3(kBlock), 0, st, n, C, T8, done);
}

void launch_inc_color(const IncBufs& b, const BinLayout& L, int round, int grid, hipStream_t st) {
  hipLaunchKernelGGL(inc_color_kernel, dim3(grid), dim3(kBlock), 0, st, b, L, round);
}
void launch_inc_detect(const KeySource& k, const IncBufs& b, const BinLayout& L, int round, int grid,
                       hipStream_t st) {
  hipLaunchKernelGGL(inc_detect_kernel, dim3(grid), dim3(kBlock), 0, st, k, b, L, round);
}
template <int MODE>
void launch_inc_sizes(const GraphView& g, const int32_t* work, int32_t* len, int32_t* words, int32_t* alen0,
                      unsigned long long* total, hipStream_t st) {
  if (g.n > 0)
    hipLaunchKernelGGL(inc_sizes_kernel<MODE>, dim3(blocks_for(g.n)), dim3(kBlock), 0, st, g, work, len, words,
                       alen0, total);
}
// Duplicates of the materialized two-hop lists (a column pair sharing
// several rows, a vertex reachable through several middle vertices) are
// removed once per call from every list longer than kDedupMin entries: the
// lists are sets, so the colorings do not change.  A workgroup walks one long
// list at a time with its own bitmap of the id range; an entry is kept when
// its atomic OR finds the bit clear.  The list is compacted in place (each
// step's entries are read before the barrier that precedes its writes), then
// the bits of the kept entries are cleared again.
constexpr int32_t kDedupMin = 4096;

__global__ __launch_bounds__(kBlock) void inc_dedup_kernel(int32_t n, const int32_t* aoff, int32_t* alen,
                                                           int32_t* A, uint32_t* bitmaps, int32_t words,
                                                           const int32_t* skip_rp) {
  __shared__ int32_t s_wc[kWavesPerBlock];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  uint32_t* bm = bitmaps + static_cast<size_t>(blockIdx.x) * static_cast<size_t>(words);
  constexpr int32_t step = kBlock * kIncBatch;
  for (int32_t v = blockIdx.x; v < n; v += gridDim.x) {
    const int32_t len = ld_dev(&alen[v]);
    if (len <= kDedupMin) continue;
    if (skip_rp && skip_rp[v + 1] - skip_rp[v] > kSetupHeavy) continue;  // built as sets already
    int32_t* L = A + ld_dev(&aoff[v]);
    int32_t kept = 0;
    for (int32_t e0 = 0; e0 < len; e0 += step) {
      int32_t x[kIncBatch];
      bool keep[kIncBatch];
      int32_t cnt = 0;
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) {
        const int32_t e = e0 + j * kBlock + tid;
        x[j] = e < len ? ld_dev(&L[e]) : -1;
      }
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j) {
        keep[j] = false;
        if (x[j] >= 0) {
          const uint32_t bit = 1u << (x[j] & 31);
          keep[j] = (atomicOr(&bm[x[j] >> 5], bit) & bit) == 0u;
        }
        cnt += keep[j] ? 1 : 0;
      }
      int32_t incl = cnt;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, kWave);
        if (lane_id() >= o) incl += y;
      }
      if (lane_id() == kWave - 1) s_wc[wave] = incl;
      __syncthreads();
      int32_t pos = kept + incl - cnt;
      int32_t tot = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wave) pos += s_wc[w];
        tot += s_wc[w];
      }
#pragma unroll
      for (int j = 0; j < kIncBatch; ++j)
        if (keep[j]) st_dev(&L[pos++], x[j]);
      kept += tot;
      __syncthreads();
    }
    for (int32_t e = tid; e < kept; e += kBlock) st_dev(&bm[ld_dev(&L[e]) >> 5], 0u);
    if (tid == 0) st_dev(&alen[v], kept);
    __syncthreads();
  }
}

// Two-hop sets of heavy (deferred) vertices built as bitmaps, for graphs
// where one bitmap of the id range per heavy vertex is affordable: every
// first-hop entry of every heavy vertex is its own thread (blockIdx.y picks
// the vertex, the x blocks stride over its entries), so the longest walk is
// spread over many workgroups instead of one; the bits then become the list,
// duplicate-free and in id order.
template <int MODE>
__global__ __launch_bounds__(kBlock) void inc_mark_kernel(GraphView g, const int32_t* deferred, int32_t i0,
                                                         uint32_t* bm, int32_t words, int32_t* alen) {
  const int32_t v = ld_dev(&deferred[i0 + static_cast<int32_t>(blockIdx.y)]);
  uint32_t* m = bm + static_cast<size_t>(blockIdx.y) * static_cast<size_t>(words);
  if (blockIdx.x == 0 && threadIdx.x == 0) st_dev(&alen[v], 0);
  const int32_t q1 = g.rp[v + 1];
  for (int32_t q = g.rp[v] + static_cast<int32_t>(blockIdx.x * kBlock + threadIdx.x); q < q1;
       q += static_cast<int32_t>(gridDim.x * kBlock)) {
    const int32_t u = g.ci[q];
    // a plain (cacheable) read first skips most atomics of bits already set;
    // a stale read only costs an atomic that was not needed
    if (MODE == kD2 && u != v && u < g.limit && !(m[u >> 5] & (1u << (u & 31))))
      atomicOr(&m[u >> 5], 1u << (u & 31));
    for (int32_t p = g.rp2[u]; p < g.rp2[u + 1]; ++p) {
      const int32_t x = g.ci2[p];
      if (x != v && x < g.limit && !(m[x >> 5] & (1u << (x & 31)))) atomicOr(&m[x >> 5], 1u << (x & 31));
    }
  }
}

__global__ __launch_bounds__(kBlock) void inc_bitmap_list_kernel(const int32_t* deferred, int32_t i0,
                                                                 const uint32_t* bm, int32_t words,
                                                                 const int32_t* aoff, int32_t* alen, int32_t* A) {
  const int32_t v = ld_dev(&deferred[i0 + static_cast<int32_t>(blockIdx.y)]);
  const uint32_t* m = bm + static_cast<size_t>(blockIdx.y) * static_cast<size_t>(words);
  int32_t* out = A + ld_dev(&aoff[v]);
  for (int32_t w0 = static_cast<int32_t>(blockIdx.x * kBlock); w0 < words;
       w0 += static_cast<int32_t>(gridDim.x * kBlock)) {
    const int32_t w = w0 + static_cast<int32_t>(threadIdx.x);
    uint32_t x = w < words ? ld_dev(&m[w]) : 0u;
    const int32_t c = __popc(x);
    int32_t incl = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(incl, o, kWave);
      if (lane_id() >= o) incl += y;
    }
    const int32_t tot = __shfl(incl, kWave - 1, kWave);
    int32_t base = 0;
    if (lane_id() == kWave - 1 && tot > 0) base = atomicAdd(&alen[v], tot);
    base = __shfl(base, kWave - 1, kWave);
    int32_t pos = base + incl - c;
    while (x) {
      const int bit = __builtin_ctz(x);
      x &= x - 1u;
      st_dev(&out[pos++], 32 * w + bit);
    }
  }
}

template <int MODE>
void launch_inc_fill(const GraphView& g, const int32_t* aoff, const int32_t* len, int32_t* A, int32_t* alen,
                     const int32_t* deferred, const int32_t* nd, int32_t* grab, bool heavy, hipStream_t st) {
  if (g.n <= 0) return;
  hipLaunchKernelGGL(inc_fill_kernel<MODE>, dim3(blocks_for(g.n)), dim3(kBlock), 0, st, g, aoff, len, A, alen);
  const int64_t wave_blocks = (static_cast<int64_t>(g.n) + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(inc_fill_wave_kernel<MODE>, dim3(static_cast<uint32_t>(wave_blocks)), dim3(kBlock), 0, st, g,
                     aoff, len, A, alen);
  if (heavy)
    hipLaunchKernelGGL(inc_fill_heavy_kernel<MODE>, dim3(std::min(blocks_for(g.n), 512)), dim3(kBlock), 0, st, g,
                       aoff, len, A, deferred, nd, grab, alen);
}

template <int MODE>
void launch_inc_bitmap_sets(const GraphView& g, const int32_t* deferred, int32_t i0, int32_t nb, uint32_t* bm,
                            int32_t words, const int32_t* aoff, int32_t* alen, int32_t* A, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(inc_mark_kernel<MODE>, dim3(kSetsBlocksPerVertex, nb), dim3(kBlock), 0, st, g, deferred, i0, bm,
                     words, alen);
  const int wx = std::max(1, std::min(kSetsBlocksPerVertex, (words + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(inc_bitmap_list_kernel, dim3(wx, nb), dim3(kBlock), 0, st, deferred, i0, bm, words, aoff, alen,
                     A);
}
int dedup_grid(int32_t words) {
  const size_t per = sizeof(uint32_t) * static_cast<size_t>(words);
  const size_t cap = static_cast<size_t>(256) << 20;  // bitmaps of all workgroups together
  return static_cast<int>(std::max<size_t>(8, std::min<size_t>(256, cap / std::max<size_t>(per, 1))));
}

void launch_inc_dedup(int32_t n, const int32_t* aoff, int32_t* alen, int32_t* A, uint32_t* bitmaps, int32_t words,
                      int grid, const int32_t* skip_rp, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(inc_dedup_kernel, dim3(grid), dim3(kBlock), 0, st, n, aoff, alen, A, bitmaps, words, skip_rp);
}

void launch_inc_init_push(const IncBufs& b, int32_t n, const int32_t* A0, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(inc_init_push_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, n, A0);
}
template <int MODE>
void launch_inc_init_pull(const GraphView& g, int32_t nnz1, const IncBufs& b, hipStream_t st) {
  if (nnz1 > 0)
    hipLaunchKernelGGL(inc_init_pull_kernel<MODE>, dim3(blocks_for(nnz1)), dim3(kBlock), 0, st, g, nnz1, b);
}
template void launch_inc_init_pull<kD2>(const GraphView&, int32_t, const IncBufs&, hipStream_t);
template void launch_inc_init_pull<kPD2>(const GraphView&, int32_t, const IncBufs&, hipStream_t);
template void launch_inc_sizes<kD1>(const GraphView&, const int32_t*, int32_t*, int32_t*, int32_t*,
                                    unsigned long long*, hipStream_t);
template void launch_inc_sizes<kD2>(const GraphView&, const int32_t*, int32_t*, int32_t*, int32_t*,
                                    unsigned long long*, hipStream_t);
template void launch_inc_sizes<kPD2>(const GraphView&, const int32_t*, int32_t*, int32_t*, int32_t*,
                                     unsigned long long*, hipStream_t);
template void launch_inc_bitmap_sets<kD2>(const GraphView&, const int32_t*, int32_t, int32_t, uint32_t*, int32_t,
                                          const int32_t*, int32_t*, int32_t*, hipStream_t);
template void launch_inc_bitmap_sets<kPD2>(const GraphView&, const int32_t*, int32_t, int32_t, uint32_t*, int32_t,
                                           const int32_t*, int32_t*, int32_t*, hipStream_t);
template void launch_inc_fill<kD2>(const GraphView&, const int32_t*, const int32_t*, int32_t*, int32_t*,
                                   const int32_t*, const int32_t*, int32_t*, bool, hipStream_t);
template void launch_inc_fill<kPD2>(const GraphView&, const int32_t*, const int32_t*, int32_t*, int32_t*,
                                    const int32_t*, const int32_t*, int32_t*, bool, hipStream_t);

int exclusive_scan_i32(const int32_t* in, int32_t* out, int32_t n_plus_1, void* tmp, size_t* tmp_bytes,
                       hipStream_t st) {
  return hipcub::DeviceScan::ExclusiveSum(tmp, *tmp_bytes, in, out, n_plus_1, st) == hipSuccess ? 0 : -1;
}

int resident_inc_blocks() {
  static int cache = 0;
  if (cache == 0) {
    int dev = 0, cus = 0, a = 0, d = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, inc_color_kernel, kBlock, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&d, inc_detect_kernel, kBlock, 0) != hipSuccess) {
      cache = 2048;
    } else {
      cache = std::max(8, (std::max(1, std::min(a, d)) * cus) / 8 * 8);
    }
  }
  return cache;
}

}  // namespace gcol
