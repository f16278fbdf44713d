// Host/device interface of the round kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace gcol {

// Degree bins: bins 0..2 map a sub-wavefront group (or a whole wavefront) to
// a vertex, bin 3 a whole workgroup, bin 4 several workgroups (split).  The
// bin of a vertex depends only on its static work (adjacency entries read per
// visit), so worklists keep their bins for the whole call.
constexpr int kBins = 5;
constexpr int kSplitBin = 4;
constexpr int kBlockBin = 3;
constexpr int kOvfWords = 1024;  // LDS overflow bitset of the workgroup bins: 32768 colors

struct GraphView {
  int32_t n;       // colorable vertices (ids [0, n))
  int32_t limit;   // D1: neighbour ids >= limit are ignored (ghost-blind phase); D2/PD2: the
                   // incremental engine's lists keep members below limit only
  const int32_t* rp;   // hop 1: D1/D2 adjacency row_ptr; PD2 CSC col_ptr (column -> rows)
  const int32_t* ci;   // hop 1: D1/D2 adjacency col_idx; PD2 CSC row_idx
  const int32_t* rp2;  // hop 2: D2 adjacency row_ptr; PD2 CSR row_ptr (row -> columns)
  const int32_t* ci2;  // hop 2: D2 adjacency col_idx; PD2 CSR col_idx
  int32_t ids = 0;     // D2/PD2: ids the walks reach (0: n); above limit, such members are
                       // constraints only (a rank's ghosts): the incremental engine keeps
                       // them out of its lists and takes their colors once, before round 1
};

struct BinLayout {
  int32_t off[kBins];     // start of each bin's region in the worklist buffers
  int32_t lanes[3];       // lanes per vertex of bins 0..2 (power of two <= 64)
  int32_t split_chunks;   // workgroups per split vertex
  int32_t grab;           // tiles of bins 0..2 taken per dynamic grab
  int32_t hi[3];          // work bounds of bins 0..2 (the incremental engine also bins its
                          // active lists by length with them)
};

// Per-round buffers (device pointers, resolved for the round's parity).
struct RoundBufs {
  int32_t* C;                 // committed colors (the output array)
  int32_t* T;                 // tentative colors
  const int32_t* work;        // static work per vertex
  const int32_t* wl_in;       // worklist W_r (bin regions; bin 4 holds split indices)
  int32_t* wl_out;            // worklist W_{r+1}
  const int32_t* cnt_in;      // |W_r| per bin
  int32_t* cnt_out;           // |W_{r+1}| per bin (zeroed by the color kernel)
  int32_t* tile_ctr;          // [0] color-kernel grab counter, [1] detect-kernel grab counter
  const int32_t* split_vertex;// split index -> vertex
  uint32_t* split_mask;       // per split index: capw words of forbidden-color bits (bit c-1)
  int32_t capw;
  uint32_t* split_ctr;        // per split index: arrival counter of its chunks
  uint32_t* split_flag;       // per split index: "lost" flag of the detect phase
  int32_t* maxc;              // largest committed color
  unsigned long long* visits; // [0] sum |W_r|, [1] sum work(W_r)
  int32_t* trace;             // |W_r| per round (nullable)
  int32_t trace_cap;
  int32_t* rounds_done;       // last round with a non-empty worklist
};

template <int MODE>
void launch_color_round(const GraphView& g, const KeySource& k, const RoundBufs& b,
                        const BinLayout& L, int round, int grid, hipStream_t st);
template <int MODE>
void launch_detect_round(const GraphView& g, const KeySource& k, const RoundBufs& b,
                         const BinLayout& L, int round, int grid, hipStream_t st);

// Workgroups a round kernel can use for the given per-bin counts: light
// chunks of kBlock entries plus heavy units.
inline int64_t round_units(const int32_t cnt[kBins], const BinLayout& L) {
  int64_t u = 0;
  for (int b = 0; b < 3; ++b) u += (cnt[b] + kBlock - 1) / kBlock;
  u += cnt[kBlockBin];
  u += static_cast<int64_t>(cnt[kSplitBin]) * L.split_chunks;
  return u;
}

// Workgroups of the round kernels that are resident on the device at once
// (occupancy x compute units), a multiple of 8 (one share per XCD).
int resident_round_blocks(int mode);

}  // namespace gcol
