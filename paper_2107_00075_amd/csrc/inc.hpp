// Interface of the incremental engine (inc.hip).
#pragma once

#include "rounds.hpp"

namespace gcol {

struct IncBufs {
  int32_t* C;                  // committed colors
  int32_t* T;                  // tentative colors
  const int32_t* work;         // static work per vertex (statistics)
  const int32_t* wl_in;        // worklist W_r (bin regions, vertex ids)
  int32_t* wl_out;             // worklist W_{r+1}
  const int32_t* cnt_in;       // |W_r| per bin
  int32_t* cnt_out;            // |W_{r+1}| per bin
  int32_t* tile_ctr;           // [1]: heavy-unit counter of the detect kernel
  const int32_t* aoff;         // list offsets (D1: row_ptr; D2/PD2: prefix of list lengths)
  const int32_t* A_in;         // active lists of round r
  int32_t* A_out;              // compacted lists (the same array as A_in after round 1: in place)
  const int32_t* alen_in;      // list lengths of round r
  int32_t* alen_out;           // list lengths for round r+1 (the same array as alen_in); after the
                               // first pass: the higher-key part at the front of a list
  int32_t* llen;               // after the first pass: the lower-key part at the back of a list
  int32_t uniform;             // 1 in round 1 without initial colors: every vertex is uncolored and
                               // every tentative color is 1
  int32_t defer_split;         // round 1 without initial colors: losers keep the read-only lists
                               // untouched (round 2 splits and compacts them)
  uint8_t* T8;                 // tentative colors as bytes, written and read in rounds <= t8_last
  int32_t t8_last;             // last round whose tentative colors all fit a byte: a color taken in
                               // round r is at most (largest initial color) + r
  uint32_t* done;              // committed vertices, one bit each (the compaction test)
  const int32_t* fw_off;       // offsets of the bitset words beyond word 0 in Fx, n+1 entries
  uint32_t* F;                 // forbidden-color bitsets, word 0 (colors 1..32) of every vertex
  uint32_t* Fx;                // their further words (bit c-1 = color c throughout)
  int32_t* maxc;               // largest committed color
  unsigned long long* acc;     // [0] sum |W|, [1] sum work, [2] list entries, [3] color bytes,
                               // [4] detect bytes, [5] pushes, [6] and [7] color and detect bytes
                               // of the tail kernel
  int32_t bytes_slot = 3;      // where this launch adds its color bytes (detect: the next slot)
  int32_t* trace;
  int32_t trace_cap;
  int32_t* rounds_done;
  int32_t round_base = 0;      // rounds the call ran before this engine run (trace and rounds_done
                               // count from there; the engine's own logic counts from 1)
};

// Vertices per light chunk of a bin with `lanes` lanes per vertex: a chunk
// takes kIncPasses passes of the workgroup's lane groups, so that a bin of
// wide groups (whose vertices are processed few at a time) is spread over
// many workgroups.
constexpr int kIncPasses = 2;
__host__ __device__ inline int32_t inc_chunk_size(int32_t lanes) {
  const int32_t c = (kBlock / lanes) * kIncPasses;
  return c < kBlock ? c : kBlock;
}
// Work units of a round: light chunks plus one unit per heavy vertex.
inline int64_t inc_round_units(const int32_t cnt[kBins], const BinLayout& L) {
  int64_t u = 0;
  for (int b = 0; b < 3; ++b) {
    const int32_t cs = inc_chunk_size(L.lanes[b]);
    u += (cnt[b] + cs - 1) / cs;
  }
  return u + cnt[kBlockBin] + cnt[kSplitBin];
}

// The buffers of every round of the tail kernel: the fields all rounds share
// (base: as for round 3 and later), the worklist ping-pong, and the unsplit
// lists of the first rounds.  Rounds are built from it with scalar selects
// (no dynamically indexed array of buffer sets, which would live in scratch).
struct IncRoundSet {
  IncBufs base;
  int32_t* wl0;
  int32_t* wl1;
  int32_t* cnt0;
  int32_t* cnt1;
  const int32_t* A0;      // the unsplit lists (round 1; round 2 when round 1 deferred the split)
  int32_t uniform1;       // round 1 is uniform
  int32_t defer1;         // round 1 defers the split to round 2
};

constexpr int32_t kErrTailBarrier = 0x100;  // error bit: a tail-kernel grid barrier gave up
constexpr int32_t kErrTailCheckin = 0x200;  // the tail kernel's workgroups were not all resident: none ran a round
constexpr int kTailBarrierSeconds = 30;     // a grid barrier of the tail kernel gives up after this long
constexpr int32_t kTailCheckinDefaultUs = 2000;  // how long the tail's workgroups wait for each other at entry
// tail-kernel barrier words (32 apart: one cache line each): top arrivals at
// 0, the generation at kBarGen, group g's arrivals at kBarGroup + 32 g, the
// entry check-in's arrivals at kBarCheckin and its decision at kBarState
constexpr int kBarGen = 32;
constexpr int kBarGroup = 64;
constexpr int kBarCheckin = kBarGroup + 32 * 8;
constexpr int kBarState = kBarCheckin + 32;
constexpr int kBarWords = kBarState + 32;
constexpr int32_t kTailDefault = 32768;     // default worklist size at which the tail kernel takes over

void launch_inc_color(const IncBufs& b, const BinLayout& L, int round, int grid, hipStream_t st);
// All remaining rounds in one cooperative launch (grid <= tail_blocks_resident());
// false if the runtime refused the launch.
// checkin_us: how long the workgroups wait for each other at entry (< 0: not
// at all); if they are not all resident by then, none runs a round and *err
// receives kErrTailCheckin.
bool launch_inc_tail(const KeySource& k, const IncRoundSet& set, const BinLayout& L, int round0, int round_cap,
                    uint32_t* bar, int32_t* err, int32_t* left, int grid, int32_t checkin_us, hipStream_t st);
// Workgroups of the tail kernel that fit on the device at once (-1: unknown).
int tail_blocks_resident();
void launch_inc_detect(const KeySource& k, const IncBufs& b, const BinLayout& L, int round, int grid,
                       hipStream_t st);
template <int MODE>
void launch_inc_sizes(const GraphView& g, const int32_t* work, int32_t* len, int32_t* words, int32_t* alen0,
                      unsigned long long* total, hipStream_t st);
// Materializes the two-hop lists: one thread per vertex of first-hop length
// up to kFillThread, a wavefront per vertex up to kSetupHeavy, and (heavy)
// one workgroup per deferred vertex.
constexpr int32_t kFillThread = 16;
template <int MODE>
void launch_inc_fill(const GraphView& g, const int32_t* aoff, const int32_t* len, int32_t* A, int32_t* alen,
                     const int32_t* deferred, const int32_t* nd, int32_t* grab, bool heavy, hipStream_t st);
// The lists of deferred vertices i0 .. i0+nb-1 as duplicate-free sets, through
// bitmaps of `words` words each (bm: nb x words, zeroed by the caller); alen
// receives the set sizes.
constexpr int kSetsBlocksPerVertex = 64;
constexpr int64_t kSetsMaxWords = int64_t{1} << 28;    // all heavy bitmaps together (1 GiB), else per-list
constexpr int64_t kSetsBatchWords = int64_t{1} << 27;  // bitmaps of one batch (512 MiB)
template <int MODE>
void launch_inc_bitmap_sets(const GraphView& g, const int32_t* deferred, int32_t i0, int32_t nb, uint32_t* bm,
                            int32_t words, const int32_t* aoff, int32_t* alen, int32_t* A, hipStream_t st);
void launch_inc_init_push(const IncBufs& b, int32_t n, const int32_t* A0, hipStream_t st);
// Initial colors of every member of each uncolored vertex's walk, lists or
// not (g.ids > g.limit), into its bitset; nnz1 = g.rp[g.n].
template <int MODE>
void launch_inc_init_pull(const GraphView& g, int32_t nnz1, const IncBufs& b, hipStream_t st);
// T8 cleared and the committed bits (n / 32 + 1 words) set from C.
void launch_inc_state_init(int32_t n, const int32_t* C, uint8_t* T8, uint32_t* done, hipStream_t st);
// Removes duplicates from the long two-hop lists (alen in: capacity, out:
// distinct entries); bitmaps: grid x words zeroed uint32 (left zeroed).
int dedup_grid(int32_t words);
// skip_rp (nullable): the first-hop row offsets; vertices deferred by their
// first-hop length are skipped (their lists were built as sets).
void launch_inc_dedup(int32_t n, const int32_t* aoff, int32_t* alen, int32_t* A, uint32_t* bitmaps, int32_t words,
                      int grid, const int32_t* skip_rp, hipStream_t st);
int resident_inc_blocks();

// Exclusive prefix sum of n+1 int32 values (the last input is 0, so out[n] is
// the total), with temporary storage from the caller.
int exclusive_scan_i32(const int32_t* in, int32_t* out, int32_t n_plus_1, void* tmp, size_t* tmp_bytes,
                       hipStream_t st);

}  // namespace gcol
