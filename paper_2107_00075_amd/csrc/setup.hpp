// Declarations of the per-call setup kernels (setup.hip).
#pragma once

#include "rounds.hpp"

namespace gcol {

// D2/PD2 vertices with a first hop longer than this are handled by a whole
// workgroup in the setup kernels.
constexpr int32_t kSetupHeavy = 1024;

struct BinSetup {
  int32_t bin_hi[kBins - 1];         // work upper bound of bins 0..3
  const int32_t* init;               // nullable initial colors
  int32_t* C;                        // committed colors (written: init or 0)
  int32_t* T;                        // tentative colors (written: init or 0)
  int32_t* work;                     // out: static work per vertex
  int8_t* bin;                       // out: bin per vertex
  int32_t* count_all;                // out: vertices per bin
  int32_t* count_unc;                // out: uncolored vertices per bin
  int32_t* maxc;                     // out: largest initial color
  int32_t* max_split_work;           // out: largest work among uncolored split vertices
  int32_t* max_work;                 // out: largest work among uncolored vertices
  unsigned long long* total_work;    // out: work of the initial worklist
  int32_t* deferred;                 // out: heavy D2/PD2 vertices (workgroup setup)
  int32_t* deferred_cnt;             // out: their number
  int32_t* deferred_grab;            // work counter of heavy_work_kernel
  unsigned long long* deferred_work; // per deferred vertex: its work, summed over slices
  int32_t* deferred_done;            // per deferred vertex: slices done
};

template <int MODE>
void launch_bin(const GraphView& g, const BinSetup& s, hipStream_t st);
void launch_scatter(int32_t n, const int32_t* C, const int8_t* bin, const BinLayout& L, int32_t* wl,
                    int32_t* cnt, int32_t* split_vertex, hipStream_t st);
void launch_validate(int32_t n_rows, int32_t n_cols, const int32_t* rp, const int32_t* ci,
                     const int32_t* rpT, const int32_t* ciT, int32_t n_trows, int square, int32_t* err,
                     hipStream_t st);
void launch_priority(int32_t n, const int32_t* gid, uint32_t hs, uint32_t* out, hipStream_t st);
// D1 ghost phase 2 (a thread per owned-row entry; loser zeroed first).
void launch_boundary(int32_t n_owned, int32_t owned_nnz, const int32_t* rp, const int32_t* ci, const int32_t* C,
                     const int32_t* ghost_colors, const KeySource& k, int32_t* loser, int32_t* gflag,
                     unsigned long long* conflicts, hipStream_t st);
// Two-hop boundary detect of the D2/PD2 ghost step (one thread per hop-1
// entry of the owned vertices; nnz1 = rp[n_owned]).  Pass 1 (set == nullptr)
// decides losers and flags and adds the conflicting walk entries to *hits;
// pass 2 (set: set_mask + 1 slots of ~0) counts distinct (v, x) pairs into
// *conflicts.  loser must be zeroed first.
template <int MODE>
void launch_boundary2(const GraphView& g, int32_t n_owned, int32_t nnz1, const int32_t* C, const int32_t* ghost_colors,
                      const KeySource& k, int32_t* loser, int32_t* gflag, unsigned long long* hits,
                      unsigned long long* set, uint64_t set_mask, unsigned long long* conflicts, hipStream_t st);
void launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long x, hipStream_t st);
void launch_boundary_uncolor(int32_t n_owned, const int32_t* loser, int32_t* C, hipStream_t st);
void launch_ghost_fill(int32_t n_owned, int32_t n_ghost, const int32_t* gc, int32_t* C, int32_t* T,
                       int32_t* maxc, hipStream_t st);
// Tentative ghost recoloring: a ghost whose color is not known yet.
constexpr int32_t kGhostUnknown = 0x7fffffff;
// One ghost layer: the local CSR over owned + ghost ids, a ghost's row being
// its owned neighbours.  cnt and fill: n_ghost + 1 zeroed words; goff:
// n_ghost + 1; rp3: n_owned + n_ghost + 1; ci3: rp[n_owned] + cut entries.
// *err = 1 if the scan failed.
void launch_ghost_rows(int32_t n_owned, int32_t n_ghost, int32_t owned_nnz, const int32_t* rp, const int32_t* ci,
                       int32_t* cnt, int32_t* goff, int32_t* fill, int32_t* rp3, int32_t* ci3, void* scan_tmp,
                       size_t scan_bytes, hipStream_t st, int* err);
// The owned-induced subgraph of a rank's local graph, in two calls: with
// ci1_or_null == nullptr, flags every owned-row entry (flag: owned_nnz + 1
// words) and scans the flags into pos (owned_nnz + 1); then, with ci1, writes
// rp1 (n_owned + 1) and the kept entries.  Returns nonzero if the scan failed.
int launch_owned_subgraph(int32_t n_owned, int32_t owned_nnz, const int32_t* rp, const int32_t* ci, int32_t* flag,
                          int32_t* pos, int32_t* rp1, int32_t* ci1_or_null, void* scan_tmp, size_t scan_bytes,
                          hipStream_t st);
// then, with ci1, copies the entries.  Returns nonzero if the scan failed.
int launch_owned_subgraph(int32_t n_owned, const int32_t* rp, const int32_t* ci, int32_t* cnt, int32_t* rp1,
                          int32_t* ci1_or_null, void* scan_tmp, size_t scan_bytes, hipStream_t st);
void launch_ghost_recolor_init(int32_t n_owned, int32_t n3, const int32_t* C, const int32_t* gc, const int32_t* gflag,
                               int32_t* init, hipStream_t st);
void launch_max_i32(int32_t n, const int32_t* a, int32_t* out, hipStream_t st);
void launch_flags_out(int32_t n, const int32_t* gflag, uint8_t* out, unsigned long long* count,
                      hipStream_t st);
void launch_copy_i32(int32_t n, const int32_t* src, int32_t* dst, hipStream_t st);

}  // namespace gcol
