// Internal declarations shared by the C-ABI translation units.
#pragma once

#include <array>
#include <mutex>
#include <vector>

#include "graphcolor.h"
#include "inc.hpp"
#include "keys.hpp"
#include "setup.hpp"

namespace gcol {

// A grow-only device buffer.  A fixed buffer is memory the library does not
// own (a region of the no-allocation entry point's static scratch array):
// it is never reallocated or freed, and asking it for more than it holds
// returns COLOR_EOVERFLOW instead of allocating.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool fixed = false;
  int ensure(size_t need, bool zero, hipStream_t st);
  void release();
  template <typename X>
  X* as() const {
    return static_cast<X*>(p);
  }
};

// Device-resident scalars of one call (one allocation, cleared per call).
struct Scalars {
  int32_t cnt[2][8];            // per-bin worklist sizes, ping-pong
  int32_t tile_ctr[2];          // dynamic unit counters of the color / detect kernels
  int32_t maxc;                 // largest committed color
  int32_t rounds_done;          // last round with a non-empty worklist
  int32_t max_split_work;       // largest work of an uncolored split vertex
  int32_t err;                  // validation error bits
  int32_t aux_max;
  int32_t pad_;
  int32_t count_all[8];
  int32_t count_unc[8];
  unsigned long long visits[8]; // [0] sum |W_r|, [1] sum work(W_r), [2] list entries, [3] color bytes,
                                // [4] detect bytes, [5] pushes, [6] + [7] tail-kernel bytes
  unsigned long long list_total; // incremental engine: entries of all lists
  int32_t max_work;              // largest work of an uncolored vertex
  int32_t deferred_cnt;          // heavy D2/PD2 vertices set up by workgroups
  int32_t deferred_grab[2];      // their work counters (work, list fill)
  uint32_t bar[kBarWords];       // tail kernel: grid-barrier words
  int32_t tail_err;              // tail kernel: error bits (a barrier gave up)
  int32_t tail_left;             // tail kernel: 1 if it stopped at the round cap with vertices left
  unsigned long long total_work;
  unsigned long long conflicts; // ghost phase-2 conflicts
  unsigned long long remote;    // ghost remote losers
  unsigned long long hits;      // D2/PD2 ghost step: conflicting two-hop walk entries
};

// Per-device workspace of the single-graph entry points.
struct Workspace {
  int device = 0;
  std::mutex mu;
  DevBuf T, C, work, bin, wl0, wl1, small, trace, split_vertex, split_ctr, split_flag, split_mask, aux0, aux1;
  DevBuf deferred, inc_len, inc_words, inc_fwoff, inc_aoff, inc_F, inc_L0, inc_Ll, inc_B0, inc_B1, inc_bm, scan_tmp;
  DevBuf inc_wl0, inc_wl1;  // incremental engine: worklists binned by active-list length
  DevBuf inc_T8, inc_done;  // incremental engine: tentative colors as bytes, committed bits
  DevBuf deferred_work, deferred_done;  // setup: per heavy D2/PD2 vertex, its work and slices done
  DevBuf rank, rk_key0, rk_key1, rk_val0, rk_val1, rk_deg0, rk_deg1, rk_tmp;  // recolorDegrees ranks
  DevBuf gr_rp, gr_ci, gr_cnt, gr_init;  // tentative ghost recoloring: local CSR with ghost rows, start colors
  DevBuf own_rp, own_ci;                 // ghost step: the owned-induced subgraph of phase 1
  DevBuf pair_set;                       // D2/PD2 ghost step: distinct conflicting (owned, ghost) pairs
  Scalars* host = nullptr;  // pinned staging for read-backs
  std::vector<hipEvent_t> events;  // pool for COLOR_FLAG_KERNEL_TIMING
  ~Workspace();
  void release();
  static constexpr int kNumBuffers = 47;
  std::array<DevBuf*, kNumBuffers> buffers();   // every DevBuf above
};

// A workspace of the current device no other call holds, returned locked
// (the lock moves into *held).
int acquire_workspace(std::unique_lock<std::mutex>* held, Workspace** out);

// State of one library call.
struct Call {
  Workspace* ws = nullptr;
  std::unique_lock<std::mutex> lock;  // holds ws for the whole call
  hipStream_t st = nullptr;
  color_params P;
  int launches = 0;
  int trace_cap = 0;
  Scalars* S = nullptr;
  Scalars* H = nullptr;
  int32_t* wl[2] = {nullptr, nullptr};
  // kernel timing (COLOR_FLAG_KERNEL_TIMING): events recorded around every
  // round kernel, resolved after the call's last synchronization
  bool timing = false;
  size_t n_events = 0;
  std::vector<int> event_kind;  // per event pair start index: 0 color, 1 detect, 2 tail, -1 none
  int color_launches = 0, detect_launches = 0;
  int tail_rounds = 0;  // rounds run by the incremental engine's tail kernel
  int tail_fallbacks = 0;  // tail launches that found their workgroups not all resident
  bool user_bins = false;  // the caller set degree-bin bounds
  int engine = 1;
  int record_event(int kind_of_next);  // records the next pool event on st
};

// run_incremental: a grid barrier of the tail kernel gave up; the call is
// repeated with per-round launches only (never returned to callers)
constexpr int kRcRetryNoTail = -1000;

void default_params(int mode, color_params* p);
int degree_rank(Call& c, int32_t m, const int32_t* deg_ptr, int32_t n_rows, const int32_t* extra_deg, KeySource& k);
void incremental_bins(int mode, int32_t bin_hi[4]);
int validate_job(const color_job& j, void* stream);
int merge_params(int mode, const color_params* user, color_params* out);
int begin_call(Call& c, int mode, const color_params* user, color_stats* stats, void* stream, int32_t n,
               int32_t n_total, Workspace* fixed_ws = nullptr);
void launch_zero_words(void* p, size_t words, hipStream_t st);
int finish_call(Call& c, color_stats* stats, int32_t num_colors_hint, int rc);

// color_d1 on a caller-provided workspace of fixed buffers (the
// no-allocation entry point): pull engine, no split vertices.
int color_d1_fixed(Workspace* ws, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
                   const uint32_t* prio, const int32_t* init_colors, int32_t* colors, color_stats* stats,
                   const color_params* params, void* stream);

int color_d2_fixed(Workspace* ws, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
                   int32_t* colors, color_stats* stats, const color_params* params, void* stream);
int color_pd2_fixed(Workspace* ws, int32_t n_rows, int32_t n_cols, const int32_t* row_ptr, const int32_t* col_idx,
                    const int32_t* col_ptr, const int32_t* row_idx, uint32_t seed, int32_t* col_colors,
                    color_stats* stats, const color_params* params, void* stream);

// Device bytes of each workspace buffer one D2/PD2 call on the incremental
// engine uses (no trace, no degree key).
struct IncPlan {
  size_t small, T, work, bin, wl0, wl1, trace, deferred, deferred_work, deferred_done;
  size_t inc_len, inc_words, inc_fwoff, inc_aoff, inc_L0, inc_Ll, inc_F, inc_B0, inc_B1, inc_bm, inc_wl0, inc_wl1,
      inc_T8, inc_done, scan_tmp;
};
// kind COLOR_KIND_D2: (rp1, ci1) = (rp2, .) = the adjacency; COLOR_KIND_PD2:
// (rp1, ci1) = the CSC, rp2 = the CSR row offsets.  HOST arrays.  Returns
// the total bytes (each buffer 256-byte aligned), 0 on error.
size_t plan_incremental(int kind, int32_t n, const int32_t* rp1, const int32_t* ci1, const int32_t* rp2,
                        IncPlan* p);
void carve_workspace(Workspace* w, char* base, const IncPlan& p);

template <int MODE>
int setup_bins(Call& c, const GraphView& g, const int32_t* init, int32_t* C, int32_t n_total, BinLayout& L,
               RoundBufs& rb, int32_t known[kBins]);
template <int MODE>
int run_incremental(Call& c, const GraphView& g, const KeySource& k, const int32_t* init, int32_t* colors,
                    BinLayout& L, int32_t known[kBins], int* fell_back, int round0 = 0);
template <int MODE>
int run_phase(Call& c, const GraphView& g, const KeySource& k, const BinLayout& L, const RoundBufs& base,
              int32_t known[kBins], int round0, int max_rounds);

}  // namespace gcol
