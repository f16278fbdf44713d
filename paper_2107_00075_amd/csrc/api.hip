// C-ABI entry points and the host round driver of libgraphcolor.
//
// Driver (Algorithm 2's "while conflicts > 0" loop, on one GPU): the static
// setup (work, bins, initial worklist) costs one host synchronization; then
// rounds are enqueued in batches of R back-to-back (color, detect) launch
// pairs with no host round trip inside a batch.  Kernels read the worklist
// sizes from device memory, so rounds enqueued after the worklist emptied
// are no-ops; the host reads the sizes once per batch and doubles R up to a
// cap, so a call with r rounds costs O(log r) synchronizations.
#include <algorithm>
#include <climits>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "api_internal.hpp"
#include "batch.hpp"

namespace gcol {

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

int DevBuf::ensure(size_t need, bool zero, hipStream_t st) {
  if (need == 0) need = 1;
  if (bytes >= need) return COLOR_OK;
  if (fixed) return COLOR_EOVERFLOW;
  if (p) {
    if (hipFree(p) != hipSuccess) return COLOR_EHIP;
    p = nullptr;
    bytes = 0;
  }
  size_t want = need + need / 4;  // headroom so slowly growing calls do not reallocate each time
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return COLOR_ENOMEM;
    }
    want = need;
  }
  bytes = want;
  if (zero && hipMemsetAsync(p, 0, want, st) != hipSuccess) return COLOR_EHIP;
  return COLOR_OK;
}

void DevBuf::release() {
  if (p && !fixed) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

Workspace::~Workspace() { release(); }

int Call::record_event(int kind_of_next) {
  std::vector<hipEvent_t>& ev = ws->events;
  if (n_events == ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return COLOR_EHIP;
    ev.push_back(e);
  }
  if (hipEventRecord(ev[n_events], st) != hipSuccess) return COLOR_EHIP;
  event_kind.push_back(kind_of_next);
  ++n_events;
  return COLOR_OK;
}

std::array<DevBuf*, Workspace::kNumBuffers> Workspace::buffers() {
  return {&T, &C, &work, &bin, &wl0, &wl1, &small, &trace, &split_vertex, &split_ctr,
          &split_flag, &split_mask, &aux0, &aux1, &deferred, &inc_len, &inc_words, &inc_fwoff, &inc_aoff,
          &inc_F, &inc_L0, &inc_Ll, &inc_B0, &inc_B1, &inc_bm, &inc_wl0, &inc_wl1, &scan_tmp,
          &deferred_work, &deferred_done, &rank, &rk_key0, &rk_key1, &rk_val0, &rk_val1, &rk_deg0,
          &rk_deg1, &rk_tmp, &gr_rp, &gr_ci, &gr_cnt, &gr_init, &own_rp, &own_ci, &pair_set, &inc_T8,
          &inc_done};
}

void Workspace::release() {
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  events.clear();
  for (DevBuf* b : buffers()) b->release();
  if (host) (void)hipHostFree(host);
  host = nullptr;
}

// Workspaces of the single-graph entry points: a pool per device.  A call
// takes a workspace no other call holds (creating one, up to
// kMaxWorkspaces per device), so calls from different host threads on
// different streams run at the same time on separate memory; beyond the cap
// a call waits for a busy workspace.  Each workspace grows to the largest
// call it served and is kept until color_release_workspace.
constexpr size_t kMaxWorkspaces = 8;

struct DevicePool {
  std::vector<Workspace*> all;
};

static std::mutex g_ws_mu;
static std::map<int, DevicePool> g_ws;

static Workspace* new_workspace(int dev, int* err) {
  Workspace* w = new Workspace();
  w->device = dev;
  if (hipHostMalloc(reinterpret_cast<void**>(&w->host), sizeof(Scalars), hipHostMallocDefault) != hipSuccess) {
    delete w;
    *err = COLOR_ENOMEM;
    return nullptr;
  }
  return w;
}

int acquire_workspace(std::unique_lock<std::mutex>* held, Workspace** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return COLOR_EHIP;
  Workspace* wait_on = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    DevicePool& pool = g_ws[dev];
    for (Workspace* w : pool.all) {
      std::unique_lock<std::mutex> l(w->mu, std::try_to_lock);
      if (l.owns_lock()) {
        *held = std::move(l);
        *out = w;
        return COLOR_OK;
      }
    }
    if (pool.all.size() < kMaxWorkspaces) {
      int err = COLOR_OK;
      Workspace* w = new_workspace(dev, &err);
      if (!w) return err;
      pool.all.push_back(w);
      *held = std::unique_lock<std::mutex>(w->mu);
      *out = w;
      return COLOR_OK;
    }
    wait_on = pool.all.front();
  }
  *held = std::unique_lock<std::mutex>(wait_on->mu);
  *out = wait_on;
  return COLOR_OK;
}

// ---------------------------------------------------------------------------
// parameters
// ---------------------------------------------------------------------------

// Degree-bin bounds (bins 0..2) for the incremental engine, on work and on
// active-list length, measured on MI355X against the pull engine's bounds:
// R-MAT scale 22 (D1) 69 -> 46 ms, the 4M x 1M power-law PD2 pattern
// 285 -> 125 ms.
void incremental_bins(int mode, int32_t bin_hi[4]) {
  if (mode == kD1) {
    bin_hi[0] = 16;
    bin_hi[1] = 96;
    bin_hi[2] = 1024;
  } else {
    bin_hi[0] = 64;
    bin_hi[1] = 256;
    bin_hi[2] = 1024;
  }
}

static bool valid_lanes(int x) {
  return x == 1 || x == 2 || x == 4 || x == 8 || x == 16 || x == 32 || x == 64;
}

void default_params(int mode, color_params* p) {
  std::memset(p, 0, sizeof(*p));
  if (mode == kD1) {
    const int32_t hi[4] = {12, 96, 2048, 65536};
    const int32_t ln[3] = {4, 16, 64};
    std::memcpy(p->bin_hi, hi, sizeof(hi));
    std::memcpy(p->lanes, ln, sizeof(ln));
    p->split_chunks = 64;
  } else if (mode == kD2) {
    const int32_t hi[4] = {64, 512, 8192, 262144};
    const int32_t ln[3] = {4, 16, 64};
    std::memcpy(p->bin_hi, hi, sizeof(hi));
    std::memcpy(p->lanes, ln, sizeof(ln));
    p->split_chunks = 64;
  } else {
    const int32_t hi[4] = {256, 2048, 32768, 524288};
    const int32_t ln[3] = {8, 32, 64};
    std::memcpy(p->bin_hi, hi, sizeof(hi));
    std::memcpy(p->lanes, ln, sizeof(ln));
    p->split_chunks = 256;
  }
  p->max_rounds = 0;
  p->rounds_per_poll = 4;
  p->tail_threshold = 0;
  p->max_workgroups = resident_round_blocks(mode);
  p->flags = 0;
  p->tail_checkin_us = kTailCheckinDefaultUs;
}

int merge_params(int mode, const color_params* user, color_params* out) {
  default_params(mode, out);
  if (!user) return COLOR_OK;
  for (int i = 0; i < 4; ++i)
    if (user->bin_hi[i] > 0) out->bin_hi[i] = user->bin_hi[i];
  for (int i = 0; i < 3; ++i) {
    if (user->lanes[i] != 0) {
      if (!valid_lanes(user->lanes[i])) return COLOR_EINVAL;
      out->lanes[i] = user->lanes[i];
    }
  }
  for (int i = 1; i < 4; ++i)
    if (out->bin_hi[i] < out->bin_hi[i - 1]) return COLOR_EINVAL;
  if (user->split_chunks < 0 || user->max_rounds < 0 || user->rounds_per_poll < 0 ||
      user->max_workgroups < 0 || user->tail_threshold < 0)
    return COLOR_EINVAL;
  if (user->split_chunks > 0) out->split_chunks = std::min(user->split_chunks, 1 << 16);
  if (user->max_rounds > 0) out->max_rounds = user->max_rounds;
  if (user->rounds_per_poll > 0) out->rounds_per_poll = std::min(user->rounds_per_poll, 1024);
  if (user->max_workgroups > 0) out->max_workgroups = user->max_workgroups;
  if (user->tail_threshold > 0) out->tail_threshold = user->tail_threshold;
  if (user->engine < 0 || user->engine > COLOR_ENGINE_INCREMENTAL) return COLOR_EINVAL;
  out->engine = user->engine;
  if (user->tail_checkin_us < -1) return COLOR_EINVAL;
  if (user->tail_checkin_us != 0) out->tail_checkin_us = user->tail_checkin_us;
  out->flags = user->flags;
  return COLOR_OK;
}

// recolorDegrees (Section 3.3; Algorithm 4 with recolorDegrees set): every
// vertex's rank in (deg, p, gid) order, built once per call in the workspace;
// k.rank then replaces the (p, gid) key in every kernel of the call.
int degree_rank(Call& c, int32_t m, const int32_t* deg_ptr, int32_t n_rows, const int32_t* extra_deg,
                KeySource& k) {
  if (m <= 0) return COLOR_OK;
  Workspace* w = c.ws;
  const size_t mm = static_cast<size_t>(m);
  const size_t tb = rank_tmp_bytes(m);
  if (tb == 0) return COLOR_EHIP;
  int e;
  if ((e = w->rank.ensure(4 * mm, false, c.st)) || (e = w->rk_key0.ensure(8 * mm, false, c.st)) ||
      (e = w->rk_key1.ensure(8 * mm, false, c.st)) || (e = w->rk_val0.ensure(4 * mm, false, c.st)) ||
      (e = w->rk_val1.ensure(4 * mm, false, c.st)) || (e = w->rk_deg0.ensure(4 * mm, false, c.st)) ||
      (e = w->rk_deg1.ensure(4 * mm, false, c.st)) || (e = w->rk_tmp.ensure(tb, false, c.st)))
    return e;
  RankBufs b{w->rk_key0.as<uint64_t>(), w->rk_key1.as<uint64_t>(), w->rk_val0.as<int32_t>(),
             w->rk_val1.as<int32_t>(), w->rk_deg0.as<uint32_t>(), w->rk_deg1.as<uint32_t>(), w->rk_tmp.p,
             w->rk_tmp.bytes};
  if (build_degree_rank(m, deg_ptr, n_rows, extra_deg, k.gid, k.prio, k.hs, b, w->rank.as<uint32_t>(), c.st))
    return COLOR_EHIP;
  c.launches += k.prio ? 5 : 3;
  k.rank = w->rank.as<uint32_t>();
  return COLOR_OK;
}

// ---------------------------------------------------------------------------
// the round loop
// ---------------------------------------------------------------------------

template <int MODE>
int run_phase(Call& c, const GraphView& g, const KeySource& k, const BinLayout& L, const RoundBufs& base,
              int32_t known[kBins], int round0, int max_rounds) {
  Scalars* S = c.S;
  Scalars* H = c.H;
  int32_t* wl[2] = {c.wl[0], c.wl[1]};
  int local = 0;
  int R = std::max(1, c.P.rounds_per_poll);
  while (true) {
    int64_t total = 0;
    for (int i = 0; i < kBins; ++i) total += known[i];
    if (total == 0) break;
    if (max_rounds > 0 && local >= max_rounds) return COLOR_ENOCONVERGE;
    const int64_t units = round_units(known, L);
    int64_t grid64 = std::min<int64_t>(units, c.P.max_workgroups);
    if (grid64 >= 8) grid64 = grid64 / 8 * 8;  // one equal share per XCD
    const int grid = static_cast<int>(std::max<int64_t>(1, grid64));
    int n_launch = R;
    if (max_rounds > 0) n_launch = std::min(n_launch, max_rounds - local);
    for (int i = 0; i < n_launch; ++i) {
      ++local;
      RoundBufs b = base;
      const int pin = (local - 1) & 1, pout = local & 1;
      b.wl_in = wl[pin];
      b.wl_out = wl[pout];
      b.cnt_in = S->cnt[pin];
      b.cnt_out = S->cnt[pout];
      if (c.timing && c.record_event(0)) return COLOR_EHIP;
      launch_color_round<MODE>(g, k, b, L, round0 + local, grid, c.st);
      if (c.timing && c.record_event(1)) return COLOR_EHIP;
      launch_detect_round<MODE>(g, k, b, L, round0 + local, grid, c.st);
      if (c.timing && c.record_event(-1)) return COLOR_EHIP;
      c.launches += 2;
      c.color_launches += 1;
      c.detect_launches += 1;
    }
    if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
    if (hipMemcpyAsync(H->cnt[local & 1], S->cnt[local & 1], sizeof(int32_t) * 8, hipMemcpyDeviceToHost,
                       c.st) != hipSuccess)
      return COLOR_EHIP;
    if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
    for (int i = 0; i < kBins; ++i) known[i] = H->cnt[local & 1][i];
    R = std::min(R * 2, 64);
  }
  return COLOR_OK;
}

template int run_phase<kD1>(Call&, const GraphView&, const KeySource&, const BinLayout&, const RoundBufs&,
                            int32_t*, int, int);
template int run_phase<kD2>(Call&, const GraphView&, const KeySource&, const BinLayout&, const RoundBufs&,
                            int32_t*, int, int);
template int run_phase<kPD2>(Call&, const GraphView&, const KeySource&, const BinLayout&, const RoundBufs&,
                             int32_t*, int, int);

// Static setup of a phase-1 worklist: work and bins, region layout, split
// scratch, initial worklist.  Leaves the initial per-bin counts in known[].
template <int MODE>
int setup_bins(Call& c, const GraphView& g, const int32_t* init, int32_t* C, int32_t n_total, BinLayout& L,
               RoundBufs& rb, int32_t known[kBins]) {
  Workspace* w = c.ws;
  Scalars* S = c.S;
  Scalars* H = c.H;
  const int32_t n = g.n;
  BinSetup s;
  for (int i = 0; i < 4; ++i) s.bin_hi[i] = c.P.bin_hi[i];
  s.init = init;
  s.C = C;
  s.T = w->T.as<int32_t>();
  s.work = w->work.as<int32_t>();
  s.bin = w->bin.as<int8_t>();
  s.count_all = S->count_all;
  s.count_unc = S->count_unc;
  s.maxc = &S->maxc;
  s.max_split_work = &S->max_split_work;
  s.max_work = &S->max_work;
  // heavy D2/PD2 vertices are set up by workgroups; D1 has none
  s.deferred = nullptr;
  s.deferred_work = nullptr;
  s.deferred_done = nullptr;
  if (MODE != kD1) {
    int e0;
    if ((e0 = w->deferred.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n, 1)), false, c.st))) return e0;
    if ((e0 = w->deferred_work.ensure(sizeof(unsigned long long) * static_cast<size_t>(std::max(n, 1)), false,
                                      c.st)))
      return e0;
    if ((e0 = w->deferred_done.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n, 1)), false, c.st)))
      return e0;
    s.deferred = w->deferred.as<int32_t>();
    s.deferred_work = w->deferred_work.as<unsigned long long>();
    s.deferred_done = w->deferred_done.as<int32_t>();
  }
  s.deferred_cnt = &S->deferred_cnt;
  s.deferred_grab = &S->deferred_grab[0];
  s.total_work = &S->total_work;
  launch_bin<MODE>(g, s, c.st);
  c.launches += 1;
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
  if (hipMemcpyAsync(H, S, sizeof(Scalars), hipMemcpyDeviceToHost, c.st) != hipSuccess) return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;

  int32_t off = 0;
  for (int i = 0; i < kBins; ++i) {
    L.off[i] = off;
    off += H->count_all[i];
  }
  for (int i = 0; i < 3; ++i) {
    L.lanes[i] = c.P.lanes[i];
    L.hi[i] = c.P.bin_hi[i];
  }
  L.split_chunks = c.P.split_chunks;
  L.grab = 4;
  const int32_t nsplit = H->count_all[kSplitBin];
  const int64_t bound = std::min<int64_t>(H->max_split_work, n_total);
  int32_t capw = static_cast<int32_t>(bound / 32 + 2);
  if (nsplit > 0) {
    int e;
    if ((e = w->split_vertex.ensure(sizeof(int32_t) * nsplit, false, c.st))) return e;
    if ((e = w->split_ctr.ensure(sizeof(uint32_t) * nsplit, true, c.st))) return e;
    if ((e = w->split_flag.ensure(sizeof(uint32_t) * nsplit, true, c.st))) return e;
    if ((e = w->split_mask.ensure(sizeof(uint32_t) * static_cast<size_t>(nsplit) * capw, true, c.st)))
      return e;
  }
  rb.C = C;
  rb.T = w->T.as<int32_t>();
  rb.work = w->work.as<int32_t>();
  rb.tile_ctr = S->tile_ctr;
  rb.split_vertex = w->split_vertex.as<int32_t>();
  rb.split_mask = w->split_mask.as<uint32_t>();
  rb.capw = capw;
  rb.split_ctr = w->split_ctr.as<uint32_t>();
  rb.split_flag = w->split_flag.as<uint32_t>();
  rb.maxc = &S->maxc;
  rb.visits = S->visits;
  rb.trace = w->trace.as<int32_t>();
  rb.trace_cap = c.trace_cap;
  rb.rounds_done = &S->rounds_done;

  launch_scatter(n, C, w->bin.as<int8_t>(), L, c.wl[0], S->cnt[0], w->split_vertex.as<int32_t>(), c.st);
  c.launches += 1;
  for (int i = 0; i < kBins; ++i) known[i] = H->count_unc[i];
  return hipGetLastError() == hipSuccess ? COLOR_OK : COLOR_EHIP;
}

template int setup_bins<kD1>(Call&, const GraphView&, const int32_t*, int32_t*, int32_t, BinLayout&,
                             RoundBufs&, int32_t*);
template int setup_bins<kD2>(Call&, const GraphView&, const int32_t*, int32_t*, int32_t, BinLayout&,
                             RoundBufs&, int32_t*);
template int setup_bins<kPD2>(Call&, const GraphView&, const int32_t*, int32_t*, int32_t, BinLayout&,
                              RoundBufs&, int32_t*);

// Clears `words` 32-bit words with a fill kernel (not hipMemsetAsync, so that
// the clear is an ordinary kernel node wherever a caller records the stream).
__global__ void zero_words_kernel(uint32_t* p, size_t words) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

void launch_zero_words(void* p, size_t words, hipStream_t st) {
  if (words == 0) return;
  hipLaunchKernelGGL(zero_words_kernel, dim3(static_cast<unsigned>((words + 255) / 256)), dim3(256), 0, st,
                     static_cast<uint32_t*>(p), words);
}

int begin_call(Call& c, int mode, const color_params* user, color_stats* stats, void* stream, int32_t n,
               int32_t n_total, Workspace* fixed_ws) {
  int e = merge_params(mode, user, &c.P);
  if (e) return e;
  c.user_bins = false;
  if (user)
    for (int i = 0; i < 3; ++i) c.user_bins = c.user_bins || user->bin_hi[i] > 0;
  // Every round commits at least the worklist vertex of highest key, so no
  // run needs more than n rounds; the default cap turns a defect into
  // COLOR_ENOCONVERGE instead of an endless loop.
  if (c.P.max_rounds == 0) c.P.max_rounds = n_total < INT_MAX ? n_total + 1 : INT_MAX;
  c.st = static_cast<hipStream_t>(stream);
  if (fixed_ws) {
    c.lock = std::unique_lock<std::mutex>(fixed_ws->mu);
    c.ws = fixed_ws;
  } else if ((e = acquire_workspace(&c.lock, &c.ws))) {
    return e;
  }
  c.trace_cap = (stats && stats->worklist_trace && stats->trace_cap > 0) ? stats->trace_cap : 0;
  c.timing = (c.P.flags & COLOR_FLAG_KERNEL_TIMING) != 0 && stats != nullptr;
  Workspace* w = c.ws;
  if ((e = w->small.ensure(sizeof(Scalars), false, c.st))) return e;
  if ((e = w->T.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n_total, 1)), false, c.st))) return e;
  if ((e = w->work.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n, 1)), false, c.st))) return e;
  if ((e = w->bin.ensure(static_cast<size_t>(std::max(n, 1)), false, c.st))) return e;
  if ((e = w->wl0.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n, 1)), false, c.st))) return e;
  if ((e = w->wl1.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n, 1)), false, c.st))) return e;
  if ((e = w->trace.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(c.trace_cap, 1)), false, c.st)))
    return e;
  c.S = w->small.as<Scalars>();
  c.H = w->host;
  c.wl[0] = w->wl0.as<int32_t>();
  c.wl[1] = w->wl1.as<int32_t>();
  static_assert(sizeof(Scalars) % 4 == 0, "Scalars is cleared in 32-bit words");
  launch_zero_words(c.S, sizeof(Scalars) / 4, c.st);
  c.launches += 1;
  return hipGetLastError() == hipSuccess ? COLOR_OK : COLOR_EHIP;
}

int finish_call(Call& c, color_stats* stats, int32_t num_colors_hint, int rc) {
  if (hipMemcpyAsync(c.H, c.S, sizeof(Scalars), hipMemcpyDeviceToHost, c.st) != hipSuccess) return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  if (stats) {
    stats->num_colors = num_colors_hint >= 0 ? num_colors_hint : c.H->maxc;
    stats->rounds = c.H->rounds_done;
    stats->vertex_visits = static_cast<int64_t>(c.H->visits[0]);
    stats->edge_visits = static_cast<int64_t>(c.H->visits[1]);
    stats->boundary_conflicts = static_cast<int64_t>(c.H->conflicts);
    stats->remote_losers = static_cast<int64_t>(c.H->remote);
    stats->kernel_launches = c.launches;
    stats->color_kernel_ns = 0;
    stats->detect_kernel_ns = 0;
    stats->color_launches = c.color_launches;
    stats->detect_launches = c.detect_launches;
    stats->engine = c.engine;
    stats->tail_rounds = c.tail_rounds;
    stats->tail_kernel_ns = 0;
    stats->tail_bytes = static_cast<int64_t>(c.H->visits[6] + c.H->visits[7]);
    stats->tail_fallbacks = c.tail_fallbacks;
    stats->list_visits = static_cast<int64_t>(c.H->visits[2]);
    stats->color_bytes = static_cast<int64_t>(c.H->visits[3]);
    stats->detect_bytes = static_cast<int64_t>(c.H->visits[4]);
    stats->pushes = static_cast<int64_t>(c.H->visits[5]);
    if (c.timing) {
      // event i opens a kernel of kind event_kind[i] that event i+1 closes
      for (size_t i = 0; i + 1 < c.n_events; ++i) {
        const int kind = c.event_kind[i];
        if (kind < 0) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c.ws->events[i], c.ws->events[i + 1]) != hipSuccess) return COLOR_EHIP;
        const int64_t ns = static_cast<int64_t>(static_cast<double>(ms) * 1e6);
        if (kind == 0) stats->color_kernel_ns += ns;
        else if (kind == 1) stats->detect_kernel_ns += ns;
        else stats->tail_kernel_ns += ns;
      }
    }
    if (c.trace_cap > 0) {
      // through a stack buffer: the no-allocation entry point shares this path
      const int nr = std::min(c.trace_cap, c.H->rounds_done);
      int32_t tmp[256];
      for (int i0 = 0; i0 < nr; i0 += 256) {
        const int k = std::min(256, nr - i0);
        if (hipMemcpy(tmp, c.ws->trace.as<int32_t>() + i0, sizeof(int32_t) * k, hipMemcpyDeviceToHost) !=
            hipSuccess)
          return COLOR_EHIP;
        for (int i = 0; i < k; ++i) stats->worklist_trace[i0 + i] = tmp[i];
      }
    }
  }
  return rc;
}

static int check_rowptr_graph(Call& c, int32_t n_rows, int32_t n_cols, const int32_t* rp, const int32_t* ci,
                              const int32_t* rpT, const int32_t* ciT, int square) {
  launch_validate(n_rows, n_cols, rp, ci, rpT, ciT, n_cols, square, &c.S->err, c.st);
  c.launches += 2;
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
  if (hipMemcpyAsync(&c.H->err, &c.S->err, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) != hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  return c.H->err ? COLOR_EGRAPH : COLOR_OK;
}

// nnz = row_ptr[n] read from the device (sizes the validation and stats).
static int read_nnz(Call& c, const int32_t* rp, int32_t n, int32_t* nnz) {
  if (hipMemcpyAsync(&c.H->err, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) != hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  *nnz = c.H->err;
  c.H->err = 0;
  return COLOR_OK;
}

// ---------------------------------------------------------------------------
// incremental engine driver
// ---------------------------------------------------------------------------
template <int MODE>
int run_incremental(Call& c, const GraphView& g, const KeySource& k, const int32_t* init, int32_t* colors,
                    BinLayout& L, int32_t known[kBins], int* fell_back, int round0) {
  Workspace* w = c.ws;
  Scalars* S = c.S;
  Scalars* H = c.H;
  const int32_t n = g.n;
  int e;
  *fell_back = 0;
  const size_t n1 = static_cast<size_t>(n) + 1;
  if ((e = w->inc_len.ensure(sizeof(int32_t) * n1, false, c.st))) return e;
  if ((e = w->inc_words.ensure(sizeof(int32_t) * n1, false, c.st))) return e;
  if ((e = w->inc_fwoff.ensure(sizeof(int32_t) * n1, false, c.st))) return e;
  if ((e = w->inc_L0.ensure(sizeof(int32_t) * n1, false, c.st))) return e;
  int32_t* len = w->inc_len.as<int32_t>();
  int32_t* words = w->inc_words.as<int32_t>();
  if (hipMemsetAsync(len + n, 0, sizeof(int32_t), c.st) != hipSuccess) return COLOR_EHIP;
  if (hipMemsetAsync(words + n, 0, sizeof(int32_t), c.st) != hipSuccess) return COLOR_EHIP;
  launch_inc_sizes<MODE>(g, w->work.as<int32_t>(), len, words, w->inc_L0.as<int32_t>(), &S->list_total, c.st);
  c.launches += 1;
  if (hipMemcpyAsync(&H->list_total, &S->list_total, sizeof(unsigned long long), hipMemcpyDeviceToHost, c.st) !=
      hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  const unsigned long long total_list = H->list_total;
  if (total_list >= static_cast<unsigned long long>(INT_MAX)) {
    *fell_back = 1;
    return COLOR_OK;
  }
  size_t tmp_bytes = 0;
  if (exclusive_scan_i32(words, w->inc_fwoff.as<int32_t>(), n + 1, nullptr, &tmp_bytes, c.st)) return COLOR_EHIP;
  if ((e = w->scan_tmp.ensure(tmp_bytes, false, c.st))) return e;
  if (exclusive_scan_i32(words, w->inc_fwoff.as<int32_t>(), n + 1, w->scan_tmp.p, &tmp_bytes, c.st))
    return COLOR_EHIP;
  const int32_t* aoff = g.rp;
  if (MODE != kD1) {
    if ((e = w->inc_aoff.ensure(sizeof(int32_t) * n1, false, c.st))) return e;
    size_t tb2 = 0;
    if (exclusive_scan_i32(len, w->inc_aoff.as<int32_t>(), n + 1, nullptr, &tb2, c.st)) return COLOR_EHIP;
    if (tb2 > tmp_bytes && (e = w->scan_tmp.ensure(tb2, false, c.st))) return e;
    tb2 = std::max(tb2, tmp_bytes);
    if (exclusive_scan_i32(len, w->inc_aoff.as<int32_t>(), n + 1, w->scan_tmp.p, &tb2, c.st)) return COLOR_EHIP;
    aoff = w->inc_aoff.as<int32_t>();
  }
  int32_t fw_total = 0;
  if (hipMemcpyAsync(&fw_total, w->inc_fwoff.as<int32_t>() + n, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) !=
      hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  const size_t list_entries = std::max<size_t>(1, total_list);
  // word 0 of every vertex's bitset, then the further words
  const size_t f_words = static_cast<size_t>(n) + static_cast<size_t>(fw_total);
  if ((e = w->inc_F.ensure(sizeof(uint32_t) * f_words, false, c.st))) return e;
  if ((e = w->inc_B0.ensure(sizeof(int32_t) * list_entries, false, c.st))) return e;
  if (hipMemsetAsync(w->inc_F.p, 0, sizeof(uint32_t) * f_words, c.st) != hipSuccess)
    return COLOR_EHIP;
  // Round 1 reads the unsplit lists (D1: the adjacency itself; D2/PD2: the
  // materialized two-hop lists) and its losers write their lists, split by
  // key, into the list array B; later rounds compact B in place (the lists
  // of a round are read and rewritten only by their own vertex's workgroup).
  int32_t* B = w->inc_B0.as<int32_t>();
  int32_t* Lb = w->inc_L0.as<int32_t>();
  if ((e = w->inc_Ll.ensure(sizeof(int32_t) * n1, false, c.st))) return e;
  const int32_t* A0 = g.ci;
  if (MODE != kD1) {
    if ((e = w->inc_B1.ensure(sizeof(int32_t) * list_entries, false, c.st))) return e;
    // heavy (deferred) vertices: their sets through one bitmap each when the
    // bitmaps of all of them together stay small, else a workgroup per list
    // and the duplicate removal below
    const int32_t words = n / 32 + 1;
    const int32_t nd = H->deferred_cnt;  // from the setup's read-back
    const bool sets = nd > 0 && static_cast<int64_t>(nd) * words <= kSetsMaxWords;
    const int32_t nb_max = sets ? static_cast<int32_t>(std::max<int64_t>(
                                      1, std::min<int64_t>(nd, kSetsBatchWords / words)))
                                : 0;
    launch_inc_fill<MODE>(g, aoff, len, B, Lb, w->deferred.as<int32_t>(), &S->deferred_cnt, &S->deferred_grab[1],
                          !sets, c.st);
    c.launches += sets ? 2 : 3;
    A0 = B;
    const int grid = dedup_grid(words);
    const size_t bm_bytes = sizeof(uint32_t) * static_cast<size_t>(words) * static_cast<size_t>(grid);
    const size_t sets_bytes = sizeof(uint32_t) * static_cast<size_t>(words) * static_cast<size_t>(nb_max);
    if ((e = w->inc_bm.ensure(std::max(bm_bytes, sets_bytes), false, c.st))) return e;
    for (int32_t i0 = 0; sets && i0 < nd; i0 += nb_max) {
      const int32_t nb = std::min(nb_max, nd - i0);
      if (hipMemsetAsync(w->inc_bm.p, 0, sizeof(uint32_t) * static_cast<size_t>(words) * nb, c.st) != hipSuccess)
        return COLOR_EHIP;
      launch_inc_bitmap_sets<MODE>(g, w->deferred.as<int32_t>(), i0, nb, w->inc_bm.as<uint32_t>(), words, aoff, Lb,
                                   B, c.st);
      c.launches += 2;
    }
    if (hipMemsetAsync(w->inc_bm.p, 0, bm_bytes, c.st) != hipSuccess) return COLOR_EHIP;
    launch_inc_dedup(n, aoff, Lb, B, w->inc_bm.as<uint32_t>(), words, grid, sets ? g.rp : nullptr, c.st);
    c.launches += 1;
    B = w->inc_B1.as<int32_t>();  // the split lists
  }
  IncBufs ib;
  ib.C = colors;
  ib.T = w->T.as<int32_t>();
  ib.work = w->work.as<int32_t>();
  ib.tile_ctr = S->tile_ctr;
  ib.aoff = aoff;
  ib.fw_off = w->inc_fwoff.as<int32_t>();
  ib.F = w->inc_F.as<uint32_t>();
  ib.Fx = ib.F + n;
  ib.maxc = &S->maxc;
  ib.acc = S->visits;
  ib.trace = w->trace.as<int32_t>();
  ib.trace_cap = c.trace_cap;
  ib.rounds_done = &S->rounds_done;
  ib.llen = w->inc_Ll.as<int32_t>();
  ib.uniform = 0;
  ib.defer_split = 0;
  ib.round_base = round0;
  // tentative colors as bytes while they fit one: a color taken in round r
  // is at most (largest initial color) + r (first fit over colors committed
  // before the round, whose largest grows by at most one per round)
  if ((e = w->inc_T8.ensure((static_cast<size_t>(n) + 3) / 4 * 4, false, c.st))) return e;
  if ((e = w->inc_done.ensure(sizeof(uint32_t) * (static_cast<size_t>(n) / 32 + 1), false, c.st))) return e;
  ib.T8 = w->inc_T8.as<uint8_t>();
  ib.done = w->inc_done.as<uint32_t>();
  ib.t8_last = std::max(0, 255 - H->maxc);
  launch_inc_state_init(n, colors, ib.T8, ib.done, c.st);
  c.launches += 1;

  if (init) {
    if constexpr (MODE != kD1) {
      if (g.ids > g.limit) {
        // walks reach members outside the lists (a rank's ghosts, fixed
        // colors): every uncolored vertex takes all its members' colors
        int32_t nnz1 = 0;
        if ((e = read_nnz(c, g.rp, n, &nnz1))) return e;
        launch_inc_init_pull<MODE>(g, nnz1, ib, c.st);
        c.launches += 1;
      }
    }
    if (g.ids <= g.limit || MODE == kD1) {
      IncBufs pb = ib;
      pb.alen_in = Lb;
      launch_inc_init_push(pb, n, A0, c.st);
      c.launches += 1;
    }
  }
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
  // Worklists binned by active-list length: a loser goes to the bin of its
  // current list, never above the bin of its static work, so bin b's region
  // holds every vertex whose static bin is b or above.  The round-1
  // worklist moves over from the static layout.
  BinLayout IL = L;
  int64_t wl_total = 0;
  {
    int64_t above = 0, cap[kBins];
    cap[kSplitBin] = known[kSplitBin];  // none: this engine bins without split units
    for (int i = kBlockBin; i >= 0; --i) {
      above += known[i];
      cap[i] = above;
    }
    for (int i = 0; i < kBins; ++i) {
      IL.off[i] = static_cast<int32_t>(std::min<int64_t>(wl_total, INT_MAX));
      wl_total += cap[i];
    }
  }
  if (wl_total >= INT_MAX) return COLOR_EOVERFLOW;
  if ((e = w->inc_wl0.ensure(sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(wl_total, 1)), false, c.st)))
    return e;
  if ((e = w->inc_wl1.ensure(sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(wl_total, 1)), false, c.st)))
    return e;
  int32_t* wl[2] = {w->inc_wl0.as<int32_t>(), w->inc_wl1.as<int32_t>()};
  for (int i = 0; i < kBins; ++i) {
    if (known[i] > 0 && hipMemcpyAsync(wl[0] + IL.off[i], c.wl[0] + L.off[i], sizeof(int32_t) * known[i],
                                       hipMemcpyDeviceToDevice, c.st) != hipSuccess)
      return COLOR_EHIP;
  }
  const int resident = std::min(resident_inc_blocks(), std::max(8, c.P.max_workgroups));
  const int max_rounds = c.P.max_rounds;
  // the buffers of round r: worklists and counts ping-pong; round 1 reads the
  // unsplit lists (and, without initial colors, takes the uniform shortcut)
  auto round_bufs = [&](int r) {
    IncBufs b = ib;
    const int pin = (r - 1) & 1, pout = r & 1;
    b.wl_in = wl[pin];
    b.wl_out = wl[pout];
    b.cnt_in = S->cnt[pin];
    b.cnt_out = S->cnt[pout];
    // without initial colors round 1's losers leave the lists unsplit (the
    // read-only adjacency or two-hop lists); round 2 reads those and writes
    // the first compacted, key-split lists, which later rounds compact in place
    b.A_in = (r == 1 || (r == 2 && !init)) ? A0 : B;
    b.A_out = B;
    b.uniform = (r == 1 && !init) ? 1 : 0;
    b.defer_split = (r == 1 && !init) ? 1 : 0;
    b.alen_in = Lb;
    b.alen_out = Lb;
    return b;
  };
  bool tail_on = !(c.P.flags & COLOR_FLAG_NO_TAIL) && tail_blocks_resident() > 0;
  const int64_t tail_at = c.P.tail_threshold > 0 ? c.P.tail_threshold : kTailDefault;
  int local = 0;
  int R = std::max(1, c.P.rounds_per_poll);
  int64_t prev_total = 0;
  int prev_local = 0;
  while (true) {
    int64_t total = 0;
    for (int i = 0; i < kBins; ++i) total += known[i];
    if (total == 0) break;
    if (max_rounds > 0 && local >= max_rounds) return COLOR_ENOCONVERGE;
    if (tail_on && total <= tail_at) {
      // the remaining rounds in one cooperative launch: no launch gaps and no
      // host polls between the (small) rounds of the tail
      int64_t g = std::max<int64_t>((total + kBlock - 1) / kBlock, inc_round_units(known, IL));
      g = std::min<int64_t>(g, std::min(tail_blocks_resident(), std::max(8, c.P.max_workgroups)));
      if (g >= 8) g = g / 8 * 8;
      IncRoundSet set;
      set.base = round_bufs(3);
      set.base.bytes_slot = 6;
      set.wl0 = wl[0];
      set.wl1 = wl[1];
      set.cnt0 = S->cnt[0];
      set.cnt1 = S->cnt[1];
      set.A0 = A0;
      set.uniform1 = init ? 0 : 1;
      set.defer1 = init ? 0 : 1;
      static_assert(offsetof(Scalars, tail_left) == offsetof(Scalars, bar) + sizeof(Scalars::bar) + sizeof(int32_t),
                    "barrier words and tail flags are cleared together");
      if (hipMemsetAsync(S->bar, 0, sizeof(S->bar) + 2 * sizeof(int32_t), c.st) != hipSuccess) return COLOR_EHIP;
      const int cap = max_rounds > 0 ? max_rounds : INT_MAX;
      if (c.timing && c.record_event(2)) return COLOR_EHIP;
      if (launch_inc_tail(k, set, IL, local + 1, cap, S->bar, &S->tail_err, &S->tail_left,
                          static_cast<int>(std::max<int64_t>(1, g)), c.P.tail_checkin_us, c.st)) {
        if (c.timing && c.record_event(-1)) return COLOR_EHIP;
        c.launches += 1;
        if (hipMemcpyAsync(&H->tail_err, &S->tail_err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c.st) !=
                hipSuccess ||
            hipMemcpyAsync(&H->rounds_done, &S->rounds_done, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) !=
                hipSuccess)
          return COLOR_EHIP;
        if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
        if (H->tail_err == kErrTailCheckin) {
          // its workgroups were not all resident: it ran nothing, so the
          // rounds go on from the same state as per-round launches
          c.tail_fallbacks += 1;
          tail_on = false;
          continue;
        }
        if (H->tail_err) return kRcRetryNoTail;  // a grid barrier gave up: the outputs are not valid
        c.tail_rounds = std::max(0, H->rounds_done - round0 - local);
        return H->tail_left ? COLOR_ENOCONVERGE : COLOR_OK;
      }
      // cooperative launch refused: per-round launches from here on
      (void)hipGetLastError();
      if (c.timing) c.event_kind.back() = -1;
      tail_on = false;
    }
    int64_t gc = std::min<int64_t>((total + kBlock - 1) / kBlock, resident);
    if (gc >= 8) gc = gc / 8 * 8;
    int64_t gd = std::min<int64_t>(inc_round_units(known, IL), resident);
    if (gd >= 8) gd = gd / 8 * 8;
    const int grid_c = static_cast<int>(std::max<int64_t>(1, gc));
    const int grid_d = static_cast<int>(std::max<int64_t>(1, gd));
    int n_launch = R;
    if (tail_on && local > prev_local && total < prev_total) {
      // poll again about when the worklist should reach the tail threshold,
      // from its geometric shrink rate over the last batch of rounds
      const double f = std::pow(static_cast<double>(total) / static_cast<double>(prev_total),
                                1.0 / static_cast<double>(local - prev_local));
      const double k = std::ceil(std::log(static_cast<double>(tail_at) / static_cast<double>(total)) / std::log(f));
      if (k >= 1.0 && k < static_cast<double>(n_launch)) n_launch = static_cast<int>(k);
    }
    prev_total = total;
    prev_local = local;
    if (max_rounds > 0) n_launch = std::min(n_launch, max_rounds - local);
    for (int i = 0; i < n_launch; ++i) {
      ++local;
      const IncBufs b = round_bufs(local);
      if (c.timing && c.record_event(0)) return COLOR_EHIP;
      launch_inc_color(b, IL, local, grid_c, c.st);
      if (c.timing && c.record_event(1)) return COLOR_EHIP;
      launch_inc_detect(k, b, IL, local, grid_d, c.st);
      if (c.timing && c.record_event(-1)) return COLOR_EHIP;
      c.launches += 2;
      c.color_launches += 1;
      c.detect_launches += 1;
    }
    if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
    if (hipMemcpyAsync(H->cnt[local & 1], S->cnt[local & 1], sizeof(int32_t) * 8, hipMemcpyDeviceToHost, c.st) !=
        hipSuccess)
      return COLOR_EHIP;
    if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
    for (int i = 0; i < kBins; ++i) known[i] = H->cnt[local & 1][i];
    // a round cap inside the tail threshold is reached by the tail kernel
    R = std::min(R * 2, 64);
  }
  return COLOR_OK;
}

template int run_incremental<kD1>(Call&, const GraphView&, const KeySource&, const int32_t*, int32_t*,
                                  BinLayout&, int32_t*, int*, int);
template int run_incremental<kD2>(Call&, const GraphView&, const KeySource&, const int32_t*, int32_t*,
                                  BinLayout&, int32_t*, int*, int);
template int run_incremental<kPD2>(Call&, const GraphView&, const KeySource&, const int32_t*, int32_t*,
                                   BinLayout&, int32_t*, int*, int);

// The input contract (COLOR_FLAG_VALIDATE), checked on the device: row
// offsets, ranges, self-loops, duplicates and symmetry (D1/D2), or that the
// CSC is the transpose of the CSR (PD2).  hop 1 = (rp, ci), hop 2 = (rp2, ci2).
template <int MODE>
static int validate_graph(Call& c, int32_t n, int32_t n_rows, const int32_t* rp, const int32_t* ci,
                          const int32_t* rp2, const int32_t* ci2) {
  int e;
  int32_t nnz = 0;
  if ((e = read_nnz(c, rp, n, &nnz))) return e;
  if (nnz < 0) return COLOR_EGRAPH;
  if (MODE == kPD2) {
    int32_t nnz2 = 0;
    if ((e = read_nnz(c, rp2, n_rows, &nnz2))) return e;
    if (nnz2 != nnz) return COLOR_EGRAPH;
    // CSC (column -> rows) against CSR (row -> columns), both directions
    if ((e = check_rowptr_graph(c, n, n_rows, rp, ci, rp2, ci2, 0))) return e;
    if ((e = check_rowptr_graph(c, n_rows, n, rp2, ci2, rp, ci, 0))) return e;
  } else {
    if ((e = check_rowptr_graph(c, n, n, rp, ci, rp, ci, 1))) return e;
  }
  return COLOR_OK;
}

int validate_job(const color_job& j, void* stream) {
  if (j.n == 0) return COLOR_OK;
  Call c;
  int e = begin_call(c, j.kind, nullptr, nullptr, stream, 1, 1);
  if (e) return e;
  if (j.kind == COLOR_KIND_D1) return validate_graph<kD1>(c, j.n, j.n, j.row_ptr, j.col_idx, j.row_ptr, j.col_idx);
  if (j.kind == COLOR_KIND_D2) return validate_graph<kD2>(c, j.n, j.n, j.row_ptr, j.col_idx, j.row_ptr, j.col_idx);
  return validate_graph<kPD2>(c, j.n, j.n_rows, j.col_ptr, j.row_idx, j.row_ptr, j.col_idx);
}

// Colors the uncolored vertices of g (colors[] is set up from init) on the
// engine the parameters name, or the library's choice.  n_total: the ids
// colors[] and the tentative colors cover.
template <int MODE>
static int run_engine(Call& c, const GraphView& g, const KeySource& k, const int32_t* init, int32_t* colors,
                      int32_t n_total, int round0 = 0) {
  const int32_t n = g.n;
  BinLayout L;
  RoundBufs rb;
  int32_t known[kBins];
  int e;
  if (c.P.engine != COLOR_ENGINE_PULL) {
    // bins without split units (the incremental engine has none; the pull
    // engine only runs on them here for graphs without heavy vertices), and
    // unless the caller set them, the incremental engine's own bounds: its
    // active lists shrink round by round, and a vertex whose list is longer
    // than one pass of a wavefront is faster on a whole workgroup
    color_params saved = c.P;
    c.P.bin_hi[3] = INT_MAX;
    if (!c.user_bins) incremental_bins(MODE, c.P.bin_hi);
    e = setup_bins<MODE>(c, g, init, colors, n_total, L, rb, known);
    c.P = saved;
    if (e) return e;
    int64_t left = 0;
    for (int i = 0; i < kBins; ++i) left += known[i];
    // library choice: the incremental engine pays off when the work is
    // concentrated in a few vertices that would be rescanned every round, or
    // when two-hop walks are long (dense D2/PD2: every revisit of a vertex
    // would re-walk thousands of entries; measured 2-12x faster)
    const double avg = static_cast<double>(c.H->total_work) / std::max<int64_t>(1, n);
    const bool skewed = c.H->max_work > 64 && c.H->max_work > 16.0 * std::max(1.0, avg);
    const bool long_walks = MODE != kD1 && avg >= 128.0;
    if (left > 0 && (c.P.engine == COLOR_ENGINE_INCREMENTAL || skewed || long_walks)) {
      int fell_back = 0;
      const int rc = run_incremental<MODE>(c, g, k, init, colors, L, known, &fell_back, round0);
      if (!fell_back) {
        c.engine = COLOR_ENGINE_INCREMENTAL;
        return rc;
      }
      // lists too large for int32 offsets: pull on the same worklists
    }
  } else {
    if ((e = setup_bins<MODE>(c, g, init, colors, n_total, L, rb, known))) return e;
  }
  c.engine = COLOR_ENGINE_PULL;
  return run_phase<MODE>(c, g, k, L, rb, known, round0, c.P.max_rounds);
}

// fixed_ws: a workspace of fixed buffers (the no-allocation entry point's
// static scratch array, the server's heavy-lane regions of its arena): the
// call allocates nothing, and a buffer asked for more than it holds fails
// the call with COLOR_EOVERFLOW.
template <int MODE>
static int color_graph_once(int32_t n, int32_t n_rows, const int32_t* rp, const int32_t* ci, const int32_t* rp2,
                       const int32_t* ci2, uint32_t seed, const uint32_t* prio, const int32_t* init,
                       int32_t* colors, color_stats* stats, const color_params* params, void* stream,
                       Workspace* fixed_ws = nullptr) {
  if (n < 0 || n_rows < 0) return COLOR_EINVAL;
  if (n > 0 && (!rp || !ci || !colors)) return COLOR_EINVAL;
  if (MODE == kPD2 && n > 0 && (!rp2 || !ci2)) return COLOR_EINVAL;
  if (n == INT_MAX || n_rows == INT_MAX) return COLOR_EOVERFLOW;
  Call c;
  int e = begin_call(c, MODE, params, stats, stream, n, n, fixed_ws);
  if (e) return e;
  if (n == 0) return finish_call(c, stats, 0, COLOR_OK);
  if (c.P.flags & COLOR_FLAG_VALIDATE) {
    if ((e = validate_graph<MODE>(c, n, n_rows, rp, ci, rp2, ci2))) return e;
  }
  GraphView g{n, n, rp, ci, MODE == kD1 ? rp : rp2, MODE == kD1 ? ci : ci2};
  if (MODE == kD2) {
    g.rp2 = rp;
    g.ci2 = ci;
  }
  KeySource k{prio, nullptr, hash_seed(seed), nullptr};
  // recolorDegrees: deg(v) is v's hop-1 row (D1/D2: adjacency; PD2: the
  // column's rows)
  if (c.P.flags & COLOR_FLAG_RECOLOR_DEGREES) {
    if ((e = degree_rank(c, n, g.rp, n, nullptr, k))) return e;
  }
  const int rc = run_engine<MODE>(c, g, k, init, colors, n);
  if (rc != COLOR_OK && rc != COLOR_ENOCONVERGE) return rc;
  return finish_call(c, stats, -1, rc);
}

// A call whose tail kernel's grid barrier gave up starts over with
// per-round launches only: the setup re-initializes every array, so the
// repeated call computes the same coloring.
template <int MODE>
static int color_graph(int32_t n, int32_t n_rows, const int32_t* rp, const int32_t* ci, const int32_t* rp2,
                       const int32_t* ci2, uint32_t seed, const uint32_t* prio, const int32_t* init,
                       int32_t* colors, color_stats* stats, const color_params* params, void* stream,
                       Workspace* fixed_ws = nullptr) {
  const int rc = color_graph_once<MODE>(n, n_rows, rp, ci, rp2, ci2, seed, prio, init, colors, stats, params,
                                        stream, fixed_ws);
  if (rc != kRcRetryNoTail) return rc;
  color_params p;
  if (params) p = *params;
  else std::memset(&p, 0, sizeof(p));
  p.flags |= COLOR_FLAG_NO_TAIL;
  return color_graph_once<MODE>(n, n_rows, rp, ci, rp2, ci2, seed, prio, init, colors, stats, &p, stream,
                                fixed_ws);
}

int color_d1_fixed(Workspace* ws, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
                   const uint32_t* prio, const int32_t* init_colors, int32_t* colors, color_stats* stats,
                   const color_params* params, void* stream) {
  return color_graph<kD1>(n, n, row_ptr, col_idx, row_ptr, col_idx, seed, prio, init_colors, colors, stats, params,
                          stream, ws);
}

int color_d2_fixed(Workspace* ws, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
                   int32_t* colors, color_stats* stats, const color_params* params, void* stream) {
  return color_graph<kD2>(n, n, row_ptr, col_idx, row_ptr, col_idx, seed, nullptr, nullptr, colors, stats, params,
                          stream, ws);
}

int color_pd2_fixed(Workspace* ws, int32_t n_rows, int32_t n_cols, const int32_t* row_ptr, const int32_t* col_idx,
                    const int32_t* col_ptr, const int32_t* row_idx, uint32_t seed, int32_t* col_colors,
                    color_stats* stats, const color_params* params, void* stream) {
  if (n_cols > 0 && n_rows > 0 && (!row_ptr || !col_idx)) return COLOR_EINVAL;
  return color_graph<kPD2>(n_cols, n_rows, col_ptr, row_idx, row_ptr, col_idx, seed, nullptr, nullptr, col_colors,
                           stats, params, stream, ws);
}

// Buffer sizes of one D2/PD2 call on the incremental engine, computed on the
// host from the graph the way the engine sizes them on the device (list
// lengths from the hop-1 and hop-2 rows, bitset words, worklists, list-
// building bitmaps, scan storage), with no trace and no degree key.
size_t plan_incremental(int kind, int32_t n, const int32_t* rp1, const int32_t* ci1, const int32_t* rp2,
                        IncPlan* p) {
  std::memset(p, 0, sizeof(*p));
  const size_t nn = static_cast<size_t>(std::max(n, 1));
  const size_t n1 = static_cast<size_t>(n) + 1;
  int64_t total = 0, fw = 0, nd = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t d1 = rp1[v + 1] - rp1[v];
    int64_t work = 0;
    for (int32_t q = rp1[v]; q < rp1[v + 1]; ++q) work += 1 + (rp2[ci1[q] + 1] - rp2[ci1[q]]);
    const int64_t len = std::max<int64_t>(0, work - (kind == COLOR_KIND_PD2 ? 2 : 1) * d1);
    total += len;
    fw += std::min<int64_t>(len, n) / 32 + 1;
    if (d1 > kSetupHeavy) ++nd;
  }
  const size_t entries = static_cast<size_t>(std::max<int64_t>(1, std::min<int64_t>(total, INT_MAX)));
  const size_t words = static_cast<size_t>(n) / 32 + 1;
  const size_t bm = sizeof(uint32_t) * words * static_cast<size_t>(dedup_grid(static_cast<int32_t>(words)));
  size_t sets = 0;
  if (nd > 0 && nd * static_cast<int64_t>(words) <= kSetsMaxWords)
    sets = sizeof(uint32_t) * words *
           static_cast<size_t>(std::max<int64_t>(1, std::min<int64_t>(nd, kSetsBatchWords / static_cast<int64_t>(words))));
  size_t scan = 0;
  if (exclusive_scan_i32(nullptr, nullptr, n + 1, nullptr, &scan, nullptr)) return 0;
  p->small = sizeof(Scalars);
  p->T = p->work = p->wl0 = p->wl1 = p->deferred = p->deferred_done = 4 * nn;
  p->bin = nn;
  p->trace = 4;
  p->deferred_work = 8 * nn;
  p->inc_len = p->inc_words = p->inc_fwoff = p->inc_aoff = p->inc_L0 = p->inc_Ll = 4 * n1;
  p->inc_F = 4 * static_cast<size_t>(std::max<int64_t>(fw, 1));
  p->inc_B0 = p->inc_B1 = 4 * entries;
  p->inc_bm = std::max(bm, sets);
  p->inc_wl0 = p->inc_wl1 = 4 * 4 * nn;  // bin regions: at most 4n entries
  p->inc_T8 = (nn + 3) / 4 * 4;  // as run_incremental sizes it
  p->inc_done = 4 * (nn / 32 + 1);
  p->scan_tmp = std::max<size_t>(scan, 1);
  size_t t = 0;
  for (size_t b : {p->small, p->T, p->work, p->bin, p->wl0, p->wl1, p->trace, p->deferred, p->deferred_work,
                   p->deferred_done, p->inc_len, p->inc_words, p->inc_fwoff, p->inc_aoff, p->inc_L0, p->inc_Ll,
                   p->inc_F, p->inc_B0, p->inc_B1, p->inc_bm, p->inc_wl0, p->inc_wl1, p->inc_T8, p->inc_done,
                   p->scan_tmp})
    t += (b + 255) / 256 * 256;
  return t;
}

// Points the buffers of w into [base, base + plan total), every buffer fixed.
void carve_workspace(Workspace* w, char* base, const IncPlan& p) {
  for (DevBuf* b : w->buffers()) {
    b->p = nullptr;
    b->bytes = 0;
    b->fixed = true;
  }
  size_t off = 0;
  auto take = [&](DevBuf& b, size_t bytes) {
    b.p = base + off;
    b.bytes = bytes;
    off += (bytes + 255) / 256 * 256;
  };
  take(w->small, p.small);
  take(w->T, p.T);
  take(w->work, p.work);
  take(w->bin, p.bin);
  take(w->wl0, p.wl0);
  take(w->wl1, p.wl1);
  take(w->trace, p.trace);
  take(w->deferred, p.deferred);
  take(w->deferred_work, p.deferred_work);
  take(w->deferred_done, p.deferred_done);
  take(w->inc_len, p.inc_len);
  take(w->inc_words, p.inc_words);
  take(w->inc_fwoff, p.inc_fwoff);
  take(w->inc_aoff, p.inc_aoff);
  take(w->inc_L0, p.inc_L0);
  take(w->inc_Ll, p.inc_Ll);
  take(w->inc_F, p.inc_F);
  take(w->inc_B0, p.inc_B0);
  take(w->inc_B1, p.inc_B1);
  take(w->inc_bm, p.inc_bm);
  take(w->inc_wl0, p.inc_wl0);
  take(w->inc_wl1, p.inc_wl1);
  take(w->inc_T8, p.inc_T8);
  take(w->inc_done, p.inc_done);
  take(w->scan_tmp, p.scan_tmp);
}

}  // namespace gcol

using namespace gcol;

extern "C" {

int color_d1(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed, const uint32_t* prio,
             const int32_t* init_colors, int32_t* colors, color_stats* stats, const color_params* params,
             void* stream) {
  return color_graph<kD1>(n, n, row_ptr, col_idx, row_ptr, col_idx, seed, prio, init_colors, colors, stats,
                          params, stream);
}

int color_d2(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed, const uint32_t* prio,
             const int32_t* init_colors, int32_t* colors, color_stats* stats, const color_params* params,
             void* stream) {
  return color_graph<kD2>(n, n, row_ptr, col_idx, row_ptr, col_idx, seed, prio, init_colors, colors, stats,
                          params, stream);
}

int color_pd2(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr, const int32_t* col_idx,
              const int32_t* col_ptr, const int32_t* row_idx, uint32_t seed, const uint32_t* prio,
              const int32_t* init_colors, int32_t* col_colors, color_stats* stats, const color_params* params,
              void* stream) {
  if (n_cols > 0 && n_rows > 0 && (!row_ptr || !col_idx)) return COLOR_EINVAL;
  // hop 1: column -> rows (CSC); hop 2: row -> columns (CSR)
  return color_graph<kPD2>(n_cols, n_rows, col_ptr, row_idx, row_ptr, col_idx, seed, prio, init_colors,
                           col_colors, stats, params, stream);
}

static int ghost_step_once(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1, const int32_t* row_ptr,
                        const int32_t* col_idx, const int32_t* gid, const int32_t* ghost_colors,
                        const int32_t* ghost_degree, uint32_t seed, const int32_t* init_owned,
                        int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats,
                        const color_params* params, void* stream) {
  if (n_owned < 0 || n_ghost < 0 || n_g1 < 0 || n_g1 > n_ghost) return COLOR_EINVAL;
  if (layers != 1 && layers != 2) return COLOR_EINVAL;
  if (static_cast<int64_t>(n_owned) + n_ghost >= INT_MAX) return COLOR_EOVERFLOW;
  if (n_owned > 0 && (!row_ptr || !col_idx || !gid || !owned_colors)) return COLOR_EINVAL;
  if (n_ghost > 0 && (!ghost_colors || !gid)) return COLOR_EINVAL;
  const bool degrees = params && (params->flags & COLOR_FLAG_RECOLOR_DEGREES);
  if (degrees && n_ghost > 0 && !ghost_degree) return COLOR_EINVAL;
  const bool grec = params && (params->flags & COLOR_FLAG_GHOST_RECOLOR);
  const int32_t m = n_owned + n_ghost;
  // with tentative ghost recoloring, phase 3 runs over every id that has a
  // row: owned and (two layers) layer-1 ghosts, or (one layer) every ghost
  const int32_t n3 = grec ? (layers == 2 ? n_owned + n_g1 : m) : n_owned;
  Call c;
  int e = begin_call(c, kD1, params, stats, stream, n3, m);
  if (e) return e;
  if (n_owned == 0) return finish_call(c, stats, 0, COLOR_OK);
  Workspace* w = c.ws;
  if ((e = w->C.ensure(sizeof(int32_t) * static_cast<size_t>(m), false, c.st))) return e;
  if ((e = w->aux0.ensure(sizeof(int32_t) * static_cast<size_t>(n_owned), false, c.st))) return e;
  if ((e = w->aux1.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n_ghost, 1)), false, c.st))) return e;
  int32_t* Cint = w->C.as<int32_t>();
  const int32_t n_rows = layers == 2 ? n_owned + n_g1 : n_owned;
  if (c.P.flags & COLOR_FLAG_VALIDATE) {
    // rows of owned (and layer-1) vertices: in range, sorted; symmetry is not
    // required for the ghost rows' partners outside the local graph
    launch_validate(n_rows, m, row_ptr, col_idx, row_ptr, col_idx, n_rows, 1, &c.S->err, c.st);
    if (hipMemcpyAsync(&c.H->err, &c.S->err, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) != hipSuccess)
      return COLOR_EHIP;
    if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
    if (c.H->err) return COLOR_EGRAPH;
    if (hipMemsetAsync(&c.S->err, 0, sizeof(int32_t), c.st) != hipSuccess) return COLOR_EHIP;
  }
  KeySource k{nullptr, gid, hash_seed(seed), nullptr};
  // recolorDegrees: an owned vertex's degree is its row (all its edges are
  // local), a ghost's is the one its owner reports
  if (degrees) {
    if ((e = degree_rank(c, m, row_ptr, n_owned, ghost_degree, k))) return e;
  }
  // phase 1: ghost-blind rounds on the owned-induced subgraph (with
  // init_owned: only over the owned vertices it leaves uncolored), built
  // once: the owned rows without their ghost entries, on either engine
  int32_t owned_nnz = 0;
  if ((e = read_nnz(c, row_ptr, n_owned, &owned_nnz))) return e;
  {
    const size_t n1 = static_cast<size_t>(n_owned) + 1;
    const size_t e1 = static_cast<size_t>(owned_nnz) + 1;
    size_t scan_bytes = 0;
    if (exclusive_scan_i32(nullptr, nullptr, owned_nnz + 1, nullptr, &scan_bytes, c.st)) return COLOR_EHIP;
    // own_rp: the subgraph's offsets, then the flags and their scan
    if ((e = w->own_rp.ensure(sizeof(int32_t) * (n1 + 2 * e1), false, c.st)) ||
        (e = w->scan_tmp.ensure(scan_bytes, false, c.st)))
      return e;
    int32_t* rp1 = w->own_rp.as<int32_t>();
    int32_t* flag = rp1 + n1;
    int32_t* pos = flag + e1;
    if (launch_owned_subgraph(n_owned, owned_nnz, row_ptr, col_idx, flag, pos, rp1, nullptr, w->scan_tmp.p,
                              w->scan_tmp.bytes, c.st))
      return COLOR_EHIP;
    int32_t nnz1 = 0;
    if ((e = read_nnz(c, pos, owned_nnz, &nnz1))) return e;
    if ((e = w->own_ci.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(nnz1, 1)), false, c.st))) return e;
    launch_owned_subgraph(n_owned, owned_nnz, row_ptr, col_idx, flag, pos, rp1, w->own_ci.as<int32_t>(), nullptr, 0,
                          c.st);
    c.launches += 3;
  }
  GraphView g1{n_owned, n_owned, w->own_rp.as<int32_t>(), w->own_ci.as<int32_t>(), w->own_rp.as<int32_t>(),
               w->own_ci.as<int32_t>()};
  int rc = run_engine<kD1>(c, g1, k, init_owned, Cint, m);
  if (rc != COLOR_OK) return rc == COLOR_ENOCONVERGE ? finish_call(c, stats, -1, rc) : rc;
  // phases 2 and 3 read the full local rows
  GraphView g{n_owned, n_owned, row_ptr, col_idx, row_ptr, col_idx};
  if (hipMemcpyAsync(&c.H->rounds_done, &c.S->rounds_done, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) !=
      hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  const int r1 = c.H->rounds_done;
  // phase 2: boundary conflicts against the ghosts' fixed colors
  int32_t* loser = w->aux0.as<int32_t>();
  int32_t* gflag = w->aux1.as<int32_t>();
  if (hipMemsetAsync(gflag, 0, sizeof(int32_t) * static_cast<size_t>(std::max(n_ghost, 1)), c.st) != hipSuccess)
    return COLOR_EHIP;
  launch_zero_words(loser, static_cast<size_t>(n_owned), c.st);
  launch_boundary(n_owned, owned_nnz, row_ptr, col_idx, Cint, ghost_colors, k, loser, gflag, &c.S->conflicts, c.st);
  launch_boundary_uncolor(n_owned, loser, Cint, c.st);
  // phase 3: ghosts become fixed committed colors; losers are recolored
  launch_ghost_fill(n_owned, n_ghost, ghost_colors, Cint, w->T.as<int32_t>(), &c.S->maxc, c.st);
  c.launches += 3;
  // the phase-3 bin setup counts afresh: per-bin totals, maxima and the
  // worklist counts, whose ping-pong halves still hold phase 1's last rounds
  static_assert(offsetof(Scalars, count_unc) == offsetof(Scalars, count_all) + sizeof(Scalars::count_all),
                "per-bin counts are cleared together");
  launch_zero_words(c.S->count_all, 16, c.st);
  launch_zero_words(c.S->cnt, sizeof(c.S->cnt) / 4, c.st);
  launch_zero_words(&c.S->max_split_work, 1, c.st);
  launch_zero_words(&c.S->max_work, 1, c.st);
  launch_zero_words(&c.S->total_work, 2, c.st);
  c.launches += 5;
  if (!grec) {
    // the owned losers on the full rows, ghosts as fixed constraints
    g.limit = m;
    BinLayout L;
    RoundBufs rb;
    int32_t known[kBins];
    if ((e = setup_bins<kD1>(c, g, Cint, Cint, m, L, rb, known))) return e;
    rc = run_phase<kD1>(c, g, k, L, rb, known, r1, c.P.max_rounds);
  } else {
    // tentative ghost recoloring (Section 3.2 save/restore; Section 3.4):
    // owned losers and losing ghosts are recolored together on the local
    // graph; the ghosts' tentative colors are dropped afterwards
    const int32_t* rp3 = row_ptr;
    const int32_t* ci3 = col_idx;
    if (layers == 1 && n_ghost > 0) {
      const size_t ng1 = static_cast<size_t>(n_ghost) + 1;
      size_t scan_bytes = 0;
      if (exclusive_scan_i32(nullptr, nullptr, n_ghost + 1, nullptr, &scan_bytes, c.st)) return COLOR_EHIP;
      if ((e = w->gr_cnt.ensure(sizeof(int32_t) * 3 * ng1, false, c.st)) ||
          (e = w->gr_rp.ensure(sizeof(int32_t) * (static_cast<size_t>(m) + 1), false, c.st)) ||
          (e = w->scan_tmp.ensure(scan_bytes, false, c.st)))
        return e;
      int32_t* cnt = w->gr_cnt.as<int32_t>();
      launch_zero_words(cnt, 3 * ng1, c.st);
      // the owned rows' entries, then the ghosts' rows: one entry per
      // owned-ghost entry of the owned rows, so at most owned_nnz more
      if ((e = w->gr_ci.ensure(sizeof(int32_t) * (2 * static_cast<size_t>(owned_nnz) + 1), false, c.st))) return e;
      int err = 0;
      launch_ghost_rows(n_owned, n_ghost, owned_nnz, row_ptr, col_idx, cnt, cnt + ng1, cnt + 2 * ng1,
                        w->gr_rp.as<int32_t>(), w->gr_ci.as<int32_t>(), w->scan_tmp.p, w->scan_tmp.bytes, c.st, &err);
      c.launches += 4;
      if (err || hipGetLastError() != hipSuccess) return COLOR_EHIP;
      rp3 = w->gr_rp.as<int32_t>();
      ci3 = w->gr_ci.as<int32_t>();
    }
    if ((e = w->gr_init.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n3, 1)), false, c.st))) return e;
    launch_ghost_recolor_init(n_owned, n3, Cint, ghost_colors, gflag, w->gr_init.as<int32_t>(), c.st);
    c.launches += 1;
    GraphView g3{n3, n3, rp3, ci3, rp3, ci3};
    g3.limit = m;
    BinLayout L3;
    RoundBufs rb3;
    int32_t known3[kBins];
    if ((e = setup_bins<kD1>(c, g3, w->gr_init.as<int32_t>(), Cint, m, L3, rb3, known3))) return e;
    rc = run_phase<kD1>(c, g3, k, L3, rb3, known3, r1, c.P.max_rounds);
  }
  if (rc != COLOR_OK && rc != COLOR_ENOCONVERGE) return rc;
  launch_flags_out(n_ghost, gflag, remote_loser, &c.S->remote, c.st);
  launch_copy_i32(n_owned, Cint, owned_colors, c.st);
  launch_max_i32(n_owned, Cint, &c.S->aux_max, c.st);
  c.launches += 3;
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
  if (hipMemcpyAsync(&c.H->aux_max, &c.S->aux_max, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) != hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  return finish_call(c, stats, c.H->aux_max, rc);
}

// A step whose tail kernel's grid barrier gave up starts over with
// per-round launches only (the same coloring).
int color_d1_ghost_step(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1, const int32_t* row_ptr,
                        const int32_t* col_idx, const int32_t* gid, const int32_t* ghost_colors,
                        const int32_t* ghost_degree, uint32_t seed, const int32_t* init_owned,
                        int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats,
                        const color_params* params, void* stream) {
  const int rc = ghost_step_once(n_owned, n_ghost, layers, n_g1, row_ptr, col_idx, gid, ghost_colors, ghost_degree,
                                 seed, init_owned, owned_colors, remote_loser, stats, params, stream);
  if (rc != kRcRetryNoTail) return rc;
  color_params p;
  if (params) p = *params;
  else std::memset(&p, 0, sizeof(p));
  p.flags |= COLOR_FLAG_NO_TAIL;
  return ghost_step_once(n_owned, n_ghost, layers, n_g1, row_ptr, col_idx, gid, ghost_colors, ghost_degree, seed,
                         init_owned, owned_colors, remote_loser, stats, &p, stream);
}

}  // extern "C"

namespace gcol {

// One rank's distance-2 (MODE kD2) or partial distance-2 (kPD2) step:
// ghost-uncolored phase 1 on the owned vertices (the two-hop walks pass
// through ghosts, whose colors and tentative colors are 0) on the engine the
// parameters name or the library's choice, the two-hop boundary detect
// against the ghosts' fixed colors, and the recoloring of the owned losers
// with the ghosts' colors as constraints on the pull engine.
template <int MODE>
static int ghost2_step_once(int32_t n_owned, int32_t n_ghost, const int32_t* rp1, const int32_t* ci1,
                            const int32_t* rp2, const int32_t* ci2, const int32_t* gid, const int32_t* ghost_colors,
                            uint32_t seed, int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats,
                            const color_params* params, void* stream) {
  if (n_owned < 0 || n_ghost < 0) return COLOR_EINVAL;
  if (static_cast<int64_t>(n_owned) + n_ghost >= INT_MAX) return COLOR_EOVERFLOW;
  if (n_owned > 0 && (!rp1 || !ci1 || !rp2 || !ci2 || !gid || !owned_colors)) return COLOR_EINVAL;
  if (n_ghost > 0 && (!ghost_colors || !gid)) return COLOR_EINVAL;
  const int32_t m = n_owned + n_ghost;
  Call c;
  int e = begin_call(c, MODE, params, stats, stream, n_owned, m);
  if (e) return e;
  if (n_owned == 0) return finish_call(c, stats, 0, COLOR_OK);
  Workspace* w = c.ws;
  if ((e = w->C.ensure(sizeof(int32_t) * static_cast<size_t>(m), false, c.st))) return e;
  if ((e = w->aux0.ensure(sizeof(int32_t) * static_cast<size_t>(n_owned), false, c.st))) return e;
  if ((e = w->aux1.ensure(sizeof(int32_t) * static_cast<size_t>(std::max(n_ghost, 1)), false, c.st))) return e;
  int32_t* Cint = w->C.as<int32_t>();
  KeySource k{nullptr, gid, hash_seed(seed), nullptr};
  // phase 1: ghosts uncolored (0 constrains nothing and never ties), on
  // either engine: the pull engine walks through the ghosts and reads their
  // zeros; the incremental engine's lists keep the owned members only
  // (limit), as a ghost can neither constrain nor beat an owned vertex here
  launch_zero_words(Cint + n_owned, static_cast<size_t>(n_ghost), c.st);
  launch_zero_words(w->T.as<int32_t>() + n_owned, static_cast<size_t>(n_ghost), c.st);
  c.launches += 2;
  GraphView g1{n_owned, n_owned, rp1, ci1, rp2, ci2};
  int rc = run_engine<MODE>(c, g1, k, nullptr, Cint, m);
  if (rc != COLOR_OK) return rc == COLOR_ENOCONVERGE ? finish_call(c, stats, -1, rc) : rc;
  GraphView g{n_owned, n_owned, rp1, ci1, rp2, ci2};
  g.limit = m;
  if (hipMemcpyAsync(&c.H->rounds_done, &c.S->rounds_done, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) !=
      hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  const int r1 = c.H->rounds_done;
  // phase 2: owned vertices against the distinct ghosts of their two-hop
  // neighbourhoods (Algorithm 5 over the owned vertices)
  int32_t* loser = w->aux0.as<int32_t>();
  int32_t* gflag = w->aux1.as<int32_t>();
  launch_zero_words(gflag, static_cast<size_t>(std::max(n_ghost, 1)), c.st);
  launch_zero_words(loser, static_cast<size_t>(n_owned), c.st);
  int32_t nnz1 = 0;
  if ((e = read_nnz(c, rp1, n_owned, &nnz1))) return e;
  launch_boundary2<MODE>(g, n_owned, nnz1, Cint, ghost_colors, k, loser, gflag, &c.S->hits, nullptr, 0,
                         &c.S->conflicts, c.st);
  if (hipMemcpyAsync(&c.H->hits, &c.S->hits, sizeof(unsigned long long), hipMemcpyDeviceToHost, c.st) !=
          hipSuccess ||
      hipStreamSynchronize(c.st) != hipSuccess)
    return COLOR_EHIP;
  if (c.H->hits > 0) {
    // distinct pairs: a set with at least twice as many slots as entries
    uint64_t slots = 1024;
    while (slots < 2 * static_cast<uint64_t>(c.H->hits)) slots <<= 1;
    if ((e = w->pair_set.ensure(sizeof(unsigned long long) * slots, false, c.st))) return e;
    launch_fill_u64(w->pair_set.as<unsigned long long>(), slots, ~0ull, c.st);
    launch_boundary2<MODE>(g, n_owned, nnz1, Cint, ghost_colors, k, loser, gflag, &c.S->hits,
                           w->pair_set.as<unsigned long long>(), slots - 1, &c.S->conflicts, c.st);
    c.launches += 2;
  }
  launch_boundary_uncolor(n_owned, loser, Cint, c.st);
  // phase 3: ghosts carry their fixed colors; the losers are recolored on
  // either engine (the incremental engine's lists keep the owned members,
  // the ghosts' colors enter the losers' bitsets once) after a fresh bin
  // setup: the per-bin totals, maxima, heavy-vertex counters and worklist
  // counts still hold phase 1's
  launch_ghost_fill(n_owned, n_ghost, ghost_colors, Cint, w->T.as<int32_t>(), &c.S->maxc, c.st);
  c.launches += 2;
  static_assert(offsetof(Scalars, deferred_grab) == offsetof(Scalars, max_work) + 2 * sizeof(int32_t),
                "max_work, deferred_cnt and deferred_grab are cleared together");
  launch_zero_words(c.S->count_all, 16, c.st);
  launch_zero_words(c.S->cnt, sizeof(c.S->cnt) / 4, c.st);
  launch_zero_words(&c.S->max_split_work, 1, c.st);
  launch_zero_words(&c.S->max_work, 4, c.st);
  launch_zero_words(&c.S->total_work, 2, c.st);
  c.launches += 5;
  GraphView g3{n_owned, n_owned, rp1, ci1, rp2, ci2};
  g3.ids = m;
  rc = run_engine<MODE>(c, g3, k, Cint, Cint, m, r1);
  if (rc != COLOR_OK && rc != COLOR_ENOCONVERGE) return rc;
  launch_flags_out(n_ghost, gflag, remote_loser, &c.S->remote, c.st);
  launch_copy_i32(n_owned, Cint, owned_colors, c.st);
  launch_max_i32(n_owned, Cint, &c.S->aux_max, c.st);
  c.launches += 3;
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
  if (hipMemcpyAsync(&c.H->aux_max, &c.S->aux_max, sizeof(int32_t), hipMemcpyDeviceToHost, c.st) != hipSuccess)
    return COLOR_EHIP;
  if (hipStreamSynchronize(c.st) != hipSuccess) return COLOR_EHIP;
  return finish_call(c, stats, c.H->aux_max, rc);
}

// A step whose tail kernel's grid barrier gave up (phase 1 on the
// incremental engine) starts over with per-round launches only (the same
// coloring).
template <int MODE>
static int ghost2_step(int32_t n_owned, int32_t n_ghost, const int32_t* rp1, const int32_t* ci1, const int32_t* rp2,
                       const int32_t* ci2, const int32_t* gid, const int32_t* ghost_colors, uint32_t seed,
                       int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats, const color_params* params,
                       void* stream) {
  const int rc = ghost2_step_once<MODE>(n_owned, n_ghost, rp1, ci1, rp2, ci2, gid, ghost_colors, seed, owned_colors,
                                        remote_loser, stats, params, stream);
  if (rc != kRcRetryNoTail) return rc;
  color_params p;
  if (params) p = *params;
  else std::memset(&p, 0, sizeof(p));
  p.flags |= COLOR_FLAG_NO_TAIL;
  return ghost2_step_once<MODE>(n_owned, n_ghost, rp1, ci1, rp2, ci2, gid, ghost_colors, seed, owned_colors,
                                remote_loser, stats, &p, stream);
}

}  // namespace gcol

extern "C" {

int color_d2_ghost(int32_t n_owned, int32_t n_ghost, int32_t n_g1, const int32_t* row_ptr, const int32_t* col_idx,
                   const int32_t* gid, const int32_t* ghost_colors, uint32_t seed, int32_t* owned_colors,
                   uint8_t* remote_loser, color_stats* stats, const color_params* params, void* stream) {
  if (n_g1 < 0 || n_g1 > n_ghost) return COLOR_EINVAL;
  return ghost2_step<kD2>(n_owned, n_ghost, row_ptr, col_idx, row_ptr, col_idx, gid, ghost_colors, seed,
                          owned_colors, remote_loser, stats, params, stream);
}

int color_pd2_ghost(int32_t n_owned, int32_t n_ghost, int32_t n_rows, const int32_t* col_ptr, const int32_t* row_idx,
                    const int32_t* row_ptr, const int32_t* col_idx, const int32_t* gid, const int32_t* ghost_colors,
                    uint32_t seed, int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats,
                    const color_params* params, void* stream) {
  if (n_rows < 0) return COLOR_EINVAL;
  if (n_owned > 0 && n_rows == 0 && (!col_ptr || !row_idx)) return COLOR_EINVAL;
  return ghost2_step<kPD2>(n_owned, n_ghost, col_ptr, row_idx, row_ptr, col_idx, gid, ghost_colors, seed,
                           owned_colors, remote_loser, stats, params, stream);
}

int color_d1_ghost(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1, const int32_t* row_ptr,
                   const int32_t* col_idx, const int32_t* gid, const int32_t* ghost_colors, uint32_t seed,
                   int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats, const color_params* params,
                   void* stream) {
  return color_d1_ghost_step(n_owned, n_ghost, layers, n_g1, row_ptr, col_idx, gid, ghost_colors, nullptr, seed,
                             nullptr, owned_colors, remote_loser, stats, params, stream);
}

int color_priority(int32_t n, const int32_t* gid, uint32_t seed, uint32_t* out, void* stream) {
  if (n < 0 || (n > 0 && !out)) return COLOR_EINVAL;
  launch_priority(n, gid, hash_seed(seed), out, static_cast<hipStream_t>(stream));
  if (hipGetLastError() != hipSuccess) return COLOR_EHIP;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return COLOR_EHIP;
  return COLOR_OK;
}

int color_release_workspace(void) {
  release_batch_workspaces();
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto& kv : g_ws) {
    for (Workspace* w : kv.second.all) {
      std::lock_guard<std::mutex> lk2(w->mu);
      w->release();
      if (hipHostMalloc(reinterpret_cast<void**>(&w->host), sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        w->host = nullptr;
    }
  }
  return COLOR_OK;
}

const char* color_strerror(int code) {
  switch (code) {
    case COLOR_OK: return "ok";
    case COLOR_EINVAL: return "invalid argument";
    case COLOR_EGRAPH: return "graph violates the input contract";
    case COLOR_EOVERFLOW: return "size exceeds int32 indexing";
    case COLOR_ENOMEM: return "out of memory";
    case COLOR_EHIP: return "HIP runtime error";
    case COLOR_ENOCONVERGE: return "round limit reached (partial coloring returned)";
    case COLOR_E2BIG: return "job exceeds the server's memory budget";
    case COLOR_EMISMATCH: return "two work mappings gave different colorings";
    case COLOR_ESCRATCH: return "graph exceeds the no-allocation entry point's scratch (COLOR_NOALLOC_MAX_N)";
    case COLOR_EQUEUED: return "job queued";
    case COLOR_EPENDING: return "job pending";
    default: return "unknown error";
  }
}

}  // extern "C"
