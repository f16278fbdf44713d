// Served form: continuous batching over the batched persistent engine.
//
// A server owns one HBM arena (the budget given at creation), a table of
// job slots in device memory and streams of default priority: the compute
// stream runs epochs of the persistent kernel, the copy stream moves admitted
// jobs' arrays in and finished jobs' colors out while an epoch runs, and each
// heavy lane (jobs with long two-hop walks, colored by the single-graph
// calls) has its own.  An epoch runs every resident job for at most
// kEpochRounds rounds (jobs park at their epoch budget and resume in the next
// epoch); between epochs the host retires finished jobs, frees their slots
// and arena space, and admits queued jobs whose footprint fits.  A job's
// coloring is the same as the single-graph call's: the engine's rounds do not
// depend on which other jobs share a launch or on where a job parks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "batch.hpp"

namespace gcol {
namespace {

// Rounds per epoch: a short epoch lets the slots of finished jobs refill
// sooner (measured on MI355X, 2,000 mixed jobs with n up to 1e5, 256 slots:
// 8 rounds 216 graphs/s closed loop, 4 rounds 248, 2 rounds 262).
constexpr int32_t kEpochRounds = 2;
constexpr size_t kAlign = 256;
constexpr int32_t kMaxSlots = 1 << 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over the arena, with coalescing of free neighbours.
class Arena {
 public:
  void init(size_t bytes) {
    free_.clear();
    free_[0] = bytes;
    total_ = bytes;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t total() const { return total_; }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0;
};

enum class JobState { Queued, Copying, Running, Draining, Done };

struct ServedJob {
  color_job desc{};       // device pointers once admitted
  int32_t nnz = 0;
  int32_t n_csr_rows = 0; // rows of the CSR (D1/D2: n; PD2: n_rows)
  JobState state = JobState::Queued;
  // host copies of the input (pinned) and the result
  int32_t* h_in = nullptr;
  size_t h_in_entries = 0;
  std::vector<int32_t> colors;
  color_stats stats{};
  int rc = COLOR_OK;      // COLOR_ENOCONVERGE when the job hit the round cap
  BatchJob rec{};         // the job record, uploaded when the job joins an epoch
  size_t footprint = 0;
  size_t arena_off = 0;
  int32_t slot = -1;
  hipEvent_t ev = nullptr;  // copy in / copy out
  bool heavy = false;       // long two-hop walks: the single-graph engine's lane
  IncPlan plan{};           // heavy: the incremental engine's buffers, carved from the job's arena region
  size_t plan_bytes = 0;
};

}  // namespace
}  // namespace gcol

using namespace gcol;

// Heavy lanes: each a worker thread with its own stream and its own
// workspace of fixed buffers (regions of the running job's arena space), so
// that several long-walk jobs, whose rounds are mostly latency-bound, overlap
// on the device.
constexpr int kHeavyLanes = 3;

struct HeavyLane {
  std::thread thread;
  hipStream_t stream = nullptr;
  Workspace ws;
};

struct color_server {
  std::mutex mu;
  int device = 0;
  int32_t max_slots = 0;
  hipStream_t compute = nullptr, copy = nullptr;
  char* arena_base = nullptr;
  Arena arena;
  BatchJob* d_jobs = nullptr;
  uint64_t* d_words = nullptr;
  int32_t* d_ctr = nullptr;
  BatchTune* d_tune = nullptr;
  BatchJob* h_jobs = nullptr;   // pinned: job table staging / read-back
  uint64_t* h_words = nullptr;
  std::vector<uint64_t> slot_job;  // slot -> job id (0 = free)
  std::deque<uint64_t> queue;
  std::map<uint64_t, ServedJob> jobs;
  uint64_t next_id = 1;
  bool in_flight = false;
  hipEvent_t epoch_done = nullptr;
  int error = COLOR_OK;
  std::vector<uint64_t> draining;  // jobs whose colors are being copied out
  // heavy lanes: jobs with long two-hop walks, each colored by the
  // single-graph call of its kind (incremental engine) on a lane's stream and
  // thread
  std::deque<uint64_t> heavy_queue;
  HeavyLane heavy[kHeavyLanes];
  std::condition_variable heavy_cv;  // wakes the heavy lanes
  std::condition_variable done_cv;   // a heavy job finished
  bool stopping = false;
};

namespace {

// Arena bytes of a job: its CSR (+ CSC), its colors, and its workspace: the
// batched engine's 16 bytes per vertex, or for a heavy-lane job every buffer
// of the single-graph incremental engine (plan_bytes), so that the server's
// device memory stays within its budget.
size_t job_footprint(const color_job& j, int32_t nnz, int32_t n_csr_rows, bool heavy, size_t plan_bytes) {
  size_t b = align_up(sizeof(int32_t) * (static_cast<size_t>(n_csr_rows) + 1)) +
             align_up(sizeof(int32_t) * static_cast<size_t>(nnz));
  if (j.kind == COLOR_KIND_PD2)
    b += align_up(sizeof(int32_t) * (static_cast<size_t>(j.n) + 1)) +
         align_up(sizeof(int32_t) * static_cast<size_t>(nnz));
  b += align_up(sizeof(int32_t) * static_cast<size_t>(std::max(j.n, 1)));
  b += heavy ? plan_bytes : sizeof(int32_t) * 4 * static_cast<size_t>(batch_stride(j.n));
  return b;
}

void free_job_resources(color_server* s, ServedJob& J) {
  if (J.slot >= 0) {
    s->slot_job[J.slot] = 0;
    J.slot = -1;
  }
  if (J.footprint) {
    s->arena.release(J.arena_off, J.footprint);
    J.footprint = 0;
  }
  if (J.h_in) {
    (void)hipHostFree(J.h_in);
    J.h_in = nullptr;
  }
  if (J.ev) {
    (void)hipEventDestroy(J.ev);
    J.ev = nullptr;
  }
}

// Places the job's arrays in its arena region and starts their copy in.
int start_copy_in(color_server* s, ServedJob& J, int32_t slot) {
  char* p = s->arena_base + J.arena_off;
  const int32_t* h = J.h_in;
  auto put = [&](size_t entries, const int32_t*& dst_const, int32_t** dst) {
    int32_t* d = reinterpret_cast<int32_t*>(p);
    p += align_up(sizeof(int32_t) * entries);
    if (entries && hipMemcpyAsync(d, h, sizeof(int32_t) * entries, hipMemcpyHostToDevice, s->copy) != hipSuccess)
      return COLOR_EHIP;
    h += entries;
    if (dst) *dst = d;
    dst_const = d;
    return COLOR_OK;
  };
  color_job& d = J.desc;
  int e;
  if ((e = put(static_cast<size_t>(J.n_csr_rows) + 1, d.row_ptr, nullptr))) return e;
  if ((e = put(static_cast<size_t>(J.nnz), d.col_idx, nullptr))) return e;
  if (d.kind == COLOR_KIND_PD2) {
    if ((e = put(static_cast<size_t>(d.n) + 1, d.col_ptr, nullptr))) return e;
    if ((e = put(static_cast<size_t>(J.nnz), d.row_idx, nullptr))) return e;
  }
  d.colors = reinterpret_cast<int32_t*>(p);
  p += align_up(sizeof(int32_t) * static_cast<size_t>(std::max(d.n, 1)));
  fill_job(d, kBatchMaxRounds, reinterpret_cast<int32_t*>(p), &J.rec);
  J.rec.stop_epoch = 1 + 2 * kEpochRounds;
  if (hipEventRecord(J.ev, s->copy) != hipSuccess) return COLOR_EHIP;
  J.slot = slot;
  J.state = JobState::Copying;
  return COLOR_OK;
}

// Admits queued jobs (FIFO, with a short look-ahead past jobs that do not fit).
int admit(color_server* s) {
  int scanned = 0;
  for (auto it = s->queue.begin(); it != s->queue.end() && scanned < 8;) {
    ServedJob& J = s->jobs[*it];
    int32_t slot = -1;
    for (int32_t i = 0; i < s->max_slots; ++i)
      if (s->slot_job[i] == 0) {
        slot = i;
        break;
      }
    if (slot < 0) return COLOR_OK;
    size_t off = 0;
    if (!s->arena.alloc(J.footprint, &off)) {
      ++scanned;
      ++it;
      continue;
    }
    J.arena_off = off;
    int e = start_copy_in(s, J, slot);
    if (e) return e;
    s->slot_job[slot] = *it;
    it = s->queue.erase(it);
  }
  return COLOR_OK;
}

// Collects a finished epoch: finished jobs start their copy out.
int collect_epoch(color_server* s) {
  for (int32_t i = 0; i < s->max_slots; ++i) {
    const uint64_t id = s->slot_job[i];
    if (!id) continue;
    ServedJob& J = s->jobs[id];
    if (J.state != JobState::Running) continue;
    const BatchJob& B = s->h_jobs[i];
    if (B.status != kJobFinished) continue;
    job_stats(B, &J.stats);
    J.rc = B.rc;
    J.colors.resize(static_cast<size_t>(J.desc.n));
    if (J.desc.n > 0 &&
        hipMemcpyAsync(J.colors.data(), J.desc.colors, sizeof(int32_t) * J.colors.size(), hipMemcpyDeviceToHost,
                       s->copy) != hipSuccess)
      return COLOR_EHIP;
    if (hipEventRecord(J.ev, s->copy) != hipSuccess) return COLOR_EHIP;
    J.state = JobState::Draining;
    s->draining.push_back(id);
  }
  return COLOR_OK;
}

// Jobs whose copy out has completed become Done and free their resources
// (a list of the draining jobs: every poll comes here, so no pass over all
// jobs).  A failed copy is an error of the server, not a copy still running.
int retire_drained(color_server* s) {
  size_t keep = 0;
  int rc = COLOR_OK;
  for (size_t i = 0; i < s->draining.size(); ++i) {
    ServedJob& J = s->jobs.at(s->draining[i]);
    const hipError_t q = hipEventQuery(J.ev);
    if (q != hipSuccess) {
      if (q != hipErrorNotReady) rc = COLOR_EHIP;
      s->draining[keep++] = s->draining[i];
      continue;
    }
    J.state = JobState::Done;
    free_job_resources(s, J);
  }
  s->draining.resize(keep);
  return rc;
}

// Launches the next epoch over every resident job (newly copied-in jobs
// join; parked jobs resume).
int launch_epoch(color_server* s) {
  int32_t active = 0;
  bool any_parked = false;
  for (int32_t i = 0; i < s->max_slots; ++i) {
    const uint64_t id = s->slot_job[i];
    if (!id) continue;
    ServedJob& J = s->jobs[id];
    const hipError_t q = J.state == JobState::Copying ? hipEventQuery(J.ev) : hipErrorNotReady;
    if (q != hipSuccess && q != hipErrorNotReady) return COLOR_EHIP;  // the copy in failed
    if (J.state == JobState::Copying && q == hipSuccess) {
      if (J.desc.n == 0) {  // nothing to color: finished at once
        job_stats(J.rec, &J.stats);
        J.state = JobState::Done;
        free_job_resources(s, J);
        continue;
      }
      s->h_jobs[i] = J.rec;
      s->h_words[i] = initial_word(J.desc.n);
      if (hipMemcpyAsync(&s->d_jobs[i], &s->h_jobs[i], sizeof(BatchJob), hipMemcpyHostToDevice, s->compute) !=
              hipSuccess ||
          hipMemcpyAsync(&s->d_words[i], &s->h_words[i], sizeof(uint64_t), hipMemcpyHostToDevice, s->compute) !=
              hipSuccess)
        return COLOR_EHIP;
      J.state = JobState::Running;
      ++active;
    } else if (J.state == JobState::Running) {
      if (s->h_jobs[i].status == kJobParked) any_parked = true;
      ++active;
    }
  }
  if (active == 0) return COLOR_OK;
  if (any_parked) {
    int e = launch_unpark(s->d_jobs, s->d_words, s->max_slots, 2 * kEpochRounds, s->compute);
    if (e) return e;
  }
  if (hipMemsetAsync(s->d_ctr, 0, sizeof(int32_t), s->compute) != hipSuccess) return COLOR_EHIP;
  const int grid = batch_resident_blocks();
  int e = launch_batch(s->d_jobs, s->d_words, s->max_slots, active, s->d_ctr, s->d_tune, grid, true, s->compute);
  if (e) return e;
  if (hipMemcpyAsync(s->h_jobs, s->d_jobs, sizeof(BatchJob) * static_cast<size_t>(s->max_slots),
                     hipMemcpyDeviceToHost, s->compute) != hipSuccess ||
      hipEventRecord(s->epoch_done, s->compute) != hipSuccess)
    return COLOR_EHIP;
  s->in_flight = true;
  return COLOR_OK;
}

// One step of the serving loop.  wait: block until the running epoch ends.
int advance(color_server* s, bool wait) {
  if (s->error) return s->error;
  int e = COLOR_OK;
  if (s->in_flight) {
    hipError_t q = wait ? hipEventSynchronize(s->epoch_done) : hipEventQuery(s->epoch_done);
    if (q == hipSuccess) {
      s->in_flight = false;
      if ((e = collect_epoch(s))) return s->error = e;
    } else if (q != hipErrorNotReady) {
      return s->error = COLOR_EHIP;
    }
  }
  if ((e = retire_drained(s))) return s->error = e;
  if ((e = admit(s))) return s->error = e;
  if (!s->in_flight) {
    if (wait) {
      // copies in flight must land before their jobs can join an epoch
      for (int32_t i = 0; i < s->max_slots; ++i) {
        const uint64_t id = s->slot_job[i];
        if (id && s->jobs[id].state == JobState::Copying && hipEventSynchronize(s->jobs[id].ev) != hipSuccess)
          return s->error = COLOR_EHIP;
      }
    }
    if ((e = launch_epoch(s))) return s->error = e;
  }
  if (wait && !s->in_flight) {
    // nothing launched: finish outstanding copies out
    for (auto& kv : s->jobs)
      if (kv.second.state == JobState::Draining && hipEventSynchronize(kv.second.ev) != hipSuccess)
        return s->error = COLOR_EHIP;
    if ((e = retire_drained(s))) return s->error = e;
  }
  return COLOR_OK;
}

bool busy(const color_server* s) {
  if (s->in_flight || !s->queue.empty()) return true;
  for (const auto& kv : s->jobs)
    if (kv.second.state != JobState::Done) return true;
  return false;
}

// Two-hop walk per visit above which a job goes to the heavy lanes (the same
// bound as the single-graph engine choice and color_batch).
constexpr double kLongWalk = 128.0;

double job_walk(const color_job& j, int32_t nnz) {
  if (j.kind == COLOR_KIND_D1 || j.n <= 0) return 0.0;
  const double d = static_cast<double>(nnz) / j.n;
  if (j.kind == COLOR_KIND_D2) return d * (d + 1.0);
  return d * (1.0 + static_cast<double>(nnz) / std::max(j.n_rows, 1));
}

// Copies a heavy job in, colors it with the single-graph call of its kind
// and copies the colors out, all on the heavy lane's stream.
int run_heavy(color_server* s, HeavyLane& lane, ServedJob& J) {
  char* p = s->arena_base + J.arena_off;
  const int32_t* h = J.h_in;
  auto put = [&](size_t entries) {
    int32_t* d = reinterpret_cast<int32_t*>(p);
    p += align_up(sizeof(int32_t) * entries);
    if (entries && hipMemcpyAsync(d, h, sizeof(int32_t) * entries, hipMemcpyHostToDevice, lane.stream) !=
                       hipSuccess)
      return static_cast<int32_t*>(nullptr);
    h += entries;
    return d;
  };
  color_job& d = J.desc;
  const int32_t* rp = put(static_cast<size_t>(J.n_csr_rows) + 1);
  const int32_t* ci = put(static_cast<size_t>(J.nnz));
  if (!rp || (J.nnz > 0 && !ci)) return COLOR_EHIP;
  const int32_t* cp = nullptr;
  const int32_t* ri = nullptr;
  if (d.kind == COLOR_KIND_PD2) {
    cp = put(static_cast<size_t>(d.n) + 1);
    ri = put(static_cast<size_t>(J.nnz));
    if (!cp || (J.nnz > 0 && !ri)) return COLOR_EHIP;
  }
  int32_t* colors = reinterpret_cast<int32_t*>(p);
  p += align_up(sizeof(int32_t) * static_cast<size_t>(std::max(d.n, 1)));
  // the engine's buffers: the rest of the job's arena region
  carve_workspace(&lane.ws, p, J.plan);
  // Per-round launches only: the light lane's persistent kernel fills the
  // device at the same time, so a cooperative tail launch would mostly find
  // its workgroups not all resident and fall back after its check-in wait.
  color_params prm;
  std::memset(&prm, 0, sizeof(prm));
  prm.flags = COLOR_FLAG_NO_TAIL;
  prm.engine = COLOR_ENGINE_INCREMENTAL;
  int rc = d.kind == COLOR_KIND_D2
               ? color_d2_fixed(&lane.ws, d.n, rp, ci, d.seed, colors, &J.stats, &prm, lane.stream)
               : color_pd2_fixed(&lane.ws, J.n_csr_rows, d.n, rp, ci, cp, ri, d.seed, colors, &J.stats, &prm,
                                 lane.stream);
  if (rc != COLOR_OK && rc != COLOR_ENOCONVERGE) return rc;
  J.rc = rc;
  J.colors.resize(static_cast<size_t>(d.n));
  if (hipMemcpyAsync(J.colors.data(), colors, sizeof(int32_t) * J.colors.size(), hipMemcpyDeviceToHost,
                     lane.stream) != hipSuccess ||
      hipStreamSynchronize(lane.stream) != hipSuccess)
    return COLOR_EHIP;
  return COLOR_OK;
}

void heavy_lane(color_server* s, int li) {
  HeavyLane& lane = s->heavy[li];
  if (hipSetDevice(s->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->error = COLOR_EHIP;
    s->done_cv.notify_all();
    return;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->heavy_cv.wait(lk, [&] { return s->stopping || !s->heavy_queue.empty(); });
    if (s->stopping) break;
    const uint64_t id = s->heavy_queue.front();
    ServedJob& J = s->jobs[id];
    size_t off = 0;
    if (!s->arena.alloc(J.footprint, &off)) {  // wait for arena space freed by the other lane
      s->heavy_cv.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    s->heavy_queue.pop_front();
    J.arena_off = off;
    J.state = JobState::Running;
    lk.unlock();
    const int e = run_heavy(s, lane, J);  // J stays put: only Done jobs are erased
    lk.lock();
    s->arena.release(J.arena_off, J.footprint);
    J.footprint = 0;
    if (J.h_in) {
      (void)hipHostFree(J.h_in);
      J.h_in = nullptr;
    }
    if (e) J.rc = e;  // this job's failure, reported by its poll; other jobs go on
    J.state = JobState::Done;
    s->done_cv.notify_all();
  }
}

void destroy_server(color_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->heavy_cv.notify_all();
  for (HeavyLane& lane : s->heavy) {
    if (lane.thread.joinable()) lane.thread.join();
    if (lane.stream) (void)hipStreamSynchronize(lane.stream);
  }
  if (s->compute) (void)hipStreamSynchronize(s->compute);
  if (s->copy) (void)hipStreamSynchronize(s->copy);
  for (auto& kv : s->jobs) free_job_resources(s, kv.second);
  if (s->epoch_done) (void)hipEventDestroy(s->epoch_done);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->d_jobs) (void)hipFree(s->d_jobs);
  if (s->d_words) (void)hipFree(s->d_words);
  if (s->d_ctr) (void)hipFree(s->d_ctr);
  if (s->d_tune) (void)hipFree(s->d_tune);
  if (s->h_jobs) (void)hipHostFree(s->h_jobs);
  if (s->h_words) (void)hipHostFree(s->h_words);
  if (s->compute) (void)hipStreamDestroy(s->compute);
  if (s->copy) (void)hipStreamDestroy(s->copy);
  for (HeavyLane& lane : s->heavy)
    if (lane.stream) (void)hipStreamDestroy(lane.stream);
  delete s;
}

}  // namespace

extern "C" {

color_server* color_server_create(size_t hbm_budget_bytes, int32_t max_slots, int* err) {
  int dummy;
  if (!err) err = &dummy;
  if (hbm_budget_bytes < kAlign || max_slots < 1 || max_slots > kMaxSlots) {
    *err = COLOR_EINVAL;
    return nullptr;
  }
  color_server* s = new color_server();
  s->max_slots = max_slots;
  const size_t ns = static_cast<size_t>(max_slots);
  auto fail = [&](int code) {
    destroy_server(s);
    *err = code;
    return static_cast<color_server*>(nullptr);
  };
  if (hipGetDevice(&s->device) != hipSuccess) return fail(COLOR_EHIP);
  if (hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->epoch_done, hipEventDisableTiming) != hipSuccess)
    return fail(COLOR_EHIP);
  for (HeavyLane& lane : s->heavy) {
    if (hipStreamCreateWithFlags(&lane.stream, hipStreamNonBlocking) != hipSuccess) return fail(COLOR_EHIP);
    if (hipHostMalloc(reinterpret_cast<void**>(&lane.ws.host), sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
      return fail(COLOR_ENOMEM);
  }
  if (hipMalloc(reinterpret_cast<void**>(&s->arena_base), hbm_budget_bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->d_jobs), sizeof(BatchJob) * ns) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->d_words), sizeof(uint64_t) * ns) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->d_ctr), kAlign) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->d_tune), sizeof(BatchTune) * 3 * kTuneClasses) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->h_jobs), sizeof(BatchJob) * ns, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->h_words), sizeof(uint64_t) * ns, hipHostMallocDefault) !=
          hipSuccess)
    return fail(COLOR_ENOMEM);
  s->arena.init(hbm_budget_bytes / kAlign * kAlign);
  std::memset(s->h_jobs, 0, sizeof(BatchJob) * ns);
  std::memset(s->h_words, 0, sizeof(uint64_t) * ns);
  for (size_t i = 0; i < ns; ++i) s->h_jobs[i].status = kJobFinished;
  std::vector<BatchTune> tune(3 * kTuneClasses);
  tune_table_for_device(tune.data());
  if (hipMemcpyAsync(s->d_tune, tune.data(), sizeof(BatchTune) * tune.size(), hipMemcpyHostToDevice, s->compute) !=
          hipSuccess ||
      hipMemcpyAsync(s->d_jobs, s->h_jobs, sizeof(BatchJob) * ns, hipMemcpyHostToDevice, s->compute) != hipSuccess ||
      hipMemsetAsync(s->d_words, 0, sizeof(uint64_t) * ns, s->compute) != hipSuccess ||
      hipStreamSynchronize(s->compute) != hipSuccess)
    return fail(COLOR_EHIP);
  s->slot_job.assign(ns, 0);
  try {
    for (int i = 0; i < kHeavyLanes; ++i) s->heavy[i].thread = std::thread(heavy_lane, s, i);
  } catch (...) {
    return fail(COLOR_ENOMEM);
  }
  *err = COLOR_OK;
  return s;
}

int color_server_submit(color_server* s, const color_host_job* job, uint64_t* job_id) {
  if (!s || !job) return COLOR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error) return s->error;
  color_job d{};
  d.kind = job->kind;
  d.n = job->n;
  d.n_rows = job->n_rows;
  d.seed = job->seed;
  // placeholders so that check_job sees the host arrays' presence
  d.row_ptr = job->row_ptr;
  d.col_idx = job->col_idx;
  d.col_ptr = job->col_ptr;
  d.row_idx = job->row_idx;
  d.colors = reinterpret_cast<int32_t*>(1);
  int e = check_job(d);
  if (e) return e;
  const int32_t n_csr_rows = d.kind == COLOR_KIND_PD2 ? d.n_rows : d.n;
  if (d.n > 0 && !d.row_ptr) return COLOR_EINVAL;
  const int32_t nnz = d.n > 0 ? job->row_ptr[n_csr_rows] : 0;
  if (nnz < 0) return COLOR_EINVAL;
  if (d.kind == COLOR_KIND_PD2 && d.n > 0 && job->col_ptr[d.n] != nnz) return COLOR_EINVAL;
  ServedJob J;
  J.nnz = nnz;
  J.n_csr_rows = n_csr_rows;
  J.heavy = job_walk(d, nnz) >= kLongWalk;
  if (J.heavy) {
    J.plan_bytes = d.kind == COLOR_KIND_D2
                       ? plan_incremental(d.kind, d.n, job->row_ptr, job->col_idx, job->row_ptr, &J.plan)
                       : plan_incremental(d.kind, d.n, job->col_ptr, job->row_idx, job->row_ptr, &J.plan);
    if (J.plan_bytes == 0) return COLOR_EHIP;
  }
  J.footprint = job_footprint(d, nnz, n_csr_rows, J.heavy, J.plan_bytes);
  if (J.footprint > s->arena.total()) return COLOR_E2BIG;
  J.h_in_entries = static_cast<size_t>(n_csr_rows) + 1 + static_cast<size_t>(nnz);
  if (d.kind == COLOR_KIND_PD2) J.h_in_entries += static_cast<size_t>(d.n) + 1 + static_cast<size_t>(nnz);
  if (hipHostMalloc(reinterpret_cast<void**>(&J.h_in), sizeof(int32_t) * J.h_in_entries, hipHostMallocDefault) !=
      hipSuccess)
    return COLOR_ENOMEM;
  int32_t* h = J.h_in;
  auto take = [&](const int32_t* src, size_t entries) {
    if (entries) std::memcpy(h, src, sizeof(int32_t) * entries);
    h += entries;
  };
  if (d.n > 0) {
    take(job->row_ptr, static_cast<size_t>(n_csr_rows) + 1);
    take(job->col_idx, static_cast<size_t>(nnz));
    if (d.kind == COLOR_KIND_PD2) {
      take(job->col_ptr, static_cast<size_t>(d.n) + 1);
      take(job->row_idx, static_cast<size_t>(nnz));
    }
  } else {
    std::memset(J.h_in, 0, sizeof(int32_t) * J.h_in_entries);
  }
  if (hipEventCreateWithFlags(&J.ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(J.h_in);
    return COLOR_EHIP;
  }
  J.desc = d;
  const uint64_t id = s->next_id++;
  s->jobs.emplace(id, J);
  if (job_id) *job_id = id;
  if (J.heavy) {
    s->heavy_queue.push_back(id);
    s->heavy_cv.notify_one();
    return COLOR_EQUEUED;
  }
  s->queue.push_back(id);
  if ((e = advance(s, false))) return e;
  return s->jobs[id].state == JobState::Queued ? COLOR_EQUEUED : COLOR_OK;
}

int color_server_poll(color_server* s, uint64_t job_id, int32_t* host_colors, color_stats* stats) {
  if (!s) return COLOR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return COLOR_EINVAL;
  int e = advance(s, false);
  if (e) return e;
  ServedJob& J = it->second;
  if (J.state != JobState::Done) return COLOR_EPENDING;
  if (host_colors && !J.colors.empty()) std::memcpy(host_colors, J.colors.data(), sizeof(int32_t) * J.colors.size());
  const int rc = J.rc;
  if (stats) *stats = J.stats;
  s->jobs.erase(it);
  return rc;
}

int color_server_drain(color_server* s) {
  if (!s) return COLOR_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  while (busy(s)) {
    int e = advance(s, true);
    if (e) return e;
    // nothing launched: the heavy lanes hold the remaining work or the arena
    // space queued jobs wait for; let it run
    if (!s->in_flight && busy(s)) s->done_cv.wait_for(lk, std::chrono::milliseconds(1));
  }
  return s->error;
}

int color_server_destroy(color_server* s) {
  if (!s) return COLOR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
  }
  destroy_server(s);
  return COLOR_OK;
}

}  // extern "C"
