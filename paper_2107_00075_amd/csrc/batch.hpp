// Batched persistent engine: many graphs colored by one launch.
//
// Every job runs the same synchronous rounds as the single-graph entry points
// (Section 3.2, Algorithms 2-4), so its colors, rounds and visit counts equal
// those of the single-graph call of its kind.  Jobs advance independently:
// each job has a phase word (epoch, units, grabbed) in device memory; the
// workgroups of the persistent kernel take units of any job's open phase by
// an atomic add on that word, and the workgroup that completes the last unit
// of a phase (a per-job atomic counter) closes it and opens the next one.
// There is no grid-wide barrier.
//
// Epochs of a job: 1 = setup A (work and bin counts), 2 = setup B (worklist
// scatter), then 2r+1 = color step of round r and 2r+2 = detect step of
// round r (r >= 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "graphcolor.h"
#include "rounds.hpp"

namespace gcol {

constexpr int kBatchBins = 4;            // bins 0..2: lane groups; bin 3: a workgroup per vertex
constexpr int32_t kBatchMaxN = 1 << 23;  // vertices per job (24-bit unit counters)
constexpr int32_t kBatchMaxRounds = 32000;
constexpr int kTuneClasses = 32;         // average-degree classes floor(log2(nnz / n))

// Tuning record of one (mode, degree class): bins and lanes per vertex.
struct BatchTune {
  int32_t bin_hi[3];
  int32_t lanes[3];
};

// Job record in device memory.  The host writes the fields up to pad0_ and
// zeroes the rest; the kernel owns the rest.
struct alignas(128) BatchJob {
  int32_t mode, n;
  uint32_t hs;          // hash_seed(seed)
  int32_t max_rounds;
  const int32_t* rp;    // hop 1 (D1/D2 adjacency; PD2 column -> rows)
  const int32_t* ci;
  const int32_t* rp2;   // hop 2 (D2 adjacency; PD2 row -> columns)
  const int32_t* ci2;
  int32_t* C;           // output colors
  int32_t* T;           // tentative colors
  int32_t* work;        // static work per vertex
  int32_t* wl0;
  int32_t* wl1;
  int32_t stop_epoch;   // the job parks instead of opening this epoch
  int32_t pad0_;
  // kernel state
  int32_t cnt_all[kBatchBins];
  int32_t off[kBatchBins + 1];
  int32_t pos[kBatchBins];
  int32_t cnt[2][kBatchBins];
  int32_t maxc;
  int32_t rounds;
  int32_t status;       // kJobRunning, kJobFinished, kJobParked
  int32_t rc;           // COLOR_OK or COLOR_ENOCONVERGE once finished
  uint32_t done;        // completed units of the open phase
  int32_t parked_epoch;
  int32_t parked_units;
  int32_t pad1_;
  unsigned long long visits[2];  // sum |W_r|, sum work(W_r)
};

enum : int32_t { kJobRunning = 0, kJobFinished = 1, kJobParked = 2 };

// Phase word: epoch (16 bits) | units (24 bits) | grabbed (24 bits).
__host__ __device__ inline uint64_t phase_word(uint32_t epoch, uint32_t units, uint32_t grabbed) {
  return (static_cast<uint64_t>(epoch) << 48) | (static_cast<uint64_t>(units) << 24) | grabbed;
}

// Launches the persistent kernel over num_jobs records; it returns when
// `active` jobs have finished or parked (counted in *retired, which the
// caller zeroes).  tune: kTuneClasses records per mode (3 x 32).
// coherent_graph: read the graph arrays with device-scope loads (graphs in
// memory that copies rewrite between launches).
int launch_batch(BatchJob* jobs, uint64_t* words, int32_t num_jobs, int32_t active, int32_t* retired,
                 const BatchTune* tune, int grid, bool coherent_graph, hipStream_t st);

// Reopens every parked job for budget_epochs more epochs.
int launch_unpark(BatchJob* jobs, uint64_t* words, int32_t num_jobs, int32_t budget_epochs, hipStream_t st);

// Workgroups of the persistent kernel resident on the device at once.
int batch_resident_blocks();

// Library default tuning table (3 x kTuneClasses records).
void default_tune_table(BatchTune* t);

// The current device's tuning table (autotuner records over the defaults).
void tune_table_for_device(BatchTune* t);

// Host helpers shared by color_batch and the server.
int check_job(const color_job& j);
int64_t batch_stride(int32_t n);  // int32 entries per workspace array of a job
void fill_job(const color_job& j, int32_t max_rounds, int32_t* base, BatchJob* out);
uint64_t initial_word(int32_t n);
void job_stats(const BatchJob& J, color_stats* st);
void release_batch_workspaces();

}  // namespace gcol
