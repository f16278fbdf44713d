// Batched persistent form: one launch colors many graphs.
//
// The kernel's workgroups are persistent workers.  Wavefront 0 of a worker
// scans the jobs' phase words (64 jobs per coalesced load), takes units of
// an open phase with one atomic add on that job's word, and the workgroup
// runs them with the same per-vertex steps as the single-graph round kernels
// (first-fit color step; detect + commit + compact).  The worker that
// completes a phase's last unit (per-job atomic counter) closes the phase:
// it computes the next phase's units from the job's worklist counts and
// publishes the new phase word.  Jobs therefore advance at their own pace,
// and a round of one job is the synchronous round of Section 3.2: its color
// units read only C, its detect units only T, and the next phase opens only
// after every unit of the previous one has completed.
//
// Unit ownership: the phase word packs (epoch, units, grabbed).  An add of k
// to the word returns the epoch and unit count it applied to; units
// [grabbed, min(grabbed + k, units)) are then owned by the caller, and while
// any of them is outstanding the phase cannot close, so the word's epoch and
// the job's counts stay put.  An add that finds grabbed >= units owns nothing.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "api_internal.hpp"
#include "batch.hpp"
#include "round_steps.hpp"

namespace gcol {

__device__ __forceinline__ uint32_t w_epoch(uint64_t w) { return static_cast<uint32_t>(w >> 48); }
__device__ __forceinline__ uint32_t w_units(uint64_t w) { return static_cast<uint32_t>(w >> 24) & 0xFFFFFFu; }
__device__ __forceinline__ uint32_t w_grabbed(uint64_t w) { return static_cast<uint32_t>(w) & 0xFFFFFFu; }

__device__ __forceinline__ void store_word(uint64_t* p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The job's static fields, read with device-scope loads: a slot's record is
// rewritten by copies between launches of the served form, and an L2 line of
// the previous record must not be read.
struct JobView {
  int32_t mode, n, max_rounds;
  uint32_t hs;
  GraphView g;
  int32_t *C, *T, *work, *wl0, *wl1;
};

template <typename X>
__device__ __forceinline__ X* ld_ptr(X* const* p) {
  return reinterpret_cast<X*>(ld_dev(reinterpret_cast<const uint64_t*>(p)));
}

__device__ __forceinline__ JobView load_job(const BatchJob* J) {
  JobView v;
  v.mode = ld_dev(&J->mode);
  v.n = ld_dev(&J->n);
  v.max_rounds = ld_dev(&J->max_rounds);
  v.hs = ld_dev(&J->hs);
  v.g.n = v.n;
  v.g.limit = v.n;
  v.g.rp = ld_ptr(&J->rp);
  v.g.ci = ld_ptr(&J->ci);
  v.g.rp2 = ld_ptr(&J->rp2);
  v.g.ci2 = ld_ptr(&J->ci2);
  v.C = ld_ptr(&J->C);
  v.T = ld_ptr(&J->T);
  v.work = ld_ptr(&J->work);
  v.wl0 = ld_ptr(&J->wl0);
  v.wl1 = ld_ptr(&J->wl1);
  return v;
}

// Tuning record of a job: its average first-hop degree class.
template <int LD>
__device__ __forceinline__ BatchTune tune_of(const JobView& J, const BatchTune* tune) {
  const int64_t nnz = gld<LD>(&J.g.rp[J.n]);
  const int64_t avg = nnz / (J.n > 0 ? J.n : 1);
  const int c = avg <= 1 ? 0 : min(kTuneClasses - 1, 63 - __builtin_clzll(static_cast<uint64_t>(avg)));
  const BatchTune* r = &tune[(J.mode - 1) * kTuneClasses + c];
  BatchTune t;  // the table is rewritten by copies between launches
  for (int i = 0; i < 3; ++i) {
    t.bin_hi[i] = ld_dev(&r->bin_hi[i]);
    t.lanes[i] = ld_dev(&r->lanes[i]);
  }
  return t;
}

__device__ __forceinline__ int bin_of(const BatchTune& t, int32_t w) {
  for (int i = 0; i < 3; ++i)
    if (w <= t.bin_hi[i]) return i;
  return 3;
}

// Units of a color/detect phase: light chunks of kBlock entries, then one
// unit per workgroup vertex.
__host__ __device__ inline uint32_t phase_units(const int32_t cnt[kBatchBins]) {
  uint32_t u = 0;
  for (int b = 0; b < 3; ++b) u += static_cast<uint32_t>((cnt[b] + kBlock - 1) / kBlock);
  return u + static_cast<uint32_t>(cnt[3]);
}

template <int MODE, int LD>
__device__ __forceinline__ int64_t job_vertex_work(const GraphView& g, int32_t v) {
  const int32_t b = gld<LD>(&g.rp[v]), e = gld<LD>(&g.rp[v + 1]);
  if (MODE == kD1) return e - b;
  int64_t w = 0;
  for (int32_t q = b; q < e; ++q) {
    const int32_t u = gld<LD>(&g.ci[q]);
    w += 1 + (gld<LD>(&g.rp2[u + 1]) - gld<LD>(&g.rp2[u]));
  }
  return w;
}

// Setup A: static work, initial colors, per-bin counts.
template <int MODE, int LD>
__device__ void setup_a_unit(BatchJob* J, const JobView& V, const BatchTune& t, int32_t u, int32_t* s_bc) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int32_t v = u * kBlock + tid;
  const bool active = v < V.n;
  int bin = -1;
  if (active) {
    const int64_t w = job_vertex_work<MODE, LD>(V.g, v);
    const int32_t wc = static_cast<int32_t>(w > INT_MAX ? INT_MAX : w);
    st_dev(&V.work[v], wc);
    st_dev(&V.C[v], 0);
    st_dev(&V.T[v], 0);
    bin = bin_of(t, wc);
  }
  for (int b = 0; b < kBatchBins; ++b) {
    const uint64_t bal = __ballot(bin == b);
    if (lane_id() == 0) s_bc[b * kWavesPerBlock + wave] = static_cast<int32_t>(__popcll(bal));
  }
  __syncthreads();
  if (tid < kBatchBins) {
    int32_t s = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) s += s_bc[tid * kWavesPerBlock + w];
    if (s) atomicAdd(&J->cnt_all[tid], s);
  }
  __syncthreads();
}

// Setup B: every vertex into its bin's region of W_1 (order within a bin is
// arbitrary; the result does not depend on it).
__device__ void setup_b_unit(BatchJob* J, const JobView& V, const BatchTune& t, int32_t u, int32_t* s_bc,
                             int32_t* s_base) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int32_t v = u * kBlock + tid;
  const bool active = v < V.n;
  const int bin = active ? bin_of(t, ld_dev(&V.work[v])) : -1;
  int32_t rank = 0;
  for (int b = 0; b < kBatchBins; ++b) {
    const uint64_t bal = __ballot(bin == b);
    if (bin == b) rank = static_cast<int32_t>(lanes_below(bal));
    if (lane_id() == 0) s_bc[b * kWavesPerBlock + wave] = static_cast<int32_t>(__popcll(bal));
  }
  __syncthreads();
  if (tid < kBatchBins) {
    int32_t tot = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      const int32_t c = s_bc[tid * kWavesPerBlock + w];
      s_bc[tid * kWavesPerBlock + w] = tot;
      tot += c;
    }
    s_base[tid] = (tot ? atomicAdd(&J->pos[tid], tot) : 0) + ld_dev(&J->off[tid]);
  }
  __syncthreads();
  if (active) st_dev(&V.wl0[s_base[bin] + s_bc[bin * kWavesPerBlock + wave] + rank], v);
  __syncthreads();
}

struct StepShared {
  uint32_t ovf[kOvfWords];
  uint64_t red[kWavesPerBlock];
  int32_t misc[4];
  int32_t ent[kBlock];
  int32_t wc[kWavesPerBlock + 1];
  int32_t cnt_in[kBatchBins];
  int32_t off[kBatchBins];
};

// Units [first, first + count) of the color (detect = false) or detect step
// of round r.
template <int MODE, int LD>
__device__ __forceinline__ void round_units(BatchJob* J, const JobView& V, const KeySource& k, const BatchTune& t, int r,
                            bool detect, uint32_t first, uint32_t count, StepShared& sh, uint64_t& work_acc,
                            int32_t& maxc_acc) {
  const int p = (r - 1) & 1;
  if (threadIdx.x < kBatchBins) {
    sh.cnt_in[threadIdx.x] = ld_dev(&J->cnt[p][threadIdx.x]);
    sh.off[threadIdx.x] = ld_dev(&J->off[threadIdx.x]);
  }
  __syncthreads();
  const GraphView& g = V.g;
  RoundBufs b{};
  b.C = V.C;
  b.T = V.T;
  b.work = V.work;
  b.wl_in = p ? V.wl1 : V.wl0;
  b.wl_out = p ? V.wl0 : V.wl1;
  b.cnt_in = J->cnt[p];
  b.cnt_out = J->cnt[p ^ 1];
  // scalars, not arrays: a dynamically indexed local array would live in
  // scratch memory
  const int32_t ch0 = (sh.cnt_in[0] + kBlock - 1) / kBlock;
  const int32_t ch1 = (sh.cnt_in[1] + kBlock - 1) / kBlock;
  const int32_t ch2 = (sh.cnt_in[2] + kBlock - 1) / kBlock;
  const int32_t light = ch0 + ch1 + ch2;
  for (uint32_t q = 0; q < count; ++q) {
    int32_t uu = static_cast<int32_t>(first + q);
    if (uu < light) {
      int bin = 0;
      if (uu >= ch0) {
        uu -= ch0;
        bin = 1;
        if (uu >= ch1) {
          uu -= ch1;
          bin = 2;
        }
      }
      const int32_t f = uu * kBlock;
      const int32_t cnt = min(kBlock, sh.cnt_in[bin] - f);
      const int32_t* wl = b.wl_in + sh.off[bin] + f;
      const int G = bin == 0 ? t.lanes[0] : (bin == 1 ? t.lanes[1] : t.lanes[2]);
      if (!detect) {
        switch (G) {
          case 1: color_chunk_group<MODE, 1, LD>(g, b, wl, cnt, work_acc); break;
          case 2: color_chunk_group<MODE, 2, LD>(g, b, wl, cnt, work_acc); break;
          case 4: color_chunk_group<MODE, 4, LD>(g, b, wl, cnt, work_acc); break;
          case 8: color_chunk_group<MODE, 8, LD>(g, b, wl, cnt, work_acc); break;
          case 16: color_chunk_group<MODE, 16, LD>(g, b, wl, cnt, work_acc); break;
          case 32: color_chunk_group<MODE, 32, LD>(g, b, wl, cnt, work_acc); break;
          default: color_chunk_group<MODE, 64, LD>(g, b, wl, cnt, work_acc); break;
        }
      } else {
        const int32_t oo = sh.off[bin];
        switch (G) {
          case 1: detect_chunk_group<MODE, 1, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
          case 2: detect_chunk_group<MODE, 2, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
          case 4: detect_chunk_group<MODE, 4, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
          case 8: detect_chunk_group<MODE, 8, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
          case 16: detect_chunk_group<MODE, 16, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
          case 32: detect_chunk_group<MODE, 32, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
          default: detect_chunk_group<MODE, 64, LD>(g, k, b, bin, wl, cnt, oo, sh.ent, sh.wc, maxc_acc); break;
        }
      }
    } else {
      const int32_t v = ld_dev(&b.wl_in[sh.off[3] + (uu - light)]);
      if (!detect) {
        color_vertex_block<MODE, LD>(g, b, v, sh.ovf, sh.red, &sh.misc[0]);
        if (threadIdx.x == 0) work_acc += static_cast<uint64_t>(ld_dev(&b.work[v]));
      } else {
        detect_vertex_block<MODE, LD>(g, k, b, v, sh.off[3], maxc_acc);
      }
    }
    __syncthreads();
  }
}

// Opens epoch e with U units, or parks the job there when its epoch budget
// is used up.
__device__ void open_phase(BatchJob* J, uint64_t* word, uint32_t e, uint32_t U, int32_t* retired) {
  atomic_reset_u32(&J->done);
  if (static_cast<int32_t>(e) >= ld_dev(&J->stop_epoch)) {
    st_dev(&J->parked_epoch, static_cast<int32_t>(e));
    st_dev(&J->parked_units, static_cast<int32_t>(U));
    st_dev(&J->status, static_cast<int32_t>(kJobParked));
    __threadfence();
    store_word(word, phase_word(e, 0, 0));
    atomicAdd(retired, 1);
    return;
  }
  __threadfence();
  store_word(word, phase_word(e, U, 0));
}

__device__ void finish_job(BatchJob* J, uint64_t* word, uint32_t e, int32_t rounds, int32_t rc,
                           int32_t* retired) {
  st_dev(&J->rounds, rounds);
  st_dev(&J->rc, rc);
  st_dev(&J->status, static_cast<int32_t>(kJobFinished));
  __threadfence();
  store_word(word, phase_word((e + 1) & 0xFFFFu, 0, 0));
  atomicAdd(retired, 1);
}

// The last unit of epoch e has completed: open the next phase.
__device__ void close_phase(BatchJob* J, int32_t n, int32_t max_rounds, uint64_t* word, uint32_t e, uint32_t U,
                            int32_t* retired) {
  if (e == 1) {
    int32_t o = 0;
    for (int b = 0; b < kBatchBins; ++b) {
      st_dev(&J->off[b], o);
      o += atomic_load_i32(&J->cnt_all[b]);
      atomic_reset_i32(&J->pos[b]);
    }
    st_dev(&J->off[kBatchBins], o);
    open_phase(J, word, 2, static_cast<uint32_t>((n + kBlock - 1) / kBlock), retired);
  } else if (e == 2) {
    int32_t c[kBatchBins];
    for (int b = 0; b < kBatchBins; ++b) {
      c[b] = atomic_load_i32(&J->cnt_all[b]);
      (void)atomicExch(&J->cnt[0][b], c[b]);
      atomic_reset_i32(&J->cnt[1][b]);
    }
    atomicAdd(&J->visits[0], static_cast<unsigned long long>(n));
    open_phase(J, word, 3, phase_units(c), retired);
  } else if (e & 1u) {
    open_phase(J, word, e + 1, U, retired);  // color step done: detect over the same worklist
  } else {
    const int32_t r = static_cast<int32_t>((e - 2) / 2);
    const int p = (r - 1) & 1;
    int32_t c[kBatchBins];
    int64_t total = 0;
    for (int b = 0; b < kBatchBins; ++b) {
      c[b] = atomic_load_i32(&J->cnt[p ^ 1][b]);
      total += c[b];
    }
    if (total == 0) {
      finish_job(J, word, e, r, COLOR_OK, retired);
    } else if (r >= max_rounds) {
      finish_job(J, word, e, r, COLOR_ENOCONVERGE, retired);
    } else {
      for (int b = 0; b < kBatchBins; ++b) atomic_reset_i32(&J->cnt[p][b]);
      atomicAdd(&J->visits[0], static_cast<unsigned long long>(total));
      open_phase(J, word, e + 1, phase_units(c), retired);
    }
  }
}

// Runs the owned units of one grab.
template <int MODE, int LD>
__device__ __forceinline__ void run_grab(BatchJob* J, const JobView& V, const BatchTune* tune, uint32_t e, uint32_t first,
                         uint32_t count, StepShared& sh, int32_t* s_bc, int32_t* s_base, uint64_t& work_acc,
                         int32_t& maxc_acc) {
  const BatchTune t = tune_of<LD>(V, tune);
  if (e == 1) {
    for (uint32_t q = 0; q < count; ++q) setup_a_unit<MODE, LD>(J, V, t, static_cast<int32_t>(first + q), s_bc);
  } else if (e == 2) {
    for (uint32_t q = 0; q < count; ++q) setup_b_unit(J, V, t, static_cast<int32_t>(first + q), s_bc, s_base);
  } else {
    const KeySource k{nullptr, nullptr, V.hs, nullptr};
    const bool detect = (e & 1u) == 0;
    const int r = static_cast<int>(detect ? (e - 2) / 2 : (e - 1) / 2);
    round_units<MODE, LD>(J, V, k, t, r, detect, first, count, sh, work_acc, maxc_acc);
  }
}

template <int LD>
__global__ __launch_bounds__(kBlock) void batch_kernel(BatchJob* jobs, uint64_t* words, int32_t num_jobs,
                                                       int32_t active, int32_t* retired, const BatchTune* tune) {
  __shared__ StepShared sh;
  __shared__ int32_t s_bc[kBatchBins * kWavesPerBlock];
  __shared__ int32_t s_base[kBatchBins];
  __shared__ int32_t s_job, s_exit;
  __shared__ uint32_t s_e, s_u, s_first, s_cnt;
  __shared__ unsigned long long s_work;
  __shared__ int32_t s_max;
  const int32_t lb = xcd_logical_block_of(gridDim.x, blockIdx.x);
  const int32_t home = static_cast<int32_t>(static_cast<int64_t>(lb) * num_jobs / gridDim.x);
  while (true) {
    if (threadIdx.x < kWave) {
      // wavefront 0: find an open phase and take units of it
      const int lane = lane_id();
      int32_t job = -1;
      uint32_t ge = 0, gu = 0, gf = 0, gc = 0;
      for (int32_t base = 0; base < num_jobs && job < 0; base += kWave) {
        const int32_t idx = base + lane;
        const bool valid = idx < num_jobs;
        int32_t j = home + idx;
        if (j >= num_jobs) j -= num_jobs;
        const uint64_t w = valid ? atomic_load_u64(&words[j]) : 0ull;
        uint64_t bal = __ballot(valid && w_grabbed(w) < w_units(w));
        while (bal) {
          const int l = __builtin_ctzll(bal);
          bal &= bal - 1ull;
          uint32_t ok = 0, e2 = 0, u2 = 0, g2 = 0, k = 0;
          if (lane == l) {
            k = min(16u, 1u + w_units(w) / (2u * gridDim.x));
            const uint64_t w2 = atomicAdd(reinterpret_cast<unsigned long long*>(&words[j]),
                                          static_cast<unsigned long long>(k));
            e2 = w_epoch(w2);
            u2 = w_units(w2);
            g2 = w_grabbed(w2);
            ok = g2 < u2 ? 1u : 0u;
          }
          ok = __shfl(ok, l, kWave);
          if (ok) {
            job = __shfl(j, l, kWave);
            ge = __shfl(e2, l, kWave);
            gu = __shfl(u2, l, kWave);
            gf = __shfl(g2, l, kWave);
            gc = min(__shfl(k, l, kWave), gu - gf);
            break;
          }
        }
      }
      if (lane == 0) {
        s_job = job;
        s_e = ge;
        s_u = gu;
        s_first = gf;
        s_cnt = gc;
        s_exit = job < 0 && atomic_load_i32(retired) >= active;
        s_work = 0ull;
        s_max = 0;
        if (job >= 0) __threadfence();
      }
    }
    __syncthreads();
    if (s_exit) break;
    const int32_t job = s_job;
    if (job < 0) {
      __builtin_amdgcn_s_sleep(16);
      __syncthreads();
      continue;
    }
    BatchJob* J = &jobs[job];
    const JobView V = load_job(J);
    const uint32_t e = s_e;
    uint64_t work_acc = 0;
    int32_t maxc_acc = 0;
    switch (V.mode) {
      case kD1: run_grab<kD1, LD>(J, V, tune, e, s_first, s_cnt, sh, s_bc, s_base, work_acc, maxc_acc); break;
      case kD2: run_grab<kD2, LD>(J, V, tune, e, s_first, s_cnt, sh, s_bc, s_base, work_acc, maxc_acc); break;
      default: run_grab<kPD2, LD>(J, V, tune, e, s_first, s_cnt, sh, s_bc, s_base, work_acc, maxc_acc); break;
    }
    work_acc = wave_sum_u64(work_acc);
    maxc_acc = wave_max_i32(maxc_acc);
    if (lane_id() == 0) {
      if (work_acc) atomicAdd(&s_work, static_cast<unsigned long long>(work_acc));
      if (maxc_acc > 0) atomicMax(&s_max, maxc_acc);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_work) atomicAdd(&J->visits[1], s_work);
      if (s_max > 0) atomicMax(&J->maxc, s_max);
      __threadfence();
      const uint32_t before = atomicAdd(&J->done, s_cnt);
      if (before + s_cnt == s_u) {
        __threadfence();
        close_phase(J, V.n, V.max_rounds, &words[job], e, s_u, retired);
      }
    }
    __syncthreads();
  }
}

__global__ void unpark_kernel(BatchJob* jobs, uint64_t* words, int32_t num_jobs, int32_t budget) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= num_jobs) return;
  BatchJob* J = &jobs[j];
  if (ld_dev(&J->status) != kJobParked) return;
  const int32_t e = ld_dev(&J->parked_epoch);
  st_dev(&J->stop_epoch, static_cast<int32_t>(min(static_cast<int64_t>(e) + budget, int64_t{0xFFFF})));
  st_dev(&J->status, static_cast<int32_t>(kJobRunning));
  atomic_reset_u32(&J->done);
  __threadfence();
  store_word(&words[j], phase_word(static_cast<uint32_t>(e), static_cast<uint32_t>(ld_dev(&J->parked_units)), 0));
}

// First-hop nnz of every job (row_ptr[n] of its hop-1 array).
__global__ void job_nnz_kernel(const BatchJob* jobs, int32_t num_jobs, int32_t* out) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= num_jobs) return;
  const BatchJob* J = &jobs[j];
  const int32_t n = ld_dev(&J->n);
  out[j] = n > 0 ? ld_dev(&ld_ptr(&J->rp)[n]) : 0;
}

int launch_batch(BatchJob* jobs, uint64_t* words, int32_t num_jobs, int32_t active, int32_t* retired,
                 const BatchTune* tune, int grid, bool coherent_graph, hipStream_t st) {
  if (coherent_graph)
    hipLaunchKernelGGL(batch_kernel<1>, dim3(grid), dim3(kBlock), 0, st, jobs, words, num_jobs, active, retired,
                       tune);
  else
    hipLaunchKernelGGL(batch_kernel<0>, dim3(grid), dim3(kBlock), 0, st, jobs, words, num_jobs, active, retired,
                       tune);
  return hipGetLastError() == hipSuccess ? COLOR_OK : COLOR_EHIP;
}

int launch_unpark(BatchJob* jobs, uint64_t* words, int32_t num_jobs, int32_t budget_epochs, hipStream_t st) {
  if (num_jobs <= 0) return COLOR_OK;
  hipLaunchKernelGGL(unpark_kernel, dim3((num_jobs + kBlock - 1) / kBlock), dim3(kBlock), 0, st, jobs, words,
                     num_jobs, budget_epochs);
  return hipGetLastError() == hipSuccess ? COLOR_OK : COLOR_EHIP;
}

int batch_resident_blocks() {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<1>, kBlock, 0) != hipSuccess)
    return 256;
  cached = std::max(8, std::max(1, per) * cus / 8 * 8);
  return cached;
}

void default_tune_table(BatchTune* t) {
  for (int m = 0; m < 3; ++m) {
    color_params p;
    default_params(m + 1, &p);
    for (int c = 0; c < kTuneClasses; ++c) {
      BatchTune& x = t[m * kTuneClasses + c];
      for (int i = 0; i < 3; ++i) {
        x.bin_hi[i] = p.bin_hi[i];
        x.lanes[i] = p.lanes[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// autotuner records (T1)
// ---------------------------------------------------------------------------

static std::mutex g_tune_mu;
static std::map<int, std::vector<BatchTune>> g_tune;   // device -> 3 x kTuneClasses
static thread_local const BatchTune* t_tune_override = nullptr;

void tune_table_for_device(BatchTune* t) {
  const size_t bytes = sizeof(BatchTune) * 3 * kTuneClasses;
  if (t_tune_override) {
    std::memcpy(t, t_tune_override, bytes);
    return;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(dev);
  if (it != g_tune.end()) std::memcpy(t, it->second.data(), bytes);
  else default_tune_table(t);
}

// ---------------------------------------------------------------------------
// host side of color_batch
// ---------------------------------------------------------------------------

struct BatchWorkspace {
  std::mutex mu;
  DevBuf table, words, ctr, tune, arrays, nnz;
  BatchJob* host = nullptr;  // pinned staging of the job table
  size_t host_cap = 0;
  ~BatchWorkspace() {
    for (DevBuf* b : {&table, &words, &ctr, &tune, &arrays, &nnz}) b->release();
    if (host) (void)hipHostFree(host);
  }
};

static std::mutex g_bws_mu;
static std::map<int, BatchWorkspace*> g_bws;

static BatchWorkspace* batch_workspace(int* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = COLOR_EHIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_bws_mu);
  auto it = g_bws.find(dev);
  if (it != g_bws.end()) return it->second;
  BatchWorkspace* w = new BatchWorkspace();
  g_bws[dev] = w;
  return w;
}

void release_batch_workspaces() {
  std::lock_guard<std::mutex> lk(g_bws_mu);
  for (auto& kv : g_bws) delete kv.second;
  g_bws.clear();
}

// int32 entries per array of a job, rounded up to 256 bytes.
int64_t batch_stride(int32_t n) { return (static_cast<int64_t>(std::max(n, 1)) + 63) / 64 * 64; }

int check_job(const color_job& j) {
  if (j.kind < COLOR_KIND_D1 || j.kind > COLOR_KIND_PD2) return COLOR_EINVAL;
  if (j.n < 0 || j.n_rows < 0) return COLOR_EINVAL;
  if (j.n > kBatchMaxN) return COLOR_EOVERFLOW;
  if (j.n > 0 && (!j.row_ptr || !j.col_idx || !j.colors)) return COLOR_EINVAL;
  if (j.kind == COLOR_KIND_PD2 && j.n > 0 && (!j.col_ptr || !j.row_idx)) return COLOR_EINVAL;
  return COLOR_OK;
}

// The job record of a job (static fields; arrays carved from `base`).
void fill_job(const color_job& j, int32_t max_rounds, int32_t* base, BatchJob* out) {
  std::memset(out, 0, sizeof(*out));
  out->mode = j.kind;
  out->n = j.n;
  out->hs = hash_seed(j.seed);
  out->max_rounds = max_rounds;
  if (j.kind == COLOR_KIND_PD2) {  // hop 1 column -> rows, hop 2 row -> columns
    out->rp = j.col_ptr;
    out->ci = j.row_idx;
    out->rp2 = j.row_ptr;
    out->ci2 = j.col_idx;
  } else {
    out->rp = out->rp2 = j.row_ptr;
    out->ci = out->ci2 = j.col_idx;
  }
  out->C = j.colors;
  const size_t n = static_cast<size_t>(batch_stride(j.n));
  out->T = base;
  out->work = base + n;
  out->wl0 = base + 2 * n;
  out->wl1 = base + 3 * n;
  out->stop_epoch = INT_MAX;
  out->status = j.n > 0 ? kJobRunning : kJobFinished;
}

uint64_t initial_word(int32_t n) {
  return n > 0 ? phase_word(1, static_cast<uint32_t>((n + kBlock - 1) / kBlock), 0) : 0ull;
}

void job_stats(const BatchJob& J, color_stats* st) {
  st->num_colors = J.maxc;
  st->rounds = J.rounds;
  st->vertex_visits = static_cast<int64_t>(J.visits[0]);
  st->edge_visits = static_cast<int64_t>(J.visits[1]);
  st->boundary_conflicts = 0;
  st->remote_losers = 0;
  st->kernel_launches = 1;
  st->color_kernel_ns = 0;
  st->detect_kernel_ns = 0;
  st->color_launches = 0;
  st->detect_launches = 0;
  st->engine = COLOR_ENGINE_BATCH;
  st->tail_rounds = 0;
  st->tail_kernel_ns = 0;
  st->tail_bytes = 0;
  st->list_visits = 0;
  st->pushes = 0;
  st->color_bytes = 0;
  st->detect_bytes = 0;
}

// Two-hop walk per visit that makes a job better served by the single-graph
// incremental engine than by the persistent kernel's pull steps (the same
// bound as the single-graph engine choice).
constexpr double kLongWalk = 128.0;

// A job's average two-hop walk, from its sizes: D2 deg (deg + 1), PD2
// (column degree)(1 + row degree), with average degrees (a lower bound of
// the true average, by convexity).  D1: 0.
double estimated_walk(const color_job& j, int32_t nnz) {
  if (j.kind == COLOR_KIND_D1 || j.n <= 0) return 0.0;
  const double d = static_cast<double>(nnz) / j.n;
  if (j.kind == COLOR_KIND_D2) return d * (d + 1.0);
  return d * (1.0 + static_cast<double>(nnz) / std::max(j.n_rows, 1));
}

int run_batch(int32_t num_jobs, const color_job* jobs, color_stats* per_job, const color_params* params,
                     void* stream, bool route_long_walks) {
  if (num_jobs < 0 || (num_jobs > 0 && !jobs)) return COLOR_EINVAL;
  int e = COLOR_OK;
  for (int i = 0; i < num_jobs; ++i)
    if ((e = check_job(jobs[i]))) return e;
  if (params && (params->max_rounds < 0 || params->max_workgroups < 0)) return COLOR_EINVAL;
  const int32_t max_rounds = (params && params->max_rounds > 0) ? std::min(params->max_rounds, kBatchMaxRounds)
                                                                : kBatchMaxRounds;
  if (params && (params->flags & COLOR_FLAG_VALIDATE)) {
    for (int i = 0; i < num_jobs; ++i)
      if ((e = validate_job(jobs[i], stream))) return e;
  }
  if (num_jobs == 0) return COLOR_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  BatchWorkspace* w = batch_workspace(&e);
  if (!w) return e;
  std::vector<int> routed;  // jobs for the single-graph engine
  {
    std::lock_guard<std::mutex> lk(w->mu);
    int64_t total = 0;
    bool two_hop = false;
    for (int i = 0; i < num_jobs; ++i) {
      total += 4 * batch_stride(jobs[i].n);
      two_hop = two_hop || (jobs[i].kind != COLOR_KIND_D1 && jobs[i].n > 0);
    }
    const size_t nj = static_cast<size_t>(num_jobs);
    if ((e = w->arrays.ensure(sizeof(int32_t) * static_cast<size_t>(total), false, st))) return e;
    if ((e = w->table.ensure(sizeof(BatchJob) * nj, false, st))) return e;
    if ((e = w->words.ensure(sizeof(uint64_t) * nj, false, st))) return e;
    if ((e = w->nnz.ensure(sizeof(int32_t) * nj, false, st))) return e;
    if ((e = w->ctr.ensure(256, false, st))) return e;
    if ((e = w->tune.ensure(sizeof(BatchTune) * 3 * kTuneClasses, false, st))) return e;
    const size_t host_bytes = sizeof(BatchJob) * nj + sizeof(uint64_t) * nj + sizeof(int32_t) * nj +
                              sizeof(BatchTune) * 3 * kTuneClasses;
    if (w->host_cap < host_bytes) {
      if (w->host) (void)hipHostFree(w->host);
      w->host = nullptr;
      w->host_cap = 0;
      if (hipHostMalloc(reinterpret_cast<void**>(&w->host), host_bytes, hipHostMallocDefault) != hipSuccess)
        return COLOR_ENOMEM;
      w->host_cap = host_bytes;
    }
    BatchJob* hj = w->host;
    uint64_t* hw = reinterpret_cast<uint64_t*>(hj + nj);
    int32_t* hn = reinterpret_cast<int32_t*>(hw + nj);
    BatchTune* ht = reinterpret_cast<BatchTune*>(hn + nj);
    int32_t* base = w->arrays.as<int32_t>();
    for (int i = 0; i < num_jobs; ++i) {
      fill_job(jobs[i], max_rounds, base, &hj[i]);
      base += 4 * batch_stride(jobs[i].n);
      hw[i] = initial_word(jobs[i].n);
    }
    tune_table_for_device(ht);
    if (hipMemcpyAsync(w->table.p, hj, sizeof(BatchJob) * nj, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w->tune.p, ht, sizeof(BatchTune) * 3 * kTuneClasses, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemsetAsync(w->ctr.p, 0, 256, st) != hipSuccess)
      return COLOR_EHIP;
    if (route_long_walks && two_hop) {
      hipLaunchKernelGGL(job_nnz_kernel, dim3((num_jobs + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                         w->table.as<BatchJob>(), num_jobs, w->nnz.as<int32_t>());
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(hn, w->nnz.p, sizeof(int32_t) * nj, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return COLOR_EHIP;
      for (int i = 0; i < num_jobs; ++i) {
        if (estimated_walk(jobs[i], hn[i]) >= kLongWalk) {
          routed.push_back(i);
          hw[i] = 0;  // no open phase: the persistent kernel never takes it
        }
      }
    }
    int32_t active = 0;
    int64_t units0 = 0;
    for (int i = 0; i < num_jobs; ++i) {
      if (hw[i] != 0) {
        ++active;
        units0 += (jobs[i].n + kBlock - 1) / kBlock;
      }
    }
    if (hipMemcpyAsync(w->words.p, hw, sizeof(uint64_t) * nj, hipMemcpyHostToDevice, st) != hipSuccess)
      return COLOR_EHIP;
    if (active > 0) {
      int grid = batch_resident_blocks();
      if (params && params->max_workgroups > 0) grid = std::min(grid, params->max_workgroups);
      grid = static_cast<int>(std::min<int64_t>(grid, std::max<int64_t>(8, (units0 + 7) / 8 * 8)));
      if ((e = launch_batch(w->table.as<BatchJob>(), w->words.as<uint64_t>(), num_jobs, active,
                            w->ctr.as<int32_t>(), w->tune.as<BatchTune>(), grid, false, st)))
        return e;
    }
    if (hipMemcpyAsync(hj, w->table.p, sizeof(BatchJob) * nj, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return COLOR_EHIP;
    int rc = COLOR_OK;
    for (int i = 0; i < num_jobs; ++i) {
      if (hw[i] == 0 && jobs[i].n > 0) continue;  // routed
      if (per_job) job_stats(hj[i], &per_job[i]);
      if (rc == COLOR_OK && hj[i].status == kJobFinished && hj[i].rc != COLOR_OK) rc = hj[i].rc;
    }
    if (rc != COLOR_OK) return rc;
  }
  // jobs with long two-hop walks: the single-graph calls (their engine choice
  // takes the incremental engine for them)
  for (int i : routed) {
    const color_job& j = jobs[i];
    color_stats* sp = per_job ? &per_job[i] : nullptr;
    if (j.kind == COLOR_KIND_D2)
      e = color_d2(j.n, j.row_ptr, j.col_idx, j.seed, nullptr, nullptr, j.colors, sp, params, stream);
    else
      e = color_pd2(j.n_rows, j.n, j.row_ptr, j.col_idx, j.col_ptr, j.row_idx, j.seed, nullptr, nullptr, j.colors,
                    sp, params, stream);
    if (e) return e;
  }
  return COLOR_OK;
}

}  // namespace gcol

extern "C" int color_batch(int32_t num_jobs, const color_job* jobs, color_stats* per_job,
                           const color_params* params, void* stream) {
  // jobs carry no degree option: the batched engine keys by (p, gid) only
  if (params && (params->flags & COLOR_FLAG_RECOLOR_DEGREES)) return COLOR_EINVAL;
  return gcol::run_batch(num_jobs, jobs, per_job, params, stream, true);
}

using namespace gcol;

namespace {

// One candidate of the autotuner: lanes of bins 0..2 and the default bounds
// scaled by 2^shift.
struct Candidate {
  int32_t lanes[3];
  int shift;
};

int read_i32(const int32_t* dev_ptr, int32_t* out, hipStream_t st) {
  if (hipMemcpyAsync(out, dev_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return COLOR_EHIP;
  return COLOR_OK;
}

}  // namespace

extern "C" int color_autotune(const color_job* job, int32_t reps, color_params* best, void* stream) {
  if (!job || reps < 1) return COLOR_EINVAL;
  int e = check_job(*job);
  if (e) return e;
  if (job->n == 0) return COLOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int mode = job->kind;
  int32_t nnz = 0;
  if ((e = read_i32((mode == COLOR_KIND_PD2 ? job->col_ptr : job->row_ptr) + job->n, &nnz, st))) return e;
  const int64_t avg = nnz / std::max(job->n, 1);
  int cls = 0;
  while (cls + 1 < kTuneClasses && (int64_t{2} << cls) <= avg) ++cls;

  std::vector<BatchTune> table(3 * kTuneClasses);
  tune_table_for_device(table.data());
  color_params defaults;
  default_params(mode, &defaults);
  static const Candidate cands[] = {
      {{4, 16, 64}, 0}, {{1, 4, 32}, 0}, {{2, 8, 64}, 0}, {{8, 32, 64}, 0}, {{16, 64, 64}, 0},
      {{4, 16, 64}, -2}, {{4, 16, 64}, 2}, {{2, 8, 64}, -2}, {{8, 32, 64}, 2},
  };
  std::vector<int32_t> ref(static_cast<size_t>(job->n)), got(static_cast<size_t>(job->n));
  double best_t = 1e300;
  BatchTune best_rec{};
  bool first = true;
  for (const Candidate& c : cands) {
    BatchTune rec;
    for (int i = 0; i < 3; ++i) {
      rec.lanes[i] = c.lanes[i];
      const int64_t b = c.shift >= 0 ? int64_t{defaults.bin_hi[i]} << c.shift : defaults.bin_hi[i] >> -c.shift;
      rec.bin_hi[i] = static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(b, i + 1), INT_MAX / 2));
    }
    std::vector<BatchTune> trial(table);
    for (int k = 0; k < kTuneClasses; ++k) trial[(mode - 1) * kTuneClasses + k] = rec;
    t_tune_override = trial.data();
    double t_min = 1e300;
    for (int r = 0; r < reps && e == COLOR_OK; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      e = run_batch(1, job, nullptr, nullptr, stream, false);
      const auto t1 = std::chrono::steady_clock::now();
      t_min = std::min(t_min, std::chrono::duration<double>(t1 - t0).count());
    }
    t_tune_override = nullptr;
    if (e) return e;
    std::vector<int32_t>& dst = first ? ref : got;
    if (hipMemcpyAsync(dst.data(), job->colors, sizeof(int32_t) * dst.size(), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return COLOR_EHIP;
    if (!first && got != ref) return COLOR_EMISMATCH;
    first = false;
    if (t_min < best_t) {
      best_t = t_min;
      best_rec = rec;
    }
  }
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COLOR_EHIP;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::vector<BatchTune>& t = g_tune[dev];
    if (t.empty()) {
      t.resize(3 * kTuneClasses);
      default_tune_table(t.data());
    }
    t[(mode - 1) * kTuneClasses + cls] = best_rec;
  }
  if (best) {
    std::memset(best, 0, sizeof(*best));
    for (int i = 0; i < 3; ++i) {
      best->bin_hi[i] = best_rec.bin_hi[i];
      best->lanes[i] = best_rec.lanes[i];
    }
    best->bin_hi[3] = INT_MAX;
  }
  return COLOR_OK;
}

extern "C" int color_autotune_reset(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return COLOR_EHIP;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.erase(dev);
  return COLOR_OK;
}
