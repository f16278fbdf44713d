// color_d1_noalloc: color_d1 for callers that cannot allocate memory.
//
// Every call runs the single-graph pull engine of color_d1 (same kernels,
// same coloring) on a workspace whose buffers are regions of one file-scope
// device array, `scratch`, sized for graphs of up to COLOR_NOALLOC_MAX_N
// vertices.  Host code never passes the array's name to a kernel or a copy:
// it takes the array's device address once per device with
// hipGetSymbolAddress (each device holds its own copy) and uses that
// address.  The workspace's buffers are marked fixed, so that a request for
// more memory than a region holds fails with COLOR_EOVERFLOW instead of
// allocating.  The only memory the path clears (the per-call scalars) is
// cleared by a fill kernel at the start of every call; the other regions are
// fully written before they are read.
#include <climits>
#include <cstring>
#include <mutex>
#include <new>

#include "api_internal.hpp"

namespace gcol {
namespace {

constexpr int32_t kMaxN = COLOR_NOALLOC_MAX_N;
constexpr int32_t kMaxTrace = 4096;
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kSmallBytes = align256(sizeof(Scalars));
constexpr size_t kVecBytes = align256(sizeof(int32_t) * static_cast<size_t>(kMaxN));
constexpr size_t kBinBytes = align256(static_cast<size_t>(kMaxN));
constexpr size_t kTraceBytes = align256(sizeof(int32_t) * static_cast<size_t>(kMaxTrace));
// scalars, T, work, bin, two worklists, worklist trace: about 17 MiB
constexpr size_t kScratchBytes = kSmallBytes + 4 * kVecBytes + kBinBytes + kTraceBytes;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
  bool ready = false;
  unsigned char* ptr = nullptr;  // this device's copy of `scratch` (device address)
  Workspace* ws = nullptr;       // constructed in ws_mem, never destroyed
  alignas(Workspace) unsigned char ws_mem[sizeof(Workspace)];
  Scalars host;                  // read-back staging in host memory
};

std::mutex g_mu;
NoAllocDevice g_dev[kMaxDevices];

// Set-up on the device's first call, with that device current.
int device_workspace(Workspace** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return COLOR_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return COLOR_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  NoAllocDevice& d = g_dev[dev];
  if (!d.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return COLOR_EHIP;
    }
    d.ptr = static_cast<unsigned char*>(p);
    Workspace* w = new (d.ws_mem) Workspace();
    w->device = dev;
    for (DevBuf* b : w->buffers()) b->fixed = true;
    size_t off = 0;
    auto take = [&](DevBuf& b, size_t bytes) {
      b.p = d.ptr + off;
      b.bytes = bytes;
      off += bytes;
    };
    take(w->small, kSmallBytes);
    take(w->T, kVecBytes);
    take(w->work, kVecBytes);
    take(w->bin, kBinBytes);
    take(w->wl0, kVecBytes);
    take(w->wl1, kVecBytes);
    take(w->trace, kTraceBytes);
    w->host = &d.host;
    d.ws = w;
    d.ready = true;
  }
  *out = d.ws;
  return COLOR_OK;
}

}  // namespace
}  // namespace gcol

using namespace gcol;

extern "C" int color_d1_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
                                const uint32_t* prio, const int32_t* init_colors, int32_t* colors,
                                color_stats* stats, const color_params* params, void* stream) {
  if (n < 0) return COLOR_EINVAL;
  if (n > kMaxN) return COLOR_ESCRATCH;
  if (params && (params->flags & (COLOR_FLAG_KERNEL_TIMING | COLOR_FLAG_RECOLOR_DEGREES))) return COLOR_EINVAL;
  if (params && params->engine == COLOR_ENGINE_INCREMENTAL) return COLOR_EINVAL;
  if (stats && stats->worklist_trace && stats->trace_cap > kMaxTrace) return COLOR_EINVAL;
  Workspace* w = nullptr;
  const int e = device_workspace(&w);
  if (e) return e;
  // the pull engine with workgroup-wide heavy vertices: the layout whose
  // buffers the scratch array holds
  color_params p;
  if (params) p = *params;
  else std::memset(&p, 0, sizeof(p));
  p.engine = COLOR_ENGINE_PULL;
  p.bin_hi[3] = INT_MAX;
  return color_d1_fixed(w, n, row_ptr, col_idx, seed, prio, init_colors, colors, stats, &p, stream);
}
