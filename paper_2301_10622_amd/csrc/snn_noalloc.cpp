// The allocation-free batch search: the device-buffer batch search with its
// workspace (prepared query entries, per-query thresholds and counters, the
// work queues and the tile candidates) in one fixed array of device memory
// that lives as long as the process, instead of buffers the index allocates.
//
// `scratch` below is a device variable. Its name, used in host code, is a
// host-side stand-in and not a device address; the address each device holds
// it at is looked up once per device with hipGetSymbolAddress and kept, and
// only that pointer is ever handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "snn.h"
#include "snn_host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // SNN_NOALLOC_SCRATCH_BYTES in snn.h
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
char *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (current), looked up on the
// first call for that device.
snn_status scratch_on(snn_index *ix, int dev, char **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return ix->hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch[dev] = (char *)ptr;
  }
  *out = g_scratch[dev];
  return SNN_OK;
}

}  // namespace

extern "C" snn_status snn_search_batch_dev_noalloc(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                                   const uint32_t *coords, const float *vals, uint32_t k,
                                                   uint32_t mode, uint32_t *out_ids, float *out_scores,
                                                   uint32_t *out_counts, void *stream) {
  if (!ix) return SNN_E_INVALID;
  static_assert(kScratchBytes == SNN_NOALLOC_SCRATCH_BYTES, "snn.h states the scratch size");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return ix->hip_fail(e, "current device");
  if (dev != ix->device)
    return ix->fail(SNN_E_INVALID, "search: device %d is current, the index lives on device %d", dev, ix->device);
  if (dev < 0 || dev >= kMaxDevices) return ix->fail(SNN_E_INVALID, "search: device %d out of range", dev);
  char *ws = nullptr;
  snn_status st = scratch_on(ix, dev, &ws);
  if (st != SNN_OK) return st;
  return snn_search_dev_in_region(ix, nq, indptr, total, coords, vals, k, mode, out_ids, out_scores, out_counts,
                                  stream, ws, kScratchBytes);
}
