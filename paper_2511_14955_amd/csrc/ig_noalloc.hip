// Featurize without allocating device memory (ig_featurize_noalloc).
//
// The entry point computes exactly what ig_featurize computes (Figure 1's Boolean rows) with the
// same kernels, but every device buffer beyond the caller's inputs and outputs (the staged batch,
// its chunk list, the per-sequence rank bitmaps, the row counts and offsets, and the CSR entries
// before their copy to the host) is carved from `scratch`, a fixed device array the library holds
// for the life of the process.  It calls no hipMalloc / hipFree.
//
// `scratch` is a file-scope __device__ array, so every GPU the library runs on holds its own copy
// at its own address.  Host code never passes the array's name to a kernel or a copy (in host code
// that name is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device when a context is created on it (noalloc_setup) and
// kept in g_scratch[].
//
// Calls share the device's copy; a per-device mutex serializes them within the process, so calls
// from several threads (or contexts) on one GPU wait for each other instead of racing.  Each call
// clears what must start at zero (the bitmaps and the data tail) with fill kernels, and the
// previous call's contents are otherwise left in place.
#include <mutex>

#include "ig_internal.h"

namespace ig {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)IG_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_setup_mu;
static void *g_scratch[NOALLOC_MAX_DEVICES];          // device address of `scratch`, per device
static std::mutex g_call_mu[NOALLOC_MAX_DEVICES];     // one no-allocation call per device at a time

// Called by ig_create with the context's device current.
int noalloc_setup(ig_ctx *c) {
  const int dev = c->cfg.device;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return IG_OK;   // the entry point refuses such devices
  std::lock_guard<std::mutex> lk(g_setup_mu);
  if (g_scratch[dev]) return IG_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return set_error(c, IG_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  }
  g_scratch[dev] = p;
  return IG_OK;
}

}  // namespace ig

using namespace ig;

extern "C" int ig_featurize_noalloc(ig_ctx *c, const void *data, uint64_t data_bytes, const uint64_t *sym_offsets,
                                    uint64_t m, uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out) {
  if (!c) return IG_EINVAL;
  const int dev = c->cfg.device;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES || !g_scratch[dev])
    return set_error(c, IG_EDEVICE, "no-allocation scratch not set up on device %d", dev);
  std::lock_guard<std::mutex> lk(g_call_mu[dev]);
  Carve a;
  a.base = reinterpret_cast<uint8_t *>(g_scratch[dev]);
  a.size = NOALLOC_SCRATCH_BYTES;
  return featurize_host(c, data, data_bytes, sym_offsets, m, indptr, indices, cap, nnz_out, &a);
}
