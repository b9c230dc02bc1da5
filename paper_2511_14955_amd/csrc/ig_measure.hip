// Attainable HBM read bandwidth of a plain streaming kernel on this device: the context for the
// scan's roofline (its input is read once per pass).  Not on the method's path.
#include "ig_internal.h"

namespace ig {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Every 16-byte element is read once (non-temporal, four loads in flight per thread); the XOR
// of the words goes to one slot per workgroup so that the loads are not removed.
__global__ void __launch_bounds__(256) k_stream_read(const u32x4_t *src, uint64_t n16, uint32_t *sink) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const u32x4_t a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + stride),
                  c = __builtin_nontemporal_load(src + i + 2 * stride), d = __builtin_nontemporal_load(src + i + 3 * stride);
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n16; i += stride) {
    const u32x4_t a = __builtin_nontemporal_load(src + i);
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  atomicXor(&s, acc);
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = s;
}

}  // namespace ig

using namespace ig;

extern "C" int ig_measure_read_bw(ig_ctx *c, uint64_t bytes, uint32_t reps, double *gb_per_s) {
  if (!c || !gb_per_s || bytes < 16 || reps == 0) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (hipSetDevice(c->cfg.device) != hipSuccess) return set_error(c, IG_EDEVICE, "hipSetDevice");
  const uint64_t n16 = bytes / 16;
  const uint32_t grid = (uint32_t)c->n_cu * 8;
  DevBuf buf, sink;
  if (dev_reserve(c, buf, n16 * 16) || dev_reserve(c, sink, (uint64_t)grid * 4)) {
    dev_release(c, buf);
    dev_release(c, sink);
    return IG_ENOMEM;
  }
  hipStream_t s = c->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(buf.p), n16 * 4, 0x9E3779B9u, s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const u32x4_t *src = reinterpret_cast<const u32x4_t *>(buf.p);
  uint32_t *out = reinterpret_cast<uint32_t *>(sink.p);
  if (e == hipSuccess) {   // one untimed launch, then reps timed ones
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, s, src, n16, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (uint32_t r = 0; r < reps && e == hipSuccess; r++) {
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, s, src, n16, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dev_release(c, buf);
  dev_release(c, sink);
  if (check_hip(c, e, "read bandwidth")) return IG_EDEVICE;
  *gb_per_s = (double)n16 * 16.0 * reps / (ms * 1e-3) / 1e9;
  return IG_OK;
}
