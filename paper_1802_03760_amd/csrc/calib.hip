// Bandwidth calibration of the device the library runs on, for reporting
// kernels against measured peaks beside the published ones: a device-to-device
// copy (HBM read + write through 16-byte vector loads and stores, grid-stride
// over 2 x 2 GiB) and an LDS read loop (every lane reads 16 bytes per step at
// conflict-free addresses from a 64 KiB table, 1024-thread workgroups, two
// per CU).  Each is timed with HIP events over several launches after a
// warm-up; the best launch is kept.
#include <functional>

#include "gj_internal.h"
#include "prim.h"

namespace gj {

__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ a, uint4* __restrict__ b, uint64_t n) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) b[i] = a[i];
}

constexpr int kLdsNT = 1024;
constexpr int kLdsWords = 16384;  // 64 KiB of u32

// Lane l of step s reads the 16-byte word (l + 64 * (w + s)) mod (words / 4)
// with w the wave index: the 64 lanes of a wave cover 1 KiB of consecutive
// addresses (no bank conflict).  The xor of what was read is stored so that
// the loop is not removed.
__global__ void __launch_bounds__(kLdsNT) k_lds_read(int steps, uint32_t* __restrict__ sink) {
  __shared__ uint4 t[kLdsWords / 4];
  for (int i = threadIdx.x; i < kLdsWords / 4; i += kLdsNT)
    t[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = 0;
  int idx = (lane + 64 * w) & (kLdsWords / 4 - 1);
  for (int s = 0; s < steps; ++s) {
    uint4 v = t[idx];
    x ^= v.x ^ v.y ^ v.z ^ v.w;
    idx = (idx + 64) & (kLdsWords / 4 - 1);
  }
  if (x == 0x9e3779b9u) sink[blockIdx.x * kLdsNT + threadIdx.x] = x;  // practically never taken
}

static double best_ms(gj_ctx* c, int reps, const std::function<void()>& launch) {
  hipEvent_t a, b;
  GJ_HIP(hipEventCreate(&a));
  GJ_HIP(hipEventCreate(&b));
  launch();  // warm-up
  double best = 1e30;
  for (int r = 0; r < reps; ++r) {
    GJ_HIP(hipEventRecord(a, c->stream));
    launch();
    GJ_HIP(hipEventRecord(b, c->stream));
    GJ_HIP(hipEventSynchronize(b));
    float ms = 0;
    GJ_HIP(hipEventElapsedTime(&ms, a, b));
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

}  // namespace gj

extern "C" gj_status gj_measure_peaks(gj_ctx* c, double* copy_gbs, double* lds_gbs) {
  if (!c) return GJ_EINVAL;
  try {
    GJ_HIP(hipSetDevice(c->device));
    if (copy_gbs) {
      const uint64_t bytes = 2ull << 30;
      gj::DevMem a(c, bytes), b(c, bytes);
      GJ_HIP(hipMemsetAsync(a.get(), 1, bytes, c->stream));
      uint64_t n = bytes / sizeof(uint4);
      unsigned grid = (unsigned)c->num_cus * 8;
      double ms = gj::best_ms(c, 5, [&] {
        gj::k_copy16<<<grid, 256, 0, c->stream>>>(a.as<const uint4>(), b.as<uint4>(), n);
      });
      GJ_HIP(hipGetLastError());
      *copy_gbs = 2.0 * bytes / (ms * 1e-3) / 1e9;
    }
    if (lds_gbs) {
      const int steps = 1 << 14;
      unsigned grid = (unsigned)c->num_cus * 2;
      gj::DevMem sink(c, (uint64_t)grid * gj::kLdsNT * sizeof(uint32_t));
      double ms = gj::best_ms(c, 5, [&] { gj::k_lds_read<<<grid, gj::kLdsNT, 0, c->stream>>>(steps, sink.as<uint32_t>()); });
      GJ_HIP(hipGetLastError());
      *lds_gbs = (double)grid * gj::kLdsNT * steps * 16.0 / (ms * 1e-3) / 1e9;
    }
    GJ_HIP(hipStreamSynchronize(c->stream));
    c->err.clear();
    return GJ_OK;
  } catch (const gj::Error& e) {
    c->err = e.msg;
    return e.code;
  }
}
