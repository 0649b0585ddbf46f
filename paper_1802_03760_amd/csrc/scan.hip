// Exclusive prefix sums (reduce, scan of block sums, downsweep).
#include "gj_internal.h"
#include "prim.h"

namespace gj {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(const Tin* __restrict__ in, uint64_t n,
                                                        Tout* __restrict__ part) {
  uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    if (idx < n) s += (uint64_t)in[idx];
  }
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) part[blockIdx.x] = (Tout)s;
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlock) k_scan_down(const Tin* __restrict__ in, uint64_t n,
                                                      const Tout* __restrict__ part_off,
                                                      Tout* __restrict__ out) {
  __shared__ Tout tile[kScanTile];
  uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    tile[i * kBlock + threadIdx.x] = idx < n ? (Tout)in[idx] : (Tout)0;
  }
  __syncthreads();
  Tout loc[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    loc[i] = tile[threadIdx.x * kScanItems + i];
    s += loc[i];
  }
  Tout total;
  Tout run = block_excl_scan<kBlock, Tout>(s, total) + (part_off ? part_off[blockIdx.x] : (Tout)0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    tile[threadIdx.x * kScanItems + i] = run;
    run += loc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    if (idx < n) out[idx] = tile[i * kBlock + threadIdx.x];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = run;
}

template <typename Tin, typename Tout>
static void scan_impl(gj_ctx* c, const Tin* in, Tout* out, uint64_t n, int level) {
  if (n == 0) {
    GJ_HIP(hipMemsetAsync(out, 0, sizeof(Tout), c->stream));
    return;
  }
  uint64_t nb = (n + kScanTile - 1) / kScanTile;
  GJ_CHECK(nb < (1ull << 31), GJ_EUNSUPPORTED, "scan too large");
  Tout* off = nullptr;  // one tile: no tile offsets
  if (nb > 1) {
    off = (Tout*)ws_get(c, "scan_off" + std::to_string(level), (nb + 1) * sizeof(Tout));
    Tout* part = (Tout*)ws_get(c, "scan_part" + std::to_string(level), nb * sizeof(Tout));
    k_scan_reduce<Tin, Tout><<<(unsigned)nb, kBlock, 0, c->stream>>>(in, n, part);
    scan_impl<Tout, Tout>(c, part, off, nb, level + 1);
  }
  k_scan_down<Tin, Tout><<<(unsigned)nb, kBlock, 0, c->stream>>>(in, n, off, out);
  GJ_HIP(hipGetLastError());
}

// The level buffers of a scan of n items (u64 tile sums, the widest any
// scan here takes), as scan_impl names them.
uint64_t scan_scratch_bytes(uint64_t n) {
  uint64_t t = 0;
  for (int level = 0; n > 0; ++level) {
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) break;
    t += ((nb + 1) * sizeof(uint64_t) + kArenaAlign - 1) & ~(kArenaAlign - 1);
    t += (nb * sizeof(uint64_t) + kArenaAlign - 1) & ~(kArenaAlign - 1);
    n = nb;
  }
  return t;
}

void scan_reserve(gj_ctx* c, uint64_t n) {
  for (int level = 0; n > 0; ++level) {
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) break;
    ws_get(c, "scan_off" + std::to_string(level), (nb + 1) * sizeof(uint64_t));
    ws_get(c, "scan_part" + std::to_string(level), nb * sizeof(uint64_t));
    n = nb;
  }
}

void scan_u32_to_u64(gj_ctx* c, const uint32_t* in, uint64_t* out, uint64_t n) {
  scan_impl<uint32_t, uint64_t>(c, in, out, n, 0);
}
void scan_u64(gj_ctx* c, const uint64_t* in, uint64_t* out, uint64_t n) {
  scan_impl<uint64_t, uint64_t>(c, in, out, n, 0);
}
void scan_u32(gj_ctx* c, const uint32_t* in, uint32_t* out, uint64_t n) {
  scan_impl<uint32_t, uint32_t>(c, in, out, n, 0);
}

}  // namespace gj
