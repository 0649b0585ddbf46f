// Stable LSD radix sort, 8-bit digits.  Each pass: per-tile digit histogram,
// exclusive scan of the digit-major histogram, stable scatter (ranks within a
// wave from eight ballots, across waves and items through LDS counters).
#include "gj_internal.h"
#include "prim.h"

namespace gj {

constexpr int kSortItems = 8;
constexpr int kSortTile = kBlock * kSortItems;
constexpr int kRadix = 256;

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
  return (uint32_t)(k >> shift) & 0xFFu;
}

template <typename K>
__global__ void __launch_bounds__(kBlock) k_hist(const K* __restrict__ keys, uint64_t n, int shift,
                                                 uint32_t* __restrict__ hist, uint32_t ntiles) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t base = (uint64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    if (idx < n) atomicAdd(&h[digit_of(keys[idx], shift)], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <typename K, bool VAL>
__global__ void __launch_bounds__(kBlock) k_scatter(const K* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                    uint64_t n, int shift,
                                                    const uint32_t* __restrict__ hist_off, uint32_t ntiles,
                                                    K* __restrict__ okeys, uint32_t* __restrict__ ovals) {
  __shared__ uint32_t base_cnt[kRadix];        // running count per digit in this tile
  __shared__ uint32_t wcnt[kBlock / 64][kRadix];
  const int lane = lane_id(), wave = wave_id();
  base_cnt[threadIdx.x] = hist_off[(uint64_t)threadIdx.x * ntiles + blockIdx.x];
  uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int i = 0; i < kSortItems; ++i) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
    bool valid = idx < n;
    K k = valid ? keys[idx] : (K)0;
    uint32_t v = 0;
    if (VAL && valid) v = vals[idx];
    uint32_t d = digit_of(k, shift);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    uint32_t rank = __popcll(peers & lanemask_lt());
    bool leader = valid && rank == 0;
    if (leader) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    {
      // one thread per digit: exclusive offsets across waves, advance base
      uint32_t run = base_cnt[threadIdx.x];
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) {
        uint32_t t = wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = run;
        run += t;
      }
      base_cnt[threadIdx.x] = run;
    }
    __syncthreads();
    if (valid) {
      uint32_t pos = wcnt[wave][d] + rank;
      okeys[pos] = k;
      if (VAL) ovals[pos] = v;
    }
    __syncthreads();
  }
}

// Up to kSmallSort (key, value) pairs sorted by one workgroup in LDS:
// bitonic sort over (key, value), padded to a power of two with the largest
// pair; equal keys end up in ascending value order.
constexpr int kSmallSort = 2048;

__global__ void __launch_bounds__(1024) k_small_sort_kv(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals, uint32_t n,
                                                        uint32_t p2, uint64_t* __restrict__ okeys,
                                                        uint32_t* __restrict__ ovals) {
  __shared__ uint64_t K[kSmallSort];
  __shared__ uint32_t V[kSmallSort];
  for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
    K[i] = i < n ? keys[i] : ~0ull;
    V[i] = i < n ? vals[i] : ~0u;
  }
  __syncthreads();
  for (uint32_t size = 2; size <= p2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
        uint32_t j = i ^ stride;
        if (j > i) {
          bool up = (i & size) == 0;
          uint64_t ki = K[i], kj = K[j];
          uint32_t vi = V[i], vj = V[j];
          bool gt = ki > kj || (ki == kj && vi > vj);
          if (gt == up) {
            K[i] = kj;
            K[j] = ki;
            V[i] = vj;
            V[j] = vi;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    okeys[i] = K[i];
    ovals[i] = V[i];
  }
}

template <typename K, bool VAL>
static void radix_pass(gj_ctx* c, const K* keys, const uint32_t* vals, K* okeys, uint32_t* ovals,
                       uint64_t n, int shift) {
  uint64_t nt = (n + kSortTile - 1) / kSortTile;
  GJ_CHECK(nt * kRadix < (1ull << 32), GJ_EUNSUPPORTED, "sort too large");
  uint32_t* hist = (uint32_t*)ws_get(c, "sort_hist", nt * kRadix * sizeof(uint32_t));
  uint32_t* hoff = (uint32_t*)ws_get(c, "sort_hoff", (nt * kRadix + 1) * sizeof(uint32_t));
  k_hist<K><<<(unsigned)nt, kBlock, 0, c->stream>>>(keys, n, shift, hist, (uint32_t)nt);
  scan_u32(c, hist, hoff, nt * kRadix);
  k_scatter<K, VAL><<<(unsigned)nt, kBlock, 0, c->stream>>>(keys, vals, n, shift, hoff,
                                                             (uint32_t)nt, okeys, ovals);
  GJ_HIP(hipGetLastError());
}

// Sorts u64 keys whose set bits lie in [0, lo_bits) and [32, 32 + hi_bits).
uint64_t* sort_u64(gj_ctx* c, uint64_t* keys, uint64_t* alt, uint64_t n, int lo_bits, int hi_bits) {
  if (n <= 1) return keys;
  for (int shift = 0; shift < 64; shift += 8) {
    bool need = shift < lo_bits || (shift >= 32 && shift - 32 < hi_bits);
    if (!need) continue;
    radix_pass<uint64_t, false>(c, keys, nullptr, alt, nullptr, n, shift);
    std::swap(keys, alt);
  }
  return keys;
}

void sort_kv_u64(gj_ctx* c, uint64_t*& key, uint32_t*& val, uint64_t*& key_alt, uint32_t*& val_alt,
                 uint64_t n, int lo_bits, int hi_bits) {
  if (n <= 1) return;
  if (n <= (uint64_t)kSmallSort) {
    // one launch instead of a histogram, scan and scatter per digit
    uint32_t p2 = 2;
    while (p2 < n) p2 <<= 1;
    k_small_sort_kv<<<1, 1024, 0, c->stream>>>(key, val, (uint32_t)n, p2, key_alt, val_alt);
    GJ_HIP(hipGetLastError());
    std::swap(key, key_alt);
    std::swap(val, val_alt);
    return;
  }
  for (int shift = 0; shift < 64; shift += 8) {
    bool need = shift < lo_bits || (shift >= 32 && shift - 32 < hi_bits);
    if (!need) continue;
    radix_pass<uint64_t, true>(c, key, val, key_alt, val_alt, n, shift);
    std::swap(key, key_alt);
    std::swap(val, val_alt);
  }
}

void sort_kv_u32(gj_ctx* c, uint32_t*& key, uint32_t*& val, uint32_t*& key_alt, uint32_t*& val_alt,
                 uint64_t n, int bits) {
  if (n <= 1) return;
  for (int shift = 0; shift < bits; shift += 8) {
    radix_pass<uint32_t, true>(c, key, val, key_alt, val_alt, n, shift);
    std::swap(key, key_alt);
    std::swap(val, val_alt);
  }
}

}  // namespace gj
