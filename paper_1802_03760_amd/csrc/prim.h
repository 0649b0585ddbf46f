// Wave64 / workgroup primitives used by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gj {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Inequality filters of symmetry breaking (Sec. 5.4): value e joining the
// prefix in slot p of a column-major frontier must exceed prefix column c
// for every bit c of `above` and stay below it for every bit of `below`.
__device__ __forceinline__ bool ineq_ok(const uint32_t* __restrict__ F, uint64_t stride, uint64_t p,
                                        uint32_t above, uint32_t below, uint32_t e) {
  if (!(above | below)) return true;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (((above | below) >> c) & 1) {
      uint32_t o = F[(uint64_t)c * stride + p];
      if ((above >> c) & 1) ok = ok && e > o;
      if ((below >> c) & 1) ok = ok && e < o;
    }
  }
  return ok;
}

// Both seed attributes at hand: bit 0 of the masks relates x1 to x0.
__device__ __forceinline__ bool seed_ineq_ok(uint32_t above, uint32_t below, uint32_t x0, uint32_t x1) {
  return (!(above & 1) || x1 > x0) && (!(below & 1) || x1 < x0);
}
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int o) {
  uint32_t lo = __shfl_up((unsigned)v, o, 64);
  uint32_t hi = __shfl_up((unsigned)(v >> 32), o, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_down_u64(uint64_t v, int o) {
  uint32_t lo = __shfl_down((unsigned)v, o, 64);
  uint32_t hi = __shfl_down((unsigned)(v >> 32), o, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((unsigned)v, src, 64);
  uint32_t hi = __shfl((unsigned)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = shfl_up_u64(v, o);
    if (l >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += shfl_down_u64(v, o);
  return shfl_u64(v, 0);
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t t = __shfl_down(v, o, 64);
    v = t > v ? t : v;
  }
  return __shfl(v, 0, 64);
}

// Exclusive scan over the workgroup (blockDim.x == NT, NT/64 waves).
// `total` receives the workgroup sum.  Contains __syncthreads.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T& total) {
  __shared__ T wsum[NT / 64];
  T inc = wave_incl_scan(v);
  if (lane_id() == 63) wsum[wave_id()] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    T s = wsum[w];
    if (w < wave_id()) before += s;
    all += s;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

// The same scan with few live registers: each wave scans, then the first
// wave scans the wave totals (sh holds NT / 64 + 1 values).  For wide
// workgroups, where the loop above keeps every wave total live at once.
// Contains __syncthreads; the caller synchronises before reusing sh.
template <int NT, typename T>
__device__ __forceinline__ T block_scan_lean(T v, T& total, T* sh) {
  constexpr int NW = NT / 64;
  const int lane = lane_id(), wave = wave_id();
  const T inc = wave_incl_scan(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const T x = lane < NW ? sh[lane] : (T)0;
    const T xi = wave_incl_scan(x);
    if (lane < NW) sh[lane] = xi - x;
    if (lane == NW - 1) sh[NW] = xi;
  }
  __syncthreads();
  total = sh[NW];
  return sh[wave] + inc - v;
}

template <int NT>
__device__ __forceinline__ uint64_t block_sum(uint64_t v) {
  __shared__ uint64_t wsum[NT / 64];
  v = wave_sum(v);
  if (lane_id() == 0) wsum[wave_id()] = v;
  __syncthreads();
  uint64_t all = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) all += wsum[w];
  __syncthreads();
  return all;
}

// Workgroup sum with few live registers (see block_scan_lean); sh holds
// NT / 64 + 1 values.  Contains __syncthreads.
template <int NT>
__device__ __forceinline__ uint64_t block_sum_lean(uint64_t v, uint64_t* sh) {
  constexpr int NW = NT / 64;
  const int lane = lane_id(), wave = wave_id();
  v = wave_sum(v);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (wave == 0) {
    const uint64_t t = wave_sum(lane < NW ? sh[lane] : 0ull);
    if (lane == 0) sh[NW] = t;
  }
  __syncthreads();
  const uint64_t all = sh[NW];
  __syncthreads();
  return all;
}

// lower_bound of x in sorted a[lo, hi): first index with a[i] >= x
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t lo,
                                                    uint32_t hi, uint32_t x) {
  uint32_t n = hi - lo;
  while (n > 0) {
    uint32_t half = n >> 1;
    if (a[lo + half] < x) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

__device__ __forceinline__ bool contains_u32(const uint32_t* __restrict__ a, uint32_t lo,
                                             uint32_t hi, uint32_t x) {
  uint32_t i = lower_bound_u32(a, lo, hi, x);
  return i < hi && a[i] == x;
}

// Row v of one direction of a version: col[lo, hi).  A log-structured update
// rewrites a row into the tail of the same column array and records it in
// the version's per-vertex map pm (offset | length << 32; ~0 for a row still
// at rp[v] .. rp[v + 1]); pm is null when no row is rewritten.
// The three loads are independent (issued together), so a map costs a
// lookup no extra latency.
__device__ __forceinline__ void row_range(const uint32_t* __restrict__ rp, const uint64_t* __restrict__ pm,
                                          uint32_t v, uint32_t& lo, uint32_t& hi) {
  uint32_t a = rp[v], b = rp[v + 1];
  if (pm) {
    uint64_t e = pm[v];
    if (e != ~0ull) {
      a = (uint32_t)e;
      b = a + (uint32_t)(e >> 32);
    }
  }
  lo = a;
  hi = b;
}

// ---------------------------------------------------------------- membership index
// A row's table descriptor: first bucket << 8 | b for a table of 2^b
// four-slot buckets; 0 = the row has no table.
constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;  // never a vertex id (ids < 2^32 - 1)

// home bucket of x among 2^b (b >= 1): the top b bits of a multiplicative
// hash
__device__ __forceinline__ uint32_t hash_home(uint32_t x, uint32_t b) { return (x * 0x9E3779B1u) >> (32 - b); }

// x in the row table `desc` (b > 0) of `slots`: buckets from the home bucket
// on until x or a bucket with an empty slot (insertion never passes one)
__device__ __forceinline__ bool hash_member(const uint32_t* __restrict__ slots, uint64_t desc, uint32_t x) {
  const uint32_t b = (uint32_t)(desc & 0xFF), mask = (1u << b) - 1;
  const uint64_t base = desc >> 8;
  uint32_t h = hash_home(x, b);
  for (;;) {
    uint4 q = *(const uint4*)(slots + 4 * (base + h));
    if (q.x == x || q.y == x || q.z == x || q.w == x) return true;
    if (q.w == kHashEmpty) return false;
    h = (h + 1) & mask;
  }
}

// p in [lo, hi) with off[p] <= g < off[p+1]; requires off[lo] <= g < off[hi].
__device__ __forceinline__ uint64_t find_segment(const uint64_t* __restrict__ off, uint64_t lo,
                                                 uint64_t hi, uint64_t g) {
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) >> 1;
    if (off[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// As find_segment, searching forward from a known lower bound lo (off[lo] <= g)
// by doubling steps first: cheap when g lies a few segments past lo.
__device__ __forceinline__ uint64_t gallop_segment(const uint64_t* __restrict__ off, uint64_t lo, uint64_t n,
                                                   uint64_t g) {
  uint64_t step = 1, hi = lo + 1;
  while (hi < n && off[hi] <= g) {
    lo = hi;
    step <<= 1;
    hi = lo + step;
  }
  if (hi > n) hi = n;
  return find_segment(off, lo, hi, g);
}

// For a wave that walks elements [base, base + 64) of a concatenation of n
// segments with offsets off (off[n] = total, base < total): the segment of
// element base, found by lane 0 and broadcast; each lane then gallops from
// it to its own element's segment, so long segments cost one search per
// wave, not one per element.
__device__ __forceinline__ uint64_t wave_first_segment(const uint64_t* __restrict__ off, uint64_t n,
                                                       uint64_t base) {
  uint64_t t0 = 0;
  if (lane_id() == 0) t0 = find_segment(off, 0, n, base);
  return shfl_u64(t0, 0);
}

}  // namespace gj
