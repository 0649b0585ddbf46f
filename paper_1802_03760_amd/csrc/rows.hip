// Output rows: lexicographic sort (LSD over columns, last attribute first) and
// consolidation of signed delta rows (sum the signs of equal rows, drop zeros).
#include "gj_internal.h"
#include "prim.h"

namespace gj {

__global__ void k_iota(uint32_t* __restrict__ idx, uint64_t n) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) idx[i] = (uint32_t)i;
}

__global__ void k_gather_key(const uint32_t* __restrict__ rows, const uint32_t* __restrict__ idx, uint64_t n,
                             int m, int col, uint32_t* __restrict__ key) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs)
    key[i] = rows[(uint64_t)idx[i] * m + col];
}

__global__ void k_gather_rows(const uint32_t* __restrict__ rows, const int8_t* __restrict__ signs,
                              const uint32_t* __restrict__ idx, uint64_t n, int m, uint32_t* __restrict__ orows,
                              int8_t* __restrict__ osigns) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) {
    uint64_t s = idx[i];
    for (int k = 0; k < m; ++k) orows[i * m + k] = rows[s * m + k];
    if (signs) osigns[i] = signs[s];
  }
}

void sort_rows(gj_ctx* c, uint32_t* rows, int8_t* signs, uint64_t n, int m, uint32_t nverts) {
  if (n <= 1) return;
  GJ_CHECK(n < (1ull << 32), GJ_EUNSUPPORTED, "too many rows to sort");
  uint32_t* idx = (uint32_t*)ws_get(c, "rs_idx", n * sizeof(uint32_t));
  uint32_t* idx2 = (uint32_t*)ws_get(c, "rs_idx2", n * sizeof(uint32_t));
  uint32_t* key = (uint32_t*)ws_get(c, "rs_key", n * sizeof(uint32_t));
  uint32_t* key2 = (uint32_t*)ws_get(c, "rs_key2", n * sizeof(uint32_t));
  unsigned gr = grid_for(n, kBlock, 1u << 16);
  k_iota<<<gr, kBlock, 0, c->stream>>>(idx, n);
  int bits = bits_for(nverts);
  if (bits == 0) bits = 1;
  for (int col = m - 1; col >= 0; --col) {
    k_gather_key<<<gr, kBlock, 0, c->stream>>>(rows, idx, n, m, col, key);
    sort_kv_u32(c, key, idx, key2, idx2, n, bits);
  }
  uint32_t* tmp = (uint32_t*)ws_get(c, "rs_rows", n * m * sizeof(uint32_t));
  int8_t* tmps = signs ? (int8_t*)ws_get(c, "rs_signs", n) : nullptr;
  k_gather_rows<<<gr, kBlock, 0, c->stream>>>(rows, signs, idx, n, m, tmp, tmps);
  GJ_HIP(hipGetLastError());
  GJ_HIP(hipMemcpyAsync(rows, tmp, n * m * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
  if (signs) GJ_HIP(hipMemcpyAsync(signs, tmps, n, hipMemcpyDeviceToDevice, c->stream));
}

__device__ __forceinline__ bool row_eq(const uint32_t* a, const uint32_t* b, int m) {
  for (int k = 0; k < m; ++k)
    if (a[k] != b[k]) return false;
  return true;
}

// run heads of equal rows: net sign of the run; flag heads with a nonzero net
__global__ void k_run_sums(const uint32_t* __restrict__ rows, const int8_t* __restrict__ signs, uint64_t n, int m,
                           int32_t* __restrict__ net, uint32_t* __restrict__ flags,
                           unsigned long long* __restrict__ total) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  int64_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) {
    const uint32_t* r = rows + i * m;
    bool head = i == 0 || !row_eq(r - m, r, m);
    int32_t s = 0;
    if (head) {
      for (uint64_t k = i; k < n && row_eq(rows + k * m, r, m); ++k) s += signs[k];
      acc += s;
    }
    net[i] = s;
    flags[i] = (head && s != 0) ? 1u : 0u;
  }
  uint64_t t = block_sum<kBlock>((uint64_t)acc);
  if (threadIdx.x == 0 && t) atomicAdd(total, (unsigned long long)t);
}

__global__ void k_run_write(const uint32_t* __restrict__ rows, const int32_t* __restrict__ net,
                            const uint32_t* __restrict__ flags, const uint64_t* __restrict__ off, uint64_t n, int m,
                            uint32_t* __restrict__ orows, int8_t* __restrict__ osigns, uint64_t cap) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) {
    if (!flags[i]) continue;
    uint64_t p = off[i];
    if (p >= cap) continue;
    if (orows)
      for (int k = 0; k < m; ++k) orows[p * m + k] = rows[i * m + k];
    if (osigns) osigns[p] = (int8_t)net[i];
  }
}

uint64_t consolidate_rows(gj_ctx* c, const uint32_t* rows, const int8_t* signs, uint64_t n, int m,
                          uint32_t* out_rows, int8_t* out_signs, uint64_t cap, int64_t* sum) {
  int32_t* net = (int32_t*)ws_get(c, "cr_net", (n + 1) * sizeof(int32_t));
  uint32_t* flags = (uint32_t*)ws_get(c, "cr_flags", (n + 1) * sizeof(uint32_t));
  uint64_t* off = (uint64_t*)ws_get(c, "cr_off", (n + 1) * sizeof(uint64_t));
  unsigned long long* tot = (unsigned long long*)ws_get(c, "cr_tot", sizeof(unsigned long long));
  GJ_HIP(hipMemsetAsync(tot, 0, sizeof(unsigned long long), c->stream));
  unsigned gr = grid_for(n, kBlock, 1u << 16);
  if (n) k_run_sums<<<gr, kBlock, 0, c->stream>>>(rows, signs, n, m, net, flags, tot);
  scan_u32_to_u64(c, flags, off, n);
  if (n) k_run_write<<<gr, kBlock, 0, c->stream>>>(rows, net, flags, off, n, m, out_rows, out_signs, cap);
  GJ_HIP(hipGetLastError());
  uint64_t T = read_u64(c, off + n);
  unsigned long long s = 0;
  read_bytes(c, &s, tot, sizeof(s));
  *sum = (int64_t)s;
  return T;
}

}  // namespace gj
