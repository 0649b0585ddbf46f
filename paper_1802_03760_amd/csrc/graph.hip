// Forward and reverse CSR indexes of the edge relation (Sec. 4.1: one forward
// and one reverse index serve every atom).  Built by sorting (src, dst) keys,
// dropping repeats and self-loops, and deriving row pointers.
#include "gj_internal.h"
#include "prim.h"

namespace gj {

__global__ void k_make_keys(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst, uint64_t m,
                            uint32_t n, uint64_t* __restrict__ keys, uint32_t* __restrict__ bad) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    uint32_t s = src[i], d = dst[i];
    if (s >= n || d >= n) atomicOr(bad, 1u);
    keys[i] = ((uint64_t)s << 32) | d;
  }
}

// keep the first of equal keys, drop self-loops
__global__ void k_unique_flags(const uint64_t* __restrict__ keys, uint64_t m, uint32_t* __restrict__ flags) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    uint64_t k = keys[i];
    bool first = i == 0 || keys[i - 1] != k;
    flags[i] = (first && (uint32_t)(k >> 32) != (uint32_t)k) ? 1u : 0u;
  }
}

__global__ void k_compact_edges(const uint64_t* __restrict__ keys, uint64_t m, const uint32_t* __restrict__ flags,
                                const uint64_t* __restrict__ off, uint32_t* __restrict__ row,
                                uint32_t* __restrict__ col, uint64_t* __restrict__ swapped) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    if (!flags[i]) continue;
    uint64_t k = keys[i], p = off[i];
    uint32_t s = (uint32_t)(k >> 32), d = (uint32_t)k;
    row[p] = s;
    col[p] = d;
    swapped[p] = ((uint64_t)d << 32) | s;
  }
}

__global__ void k_split_keys(const uint64_t* __restrict__ keys, uint64_t m, uint32_t* __restrict__ row,
                             uint32_t* __restrict__ col) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    uint64_t k = keys[i];
    row[i] = (uint32_t)(k >> 32);
    col[i] = (uint32_t)k;
  }
}

// rp[v] = first entry of row v in a row-sorted entry list (rp[n] = m)
__global__ void k_rowptr(const uint32_t* __restrict__ row, uint64_t m, uint32_t n, uint32_t* __restrict__ rp) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
    uint64_t lo = 0, len = m;
    while (len > 0) {
      uint64_t half = len >> 1;
      if (row[lo + half] < v) {
        lo += half + 1;
        len -= half + 1;
      } else {
        len = half;
      }
    }
    rp[v] = (uint32_t)lo;
  }
}

__global__ void __launch_bounds__(kBlock) k_maxdeg(const uint32_t* __restrict__ rp, uint32_t n,
                                                   uint32_t* __restrict__ out) {
  __shared__ uint32_t wbest[kBlock / 64];
  uint32_t best = 0;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    uint32_t d = rp[v + 1] - rp[v];
    best = d > best ? d : best;
  }
  best = wave_max(best);
  if (lane_id() == 0) wbest[wave_id()] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) best = wbest[w] > best ? wbest[w] : best;
    atomicMax(out, best);  // one atomic per workgroup
  }
}

void version_alloc(gj_ctx* c, Version& v, uint32_t n, uint64_t cap) {
  if (cap < 1) cap = 1;
  ++v.gen;  // the slot is about to be rewritten
  for (int d = 0; d < 2; ++d) {
    if (!v.d[d].rp) v.d[d].rp = (uint32_t*)dev_alloc(c, ((uint64_t)n + 1) * sizeof(uint32_t));
    if (cap > v.cap) {
      // a failure part-way leaves this direction without arrays and the
      // slot's capacity at 0, so the next call allocates them again
      dev_free(c, v.d[d].col);
      dev_free(c, v.d[d].row);
      v.d[d].col = nullptr;
      v.d[d].row = nullptr;
      if (d == 0) v.cap = 0;
      v.d[d].col = (uint32_t*)dev_alloc(c, cap * sizeof(uint32_t));
      v.d[d].row = (uint32_t*)dev_alloc(c, cap * sizeof(uint32_t));
    }
  }
  if (cap > v.cap) v.cap = cap;
}

void version_free(gj_ctx* c, Version& v) {
  for (int d = 0; d < 2; ++d) {
    dev_free(c, v.d[d].rp);
    dev_free(c, v.d[d].col);
    dev_free(c, v.d[d].row);
    v.d[d] = CsrDir{};
  }
  v.cap = v.m = 0;
}

int bits_for(uint32_t n) {
  int b = 0;
  while (b < 32 && ((uint64_t)1 << b) < n) ++b;
  return b;
}

void version_finish(gj_ctx* c, Version& v, uint32_t n, bool from_update) {
  ++v.gen;
  uint32_t* mx = (uint32_t*)ws_get(c, "maxdeg", 2 * sizeof(uint32_t));
  if (!from_update) {
    GJ_HIP(hipMemsetAsync(mx, 0, 2 * sizeof(uint32_t), c->stream));
    for (int d = 0; d < 2; ++d) {
      k_rowptr<<<grid_for((uint64_t)n + 1, kBlock, 1u << 16), kBlock, 0, c->stream>>>(v.d[d].row, v.m, n,
                                                                                        v.d[d].rp);
      k_maxdeg<<<grid_for(n, kBlock * 16, 1024), kBlock, 0, c->stream>>>(v.d[d].rp, n, mx + d);
    }
    GJ_HIP(hipGetLastError());
  }
  uint32_t h[2];
  read_bytes(c, h, mx, sizeof(h));
  v.max_deg[0] = h[0];
  v.max_deg[1] = h[1];
}

void graph_build(gj_ctx* c, gj_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m) {
  uint32_t n = g->n;
  int bits = bits_for(n);
  uint64_t* keys = (uint64_t*)ws_get(c, "gb_keys", (m + 1) * sizeof(uint64_t));
  uint64_t* alt = (uint64_t*)ws_get(c, "gb_alt", (m + 1) * sizeof(uint64_t));
  uint32_t* bad = (uint32_t*)ws_get(c, "gb_bad", sizeof(uint32_t));
  GJ_HIP(hipMemsetAsync(bad, 0, sizeof(uint32_t), c->stream));
  unsigned gr = grid_for(m, kBlock, 1u << 16);
  if (m) k_make_keys<<<gr, kBlock, 0, c->stream>>>(d_src, d_dst, m, n, keys, bad);
  GJ_HIP(hipGetLastError());
  uint32_t hbad = 0;
  read_bytes(c, &hbad, bad, sizeof(hbad));
  GJ_CHECK(!hbad, GJ_EINVAL, "vertex id >= num_vertices");
  uint64_t* sorted = sort_u64(c, keys, alt, m, bits, bits);
  uint64_t* other = sorted == keys ? alt : keys;
  uint32_t* flags = (uint32_t*)ws_get(c, "gb_flags", (m + 1) * sizeof(uint32_t));
  uint64_t* off = (uint64_t*)ws_get(c, "gb_off", (m + 1) * sizeof(uint64_t));
  if (m) k_unique_flags<<<gr, kBlock, 0, c->stream>>>(sorted, m, flags);
  scan_u32_to_u64(c, flags, off, m);
  uint64_t mu = read_u64(c, off + m);
  Version& v = g->ver[g->cur];
  // the same growth room as the versions updates write, so that no slot is
  // reallocated when updates come back round to it
  version_alloc(c, v, n, mu + mu / 16 + (1ull << 20));
  v.m = mu;
  if (m) k_compact_edges<<<gr, kBlock, 0, c->stream>>>(sorted, m, flags, off, v.d[0].row, v.d[0].col, other);
  uint64_t* other_alt = sorted;  // free for reuse now
  uint64_t* rsorted = sort_u64(c, other, other_alt, mu, bits, bits);
  if (mu) k_split_keys<<<grid_for(mu, kBlock, 1u << 16), kBlock, 0, c->stream>>>(rsorted, mu, v.d[1].row, v.d[1].col);
  GJ_HIP(hipGetLastError());
  version_finish(c, v, n, false);
}

// ---------------------------------------------------------------- renaming by degree (Sec. 5.4)
// Both directions of every input edge as (src, dst) keys.
__global__ void k_make_sym_keys(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst, uint64_t m,
                                uint32_t n, uint64_t* __restrict__ keys, uint32_t* __restrict__ bad) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    uint32_t s = src[i], d = dst[i];
    if (s >= n || d >= n) atomicOr(bad, 1u);
    keys[i] = ((uint64_t)s << 32) | d;
    keys[m + i] = ((uint64_t)d << 32) | s;
  }
}

// (degree, id) of every vertex; the degree is its row length in the
// symmetric edge set, i.e. the number of distinct neighbours
__global__ void k_degree_keys(const uint32_t* __restrict__ rp, uint32_t n, uint64_t* __restrict__ vkeys) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    vkeys[v] = ((uint64_t)(rp[v + 1] - rp[v]) << 32) | v;
}

// new id = rank in (degree, id) order
__global__ void k_rank_ids(const uint64_t* __restrict__ vkeys, uint32_t n, uint32_t* __restrict__ old_of_new,
                           uint32_t* __restrict__ new_of_old) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint32_t o = (uint32_t)vkeys[i];
    old_of_new[i] = o;
    new_of_old[o] = (uint32_t)i;
  }
}

// Renames both ends; with `up_only` an edge that does not go from a lower new
// id to a higher one is written as a self-loop, which the build drops.
__global__ void k_rename_edges(const uint32_t* __restrict__ row, const uint32_t* __restrict__ col, uint64_t m,
                               const uint32_t* __restrict__ new_of_old, int up_only, uint32_t* __restrict__ osrc,
                               uint32_t* __restrict__ odst) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    uint32_t u = new_of_old[row[i]], v = new_of_old[col[i]];
    osrc[i] = u;
    odst[i] = (up_only && !(u < v)) ? u : v;
  }
}

void graph_build_sym(gj_ctx* c, gj_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                     bool degree_order, bool undirected) {
  uint32_t n = g->n;
  int bits = bits_for(n);
  uint64_t m2 = 2 * m;
  struct Temps {  // freed on every exit, errors included
    gj_ctx* c;
    std::vector<void*> p;
    ~Temps() {
      for (void* x : p) dev_free(c, x);
    }
  } tmp{c, {}};
  auto alloc = [&](size_t bytes) {
    void* p = dev_alloc(c, bytes ? bytes : 1);
    tmp.p.push_back(p);
    return p;
  };
  uint64_t* keys = (uint64_t*)alloc((m2 + 1) * sizeof(uint64_t));
  uint64_t* alt = (uint64_t*)alloc((m2 + 1) * sizeof(uint64_t));
  uint32_t* flags = (uint32_t*)alloc((m2 + 1) * sizeof(uint32_t));
  uint64_t* off = (uint64_t*)alloc((m2 + 1) * sizeof(uint64_t));
  uint32_t* bad = (uint32_t*)alloc(sizeof(uint32_t));
  GJ_HIP(hipMemsetAsync(bad, 0, sizeof(uint32_t), c->stream));
  unsigned gr = grid_for(m, kBlock, 1u << 16), gr2 = grid_for(m2, kBlock, 1u << 16);
  if (m) k_make_sym_keys<<<gr, kBlock, 0, c->stream>>>(d_src, d_dst, m, n, keys, bad);
  GJ_HIP(hipGetLastError());
  uint32_t hbad = 0;
  read_bytes(c, &hbad, bad, sizeof(hbad));
  GJ_CHECK(!hbad, GJ_EINVAL, "vertex id >= num_vertices");
  // the symmetric edge set: both directions of every distinct pair, no loops
  uint64_t* sorted = sort_u64(c, keys, alt, m2, bits, bits);
  uint64_t* other = sorted == keys ? alt : keys;
  if (m2) k_unique_flags<<<gr2, kBlock, 0, c->stream>>>(sorted, m2, flags);
  scan_u32_to_u64(c, flags, off, m2);
  uint64_t ms = read_u64(c, off + m2);
  uint32_t* srow = (uint32_t*)alloc((ms + 1) * sizeof(uint32_t));
  uint32_t* scol = (uint32_t*)alloc((ms + 1) * sizeof(uint32_t));
  if (m2) k_compact_edges<<<gr2, kBlock, 0, c->stream>>>(sorted, m2, flags, off, srow, scol, other);
  const uint32_t *es = srow, *ed = scol;
  if (degree_order) {
    uint32_t* rp = (uint32_t*)alloc(((uint64_t)n + 1) * sizeof(uint32_t));
    uint64_t* vk = (uint64_t*)alloc((uint64_t)n * sizeof(uint64_t));
    uint64_t* vk2 = (uint64_t*)alloc((uint64_t)n * sizeof(uint64_t));
    uint32_t* new_of_old = (uint32_t*)alloc((uint64_t)n * sizeof(uint32_t));
    unsigned gn = grid_for((uint64_t)n + 1, kBlock, 1u << 16);
    k_rowptr<<<gn, kBlock, 0, c->stream>>>(srow, ms, n, rp);
    k_degree_keys<<<gn, kBlock, 0, c->stream>>>(rp, n, vk);
    uint64_t* vs = sort_u64(c, vk, vk2, n, bits, bits);
    g->old_of_new = (uint32_t*)dev_alloc(c, (uint64_t)n * sizeof(uint32_t));
    k_rank_ids<<<gn, kBlock, 0, c->stream>>>(vs, n, g->old_of_new, new_of_old);
    uint32_t* osrc = (uint32_t*)alloc((ms + 1) * sizeof(uint32_t));
    uint32_t* odst = (uint32_t*)alloc((ms + 1) * sizeof(uint32_t));
    if (ms)
      k_rename_edges<<<grid_for(ms, kBlock, 1u << 16), kBlock, 0, c->stream>>>(srow, scol, ms, new_of_old,
                                                                               undirected ? 0 : 1, osrc, odst);
    es = osrc;
    ed = odst;
  }
  GJ_HIP(hipGetLastError());
  graph_build(c, g, es, ed, ms);
  GJ_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace gj
