// Membership index of one direction of a graph version: the paper's O(1)
// membership test on extension sets (Sec. 2.2, where each index answers
// "is e in Ext(p)" in constant time) for the generic propose kernels.
//
// Every row with at least `min_deg` entries (option hash_min_degree) gets its
// own open-addressing table of 2^b buckets of four u32 slots (b the smallest
// with load <= 1/2), empty slots ~0.  A value's home bucket is the top b bits
// of a multiplicative hash; insertion takes the first empty slot from there
// on (slots within a bucket in order, then the next bucket, wrapping), so
// that a probe may stop at the first bucket with an empty slot.  desc[v] =
// (first bucket of v's table) << 8 | b, or 0 for a row without a table
// (searched as before).  A probe is one 16-byte load in most cases, where a
// binary search over a hub row of 10^5 entries is 17 dependent loads.
#include "gj_internal.h"
#include "prim.h"

namespace gj {

__global__ void k_hash_bits(const uint32_t* __restrict__ rp, uint32_t n, uint32_t min_deg, uint32_t* __restrict__ nb,
                            uint8_t* __restrict__ bits) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gs) {
    uint64_t d = rp[v + 1] - rp[v];
    uint32_t b = 0;
    if (d >= min_deg) {
      b = 1;
      while ((4ull << b) < 2 * d) ++b;  // 4 * 2^b slots >= 2d: load <= 1/2
    }
    bits[v] = (uint8_t)b;
    nb[v] = b ? (1u << b) : 0u;
  }
}

__global__ void k_hash_desc(const uint64_t* __restrict__ boff, const uint8_t* __restrict__ bits, uint32_t n,
                            uint64_t* __restrict__ desc) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gs)
    desc[v] = bits[v] ? (boff[v] << 8) | bits[v] : 0ull;
}

// one thread per index entry (row v = row[e], value col[e])
__global__ void k_hash_insert(const uint32_t* __restrict__ row, const uint32_t* __restrict__ col, uint64_t m,
                              const uint64_t* __restrict__ desc, uint32_t* __restrict__ slots) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gs) {
    uint64_t dd = desc[row[e]];
    uint32_t b = (uint32_t)(dd & 0xFF);
    if (!b) continue;
    uint32_t x = col[e];
    uint64_t base = dd >> 8;
    uint32_t mask = (1u << b) - 1, h = hash_home(x, b);
    for (;;) {
      uint32_t* bk = slots + 4 * (base + h);
      bool done = false;
      for (int s = 0; s < 4 && !done; ++s)
        done = atomicCAS(bk + s, kHashEmpty, x) == kHashEmpty;
      if (done) break;
      h = (h + 1) & mask;  // the table holds at most half its slots: a free one exists
    }
  }
}

static void hash_dir(gj_ctx* alloc_ctx, gj_ctx* c, const CsrDir& d, uint64_t m, uint32_t n, uint32_t min_deg,
                     HashDir& h) {
  uint32_t* nb = (uint32_t*)ws_get(c, "hash_nb", ((uint64_t)n + 1) * sizeof(uint32_t));
  uint8_t* bits = (uint8_t*)ws_get(c, "hash_bits", (uint64_t)n + 1);
  uint64_t* boff = (uint64_t*)ws_get(c, "hash_boff", ((uint64_t)n + 1) * sizeof(uint64_t));
  unsigned gn = grid_for(n, kBlock, 1u << 16);
  k_hash_bits<<<gn, kBlock, 0, c->stream>>>(d.rp, n, min_deg, nb, bits);
  scan_u32_to_u64(c, nb, boff, n);
  uint64_t buckets = read_u64(c, boff + n);
  if (!h.desc) h.desc = (uint64_t*)dev_alloc(alloc_ctx, (uint64_t)n * sizeof(uint64_t));
  if (buckets > h.buckets_cap) {
    dev_free(alloc_ctx, h.slots);
    h.slots = nullptr;
    h.buckets_cap = 0;
    uint64_t want = buckets + buckets / 8 + 1024;
    h.slots = (uint32_t*)dev_alloc(alloc_ctx, want * 4 * sizeof(uint32_t));
    h.buckets_cap = want;
  }
  k_hash_desc<<<gn, kBlock, 0, c->stream>>>(boff, bits, n, h.desc);
  if (buckets) GJ_HIP(hipMemsetAsync(h.slots, 0xFF, buckets * 4 * sizeof(uint32_t), c->stream));
  if (m) k_hash_insert<<<grid_for(m, kBlock, 1u << 16), kBlock, 0, c->stream>>>(d.row, d.col, m, h.desc, h.slots);
  GJ_HIP(hipGetLastError());
}

void hash_free(gj_ctx* c, Version& v) {
  for (int d = 0; d < 2; ++d) {
    dev_free(c, v.h[d].desc);
    dev_free(c, v.h[d].slots);
    v.h[d] = HashDir{};
  }
  v.hash_gen = ~0ull;
}

// The index of a version is used when it was built for the version's
// current contents and no row of the view is remapped by log-structured
// updates.  `v` may be a graph slot or a copy of one (the server reads
// copies): the index is built into the slot that holds the same arrays and
// contents, and the copy receives it.
void hash_ensure(gj_ctx* c, const gj_graph* gc, const Version& v) {
  if (!c->hash_index || !c->hash_build || v.pmap[0] || v.pmap[1] || v.m == 0) return;
  Version& view = const_cast<Version&>(v);
  if (view.hash_gen == view.gen && view.hash_min == c->hash_min_degree) return;
  gj_graph* g = const_cast<gj_graph*>(gc);
  std::lock_guard<std::mutex> lk(g->hash_mu);  // one build per slot, whichever context asks first
  Version* slot = nullptr;
  for (Version& s : g->ver)
    if (s.d[0].col == v.d[0].col && s.gen == v.gen) slot = &s;
  if (!slot) return;
  if (slot->hash_gen != slot->gen || slot->hash_min != c->hash_min_degree) {
    slot->hash_gen = ~0ull;
    for (int d = 0; d < 2; ++d) hash_dir(g->ctx, c, slot->d[d], slot->m, g->n, c->hash_min_degree, slot->h[d]);
    GJ_HIP(hipStreamSynchronize(c->stream));  // complete before another stream reads it
    slot->hash_gen = slot->gen;
    slot->hash_min = c->hash_min_degree;
    ++c->hash_builds;
  }
  if (slot != &view) {
    view.h[0] = slot->h[0];
    view.h[1] = slot->h[1];
    view.hash_gen = slot->hash_gen;
    view.hash_min = slot->hash_min;
  }
}

bool hash_note_work(gj_ctx* c, const gj_graph* gc, const Version& v, uint64_t W) {
  Version& view = const_cast<Version&>(v);
  if (view.hash_gen == view.gen && view.hash_min == c->hash_min_degree) return true;
  if (!c->hash_index || !c->hash_build || v.pmap[0] || v.pmap[1] || v.m == 0) return false;
  if (view.work_gen != view.gen) {
    view.work_gen = view.gen;
    view.probe_work = 0;
  }
  view.probe_work += W;
  if (view.probe_work < c->hash_build_work * v.m) return false;
  hash_ensure(c, gc, v);
  return view.hash_gen == view.gen;
}

}  // namespace gj
