// The triangle relation as an index for ternary atoms (Sec. 5.4: the paper
// materialises all triangles as a relation tri(a_i, a_j, a_k) indexed by
// (a_i, a_j)).  For every forward edge (x, y), in edge order, the ascending
// list out(x) & out(y) -- the third vertices of the transitive triangles on
// that edge -- stored as a CSR over edge positions with 64-bit row pointers.
//
// It is the third stage of the transitive triangle query over P_2 = all
// edges, run with the ordinary stage kernels in seed chunks: a first pass
// counts the survivors of every edge (k_propose mode 3) and turns the counts
// into row pointers; a second pass repeats the same proposals and writes the
// survivors' values in candidate order, which is edge order and, within an
// edge, ascending.
#include <cstring>
#include <vector>

#include "gj_internal.h"
#include "prim.h"

namespace gj {

__global__ void k_add_base(const uint64_t* __restrict__ scan, uint64_t k, uint64_t base, uint64_t* __restrict__ out) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= k; i += gs) out[i] = base + scan[i];
}

void tri_index_free(gj_graph* g) {
  dev_free(g->ctx, g->tri.rp);
  dev_free(g->ctx, g->tri.col);
  g->tri = TriIndex{};
}

void tri_index_build(gj_ctx* c, gj_graph* g) {
  tri_index_free(g);
  const Version& v = g->ver[g->cur];
  uint64_t m = v.m;
  // owned by the graph from the start (freed by gj_graph_destroy or the next
  // build if this one fails); valid once version and slot are set at the end
  TriIndex& t = g->tri;
  t.rp = (uint64_t*)dev_alloc(c, (m + 1) * sizeof(uint64_t));
  // third attribute bound by out(x) and out(y)
  StageDesc d;
  memset(&d, 0, sizeof(d));
  d.j = 2;
  d.k = 2;
  for (int a = 0; a < kMaxBind; ++a) {
    d.col[a] = a == 1 ? 1 : 0;
    d.rp[a] = v.d[0].rp;
    d.adj[a] = v.d[0].col;
    d.col2[a] = -1;
  }
  uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(c->seed_chunk, m));
  uint64_t piece = c->frontier_cap;
  uint64_t words = piece / 64 + 2;
  uint32_t* F = (uint32_t*)ws_get(c, "tri_F", 2 * chunk * sizeof(uint32_t) + 16);
  uint32_t* minc = (uint32_t*)ws_get(c, "tri_minc", chunk * sizeof(uint32_t) + 16);
  uint8_t* mini = (uint8_t*)ws_get(c, "tri_mini", chunk + 16);
  uint64_t* off = (uint64_t*)ws_get(c, "tri_off", (chunk + 1) * sizeof(uint64_t));
  uint32_t* cnt = (uint32_t*)ws_get(c, "tri_cnt", chunk * sizeof(uint32_t) + 16);
  uint64_t* cscan = (uint64_t*)ws_get(c, "tri_cscan", (chunk + 1) * sizeof(uint64_t));
  uint64_t* mask = (uint64_t*)ws_get(c, "tri_mask", words * sizeof(uint64_t));
  uint32_t* wcnt = (uint32_t*)ws_get(c, "tri_wcnt", words * sizeof(uint32_t));
  uint64_t* woff = (uint64_t*)ws_get(c, "tri_woff", (words + 1) * sizeof(uint64_t));
  auto load_chunk = [&](uint64_t s, uint64_t k) {
    GJ_HIP(hipMemcpyAsync(F, v.d[0].row + s, k * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
    GJ_HIP(hipMemcpyAsync(F + chunk, v.d[0].col + s, k * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
    launch_count_min(c, F, chunk, k, d, minc, mini);
    scan_u32_to_u64(c, minc, off, k);
    return read_u64(c, off + k);
  };
  // pass 1: triangles per edge -> row pointers
  std::vector<uint64_t> base(1, 0);
  for (uint64_t s = 0; s < m; s += chunk) {
    uint64_t k = std::min(chunk, m - s);
    uint64_t W = load_chunk(s, k);
    GJ_HIP(hipMemsetAsync(cnt, 0, k * sizeof(uint32_t), c->stream));
    if (W) launch_propose(c, 3, F, chunk, k, off, mini, d, 0, W, nullptr, cnt, nullptr, nullptr);
    scan_u32_to_u64(c, cnt, cscan, k);
    k_add_base<<<grid_for(k + 1, kBlock, 1u << 16), kBlock, 0, c->stream>>>(cscan, k, base.back(), t.rp + s);
    GJ_HIP(hipGetLastError());
    base.push_back(base.back() + read_u64(c, cscan + k));
  }
  if (m == 0) GJ_HIP(hipMemsetAsync(t.rp, 0, sizeof(uint64_t), c->stream));
  t.size = base.back();
  t.col = (uint32_t*)dev_alloc(c, std::max<uint64_t>(t.size, 1) * sizeof(uint32_t));
  // pass 2: the same proposals, survivors' values in candidate order
  size_t ci = 0;
  for (uint64_t s = 0; s < m; s += chunk, ++ci) {
    uint64_t k = std::min(chunk, m - s);
    uint64_t W = load_chunk(s, k);
    uint64_t at = base[ci];
    for (uint64_t w0 = 0; w0 < W; w0 += piece) {
      uint64_t w1 = std::min(W, w0 + piece);
      uint64_t nw = (w1 - w0 + 63) >> 6;
      launch_propose(c, 0, F, chunk, k, off, mini, d, w0, w1, mask, wcnt, nullptr, nullptr);
      scan_u32_to_u64(c, wcnt, woff, nw);
      uint64_t T = read_u64(c, woff + nw);
      if (T) launch_emit_values(c, F, chunk, k, off, mini, d, w0, w1, mask, woff, t.col, at, t.size);
      at += T;
    }
    GJ_CHECK(at == base[ci + 1], GJ_EDEVICE, "triangle index passes disagree");
  }
  GJ_HIP(hipStreamSynchronize(c->stream));
  t.version = g->version;
  t.slot = g->cur;
}

}  // namespace gj
