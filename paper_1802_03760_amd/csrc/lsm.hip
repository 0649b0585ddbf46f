// Log-structured updates: the multi-version index of Sec. 4.3 on one GPU.
//
// The paper's index holds a compacted index of old data, per-vertex
// log-structured lists of committed changes that can be merged one vertex at
// a time, and the uncommitted changes in order.  Here the compacted index is a
// version slot (both CSR directions).  An update batch dE (already sorted and
// classified against the current version) rewrites only the rows it touches:
// each is merged with its run of dE and appended to the slack of the same
// column array past the slot's m, and a per-vertex map records where the row
// now lives.  The maps are double-buffered: the one of the current version
// stays untouched while the one of the next version is written, so the old
// and the new version of the batch are both readable while its delta queries
// run (atoms before i read the new one, atoms after i the old one).  An
// update thus writes the touched rows and the map entries of the rows
// rewritten before it, not both indexes.  When the slack is used up, or when
// a reader needs a plain CSR, every row is merged into another slot (a
// compaction), which becomes current.
#include <algorithm>
#include <cstring>

#include "gj_internal.h"
#include "lsm.h"
#include "prim.h"

namespace gj {

// ---------------------------------------------------------------- kernels
__global__ void k_lsm_heads(const uint32_t* __restrict__ r, const int8_t* __restrict__ g, uint64_t k,
                            uint32_t* __restrict__ head, uint32_t* __restrict__ insf) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) {
    head[i] = (i == 0 || r[i] != r[i - 1]) ? 1u : 0u;
    insf[i] = g[i] > 0 ? 1u : 0u;
  }
}

// Run t of dE (one touched vertex): its vertex and first entry; dlo[nt] = k.
__global__ void k_lsm_runs(const uint32_t* __restrict__ r, uint64_t k, const uint32_t* __restrict__ head,
                           const uint64_t* __restrict__ hscan, uint32_t* __restrict__ tv, uint32_t* __restrict__ dlo) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) {
    if (i == 0) dlo[hscan[k]] = (uint32_t)k;
    if (!head[i]) continue;
    uint64_t t = hscan[i];
    tv[t] = r[i];
    dlo[t] = (uint32_t)i;
  }
}

// Per run t: the vertex's row in the current version (olo, olen), its length
// after the batch (every delete of dE removes a present entry, every insert
// adds an absent one), and whether the vertex has no rewritten row yet.
__global__ void k_lsm_sizes(const uint32_t* __restrict__ tv, const uint32_t* __restrict__ dlo, uint64_t nt,
                            const uint64_t* __restrict__ ins_scan, const uint32_t* __restrict__ rp,
                            const uint64_t* __restrict__ pm, uint32_t* __restrict__ olo,
                            uint32_t* __restrict__ olen, uint32_t* __restrict__ nlen, uint32_t* __restrict__ fresh) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gs) {
    uint32_t v = tv[t], a = dlo[t], b = dlo[t + 1];
    uint32_t ins = (uint32_t)(ins_scan[b] - ins_scan[a]);
    uint32_t del = (b - a) - ins;
    uint32_t lo, hi;
    row_range(rp, pm, v, lo, hi);
    olo[t] = lo;
    olen[t] = hi - lo;
    nlen[t] = hi - lo + ins - del;
    fresh[t] = (!pm || pm[v] == ~0ull) ? 1u : 0u;
  }
}

// Entry i of the concatenated old rows of the touched vertices, to its place
// in the rewritten row (deleted entries dropped).  Reads and writes share col:
// old rows lie below the append point, rewritten ones above it.
__global__ void k_lsm_move(const uint64_t* __restrict__ ooff, uint64_t nt, uint64_t tot,
                           const uint32_t* __restrict__ olo, const uint32_t* __restrict__ dlo,
                           const uint32_t* __restrict__ dx, const uint64_t* __restrict__ ins_scan,
                           const uint64_t* __restrict__ noff, uint64_t abase, uint32_t* col) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gs) {
    uint64_t t = find_segment(ooff, 0, nt, i);
    uint32_t j = (uint32_t)(i - ooff[t]);
    uint32_t x = col[olo[t] + j];
    uint32_t a = dlo[t], b = dlo[t + 1];
    uint32_t p = lower_bound_u32(dx, a, b, x);
    if (p < b && dx[p] == x) continue;  // deleted
    uint32_t ins_before = (uint32_t)(ins_scan[p] - ins_scan[a]);
    uint32_t del_before = (p - a) - ins_before;
    col[abase + noff[t] + j + ins_before - del_before] = x;
  }
}

// Inserted entries of dE to their places in the rewritten rows: every entry
// of the run before i is below x, and every delete among them an old entry.
__global__ void k_lsm_ins(const uint32_t* __restrict__ dx, const int8_t* __restrict__ dg, uint64_t k,
                          const uint64_t* __restrict__ hscan, const uint32_t* __restrict__ dlo,
                          const uint32_t* __restrict__ olo, const uint32_t* __restrict__ olen,
                          const uint64_t* __restrict__ ins_scan, const uint64_t* __restrict__ noff, uint64_t abase,
                          uint32_t* col) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) {
    if (dg[i] < 0) continue;
    uint64_t t = hscan[i + 1] - 1;
    uint32_t a = dlo[t], x = dx[i];
    uint32_t less = lower_bound_u32(col, olo[t], olo[t] + olen[t], x) - olo[t];
    uint32_t ins_before = (uint32_t)(ins_scan[i] - ins_scan[a]);
    uint32_t del_before = ((uint32_t)i - a) - ins_before;
    col[abase + noff[t] + less - del_before + ins_before] = x;
  }
}

__global__ void k_lsm_copy_map(const uint32_t* __restrict__ keys, uint64_t nkeys, const uint64_t* __restrict__ from,
                               uint64_t* __restrict__ to) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nkeys; i += gs) {
    uint32_t v = keys[i];
    to[v] = from[v];
  }
}

__global__ void k_lsm_set_map(const uint32_t* __restrict__ tv, uint64_t nt, const uint64_t* __restrict__ noff,
                              const uint32_t* __restrict__ nlen, uint64_t abase, const uint32_t* __restrict__ fresh,
                              const uint64_t* __restrict__ fscan, uint64_t nkeys, uint64_t* __restrict__ to,
                              uint32_t* __restrict__ keys) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gs) {
    uint32_t v = tv[t];
    to[v] = (abase + noff[t]) | ((uint64_t)nlen[t] << 32);
    if (fresh[t]) keys[nkeys + fscan[t]] = v;
  }
}

__global__ void k_lsm_unset(const uint32_t* __restrict__ keys, uint64_t nkeys, uint64_t* __restrict__ m0,
                            uint64_t* __restrict__ m1) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nkeys; i += gs) {
    uint32_t v = keys[i];
    m0[v] = ~0ull;
    m1[v] = ~0ull;
  }
}

// ---- compaction
__global__ void k_view_deg(const uint32_t* __restrict__ rp, const uint64_t* __restrict__ pm, uint32_t n,
                           uint32_t* __restrict__ deg) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gs) {
    uint32_t lo, hi;
    row_range(rp, pm, (uint32_t)v, lo, hi);
    deg[v] = hi - lo;
  }
}

// entries of the compacted slot whose row was not rewritten
__global__ void k_copy_base(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ col,
                            const uint32_t* __restrict__ row, uint64_t m, const uint64_t* __restrict__ pm,
                            const uint32_t* __restrict__ nrp, uint32_t* __restrict__ ncol,
                            uint32_t* __restrict__ nrow) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gs) {
    uint32_t r = row[e];
    if (pm[r] != ~0ull) continue;
    uint64_t pos = (uint64_t)nrp[r] + (e - rp[r]);
    ncol[pos] = col[e];
    nrow[pos] = r;
  }
}

__global__ void k_key_lens(const uint32_t* __restrict__ keys, uint64_t nkeys, const uint64_t* __restrict__ pm,
                           uint32_t* __restrict__ lens) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nkeys; i += gs)
    lens[i] = (uint32_t)(pm[keys[i]] >> 32);
}

// the entries of the rewritten rows, in key-list order (koff: their offsets)
__global__ void __launch_bounds__(kBlock) k_copy_rows(const uint32_t* __restrict__ keys,
                                                      const uint64_t* __restrict__ koff, uint64_t nkeys,
                                                      uint64_t tot, const uint64_t* __restrict__ pm,
                                                      const uint32_t* __restrict__ col,
                                                      const uint32_t* __restrict__ nrp, uint32_t* __restrict__ ncol,
                                                      uint32_t* __restrict__ nrow) {
  const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) << 6; base < tot;
       base += waves << 6) {
    uint64_t t0 = wave_first_segment(koff, nkeys, base);
    uint64_t i = base + lane_id();
    if (i >= tot) continue;
    uint64_t t = gallop_segment(koff, t0, nkeys, i);
    uint32_t v = keys[t];
    uint32_t j = (uint32_t)(i - koff[t]);
    uint64_t dst = (uint64_t)nrp[v] + j;
    ncol[dst] = col[(uint32_t)pm[v] + j];
    nrow[dst] = v;
  }
}

// ---------------------------------------------------------------- host
// allocates whatever an earlier call did not (one that failed part-way
// leaves the rest null, never a half-initialised map)
static void lsm_alloc(gj_ctx* c, gj_graph* g) {
  LsmState& L = g->lsm;
  uint64_t bytes = (uint64_t)g->n * sizeof(uint64_t);
  for (int b = 0; b < 2; ++b)
    for (int d = 0; d < 2; ++d) {
      if (L.map[b][d]) continue;
      uint64_t* p = (uint64_t*)dev_alloc(c, bytes);
      hipError_t e = hipMemsetAsync(p, 0xFF, bytes, c->stream);
      if (e != hipSuccess) dev_free(c, p);
      GJ_HIP(e);
      L.map[b][d] = p;
    }
  for (int d = 0; d < 2; ++d)
    if (!L.keys[d]) L.keys[d] = (uint32_t*)dev_alloc(c, (uint64_t)g->n * sizeof(uint32_t));
}

void lsm_free(gj_graph* g) {
  LsmState& L = g->lsm;
  for (int b = 0; b < 2; ++b)
    for (int d = 0; d < 2; ++d) dev_free(g->ctx, L.map[b][d]);
  for (int d = 0; d < 2; ++d) dev_free(g->ctx, L.keys[d]);
  L = LsmState{};
}

void lsm_clear(gj_ctx* c, gj_graph* g) {
  // every entry other than ~0 in either map belongs to a vertex of the key list
  LsmState& L = g->lsm;
  for (int d = 0; d < 2; ++d)
    if (L.map[0][d] && L.nkeys[d])
      k_lsm_unset<<<grid_for(L.nkeys[d], kBlock, 1u << 16), kBlock, 0, c->stream>>>(L.keys[d], L.nkeys[d],
                                                                                    L.map[0][d], L.map[1][d]);
  GJ_HIP(hipGetLastError());
  L.on = false;
  L.cur_map = 0;
  L.nkeys[0] = L.nkeys[1] = 0;
  L.used[0] = L.used[1] = 0;
}

const uint64_t* lsm_row_offsets(gj_ctx* c, const gj_graph* g, int d, uint64_t& total) {
  const LsmState& L = g->lsm;
  total = 0;
  if (!L.on || !L.nkeys[d]) return nullptr;
  const std::string tag = d ? "r" : "f";
  uint64_t nk = L.nkeys[d];
  uint32_t* lens = (uint32_t*)ws_get(c, "lsm_klen" + tag, (nk + 1) * sizeof(uint32_t));
  uint64_t* off = (uint64_t*)ws_get(c, "lsm_koff" + tag, (nk + 1) * sizeof(uint64_t));
  k_key_lens<<<grid_for(nk, kBlock, 1u << 16), kBlock, 0, c->stream>>>(L.keys[d], nk, L.map[L.cur_map][d], lens);
  GJ_HIP(hipGetLastError());
  scan_u32_to_u64(c, lens, off, nk);
  total = read_u64(c, off + nk);
  return off;
}

void graph_compact(gj_ctx* c, gj_graph* g) {
  LsmState& L = g->lsm;
  if (!L.on) return;
  uint32_t n = g->n;
  int s = g->cur < 2 ? 1 - g->cur : 0;
  Version& ov = g->ver[g->cur];
  Version& nv = g->ver[s];
  uint64_t m = L.m;
  // room for the rows appended by the updates that follow: m / 2 + 2^22
  // entries per direction, reallocated only when less than half of that is
  // left (a graph that grows would otherwise reallocate at every compaction)
  uint64_t room = m / 2 + (1ull << 22);
  if (m + room / 2 > nv.cap) version_alloc(c, nv, n, m + room);
  ++nv.gen;
  uint32_t* deg = (uint32_t*)ws_get(c, "lsm_deg", ((uint64_t)n + 1) * sizeof(uint32_t));
  for (int d = 0; d < 2; ++d) {
    const uint64_t* pm = L.map[L.cur_map][d];
    k_view_deg<<<grid_for(n, kBlock, 1u << 16), kBlock, 0, c->stream>>>(ov.d[d].rp, pm, n, deg);
    scan_u32(c, deg, nv.d[d].rp, n);
    if (ov.m)
      k_copy_base<<<grid_for(ov.m, kBlock, 1u << 16), kBlock, 0, c->stream>>>(ov.d[d].rp, ov.d[d].col, ov.d[d].row,
                                                                             ov.m, pm, nv.d[d].rp, nv.d[d].col,
                                                                             nv.d[d].row);
    uint64_t tot = 0;
    const uint64_t* koff = lsm_row_offsets(c, g, d, tot);
    if (tot)
      k_copy_rows<<<grid_for(tot, kBlock, 1u << 16), kBlock, 0, c->stream>>>(
          L.keys[d], koff, L.nkeys[d], tot, pm, ov.d[d].col, nv.d[d].rp, nv.d[d].col, nv.d[d].row);
    GJ_HIP(hipGetLastError());
  }
  nv.m = m;
  version_finish(c, nv, n, false);
  g->cur = s;
  lsm_clear(c, g);
  ++c->lsm_compactions;
  GJ_HIP(hipStreamSynchronize(c->stream));
}

namespace {

// Scratch and sizes of one direction of one update.
struct DirPlan {
  const uint32_t* r;
  const uint32_t* x;
  const int8_t* g;
  uint64_t k = 0;
  uint32_t *head, *insf, *tv, *dlo, *olo, *olen, *nlen, *fresh;
  uint64_t *hscan, *ins_scan, *noff, *ooff, *fscan;
  uint64_t nt = 0, tot_new = 0, tot_old = 0, nfresh = 0, ins = 0;
};

std::string tag_of(int d) { return d ? "r" : "f"; }

uint32_t* ws32(gj_ctx* c, const char* name, int d, uint64_t cnt) {
  return (uint32_t*)ws_get(c, std::string("lsm_") + name + tag_of(d), (cnt + 1) * sizeof(uint32_t));
}
uint64_t* ws64(gj_ctx* c, const char* name, int d, uint64_t cnt) {
  return (uint64_t*)ws_get(c, std::string("lsm_") + name + tag_of(d), (cnt + 1) * sizeof(uint64_t));
}

// runs of dE per touched vertex, and insert counts (phase 1 of the sizing)
void runs(gj_ctx* c, int d, DirPlan& P) {
  uint64_t k = P.k;
  P.head = ws32(c, "head", d, k);
  P.insf = ws32(c, "insf", d, k);
  P.hscan = ws64(c, "hscan", d, k);
  P.ins_scan = ws64(c, "inss", d, k);
  k_lsm_heads<<<grid_for(k, kBlock, 1u << 16), kBlock, 0, c->stream>>>(P.r, P.g, k, P.head, P.insf);
  scan_u32_to_u64(c, P.head, P.hscan, k);
  scan_u32_to_u64(c, P.insf, P.ins_scan, k);
}

// per touched vertex, its current row and its length after the batch
// (phase 2, once the number of touched vertices nt is known)
void sizes(gj_ctx* c, gj_graph* g, int d, DirPlan& P) {
  uint64_t k = P.k, nt = P.nt;
  P.tv = ws32(c, "tv", d, nt);
  P.dlo = ws32(c, "dlo", d, nt + 1);
  P.olo = ws32(c, "olo", d, nt);
  P.olen = ws32(c, "olen", d, nt);
  P.nlen = ws32(c, "nlen", d, nt);
  P.fresh = ws32(c, "fresh", d, nt);
  P.noff = ws64(c, "noff", d, nt);
  P.ooff = ws64(c, "ooff", d, nt);
  P.fscan = ws64(c, "fscan", d, nt);
  k_lsm_runs<<<grid_for(k, kBlock, 1u << 16), kBlock, 0, c->stream>>>(P.r, k, P.head, P.hscan, P.tv, P.dlo);
  const LsmState& L = g->lsm;
  const uint64_t* pm = L.on ? L.map[L.cur_map][d] : nullptr;
  k_lsm_sizes<<<grid_for(nt, kBlock, 1u << 16), kBlock, 0, c->stream>>>(
      P.tv, P.dlo, nt, P.ins_scan, g->ver[g->cur].d[d].rp, pm, P.olo, P.olen, P.nlen, P.fresh);
  GJ_HIP(hipGetLastError());
  scan_u32_to_u64(c, P.nlen, P.noff, nt);
  scan_u32_to_u64(c, P.olen, P.ooff, nt);
  scan_u32_to_u64(c, P.fresh, P.fscan, nt);
}

void measure(gj_ctx* c, gj_graph* g, DirPlan (&P)[2]) {
  for (int d = 0; d < 2; ++d) runs(c, d, P[d]);
  uint64_t h[4];
  read_u64s(c, {P[0].hscan + P[0].k, P[0].ins_scan + P[0].k, P[1].hscan + P[1].k, P[1].ins_scan + P[1].k}, h);
  for (int d = 0; d < 2; ++d) {
    P[d].nt = h[2 * d];
    P[d].ins = h[2 * d + 1];
    sizes(c, g, d, P[d]);
  }
  uint64_t t[6];
  read_u64s(c, {P[0].noff + P[0].nt, P[0].ooff + P[0].nt, P[0].fscan + P[0].nt, P[1].noff + P[1].nt,
                P[1].ooff + P[1].nt, P[1].fscan + P[1].nt},
            t);
  for (int d = 0; d < 2; ++d) {
    P[d].tot_new = t[3 * d];
    P[d].tot_old = t[3 * d + 1];
    P[d].nfresh = t[3 * d + 2];
  }
}

// the rows of both directions appended, and the next version's map written
void write_rows(gj_ctx* c, gj_graph* g, const DirPlan (&P)[2], uint64_t k, LsmCommit& commit) {
  LsmState& L = g->lsm;
  Version& base = g->ver[g->cur];
  const int nb = 1 - L.cur_map;
  for (int d = 0; d < 2; ++d) {
    const DirPlan& p = P[d];
    uint64_t abase = base.m + L.used[d];
    if (p.tot_old)
      k_lsm_move<<<grid_for(p.tot_old, kBlock, 1u << 16), kBlock, 0, c->stream>>>(
          p.ooff, p.nt, p.tot_old, p.olo, p.dlo, p.x, p.ins_scan, p.noff, abase, base.d[d].col);
    k_lsm_ins<<<grid_for(k, kBlock, 1u << 16), kBlock, 0, c->stream>>>(p.x, p.g, k, p.hscan, p.dlo, p.olo, p.olen,
                                                                      p.ins_scan, p.noff, abase, base.d[d].col);
    if (L.nkeys[d])
      k_lsm_copy_map<<<grid_for(L.nkeys[d], kBlock, 1u << 16), kBlock, 0, c->stream>>>(
          L.keys[d], L.nkeys[d], L.map[L.cur_map][d], L.map[nb][d]);
    k_lsm_set_map<<<grid_for(p.nt, kBlock, 1u << 16), kBlock, 0, c->stream>>>(
        p.tv, p.nt, p.noff, p.nlen, abase, p.fresh, p.fscan, L.nkeys[d], L.map[nb][d], L.keys[d]);
    GJ_HIP(hipGetLastError());
    commit.used[d] = L.used[d] + p.tot_new;
    commit.nkeys[d] = L.nkeys[d] + p.nfresh;
  }
}

// Whether this update appends its rows: they fit the current slot's slack,
// and they are at most an eighth of the edges (2^16 entries at least) per
// direction.  A larger batch touches most of the heavy rows, so writing both
// indexes anew costs little more than appending them, and leaves the slack
// to the small batches that follow.
bool appends(const gj_ctx* c, const gj_graph* g, const DirPlan (&P)[2]) {
  const Version& v = g->ver[g->cur];
  const uint64_t m = g->lsm.on ? g->lsm.m : v.m;
  uint64_t room = v.cap - v.m;
  if (c->lsm_max_patch) room = std::min(room, c->lsm_max_patch);
  for (int d = 0; d < 2; ++d) {
    uint64_t end = g->lsm.used[d] + P[d].tot_new;
    if (end > room || v.m + end > 0xFFFFFFFFull) return false;
    if (P[d].tot_new > std::max<uint64_t>(m / 8, 1u << 16)) return false;
  }
  return true;
}

}  // namespace

bool lsm_update(gj_ctx* c, gj_graph* g, const uint32_t* const (&r)[2], const uint32_t* const (&x)[2],
                const int8_t* const (&sg)[2], uint64_t k, Version& oldv, Version& newv, LsmCommit& commit) {
  // a batch this large touches most heavy rows: it is written as a new
  // version without sizing its rows first
  if (k >= c->lsm_fold_min) return false;
  lsm_alloc(c, g);
  DirPlan P[2];
  for (int d = 0; d < 2; ++d) {
    P[d].r = r[d];
    P[d].x = x[d];
    P[d].g = sg[d];
    P[d].k = k;
  }
  measure(c, g, P);
  if (!appends(c, g, P)) return false;
  LsmState& L = g->lsm;
  Version& base = g->ver[g->cur];
  const int nb = 1 - L.cur_map;
  try {
    write_rows(c, g, P, k, commit);
  } catch (...) {
    lsm_abort(c, g);  // the next map may be partly written
    throw;
  }
  // every insert and delete of dE appears once per direction
  uint64_t ins = P[0].ins, del = k - P[0].ins;
  const uint64_t m0 = L.on ? L.m : base.m;
  commit.m = m0 + ins - del;
  oldv = base;
  newv = base;
  for (int d = 0; d < 2; ++d) {
    oldv.pmap[d] = L.on ? L.map[L.cur_map][d] : nullptr;
    newv.pmap[d] = L.map[nb][d];
  }
  oldv.m = m0;
  newv.m = commit.m;
  return true;
}

void lsm_commit(gj_graph* g, const LsmCommit& commit) {
  LsmState& L = g->lsm;
  for (int d = 0; d < 2; ++d) {
    L.used[d] = commit.used[d];
    L.nkeys[d] = commit.nkeys[d];
  }
  L.m = commit.m;
  L.cur_map = 1 - L.cur_map;
  L.on = true;
}

void lsm_abort(gj_ctx* c, gj_graph* g) {
  // the next version's map may hold entries of vertices outside the key list:
  // make it equal to the current one again
  LsmState& L = g->lsm;
  if (!L.map[0][0]) return;
  const int nb = 1 - L.cur_map;
  uint64_t bytes = (uint64_t)g->n * sizeof(uint64_t);
  for (int d = 0; d < 2; ++d) {
    (void)hipMemsetAsync(L.map[nb][d], 0xFF, bytes, c->stream);
    if (L.on && L.nkeys[d])
      k_lsm_copy_map<<<grid_for(L.nkeys[d], kBlock, 1u << 16), kBlock, 0, c->stream>>>(
          L.keys[d], L.nkeys[d], L.map[L.cur_map][d], L.map[nb][d]);
  }
  (void)hipStreamSynchronize(c->stream);
}

}  // namespace gj
