// Delta queries (Delta-GJ, Sec. 3.3.1; Delta-BiGJoin, Sec. 3.3.2 and 4.3).
//
// An update batch is normalised into a signed edge change dE, the next
// version of both indexes is built next to the current one (old and new stay
// resident together, the two versions every dQ_i reads), and for every atom i
// of every query the delta query dQ_i runs through the same stage kernels as
// the static path: seeded with dE on R_i's attributes, atoms before i read the
// new version and atoms after i the old one, each prefix carrying the sign of
// its seed.  The signed outputs of all dQ_i are consolidated per tuple.
#include <algorithm>
#include <cstring>

#include "batch.h"
#include "engine.h"
#include "gj_internal.h"
#include "lsm.h"
#include "owner.h"
#include <thread>
#include "prim.h"

namespace gj {

// ---------------------------------------------------------------- batch normalisation
__global__ void k_batch_keys(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                             const int8_t* __restrict__ sign, uint64_t b, uint32_t n, uint64_t* __restrict__ keys,
                             uint32_t* __restrict__ vals, uint32_t* __restrict__ bad) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += gs) {
    uint32_t s = src[i], d = dst[i];
    int8_t g = sign[i];
    if (s >= n || d >= n || (g != 1 && g != -1)) {
      // the batch is rejected once the flag is read; until then the row
      // stands in as the self-loop (0, 0), which no later kernel looks up
      atomicOr(bad, 1u);
      s = d = 0;
    }
    keys[i] = ((uint64_t)s << 32) | d;
    vals[i] = g > 0 ? 1u : 0u;
  }
}

// One flag per distinct (src, dst) of the sorted batch: 1 if it changes the
// graph.  counters: [0] no-op inserts, [1] no-op deletes, [2] conflicts.
__global__ void k_batch_classify(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ins, uint64_t b,
                                 const uint32_t* __restrict__ rp, const uint32_t* __restrict__ col,
                                 const uint64_t* __restrict__ pm, uint32_t* __restrict__ flags, int8_t* __restrict__ dsign,
                                 unsigned long long* __restrict__ counters) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += gs) {
    uint64_t k = keys[i];
    flags[i] = 0;
    if (i > 0 && keys[i - 1] == k) continue;  // not the head of its run
    uint32_t s = (uint32_t)(k >> 32), d = (uint32_t)k;
    bool any_ins = false, any_del = false;
    for (uint64_t j = i; j < b && keys[j] == k; ++j) {
      if (ins[j])
        any_ins = true;
      else
        any_del = true;
    }
    if (s == d) continue;  // self-loops are dropped
    if (any_ins && any_del) {
      atomicAdd(counters + 2, 1ull);
      continue;
    }
    uint32_t lo, hi;
    row_range(rp, pm, s, lo, hi);
    bool present = contains_u32(col, lo, hi, d);
    if (any_ins && present) {
      atomicAdd(counters + 0, 1ull);
      continue;
    }
    if (any_del && !present) {
      atomicAdd(counters + 1, 1ull);
      continue;
    }
    flags[i] = 1;
    dsign[i] = any_ins ? (int8_t)1 : (int8_t)-1;
  }
}

__global__ void k_batch_compact(const uint64_t* __restrict__ keys, const int8_t* __restrict__ dsign,
                                const uint32_t* __restrict__ flags, const uint64_t* __restrict__ off, uint64_t b,
                                uint32_t* __restrict__ es, uint32_t* __restrict__ ed, int8_t* __restrict__ eg,
                                uint64_t* __restrict__ swapped, uint32_t* __restrict__ sidx) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += gs) {
    if (!flags[i]) continue;
    uint64_t p = off[i], k = keys[i];
    es[p] = (uint32_t)(k >> 32);
    ed[p] = (uint32_t)k;
    eg[p] = dsign[i];
    swapped[p] = (k << 32) | (k >> 32);
    sidx[p] = (uint32_t)p;
  }
}

// ---------------------------------------------------------------- versioned index update
// dE of one direction: rows r[i], values x[i], signs g[i], sorted by (r, x);
// drp = per-row ranges of dE (n + 1); ins_scan = exclusive scan of insert flags.
struct DeltaDir {
  const uint32_t* r;
  const uint32_t* x;
  const int8_t* g;
  const uint32_t* drp;
  const uint64_t* ins_scan;
};

__global__ void k_ins_flags(const int8_t* __restrict__ g, uint64_t k, uint32_t* __restrict__ f) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) f[i] = g[i] > 0 ? 1u : 0u;
}

// Per row v of one direction: drp[v], where the rows of dE (sorted) reach v;
// the row's new degree deg[v]; and the largest new degree, folded into
// *maxdeg by at most one atomicMax per workgroup (launched with few
// workgroups for that reason).  A wave covers 63 rows at a time: its lane 63
// only finds where row v + 1 starts, for lane 62.
__global__ void __launch_bounds__(kBlock) k_delta_rows(const uint32_t* __restrict__ r, uint64_t k,
                                                       const uint64_t* __restrict__ ins_scan,
                                                       const uint32_t* __restrict__ rp,
                                                       const uint64_t* __restrict__ pm, uint32_t n,
                                                       uint32_t* __restrict__ drp, uint32_t* __restrict__ deg,
                                                       uint32_t* __restrict__ maxdeg) {
  __shared__ uint32_t wbest[kBlock / 64];
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  uint32_t best = 0;
  for (uint64_t base = wave * 63; base <= n; base += waves * 63) {
    uint64_t v = base + lane;
    uint64_t lo = k;
    if (v <= n) {
      uint64_t len = k;
      lo = 0;
      while (len > 0) {
        uint64_t half = len >> 1;
        if (r[lo + half] < v) {
          lo += half + 1;
          len -= half + 1;
        } else {
          len = half;
        }
      }
      drp[v] = (uint32_t)lo;
    }
    uint32_t hi = __shfl_down((uint32_t)lo, 1, 64);
    if (lane < 63 && v < n) {
      uint32_t ins = (uint32_t)(ins_scan[hi] - ins_scan[lo]);
      uint32_t del = (hi - (uint32_t)lo) - ins;
      uint32_t olo, ohi;
      row_range(rp, pm, (uint32_t)v, olo, ohi);
      uint32_t d = ohi - olo + ins - del;
      deg[v] = d;
      best = d > best ? d : best;
    }
  }
  best = wave_max(best);
  if (lane == 0) wbest[wave_id()] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) best = wbest[w] > best ? wbest[w] : best;
    // the atomics of many workgroups on one word serialise: most are skipped
    if (best > __hip_atomic_load(maxdeg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(maxdeg, best);
  }
}

// copy the surviving old entries to their new positions.  A workgroup moves a
// tile of kMoveU * kBlock consecutive entries, each thread kMoveU of them
// kBlock apart, with every load of a tile issued before the row lookups that
// depend on them, so that a wave has kMoveU independent loads in flight.
// Rows that a log-structured update rewrote (pm, when not null) are moved by
// k_move_rewritten instead.
constexpr int kMoveU = 4;
__global__ void __launch_bounds__(kBlock) k_move_old(const uint32_t* __restrict__ orp,
                                                     const uint32_t* __restrict__ ocol,
                                                     const uint32_t* __restrict__ orow, uint64_t om,
                                                     const uint64_t* __restrict__ pm, DeltaDir D,
                                                     const uint32_t* __restrict__ nrp, uint32_t* __restrict__ ncol,
                                                     uint32_t* __restrict__ nrow) {
  const uint64_t tile = (uint64_t)kBlock * kMoveU;
  for (uint64_t base = (uint64_t)blockIdx.x * tile; base < om; base += (uint64_t)gridDim.x * tile) {
    uint32_t r[kMoveU], x[kMoveU], a[kMoveU], b[kMoveU], np[kMoveU], op[kMoveU];
    bool moved[kMoveU];
#pragma unroll
    for (int u = 0; u < kMoveU; ++u) {
      uint64_t e = base + (uint64_t)u * kBlock + threadIdx.x;
      r[u] = 0;  // row 0 exists: the lookups below stay in bounds past the end
      x[u] = 0;
      if (e < om) {
        r[u] = orow[e];
        x[u] = ocol[e];
      }
    }
#pragma unroll
    for (int u = 0; u < kMoveU; ++u) {
      a[u] = D.drp[r[u]];
      b[u] = D.drp[r[u] + 1];
      np[u] = nrp[r[u]];
      op[u] = orp[r[u]];
      moved[u] = pm && pm[r[u]] != ~0ull;
    }
#pragma unroll
    for (int u = 0; u < kMoveU; ++u) {
      uint64_t e = base + (uint64_t)u * kBlock + threadIdx.x;
      if (e >= om || moved[u]) continue;
      uint64_t pos = (uint64_t)np[u] + (e - op[u]);
      if (a[u] != b[u]) {
        uint32_t i = lower_bound_u32(D.x, a[u], b[u], x[u]);
        if (i < b[u] && D.x[i] == x[u]) continue;  // deleted (an insert of a present edge never reaches dE)
        uint32_t ins_before = (uint32_t)(D.ins_scan[i] - D.ins_scan[a[u]]);
        uint32_t del_before = (i - a[u]) - ins_before;
        pos = pos + ins_before - del_before;
      }
      ncol[pos] = x[u];
      nrow[pos] = r[u];
    }
  }
}

// the surviving entries of the rows a log-structured update rewrote (keys:
// their vertices, koff: the offsets of their rows in key-list order, tot
// entries; pm: where each row lies in ocol), spread over the grid entry by
// entry so that long rows do not serialise on one wave
__global__ void __launch_bounds__(kBlock) k_move_rewritten(const uint32_t* __restrict__ keys,
                                                           const uint64_t* __restrict__ koff, uint64_t nkeys,
                                                           uint64_t tot, const uint64_t* __restrict__ pm,
                                                           const uint32_t* __restrict__ ocol, DeltaDir D,
                                                           const uint32_t* __restrict__ nrp,
                                                           uint32_t* __restrict__ ncol, uint32_t* __restrict__ nrow) {
  const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) << 6; base < tot;
       base += waves << 6) {
    uint64_t t0 = wave_first_segment(koff, nkeys, base);
    uint64_t e = base + lane_id();
    if (e >= tot) continue;
    uint64_t t = gallop_segment(koff, t0, nkeys, e);
    uint32_t v = keys[t];
    uint32_t j = (uint32_t)(e - koff[t]);
    uint32_t x = ocol[(uint32_t)pm[v] + j];
    uint32_t a = D.drp[v], b = D.drp[v + 1];
    uint64_t pos = (uint64_t)nrp[v] + j;
    if (a != b) {
      uint32_t i = lower_bound_u32(D.x, a, b, x);
      if (i < b && D.x[i] == x) continue;  // deleted
      uint32_t ins_before = (uint32_t)(D.ins_scan[i] - D.ins_scan[a]);
      uint32_t del_before = (i - a) - ins_before;
      pos = pos + ins_before - del_before;
    }
    ncol[pos] = x;
    nrow[pos] = v;
  }
}

// place the inserted entries
__global__ void k_place_ins(const uint32_t* __restrict__ orp, const uint32_t* __restrict__ ocol,
                            const uint64_t* __restrict__ pm, DeltaDir D, uint64_t k,
                            const uint32_t* __restrict__ nrp, uint32_t* __restrict__ ncol,
                            uint32_t* __restrict__ nrow) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) {
    if (D.g[i] < 0) continue;
    uint32_t r = D.r[i], x = D.x[i];
    uint32_t a = D.drp[r];
    uint32_t olo, ohi;
    row_range(orp, pm, r, olo, ohi);
    uint32_t old_less = lower_bound_u32(ocol, olo, ohi, x) - olo;
    uint32_t ins_before = (uint32_t)(D.ins_scan[i] - D.ins_scan[a]);
    uint32_t del_before = ((uint32_t)i - a) - ins_before;  // every delete below x is an old entry below x
    uint64_t pos = (uint64_t)nrp[r] + old_less - del_before + ins_before;
    ncol[pos] = x;
    nrow[pos] = r;
  }
}

__global__ void k_unswap(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx,
                         const int8_t* __restrict__ g, uint64_t k, uint32_t* __restrict__ r, uint32_t* __restrict__ x,
                         int8_t* __restrict__ og) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) {
    r[i] = (uint32_t)(keys[i] >> 32);
    x[i] = (uint32_t)keys[i];
    og[i] = g[idx[i]];
  }
}

// Rows appended by log-structured updates to one direction of the current
// version: their map, vertices and offsets (see lsm_row_offsets).
struct Rewritten {
  const uint64_t* pm = nullptr;
  const uint32_t* keys = nullptr;
  const uint64_t* koff = nullptr;
  uint64_t nkeys = 0, tot = 0;
};

// One direction of the next version, from the current one: the slot od with
// om entries, and the rows appended since (rw).
static void update_dir(gj_ctx* c, uint32_t n, const CsrDir& od, uint64_t om, const Rewritten& rw,
                       const uint32_t* r, const uint32_t* x, const int8_t* g, uint64_t k, CsrDir& nd,
                       const std::string& tag, uint32_t* maxdeg) {
  const uint64_t* pm = rw.pm;
  uint32_t* drp = (uint32_t*)ws_get(c, "up_drp" + tag, ((uint64_t)n + 1) * sizeof(uint32_t));
  uint32_t* insf = (uint32_t*)ws_get(c, "up_insf" + tag, (k + 1) * sizeof(uint32_t));
  uint64_t* ins_scan = (uint64_t*)ws_get(c, "up_inss" + tag, (k + 1) * sizeof(uint64_t));
  uint32_t* deg = (uint32_t*)ws_get(c, "up_deg", ((uint64_t)n + 1) * sizeof(uint32_t));
  unsigned gn = grid_for(((uint64_t)n + 63) / 63 * 64, kBlock, 2048);  // a wave per 63 rows
  unsigned gk = grid_for(k, kBlock, 1u << 16);
  k_ins_flags<<<gk, kBlock, 0, c->stream>>>(g, k, insf);
  scan_u32_to_u64(c, insf, ins_scan, k);
  k_delta_rows<<<gn, kBlock, 0, c->stream>>>(r, k, ins_scan, od.rp, pm, n, drp, deg, maxdeg);
  DeltaDir D{r, x, g, drp, ins_scan};
  scan_u32(c, deg, nd.rp, n);
  if (om)
    k_move_old<<<grid_for((om + kMoveU - 1) / kMoveU, kBlock, 1u << 16), kBlock, 0, c->stream>>>(
        od.rp, od.col, od.row, om, pm, D, nd.rp, nd.col, nd.row);
  if (pm && rw.tot)
    k_move_rewritten<<<grid_for(rw.tot, kBlock, 1u << 16), kBlock, 0, c->stream>>>(
        rw.keys, rw.koff, rw.nkeys, rw.tot, pm, od.col, D, nd.rp, nd.col, nd.row);
  k_place_ins<<<gk, kBlock, 0, c->stream>>>(od.rp, od.col, pm, D, k, nd.rp, nd.col, nd.row);
  GJ_HIP(hipGetLastError());
}

static void add_stats(gj_stats& a, const gj_stats& b) {
  for (int j = 0; j <= GJ_MAX_ATTRS; ++j) {
    a.prefixes[j] += b.prefixes[j];
    a.extensions[j] += b.extensions[j];
  }
  a.kernel_ms += b.kernel_ms;
  a.kernel_launches += b.kernel_launches;
}

// One dQ_i of a count-only query on the depth-first path (signed sum of its
// outputs and its counters), on context c.
static void delta_count_one(gj_ctx* c, const gj_query* q, int i, const Version& ov, const Version& nv,
                            const uint32_t* es, const uint32_t* ed, const int8_t* eg, uint64_t k, int64_t& ws,
                            uint64_t& matches, gj_stats& st) {
  PlanH P = make_plan(q, delta_order(q, i), i);
  Views V{&ov, &nv, i};
  Runner R(c, P, V, true, false, std::max<uint64_t>(1, std::min<uint64_t>(c->seed_chunk, k)));
  R.seed(es, ed, eg, k);
  R.finish(matches, ws);
  st = R.st;
}

void apply_updates(gj_ctx* c, gj_graph* g, const uint32_t* src, const uint32_t* dst, const int8_t* sign, uint64_t b,
                   int on_device, const gj_query* const* qs, uint32_t nq, int64_t* count_delta,
                   uint32_t* const* out_rows, int8_t* const* out_signs, const uint64_t* cap, uint64_t* n_delta,
                   gj_stats* stats, bool& overflow, int target, const std::vector<gj_ctx*>* lanes) {
  overflow = false;
  uint32_t n = g->n;
  int bits = bits_for(n);
  // log-structured updates for the plain entry point only: a caller that
  // names the slot (the server) keeps every version a plain CSR
  const bool lsm = c->lsm_updates && target < 0;
  LsmState& L = g->lsm;
  GJ_CHECK(target < 0 || (target < kMaxVersions && target != g->cur), GJ_EINVAL,
           "update target is the current version");
  c->last_delta.assign(nq, gj_ctx::LastDelta{});
  for (uint32_t k = 0; k < nq; ++k) {
    if (count_delta) count_delta[k] = 0;
    if (n_delta) n_delta[k] = 0;
    if (stats) memset(&stats[k], 0, sizeof(gj_stats));
  }
  GJ_CHECK(b < (1ull << 32), GJ_EUNSUPPORTED, "update batch of 2^32 rows or more");
  // ---- upload and normalise the batch
  const uint32_t *ds = src, *dd = dst;
  const int8_t* dg = sign;
  if (!on_device && b) {
    uint32_t* s2 = (uint32_t*)ws_get(c, "ub_src", b * sizeof(uint32_t));
    uint32_t* d2 = (uint32_t*)ws_get(c, "ub_dst", b * sizeof(uint32_t));
    int8_t* g2 = (int8_t*)ws_get(c, "ub_sign", b);
    GJ_HIP(hipMemcpyAsync(s2, src, b * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    GJ_HIP(hipMemcpyAsync(d2, dst, b * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    GJ_HIP(hipMemcpyAsync(g2, sign, b, hipMemcpyHostToDevice, c->stream));
    ds = s2;
    dd = d2;
    dg = g2;
  }
  uint64_t* keys = (uint64_t*)ws_get(c, "ub_keys", (b + 1) * sizeof(uint64_t));
  uint64_t* keys2 = (uint64_t*)ws_get(c, "ub_keys2", (b + 1) * sizeof(uint64_t));
  uint32_t* vals = (uint32_t*)ws_get(c, "ub_vals", (b + 1) * sizeof(uint32_t));
  uint32_t* vals2 = (uint32_t*)ws_get(c, "ub_vals2", (b + 1) * sizeof(uint32_t));
  // counters of the classification (no-op inserts, no-op deletes,
  // conflicts), then the flag of an invalid row; read with the number of
  // changes in one synchronisation
  unsigned long long* cnt = (unsigned long long*)ws_get(c, "ub_cnt", 4 * sizeof(unsigned long long));
  uint32_t* bad = (uint32_t*)(cnt + 3);
  GJ_HIP(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), c->stream));
  unsigned gb = grid_for(b, kBlock, 1u << 16);
  if (b) k_batch_keys<<<gb, kBlock, 0, c->stream>>>(ds, dd, dg, b, n, keys, vals, bad);
  sort_kv_u64(c, keys, vals, keys2, vals2, b, bits, bits);
  uint32_t* flags = (uint32_t*)ws_get(c, "ub_flags", (b + 1) * sizeof(uint32_t));
  int8_t* dsign = (int8_t*)ws_get(c, "ub_dsign", b + 1);
  uint64_t* off = (uint64_t*)ws_get(c, "ub_off", (b + 1) * sizeof(uint64_t));
  // the current version as the update reads it: the slot ver[cur], plus the
  // rows appended by log-structured updates since its last rewrite
  Version cur_view = g->ver[g->cur];
  if (L.on) {
    for (int d = 0; d < 2; ++d) cur_view.pmap[d] = L.map[L.cur_map][d];
    cur_view.m = L.m;
  }
  if (b)
    k_batch_classify<<<gb, kBlock, 0, c->stream>>>(keys, vals, b, cur_view.d[0].rp, cur_view.d[0].col,
                                                   cur_view.pmap[0], flags, dsign, cnt);
  scan_u32_to_u64(c, flags, off, b);
  uint64_t hc[5];
  read_u64s(c, {(const uint64_t*)cnt, (const uint64_t*)cnt + 1, (const uint64_t*)cnt + 2, (const uint64_t*)cnt + 3,
                off + b}, hc);
  GJ_CHECK(!hc[3], GJ_EINVAL, "update batch: vertex id >= num_vertices or sign not +-1");
  GJ_CHECK(hc[2] == 0, GJ_EINVAL, "update batch inserts and deletes the same edge");
  uint64_t k = hc[4];
  // dE sorted by (src, dst) and by (dst, src)
  uint32_t* es = (uint32_t*)ws_get(c, "de_src", (k + 1) * sizeof(uint32_t));
  uint32_t* ed = (uint32_t*)ws_get(c, "de_dst", (k + 1) * sizeof(uint32_t));
  int8_t* eg = (int8_t*)ws_get(c, "de_sign", k + 1);
  uint64_t* sw = (uint64_t*)ws_get(c, "de_sw", (k + 1) * sizeof(uint64_t));
  uint64_t* sw2 = (uint64_t*)ws_get(c, "de_sw2", (k + 1) * sizeof(uint64_t));
  uint32_t* si = (uint32_t*)ws_get(c, "de_si", (k + 1) * sizeof(uint32_t));
  uint32_t* si2 = (uint32_t*)ws_get(c, "de_si2", (k + 1) * sizeof(uint32_t));
  if (b) k_batch_compact<<<gb, kBlock, 0, c->stream>>>(keys, dsign, flags, off, b, es, ed, eg, sw, si);
  GJ_HIP(hipGetLastError());
  for (uint32_t q = 0; q < nq; ++q) {
    if (stats) {
      stats[q].noop_inserts = hc[0];
      stats[q].noop_deletes = hc[1];
    }
  }
  if (k == 0) return;  // nothing changes: same version
  sort_kv_u64(c, sw, si, sw2, si2, k, bits, bits);
  uint32_t* rs = (uint32_t*)ws_get(c, "de_rsrc", (k + 1) * sizeof(uint32_t));
  uint32_t* rd = (uint32_t*)ws_get(c, "de_rdst", (k + 1) * sizeof(uint32_t));
  int8_t* rg = (int8_t*)ws_get(c, "de_rsign", k + 1);
  k_unswap<<<grid_for(k, kBlock, 1u << 16), kBlock, 0, c->stream>>>(sw, si, eg, k, rd, rs, rg);
  // ---- next version: the touched rows appended (log-structured), else both
  // indexes written into another slot from the current version (appended
  // rows included, which ends their epoch)
  Version lsm_old, lsm_new;
  LsmCommit commit;
  const bool patched =
      lsm && lsm_update(c, g, {es, rd}, {ed, rs}, {eg, rg}, k, lsm_old, lsm_new, commit);
  struct AbortGuard {  // an uncommitted log-structured update leaves the maps as they were
    gj_ctx* c;
    gj_graph* g;
    bool armed;
    ~AbortGuard() {
      if (armed) lsm_abort(c, g);
    }
  } guard{c, g, patched};
  if (!patched) {
    if (target < 0) target = g->cur < 2 ? 1 - g->cur : 0;
    const Version& bv = g->ver[g->cur];
    Version& nv = g->ver[target];
    // upper bound of the new edge count: old + all of dE, with slack so that a
    // growing graph does not reallocate the spare version on every batch
    uint64_t need = cur_view.m + k;
    if (need > nv.cap) version_alloc(c, nv, n, need + need / 16 + (1u << 20));
    ++nv.gen;  // rewritten from here on: its membership index no longer holds
    uint32_t* mx = (uint32_t*)ws_get(c, "maxdeg", 2 * sizeof(uint32_t));
    GJ_HIP(hipMemsetAsync(mx, 0, 2 * sizeof(uint32_t), c->stream));
    for (int d = 0; d < 2; ++d) {
      Rewritten rw;
      if (L.on) {
        rw.pm = cur_view.pmap[d];
        rw.keys = L.keys[d];
        rw.nkeys = L.nkeys[d];
        rw.koff = lsm_row_offsets(c, g, d, rw.tot);
      }
      update_dir(c, n, bv.d[d], bv.m, rw, d ? rd : es, d ? rs : ed, d ? rg : eg, k, nv.d[d], d ? "r" : "f", mx + d);
    }
    // the new edge count and the largest degrees (written by the update), in
    // one synchronisation
    uint32_t h3[3];
    read_u32s(c, {nv.d[0].rp + n, mx, mx + 1}, h3);
    nv.m = h3[0];
    ++nv.gen;  // written (as version_finish marks a slot)
    nv.max_deg[0] = h3[1];
    nv.max_deg[1] = h3[2];
  }
  const Version& ov = patched ? lsm_old : cur_view;
  const Version& nv = patched ? lsm_new : g->ver[target];
  // ---- delta queries
  std::vector<char> done(nq, 0);
  // Count-only queries whose every dQ_i extends the seed edge by one attribute
  // bound by one atom on each seed attribute (the triangle shapes): each dQ_i
  // runs the owner-grouped kernel over the signed seeds, grouped by source
  // (the forward delta rows) and by destination (the reverse ones), for
  // batches with enough changes to pay for its planning over every vertex.
  if (c->strategy != 1 && k >= c->delta_owner_min && !patched && !ov.pmap[0]) {
    const uint32_t* drp_f = (const uint32_t*)ws_get(c, "up_drpf", ((uint64_t)n + 1) * sizeof(uint32_t));
    const uint32_t* drp_r = (const uint32_t*)ws_get(c, "up_drpr", ((uint64_t)n + 1) * sizeof(uint32_t));
    for (uint32_t qi = 0; qi < nq; ++qi) {
      bool want_rows = (out_rows && out_rows[qi]) || (out_signs && out_signs[qi]);
      const gj_query* q = qs[qi];
      if (want_rows || q->m != 3) continue;
      std::vector<PlanH> plans;
      bool ok = true;
      for (int i = 0; i < (int)q->atoms.size() && ok; ++i) {
        plans.push_back(make_plan(q, delta_order(q, i), i));
        const PlanH& P = plans.back();
        ok = P.filters.empty() && !P.has_ineq() && P.bind[2].size() == 2 && P.bind[2][0].col != P.bind[2][1].col;
      }
      if (!ok) continue;
      gj_stats acc{};
      int64_t cd = 0;
      uint64_t raw = 0;
      for (int i = 0; i < (int)plans.size(); ++i) {
        const PlanH& P = plans[i];
        Views V{&ov, &nv, i};
        const BindH& A = P.bind[2][0].col == 0 ? P.bind[2][0] : P.bind[2][1];
        const BindH& B = P.bind[2][0].col == 0 ? P.bind[2][1] : P.bind[2][0];
        const Version& VA = V.of(A.atom);
        const Version& VB = V.of(B.atom);
        OwnerArgs oa{VA.d[A.dir].rp, VA.d[A.dir].col, VB.d[B.dir].rp, VB.d[B.dir].col, drp_f, ed, drp_r, rs,
                     n, eg, rg};
        KernelTimer timer(c);
        uint64_t mt = 0, ex = 0;
        int64_t ws = 0;
        owner_count(c, oa, es, ed, rd, rs, k, timer, mt, ex, &ws);
        acc.prefixes[2] += k;
        acc.extensions[2] += ex;
        acc.prefixes[3] += mt;
        acc.kernel_ms += timer.total_ms();
        acc.kernel_launches += timer.launches();
        cd += ws;
        raw += mt;
      }
      done[qi] = 1;
      if (count_delta) count_delta[qi] = cd;
      if (n_delta) n_delta[qi] = 0;
      if (stats) {
        acc.noop_inserts = hc[0];
        acc.noop_deletes = hc[1];
        acc.raw_emissions = raw;
        acc.matches = raw;
        stats[qi] = acc;
      }
    }
  }
  // With delta lanes (other contexts, each with its own stream), the
  // count-only dQ_i of a large enough batch run depth-first side by side,
  // one host thread per lane, instead of through the fused pipeline: their
  // host-driven stages overlap and their kernels share the device.
  const bool use_lanes = lanes && !lanes->empty() && k >= c->delta_lane_min;
  if (use_lanes) {
    struct Job {
      uint32_t qi;
      int i;
      int64_t ws = 0;
      uint64_t matches = 0;
      gj_stats st{};
    };
    std::vector<Job> jobs;
    for (uint32_t qi = 0; qi < nq; ++qi) {
      bool want_rows = (out_rows && out_rows[qi]) || (out_signs && out_signs[qi]);
      if (want_rows || done[qi]) continue;
      for (int i = 0; i < (int)qs[qi]->atoms.size(); ++i) jobs.push_back(Job{qi, i});
    }
    if (!jobs.empty()) {
      // the seeds and the new version are complete before other streams read them
      GJ_HIP(hipStreamSynchronize(c->stream));
      const size_t nw = std::min(jobs.size(), lanes->size() + 1);
      std::vector<Error> errs(nw);
      std::vector<char> failed(nw, 0);
      auto work = [&](size_t w) {
        gj_ctx* x = w == 0 ? c : (*lanes)[w - 1];
        try {
          if (w) GJ_HIP(hipSetDevice(x->device));
          for (size_t j = w; j < jobs.size(); j += nw) {
            Job& J = jobs[j];
            delta_count_one(x, qs[J.qi], J.i, ov, nv, es, ed, eg, k, J.ws, J.matches, J.st);
          }
        } catch (const Error& e) {
          errs[w] = e;
          failed[w] = 1;
        } catch (const std::exception& e) {
          errs[w] = Error{GJ_EDEVICE, e.what()};
          failed[w] = 1;
        }
      };
      std::vector<std::thread> th;
      try {
        for (size_t w = 1; w < nw; ++w) th.emplace_back(work, w);
      } catch (...) {
        for (auto& t : th) t.join();
        throw Error{GJ_ENOMEM, "cannot start a delta lane thread"};
      }
      work(0);
      for (auto& t : th) t.join();
      for (size_t w = 0; w < nw; ++w)
        if (failed[w]) throw errs[w];
      std::vector<gj_stats> acc(nq);
      std::vector<int64_t> cd(nq, 0);
      std::vector<uint64_t> raw(nq, 0);
      for (const Job& J : jobs) {
        add_stats(acc[J.qi], J.st);
        cd[J.qi] += J.ws;
        raw[J.qi] += J.matches;
        done[J.qi] = 1;
      }
      for (const Job& J : jobs) {
        const uint32_t qi = J.qi;
        if (count_delta) count_delta[qi] = cd[qi];
        if (n_delta) n_delta[qi] = 0;
        if (stats) {
          gj_stats a = acc[qi];
          a.noop_inserts = hc[0];
          a.noop_deletes = hc[1];
          a.raw_emissions = raw[qi];
          a.matches = raw[qi];
          stats[qi] = a;
        }
      }
    }
  }
  // Queries that only need count deltas: every dQ_i of all of them runs as
  // one fused, graph-captured pipeline with signed seeds.
  if (c->delta_fused && !use_lanes) {
    std::vector<gj::ReqSpec> specs;
    std::vector<uint32_t> owner;
    for (uint32_t qi = 0; qi < nq; ++qi) {
      bool want_rows = (out_rows && out_rows[qi]) || (out_signs && out_signs[qi]);
      if (want_rows || done[qi]) continue;
      const gj_query* q = qs[qi];
      for (int i = 0; i < (int)q->atoms.size(); ++i) {
        ReqSpec r{make_plan(q, delta_order(q, i), i), Views{&ov, &nv, i}};
        r.row = es;
        r.col = ed;
        r.w = eg;
        r.lo = 0;
        r.len = k;
        specs.push_back(std::move(r));
        owner.push_back(qi);
      }
    }
    if (!specs.empty()) {
      std::vector<uint64_t> cnts(specs.size());
      std::vector<int64_t> ws(specs.size());
      std::vector<gj_stats> sts(specs.size());
      bool ov_b = false;
      if (!c->batch) c->batch = new BatchExec();
      c->batch->run_specs(c, specs, cnts.data(), ws.data(), sts.data(), ov_b);
      if (!ov_b) {
        std::vector<gj_stats> acc(nq);
        std::vector<int64_t> cd(nq, 0);
        std::vector<uint64_t> raw(nq, 0);
        std::vector<char> fused(nq, 0);
        for (size_t x = 0; x < specs.size(); ++x) {
          uint32_t qi = owner[x];
          add_stats(acc[qi], sts[x]);
          acc[qi].kernel_ms = sts[x].kernel_ms;  // one launch for all
          acc[qi].kernel_launches = 1;
          cd[qi] += ws[x];
          raw[qi] += cnts[x];
          fused[qi] = 1;
          done[qi] = 1;
        }
        for (uint32_t qi = 0; qi < nq; ++qi) {
          if (!fused[qi]) continue;
          if (count_delta) count_delta[qi] = cd[qi];
          if (n_delta) n_delta[qi] = 0;
          if (stats) {
            acc[qi].noop_inserts = hc[0];
            acc[qi].noop_deletes = hc[1];
            acc[qi].raw_emissions = raw[qi];
            acc[qi].matches = raw[qi];
            stats[qi] = acc[qi];
          }
        }
      } else {
        ++c->batch_fallbacks;
      }
    }
  }
  for (uint32_t qi = 0; qi < nq; ++qi) {
    if (done[qi]) continue;
    const gj_query* q = qs[qi];
    bool want_rows = (out_rows && out_rows[qi]) || (out_signs && out_signs[qi]);
    gj_stats acc{};
    int64_t cd = 0;
    uint64_t raw = 0;
    // every dQ_i's signed rows, concatenated (freed on every exit)
    DevMem all_rows_m, all_signs_m;
    uint64_t all_n = 0, all_cap = 0;
    for (int i = 0; i < (int)q->atoms.size(); ++i) {
      PlanH P = make_plan(q, delta_order(q, i), i);
      Views V{&ov, &nv, i};
      Runner R(c, P, V, true, want_rows, std::max<uint64_t>(1, std::min<uint64_t>(c->seed_chunk, k)));
      if (want_rows) R.own_rows(~0ull, true);
      R.seed(es, ed, eg, k);
      uint64_t matches = 0;
      int64_t ws = 0;
      R.finish(matches, ws);
      add_stats(acc, R.st);
      raw += matches;
      if (!want_rows) {
        cd += ws;
        continue;
      }
      if (matches) {
        if (all_n + matches > all_cap) {
          uint64_t ncap = std::max<uint64_t>(all_n + matches, all_cap * 2);
          DevMem nr(c, ncap * q->m * sizeof(uint32_t));
          DevMem ns(c, ncap);
          if (all_n) {
            GJ_HIP(hipMemcpyAsync(nr.get(), all_rows_m.get(), all_n * q->m * sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, c->stream));
            GJ_HIP(hipMemcpyAsync(ns.get(), all_signs_m.get(), all_n, hipMemcpyDeviceToDevice, c->stream));
            GJ_HIP(hipStreamSynchronize(c->stream));
          }
          all_rows_m = std::move(nr);
          all_signs_m = std::move(ns);
          all_cap = ncap;
        }
        GJ_HIP(hipMemcpyAsync(all_rows_m.as<uint32_t>() + all_n * q->m, R.rows, matches * q->m * sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, c->stream));
        GJ_HIP(hipMemcpyAsync(all_signs_m.as<int8_t>() + all_n, R.rsign, matches, hipMemcpyDeviceToDevice,
                              c->stream));
        GJ_HIP(hipStreamSynchronize(c->stream));
        all_n += matches;
      }
    }
    uint64_t nd = 0;
    if (want_rows) {
      uint32_t* all_rows = all_rows_m.as<uint32_t>();
      int8_t* all_signs = all_signs_m.as<int8_t>();
      {
        gj_ctx::LastDelta& ld = c->last_delta[qi];
        ld.kept = true;
        ld.m = q->m;
        if (all_n) {
          sort_rows(c, all_rows, all_signs, all_n, q->m, n);
          ld.rows = (uint32_t*)ws_get(c, "dq_res_rows" + std::to_string(qi), all_n * q->m * sizeof(uint32_t));
          ld.signs = (int8_t*)ws_get(c, "dq_res_signs" + std::to_string(qi), all_n);
          nd = consolidate_rows(c, all_rows, all_signs, all_n, q->m, ld.rows, ld.signs, all_n, &cd);
          ld.n = nd;
          uint64_t ucap = cap ? cap[qi] : 0;
          uint64_t w = std::min(nd, ucap);
          uint32_t* orow = out_rows ? out_rows[qi] : nullptr;
          int8_t* osg = out_signs ? out_signs[qi] : nullptr;
          hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
          if (orow && w) GJ_HIP(hipMemcpyAsync(orow, ld.rows, w * q->m * sizeof(uint32_t), kind, c->stream));
          if (osg && w) GJ_HIP(hipMemcpyAsync(osg, ld.signs, w, kind, c->stream));
          GJ_HIP(hipStreamSynchronize(c->stream));
          if (nd > ucap) overflow = true;
        }
      }
    }
    if (count_delta) count_delta[qi] = cd;
    if (n_delta) n_delta[qi] = nd;
    if (stats) {
      acc.noop_inserts = hc[0];
      acc.noop_deletes = hc[1];
      acc.raw_emissions = raw;
      acc.matches = raw;
      stats[qi] = acc;
    }
  }
  if (patched) {
    guard.armed = false;
    lsm_commit(g, commit);
  } else {
    g->cur = target;
    if (L.on) {  // the appended rows are in the new version now
      lsm_clear(c, g);
      ++c->lsm_folds;
    }
  }
  g->version += 1;
}

}  // namespace gj
