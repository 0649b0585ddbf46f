// Generic Join prefix-extension stage P_j -> P_{j+1} (Sec. 2.2; the three
// steps of the dataflow primitive, Sec. 3.1): count-minimisation over the
// atoms binding the next attribute, proposal from the smallest extension set,
// and intersection of every proposal with the other sets.
//
// Frontiers are column-major: column c of prefix p at F[c * stride + p].  The
// candidates of a stage form one index space [0, W): prefix p owns
// [off[p], off[p+1]) with off the exclusive scan of its smallest set size, so
// work is split in equal candidate ranges whatever the degree skew (the
// (prefix, range) split of Sec. 3.4, applied inside the GPU).  Each wave takes
// 64 consecutive candidates, keeps a 64-bit ballot of the survivors, and a
// later pass writes survivors in candidate order, so every frontier stays
// sorted in the order's lexicographic order.
#include "gj_internal.h"
#include "prim.h"

namespace gj {

// ---------------------------------------------------------------- seeding P_2
// Seed pairs (x0[i], x1[i]) (the seed atom's edges, or a signed update batch)
// pass the membership filters of the other atoms over the first two attributes.
__global__ void k_seed_flags(const uint32_t* __restrict__ x0, const uint32_t* __restrict__ x1, uint64_t cnt,
                             SeedFilter f, uint32_t* __restrict__ flags) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
    uint32_t x[2] = {x0[i], x1[i]};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < kMaxBind; ++a) {
      if (a < f.n && ok) {
        uint32_t key = f.key[a] ? x[1] : x[0];
        uint32_t val = f.val[a] ? x[1] : x[0];
        uint32_t lo, hi;
        row_range(f.rp[a], f.pm[a], key, lo, hi);
        ok = contains_u32(f.adj[a], lo, hi, val);
      }
    }
    flags[i] = (ok && seed_ineq_ok(f.above, f.below, x[0], x[1])) ? 1u : 0u;
  }
}

__global__ void k_seed_scatter(const uint32_t* __restrict__ x0, const uint32_t* __restrict__ x1,
                               const int8_t* __restrict__ w, uint64_t cnt, const uint32_t* __restrict__ flags,
                               const uint64_t* __restrict__ off, uint32_t* __restrict__ F, uint64_t stride,
                               int8_t* __restrict__ Fw) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gs) {
    if (!flags[i]) continue;
    uint64_t p = off[i];
    F[p] = x0[i];
    F[stride + p] = x1[i];
    if (Fw) Fw[p] = w ? w[i] : (int8_t)1;
  }
}

// Ternary binding a (Sec. 5.4) for prefix p: the third vertices of the pair
// in columns col, col2 are tcol[lo, lo + size); size 0 if the pair is no edge.
__device__ __forceinline__ uint32_t tri_set(const StageDesc& d, int a, const uint32_t* __restrict__ F,
                                            uint64_t stride, uint64_t p, uint64_t& lo) {
  uint32_t x = F[(uint64_t)d.col[a] * stride + p], y = F[(uint64_t)d.col2[a] * stride + p];
  uint32_t b = d.erp[x], e = d.erp[x + 1];
  uint32_t i = lower_bound_u32(d.ecol, b, e, y);
  if (i >= e || d.ecol[i] != y) {
    lo = 0;
    return 0;
  }
  lo = d.trp[i];
  return (uint32_t)(d.trp[i + 1] - lo);
}

// ---------------------------------------------------------------- count-minimisation
// min_c = smallest extension-set size over the binding atoms, min_i = its
// binding index (ties: lowest, i.e. lowest atom index).  With d.ent, also the
// prefix's records: where the proposing row starts, and for every other atom
// its table descriptor or row range, so that the propose and emit kernels
// read one record per atom instead of the frontier, row pointers and maps.
__global__ void k_count_min(const uint32_t* __restrict__ F, uint64_t stride, uint64_t n, StageDesc d,
                            uint32_t* __restrict__ minc, uint8_t* __restrict__ mini) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    uint32_t best = 0xFFFFFFFFu;
    int bi = 0;
    uint32_t rlo[kMaxBind], rlen[kMaxBind], rv[kMaxBind];
#pragma unroll
    for (int a = 0; a < kMaxBind; ++a) {
      rlo[a] = rlen[a] = rv[a] = 0;
      if (a < d.k) {
        uint32_t c;
        if (d.col2[a] >= 0) {
          uint64_t lo;
          c = tri_set(d, a, F, stride, p, lo);
        } else {
          uint32_t v = F[(uint64_t)d.col[a] * stride + p], lo, hi;
          row_range(d.rp[a], d.pm[a], v, lo, hi);
          c = hi - lo;
          rlo[a] = lo;
          rlen[a] = c;
          rv[a] = v;
        }
        if (c < best) {
          best = c;
          bi = a;
        }
      }
    }
    minc[p] = best;
    mini[p] = (uint8_t)bi;
    if (d.ent && best) {
      uint32_t start = 0;
#pragma unroll
      for (int a = 0; a < kMaxBind; ++a) {
        if (a >= d.k) continue;
        if (a == bi) {
          start = rlo[a];
          continue;
        }
        uint64_t r = kEntRange | ((uint64_t)rlen[a] << 32) | rlo[a];
        if (d.hd[a]) {
          uint64_t dd = d.hd[a][rv[a]];
          if (dd) r = dd;
        }
        d.ent[(uint64_t)a * d.es + p] = r;
      }
      d.pl[p] = start;
    }
  }
}

// ---------------------------------------------------------------- propose + intersect
// Candidate g of the range: its prefix p, the proposing atom, the proposed value.
struct Cand {
  uint64_t p;
  uint32_t e;
  int am;
};

template <bool REC>
__device__ __forceinline__ Cand resolve(const uint32_t* __restrict__ F, uint64_t stride,
                                        const uint64_t* __restrict__ off, const uint8_t* __restrict__ mini,
                                        const StageDesc& d, uint64_t plo, uint64_t phi, uint64_t g) {
  Cand c;
  c.p = find_segment(off, plo, phi, g);
  uint32_t k = (uint32_t)(g - off[c.p]);
  c.am = mini[c.p];
  if (REC) {
    const uint32_t* adj;
    switch (c.am) {
#define GJ_PICK(A) \
  case A:          \
    adj = d.adj[A]; \
    break;
      GJ_PICK(1) GJ_PICK(2) GJ_PICK(3) GJ_PICK(4) GJ_PICK(5) GJ_PICK(6) GJ_PICK(7)
#undef GJ_PICK
      default:
        adj = d.adj[0];
        break;
    }
    c.e = adj[d.pl[c.p] + k];
    return c;
  }
  if (d.ntri) {
    bool tri = false;
#pragma unroll
    for (int a = 0; a < kMaxBind; ++a)
      if (a == c.am && d.col2[a] >= 0) tri = true;
    if (tri) {
      uint64_t lo = 0;
#pragma unroll
      for (int a = 0; a < kMaxBind; ++a)
        if (a == c.am) tri_set(d, a, F, stride, c.p, lo);
      c.e = d.tcol[lo + k];
      return c;
    }
  }
  // the proposing atom's arrays by a switch on its (per-lane) index: a
  // select loop over the atoms is turned into an indexed read of the kernel
  // argument, which the compiler copies to private memory in every lane
  const uint32_t* rp;
  const uint32_t* adj;
  const uint64_t* pm;
  int col;
  switch (c.am) {
#define GJ_PICK(A)  \
  case A:           \
    rp = d.rp[A];   \
    adj = d.adj[A]; \
    pm = d.pm[A];   \
    col = d.col[A]; \
    break;
    GJ_PICK(1) GJ_PICK(2) GJ_PICK(3) GJ_PICK(4) GJ_PICK(5) GJ_PICK(6) GJ_PICK(7)
#undef GJ_PICK
    default:
      rp = d.rp[0];
      adj = d.adj[0];
      pm = d.pm[0];
      col = d.col[0];
      break;
  }
  uint32_t v = F[(uint64_t)col * stride + c.p], lo, hi;
  row_range(rp, pm, v, lo, hi);
  c.e = adj[lo + k];
  return c;
}

template <bool REC>
__device__ __forceinline__ bool intersect_all(const uint32_t* __restrict__ F, uint64_t stride, const StageDesc& d,
                                              const Cand& c) {
  bool keep = ineq_ok(F, stride, c.p, d.above, d.below, c.e);
#pragma unroll
  for (int a = 0; a < kMaxBind; ++a) {
    if (a < d.k && a != c.am && keep) {
      if (d.col2[a] >= 0) {
        uint64_t lo;
        uint32_t len = tri_set(d, a, F, stride, c.p, lo);
        keep = contains_u32(d.tcol + lo, 0, len, c.e);
        continue;
      }
      if (REC) {
        const uint64_t r = d.ent[(uint64_t)a * d.es + c.p];
        if (r & kEntRange) {
          const uint32_t lo = (uint32_t)r;
          keep = contains_u32(d.adj[a], lo, lo + (uint32_t)((r >> 32) & 0x7FFFFFFFu), c.e);
        } else {
          keep = hash_member(d.hs[a], r, c.e);
        }
        continue;
      }
      uint32_t u = F[(uint64_t)d.col[a] * stride + c.p], lo, hi;
      uint64_t dd = d.hd[a] ? d.hd[a][u] : 0ull;
      if (dd) {
        keep = hash_member(d.hs[a], dd, c.e);
        continue;
      }
      row_range(d.rp[a], d.pm[a], u, lo, hi);
      keep = contains_u32(d.adj[a], lo, hi, c.e);
    }
  }
  return keep;
}

// Membership tests of U candidates of a lane in lockstep: every step of their
// binary searches issues the U loads before any comparison, so a wave keeps
// U dependent-load chains in flight instead of one (the searches are bound by
// load latency, not bandwidth).  Binary bindings only.
template <int U, bool REC>
__device__ __forceinline__ void intersect_lockstep(const uint32_t* __restrict__ F, uint64_t stride,
                                                   const StageDesc& d, const Cand (&c)[U], bool (&keep)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (keep[u]) keep[u] = ineq_ok(F, stride, c[u].p, d.above, d.below, c[u].e);
#pragma unroll
  for (int a = 0; a < kMaxBind; ++a) {
    if (a < d.k) {
      const uint32_t* arr = d.adj[a];
      uint32_t lo[U], hi[U], n[U];
      uint64_t dd[U];
      bool act[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        act[u] = keep[u] && a != c[u].am;
        lo[u] = hi[u] = n[u] = 0;
        dd[u] = 0;
        if (REC) {
          if (!act[u]) continue;
          const uint64_t r = d.ent[(uint64_t)a * d.es + c[u].p];
          if (r & kEntRange) {
            lo[u] = (uint32_t)r;
            n[u] = (uint32_t)((r >> 32) & 0x7FFFFFFFu);
            hi[u] = lo[u] + n[u];
          } else {
            dd[u] = r;
          }
        } else if (act[u]) {
          uint32_t x = F[(uint64_t)d.col[a] * stride + c[u].p];
          if (d.hd[a]) dd[u] = d.hd[a][x];
          if (!dd[u]) {
            row_range(d.rp[a], d.pm[a], x, lo[u], hi[u]);
            n[u] = hi[u] - lo[u];
          }
        }
      }
      if (d.hd[a]) {
        // rows with a table: probes in lockstep, one bucket load per step
        uint32_t h[U];
        bool pend[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          pend[u] = dd[u] != 0;
          h[u] = pend[u] ? hash_home(c[u].e, (uint32_t)(dd[u] & 0xFF)) : 0u;
        }
        for (;;) {
          bool any = false;
#pragma unroll
          for (int u = 0; u < U; ++u) any = any || pend[u];
          if (!any) break;
          uint4 q[U];
#pragma unroll
          for (int u = 0; u < U; ++u)
            q[u] = pend[u] ? *(const uint4*)(d.hs[a] + 4 * ((dd[u] >> 8) + h[u])) : make_uint4(0, 0, 0, 0);
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (!pend[u]) continue;
            const uint32_t e = c[u].e;
            if (q[u].x == e || q[u].y == e || q[u].z == e || q[u].w == e) {
              keep[u] = true;
              pend[u] = false;
            } else if (q[u].w == kHashEmpty) {
              keep[u] = false;
              pend[u] = false;
            } else {
              h[u] = (h[u] + 1) & ((1u << (uint32_t)(dd[u] & 0xFF)) - 1);
            }
          }
        }
      }
      for (;;) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) any = any || n[u] > 0;
        if (!any) break;
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = n[u] > 0 ? arr[lo[u] + (n[u] >> 1)] : 0u;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (n[u] > 0) {
            uint32_t half = n[u] >> 1;
            if (v[u] < c[u].e) {
              lo[u] += half + 1;
              n[u] -= half + 1;
            } else {
              n[u] = half;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (act[u] && !dd[u]) keep[u] = lo[u] < hi[u] && arr[lo[u]] == c[u].e;
    }
  }
}

// MODE 0: write survivor ballots mask[word] and counts wcnt[word].
// MODE 1: acc[0] += survivors.
// MODE 2: acc[0] += survivors, acc[1] += sum of survivor weights (signed).
// MODE 3: wcnt[p] += survivors of prefix p (a prefix's candidates are
//         consecutive, so a wave adds once per prefix it touches).
// A wave takes U words (64 candidates each) per step, one candidate of each
// per lane, and tests their memberships in lockstep.
template <int MODE, int U, bool REC>
__global__ void __launch_bounds__(kBlock) k_propose(const uint32_t* __restrict__ F, uint64_t stride, uint64_t n,
                                                    const uint64_t* __restrict__ off,
                                                    const uint8_t* __restrict__ mini, StageDesc d, uint64_t w0,
                                                    uint64_t w1, uint64_t* __restrict__ mask,
                                                    uint32_t* __restrict__ wcnt, const int8_t* __restrict__ wt,
                                                    unsigned long long* __restrict__ acc) {
  const int lane = lane_id();
  const uint64_t nwords = (w1 - w0 + 63) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  uint64_t cnt = 0;
  int64_t wsum = 0;
  // each wave walks a contiguous run of words, galloping forward over prefixes
  const uint64_t per = (nwords + nwaves - 1) / nwaves;
  const uint64_t wbeg = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * per;
  const uint64_t wend = wbeg + per < nwords ? wbeg + per : nwords;
  uint64_t plo = 0, phi;
  for (uint64_t wd = wbeg; wd < wend; wd += U) {
    const uint64_t wl = wd + U < wend ? wd + U : wend;  // words [wd, wl) this step
    uint64_t gf = w0 + (wd << 6);
    uint64_t gl = w0 + (wl << 6) - 1 < w1 ? w0 + (wl << 6) - 1 : w1 - 1;
    plo = gallop_segment(off, plo, n, gf);
    phi = gallop_segment(off, plo, n, gl) + 1;
    Cand c[U];
    bool keep[U];
    uint64_t pp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t g = gf + ((uint64_t)u << 6) + lane;
      keep[u] = wd + u < wl && g < w1;
      pp[u] = ~0ull;
      c[u].p = 0;
      c[u].e = 0;
      c[u].am = 0;
      if (keep[u]) {
        c[u] = resolve<REC>(F, stride, off, mini, d, plo, phi, g);
        pp[u] = c[u].p;
      }
    }
    if (U == 1 || d.ntri) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (keep[u]) keep[u] = intersect_all<REC>(F, stride, d, c[u]);
    } else {
      intersect_lockstep<U, REC>(F, stride, d, c, keep);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t b = __ballot(keep[u]);
      if (MODE == 0) {
        if (lane == 0 && wd + u < wl) {
          mask[wd + u] = b;
          wcnt[wd + u] = (uint32_t)__popcll(b);
        }
      } else if (MODE == 3) {
        // lanes of one prefix form a run; the first lane of each run adds the
        // survivors of the run
        uint64_t prev = shfl_up_u64(pp[u], 1);
        bool start = pp[u] != ~0ull && (lane == 0 || prev != pp[u]);
        uint64_t sb = __ballot(start);
        if (start) {
          uint64_t later = lane == 63 ? 0ull : (sb >> (lane + 1)) << (lane + 1);
          int end = later ? __ffsll((unsigned long long)later) - 1 : 64;
          uint64_t run = (end == 64 ? ~0ull : ((1ull << end) - 1)) & ~lanemask_lt();
          uint32_t k = (uint32_t)__popcll(b & run);
          if (k) atomicAdd(wcnt + pp[u], k);
        }
      } else {
        cnt += keep[u] ? 1 : 0;
        if (MODE == 2 && keep[u]) wsum += wt[c[u].p];
      }
    }
  }
  if (MODE == 1 || MODE == 2) {
    uint64_t t = block_sum<kBlock>(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(acc, (unsigned long long)t);
    if (MODE == 2) {
      uint64_t s = block_sum<kBlock>((uint64_t)wsum);
      if (threadIdx.x == 0 && s) atomicAdd(acc + 1, (unsigned long long)s);
    }
  }
}

// Writes the survivors of [w0, w1) in candidate order.
// KIND 0: prefixes p . e into frontier G (j + 1 columns), weights to Gw.
// KIND 1: rows of map.m values in attribute order at rows[(obase+pos)*m],
// signs to osign, only for obase + pos < ocap.
// KIND 2: the new values only, at G[obase + pos] for obase + pos < ocap.
template <int KIND, bool REC>
__global__ void __launch_bounds__(kBlock) k_emit(const uint32_t* __restrict__ F, uint64_t stride, uint64_t n,
                                                 const uint64_t* __restrict__ off, const uint8_t* __restrict__ mini,
                                                 StageDesc d, uint64_t w0, uint64_t w1,
                                                 const uint64_t* __restrict__ mask, const uint64_t* __restrict__ woff,
                                                 const int8_t* __restrict__ wt, uint32_t* __restrict__ G,
                                                 uint64_t gstride, int8_t* __restrict__ Gw, RowMap map,
                                                 uint64_t obase, uint64_t ocap) {
  const int lane = lane_id();
  const uint64_t nwords = (w1 - w0 + 63) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t per = (nwords + nwaves - 1) / nwaves;
  const uint64_t wbeg = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * per;
  const uint64_t wend = wbeg + per < nwords ? wbeg + per : nwords;
  uint64_t plo = 0, phi;
  for (uint64_t wd = wbeg; wd < wend; ++wd) {
    uint64_t b = mask[wd];
    if (b == 0) continue;
    uint64_t gf = w0 + (wd << 6);
    uint64_t gl = gf + 63 < w1 ? gf + 63 : w1 - 1;
    plo = gallop_segment(off, plo, n, gf);
    phi = gallop_segment(off, plo, n, gl) + 1;
    if (!((b >> lane) & 1)) continue;
    Cand c = resolve<REC>(F, stride, off, mini, d, plo, phi, gf + lane);
    uint64_t pos = woff[wd] + __popcll(b & lanemask_lt());
    if (KIND == 2) {
      if (obase + pos < ocap) G[obase + pos] = c.e;
    } else if (KIND == 0) {
      for (int col = 0; col < d.j; ++col) G[(uint64_t)col * gstride + pos] = F[(uint64_t)col * stride + c.p];
      G[(uint64_t)d.j * gstride + pos] = c.e;
      if (Gw) Gw[pos] = wt ? wt[c.p] : (int8_t)1;
    } else {
      uint64_t r = obase + pos;
      if (r >= ocap) continue;
      uint32_t* row = G + r * (uint64_t)map.m;
      for (int col = 0; col < d.j; ++col) row[map.attr[col]] = F[(uint64_t)col * stride + c.p];
      row[map.attr[d.j]] = c.e;
      if (Gw) Gw[r] = wt ? wt[c.p] : (int8_t)1;
    }
  }
}

// Rows of a two-attribute query straight from P_2.
__global__ void k_rows_from_frontier(const uint32_t* __restrict__ F, uint64_t stride, uint64_t n,
                                     const int8_t* __restrict__ wt, RowMap map, uint32_t* __restrict__ rows,
                                     int8_t* __restrict__ osign, uint64_t obase, uint64_t ocap,
                                     unsigned long long* __restrict__ acc) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  int64_t ws = 0;
  uint64_t cnt = 0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    int8_t w = wt ? wt[p] : (int8_t)1;
    ws += w;
    ++cnt;
    uint64_t r = obase + p;
    if (rows && r < ocap) {
      for (int col = 0; col < map.m; ++col) rows[r * map.m + map.attr[col]] = F[(uint64_t)col * stride + p];
      if (osign) osign[r] = w;
    }
  }
  uint64_t t = block_sum<kBlock>(cnt);
  uint64_t s = block_sum<kBlock>((uint64_t)ws);
  if (threadIdx.x == 0) {
    atomicAdd(acc, (unsigned long long)t);
    atomicAdd(acc + 1, (unsigned long long)s);
  }
}

// ---------------------------------------------------------------- host launchers
void launch_seed(gj_ctx* c, const uint32_t* x0, const uint32_t* x1, const int8_t* w, uint64_t cnt,
                 const SeedFilter& f, uint32_t* flags, uint64_t* off, uint32_t* F, uint64_t stride,
                 int8_t* Fw) {
  unsigned gr = grid_for(cnt, kBlock, 1u << 16);
  k_seed_flags<<<gr, kBlock, 0, c->stream>>>(x0, x1, cnt, f, flags);
  scan_u32_to_u64(c, flags, off, cnt);
  k_seed_scatter<<<gr, kBlock, 0, c->stream>>>(x0, x1, w, cnt, flags, off, F, stride, Fw);
  GJ_HIP(hipGetLastError());
}

void launch_count_min(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const StageDesc& d,
                      uint32_t* minc, uint8_t* mini) {
  k_count_min<<<grid_for(n, kBlock, 1u << 16), kBlock, 0, c->stream>>>(F, stride, n, d, minc, mini);
  GJ_HIP(hipGetLastError());
}

static unsigned propose_grid(gj_ctx* c, uint64_t words) {
  uint64_t waves = words;
  uint64_t cap = (uint64_t)c->num_cus * 32;  // persistent-ish: 32 waves per CU
  if (waves > cap * 4) waves = cap * 4;
  return grid_for(waves, kBlock / 64, 1u << 20);
}

void launch_propose(gj_ctx* c, int mode, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off,
                    const uint8_t* mini, const StageDesc& d, uint64_t w0, uint64_t w1, uint64_t* mask,
                    uint32_t* wcnt, const int8_t* wt, unsigned long long* acc) {
  uint64_t words = (w1 - w0 + 63) >> 6;
  unsigned gr = propose_grid(c, words);
  // ternary bindings search one candidate at a time: wider steps only cost occupancy
  int u = d.ntri && c->propose_u > 2 ? 2 : c->propose_u;
  // with per-prefix records, instances without the frontier-resolution code
  switch (mode * 16 + u * 2 + (d.ent ? 1 : 0)) {
#define GJ_PROPOSE(M, U)                                                                                        \
  case M * 16 + U * 2:                                                                                         \
    k_propose<M, U, false><<<gr, kBlock, 0, c->stream>>>(F, stride, n, off, mini, d, w0, w1, mask, wcnt, wt, acc); \
    break;                                                                                                     \
  case M * 16 + U * 2 + 1:                                                                                     \
    k_propose<M, U, true><<<gr, kBlock, 0, c->stream>>>(F, stride, n, off, mini, d, w0, w1, mask, wcnt, wt, acc);  \
    break;
    GJ_PROPOSE(0, 1) GJ_PROPOSE(0, 2) GJ_PROPOSE(0, 4)
    GJ_PROPOSE(1, 1) GJ_PROPOSE(1, 2) GJ_PROPOSE(1, 4)
    GJ_PROPOSE(2, 1) GJ_PROPOSE(2, 2) GJ_PROPOSE(2, 4)
    GJ_PROPOSE(3, 1) GJ_PROPOSE(3, 2) GJ_PROPOSE(3, 4)
#undef GJ_PROPOSE
    default:
      throw Error{GJ_EINVAL, "bad propose mode or width"};
  }
  GJ_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(kBlock) k_factor_sum(const uint32_t* __restrict__ cnt, uint64_t stride,
                                                       uint64_t n, int T, unsigned long long* __restrict__ acc) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  uint64_t s = 0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    uint64_t prod = cnt[p];
    for (int t = 1; t < T; ++t) prod *= cnt[(uint64_t)t * stride + p];
    s += prod;
  }
  uint64_t tot = block_sum<kBlock>(s);
  if (threadIdx.x == 0 && tot) atomicAdd(acc, (unsigned long long)tot);
}

void launch_factor_sum(gj_ctx* c, const uint32_t* cnt, uint64_t stride, uint64_t n, int T,
                       unsigned long long* acc) {
  k_factor_sum<<<grid_for(n, kBlock, 4096), kBlock, 0, c->stream>>>(cnt, stride, n, T, acc);
  GJ_HIP(hipGetLastError());
}

void launch_emit(gj_ctx* c, bool final_rows, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off,
                 const uint8_t* mini, const StageDesc& d, uint64_t w0, uint64_t w1, const uint64_t* mask,
                 const uint64_t* woff, const int8_t* wt, uint32_t* G, uint64_t gstride, int8_t* Gw,
                 const RowMap& map, uint64_t obase, uint64_t ocap) {
  uint64_t words = (w1 - w0 + 63) >> 6;
  unsigned gr = propose_grid(c, words);
#define GJ_EMIT(K, R)                                                                                       \
  k_emit<K, R><<<gr, kBlock, 0, c->stream>>>(F, stride, n, off, mini, d, w0, w1, mask, woff, wt, G, gstride, Gw, \
                                             map, obase, ocap)
  if (final_rows) {
    if (d.ent)
      GJ_EMIT(1, true);
    else
      GJ_EMIT(1, false);
  } else {
    if (d.ent)
      GJ_EMIT(0, true);
    else
      GJ_EMIT(0, false);
  }
#undef GJ_EMIT
  GJ_HIP(hipGetLastError());
}

void launch_emit_values(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off,
                        const uint8_t* mini, const StageDesc& d, uint64_t w0, uint64_t w1, const uint64_t* mask,
                        const uint64_t* woff, uint32_t* out, uint64_t obase, uint64_t ocap) {
  uint64_t words = (w1 - w0 + 63) >> 6;
  unsigned gr = propose_grid(c, words);
  RowMap map{};
  GJ_CHECK(!d.ent, GJ_EINVAL, "per-prefix records with ternary bindings");
  k_emit<2, false><<<gr, kBlock, 0, c->stream>>>(F, stride, n, off, mini, d, w0, w1, mask, woff, nullptr, out, 0,
                                                 nullptr, map, obase, ocap);
  GJ_HIP(hipGetLastError());
}

void launch_rows_from_frontier(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const int8_t* wt,
                               const RowMap& map, uint32_t* rows, int8_t* osign, uint64_t obase, uint64_t ocap,
                               unsigned long long* acc) {
  k_rows_from_frontier<<<grid_for(n, kBlock, 1u << 14), kBlock, 0, c->stream>>>(F, stride, n, wt, map, rows,
                                                                                 osign, obase, ocap, acc);
  GJ_HIP(hipGetLastError());
}

}  // namespace gj
