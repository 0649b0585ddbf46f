// Host side of the plain Generic Join path: query plans, the depth-first
// batch scheduler over bounded frontiers, and the static entry point.
//
// Scheduling follows the BiGJoin batching rule (Sec. 3.2 with the batching
// optimisation of Sec. 3.1.2): candidates of a stage are proposed in batches
// of at most B = frontier_cap, and each batch's survivors are extended to the
// end before the next batch of the shallower stage is proposed (the deepest
// stage with work always goes first).  Every frontier buffer therefore holds
// at most B prefixes, and memory stays O(m * B) beside the indexes (Lemma 3.1).
#include <algorithm>
#include <cstring>

#include "engine.h"
#include "gj_internal.h"
#include "owner.h"
#include "run.h"

namespace gj {

PlanH make_plan(const gj_query* q, const std::vector<int>& order, int forced_seed) {
  PlanH P;
  P.m = q->m;
  P.order = order;
  std::vector<int> pos(q->m);
  for (int j = 0; j < q->m; ++j) pos[order[j]] = j;
  P.bind.assign(q->m, {});
  for (int i = 0; i < (int)q->atoms.size(); ++i) {
    int s = q->atoms[i].src_attr, d = q->atoms[i].dst_attr;
    int j = std::max(pos[s], pos[d]);
    if (j == 1) {
      bool is_seed = forced_seed >= 0 ? i == forced_seed : P.seed_atom < 0;
      if (is_seed) {
        P.seed_atom = i;
        P.seed_fwd = pos[s] == 0;
      } else {
        // keep (x0, x1) iff edge(x_s, x_d): x_d in out(x_s)
        P.filters.push_back({i, pos[s], pos[d]});
      }
    } else if (pos[d] == j) {
      P.bind[j].push_back({i, pos[s], 0});  // edge(y, x): x in out(y)
    } else {
      P.bind[j].push_back({i, pos[d], 1});  // edge(x, y): x in in(y)
    }
  }
  // ternary atoms bind their third attribute, after the binary atoms
  for (const gj_tri_atom& t : q->tris) {
    BindH b{-1, pos[t.x_attr], 0, pos[t.y_attr]};
    P.bind[pos[t.z_attr]].push_back(b);
  }
  P.ntri = (int)q->tris.size();
  // trailing run of attributes that share no atom and no inequality
  auto linked = [&](int x, int y) {
    for (const gj_atom& at : q->atoms)
      if ((at.src_attr == x && at.dst_attr == y) || (at.src_attr == y && at.dst_attr == x)) return true;
    for (const gj_less& l : q->less)
      if ((l.lo_attr == x && l.hi_attr == y) || (l.lo_attr == y && l.hi_attr == x)) return true;
    for (const gj_tri_atom& t : q->tris) {
      bool hx = t.x_attr == x || t.y_attr == x || t.z_attr == x;
      bool hy = t.x_attr == y || t.y_attr == y || t.z_attr == y;
      if (hx && hy) return true;
    }
    return false;
  };
  int j0 = q->m - 1;
  while (j0 - 1 >= 2) {
    bool free_ = true;
    for (int t = j0; t < q->m; ++t) free_ = free_ && !linked(order[j0 - 1], order[t]);
    if (!free_) break;
    --j0;
  }
  P.fact_from = q->m - j0 >= 2 ? j0 : 0;
  // a_x < a_y is checked when the later of the two is bound (Sec. 5.4)
  P.above.assign(q->m, 0u);
  P.below.assign(q->m, 0u);
  for (const gj_less& l : q->less) {
    int jx = pos[l.lo_attr], jy = pos[l.hi_attr];
    if (jy > jx)
      P.above[jy] |= 1u << jx;
    else
      P.below[jx] |= 1u << jy;
  }
  for (int j = 2; j < q->m; ++j)
    GJ_CHECK(P.bind[j].size() <= (size_t)kMaxBind, GJ_EUNSUPPORTED, "more than 8 atoms bind one attribute");
  GJ_CHECK(P.filters.size() <= (size_t)kMaxBind, GJ_EUNSUPPORTED, "more than 8 atoms over the first two attributes");
  return P;
}

StageDesc stage_desc(const PlanH& P, const Views& V, int j) {
  StageDesc d;
  memset(&d, 0, sizeof(d));
  d.j = j;
  d.k = (int)P.bind[j].size();
  d.above = P.above[j];
  d.below = P.below[j];
  for (int a = 0; a < kMaxBind; ++a) d.col2[a] = -1;
  for (int a = 0; a < d.k; ++a) {
    const BindH& b = P.bind[j][a];
    d.col[a] = b.col;
    if (b.col2 >= 0) {  // ternary: the triangle index of the version read
      d.col2[a] = b.col2;
      ++d.ntri;
      continue;
    }
    const Version& v = V.of(b.atom);
    d.rp[a] = v.d[b.dir].rp;
    d.adj[a] = v.d[b.dir].col;
    d.pm[a] = v.pmap[b.dir];
    if (V.hash && !d.pm[a] && v.hash_gen == v.gen && v.h[b.dir].desc) {
      d.hd[a] = v.h[b.dir].desc;
      d.hs[a] = v.h[b.dir].slots;
    }
  }
  if (d.ntri) {
    GJ_CHECK(V.tri && V.tri->rp, GJ_EINVAL, "ternary atom without a triangle index");
    d.trp = V.tri->rp;
    d.tcol = V.tri->col;
    d.erp = V.old_v->d[0].rp;
    d.ecol = V.old_v->d[0].col;
  }
  for (int a = d.k; a < kMaxBind; ++a) {
    d.col[a] = 0;
    d.rp[a] = d.rp[0];
    d.adj[a] = d.adj[0];
    d.pm[a] = d.pm[0];
  }
  return d;
}

SeedFilter seed_filter(const PlanH& P, const Views& V) {
  SeedFilter f;
  memset(&f, 0, sizeof(f));
  f.n = (int)P.filters.size();
  f.above = P.above[1];
  f.below = P.below[1];
  for (int a = 0; a < f.n; ++a) {
    const Version& v = V.of(P.filters[a].atom);
    f.key[a] = P.filters[a].key;
    f.val[a] = P.filters[a].val;
    f.rp[a] = v.d[0].rp;
    f.adj[a] = v.d[0].col;
    f.pm[a] = v.pmap[0];
  }
  return f;
}

// Order of dQ_i: the atom's (src, dst), then repeatedly the earliest attribute
// of the global order that shares an atom with a bound attribute.
std::vector<int> delta_order(const gj_query* q, int i) {
  std::vector<int> ord = {q->atoms[i].src_attr, q->atoms[i].dst_attr};
  std::vector<int> bound(q->m, 0);
  bound[ord[0]] = bound[ord[1]] = 1;
  while ((int)ord.size() < q->m) {
    int pick = -1;
    for (int a : q->order) {
      if (bound[a]) continue;
      bool adj = false;
      for (auto& at : q->atoms)
        if ((at.src_attr == a && bound[at.dst_attr]) || (at.dst_attr == a && bound[at.src_attr])) adj = true;
      if (adj) {
        pick = a;
        break;
      }
    }
    GJ_CHECK(pick >= 0, GJ_EINVAL, "query graph is not connected");
    ord.push_back(pick);
    bound[pick] = 1;
  }
  return ord;
}

// Plans of the static order and of every delta query must fit the kernels.
void PlanHCheck(const gj_query* q) {
  make_plan(q, q->order, -1);
  if (!q->tris.empty()) return;  // no delta queries over the triangle relation
  for (int i = 0; i < (int)q->atoms.size(); ++i) make_plan(q, delta_order(q, i), i);
}

// ---------------------------------------------------------------- Runner
Runner::Runner(gj_ctx* c_, const PlanH& P_, const Views& V_, bool weighted_, bool collect_, uint64_t seed_cap)
    : c(c_), P(P_), V(V_), weighted(weighted_), collect(collect_), timer(c_) {
  map.m = P.m;
  for (int k = 0; k < P.m; ++k) map.attr[k] = P.order[k];
  uint64_t fcap = c->frontier_cap;
  for (int j = 2; j < P.m; ++j) {
    Level& l = L[j];
    l.cap = j == 2 ? seed_cap : fcap;
    std::string t = "L" + std::to_string(j) + "_";
    l.F = (uint32_t*)ws_get(c, t + "F", l.cap * j * sizeof(uint32_t) + 16);
    l.Fw = weighted ? (int8_t*)ws_get(c, t + "Fw", l.cap + 16) : nullptr;
    l.minc = (uint32_t*)ws_get(c, t + "minc", l.cap * sizeof(uint32_t) + 16);
    l.mini = (uint8_t*)ws_get(c, t + "mini", l.cap + 16);
    l.off = (uint64_t*)ws_get(c, t + "off", (l.cap + 1) * sizeof(uint64_t));
    uint64_t words = fcap / 64 + 2;
    l.mask = (uint64_t*)ws_get(c, t + "mask", words * sizeof(uint64_t));
    l.wcnt = (uint32_t*)ws_get(c, t + "wcnt", words * sizeof(uint32_t));
    l.woff = (uint64_t*)ws_get(c, t + "woff", (words + 1) * sizeof(uint64_t));
    // the allocation-free count keeps to the frontier-only form (its batch
    // bounds are sized without the records)
    if (!c->arena.on && P.ntri == 0) {
      l.pl = (uint32_t*)ws_get(c, t + "pl", l.cap * sizeof(uint32_t) + 16);
      l.ent = (uint64_t*)ws_get(c, t + "ent", l.cap * P.bind[j].size() * sizeof(uint64_t) + 16);
    }
  }
  if (P.m == 2) {
    Level& l = L[2];
    l.cap = seed_cap;
    l.F = (uint32_t*)ws_get(c, "L2_F", l.cap * 2 * sizeof(uint32_t) + 16);
    l.Fw = weighted ? (int8_t*)ws_get(c, "L2_Fw", l.cap + 16) : nullptr;
  }
  acc = (unsigned long long*)ws_get(c, "acc", 4 * sizeof(unsigned long long));
  GJ_HIP(hipMemsetAsync(acc, 0, 4 * sizeof(unsigned long long), c->stream));
  seed_flags = (uint32_t*)ws_get(c, "seed_flags", (seed_cap + 1) * sizeof(uint32_t));
  seed_off = (uint64_t*)ws_get(c, "seed_off", (seed_cap + 1) * sizeof(uint64_t));
}

static uint64_t arena_piece(uint64_t b) { return (b + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// Mirrors the Runner constructor's buffers for a count-only, unweighted run.
uint64_t runner_scratch_bytes(int m, uint64_t seed_cap, uint64_t fcap) {
  uint64_t t = 0, words = fcap / 64 + 2;
  for (int j = 2; j < m; ++j) {
    uint64_t cap = j == 2 ? seed_cap : fcap;
    t += arena_piece(cap * j * sizeof(uint32_t) + 16) + arena_piece(cap * sizeof(uint32_t) + 16) +
         arena_piece(cap + 16) + arena_piece((cap + 1) * sizeof(uint64_t)) + arena_piece(words * sizeof(uint64_t)) +
         arena_piece(words * sizeof(uint32_t)) + arena_piece((words + 1) * sizeof(uint64_t));
  }
  if (m == 2) t += arena_piece(seed_cap * 2 * sizeof(uint32_t) + 16);
  t += arena_piece(4 * sizeof(unsigned long long)) + arena_piece((seed_cap + 1) * sizeof(uint32_t)) +
       arena_piece((seed_cap + 1) * sizeof(uint64_t));
  return t + scan_scratch_bytes(std::max(seed_cap, fcap) + 1);
}

Runner::~Runner() {
  if (rows_owned) dev_free(c, rows);
  if (signs_owned) dev_free(c, rsign);
}

void Runner::use_rows(uint32_t* dev_rows, int8_t* dev_signs, uint64_t cap) {
  rows = dev_rows;
  rsign = dev_signs;
  rcap = cap;
  rows_alloc = cap;
}

void Runner::own_rows(uint64_t cap, bool with_signs) {
  rows_owned = true;
  signs_owned = with_signs;
  rcap = cap;
  rows_alloc = 0;
  want_signs = with_signs;
}

// grows an internal row buffer (keeping its contents) to hold `need` rows
void Runner::ensure_rows(uint64_t need) {
  if (!rows_owned || need <= rows_alloc) return;
  uint64_t want = std::max<uint64_t>(need, rows_alloc * 2);
  want = std::min<uint64_t>(std::max<uint64_t>(want, 1024), rcap);
  if (want <= rows_alloc) return;
  DevMem nr(c, want * P.m * sizeof(uint32_t));
  DevMem ns;
  if (want_signs) ns = DevMem(c, want);
  if (rows_alloc) {
    GJ_HIP(hipMemcpyAsync(nr.get(), rows, rows_alloc * P.m * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
    if (ns.get()) GJ_HIP(hipMemcpyAsync(ns.get(), rsign, rows_alloc, hipMemcpyDeviceToDevice, c->stream));
    GJ_HIP(hipStreamSynchronize(c->stream));
  }
  dev_free(c, rows);
  dev_free(c, rsign);
  rows = (uint32_t*)nr.release();
  rsign = (int8_t*)ns.release();
  rows_alloc = want;
}

void Runner::seed(const uint32_t* x0, const uint32_t* x1, const int8_t* w, uint64_t cnt) {
  uint64_t chunk = L[2].cap;
  SeedFilter f = seed_filter(P, V);
  for (uint64_t s = 0; s < cnt; s += chunk) {
    uint64_t k = std::min(chunk, cnt - s);
    launch_seed(c, x0 + s, x1 + s, w ? w + s : nullptr, k, f, seed_flags, seed_off, L[2].F, L[2].cap,
                weighted ? L[2].Fw : nullptr);
    uint64_t n2 = read_u64(c, seed_off + k);
    stage(2, n2);
  }
}

void Runner::stage(int j, uint64_t n) {
  st.prefixes[j] += n;
  Level& l = L[j];
  if (j == P.m) {  // two-attribute query: P_2 is the result
    if (collect) ensure_rows(std::min(rcap, nrows + n));
    launch_rows_from_frontier(c, l.F, l.cap, n, l.Fw, map, collect ? rows : nullptr, collect ? rsign : nullptr,
                              nrows, collect ? std::min(rcap, rows_alloc) : 0, acc);
    nrows += n;
    return;
  }
  if (n == 0) return;
  if (!collect && !weighted && c->factorise && P.fact_from && j == P.fact_from) {
    factorised(j, n);
    return;
  }
  StageDesc d = desc(j, j);
  launch_count_min(c, l.F, l.cap, n, d, l.minc, l.mini);
  scan_u32_to_u64(c, l.minc, l.off, n);
  uint64_t W = read_u64(c, l.off + n);
  st.extensions[j] += W;
  if (W == 0) return;
  // a static read that tests membership counts its candidates towards the
  // version's index, built once they pay for it (the records are written
  // again to name the new tables; the counts do not change)
  if (V.graph && d.k >= 2 && !d.hd[0] && !d.hd[1] && hash_note_work(c, V.graph, *V.old_v, W)) {
    d = desc(j, j);
    if (d.ent) launch_count_min(c, l.F, l.cap, n, d, l.minc, l.mini);
  }
  bool final = j + 1 == P.m;
  RunDesc rd;
  // Static counts only: the seeds of a delta query are one batch of changes,
  // whose prefixes rarely share a source, so its runs hold a few prefixes
  // each and staging them was measured slower than the per-candidate kernel.
  if (final && !collect && !weighted && c->run_stage && c->strategy != 1 && !c->arena.on &&
      W >= c->run_stage_min && run_desc(d, rd)) {
    // prefix runs sharing their old sets take the run kernels; the rest of
    // the candidates the per-candidate kernel
    uint64_t* off2 = (uint64_t*)ws_get(c, "run_off2", (l.cap + 1) * sizeof(uint64_t));
    uint64_t W2 = 0;
    if (run_count(c, l.F, l.cap, n, l.off, l.minc, d, rd, weighted ? l.Fw : nullptr, acc, off2, W2, timer)) {
      if (W2) {
        timer.start();
        launch_propose(c, weighted ? 2 : 1, l.F, l.cap, n, off2, l.mini, d, 0, W2, nullptr, nullptr, l.Fw, acc);
        timer.stop();
      }
      return;
    }
  }
  if (final && !collect) {
    timer.start();
    launch_propose(c, weighted ? 2 : 1, l.F, l.cap, n, l.off, l.mini, d, 0, W, nullptr, nullptr, l.Fw, acc);
    timer.stop();
    return;
  }
  uint64_t piece = c->frontier_cap;
  for (uint64_t w0 = 0; w0 < W; w0 += piece) {
    uint64_t w1 = std::min(W, w0 + piece);
    uint64_t words = (w1 - w0 + 63) >> 6;
    timer.start();
    launch_propose(c, 0, l.F, l.cap, n, l.off, l.mini, d, w0, w1, l.mask, l.wcnt, nullptr, nullptr);
    timer.stop();
    scan_u32_to_u64(c, l.wcnt, l.woff, words);
    uint64_t T = read_u64(c, l.woff + words);
    if (T == 0) continue;
    if (final) {
      st.prefixes[j + 1] += T;
      ensure_rows(std::min(rcap, nrows + T));
      launch_emit(c, true, l.F, l.cap, n, l.off, l.mini, d, w0, w1, l.mask, l.woff, l.Fw, rows, 0, rsign, map,
                  nrows, std::min(rcap, rows_alloc));
      nrows += T;
    } else {
      Level& nl = L[j + 1];
      launch_emit(c, false, l.F, l.cap, n, l.off, l.mini, d, w0, w1, l.mask, l.woff, l.Fw, nl.F, nl.cap,
                  weighted ? nl.Fw : nullptr, map, 0, 0);
      stage(j + 1, T);
    }
  }
}

// Factorised count (Sec. 5.4): the attributes at positions j0..m-1 share no
// atom, so each one's extension set is a function of the prefix in P_j0 and a
// prefix contributes the product of their extension counts.  Per trailing
// attribute: count-minimisation, scan, and a propose pass that counts the
// survivors of every prefix; then one pass sums the products.  The prefixes
// inside the run are never materialised.
void Runner::factorised(int j0, uint64_t n) {
  Level& l = L[j0];
  int T = P.m - j0;
  uint32_t* cnt = (uint32_t*)ws_get(c, "fact_cnt", (uint64_t)T * l.cap * sizeof(uint32_t) + 16);
  bool zero = false;
  for (int t = j0; t < P.m; ++t) {
    StageDesc d = desc(t, j0);  // its columns and inequalities all lie before j0
    launch_count_min(c, l.F, l.cap, n, d, l.minc, l.mini);
    scan_u32_to_u64(c, l.minc, l.off, n);
    uint64_t W = read_u64(c, l.off + n);
    st.extensions[t] += W;
    if (W == 0) zero = true;
    if (zero) continue;  // the products are all zero; the proposals are still counted
    uint32_t* ct = cnt + (uint64_t)(t - j0) * l.cap;
    GJ_HIP(hipMemsetAsync(ct, 0, n * sizeof(uint32_t), c->stream));
    timer.start();
    launch_propose(c, 3, l.F, l.cap, n, l.off, l.mini, d, 0, W, nullptr, ct, nullptr, nullptr);
    timer.stop();
  }
  if (!zero) launch_factor_sum(c, cnt, l.cap, n, T, acc);
}

// Stage j's descriptor over the prefixes of level lvl, with that level's
// record buffers when every binding atom is binary, the buffers hold one
// record per atom, and every row it may read stays below 2^31 entries.
StageDesc Runner::desc(int j, int lvl) {
  StageDesc d = stage_desc(P, V, j);
  const Level& l = L[lvl];
  if (!l.ent || d.ntri || P.bind[j].size() > P.bind[lvl].size()) return d;
  for (const BindH& b : P.bind[j]) {
    const Version& v = V.of(b.atom);
    if (v.max_deg[0] >= (1u << 30) || v.max_deg[1] >= (1u << 30)) return d;
  }
  d.pl = l.pl;
  d.ent = l.ent;
  d.es = l.cap;
  return d;
}

// counts: acc[0] unsigned matches, acc[1] signed weight sum
void Runner::finish(uint64_t& matches, int64_t& wsum) {
  unsigned long long h[2];
  read_bytes(c, h, acc, sizeof(h));
  if (collect) {
    matches = nrows;
    wsum = 0;
  } else {
    matches = P.m == 2 ? nrows : h[0];
    wsum = (int64_t)h[1];
  }
  if (P.m >= 3) st.prefixes[P.m] = matches;
  st.kernel_ms = timer.total_ms();
  st.kernel_launches = timer.launches();
}

static bool identity(const std::vector<int>& o) {
  for (int i = 0; i < (int)o.size(); ++i)
    if (o[i] != i) return false;
  return true;
}

void run_static(gj_ctx* c, const gj_graph* g, const gj_query* q, int mode, uint64_t lo, uint64_t hi,
                uint32_t* out, uint64_t cap, int out_on_device, gj_stats* st, bool& overflow, const Version* ver) {
  PlanH P = make_plan(q, q->order, -1);
  const Version& v = ver ? *ver : g->ver[g->cur];
  Views V{&v, &v, -1};
  if (P.ntri) {
    GJ_CHECK(!ver, GJ_EUNSUPPORTED, "queries with ternary atoms run only through gj_run");
    GJ_CHECK(g->tri.rp && g->tri.version == g->version && g->tri.slot == g->cur, GJ_EINVAL,
             "no triangle index for the graph's current version (gj_graph_index_triangles)");
    V.tri = &g->tri;
  }
  int dir = P.seed_fwd ? 0 : 1;
  hi = std::min<uint64_t>(hi, v.m);
  lo = std::min<uint64_t>(lo, hi);
  bool collect = mode == GJ_MODE_ENUMERATE;
  // Owner-grouped kernel: counting a three-attribute query over all seed
  // edges whose last attribute is bound by one atom on each seed attribute.
  if (!collect && c->strategy != 1 && P.m == 3 && P.filters.empty() && !P.has_ineq() && !P.ntri && lo == 0 &&
      hi == v.m &&
      P.bind[2].size() == 2 && P.bind[2][0].col != P.bind[2][1].col) {
    const BindH& A = P.bind[2][0].col == 0 ? P.bind[2][0] : P.bind[2][1];
    const BindH& B = P.bind[2][0].col == 0 ? P.bind[2][1] : P.bind[2][0];
    OwnerArgs a{v.d[A.dir].rp, v.d[A.dir].col, v.d[B.dir].rp, v.d[B.dir].col,
                v.d[dir].rp,   v.d[dir].col,   v.d[1 - dir].rp, v.d[1 - dir].col, g->n};
    KernelTimer timer(c);
    uint64_t matches = 0, ext = 0;
    if (!ver) {
      // the graph's current slot keeps the plan (tasks by owner and partner
      // range, a function of its degrees) for later counts of this version
      gj_graph* gm = const_cast<gj_graph*>(g);
      std::lock_guard<std::mutex> lk(gm->hash_mu);
      Version& slot = gm->ver[gm->cur];
      owner_count(c, a, v.d[dir].row, v.d[dir].col, v.d[1 - dir].row, v.d[1 - dir].col, v.m, timer, matches, ext,
                  nullptr, &slot.plan, slot.gen, gm->ctx);
    } else {
      owner_count(c, a, v.d[dir].row, v.d[dir].col, v.d[1 - dir].row, v.d[1 - dir].col, v.m, timer, matches,
                  ext);
    }
    gj_stats s{};
    s.prefixes[2] = v.m;
    s.extensions[2] = ext;
    s.prefixes[3] = matches;
    s.matches = matches;
    s.kernel_ms = timer.total_ms();
    s.kernel_launches = timer.launches();
    *st = s;
    return;
  }
  // Transitive 4-clique and diamond: grouped by seed edge (forward seeds,
  // stage bindings all out-lists of exactly the given columns).
  auto out_of = [&](int j, int cols) {
    int seen = 0;
    for (const BindH& b : P.bind[j]) {
      if (b.dir != 0 || b.col2 >= 0 || ((cols >> b.col) & 1) == 0 || ((seen >> b.col) & 1)) return false;
      seen |= 1 << b.col;
    }
    return seen == cols;
  };
  int shape = -1;
  if (!collect && c->strategy != 1 && P.m == 4 && P.filters.empty() && !P.ntri && P.seed_fwd && lo == 0 &&
      hi == v.m) {
    if (out_of(2, 0b011) && out_of(3, 0b111)) shape = 0;       // a2: a0, a1; a3: a0, a1, a2
    else if (out_of(2, 0b001) && out_of(3, 0b110)) shape = 1;  // a2: a0; a3: a1, a2
  }
  // transitive 5-clique: every atom out of an earlier attribute
  if (!collect && c->strategy != 1 && P.m == 5 && P.filters.empty() && !P.ntri && P.seed_fwd && lo == 0 &&
      hi == v.m && out_of(2, 0b0011) && out_of(3, 0b0111) && out_of(4, 0b1111)) {
    KernelTimer timer(c);
    uint64_t o[7];
    uint32_t *x0 = nullptr, *x1 = nullptr;
    uint64_t left = 0;
    const uint64_t* hd = nullptr;  // the version's membership index, as for the 4-clique below
    const uint32_t* hs = nullptr;
    if (c->hash_index && !v.pmap[0] && !v.pmap[1]) {
      hash_ensure(c, g, v);
      if (v.hash_gen == v.gen && v.h[0].desc) {
        hd = v.h[0].desc;
        hs = v.h[0].slots;
      }
    }
    clique5_count(c, v, P.above.data(), P.below.data(), hd, hs, timer, o, x0, x1, left);
    gj_stats s{};
    uint64_t mrest = 0;
    if (left) {  // seeds whose common neighbourhood outgrew LDS
      Runner R(c, P, V, false, false, std::max<uint64_t>(1, std::min<uint64_t>(c->seed_chunk, left)));
      R.seed(x0, x1, nullptr, left);
      int64_t ws = 0;
      R.finish(mrest, ws);
      s = R.st;
    }
    s.prefixes[2] += o[1];
    s.extensions[2] += o[2];
    s.prefixes[3] += o[3];
    s.extensions[3] += o[4];
    s.prefixes[4] += o[5];
    s.extensions[4] += o[6];
    s.matches = mrest + o[0];
    s.prefixes[5] = s.matches;
    s.kernel_ms += timer.total_ms();
    s.kernel_launches += timer.launches();
    *st = s;
    return;
  }
  // 4-cycle: a2 from out(a1), a3 from out(a2) and in(a0)
  auto is_bind = [&](const BindH& b, int col, int dir) { return b.col == col && b.dir == dir && b.col2 < 0; };
  bool cycle4 = !collect && c->strategy != 1 && P.m == 4 && P.filters.empty() && !P.has_ineq() && !P.ntri &&
                P.seed_fwd && lo == 0 && hi == v.m && P.bind[2].size() == 1 && is_bind(P.bind[2][0], 1, 0) &&
                P.bind[3].size() == 2 &&
                ((is_bind(P.bind[3][0], 2, 0) && is_bind(P.bind[3][1], 0, 1)) ||
                 (is_bind(P.bind[3][1], 2, 0) && is_bind(P.bind[3][0], 0, 1)));
  if ((shape == 1 && !P.has_ineq()) || cycle4) {  // diamond / 4-cycle: 2-path counts per a0
    KernelTimer timer(c);
    uint64_t o[3];
    if (cycle4)
      cycle4_2p_count(c, v, g->n, timer, o);
    else
      diamond2p_count(c, v, g->n, timer, o);
    gj_stats s{};
    s.prefixes[2] = v.m;
    s.extensions[2] = s.prefixes[3] = o[1];
    s.extensions[3] = o[2];
    s.matches = s.prefixes[4] = o[0];
    s.kernel_ms = timer.total_ms();
    s.kernel_launches = timer.launches();
    *st = s;
    return;
  }
  if (shape >= 0) {
    KernelTimer timer(c);
    uint64_t o[5];
    uint32_t *x0 = nullptr, *x1 = nullptr;
    uint64_t left = 0;
    // the membership index of the version (built here if missing: a whole
    // count probes rows many times over), for the probes of rows in memory
    const uint64_t* hd = nullptr;
    const uint32_t* hs = nullptr;
    if (c->hash_index && !v.pmap[0] && !v.pmap[1]) {
      hash_ensure(c, g, v);
      if (v.hash_gen == v.gen && v.h[0].desc) {
        hd = v.h[0].desc;
        hs = v.h[0].slots;
      }
    }
    edge4_count(c, v, shape, P.above.data(), P.below.data(), hd, hs, timer, o, x0, x1, left);
    gj_stats s{};
    uint64_t mrest = 0;
    if (left) {  // seeds whose common neighbourhood outgrew LDS
      Runner R(c, P, V, false, false, std::max<uint64_t>(1, std::min<uint64_t>(c->seed_chunk, left)));
      R.seed(x0, x1, nullptr, left);
      int64_t ws = 0;
      R.finish(mrest, ws);
      s = R.st;
    }
    s.prefixes[2] += o[4];  // seeds that pass the inequalities (the depth-first rest counted its own)
    s.extensions[2] += o[2];
    s.prefixes[3] += o[1];
    s.extensions[3] += o[3];
    s.matches = mrest + o[0];
    s.prefixes[4] = s.matches;
    s.kernel_ms += timer.total_ms();
    s.kernel_launches += timer.launches();
    *st = s;
    return;
  }
  uint64_t seed_cap = std::max<uint64_t>(1, std::min<uint64_t>(c->seed_chunk, hi - lo));
  V.graph = g;  // membership indexes are built on demand (Runner::stage)
  Runner R(c, P, V, false, collect, seed_cap);
  if (collect) {
    if (out_on_device)
      R.use_rows(out, nullptr, cap);
    else
      R.own_rows(cap, false);
  }
  R.seed(v.d[dir].row + lo, v.d[dir].col + lo, nullptr, hi - lo);
  uint64_t matches = 0;
  int64_t ws = 0;
  R.finish(matches, ws);
  overflow = collect && matches > cap;
  if (collect && !overflow && matches > 1 && !identity(P.order))
    sort_rows(c, R.rows, nullptr, matches, P.m, g->n);
  if (collect && !overflow && !out_on_device && matches)
    GJ_HIP(hipMemcpyAsync(out, R.rows, matches * P.m * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  GJ_HIP(hipStreamSynchronize(c->stream));
  R.st.matches = matches;
  *st = R.st;
}

}  // namespace gj
