// CPU oracle for Generic Join subgraph queries -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct implementation of what the GPU library
// computes.  Only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark may load it; the GPU library never does.  It shares no code,
// headers or tables with the GPU library.
//
// Paper: Ammar, McSherry, Salihoglu, Joglekar, "Distributed Evaluation of
// Subgraph Queries Using Worst-case Optimal Low-Memory Dataflows" (VLDB 2018).
//
//  * A subgraph query is a multiway self-join of the edge relation: one
//    attribute per query vertex, one atom edge(a_i, a_j) per query edge
//    (Sec. 1.1; Sec. 2.1 notation).  Join semantics: a match is any tuple of
//    vertices that satisfies every atom (no distinctness requirement).
//  * Generic Join (Sec. 2.2, Fig. 1): attributes are bound one at a time in a
//    global order; a prefix is extended by the values present in every
//    extension set Ext^i_j(p) of the relations that bind the next attribute,
//    proposing from the smallest set and checking the proposals against the
//    others.
//  * The evaluated implementation seeds P_2 from the edges of an atom over the
//    first two attributes (Sec. 4.2) and runs count-minimisation, proposal and
//    intersection per stage (Sec. 3.1, Sec. 4.1); extension sets are the
//    out- and in-neighbour lists (forward and reverse indices, Sec. 4.1).
//  * Delta-GJ (Sec. 3.3.1): dQ_i = R'_1..R'_{i-1}, dR_i, R_{i+1}..R_n, each
//    ordered starting with R_i's attributes; the signed union of the dQ_i is
//    the change of the output.
//  * Symmetry breaking (Sec. 5.4): a query may carry inequalities a_x < a_y
//    between attributes, applied as filters to the prefixes: a prefix that
//    binds both attributes is dropped unless the inequality holds.  The
//    filters do not change which set is proposed from, so the extension
//    counters are those of the query without them.
//  * Ternary relations (Sec. 5.4): an atom tri(a_x, a_y, a_z) holds when
//    x -> y, x -> z and y -> z are all edges.  It binds a_z once a_x and a_y
//    are bound; its extension set is out(x) intersected with out(y) when
//    x -> y, else empty.  The oracle computes that set from the definition
//    every time (no index).
//  * Factorised counting (Sec. 5.4): when the last attributes of the order
//    share no atom and no inequality, each one's extensions depend only on the
//    prefix before them, so a count multiplies their extension-set sizes
//    instead of enumerating the combinations.  Counters then cover the work
//    done: extensions[t] sums the smallest set of attribute t over the
//    prefixes where the trailing run starts; the prefixes inside the run are
//    not materialised (0); prefixes[m] is the count.
//
// Readings where the paper is silent (each is listed with its reason in the
// design notes): count-minimisation ties go to the lowest atom index; the
// remaining attributes of dQ_i follow the global order, taking next the
// earliest attribute that shares an atom with a bound one; update batches drop
// self-loops, collapse repeats, ignore no-op operations and reject a batch
// that inserts and deletes one edge; output rows are in attribute-index order,
// sorted ascending as unsigned tuples.
#include <algorithm>
#include <iterator>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <thread>
#include <utility>
#include <vector>

namespace {

constexpr int kMaxAttrs = 8;
constexpr int kMaxAtoms = 16;
constexpr int kMaxLess = 28;  // every pair of 8 attributes once

enum { OR_OK = 0, OR_EINVAL = 1, OR_EOVERFLOW = 4 };

// Edge relation held as per-vertex sorted neighbour vectors (out and in).
struct Graph {
  uint32_t n = 0;
  uint64_t m = 0;  // number of edges
  std::vector<std::vector<uint32_t>> out, in;
  uint64_t noop_inserts = 0, noop_deletes = 0, dropped_loops = 0;

  bool has(uint32_t u, uint32_t v) const {
    const auto& l = out[u];
    return std::binary_search(l.begin(), l.end(), v);
  }
  // `s`: the edge set, sorted ascending by (src, dst), no repeats
  void rebuild_lists(const std::vector<std::pair<uint32_t, uint32_t>>& s) {
    out.assign(n, {});
    in.assign(n, {});
    for (auto& e : s) {
      out[e.first].push_back(e.second);
      in[e.second].push_back(e.first);
    }
    for (auto& l : out) std::sort(l.begin(), l.end());
    for (auto& l : in) std::sort(l.begin(), l.end());
    m = s.size();
    stale = true;
  }
  // The edge set in (src, dst) order and in (dst, src) order; position in
  // these is the "edge index" of the forward / reverse direction.  Read off
  // the neighbour lists (already in that order) after every change.
  const std::vector<std::pair<uint32_t, uint32_t>>& fwd_edges() const {
    refresh();
    return fwd_;
  }
  const std::vector<std::pair<uint32_t, uint32_t>>& rev_edges() const {
    refresh();
    return rev_;
  }
  void mark_changed() { stale = true; }

 private:
  mutable std::vector<std::pair<uint32_t, uint32_t>> fwd_, rev_;
  mutable bool stale = true;
  void refresh() const {
    if (!stale) return;
    fwd_.clear();
    rev_.clear();
    fwd_.reserve(m);
    rev_.reserve(m);
    for (uint32_t u = 0; u < n; ++u)
      for (uint32_t v : out[u]) fwd_.push_back({u, v});
    for (uint32_t v = 0; v < n; ++v)
      for (uint32_t u : in[v]) rev_.push_back({v, u});
    stale = false;
  }
};

// One version of the relation for a delta query: the graph as it is, or the
// graph with the neighbour lists of the vertices an update batch touches
// replaced by their lists after the batch (`out_new`, `in_new`).
struct VersionView {
  const Graph* g = nullptr;
  const std::map<uint32_t, std::vector<uint32_t>>* out_new = nullptr;
  const std::map<uint32_t, std::vector<uint32_t>>* in_new = nullptr;
  const std::vector<uint32_t>& out(uint32_t v) const {
    if (out_new) {
      auto it = out_new->find(v);
      if (it != out_new->end()) return it->second;
    }
    return g->out[v];
  }
  const std::vector<uint32_t>& in(uint32_t v) const {
    if (in_new) {
      auto it = in_new->find(v);
      if (it != in_new->end()) return it->second;
    }
    return g->in[v];
  }
  bool has(uint32_t u, uint32_t v) const {
    const auto& l = out(u);
    return std::binary_search(l.begin(), l.end(), v);
  }
};

struct Atom {
  int s, d;
};

struct Query {
  int m = 0;
  std::vector<Atom> atoms;
  std::vector<int> order;  // order[j] = attribute bound at position j
  std::vector<Atom> less;  // (x, y): the value of a_x is below that of a_y
  struct Tri {
    int x, y, z;
  };
  std::vector<Tri> tris;   // tri(a_x, a_y, a_z)
};

// An extension set reference: the neighbour list of the value in prefix
// column `col`, outgoing (`out_dir`) or incoming, in the old or new version;
// or, for a ternary atom (tri >= 0), the third vertices of the pair in
// columns col, col2.
struct Binding {
  int atom;
  int col;
  bool out_dir;
  int tri = -1;
  int col2 = -1;
};

bool valid_query(const Query& q) {
  if (q.m < 2 || q.m > kMaxAttrs) return false;
  if (q.atoms.empty() || (int)q.atoms.size() > kMaxAtoms) return false;
  if ((int)q.order.size() != q.m) return false;
  std::vector<int> seen(q.m, 0);
  for (int a : q.order) {
    if (a < 0 || a >= q.m || seen[a]) return false;
    seen[a] = 1;
  }
  for (auto& at : q.atoms) {
    if (at.s < 0 || at.s >= q.m || at.d < 0 || at.d >= q.m) return false;
    if (at.s == at.d) return false;
  }
  if ((int)q.less.size() > kMaxLess) return false;
  if ((int)(q.atoms.size() + q.tris.size()) > kMaxAtoms) return false;
  for (auto& t : q.tris) {
    if (t.x < 0 || t.x >= q.m || t.y < 0 || t.y >= q.m || t.z < 0 || t.z >= q.m) return false;
    if (t.x == t.y || t.x == t.z || t.y == t.z) return false;
  }
  for (auto& l : q.less)
    if (l.s < 0 || l.s >= q.m || l.d < 0 || l.d >= q.m || l.s == l.d) return false;
  std::vector<int> pos(q.m);
  for (int j = 0; j < q.m; ++j) pos[q.order[j]] = j;
  // the first two attributes must share an atom (P_2 is seeded from edges)
  bool seed = false;
  for (auto& at : q.atoms)
    if (std::max(pos[at.s], pos[at.d]) == 1) seed = true;
  if (!seed) return false;
  // a ternary atom binds its third attribute, after the other two
  for (auto& t : q.tris)
    if (pos[t.z] < std::max(pos[t.x], pos[t.y]) || pos[t.z] < 2) return false;
  // every later attribute needs an atom to an earlier one
  for (int j = 2; j < q.m; ++j) {
    bool any = false;
    for (auto& at : q.atoms)
      if (std::max(pos[at.s], pos[at.d]) == j) any = true;
    for (auto& t : q.tris)
      if (pos[t.z] == j) any = true;
    if (!any) return false;
  }
  return true;
}

// Per-query plan derived from the order: the seed atom (lowest index over the
// first two attributes), filter atoms over the same two, and for every later
// position j the atoms binding order[j] with their bound column.
// An inequality checked when position `later` is bound: the value there must
// be above (above = true) or below the value in prefix column `col`.
struct Ineq {
  int col;
  bool above;
};

struct Plan {
  int seed_atom = -1;
  bool seed_fwd = true;  // P_2 = (u, v) with u -> v (true) or v -> u (false)
  std::vector<int> filters;
  std::vector<std::vector<Binding>> bind;  // bind[j], j = 2..m-1
  std::vector<std::vector<Ineq>> ineq;     // ineq[j], j = 1..m-1
  int fact_from = 0;  // first position of a trailing independent run of >= 2, else 0
};

// Does value e at position j satisfy the inequalities against the prefix?
bool ineq_ok(const Plan& p, int j, const std::vector<uint32_t>& prefix, uint32_t e) {
  for (const Ineq& iq : p.ineq[j]) {
    uint32_t o = prefix[iq.col];
    if (iq.above ? !(e > o) : !(e < o)) return false;
  }
  return true;
}

Plan make_plan(const Query& q) {
  Plan p;
  std::vector<int> pos(q.m);
  for (int j = 0; j < q.m; ++j) pos[q.order[j]] = j;
  for (int i = 0; i < (int)q.atoms.size(); ++i) {
    const Atom& at = q.atoms[i];
    if (std::max(pos[at.s], pos[at.d]) == 1) {
      if (p.seed_atom < 0) {
        p.seed_atom = i;
        p.seed_fwd = pos[at.s] == 0;
      } else {
        p.filters.push_back(i);
      }
    }
  }
  p.bind.assign(q.m, {});
  for (int i = 0; i < (int)q.atoms.size(); ++i) {
    const Atom& at = q.atoms[i];
    int j = std::max(pos[at.s], pos[at.d]);
    if (j < 2) continue;
    // the atom binds attribute order[j]; its other end is already bound
    if (pos[at.d] == j)  // edge(y, x): x ranges over out(y)
      p.bind[j].push_back({i, pos[at.s], true});
    else  // edge(x, y): x ranges over in(y)
      p.bind[j].push_back({i, pos[at.d], false});
  }
  // ternary atoms bind their third attribute, after the binary ones
  for (int i = 0; i < (int)q.tris.size(); ++i) {
    const Query::Tri& t = q.tris[i];
    p.bind[pos[t.z]].push_back({-1, pos[t.x], true, i, pos[t.y]});
  }
  // the longest run of trailing positions whose attributes share no atom and
  // no inequality (positions 0 and 1 are the seed)
  auto linked = [&](int x, int y) {
    for (auto& at : q.atoms)
      if ((at.s == x && at.d == y) || (at.s == y && at.d == x)) return true;
    for (auto& l : q.less)
      if ((l.s == x && l.d == y) || (l.s == y && l.d == x)) return true;
    for (auto& t : q.tris) {
      bool hx = t.x == x || t.y == x || t.z == x, hy = t.x == y || t.y == y || t.z == y;
      if (hx && hy) return true;
    }
    return false;
  };
  int j0 = q.m - 1;
  while (j0 - 1 >= 2) {
    bool free_ = true;
    for (int t = j0; t < q.m; ++t) free_ = free_ && !linked(q.order[j0 - 1], q.order[t]);
    if (!free_) break;
    --j0;
  }
  p.fact_from = q.m - j0 >= 2 ? j0 : 0;
  // a_x < a_y is checked when the later of the two is bound
  p.ineq.assign(q.m, {});
  for (const Atom& l : q.less) {
    int jx = pos[l.s], jy = pos[l.d];
    if (jy > jx)
      p.ineq[jy].push_back({jx, true});   // new a_y must exceed a_x
    else
      p.ineq[jx].push_back({jy, false});  // new a_x must stay below a_y
  }
  return p;
}

// Which version of the relation an atom reads: for delta query dQ_i, atoms
// before i read the new graph, atoms after i the old one (Sec. 3.3.1).
struct Views {
  VersionView v_old;
  VersionView v_new;
  int delta_atom;  // -1: every atom reads v_old
  const VersionView& of(int atom) const {
    return (delta_atom >= 0 && atom < delta_atom) ? v_new : v_old;
  }
};

// The extension set of binding b for a prefix: a neighbour list of the
// graph, or for a ternary atom (static runs only: it reads the one graph) the
// set written into `scratch`.
const std::vector<uint32_t>& ext_list(const Views& v, const Binding& b, const std::vector<uint32_t>& prefix,
                                      std::vector<uint32_t>& scratch) {
  if (b.tri >= 0) {
    const VersionView& g = v.v_old;
    uint32_t x = prefix[b.col], y = prefix[b.col2];
    scratch.clear();
    if (g.has(x, y))
      std::set_intersection(g.out(x).begin(), g.out(x).end(), g.out(y).begin(), g.out(y).end(),
                            std::back_inserter(scratch));
    return scratch;
  }
  const VersionView& g = v.of(b.atom);
  return b.out_dir ? g.out(prefix[b.col]) : g.in(prefix[b.col]);
}

struct Counters {
  uint64_t prefixes[kMaxAttrs + 1] = {0};
  uint64_t extensions[kMaxAttrs + 1] = {0};
  uint64_t matches = 0;
  bool overflow = false;
  void add(uint64_t& slot, uint64_t x) {
    if (__builtin_add_overflow(slot, x, &slot)) overflow = true;
  }
  void merge(const Counters& o) {
    for (int j = 0; j <= kMaxAttrs; ++j) {
      add(prefixes[j], o.prefixes[j]);
      add(extensions[j], o.extensions[j]);
    }
    add(matches, o.matches);
    overflow = overflow || o.overflow;
  }
};

// Extends one prefix (in position order) through stages j..m-1, depth first.
// Count-minimisation picks the smallest extension set (ties: lowest atom
// index), proposes its values in ascending order and keeps a value only if
// every other binding set contains it (Sec. 3.1 steps; Sec. 4.1 operators).
// Count-minimisation and intersection of position j's sets for one prefix:
// returns the number of values kept and adds the proposals to the counters.
uint64_t count_extensions(const Plan& plan, const Views& views, int j,
                          const std::vector<uint32_t>& prefix, Counters& c) {
  const std::vector<Binding>& B = plan.bind[j];
  std::vector<uint32_t> scratch[kMaxAtoms];
  const std::vector<uint32_t>* sets[kMaxAtoms] = {};
  for (size_t i = 0; i < B.size(); ++i) sets[i] = &ext_list(views, B[i], prefix, scratch[i]);
  size_t best = 0;
  for (size_t i = 1; i < B.size(); ++i)
    if (sets[i]->size() < sets[best]->size()) best = i;
  const std::vector<uint32_t>& prop = *sets[best];
  c.add(c.extensions[j], prop.size());
  uint64_t kept = 0;
  for (uint32_t e : prop) {
    bool keep = true;
    for (size_t i = 0; i < B.size() && keep; ++i) {
      if (i == best) continue;
      keep = std::binary_search(sets[i]->begin(), sets[i]->end(), e);
    }
    if (keep && ineq_ok(plan, j, prefix, e)) ++kept;
  }
  return kept;
}

void extend(const Query& q, const Plan& plan, const Views& views, int j,
            std::vector<uint32_t>& prefix, Counters& c, bool collect,
            std::vector<uint32_t>& rows, bool factorise = false) {
  c.add(c.prefixes[j], 1);
  if (factorise && !collect && j == plan.fact_from && j > 0) {
    // the trailing attributes are independent given the prefix: the number
    // of matches extending it is the product of their extension counts
    uint64_t prod = 1;
    for (int t = j; t < q.m; ++t) {
      uint64_t k = count_extensions(plan, views, t, prefix, c);
      if (__builtin_mul_overflow(prod, k, &prod)) c.overflow = true;
    }
    c.add(c.matches, prod);
    c.add(c.prefixes[q.m], prod);
    return;
  }
  if (j == q.m) {
    c.add(c.matches, 1);
    if (collect) {
      // store in attribute-index order
      uint32_t row[kMaxAttrs];
      for (int k = 0; k < q.m; ++k) row[q.order[k]] = prefix[k];
      rows.insert(rows.end(), row, row + q.m);
    }
    return;
  }
  const std::vector<Binding>& B = plan.bind[j];
  std::vector<uint32_t> scratch[kMaxAtoms];
  const std::vector<uint32_t>* sets[kMaxAtoms] = {};
  for (size_t i = 0; i < B.size(); ++i) sets[i] = &ext_list(views, B[i], prefix, scratch[i]);
  size_t best = 0;
  for (size_t i = 1; i < B.size(); ++i)
    if (sets[i]->size() < sets[best]->size()) best = i;  // strict: ties keep the lower binding
  const std::vector<uint32_t>& prop = *sets[best];
  c.add(c.extensions[j], prop.size());
  for (uint32_t e : prop) {
    bool keep = true;
    for (size_t i = 0; i < B.size() && keep; ++i) {
      if (i == best) continue;
      keep = std::binary_search(sets[i]->begin(), sets[i]->end(), e);
    }
    if (!keep || !ineq_ok(plan, j, prefix, e)) continue;
    prefix.push_back(e);
    extend(q, plan, views, j + 1, prefix, c, collect, rows, factorise);
    prefix.pop_back();
  }
}

// Does seed pair (x0, x1) (values of order[0], order[1]) satisfy atom i?
bool pair_ok(const Query& q, const Views& v, int atom, uint32_t x0, uint32_t x1) {
  const Atom& at = q.atoms[atom];
  uint32_t s = at.s == q.order[0] ? x0 : x1;
  uint32_t d = at.s == q.order[0] ? x1 : x0;
  return v.of(atom).has(s, d);
}

// Runs the edge-seeded Generic Join on seed edges [lo, hi) of the seed
// atom's edge list, in the seed atom's version.
void run_seeds(const Query& q, const Plan& plan, const Views& views,
               uint64_t lo, uint64_t hi, Counters& c, bool collect,
               std::vector<uint32_t>& rows, bool factorise) {
  const Graph& g = *views.of(plan.seed_atom).g;
  const auto& E = plan.seed_fwd ? g.fwd_edges() : g.rev_edges();
  std::vector<uint32_t> prefix;
  prefix.reserve(q.m);
  for (uint64_t k = lo; k < hi && k < E.size(); ++k) {
    uint32_t x0 = E[k].first, x1 = E[k].second;
    bool ok = true;
    for (int f : plan.filters) ok = ok && pair_ok(q, views, f, x0, x1);
    prefix.assign({x0});
    if (!ok || !ineq_ok(plan, 1, prefix, x1)) continue;
    prefix.assign({x0, x1});
    extend(q, plan, views, 2, prefix, c, collect, rows, factorise);
  }
}

void sort_rows(std::vector<uint32_t>& rows, int m) {
  size_t n = rows.size() / m;
  std::vector<std::vector<uint32_t>> t(n);
  for (size_t i = 0; i < n; ++i) t[i].assign(rows.begin() + i * m, rows.begin() + (i + 1) * m);
  std::sort(t.begin(), t.end());
  for (size_t i = 0; i < n; ++i) std::copy(t[i].begin(), t[i].end(), rows.begin() + i * m);
}

struct Result {
  int m = 0;
  Counters c;
  std::vector<uint32_t> rows;   // attribute-index order, sorted
  std::vector<int8_t> signs;    // delta results only
  int64_t count_delta = 0;
  uint64_t raw_emissions = 0;   // delta: signed outputs before consolidation
};

// The query's inequalities: lx[k] < ly[k] for k < num_less; its ternary atoms
// tri(tx[k], ty[k], tz[k]) for k < num_tri.
bool parse_query(int num_attrs, const uint8_t* as, const uint8_t* ad, int num_atoms,
                 const uint8_t* order, const uint8_t* lx, const uint8_t* ly, int num_less,
                 Query& q, const uint8_t* tx = nullptr, const uint8_t* ty = nullptr,
                 const uint8_t* tz = nullptr, int num_tri = 0) {
  if (num_attrs < 0 || num_attrs > kMaxAttrs || num_atoms < 0 || num_atoms > kMaxAtoms ||
      num_less < 0 || num_less > kMaxLess)
    return false;
  q.m = num_attrs;
  q.atoms.clear();
  for (int i = 0; i < num_atoms; ++i) q.atoms.push_back({as[i], ad[i]});
  q.order.assign(order, order + num_attrs);
  q.less.clear();
  for (int i = 0; i < num_less; ++i) q.less.push_back({lx[i], ly[i]});
  q.tris.clear();
  if (num_tri < 0 || num_tri > kMaxAtoms) return false;
  for (int i = 0; i < num_tri; ++i) q.tris.push_back({tx[i], ty[i], tz[i]});
  return valid_query(q);
}

// Order of dQ_i: the atom's (src, dst), then repeatedly the earliest attribute
// in the global order that shares an atom with an already-bound attribute.
std::vector<int> delta_order(const Query& q, int i) {
  std::vector<int> ord = {q.atoms[i].s, q.atoms[i].d};
  std::vector<int> bound(q.m, 0);
  bound[ord[0]] = bound[ord[1]] = 1;
  while ((int)ord.size() < q.m) {
    int pick = -1;
    for (int a : q.order) {
      if (bound[a]) continue;
      bool adj = false;
      for (auto& at : q.atoms)
        if ((at.s == a && bound[at.d]) || (at.d == a && bound[at.s])) adj = true;
      if (adj) { pick = a; break; }
    }
    if (pick < 0) return {};
    ord.push_back(pick);
    bound[pick] = 1;
  }
  return ord;
}

}  // namespace

extern "C" {

// Graph: drops self-loops and repeated edges.  Vertex ids must be < n.
void* or_graph_new(uint32_t n, const uint32_t* src, const uint32_t* dst, uint64_t m) {
  std::vector<std::pair<uint32_t, uint32_t>> s;
  s.reserve(m);
  Graph* g = new Graph();
  g->n = n;
  for (uint64_t i = 0; i < m; ++i) {
    if (src[i] >= n || dst[i] >= n) { delete g; return nullptr; }
    if (src[i] == dst[i]) { ++g->dropped_loops; continue; }
    s.push_back({src[i], dst[i]});
  }
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  g->rebuild_lists(s);
  return g;
}

void* or_graph_copy(const void* g) { return new Graph(*(const Graph*)g); }
void or_graph_free(void* g) { delete (Graph*)g; }
uint64_t or_graph_edges(const void* g) { return ((const Graph*)g)->m; }
uint32_t or_graph_vertices(const void* g) { return ((const Graph*)g)->n; }
void or_graph_edge_list(const void* gp, uint32_t* src, uint32_t* dst) {
  const Graph* g = (const Graph*)gp;
  const auto& E = g->fwd_edges();
  for (size_t i = 0; i < E.size(); ++i) {
    src[i] = E[i].first;
    dst[i] = E[i].second;
  }
}

int or_query_valid(int num_attrs, const uint8_t* as, const uint8_t* ad, int num_atoms,
                   const uint8_t* order, const uint8_t* lx, const uint8_t* ly, int num_less,
                   const uint8_t* tx, const uint8_t* ty, const uint8_t* tz, int num_tri) {
  Query q;
  return parse_query(num_attrs, as, ad, num_atoms, order, lx, ly, num_less, q, tx, ty, tz, num_tri) ? 1
                                                                                                  : 0;
}

// Edge-seeded Generic Join over seed edges [seed_lo, seed_hi) of the seed
// atom (clamped to the edge count).  collect != 0 keeps the matching rows.
// Seeds are split over `threads` std::threads in contiguous chunks; the
// result does not depend on the thread count.
void* or_run(const void* gp, int num_attrs, const uint8_t* as, const uint8_t* ad,
             int num_atoms, const uint8_t* order, const uint8_t* lx, const uint8_t* ly,
             int num_less, const uint8_t* tx, const uint8_t* ty, const uint8_t* tz, int num_tri,
             int collect, int factorise, uint64_t seed_lo, uint64_t seed_hi, int threads,
             int* status) {
  const Graph* g = (const Graph*)gp;
  Query q;
  if (!parse_query(num_attrs, as, ad, num_atoms, order, lx, ly, num_less, q, tx, ty, tz, num_tri)) {
    *status = OR_EINVAL;
    return nullptr;
  }
  Plan plan = make_plan(q);
  Views views{VersionView{g}, VersionView{g}, -1};
  const auto& E = plan.seed_fwd ? g->fwd_edges() : g->rev_edges();
  uint64_t hi = std::min<uint64_t>(seed_hi, E.size());
  uint64_t lo = std::min<uint64_t>(seed_lo, hi);
  if (threads < 1) threads = 1;
  uint64_t span = hi - lo;
  if ((uint64_t)threads > span) threads = span ? (int)span : 1;
  std::vector<Counters> cs(threads);
  std::vector<std::vector<uint32_t>> rs(threads);
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) {
    uint64_t a = lo + span * t / threads, b = lo + span * (t + 1) / threads;
    pool.emplace_back([&, t, a, b] {
      run_seeds(q, plan, views, a, b, cs[t], collect != 0, rs[t], factorise != 0);
    });
  }
  for (auto& th : pool) th.join();
  Result* r = new Result();
  r->m = q.m;
  for (int t = 0; t < threads; ++t) {
    r->c.merge(cs[t]);
    r->rows.insert(r->rows.end(), rs[t].begin(), rs[t].end());
  }
  // P_2 counts seeds that passed the filters; prefixes[m] == matches
  if (collect) sort_rows(r->rows, q.m);
  *status = r->c.overflow ? OR_EOVERFLOW : OR_OK;
  return r;
}

// Textbook Generic Join (Fig. 1): starts from P_0 = {()}; an atom whose other
// attribute is not yet bound contributes the projection of the relation on
// the new attribute ({v : out(v) nonempty} or {v : in(v) nonempty}).
// Returns every P_j, j = 1..m, concatenated (position order); sizes[j] = |P_j|.
void* or_run_textbook(const void* gp, int num_attrs, const uint8_t* as, const uint8_t* ad,
                      int num_atoms, const uint8_t* order, uint64_t* sizes, int* status) {
  const Graph* g = (const Graph*)gp;
  Query q;
  q.m = num_attrs;
  for (int i = 0; i < num_atoms; ++i) q.atoms.push_back({as[i], ad[i]});
  q.order.assign(order, order + num_attrs);
  if (num_attrs < 1 || num_attrs > kMaxAttrs) { *status = OR_EINVAL; return nullptr; }
  std::vector<int> pos(q.m);
  for (int j = 0; j < q.m; ++j) pos[q.order[j]] = j;
  std::vector<uint32_t> has_out, has_in;
  for (uint32_t v = 0; v < g->n; ++v) {
    if (!g->out[v].empty()) has_out.push_back(v);
    if (!g->in[v].empty()) has_in.push_back(v);
  }
  Result* r = new Result();
  r->m = q.m;
  std::vector<std::vector<uint32_t>> P = {{}};  // P_0 = {()}
  for (int j = 0; j < q.m; ++j) {
    int x = q.order[j];
    std::vector<std::vector<uint32_t>> next;
    for (auto& p : P) {
      std::vector<const std::vector<uint32_t>*> sets;
      for (auto& at : q.atoms) {
        if (at.s == x && at.d != x) {
          if (pos[at.d] < j) sets.push_back(&g->in[p[pos[at.d]]]);
          else sets.push_back(&has_out);
        } else if (at.d == x && at.s != x) {
          if (pos[at.s] < j) sets.push_back(&g->out[p[pos[at.s]]]);
          else sets.push_back(&has_in);
        }
      }
      if (sets.empty()) { *status = OR_EINVAL; delete r; return nullptr; }
      size_t best = 0;
      for (size_t i = 1; i < sets.size(); ++i)
        if (sets[i]->size() < sets[best]->size()) best = i;
      for (uint32_t e : *sets[best]) {
        bool keep = true;
        for (size_t i = 0; i < sets.size() && keep; ++i)
          if (i != best) keep = std::binary_search(sets[i]->begin(), sets[i]->end(), e);
        if (!keep) continue;
        auto np = p;
        np.push_back(e);
        next.push_back(np);
      }
    }
    P.swap(next);
    sizes[j + 1] = P.size();
    for (auto& p : P) r->rows.insert(r->rows.end(), p.begin(), p.end());
  }
  *status = OR_OK;
  return r;
}

// Applies a signed update batch to the graph (in place) and returns, for the
// given query, the change of its output (Delta-GJ, Sec. 3.3.1).
// Normalisation: self-loops dropped, repeated rows collapse, an insertion of
// a present edge and a deletion of an absent edge are no-ops (counted); a
// batch that both inserts and deletes one edge is rejected (status EINVAL,
// graph unchanged).  Pass num_atoms = 0 to only apply the batch.
// want_rows != 0: the signed outputs of all dQ_i are consolidated per tuple
// (weights summed, zeros dropped) into sorted rows with signs.  Otherwise
// only their sums are kept: count_delta is the sum of the signed outputs
// (consolidation regroups them and cannot change it) and raw_emissions their
// number.  The seeds of each dQ_i are split over `threads` std::threads in
// contiguous chunks; nothing depends on the thread count.
void* or_delta(void* gp, const uint32_t* src, const uint32_t* dst, const int8_t* sign,
               uint64_t b, int num_attrs, const uint8_t* as, const uint8_t* ad,
               int num_atoms, const uint8_t* order, const uint8_t* lx, const uint8_t* ly,
               int num_less, int want_rows, int threads, int* status) {
  Graph* g = (Graph*)gp;
  Query q;
  bool have_query = num_atoms > 0;
  if (have_query && !parse_query(num_attrs, as, ad, num_atoms, order, lx, ly, num_less, q)) {
    *status = OR_EINVAL;
    return nullptr;
  }
  std::set<std::pair<uint32_t, uint32_t>> ins, del;
  for (uint64_t i = 0; i < b; ++i) {
    if (src[i] >= g->n || dst[i] >= g->n || (sign[i] != 1 && sign[i] != -1)) {
      *status = OR_EINVAL;
      return nullptr;
    }
    if (src[i] == dst[i]) continue;
    (sign[i] > 0 ? ins : del).insert({src[i], dst[i]});
  }
  for (auto& e : ins)
    if (del.count(e)) { *status = OR_EINVAL; return nullptr; }
  // the signed change dE: inserted edges absent before, deleted edges present
  std::vector<std::pair<std::pair<uint32_t, uint32_t>, int>> dE;
  uint64_t noop_i = 0, noop_d = 0;
  for (auto& e : ins) {
    if (g->has(e.first, e.second)) ++noop_i;
    else dE.push_back({e, +1});
  }
  for (auto& e : del) {
    if (!g->has(e.first, e.second)) ++noop_d;
    else dE.push_back({e, -1});
  }
  // the new version: every list dE touches, rewritten; the others shared
  std::map<uint32_t, std::vector<uint32_t>> out_new, in_new;
  for (auto& x : dE) {
    uint32_t u = x.first.first, v = x.first.second;
    if (!out_new.count(u)) out_new[u] = g->out[u];
    if (!in_new.count(v)) in_new[v] = g->in[v];
  }
  for (auto& x : dE) {
    uint32_t u = x.first.first, v = x.first.second;
    std::vector<uint32_t>& o = out_new[u];
    std::vector<uint32_t>& i = in_new[v];
    if (x.second > 0) {
      o.insert(std::lower_bound(o.begin(), o.end(), v), v);
      i.insert(std::lower_bound(i.begin(), i.end(), u), u);
    } else {
      o.erase(std::lower_bound(o.begin(), o.end(), v));
      i.erase(std::lower_bound(i.begin(), i.end(), u));
    }
  }
  Result* r = new Result();
  r->m = q.m;
  if (threads < 1) threads = 1;
  if (have_query) {
    std::map<std::vector<uint32_t>, int64_t> acc;
    for (int i = 0; i < (int)q.atoms.size(); ++i) {
      Query qi = q;
      qi.order = delta_order(q, i);
      if ((int)qi.order.size() != q.m) { *status = OR_EINVAL; delete r; return nullptr; }
      Plan plan = make_plan(qi);
      // the seed atom of dQ_i must be atom i itself: other atoms over the
      // same two attributes become filters in their own version
      plan.filters.clear();
      for (int k = 0; k < (int)q.atoms.size(); ++k) {
        if (k == i) continue;
        const Atom& at = q.atoms[k];
        bool same = (at.s == q.atoms[i].s && at.d == q.atoms[i].d) ||
                    (at.s == q.atoms[i].d && at.d == q.atoms[i].s);
        if (same) plan.filters.push_back(k);
      }
      plan.seed_atom = i;
      plan.seed_fwd = true;
      Views views{VersionView{g}, VersionView{g, &out_new, &in_new}, i};
      // per thread: counters, signed match sum, emissions, and (want_rows)
      // the emitted rows with the weight of their seed
      struct Part {
        Counters c;
        int64_t wsum = 0;
        uint64_t raw = 0;
        std::vector<uint32_t> rows;
        std::vector<int8_t> w;
      };
      int nt = (uint64_t)threads > dE.size() ? std::max<int>(1, (int)dE.size()) : threads;
      std::vector<Part> parts(nt);
      std::vector<std::thread> pool;
      for (int t = 0; t < nt; ++t) {
        uint64_t a = dE.size() * t / nt, e = dE.size() * (t + 1) / nt;
        pool.emplace_back([&, t, a, e] {
          Part& P = parts[t];
          for (uint64_t s = a; s < e; ++s) {
            const auto& x = dE[s];
            uint32_t x0 = x.first.first, x1 = x.first.second;
            bool ok = true;
            for (int f : plan.filters) ok = ok && pair_ok(qi, views, f, x0, x1);
            std::vector<uint32_t> prefix = {x0};
            if (!ok || !ineq_ok(plan, 1, prefix, x1)) continue;
            prefix.push_back(x1);
            uint64_t before = P.c.matches;
            size_t rbefore = P.rows.size();
            extend(qi, plan, views, 2, prefix, P.c, want_rows != 0, P.rows);
            uint64_t k = P.c.matches - before;
            P.raw += k;
            P.wsum += (int64_t)k * x.second;
            if (want_rows) P.w.insert(P.w.end(), (P.rows.size() - rbefore) / q.m, (int8_t)x.second);
          }
        });
      }
      for (auto& th : pool) th.join();
      for (Part& P : parts) {
        r->c.merge(P.c);
        r->raw_emissions += P.raw;
        r->count_delta += P.wsum;
        for (size_t k = 0; k < P.w.size(); ++k) {
          std::vector<uint32_t> t(P.rows.begin() + k * q.m, P.rows.begin() + (k + 1) * q.m);
          acc[t] += P.w[k];
        }
      }
    }
    if (want_rows) {
      int64_t sum = 0;
      for (auto& kv : acc) {
        if (kv.second == 0) continue;
        r->rows.insert(r->rows.end(), kv.first.begin(), kv.first.end());
        r->signs.push_back((int8_t)kv.second);
        sum += kv.second;
      }
      if (sum != r->count_delta) { *status = OR_EINVAL; delete r; return nullptr; }
    }
  }
  // commit the new version
  for (auto& kv : out_new) g->out[kv.first].swap(kv.second);
  for (auto& kv : in_new) g->in[kv.first].swap(kv.second);
  for (auto& x : dE) g->m += x.second > 0 ? 1 : (uint64_t)-1;
  g->mark_changed();
  g->noop_inserts += noop_i;
  g->noop_deletes += noop_d;
  *status = OR_OK;
  return r;
}

// Counts of two four-attribute queries by counting 2-paths, the reference
// for graphs where Generic Join itself is too slow on the host:
//  kind 0, the diamond edge(a0,a1), edge(a0,a2), edge(a1,a3), edge(a2,a3):
//    with k(a0, a3) = |{a1 : a0 -> a1 -> a3}| the number of 2-paths, the
//    matches are the pairs of 2-paths from a0 to a3 (a1 = a2 allowed, join
//    semantics), so count = sum over a0, a3 of k(a0, a3)^2;
//  kind 1, the 4-cycle edge(a0,a1), edge(a1,a2), edge(a2,a3), edge(a3,a0):
//    a match is a 2-path a0 -> a1 -> a2 and a 2-path a2 -> a3 -> a0, so
//    count = sum over a0, a2 of k(a0, a2) * k(a2, a0).
// Also the per-stage counters of Generic Join in the order a0, a1, a2, a3
// (edge-seeded form, Sec. 4.2), each summed from its definition:
//  prefixes[2] = |E|;
//  diamond:  a2 ranges over out(a0) alone, so extensions[2] = prefixes[3] =
//            sum over edges (a0, a1) of |out(a0)|; a3 is proposed from the
//            smaller of out(a1), out(a2): extensions[3] = sum over
//            (a0, a1, a2) of min(|out(a1)|, |out(a2)|);
//  4-cycle:  a2 ranges over out(a1): extensions[2] = prefixes[3] = sum over
//            edges (a0, a1) of |out(a1)|; a3 from the smaller of out(a2) and
//            in(a0): extensions[3] = sum over 2-paths (a0, a1, a2) of
//            min(|out(a2)|, |in(a0)|);
//  prefixes[4] = count.
// out[0..5] = count, prefixes[2], extensions[2], prefixes[3], extensions[3],
// prefixes[4].  Work is split over `threads` std::threads by vertex ranges.
int or_twopath(const void* gp, int kind, int threads, uint64_t* out) {
  const Graph* g = (const Graph*)gp;
  if (kind != 0 && kind != 1) return OR_EINVAL;
  if (threads < 1) threads = 1;
  const uint32_t n = g->n;
  std::vector<uint64_t> res(3 * threads, 0);
  std::vector<int> ovf(threads, 0);
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&, t] {
      uint64_t count = 0, ext2 = 0, ext3 = 0;
      bool over = false;
      std::vector<uint32_t> k(n, 0), back(n, 0), seen;
      std::vector<uint32_t> da, db;
      for (uint64_t v = (uint64_t)n * t / threads; v < (uint64_t)n * (t + 1) / threads; ++v) {
        const uint32_t a0 = (uint32_t)v;
        // count: 2-paths from a0, by end vertex
        seen.clear();
        for (uint32_t a1 : g->out[a0])
          for (uint32_t a2 : g->out[a1]) {
            if (k[a2] == 0) seen.push_back(a2);
            ++k[a2];
          }
        if (kind == 0) {
          for (uint32_t e : seen) {
            uint64_t sq = (uint64_t)k[e] * k[e];
            over = over || __builtin_add_overflow(count, sq, &count);
          }
        } else {
          // 2-paths into a0, by start vertex
          for (uint32_t a3 : g->in[a0])
            for (uint32_t a2 : g->in[a3]) ++back[a2];
          for (uint32_t e : seen) {
            uint64_t pr = (uint64_t)k[e] * back[e];
            over = over || __builtin_add_overflow(count, pr, &count);
          }
          for (uint32_t a3 : g->in[a0])
            for (uint32_t a2 : g->in[a3]) back[a2] = 0;
        }
        for (uint32_t e : seen) k[e] = 0;
        // counters, grouped by vertex w = a0
        const uint32_t w = a0;
        if (kind == 0) {
          // the seed edges (w, a1) each propose |out(w)| values of a2; the
          // prefixes (w, a1, a2) range over out(w) x out(w)
          uint64_t d0 = g->out[w].size();
          ext2 += d0 * d0;
          da.clear();
          for (uint32_t a1 : g->out[w]) da.push_back((uint32_t)g->out[a1].size());
          for (uint32_t x : da)
            for (uint32_t y : da) ext3 += std::min(x, y);
        } else {
          // the prefixes (a0, a1, a2) are the 2-paths; here those whose middle
          // vertex a1 is w: a0 ranges over in(w), a2 over out(w)
          uint64_t di = g->in[w].size(), dout = g->out[w].size();
          ext2 += di * dout;
          da.clear();
          db.clear();
          for (uint32_t x : g->in[w]) da.push_back((uint32_t)g->in[x].size());
          for (uint32_t y : g->out[w]) db.push_back((uint32_t)g->out[y].size());
          for (uint32_t x : da)
            for (uint32_t y : db) ext3 += std::min(x, y);
        }
      }
      res[3 * t] = count;
      res[3 * t + 1] = ext2;
      res[3 * t + 2] = ext3;
      ovf[t] = over ? 1 : 0;
    });
  }
  for (auto& th : pool) th.join();
  uint64_t count = 0, ext2 = 0, ext3 = 0;
  bool over = false;
  for (int t = 0; t < threads; ++t) {
    over = over || ovf[t] || __builtin_add_overflow(count, res[3 * t], &count) ||
           __builtin_add_overflow(ext2, res[3 * t + 1], &ext2) ||
           __builtin_add_overflow(ext3, res[3 * t + 2], &ext3);
  }
  out[0] = count;
  out[1] = g->m;
  out[2] = ext2;
  out[3] = ext2;
  out[4] = ext3;
  out[5] = count;
  return over ? OR_EOVERFLOW : OR_OK;
}

uint64_t or_result_matches(const void* r) { return ((const Result*)r)->c.matches; }
void or_result_counters(const void* rp, uint64_t* prefixes, uint64_t* extensions) {
  const Result* r = (const Result*)rp;
  for (int j = 0; j <= kMaxAttrs; ++j) {
    prefixes[j] = r->c.prefixes[j];
    extensions[j] = r->c.extensions[j];
  }
}
uint64_t or_result_num_rows(const void* r) {
  const Result* x = (const Result*)r;
  return x->m ? x->rows.size() / x->m : 0;
}
void or_result_rows(const void* r, uint32_t* out) {
  const Result* x = (const Result*)r;
  std::copy(x->rows.begin(), x->rows.end(), out);
}
void or_result_signs(const void* r, int8_t* out) {
  const Result* x = (const Result*)r;
  std::copy(x->signs.begin(), x->signs.end(), out);
}
int64_t or_result_count_delta(const void* r) { return ((const Result*)r)->count_delta; }
uint64_t or_result_raw_emissions(const void* r) { return ((const Result*)r)->raw_emissions; }
void or_graph_noops(const void* gp, uint64_t* ins, uint64_t* del) {
  *ins = ((const Graph*)gp)->noop_inserts;
  *del = ((const Graph*)gp)->noop_deletes;
}
void or_result_free(void* r) { delete (Result*)r; }

}  // extern "C"
