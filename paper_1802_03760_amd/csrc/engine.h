// Query plans and the depth-first stage runner shared by the static and the
// delta entry points.
#pragma once

#include <vector>

#include "gj_internal.h"

namespace gj {

struct BindH {
  int atom, col, dir;  // extension set: dir 0 out(prefix[col]), 1 in(prefix[col])
  int col2 = -1;       // ternary atom: the third vertices of (prefix[col], prefix[col2])
};
struct FilterH {
  int atom, key, val;  // seed pair kept iff x[val] in out(x[key])
};

// Plan of one global order: the seed atom of P_2, filters over the first two
// attributes, and per position j >= 2 the atoms binding order[j].
struct PlanH {
  int m = 0;
  std::vector<int> order;
  int seed_atom = -1;
  bool seed_fwd = true;
  std::vector<FilterH> filters;
  std::vector<std::vector<BindH>> bind;
  // inequalities checked when position j is bound: the value there must
  // exceed the prefix columns in above[j] and stay below those in below[j]
  std::vector<uint32_t> above, below;
  // first position of a trailing run of >= 2 attributes that share no atom
  // and no inequality (their extensions depend only on the prefix before the
  // run, so counts may multiply), else 0
  int fact_from = 0;
  int ntri = 0;  // ternary atoms
  bool has_ineq() const {
    for (int j = 0; j < m; ++j)
      if (above[j] | below[j]) return true;
    return false;
  }
};

PlanH make_plan(const gj_query* q, const std::vector<int>& order, int forced_seed);
std::vector<int> delta_order(const gj_query* q, int i);
void PlanHCheck(const gj_query* q);

// Versions read by each atom: delta query dQ_i reads the new version for
// atoms before i and the old one for atoms after i (Sec. 3.3.1).
struct Views {
  const Version* old_v;
  const Version* new_v;
  int delta_atom;  // -1: every atom reads old_v
  const TriIndex* tri = nullptr;  // for ternary atoms (static runs)
  bool hash = true;               // membership indexes may be used where built
  const gj_graph* graph = nullptr;  // static reads: the graph whose indexes may be built
  const Version& of(int atom) const {
    return (delta_atom >= 0 && atom < delta_atom) ? *new_v : *old_v;
  }
};

StageDesc stage_desc(const PlanH& P, const Views& V, int j);
SeedFilter seed_filter(const PlanH& P, const Views& V);

struct Level {
  uint64_t cap = 0;
  uint32_t* F = nullptr;
  int8_t* Fw = nullptr;
  uint32_t* minc = nullptr;
  uint8_t* mini = nullptr;
  uint64_t* off = nullptr;
  uint64_t* mask = nullptr;
  uint32_t* wcnt = nullptr;
  uint64_t* woff = nullptr;
  // per-prefix records of count-minimisation (StageDesc::pl, ent), or null
  uint32_t* pl = nullptr;
  uint64_t* ent = nullptr;
};

class Runner {
 public:
  Runner(gj_ctx* c, const PlanH& P, const Views& V, bool weighted, bool collect, uint64_t seed_cap);
  ~Runner();
  void use_rows(uint32_t* dev_rows, int8_t* dev_signs, uint64_t cap);
  void own_rows(uint64_t cap, bool with_signs);
  void seed(const uint32_t* x0, const uint32_t* x1, const int8_t* w, uint64_t cnt);
  void finish(uint64_t& matches, int64_t& wsum);

  gj_ctx* c;
  const PlanH& P;
  Views V;
  bool weighted, collect;
  gj_stats st{};
  KernelTimer timer;
  uint32_t* rows = nullptr;
  int8_t* rsign = nullptr;
  uint64_t rcap = 0, rows_alloc = 0, nrows = 0;

 private:
  void stage(int j, uint64_t n);
  StageDesc desc(int j, int lvl);
  void factorised(int j0, uint64_t n);
  void ensure_rows(uint64_t need);
  Level L[GJ_MAX_ATTRS + 1];
  RowMap map;
  unsigned long long* acc = nullptr;
  uint32_t* seed_flags = nullptr;
  uint64_t* seed_off = nullptr;
  bool rows_owned = false, signs_owned = false, want_signs = false;
};

}  // namespace gj
