// Owner-grouped first-stage intersection (see owner.hip).
#pragma once

#include "gj_internal.h"

namespace gj {

// Seed edges (x0, x1); LA = extension set of the atom on x0, LB = of the atom
// on x1; S0 = seed index (partners x1 of x0), S1 = its transpose (partners x0
// of x1).  Each pair (rp, adj) is a CSR row-pointer and column array.
struct OwnerArgs {
  const uint32_t *rpA, *adjA;
  const uint32_t *rpB, *adjB;
  const uint32_t *rpS0, *adjS0;
  const uint32_t *rpS1, *adjS1;
  uint32_t n;
  // optional signs of the seed edges (null: all +1), in S0 order (seed-index
  // order, as seed_row/seed_col) and in S1 order (transposed order)
  const int8_t* sg0 = nullptr;
  const int8_t* sg1 = nullptr;
};

// matches = sum over all seed edges of |LA(x0) ∩ LB(x1)|;
// extensions = sum of min(|LA(x0)|, |LB(x1)|); wsum = the same sum as
// matches with each edge's term times its sign.  seed_row/seed_col: the E
// seed edges as (x0, x1) in seed-index order; t_row/t_col: the same edges in
// transposed-index order as (x1, x0).
// plan (with gen, the version's generation, and pc, the context that owns
// the graph's memory): a static count's plan kept with the version, reused
// while valid, else built and stored there; null: planned for this call only.
void owner_count(gj_ctx* c, const OwnerArgs& a, const uint32_t* seed_row, const uint32_t* seed_col,
                 const uint32_t* t_row, const uint32_t* t_col, uint64_t E, KernelTimer& timer, uint64_t& matches,
                 uint64_t& extensions, int64_t* wsum = nullptr, OwnerPlan* plan = nullptr, uint64_t gen = 0,
                 gj_ctx* pc = nullptr);

}  // namespace gj
