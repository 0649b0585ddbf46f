// Log-structured updates (see lsm.hip).
#pragma once

#include "gj_internal.h"

namespace gj {

// State of the graph after an update whose delta queries completed.
struct LsmCommit {
  uint64_t used[2] = {0, 0};
  uint64_t nkeys[2] = {0, 0};
  uint64_t m = 0;
};

// Rewrites the rows touched by dE (per direction d: rows r[d], values x[d],
// signs sg[d], k entries sorted by (r, x), every insert absent from and every
// delete present in the current version) into the current slot's slack, and
// writes the next version's map.  oldv / newv become the two versions the
// delta queries read.  Compacts first when the slack is used up; returns
// false when the rows do not fit even then (the caller rewrites both
// indexes).  The graph is unchanged until lsm_commit; lsm_abort undoes the
// map writes of an update that is not committed.
bool lsm_update(gj_ctx* c, gj_graph* g, const uint32_t* const (&r)[2], const uint32_t* const (&x)[2],
                const int8_t* const (&sg)[2], uint64_t k, Version& oldv, Version& newv, LsmCommit& commit);
void lsm_commit(gj_graph* g, const LsmCommit& commit);
void lsm_abort(gj_ctx* c, gj_graph* g);

}  // namespace gj
