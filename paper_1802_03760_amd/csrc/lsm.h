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
// delta queries read.  Returns false, writing nothing, when the rows do not
// fit the slack or exceed an eighth of the edges: the caller then writes both
// indexes anew from the current version, appended rows included, and calls
// lsm_clear.  The graph is unchanged until lsm_commit; lsm_abort undoes the
// map writes of an update that is not committed.
bool lsm_update(gj_ctx* c, gj_graph* g, const uint32_t* const (&r)[2], const uint32_t* const (&x)[2],
                const int8_t* const (&sg)[2], uint64_t k, Version& oldv, Version& newv, LsmCommit& commit);
void lsm_commit(gj_graph* g, const LsmCommit& commit);
void lsm_abort(gj_ctx* c, gj_graph* g);
// Offsets (device, nkeys + 1 entries) of the current version's rewritten rows
// of direction d in key-list order; total = their summed length (null, 0
// when none).
const uint64_t* lsm_row_offsets(gj_ctx* c, const gj_graph* g, int d, uint64_t& total);
// ends the epoch of appended rows: maps back to "row in the slot", nothing used
void lsm_clear(gj_ctx* c, gj_graph* g);

}  // namespace gj
