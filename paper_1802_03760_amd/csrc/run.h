// Last-stage counts grouped by prefix runs (run.hip).
#pragma once

#include "gj_internal.h"

namespace gj {

// How a stage's binding atoms split for run.hip: the old ones (old_mask, nold)
// read columns below r, which key the runs; newa is the one atom reading the
// last bound column (-1: none).  The rest are the context's options.
struct RunDesc {
  int r;
  int nold;
  uint32_t old_mask;
  int newa;
  uint32_t ratio;      // stream the new set when it holds at most ratio x |S| values
  uint64_t min_work;   // staged runs: at least this many count-minimised candidates
  uint64_t task_work;  // candidates per task beyond the build's share
  uint32_t reuse;      // staged runs: candidates at least this many times the shared set bound
};

// Whether stage d can run grouped by prefix runs (binary atoms only, at least
// one old atom, at most one new atom); fills rd's split.
bool run_desc(const StageDesc& d, RunDesc& rd);

// Plans the last stage by runs; when the staged runs make at least
// run_min_tasks tasks, counts their survivors into acc (acc[1]: the signed
// sum with prefix weights wt), writes to off2 the exclusive scan of minc
// with the staged prefixes' counts zeroed, sets W2 = off2[n] (the candidate
// space left to the per-candidate kernel) and returns true.  Otherwise
// counts nothing and returns false (the per-candidate kernel takes the whole
// stage).
bool run_count(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off, const uint32_t* minc,
               const StageDesc& d, RunDesc rd, const int8_t* wt, unsigned long long* acc, uint64_t* off2,
               uint64_t& W2, KernelTimer& timer);

}  // namespace gj
