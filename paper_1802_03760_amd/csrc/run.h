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
};

// Whether stage d can run grouped by prefix runs (binary atoms only, at least
// one old atom, at most one new atom); fills rd's split.
bool run_desc(const StageDesc& d, RunDesc& rd);

// Counts the last stage's survivors of the staged runs into acc (acc[1]: the
// signed sum with prefix weights wt) and zeroes the other runs' counts in
// minc, whose exclusive scan it writes to off2; returns off2[n], the size of
// the candidate space left to the per-candidate kernel.
uint64_t run_count(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off, uint32_t* minc,
                   const StageDesc& d, RunDesc rd, const int8_t* wt, unsigned long long* acc, uint64_t* off2,
                   KernelTimer& timer);

}  // namespace gj
