// Seed-work estimates for the request scheduler of the server (see sched.hip).
#pragma once

#include <vector>

#include "engine.h"

namespace gj {

// One count request to estimate: its plan, the version it reads, and its
// seed slice [lo, lo + len) summed in blocks of bs consecutive seeds.
struct WorkReq {
  const PlanH* P = nullptr;
  const Version* v = nullptr;
  uint64_t lo = 0, len = 0;
  uint32_t bs = 1;
};

// Estimated work per block, concatenated over the requests: request i owns
// out[off[i] .. off[i + 1]).  Runs on the context stream and synchronises.
void seed_work(gj_ctx* c, const std::vector<WorkReq>& reqs, std::vector<uint64_t>& out, std::vector<uint64_t>& off);

}  // namespace gj
