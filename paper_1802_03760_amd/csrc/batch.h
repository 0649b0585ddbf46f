// Batched multi-request execution (see batch.hip).
#pragma once

#include <vector>

#include "engine.h"
#include "gj_internal.h"

namespace gj {

// One request of a fused run: a query plan, the versions its atoms read, and
// its seeds (x0 = row[lo + i], x1 = col[lo + i], signed by w[lo + i] if w is
// not null) for i < len.
struct ReqSpec {
  PlanH P;
  Views V;
  const uint32_t* row = nullptr;
  const uint32_t* col = nullptr;
  const int8_t* w = nullptr;
  uint64_t lo = 0, len = 0;
};

class BatchExec {
 public:
  struct Impl;
  BatchExec();
  ~BatchExec();
  // counts of nreq (query, seed slice) requests on the current version of g;
  // overflow = a level exceeded the capacity (results not set)
  void run(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* lo,
           const uint64_t* hi, uint64_t* counts, gj_stats* stats, bool& overflow, const Version* ver = nullptr);
  // general form: per request the match count, the signed sum of match
  // weights and the per-level counters (any output may be null)
  void run_specs(gj_ctx* c, const std::vector<ReqSpec>& specs, uint64_t* counts, int64_t* wsums, gj_stats* stats,
                 bool& overflow);

 private:
  Impl* p;
};

void batch_destroy(gj_ctx* c);

}  // namespace gj
