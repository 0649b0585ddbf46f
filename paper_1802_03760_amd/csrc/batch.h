// Batched multi-request execution (see batch.hip).
#pragma once

#include "gj_internal.h"

namespace gj {

class BatchExec {
 public:
  struct Impl;
  BatchExec();
  ~BatchExec();
  // counts of nreq (query, seed slice) requests on the current version of g;
  // overflow = a level exceeded the frontier capacity (results not set)
  void run(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* lo,
           const uint64_t* hi, uint64_t* counts, gj_stats* stats, bool& overflow);

 private:
  Impl* p;
};

void batch_destroy(gj_ctx* c);

}  // namespace gj
