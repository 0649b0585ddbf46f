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

// Device table entry of one request of a fused run: its seeds, seed
// filters and the stage descriptor of every level.
struct BReq {
  uint32_t m;
  uint32_t pad;
  uint64_t seed_lo;
  const uint32_t* seed_row;
  const uint32_t* seed_col;
  const int8_t* seed_w;  // signed seeds of a delta query, or null (+1)
  SeedFilter filt;
  StageDesc st[GJ_MAX_ATTRS];
};

// header of the device state: sizes and flags read by every kernel
struct BHead {
  uint32_t nreq;
  uint32_t lin;        // tuned: linear search below this extension-set size
  uint32_t claim_words;  // tuned: words (64 candidates each) a wave claims at a time
  uint64_t seeds;      // total seed edges over all requests
  unsigned long long nlev[GJ_MAX_ATTRS + 1];
  unsigned long long claim[GJ_MAX_ATTRS + 1];  // next unclaimed word chunk per level
  uint32_t overflow;
  // levels whose last-stage prefixes may be grouped by runs (set per batch by
  // the host), and the live size the run kernels take there (0 elsewhere)
  uint32_t runon[GJ_MAX_ATTRS + 1];
  unsigned long long nrun[GJ_MAX_ATTRS + 1];
  // level j regrouped by parent prefix before its stage: its live size and
  // that of level j - 1 (both 0 where it is not)
  unsigned long long nreg[GJ_MAX_ATTRS + 1];
  unsigned long long nregp[GJ_MAX_ATTRS + 1];
};


constexpr int kStat = GJ_MAX_ATTRS + 1;

// Exclusive scan of the live part (H->nlev[j], at most cap entries) of a
// level-sized u32 array into out (out[n] = total), in device memory only
// (three launches, capturable): part / part_off hold the tile sums.
void bt_scan(hipStream_t st, const uint32_t* in, const BHead* H, int j, uint64_t cap, uint64_t* part,
             uint64_t* part_off, uint64_t* out);
// The same over the first *n entries (n in device memory, at most cap).
void bt_scan_n(hipStream_t st, const uint32_t* in, const unsigned long long* n, uint64_t cap, uint64_t* part,
               uint64_t* part_off, uint64_t* out);

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
