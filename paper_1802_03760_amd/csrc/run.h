// Last-stage counts grouped by prefix runs (run.hip).
#pragma once

#include "gj_internal.h"

namespace gj {

// How a stage's binding atoms split for run.hip: the old ones (old_mask, nold)
// read columns below r, which key the runs; newa is the one atom reading the
// last bound column (-1: none).  The rest are the context's options.
struct RunDesc {
  int ok;  // fused pipeline's table: this request's stage at this level takes the run kernels
  int r;
  int nold;
  uint32_t old_mask;
  int newa;
  uint32_t ratio;      // stream the new set when it holds at most ratio x |S| values
  uint64_t min_work;   // staged runs: at least this many count-minimised candidates
  uint64_t task_work;  // candidates per task beyond the build's share
  uint32_t reuse;      // staged runs: candidates at least this many times the shared set bound
  uint32_t big;        // 0: runs whose shared set needs the large shape are not staged
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

// ---------------------------------------------------------------- fused pipeline
// Device buffers of the run kernels inside the fused pipeline, shared by its
// levels (which run one after another): sized for levels of at most cap
// prefixes (larger levels keep the per-candidate kernel).
struct RunFusedBufs {
  uint64_t cap = 0;
  uint32_t *head = nullptr, *rs = nullptr, *tcnt = nullptr, *tcnt_big = nullptr, *minc2 = nullptr;
  uint64_t *hoff = nullptr, *toff = nullptr, *toff_big = nullptr, *off2 = nullptr;
  uint8_t* staged = nullptr;
  unsigned int* counter = nullptr;  // two task counters
  uint32_t* sv = nullptr;           // the large shape's shared values, per workgroup
  unsigned long long* stats = nullptr;  // the context's run sums (run_stats_get)
  int num_cus = 0;
};

// bytes of RunFusedBufs for levels of cap prefixes on num_cus CUs
uint64_t run_fused_bytes(uint64_t cap, int num_cus);
// carves RunFusedBufs out of one device allocation of run_fused_bytes bytes
void run_fused_carve(RunFusedBufs& b, void* base, uint64_t cap, int num_cus, unsigned long long* stats);
// the context's run sums (allocated and cleared at first use, outside any
// stream capture)
unsigned long long* run_stats_get(gj_ctx* c);
// Enqueues (capturable: every size is read from device memory) the run path
// of level j of the fused pipeline, whose levels hold cap prefixes at most:
// the runs of the requests whose split RDt[r * (GJ_MAX_ATTRS + 1) + j] is ok
// are counted into cnt[r], pre (next level's prefixes) and wsum[r], and
// b.off2 gets the candidate space left to the fused propose kernel, which
// takes it where H->nrun[j] > 0.  R, H: the fused pipeline's request table
// and header (batch.h); off, minc: the level's count-minimised candidate
// offsets and counts; part, part_off: the pipeline's scan scratch.
struct BReq;
struct BHead;
void run_fused_level(hipStream_t st, const RunFusedBufs& b, const BReq* R, const RunDesc* RDt, BHead* H, int j,
                     const uint32_t* F, const uint32_t* rid, uint64_t cap, const uint64_t* off,
                     const uint32_t* minc, uint64_t* part, uint64_t* part_off, unsigned long long* cnt,
                     unsigned long long* pre, unsigned long long* wsum);

}  // namespace gj
