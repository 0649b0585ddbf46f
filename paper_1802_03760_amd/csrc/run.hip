// Last-stage counts grouped by prefix runs.
//
// The atoms binding attribute j split into new ones, whose other attribute
// is the last bound column j-1, and old ones, which read earlier columns.
// Consecutive prefixes of a frontier that agree on every column an old atom
// reads (a run; frontiers are written in lexicographic order, so such
// prefixes sit together) have the same old extension sets, hence the same
// intersection S of them.  Generic Join's proposal and intersection for a
// prefix p of the run (Sec. 2.2, Sec. 4.1) then reduce to |S & new set of p|
// within p's inequality range.  One workgroup builds S once per run (or per
// share of a long run) into an LDS hash table, so its membership tests are
// O(1) LDS probes, and per prefix takes the cheaper side by the ratio of the
// two sizes: the new set streamed from memory (coalesced) through the table
// when it holds at most `run_ratio` x |S| values, else S's values probed
// against the new set's own table or row.  A run's prefixes are cut into
// tasks of about equal work (the balanced split of Sec. 3.4), claimed from a
// device counter.  Runs whose S could outgrow the table, or whose work would
// not repay the build, keep the per-candidate kernel: their counts of
// candidates stay in a second candidate space, the staged runs' set to zero.
#include <algorithm>
#include <cstring>

#include "batch.h"
#include "gj_internal.h"
#include "prim.h"
#include "run.h"

namespace gj {

// Two workgroup shapes: small shared sets (at most 4,096 values, a 32 KiB
// table and S's values in LDS, two workgroups of 512 threads per CU) and
// large ones (at most 24,576 values, a 128 KiB table at load <= 3/4, S's
// values in a per-workgroup global buffer, one workgroup of 1,024 threads per
// CU).  Larger sets stay with the per-candidate kernel.
template <bool BIG>
struct RunShape;
template <>
struct RunShape<false> {
  static constexpr int NT = 512;
  static constexpr uint32_t CAP = 4096;
  static constexpr int LOG_SLOTS = 13;
  static constexpr int U = 2;  // windows per wave per step, their loads issued together
  static constexpr int UF = 3;  // the same in the fused form (fewer live registers elsewhere)
};
template <>
struct RunShape<true> {
  static constexpr int NT = 1024;
  static constexpr uint32_t CAP = 24576;
  static constexpr int LOG_SLOTS = 15;
  static constexpr int U = 1;
  static constexpr int UF = 2;
};
constexpr uint32_t kRunCap = RunShape<false>::CAP;
constexpr uint32_t kRunCapBig = RunShape<true>::CAP;
constexpr uint32_t kRunChunk = 512;  // prefixes per chunk (one thread each)
constexpr uint32_t kRunEmpty = 0xFFFFFFFFu;

// ---------------------------------------------------------------- planning
// head[p] = 1 where a run starts: p = 0, or a key column differs from p - 1.
__global__ void k_run_heads(const uint32_t* __restrict__ F, uint64_t stride, uint64_t n, int r,
                            uint32_t* __restrict__ head) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    uint32_t h = p == 0;
    for (int c = 0; c < r && !h; ++c) h = F[(uint64_t)c * stride + p] != F[(uint64_t)c * stride + p - 1];
    head[p] = h;
  }
}

// rs[run] = its first prefix; rs[runs] = n
// (also clears the task counter of the counting kernel)
// (n: *np when np is not null)
__global__ void k_run_starts(const uint32_t* __restrict__ head, const uint64_t* __restrict__ hoff, uint64_t n_arg,
                             const unsigned long long* __restrict__ np, uint32_t* __restrict__ rs,
                             unsigned int* __restrict__ counter) {
  const uint64_t n = np ? *np : n_arg;
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  if (blockIdx.x == 0 && threadIdx.x < 2) counter[threadIdx.x] = 0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    if (head[p]) rs[hoff[p]] = (uint32_t)p;
    if (p + 1 == n) rs[hoff[n]] = (uint32_t)n;
  }
}

// Row of binding atom a of the stage for value v (a a compile-time index in
// every caller, so the descriptor's arrays are read without a private copy).
__device__ __forceinline__ void atom_row(const StageDesc& d, int a, uint32_t v, uint32_t& lo, uint32_t& len) {
  uint32_t hi;
  row_range(d.rp[a], d.pm[a], v, lo, hi);
  len = hi - lo;
}

// The plan of the run headed by prefix p (ending before prefix e): the size
// bound of S (smallest old set), the run's candidates in the count-minimised
// space, whether it is staged (st) and with which shape (big), its number of
// tasks (t), and its candidates added to ws by outcome (staged, shared set
// too large, too little work).
__device__ __forceinline__ void run_plan_one(const uint32_t* __restrict__ F, uint64_t stride, uint64_t p, uint64_t e,
                                             const uint64_t* __restrict__ off, const StageDesc& d, const RunDesc& rd,
                                             bool& st, bool& big, uint32_t& t, uint64_t (&ws)[3]) {
  uint32_t B = 0xFFFFFFFFu;
#pragma unroll
  for (int a = 0; a < kMaxBind; ++a) {
    if (a < d.k && ((rd.old_mask >> a) & 1)) {
      uint32_t lo, len;
      atom_row(d, a, F[(uint64_t)d.col[a] * stride + p], lo, len);
      B = len < B ? len : B;
    }
  }
  uint64_t W = off[e] - off[p];
  st = B <= (rd.big ? kRunCapBig : kRunCap) && W >= rd.min_work && W >= (uint64_t)rd.reuse * B;
  big = B > kRunCap;
  t = 0;
  if (st) {
    uint64_t per = rd.task_work + 8ull * B * (uint64_t)rd.nold;
    uint64_t k = (W + per - 1) / per;
    uint64_t kids = e - p;
    t = (uint32_t)(k < 1 ? 1 : (k > kids ? kids : k));
  }
  ws[st ? 0 : (B > kRunCapBig ? 1 : 2)] += W;
}

__device__ __forceinline__ void run_plan_sums(const uint64_t (&ws)[3], unsigned long long* __restrict__ wsum) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    uint64_t b = block_sum<kBlock>(ws[i]);
    if (threadIdx.x == 0 && b) atomicAdd(wsum + i, (unsigned long long)b);
  }
}

// Per run (at its head): staged[run], and its number of tasks in the shape's
// array (tcnt or tcnt_big at the head; 0 elsewhere and for unstaged runs).
__global__ void k_run_plan(const uint32_t* __restrict__ F, uint64_t stride, uint64_t n,
                           const uint64_t* __restrict__ off, const uint32_t* __restrict__ head,
                           const uint64_t* __restrict__ hoff, const uint32_t* __restrict__ rs, StageDesc d,
                           RunDesc rd, uint32_t* __restrict__ tcnt, uint32_t* __restrict__ tcnt_big,
                           uint8_t* __restrict__ staged, unsigned long long* __restrict__ wsum) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  uint64_t ws[3] = {0, 0, 0};
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    uint32_t t = 0;
    bool big = false, st = false;
    if (head[p]) {
      uint64_t run = hoff[p];
      run_plan_one(F, stride, p, rs[run + 1], off, d, rd, st, big, t, ws);
      staged[run] = st ? 1 : 0;
    }
    tcnt[p] = big ? 0 : t;
    tcnt_big[p] = big ? t : 0;
  }
  run_plan_sums(ws, wsum);
}

// The per-candidate kernel's counts: zero for prefixes of staged runs
// (n: *np when np is not null).
__global__ void k_run_direct(const uint32_t* __restrict__ head, const uint64_t* __restrict__ hoff,
                             const uint8_t* __restrict__ staged, uint64_t n_arg,
                             const unsigned long long* __restrict__ np, const uint32_t* __restrict__ minc,
                             uint32_t* __restrict__ minc2) {
  const uint64_t n = np ? *np : n_arg;
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    uint64_t rid = hoff[p] + head[p] - 1;
    minc2[p] = staged[rid] ? 0u : minc[p];
  }
}

// ---------------------------------------------------------------- LDS table
// Open addressing over buckets of four u32 slots (one 16-byte read each);
// insertion fills the first empty slot from the home bucket on, so a bucket
// with an empty last slot ends an unsuccessful search.
__device__ __forceinline__ void run_insert(uint32_t* H, uint32_t x, int shift, uint32_t bmask) {
  uint32_t b = (x * 0x9E3779B1u) >> shift;
  for (;;) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (atomicCAS(&H[4 * b + k], kRunEmpty, x) == kRunEmpty) return;
    b = (b + 1) & bmask;
  }
}

__device__ __forceinline__ bool run_probe(const uint32_t* H, uint32_t x, int shift, uint32_t bmask) {
  const uint4* B = reinterpret_cast<const uint4*>(H);
  uint32_t b = (x * 0x9E3779B1u) >> shift;
  for (;;) {
    uint4 q = B[b];
    if (min(min(q.x ^ x, q.y ^ x), min(q.z ^ x, q.w ^ x)) == 0u) return true;
    if (q.w == kRunEmpty) return false;
    b = (b + 1) & bmask;
  }
}

// first i in [lo, hi) with a[i] >= x, else hi
__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* __restrict__ a, uint64_t lo, uint64_t hi,
                                                    uint64_t x) {
  uint64_t n = hi - lo;
  while (n > 0) {
    uint64_t half = n >> 1;
    if (a[lo + half] < x) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

// Exclusive scan over a workgroup of NT threads with few live registers: a
// scan in each wave, then the wave totals scanned by the first wave.  sh
// holds NT / 64 + 1 values; the caller synchronises before reusing it.
template <int NT>
__device__ __forceinline__ uint64_t run_block_scan(uint64_t v, uint64_t& total, uint64_t* sh) {
  constexpr int NW = NT / 64;
  const int lane = lane_id(), wave = wave_id();
  const uint64_t inc = wave_incl_scan(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const uint64_t x = lane < NW ? sh[lane] : 0ull;
    const uint64_t xi = wave_incl_scan(x);
    if (lane < NW) sh[lane] = xi - x;
    if (lane == NW - 1) sh[NW] = xi;
  }
  __syncthreads();
  total = sh[NW];
  return sh[wave] + inc - v;
}

// OR of a 64-bit value over the wave
__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    lo |= __shfl_xor(lo, o, 64);
    hi |= __shfl_xor(hi, o, 64);
  }
  return ((uint64_t)hi << 32) | lo;
}

// last i in [0, n) with w[i] <= q (w ascending, w[0] = 0 <= q < w[n])
__device__ __forceinline__ uint32_t run_owner(const uint32_t* w, uint32_t n, uint32_t q) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (w[mid] <= q)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// x in the new atom's set of a prefix: its table (desc != 0) or its row
__device__ __forceinline__ bool mem_member(const uint32_t* __restrict__ adj, const uint32_t* __restrict__ hs,
                                           uint64_t desc, uint32_t lo, uint32_t len, uint32_t x) {
  if (desc) return hash_member(hs, desc, x);
  return contains_u32(adj, lo, lo + len, x);
}

// Membership of U values in the new sets of their prefixes, in lockstep
// (each step issues the loads of every pending value before comparing):
// want[u] asks for x[u] in the set with table descriptor desc[u] in hs, or,
// without a table, in the sorted row adj[lo[u], lo[u] + len[u]).
template <int U>
__device__ __forceinline__ void member_lockstep(const uint32_t* __restrict__ adj, const uint32_t* __restrict__ hs,
                                                const uint64_t (&desc)[U], const uint32_t (&lo)[U],
                                                const uint32_t (&len)[U], const uint32_t (&x)[U],
                                                const bool (&want)[U], bool (&hit)[U]) {
  bool pend[U];
  uint32_t h[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    pend[u] = want[u] && desc[u] != 0;
    h[u] = pend[u] ? hash_home(x[u], (uint32_t)(desc[u] & 0xFF)) : 0u;
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < U; ++u) any = any || pend[u];
    if (!any) break;
    uint4 q[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      q[u] = pend[u] ? *(const uint4*)(hs + 4 * ((desc[u] >> 8) + h[u])) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!pend[u]) continue;
      const uint32_t e = x[u];
      if (q[u].x == e || q[u].y == e || q[u].z == e || q[u].w == e) {
        hit[u] = true;
        pend[u] = false;
      } else if (q[u].w == kHashEmpty) {
        pend[u] = false;
      } else {
        h[u] = (h[u] + 1) & ((1u << (uint32_t)(desc[u] & 0xFF)) - 1);
      }
    }
  }
  uint32_t l[U], n[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    l[u] = lo[u];
    n[u] = want[u] && desc[u] == 0 ? len[u] : 0u;
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < U; ++u) any = any || n[u] > 0;
    if (!any) break;
    uint32_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = n[u] > 0 ? adj[l[u] + (n[u] >> 1)] : 0u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (n[u] > 0) {
        const uint32_t half = n[u] >> 1;
        if (v[u] < x[u]) {
          l[u] += half + 1;
          n[u] -= half + 1;
        } else {
          n[u] = half;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (want[u] && desc[u] == 0) hit[u] = l[u] < lo[u] + len[u] && adj[l[u]] == x[u];
}

// ---------------------------------------------------------------- counting kernel
// A task's stage and run split: the launch's own (one stage of one query),
// or, in the fused pipeline (FUSED), those of the request its run belongs to.
template <bool FUSED>
__device__ __forceinline__ const StageDesc& task_desc(const StageDesc& own, const BReq* __restrict__ R, uint32_t r,
                                                      int j) {
  if constexpr (FUSED)
    return R[r].st[j];
  else
    return own;
}
template <bool FUSED>
__device__ __forceinline__ const RunDesc& task_split(const RunDesc& own, const RunDesc* __restrict__ RDt, uint32_t r,
                                                     int j) {
  if constexpr (FUSED)
    return RDt[(uint64_t)r * kStat + j];
  else
    return own;
}

// FUSED: the level's live size is *np, a run's request is rid[head], and
// each task adds its survivors to that request's match count fcnt, prefix
// counter fpre of the next level and weight sum fws (static requests only:
// weight 1); acc is not used.
template <bool SIGNED, bool BIG, bool FUSED>
__global__ void __launch_bounds__(RunShape<BIG>::NT) __attribute__((amdgpu_waves_per_eu(4))) k_run_count(const uint32_t* __restrict__ F, uint64_t stride,
                                                                 uint64_t n_arg, const uint64_t* __restrict__ off,
                                                                 const uint64_t* __restrict__ hoff,
                                                                 const uint32_t* __restrict__ rs,
                                                                 const uint64_t* __restrict__ toff, StageDesc d_own,
                                                                 RunDesc rd_own, const int8_t* __restrict__ wt,
                                                                 uint32_t* __restrict__ sv_glob,
                                                                 unsigned int* __restrict__ counter,
                                                                 unsigned long long* __restrict__ acc,
                                                                 unsigned long long* __restrict__ wsum,
                                                                 const BReq* __restrict__ R, int jl,
                                                                 const uint32_t* __restrict__ rid,
                                                                 const RunDesc* __restrict__ RDt,
                                                                 const unsigned long long* __restrict__ np,
                                                                 unsigned long long* __restrict__ fcnt,
                                                                 unsigned long long* __restrict__ fpre,
                                                                 unsigned long long* __restrict__ fws) {
  constexpr int kRunNT = RunShape<BIG>::NT;
  constexpr int kRunU = FUSED ? RunShape<BIG>::UF : RunShape<BIG>::U;
  constexpr int kRunLogSlots = RunShape<BIG>::LOG_SLOTS;
  __shared__ __attribute__((aligned(16))) uint32_t H[1 << kRunLogSlots];
  // S's values: in LDS (small shape) or this workgroup's global buffer
  __shared__ uint32_t SvL[BIG ? 1 : RunShape<BIG>::CAP];
  uint32_t* const SvG = sv_glob + (uint64_t)blockIdx.x * RunShape<BIG>::CAP;
  // the chunk's prefixes with work: unit offsets; row start, length (top
  // bit: streamed) and inequality range; table descriptor; weight
  __shared__ uint32_t coff[kRunChunk + 1];
  __shared__ uint4 cmeta[kRunChunk];
  __shared__ uint64_t cdesc[kRunChunk];
  __shared__ int8_t cw[kRunChunk];
  __shared__ uint64_t s_cs, s_ce, s_head;
  __shared__ uint64_t s_scan[kRunNT / 64 + 1];
  __shared__ uint32_t s_task, s_nS, s_small;
  __shared__ uint32_t s_olo[kMaxBind], s_olen[kMaxBind];
  __shared__ uint64_t s_odesc[kMaxBind];
  const int tid = threadIdx.x;
  const uint64_t n = FUSED ? (uint64_t)*np : n_arg;
  const uint64_t ntask = toff[n];
  uint64_t hits = 0, units = 0, builds = 0, belems = 0;
  int64_t whits = 0;
  uint64_t cached = ~0ull;  // head of the run whose S is in the table
  uint32_t nS = 0;
  int shift = 0;
  uint32_t bmask = 0;
  for (;;) {
    if (tid == 0) {
      uint32_t t = atomicAdd(counter, 1u);
      s_task = t;
      if (t < ntask) {
        // the run (head prefix) of task t, its prefixes, and this task's share
        // of them by equal parts of the run's candidates
        uint64_t s = find_segment(toff, 0, n, t);
        uint64_t e = rs[hoff[s] + 1];
        uint64_t nt = toff[s + 1] - toff[s], i = t - toff[s];
        uint64_t W = off[e] - off[s];
        uint64_t q = W / nt, rm = W % nt;
        uint64_t g0 = off[s] + q * i + rm * i / nt, g1 = off[s] + q * (i + 1) + rm * (i + 1) / nt;
        s_cs = i == 0 ? s : lower_bound_u64(off, s, e, g0);
        s_ce = i + 1 == nt ? e : lower_bound_u64(off, s, e, g1);
        s_head = s;
      }
    }
    __syncthreads();
    if (s_task >= ntask) break;
    const uint64_t head = s_head, cs = s_cs, ce = s_ce;
    const uint32_t rq = FUSED ? __builtin_amdgcn_readfirstlane(rid[head]) : 0u;
    const StageDesc& d = task_desc<FUSED>(d_own, R, rq, jl);
    const RunDesc& rd = task_split<FUSED>(rd_own, RDt, rq, jl);
    // the new atom's arrays (uniform over the task)
    const uint32_t* nrp = nullptr;
    const uint32_t* nadj = nullptr;
    const uint64_t* npm = nullptr;
    const uint64_t* nhd = nullptr;
    const uint32_t* nhs = nullptr;
    int ncol = 0;
    switch (rd.newa) {
#define GJ_NEWA(A)     \
  case A:              \
    nrp = d.rp[A];     \
    nadj = d.adj[A];   \
    npm = d.pm[A];     \
    nhd = d.hd[A];     \
    nhs = d.hs[A];     \
    ncol = d.col[A];   \
    break;
      GJ_NEWA(0) GJ_NEWA(1) GJ_NEWA(2) GJ_NEWA(3) GJ_NEWA(4) GJ_NEWA(5) GJ_NEWA(6) GJ_NEWA(7)
#undef GJ_NEWA
      default:
        break;
    }
    if (cs < ce && head != cached) {
      // S = the intersection of the old sets of the run: the smallest one
      // streamed, each value tested in the others (their tables or rows)
      if (tid == 0) {
        uint32_t best = 0xFFFFFFFFu;
        int bi = 0;
#pragma unroll
        for (int a = 0; a < kMaxBind; ++a) {
          if (a < d.k && ((rd.old_mask >> a) & 1)) {
            uint32_t v = F[(uint64_t)d.col[a] * stride + head], lo, len;
            atom_row(d, a, v, lo, len);
            s_olo[a] = lo;
            s_olen[a] = len;
            s_odesc[a] = d.hd[a] ? d.hd[a][v] : 0ull;
            if (len < best) {
              best = len;
              bi = a;
            }
          }
        }
        s_small = (uint32_t)bi;
        s_nS = 0;
      }
      for (uint32_t k = tid; k < (1u << kRunLogSlots); k += kRunNT) H[k] = kRunEmpty;
      __syncthreads();
      const int small = (int)s_small;
      const uint32_t slen = s_olen[small], slo = s_olo[small];
      // table of 2^lg slots, lg >= log2(4 |S| bound) where it fits (load <= 1/4),
      // else the whole table (load <= 1/2 small, <= 3/4 large)
      int lg = 6;
      while ((1u << lg) < 4 * slen && lg < kRunLogSlots) ++lg;
      shift = 32 - (lg - 2);
      bmask = (1u << (lg - 2)) - 1;
      const uint32_t* sadj = d.adj[0];
      switch (small) {
#define GJ_SMALL(A)    \
  case A:              \
    sadj = d.adj[A];   \
    break;
        GJ_SMALL(1) GJ_SMALL(2) GJ_SMALL(3) GJ_SMALL(4) GJ_SMALL(5) GJ_SMALL(6) GJ_SMALL(7)
#undef GJ_SMALL
        default:
          break;
      }
      for (uint32_t k0 = 0; k0 < slen; k0 += kRunNT) {
        uint32_t k = k0 + tid;
        bool in = k < slen;
        uint32_t x = in ? sadj[slo + k] : 0u;
#pragma unroll
        for (int a = 0; a < kMaxBind; ++a) {
          if (a < d.k && ((rd.old_mask >> a) & 1) && a != small && in)
            in = mem_member(d.adj[a], d.hs[a], s_odesc[a], s_olo[a], s_olen[a], x);
        }
        uint64_t bal = __ballot(in);
        uint32_t base = 0;
        if (lane_id() == 0 && bal) base = atomicAdd(&s_nS, (uint32_t)__popcll(bal));
        base = __shfl(base, 0, 64);
        if (in) {
          const uint32_t pos = base + (uint32_t)__popcll(bal & lanemask_lt());
          if (BIG)
            SvG[pos] = x;
          else
            SvL[pos] = x;
          run_insert(H, x, shift, bmask);
        }
      }
      if (BIG) __threadfence_block();  // S's values in memory are seen by the whole workgroup
      __syncthreads();
      nS = s_nS;
      cached = head;
      builds += 1;
      belems += slen;
    }
    // the task's prefixes, kRunChunk at a time (none when S is empty)
    for (uint64_t cb = cs; cb < ce && nS; cb += kRunChunk) {
      const uint32_t cn = (uint32_t)(ce - cb < kRunChunk ? ce - cb : kRunChunk);
      uint32_t u = 0;
      uint32_t lo = 0, len = 0, lb = 0, ub = 0xFFFFFFFFu;
      uint64_t desc = 0;
      bool stream = false;
      int8_t w8 = 1;
      if ((uint32_t)tid < cn) {
        const uint64_t p = cb + tid;
        if (d.above | d.below) {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if (((d.above | d.below) >> c) & 1) {
              uint32_t o = F[(uint64_t)c * stride + p];
              if ((d.above >> c) & 1) lb = max(lb, o + 1);
              if ((d.below >> c) & 1) ub = min(ub, o);
            }
          }
        }
        if (rd.newa >= 0) {
          uint32_t v = F[(uint64_t)ncol * stride + p], hi;
          row_range(nrp, npm, v, lo, hi);
          len = hi - lo;
          desc = nhd ? nhd[v] : 0ull;
          stream = (uint64_t)len <= (uint64_t)rd.ratio * nS;
          u = stream ? len : nS;
        } else {
          u = nS;
        }
        if (lb >= ub) u = 0;
        if (SIGNED) w8 = wt[p];
      }
      // prefixes with work, compacted in order: their unit offsets (low
      // half) and positions (high half) by one workgroup scan
      uint64_t tot;
      const uint64_t ex = run_block_scan<kRunNT>((uint64_t)u | ((uint64_t)(u != 0) << 32), tot, s_scan);
      const uint32_t total = (uint32_t)tot, cnz = (uint32_t)(tot >> 32);
      if (u) {
        const uint32_t k = (uint32_t)(ex >> 32);
        coff[k] = (uint32_t)ex;
        cmeta[k] = make_uint4(lo, len | (stream ? 0x80000000u : 0u), lb, ub);
        cdesc[k] = desc;
        if (SIGNED) cw[k] = w8;
      }
      if (tid == 0) coff[cnz] = total;
      units += total;
      __syncthreads();
      // Each wave walks a contiguous run of 64-unit windows of the chunk's
      // unit space.  The prefix holding a window's first unit is carried from
      // window to window: lane l reads where prefix i0 + 1 + l starts, the
      // starts that fall in the window form a bit mask (every prefix has
      // work, so at most 64 start there), and lane j's prefix is i0 plus
      // the starts at or before j.  kRunU windows per step, their loads
      // issued together.
      constexpr uint32_t kWaves = kRunNT / 64;
      const uint32_t lane = (uint32_t)lane_id();
      const uint32_t nwin = (total + 63) >> 6;
      const uint32_t per = (nwin + kWaves - 1) / kWaves;
      const uint32_t wb = (uint32_t)wave_id() * per, we = min(nwin, wb + per);
      uint32_t i0 = wb < we ? run_owner(coff, cnz, wb << 6) : 0u;
      for (uint32_t wv = wb; wv < we; wv += kRunU) {
        uint32_t ci[kRunU], xv[kRunU], slo[kRunU], sln[kRunU], lbv[kRunU], ubv[kRunU];
        uint64_t sds[kRunU];
        bool act[kRunU], sm[kRunU], hit[kRunU];
#pragma unroll
        for (int k = 0; k < kRunU; ++k) {
          const uint32_t qw = (wv + k) << 6, q = qw + lane;
          const bool wok = wv + k < we;
          uint64_t bit = 0;
          const uint32_t nb = i0 + 1 + lane;
          if (wok && nb < cnz) {
            const uint32_t b = coff[nb] - qw;
            if (b < 64) bit = 1ull << b;
          }
          const uint64_t smask = wave_or(bit);
          const uint32_t i = i0 + (uint32_t)__popcll(smask & ((2ull << lane) - 1));
          i0 += (uint32_t)__popcll(smask);
          act[k] = wok && q < total;
          ci[k] = act[k] ? i : 0u;
          const uint4 mt = cmeta[ci[k]];
          const uint32_t t = q - coff[ci[k]];
          sm[k] = act[k] && !(mt.y >> 31);
          slo[k] = mt.x;
          sln[k] = mt.y & 0x7FFFFFFFu;
          lbv[k] = mt.z;
          ubv[k] = mt.w;
          xv[k] = !act[k] ? 0u : (sm[k] ? (BIG ? SvG[t] : SvL[t]) : nadj[mt.x + t]);
        }
        // streamed values: one LDS probe each
#pragma unroll
        for (int k = 0; k < kRunU; ++k) hit[k] = act[k] && !sm[k] && run_probe(H, xv[k], shift, bmask);
        // S's values: membership in the prefix's new set in memory
        if (rd.newa >= 0) {
#pragma unroll
          for (int k = 0; k < kRunU; ++k) sds[k] = sm[k] ? cdesc[ci[k]] : 0ull;
          member_lockstep<kRunU>(nadj, nhs, sds, slo, sln, xv, sm, hit);
        } else {
#pragma unroll
          for (int k = 0; k < kRunU; ++k) hit[k] = hit[k] || sm[k];
        }
#pragma unroll
        for (int k = 0; k < kRunU; ++k) {
          if (act[k] && hit[k] && xv[k] >= lbv[k] && xv[k] < ubv[k]) {
            ++hits;
            if (SIGNED) whits += cw[ci[k]];
          }
        }
      }
      __syncthreads();  // the chunk's arrays are read before the next chunk writes them
    }
    if (FUSED) {
      // the task's survivors to its request's counters
      const uint64_t t = block_sum_lean<kRunNT>(hits, s_scan);
      if (tid == 0 && t) {
        atomicAdd(fcnt + rq, (unsigned long long)t);
        atomicAdd(fpre + (uint64_t)rq * kStat + jl + 1, (unsigned long long)t);
        atomicAdd(fws + rq, (unsigned long long)t);
      }
      hits = 0;
    }
    __syncthreads();  // every thread has read this task's shared values before thread 0 claims the next
  }
  if (!FUSED) {
    uint64_t tsum = block_sum<kRunNT>(hits);
    if (tid == 0 && tsum) atomicAdd(acc, (unsigned long long)tsum);
  }
  if (tid == 0) {
    atomicAdd(wsum + 3, (unsigned long long)units);
    atomicAdd(wsum + 4, (unsigned long long)builds);
    atomicAdd(wsum + 5, (unsigned long long)belems);
  }
  if (SIGNED) {
    uint64_t s = block_sum<kRunNT>((uint64_t)whits);
    if (tid == 0 && s) atomicAdd(acc + 1, (unsigned long long)s);
  }
}

// ---------------------------------------------------------------- host
bool run_desc(const StageDesc& d, RunDesc& rd) {
  if (d.ntri || d.k < 1) return false;
  memset(&rd, 0, sizeof(rd));
  rd.newa = -1;
  int r = 0;
  for (int a = 0; a < d.k; ++a) {
    if (d.col[a] == d.j - 1) {
      if (rd.newa >= 0) return false;  // two new atoms: not handled here
      rd.newa = a;
    } else {
      rd.old_mask |= 1u << a;
      ++rd.nold;
      r = std::max(r, d.col[a] + 1);
    }
  }
  if (rd.nold == 0) return false;
  rd.r = r;
  return true;
}

unsigned long long* run_stats_get(gj_ctx* c) {
  if (!c->run_stats) {
    c->run_stats = (unsigned long long*)ws_get(c, "run_stats", 8 * sizeof(unsigned long long));
    GJ_HIP(hipMemsetAsync(c->run_stats, 0, 8 * sizeof(unsigned long long), c->stream));
  }
  return c->run_stats;
}

bool run_count(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off, const uint32_t* minc,
               const StageDesc& d, RunDesc rd, const int8_t* wt, unsigned long long* acc, uint64_t* off2,
               uint64_t& W2, KernelTimer& timer) {
  rd.ratio = c->run_ratio;
  rd.min_work = c->run_min_work;
  rd.task_work = c->run_task_work;
  rd.reuse = c->run_reuse;
  rd.big = c->run_big ? 1u : 0u;
  uint32_t* head = (uint32_t*)ws_get(c, "run_head", n * sizeof(uint32_t) + 16);
  uint64_t* hoff = (uint64_t*)ws_get(c, "run_hoff", (n + 1) * sizeof(uint64_t));
  uint32_t* rs = (uint32_t*)ws_get(c, "run_rs", (n + 1) * sizeof(uint32_t));
  uint32_t* tcnt = (uint32_t*)ws_get(c, "run_tcnt", n * sizeof(uint32_t) + 16);
  uint32_t* tcnt_big = (uint32_t*)ws_get(c, "run_tcnt_big", n * sizeof(uint32_t) + 16);
  uint32_t* minc2 = (uint32_t*)ws_get(c, "run_minc2", n * sizeof(uint32_t) + 16);
  uint64_t* toff = (uint64_t*)ws_get(c, "run_toff", (n + 1) * sizeof(uint64_t));
  uint64_t* toff_big = (uint64_t*)ws_get(c, "run_toff_big", (n + 1) * sizeof(uint64_t));
  uint8_t* staged = (uint8_t*)ws_get(c, "run_staged", n + 16);
  // two task counters (cleared by k_run_starts)
  unsigned int* counter = (unsigned int*)ws_get(c, "run_counter", 16);
  // context-lifetime sums: candidates by plan outcome, and units, builds and
  // built values of the counting kernels (read by gj_ctx_get_option)
  unsigned long long* wsum = run_stats_get(c);
  unsigned gr = grid_for(n, kBlock, 1u << 16);
  k_run_heads<<<gr, kBlock, 0, c->stream>>>(F, stride, n, rd.r, head);
  scan_u32_to_u64(c, head, hoff, n);
  k_run_starts<<<gr, kBlock, 0, c->stream>>>(head, hoff, n, nullptr, rs, counter);
  k_run_plan<<<gr, kBlock, 0, c->stream>>>(F, stride, n, off, head, hoff, rs, d, rd, tcnt, tcnt_big, staged, wsum);
  scan_u32_to_u64(c, tcnt, toff, n);
  scan_u32_to_u64(c, tcnt_big, toff_big, n);
  k_run_direct<<<gr, kBlock, 0, c->stream>>>(head, hoff, staged, n, nullptr, minc, minc2);
  scan_u32_to_u64(c, minc2, off2, n);
  GJ_HIP(hipGetLastError());
  uint64_t h[3];
  read_u64s(c, {off2 + n, toff + n, toff_big + n}, h);
  // too few tasks to occupy the device: a workgroup works through a task
  // alone, so the per-candidate kernel, which spreads every candidate over
  // the whole device, is faster for the stage
  if (h[1] + h[2] < (uint64_t)c->run_min_tasks) {
    c->run_declined += 1;
    return false;
  }
  W2 = h[0];
  if (h[1]) {
    unsigned g = (unsigned)std::min<uint64_t>(h[1], (uint64_t)c->num_cus * 2);
    timer.start();
    if (wt)
      k_run_count<true, false, false><<<g, RunShape<false>::NT, 0, c->stream>>>(F, stride, n, off, hoff, rs, toff, d, rd, wt,
                                                                         nullptr, counter, acc, wsum, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    else
      k_run_count<false, false, false><<<g, RunShape<false>::NT, 0, c->stream>>>(F, stride, n, off, hoff, rs, toff, d, rd,
                                                                          wt, nullptr, counter, acc, wsum, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    timer.stop();
    GJ_HIP(hipGetLastError());
  }
  if (h[2]) {
    unsigned g = (unsigned)std::min<uint64_t>(h[2], (uint64_t)c->num_cus);
    uint32_t* sv = (uint32_t*)ws_get(c, "run_sv", (uint64_t)g * kRunCapBig * sizeof(uint32_t));
    timer.start();
    if (wt)
      k_run_count<true, true, false><<<g, RunShape<true>::NT, 0, c->stream>>>(F, stride, n, off, hoff, rs, toff_big, d, rd,
                                                                       wt, sv, counter + 1, acc, wsum, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    else
      k_run_count<false, true, false><<<g, RunShape<true>::NT, 0, c->stream>>>(F, stride, n, off, hoff, rs, toff_big, d, rd,
                                                                        wt, sv, counter + 1, acc, wsum, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    timer.stop();
    GJ_HIP(hipGetLastError());
  }
  c->run_tasks += h[1] + h[2];
  c->run_tasks_big += h[2];
  return true;
}

// ---------------------------------------------------------------- fused pipeline
// Level j of the fused pipeline holds the prefixes of every request, each
// tagged with its request (rid); a request's stage and run split come from
// the request table R and the split table RDt (ok = 0: the request's
// prefixes stay with the per-candidate kernel).  Every size is read from
// device memory, so the launches below can be captured once and replayed.

// the live size the run kernels take at level j: 0 where the host left the
// level off or where it holds more than rcap prefixes (the run buffers' size)
__global__ void k_runf_setn(BHead* __restrict__ H, int j, uint64_t cap, uint64_t rcap) {
  if (threadIdx.x == 0) {
    const uint64_t nl = H->nlev[j] < cap ? H->nlev[j] : cap;
    H->nrun[j] = H->runon[j] && nl <= rcap ? nl : 0ull;
  }
}

// head[p] = 1 where a run starts: a request's first prefix, or, for a
// request that takes the run kernels, a key column that differs from p - 1
// (a request left to the per-candidate kernel is one run per stretch)
__global__ void k_runf_heads(const uint32_t* __restrict__ F, uint64_t stride, const unsigned long long* __restrict__ np,
                             const uint32_t* __restrict__ rid, const RunDesc* __restrict__ RDt, int j,
                             uint32_t* __restrict__ head) {
  const uint64_t n = *np;
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    const uint32_t r = rid[p];
    uint32_t h = p == 0 || rid[p - 1] != r;
    if (!h) {
      const RunDesc& rd = RDt[(uint64_t)r * kStat + j];
      if (rd.ok)
        for (int c = 0; c < rd.r && !h; ++c) h = F[(uint64_t)c * stride + p] != F[(uint64_t)c * stride + p - 1];
    }
    head[p] = h;
  }
}

// k_run_plan over the level, each run planned with its request's stage
__global__ void k_runf_plan(const uint32_t* __restrict__ F, uint64_t stride, const unsigned long long* __restrict__ np,
                            const uint64_t* __restrict__ off, const uint32_t* __restrict__ head,
                            const uint64_t* __restrict__ hoff, const uint32_t* __restrict__ rs,
                            const BReq* __restrict__ R, const RunDesc* __restrict__ RDt,
                            const uint32_t* __restrict__ rid, int j, uint32_t* __restrict__ tcnt,
                            uint32_t* __restrict__ tcnt_big, uint8_t* __restrict__ staged,
                            unsigned long long* __restrict__ wsum) {
  const uint64_t n = *np;
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  uint64_t ws[3] = {0, 0, 0};
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gs) {
    uint32_t t = 0;
    bool big = false, st = false;
    if (head[p]) {
      const uint64_t run = hoff[p];
      const uint32_t r = rid[p];
      const RunDesc& rd = RDt[(uint64_t)r * kStat + j];
      if (rd.ok) run_plan_one(F, stride, p, rs[run + 1], off, R[r].st[j], rd, st, big, t, ws);
      staged[run] = st ? 1 : 0;
    }
    tcnt[p] = big ? 0 : t;
    tcnt_big[p] = big ? t : 0;
  }
  run_plan_sums(ws, wsum);
}

namespace {
constexpr uint64_t kFusedAlign = 256;
uint64_t fused_round(uint64_t b) { return (b + kFusedAlign - 1) / kFusedAlign * kFusedAlign; }
}  // namespace

uint64_t run_fused_bytes(uint64_t cap, int num_cus) {
  const uint64_t n1 = cap + 1;
  return 5 * fused_round(n1 * sizeof(uint32_t)) + 4 * fused_round(n1 * sizeof(uint64_t)) + fused_round(n1) +
         fused_round(2 * sizeof(unsigned int)) + fused_round((uint64_t)num_cus * kRunCapBig * sizeof(uint32_t));
}

void run_fused_carve(RunFusedBufs& b, void* base, uint64_t cap, int num_cus, unsigned long long* stats) {
  const uint64_t n1 = cap + 1;
  char* q = (char*)base;
  auto take = [&](uint64_t bytes) {
    char* r = q;
    q += fused_round(bytes);
    return (void*)r;
  };
  b.cap = cap;
  b.num_cus = num_cus;
  b.head = (uint32_t*)take(n1 * sizeof(uint32_t));
  b.rs = (uint32_t*)take(n1 * sizeof(uint32_t));
  b.tcnt = (uint32_t*)take(n1 * sizeof(uint32_t));
  b.tcnt_big = (uint32_t*)take(n1 * sizeof(uint32_t));
  b.minc2 = (uint32_t*)take(n1 * sizeof(uint32_t));
  b.hoff = (uint64_t*)take(n1 * sizeof(uint64_t));
  b.toff = (uint64_t*)take(n1 * sizeof(uint64_t));
  b.toff_big = (uint64_t*)take(n1 * sizeof(uint64_t));
  b.off2 = (uint64_t*)take(n1 * sizeof(uint64_t));
  b.staged = (uint8_t*)take(n1);
  b.counter = (unsigned int*)take(2 * sizeof(unsigned int));
  b.sv = (uint32_t*)take((uint64_t)num_cus * kRunCapBig * sizeof(uint32_t));
  b.stats = stats;
}

void run_fused_level(hipStream_t st, const RunFusedBufs& b, const BReq* R, const RunDesc* RDt, BHead* H, int j,
                     const uint32_t* F, const uint32_t* rid, uint64_t cap, const uint64_t* off,
                     const uint32_t* minc, uint64_t* part, uint64_t* part_off, unsigned long long* cnt,
                     unsigned long long* pre, unsigned long long* wsum) {
  GJ_CHECK(b.cap <= cap, GJ_EINVAL, "run buffers larger than the level capacity");
  const unsigned long long* np = &H->nrun[j];
  const uint64_t rc = b.cap;
  const unsigned gr = (unsigned)b.num_cus * 8;  // grid-stride over the live level
  k_runf_setn<<<1, 64, 0, st>>>(H, j, cap, rc);
  k_runf_heads<<<gr, kBlock, 0, st>>>(F, cap, np, rid, RDt, j, b.head);
  bt_scan_n(st, b.head, np, rc, part, part_off, b.hoff);
  k_run_starts<<<gr, kBlock, 0, st>>>(b.head, b.hoff, 0, np, b.rs, b.counter);
  k_runf_plan<<<gr, kBlock, 0, st>>>(F, cap, np, off, b.head, b.hoff, b.rs, R, RDt, rid, j, b.tcnt, b.tcnt_big,
                                     b.staged, b.stats);
  bt_scan_n(st, b.tcnt, np, rc, part, part_off, b.toff);
  bt_scan_n(st, b.tcnt_big, np, rc, part, part_off, b.toff_big);
  k_run_direct<<<gr, kBlock, 0, st>>>(b.head, b.hoff, b.staged, 0, np, minc, b.minc2);
  bt_scan_n(st, b.minc2, np, rc, part, part_off, b.off2);
  const StageDesc d0{};
  const RunDesc rd0{};
  // a fixed grid (idle workgroups exit at once): two small-shape workgroups
  // per CU, one large-shape one
  k_run_count<false, false, true><<<(unsigned)b.num_cus * 2, RunShape<false>::NT, 0, st>>>(
      F, cap, 0, off, b.hoff, b.rs, b.toff, d0, rd0, nullptr, nullptr, b.counter, nullptr, b.stats, R, j, rid, RDt,
      np, cnt, pre, wsum);
  k_run_count<false, true, true><<<(unsigned)b.num_cus, RunShape<true>::NT, 0, st>>>(
      F, cap, 0, off, b.hoff, b.rs, b.toff_big, d0, rd0, nullptr, b.sv, b.counter + 1, nullptr, b.stats, R, j, rid,
      RDt, np, cnt, pre, wsum);
  GJ_HIP(hipGetLastError());
}

}  // namespace gj
