// Batched execution: many count requests (query, seed slice) fused stage by
// stage into one pipeline whose sizes live in device memory, captured once as
// a hipGraph and replayed.
//
// Every prefix carries the id of its request; the per-request query plans
// (seed index, filters, binding atoms of every stage, in the version the
// request reads) sit in a device table.  Level j holds the prefixes of length
// j of every request that has not finished; one count-minimisation pass, one
// scan and one propose+intersect pass per level serve all of them, so
// frontiers of very different sizes share launches (the synchronous dataflow
// primitive of Sec. 3.1.1 applied to all requests at once).  Requests whose
// query ends at attribute j+1 are counted there; the others are compacted into
// level j+1 with one atomic per wave.  If a level would exceed its capacity
// the run reports it and the host reruns the batch one request at a time on
// the depth-first path, whose frontiers are bounded.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "batch.h"
#include "engine.h"
#include "gj_internal.h"
#include "prim.h"
#include "run.h"

namespace gj {



__device__ __forceinline__ bool member(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi, uint32_t x,
                                       uint32_t lin) {
  if (hi - lo <= lin) {
    for (uint32_t i = lo; i < hi; ++i) {
      uint32_t y = a[i];
      if (y >= x) return y == x;
    }
    return false;
  }
  return contains_u32(a, lo, hi, x);
}

// Wave-resident accumulator of arr[key] += val: runs of iterations that agree
// on one key add in registers and flush with a single atomic when the key
// changes (or at the end); a wave mixing keys reduces per distinct key.  key
// and the running sum are wave-uniform.
struct WaveAcc {
  uint32_t key = 0xFFFFFFFFu;
  uint64_t sum = 0;
  __device__ __forceinline__ void flush(unsigned long long* arr) {
    if (lane_id() == 0 && sum && key != 0xFFFFFFFFu) atomicAdd(&arr[key], (unsigned long long)sum);
    sum = 0;
  }
  __device__ __forceinline__ void add(unsigned long long* arr, uint32_t k, uint64_t val, bool active, bool unit) {
    uint64_t act = __ballot(active);
    if (!act) return;
    int leader = __ffsll((unsigned long long)act) - 1;
    uint32_t k0 = __builtin_amdgcn_readfirstlane(__shfl(k, leader, 64));
    if (__ballot(active && k != k0) == 0) {
      uint64_t s = unit ? (uint64_t)__popcll(act) : wave_sum(active ? val : 0);
      if (k0 != key) {
        flush(arr);
        key = k0;
      }
      sum += s;
    } else {
      // mixed keys: one reduction and one atomic per distinct key
      bool todo = active;
      while (__ballot(todo)) {
        uint64_t m = __ballot(todo);
        int l = __ffsll((unsigned long long)m) - 1;
        uint32_t kc = __builtin_amdgcn_readfirstlane(__shfl(k, l, 64));
        bool mine = todo && k == kc;
        uint64_t s = unit ? (uint64_t)__popcll(__ballot(mine)) : wave_sum(mine ? val : 0);
        if (lane_id() == l && s) atomicAdd(&arr[kc], (unsigned long long)s);
        todo = todo && !mine;
      }
    }
  }
};

// wave-level slot reservation for the active lanes in an unordered buffer
__device__ __forceinline__ uint64_t wave_reserve(unsigned long long* counter, bool active) {
  uint64_t b = __ballot(active);
  uint64_t base = 0;
  if (lane_id() == 0 && b) base = atomicAdd(counter, (unsigned long long)__popcll(b));
  base = shfl_u64(base, 0);
  return base + __popcll(b & lanemask_lt());
}

__global__ void k_bt_clear(unsigned long long* __restrict__ p, uint64_t n) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) p[i] = 0;
}

__global__ void k_bt_head_reset(BHead* h) {
  if (threadIdx.x == 0) {
    for (int j = 0; j <= GJ_MAX_ATTRS; ++j) h->nlev[j] = h->claim[j] = 0;
    h->overflow = 0;
  }
}

// P_2 of every request: seed g of the concatenated seed space -> request r.
// A wave takes blocks of kSeedBlock consecutive seeds: it first counts the
// block's survivors, reserves their slots with one atomic, then writes them
// in seed order, so the prefixes of a run (seeds sharing x0) stay together
// across a block instead of being cut every 64 seeds.
constexpr uint32_t kSeedSub = 16;               // 64-seed steps per block
constexpr uint64_t kSeedBlock = 64 * kSeedSub;  // seeds per block

// The seed's request, values, weight, and whether it is in P_2 (keep) and
// ends its query there (fin).
__device__ __forceinline__ void seed_at(const BReq* __restrict__ R, const uint64_t* __restrict__ roff,
                                        uint32_t nreq, uint64_t g, uint32_t& r, uint32_t& x0, uint32_t& x1,
                                        int8_t& w, bool& keep, bool& fin) {
  r = (uint32_t)find_segment(roff, 0, nreq, g);
  const BReq& q = R[r];
  const uint64_t e = q.seed_lo + (g - roff[r]);
  x0 = q.seed_row[e];
  x1 = q.seed_col[e];
  w = q.seed_w ? q.seed_w[e] : (int8_t)1;
  keep = true;
  const uint32_t x[2] = {x0, x1};
  for (int a = 0; a < q.filt.n && keep; ++a) {
    const uint32_t key = x[q.filt.key[a]], val = x[q.filt.val[a]];
    uint32_t lo, hi;
    row_range(q.filt.rp[a], q.filt.pm[a], key, lo, hi);
    keep = contains_u32(q.filt.adj[a], lo, hi, val);
  }
  keep = keep && seed_ineq_ok(q.filt.above, q.filt.below, x0, x1);
  fin = q.m == 2;
}

__global__ void __launch_bounds__(kBlock) k_bt_seed(const BReq* __restrict__ R, const uint64_t* __restrict__ roff,
                                                    BHead* __restrict__ H, uint32_t* __restrict__ F,
                                                    uint32_t* __restrict__ rid, int8_t* __restrict__ Fw, uint64_t cap,
                                                    unsigned long long* __restrict__ cnt,
                                                    unsigned long long* __restrict__ pre,
                                                    unsigned long long* __restrict__ wsum) {
  const uint32_t nreq = H->nreq;
  const uint64_t total = H->seeds;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const int lane = lane_id();
  WaveAcc a_pre, a_cnt, a_ws;
  for (uint64_t blk = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; blk * kSeedBlock < total;
       blk += nwaves) {
    const uint64_t b0 = blk * kSeedBlock;
    // pass 1: counters, and the block's survivors that go on to level 3
    uint32_t nstore = 0;
    for (uint32_t k = 0; k < kSeedSub; ++k) {
      const uint64_t g = b0 + (uint64_t)k * 64 + lane;
      const bool valid = g < total;
      uint32_t r = 0, x0 = 0, x1 = 0;
      int8_t w = 1;
      bool keep = false, fin = false;
      if (valid) seed_at(R, roff, nreq, g, r, x0, x1, w, keep, fin);
      a_pre.add(pre, r * kStat + 2, 1, valid && keep, true);
      a_cnt.add(cnt, r, 1, valid && keep && fin, true);
      a_ws.add(wsum, r, (uint64_t)(int64_t)w, valid && keep && fin, false);
      nstore += (uint32_t)__popcll(__ballot(valid && keep && !fin));
    }
    if (nstore == 0) continue;
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd(&H->nlev[2], (unsigned long long)nstore);
    base = shfl_u64(base, 0);
    // pass 2: the survivors in seed order
    for (uint32_t k = 0; k < kSeedSub; ++k) {
      const uint64_t g = b0 + (uint64_t)k * 64 + lane;
      const bool valid = g < total;
      uint32_t r = 0, x0 = 0, x1 = 0;
      int8_t w = 1;
      bool keep = false, fin = false;
      if (valid) seed_at(R, roff, nreq, g, r, x0, x1, w, keep, fin);
      const bool store = valid && keep && !fin;
      const uint64_t bal = __ballot(store);
      if (store) {
        const uint64_t pos = base + (uint64_t)__popcll(bal & lanemask_lt());
        if (pos < cap) {
          F[pos] = x0;
          F[cap + pos] = x1;
          rid[pos] = r;
          Fw[pos] = w;
        } else {
          atomicOr(&H->overflow, 1u);
        }
      }
      base += (uint64_t)__popcll(bal);
    }
  }
  a_pre.flush(pre);
  a_cnt.flush(cnt);
  a_ws.flush(wsum);
}

// The lanes of a wave are served one request at a time: the first pending
// request id is made wave-uniform, its plan is read with scalar loads into
// registers (loops over binding atoms fully unrolled), and the lanes of that
// request run; a wave spanning a request boundary takes a second pass.
__device__ __forceinline__ uint32_t first_pending(uint32_t r, bool todo) {
  uint64_t m = __ballot(todo);
  int l = __ffsll((unsigned long long)m) - 1;
  return __builtin_amdgcn_readfirstlane(__shfl(r, l, 64));
}

__global__ void __launch_bounds__(kBlock) k_bt_count_min(const BReq* __restrict__ R, int j, BHead* __restrict__ H,
                                                         const uint32_t* __restrict__ F,
                                                         const uint32_t* __restrict__ rid, uint64_t cap,
                                                         uint32_t* __restrict__ minc, uint8_t* __restrict__ mini,
                                                         unsigned long long* __restrict__ ext) {
  uint64_t n = H->nlev[j] < cap ? H->nlev[j] : cap;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  WaveAcc a_ext;
  for (uint64_t base = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) << 6; base < n;
       base += nwaves * 64) {
    uint64_t p = base + lane_id();
    bool valid = p < n;
    uint32_t r = valid ? rid[p] : 0u, best = 0;
    bool todo = valid;
    while (__ballot(todo)) {
      uint32_t rc = first_pending(r, todo);
      const StageDesc d = R[rc].st[j];
      if (todo && r == rc) {
        best = 0xFFFFFFFFu;
        int bi = 0;
#pragma unroll
        for (int a = 0; a < kMaxBind; ++a) {
          if (a < d.k) {
            uint32_t v = F[(uint64_t)d.col[a] * cap + p], lo, hi;
            row_range(d.rp[a], d.pm[a], v, lo, hi);
            uint32_t c = hi - lo;
            if (c < best) {
              best = c;
              bi = a;
            }
          }
        }
        minc[p] = best;
        mini[p] = (uint8_t)bi;
        todo = false;
      }
    }
    a_ext.add(ext, r * kStat + j, best, valid, false);
  }
  a_ext.flush(ext);
}

__global__ void __launch_bounds__(kBlock) k_bt_propose(const BReq* __restrict__ R, int j, BHead* __restrict__ H,
                                                       const uint32_t* __restrict__ F,
                                                       const uint32_t* __restrict__ rid, uint64_t cap,
                                                       const uint64_t* __restrict__ off_all,
                                                       const uint64_t* __restrict__ off_left,
                                                       const uint8_t* __restrict__ mini, const int8_t* __restrict__ Fw,
                                                       uint32_t* __restrict__ G, uint32_t* __restrict__ grid_,
                                                       int8_t* __restrict__ Gw, uint64_t gcap,
                                                       uint32_t* __restrict__ par, uint64_t par_cap,
                                                       unsigned long long* __restrict__ cnt,
                                                       unsigned long long* __restrict__ pre,
                                                       unsigned long long* __restrict__ wsum) {
  const uint64_t n = H->nlev[j] < cap ? H->nlev[j] : cap;
  // the candidates the run kernels left (staged runs' prefixes have none),
  // where they took the level
  const uint64_t* __restrict__ off = H->nrun[j] > 0 ? off_left : off_all;
  const uint64_t W = off[n];
  const uint32_t lin = H->lin;
  const uint64_t claim = H->claim_words;
  const int lane = lane_id();
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t nwords = (W + 63) >> 6;
  (void)nwaves;
  WaveAcc a_pre, a_cnt, a_ws;
  // waves claim chunks of `claim` words from a device counter and walk each
  // chunk galloping forward over the prefixes
  for (;;) {
    uint64_t cb = 0;
    if (lane == 0) cb = atomicAdd(&H->claim[j], 1ull);
    cb = shfl_u64(cb, 0) * claim;
    if (cb >= nwords) break;
    uint64_t ce = cb + claim < nwords ? cb + claim : nwords;
    uint64_t plo = find_segment(off, 0, n, cb << 6);
  for (uint64_t wd = cb; wd < ce; ++wd) {
    uint64_t gf = wd << 6;
    uint64_t gl = gf + 63 < W ? gf + 63 : W - 1;
    plo = gallop_segment(off, plo, n, gf);
    uint64_t phi = gallop_segment(off, plo, n, gl) + 1;
    uint64_t g = gf + lane;
    bool valid = g < W, keep = false, fin = false;
    uint32_t r = 0, e = 0;
    uint64_t p = 0;
    if (valid) {
      p = find_segment(off, plo, phi, g);
      r = rid[p];
    }
    bool todo = valid;
    while (__ballot(todo)) {
      uint32_t rc = first_pending(r, todo);
      const StageDesc d = R[rc].st[j];
      const uint32_t mc = R[rc].m;
      if (todo && r == rc) {
        uint32_t k = (uint32_t)(g - off[p]);
        int am = mini[p];
        const uint32_t* rp_m = d.rp[0];
        const uint32_t* adj_m = d.adj[0];
        const uint64_t* pm_m = d.pm[0];
        int col_m = d.col[0];
#pragma unroll
        for (int a = 1; a < kMaxBind; ++a) {
          if (a == am) {
            rp_m = d.rp[a];
            adj_m = d.adj[a];
            pm_m = d.pm[a];
            col_m = d.col[a];
          }
        }
        uint32_t v = F[(uint64_t)col_m * cap + p], vlo, vhi;
        row_range(rp_m, pm_m, v, vlo, vhi);
        e = adj_m[vlo + k];
        keep = ineq_ok(F, cap, p, d.above, d.below, e);
#pragma unroll
        for (int a = 0; a < kMaxBind; ++a) {
          if (a < d.k && a != am && keep) {
            uint32_t u = F[(uint64_t)d.col[a] * cap + p], lo, hi;
            uint64_t dd = d.hd[a] ? d.hd[a][u] : 0ull;
            if (dd) {
              keep = hash_member(d.hs[a], dd, e);
            } else {
              row_range(d.rp[a], d.pm[a], u, lo, hi);
              keep = member(d.adj[a], lo, hi, e, lin);
            }
          }
        }
        fin = mc == (uint32_t)(j + 1);
        todo = false;
      }
    }
    int8_t w = valid ? Fw[p] : (int8_t)0;
    a_pre.add(pre, r * kStat + j + 1, 1, valid && keep, true);
    a_cnt.add(cnt, r, 1, valid && keep && fin, true);
    a_ws.add(wsum, r, (uint64_t)(int64_t)w, valid && keep && fin, false);
    bool store = valid && keep && !fin;
    uint64_t pos = wave_reserve(&H->nlev[j + 1], store);
    if (store) {
      if (pos < gcap) {
        for (int c = 0; c < j; ++c) G[(uint64_t)c * gcap + pos] = F[(uint64_t)c * cap + p];
        G[(uint64_t)j * gcap + pos] = e;
        grid_[pos] = r;
        Gw[pos] = w;
        if (pos < par_cap) par[pos] = (uint32_t)p;
      } else {
        atomicOr(&H->overflow, 1u);
      }
    }
  }
  }
  a_pre.flush(pre);
  a_cnt.flush(cnt);
  a_ws.flush(wsum);
}

// ---------------------------------------------------------------- device-size scan
constexpr int kBtTile = kBlock * 8;

// The scan kernels walk tiles with a fixed grid and stop at the live level
// size, so a small level costs a few tiles whatever the capacity.
constexpr unsigned kScanGrid = 1024;

__global__ void __launch_bounds__(kBlock) k_bt_scan_reduce(const uint32_t* __restrict__ in,
                                                           const unsigned long long* __restrict__ np, uint64_t cap,
                                                           uint64_t* __restrict__ part) {
  uint64_t n = *np < cap ? *np : cap;
  uint64_t tiles = (n + kBtTile - 1) / kBtTile + 1;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    uint64_t base = t * kBtTile;
    uint64_t s = 0;
    for (int i = 0; i < 8; ++i) {
      uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
      if (idx < n) s += in[idx];
    }
    s = block_sum<kBlock>(s);
    if (threadIdx.x == 0) part[t] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_bt_scan_down(const uint32_t* __restrict__ in,
                                                         const unsigned long long* __restrict__ np, uint64_t cap,
                                                         const uint64_t* __restrict__ part_off,
                                                         uint64_t* __restrict__ out) {
  __shared__ uint64_t tile[kBtTile];
  uint64_t n = *np < cap ? *np : cap;
  uint64_t tiles = (n + kBtTile - 1) / kBtTile + 1;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    uint64_t base = t * kBtTile;
    for (int i = 0; i < 8; ++i) {
      uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
      tile[i * kBlock + threadIdx.x] = idx < n ? in[idx] : 0;
    }
    __syncthreads();
    uint64_t loc[8], s = 0;
    for (int i = 0; i < 8; ++i) {
      loc[i] = tile[threadIdx.x * 8 + i];
      s += loc[i];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<kBlock, uint64_t>(s, tot) + part_off[t];
    for (int i = 0; i < 8; ++i) {
      tile[threadIdx.x * 8 + i] = run;
      run += loc[i];
    }
    __syncthreads();
    for (int i = 0; i < 8; ++i) {
      uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
      if (idx <= n) out[idx] = idx < n ? tile[i * kBlock + threadIdx.x] : part_off[tiles];
    }
    __syncthreads();
  }
}

// exclusive scan of the block sums of the live tiles, one workgroup
__global__ void __launch_bounds__(kBlock) k_bt_scan_parts(const uint64_t* __restrict__ part,
                                                          const unsigned long long* __restrict__ np, uint64_t cap,
                                                          uint64_t* __restrict__ out) {
  uint64_t nl = *np < cap ? *np : cap;
  uint64_t n = (nl + kBtTile - 1) / kBtTile + 1;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < n; base += kBtTile) {
    uint64_t loc[8], s = 0;
    for (int i = 0; i < 8; ++i) {
      uint64_t idx = base + (uint64_t)threadIdx.x * 8 + i;
      loc[i] = idx < n ? part[idx] : 0;
      s += loc[i];
    }
    uint64_t tot;
    uint64_t run = carry + block_excl_scan<kBlock, uint64_t>(s, tot);
    for (int i = 0; i < 8; ++i) {
      uint64_t idx = base + (uint64_t)threadIdx.x * 8 + i;
      if (idx < n) out[idx] = run;
      run += loc[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

void bt_scan_n(hipStream_t st, const uint32_t* in, const unsigned long long* n, uint64_t cap, uint64_t* part,
               uint64_t* part_off, uint64_t* out) {
  k_bt_scan_reduce<<<kScanGrid, kBlock, 0, st>>>(in, n, cap, part);
  k_bt_scan_parts<<<1, kBlock, 0, st>>>(part, n, cap, part_off);
  k_bt_scan_down<<<kScanGrid, kBlock, 0, st>>>(in, n, cap, part_off, out);
}

void bt_scan(hipStream_t st, const uint32_t* in, const BHead* H, int j, uint64_t cap, uint64_t* part,
             uint64_t* part_off, uint64_t* out) {
  bt_scan_n(st, in, &H->nlev[j], cap, part, part_off, out);
}

// ---------------------------------------------------------------- regrouping by parent
// The fused propose kernel writes a level in the order its waves reserve
// space, so the children of one prefix arrive in pieces of at most 64 (one
// word of candidates each) spread over the level.  Before a level whose last
// stage takes the run kernels, a counting sort by parent index puts the
// children of every prefix side by side (in arbitrary order among
// themselves), so the runs, whose key columns are all parent columns, come
// whole.  Levels or parent levels above the buffers' size keep their order.

__global__ void k_bt_reg_setn(BHead* __restrict__ H, int j, uint64_t cap, uint64_t rcap) {
  if (threadIdx.x == 0) {
    const uint64_t nc = H->nlev[j] < cap ? H->nlev[j] : cap;
    const uint64_t np = H->nlev[j - 1] < cap ? H->nlev[j - 1] : cap;
    const bool on = H->runon[j] && nc <= rcap && np <= rcap;
    H->nreg[j] = on ? nc : 0ull;
    H->nregp[j] = on ? np : 0ull;
  }
}

__global__ void k_bt_reg_clear(uint32_t* __restrict__ hist, const unsigned long long* __restrict__ np) {
  const uint64_t n = *np;
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) hist[i] = 0;
}

// children per parent: one atomic per distinct parent in a wave (a wave's
// lanes hold a few pieces, each of one parent)
__global__ void __launch_bounds__(kBlock) k_bt_reg_hist(const uint32_t* __restrict__ par,
                                                        const unsigned long long* __restrict__ nc,
                                                        uint32_t* __restrict__ hist) {
  const uint64_t n = *nc;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) << 6; base < n;
       base += nwaves * 64) {
    const uint64_t i = base + lane_id();
    const bool valid = i < n;
    const uint32_t k = valid ? par[i] : 0u;
    bool todo = valid;
    while (__ballot(todo)) {
      const uint32_t kc = first_pending(k, todo);
      const bool mine = todo && k == kc;
      const uint64_t mm = __ballot(mine);
      if (lane_id() == __ffsll((unsigned long long)mm) - 1) atomicAdd(&hist[kc], (uint32_t)__popcll(mm));
      todo = todo && !mine;
    }
  }
}

// Each child to its slot in its parent's range (poff[parent] + a slot taken
// by counting the parent's histogram entry down, once per distinct parent in
// a wave): columns, request and weight into the staging buffers.
__global__ void __launch_bounds__(kBlock) k_bt_reg_scatter(const uint32_t* __restrict__ par,
                                                           const unsigned long long* __restrict__ nc,
                                                           uint32_t* __restrict__ hist,
                                                           const uint64_t* __restrict__ poff, int j,
                                                           const uint32_t* __restrict__ F, uint64_t cap,
                                                           const uint32_t* __restrict__ rid,
                                                           const int8_t* __restrict__ Fw,
                                                           uint32_t* __restrict__ T, uint64_t rcap,
                                                           uint32_t* __restrict__ trid, int8_t* __restrict__ tw) {
  const uint64_t n = *nc;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) << 6; base < n;
       base += nwaves * 64) {
    const uint64_t i = base + lane_id();
    const bool valid = i < n;
    const uint32_t k = valid ? par[i] : 0u;
    uint32_t slot = 0;
    bool todo = valid;
    while (__ballot(todo)) {
      const uint32_t kc = first_pending(k, todo);
      const bool mine = todo && k == kc;
      const uint64_t mm = __ballot(mine);
      const int leader = __ffsll((unsigned long long)mm) - 1;
      const uint32_t cntk = (uint32_t)__popcll(mm);
      uint32_t top = 0;
      if (lane_id() == leader) top = atomicSub(&hist[kc], cntk);
      top = __shfl(top, leader, 64);
      if (mine) slot = top - cntk + (uint32_t)__popcll(mm & lanemask_lt());
      todo = todo && !mine;
    }
    if (valid) {
      const uint64_t pos = poff[k] + slot;
      for (int c = 0; c < j; ++c) T[(uint64_t)c * rcap + pos] = F[(uint64_t)c * cap + i];
      trid[pos] = rid[i];
      tw[pos] = Fw[i];
    }
  }
}

__global__ void k_bt_reg_copy(const unsigned long long* __restrict__ nc, int j, const uint32_t* __restrict__ T,
                              uint64_t rcap, const uint32_t* __restrict__ trid, const int8_t* __restrict__ tw,
                              uint32_t* __restrict__ F, uint64_t cap, uint32_t* __restrict__ rid,
                              int8_t* __restrict__ Fw) {
  const uint64_t n = *nc;
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) {
    for (int c = 0; c < j; ++c) F[(uint64_t)c * cap + i] = T[(uint64_t)c * rcap + i];
    rid[i] = trid[i];
    Fw[i] = tw[i];
  }
}

// ---------------------------------------------------------------- executor
struct BatchExec::Impl {
  uint32_t max_req = 0;
  int max_m = 0;
  uint64_t cap = 0;
  BReq* d_req = nullptr;
  uint64_t* d_roff = nullptr;
  BHead* d_head = nullptr;
  unsigned long long* d_stat = nullptr;  // cnt[mr], wsum[mr], pre[mr * kStat], ext[mr * kStat]
  uint32_t* F[GJ_MAX_ATTRS + 1] = {};
  uint32_t* rid[GJ_MAX_ATTRS + 1] = {};
  int8_t* W[GJ_MAX_ATTRS + 1] = {};
  uint32_t* minc[GJ_MAX_ATTRS + 1] = {};
  uint8_t* mini[GJ_MAX_ATTRS + 1] = {};
  uint64_t* off[GJ_MAX_ATTRS + 1] = {};
  uint64_t* part = nullptr;
  uint64_t* part_off = nullptr;
  uint64_t nparts = 0;
  // run kernels of the last stage (run.h), when captured into the pipeline:
  // their buffers and the per-request, per-level split table
  bool runs = false;
  RunFusedBufs rb;
  RunDesc* d_rdt = nullptr;
  // regrouping by parent (levels of at most rcap prefixes): the parent index
  // of each prefix of the level being written, the per-parent histogram and
  // offsets, and staging for the regrouped level (columns stride rcap)
  uint64_t rcap = 0;
  uint32_t* par = nullptr;
  uint32_t* rg_hist = nullptr;
  uint64_t* rg_off = nullptr;
  uint32_t* rg_F = nullptr;
  uint32_t* rg_rid = nullptr;
  int8_t* rg_w = nullptr;
  void* h_stage = nullptr;  // pinned staging for the request table and results
  size_t h_stage_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned grid_cfg = 0;
  std::vector<void*> allocs;
  gj_ctx* owner = nullptr;  // the context whose allocator holds allocs

  uint64_t stat_words() const { return (uint64_t)max_req * (2 + 2 * kStat); }
  uint64_t rdt_entries() const { return (uint64_t)max_req * kStat; }
  unsigned long long* cnt() { return d_stat; }
  unsigned long long* wsum() { return d_stat + max_req; }
  unsigned long long* pre() { return d_stat + 2ull * max_req; }
  unsigned long long* ext() { return d_stat + 2ull * max_req + (uint64_t)max_req * kStat; }
  std::vector<size_t> alloc_bytes;
  void* alloc(size_t b) {
    void* p = dev_alloc(owner, b);
    allocs.push_back(p);
    alloc_bytes.push_back(b);
    return p;
  }
  ~Impl() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : allocs) dev_free(owner, p);
    if (h_stage) (void)hipHostFree(h_stage);
  }
};

BatchExec::BatchExec() : p(new Impl) {}
BatchExec::~BatchExec() { delete p; }

static void enqueue(gj_ctx* c, BatchExec::Impl& s, unsigned grid) {
  hipStream_t st = c->stream;
  k_bt_head_reset<<<1, 64, 0, st>>>(s.d_head);
  k_bt_clear<<<grid_for(s.stat_words(), kBlock, 1024), kBlock, 0, st>>>(s.d_stat, s.stat_words());
  k_bt_seed<<<grid, kBlock, 0, st>>>(s.d_req, s.d_roff, s.d_head, s.F[2], s.rid[2], s.W[2], s.cap, s.cnt(),
                                     s.pre(), s.wsum());
  for (int j = 2; j < s.max_m; ++j) {
    if (s.runs && j >= 3) {
      // children of one prefix side by side for the run kernels (a no-op
      // where the host left level j off or it is too large)
      const unsigned gr = (unsigned)c->num_cus * 8;
      const unsigned long long* nc = &s.d_head->nreg[j];
      const unsigned long long* np = &s.d_head->nregp[j];
      k_bt_reg_setn<<<1, 64, 0, st>>>(s.d_head, j, s.cap, s.rcap);
      k_bt_reg_clear<<<gr, kBlock, 0, st>>>(s.rg_hist, np);
      k_bt_reg_hist<<<gr, kBlock, 0, st>>>(s.par, nc, s.rg_hist);
      bt_scan_n(st, s.rg_hist, np, s.rcap, s.part, s.part_off, s.rg_off);
      k_bt_reg_scatter<<<gr, kBlock, 0, st>>>(s.par, nc, s.rg_hist, s.rg_off, j, s.F[j], s.cap, s.rid[j], s.W[j],
                                              s.rg_F, s.rcap, s.rg_rid, s.rg_w);
      k_bt_reg_copy<<<gr, kBlock, 0, st>>>(nc, j, s.rg_F, s.rcap, s.rg_rid, s.rg_w, s.F[j], s.cap, s.rid[j],
                                           s.W[j]);
    }
    // latency-bound, no dynamic claiming: oversubscribe (idle blocks exit at once)
    k_bt_count_min<<<grid_for(s.cap, kBlock * 4, 8192), kBlock, 0, st>>>(s.d_req, j, s.d_head, s.F[j], s.rid[j],
                                                                         s.cap, s.minc[j], s.mini[j], s.ext());
    bt_scan(st, s.minc[j], s.d_head, j, s.cap, s.part, s.part_off, s.off[j]);
    if (s.runs)
      run_fused_level(st, s.rb, s.d_req, s.d_rdt, s.d_head, j, s.F[j], s.rid[j], s.cap, s.off[j], s.minc[j], s.part,
                      s.part_off, s.cnt(), s.pre(), s.wsum());
    bool last = j + 1 >= s.max_m;
    k_bt_propose<<<grid, kBlock, 0, st>>>(s.d_req, j, s.d_head, s.F[j], s.rid[j], s.cap, s.off[j],
                                         s.runs ? s.rb.off2 : s.off[j], s.mini[j], s.W[j],
                                         last ? nullptr : s.F[j + 1], last ? nullptr : s.rid[j + 1],
                                         last ? nullptr : s.W[j + 1], last ? 0 : s.cap,
                                         last || !s.runs ? nullptr : s.par, last || !s.runs ? 0 : s.rcap, s.cnt(),
                                         s.pre(), s.wsum());
  }
}

void BatchExec::run_specs(gj_ctx* c, const std::vector<ReqSpec>& specs, uint64_t* counts, int64_t* wsums,
                          gj_stats* stats, bool& overflow) {
  overflow = false;
  uint32_t nreq = (uint32_t)specs.size();
  if (!nreq) return;
  int max_m = 2;
  for (auto& r : specs) max_m = std::max(max_m, r.P.m);
  uint64_t cap = c->batch_cap;
  unsigned grid = (unsigned)c->num_cus * (c->batch_waves_per_cu / 4 > 0 ? c->batch_waves_per_cu / 4 : 1);
  Impl& s = *p;
  // the run kernels enter the captured pipeline once a batch has a request
  // whose last stage they can take (static counts; a context that only runs
  // signed delta batches never allocates their buffers), and stay
  auto groupable = [&](const ReqSpec& r) {
    RunDesc rd;
    return !r.w && r.P.m >= 3 && c->run_stage && c->strategy != 1 && run_desc(stage_desc(r.P, r.V, r.P.m - 1), rd);
  };
  bool runs = false;
  if (c->batch_run) {
    runs = s.runs;
    for (uint32_t i = 0; i < nreq && !runs; ++i) runs = groupable(specs[i]);
  }
  bool rebuild = nreq > s.max_req || max_m > s.max_m || cap != s.cap || grid != s.grid_cfg || runs != s.runs ||
                 !s.exec;
  if (rebuild) {
    uint32_t mr = std::max<uint32_t>(nreq, std::max<uint32_t>(s.max_req, 64));
    int mm = std::max(max_m, std::max(s.max_m, 3));
    GJ_HIP(hipStreamSynchronize(c->stream));
    delete p;
    p = new Impl;
    Impl& t = *p;
    t.owner = c;
    t.max_req = mr;
    t.max_m = mm;
    t.cap = cap;
    t.grid_cfg = grid;
    t.d_req = (BReq*)t.alloc(sizeof(BReq) * mr);
    t.d_roff = (uint64_t*)t.alloc(sizeof(uint64_t) * (mr + 1));
    t.d_head = (BHead*)t.alloc(sizeof(BHead));
    t.d_stat = (unsigned long long*)t.alloc(sizeof(unsigned long long) * t.stat_words());
    for (int j = 2; j < mm; ++j) {
      t.F[j] = (uint32_t*)t.alloc(cap * j * sizeof(uint32_t));
      t.rid[j] = (uint32_t*)t.alloc(cap * sizeof(uint32_t));
      t.W[j] = (int8_t*)t.alloc(cap);
      t.minc[j] = (uint32_t*)t.alloc(cap * sizeof(uint32_t));
      t.mini[j] = (uint8_t*)t.alloc(cap);
      t.off[j] = (uint64_t*)t.alloc((cap + 1) * sizeof(uint64_t));
    }
    t.nparts = (cap + kBtTile - 1) / kBtTile + 1;
    t.part = (uint64_t*)t.alloc(t.nparts * sizeof(uint64_t));
    t.part_off = (uint64_t*)t.alloc((t.nparts + 1) * sizeof(uint64_t));
    t.runs = runs;
    if (runs) {
      // levels of up to 2^25 prefixes take the run kernels (larger ones keep
      // the per-candidate kernel), so the buffers stay below 2 GB
      const uint64_t rcap = std::min<uint64_t>(cap, 1ull << 25);
      unsigned long long* stats = run_stats_get(c);  // cleared here, outside the capture
      run_fused_carve(t.rb, t.alloc(run_fused_bytes(rcap, c->num_cus)), rcap, c->num_cus, stats);
      t.d_rdt = (RunDesc*)t.alloc(sizeof(RunDesc) * t.rdt_entries());
      t.rcap = rcap;
      if (mm > 3) {
        t.par = (uint32_t*)t.alloc(rcap * sizeof(uint32_t));
        t.rg_hist = (uint32_t*)t.alloc((rcap + 1) * sizeof(uint32_t));
        t.rg_off = (uint64_t*)t.alloc((rcap + 1) * sizeof(uint64_t));
        t.rg_F = (uint32_t*)t.alloc(rcap * (mm - 1) * sizeof(uint32_t));
        t.rg_rid = (uint32_t*)t.alloc(rcap * sizeof(uint32_t));
        t.rg_w = (int8_t*)t.alloc(rcap);
      }
    }
    // touch every buffer once now (a fill at copy speed, outside the
    // capture), so that the first use of freshly mapped device memory is
    // paid at the build, not in a replay
    for (size_t i = 0; i < t.allocs.size(); ++i)
      GJ_HIP(hipMemsetAsync(t.allocs[i], 0, t.alloc_bytes[i], c->stream));
    t.h_stage_bytes = sizeof(BHead) + sizeof(BReq) * mr + sizeof(uint64_t) * (mr + 1) +
                      sizeof(unsigned long long) * t.stat_words() + sizeof(RunDesc) * t.rdt_entries();
    GJ_HIP(hipHostMalloc(&t.h_stage, t.h_stage_bytes, hipHostMallocDefault));
    // capture the level pipeline once; it reads every size from device memory
    GJ_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    enqueue(c, t, grid);
    hipError_t ce = hipStreamEndCapture(c->stream, &t.graph);
    GJ_CHECK(ce == hipSuccess, GJ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    GJ_HIP(hipGraphInstantiate(&t.exec, t.graph, nullptr, nullptr, 0));
  }
  Impl& t = *p;
  char* hs = (char*)t.h_stage;
  BHead* hh = (BHead*)hs;
  BReq* hr = (BReq*)(hs + sizeof(BHead));
  uint64_t* ho = (uint64_t*)(hr + t.max_req);
  memset(hh, 0, sizeof(BHead));
  uint64_t tot = 0;
  for (uint32_t i = 0; i < nreq; ++i) {
    const ReqSpec& r = specs[i];
    BReq& b = hr[i];
    memset(&b, 0, sizeof(b));
    b.m = (uint32_t)r.P.m;
    b.seed_lo = r.lo;
    b.seed_row = r.row;
    b.seed_col = r.col;
    b.seed_w = r.w;
    b.filt = seed_filter(r.P, r.V);
    for (int j = 2; j < r.P.m; ++j) b.st[j] = stage_desc(r.P, r.V, j);
    ho[i] = tot;
    tot += r.len;
  }
  ho[nreq] = tot;
  unsigned long long* res = (unsigned long long*)(ho + t.max_req + 1);
  if (t.runs) {
    // the split of each request's last stage where the run kernels can take
    // it (static counts only; signed delta seeds keep the per-candidate kernel)
    RunDesc* hd = (RunDesc*)(res + t.stat_words());
    memset(hd, 0, sizeof(RunDesc) * (uint64_t)nreq * kStat);
    for (uint32_t i = 0; i < nreq; ++i) {
      const ReqSpec& r = specs[i];
      const int j = r.P.m - 1;
      RunDesc& rd = hd[(uint64_t)i * kStat + j];
      if (j < 2 || r.w || !c->run_stage || c->strategy == 1 || !run_desc(hr[i].st[j], rd)) continue;
      rd.ok = 1;
      rd.ratio = c->run_ratio;
      rd.min_work = c->run_min_work;
      rd.task_work = c->run_task_work;
      rd.reuse = c->run_reuse;
      rd.big = c->run_big ? 1u : 0u;
      hh->runon[j] = 1;
    }
    GJ_HIP(hipMemcpyAsync(t.d_rdt, hd, sizeof(RunDesc) * (uint64_t)nreq * kStat, hipMemcpyHostToDevice,
                          c->stream));
  }
  hh->nreq = nreq;
  hh->lin = c->batch_lin;
  hh->claim_words = c->batch_claim_words;
  hh->seeds = tot;
  GJ_HIP(hipMemcpyAsync(t.d_req, hr, sizeof(BReq) * nreq, hipMemcpyHostToDevice, c->stream));
  GJ_HIP(hipMemcpyAsync(t.d_roff, ho, sizeof(uint64_t) * (nreq + 1), hipMemcpyHostToDevice, c->stream));
  GJ_HIP(hipMemcpyAsync(t.d_head, hh, sizeof(BHead), hipMemcpyHostToDevice, c->stream));
  KernelTimer timer(c);
  timer.start();
  GJ_HIP(hipGraphLaunch(t.exec, c->stream));
  timer.stop();
  GJ_HIP(hipMemcpyAsync(res, t.d_stat, t.stat_words() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                        c->stream));
  GJ_HIP(hipMemcpyAsync(hh, t.d_head, sizeof(BHead), hipMemcpyDeviceToHost, c->stream));
  double kms = timer.total_ms();  // synchronises
  overflow = hh->overflow != 0;
  if (overflow) return;
  const uint64_t mr = t.max_req;
  for (uint32_t i = 0; i < nreq; ++i) {
    if (counts) counts[i] = res[i];
    if (wsums) wsums[i] = (int64_t)res[mr + i];
    if (stats) {
      gj_stats st{};
      st.matches = res[i];
      for (int j = 0; j < kStat; ++j) {
        st.prefixes[j] = res[2 * mr + (uint64_t)i * kStat + j];
        st.extensions[j] = res[2 * mr + mr * kStat + (uint64_t)i * kStat + j];
      }
      st.kernel_ms = kms;
      st.kernel_launches = 1;
      stats[i] = st;
    }
  }
}

void BatchExec::run(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* lo,
                    const uint64_t* hi, uint64_t* counts, gj_stats* stats, bool& overflow, const Version* ver) {
  const Version& v = ver ? *ver : g->ver[g->cur];
  Views V{&v, &v, -1};
  std::vector<ReqSpec> specs;
  specs.reserve(nreq);
  for (uint32_t i = 0; i < nreq; ++i) {
    ReqSpec r{make_plan(qs[i], qs[i]->order, -1), V};
    int dir = r.P.seed_fwd ? 0 : 1;
    uint64_t h = std::min<uint64_t>(hi[i], v.m), l = std::min<uint64_t>(lo[i], h);
    r.row = v.d[dir].row;
    r.col = v.d[dir].col;
    r.w = nullptr;
    r.lo = l;
    r.len = h - l;
    specs.push_back(std::move(r));
  }
  run_specs(c, specs, counts, nullptr, stats, overflow);
}

void batch_destroy(gj_ctx* c) {
  delete c->batch;
  c->batch = nullptr;
}

}  // namespace gj
