// Whole counts of two four-attribute queries grouped by seed edge (a0, a1):
// the transitive 4-clique (every atom from an earlier attribute of the order
// to a later one), where Generic Join binds a2 from L = out(a0) & out(a1)
// and a3 from L & out(a2) (Sec. 2.2); and the diamond edge(a0,a1),
// edge(a0,a2), edge(a1,a3), edge(a2,a3), where a2 ranges over out(a0) and
// a3 over out(a1) & out(a2).  In both, a3 ranges over S & out(a2) with S
// (L, or out(a1)) fixed by the edge, so one wave per seed edge puts S in its
// LDS share once and counts |S & out(a2)| for every a2, probing whichever
// side is smaller: out(a2)'s values against S in LDS, or S's values against
// out(a2) in memory.  The probes of all a2 of an edge (in chunks of the
// offsets' LDS share) form one flattened index space over the wave.
//
// The counters are those of the depth-first evaluation: extensions[2] sums
// the stage-2 count-minimisation (min(d0, d1), or d0) over the edges,
// prefixes[3] the a2 per edge, extensions[3] the stage-3 minimum (min(d0, d1,
// d2), or min(d1, d2)) over the prefixes.  An edge whose S does not fit the
// wave's LDS share is left to the depth-first path (its id appended to a
// list) and contributes nothing here.
#include <algorithm>

#include "gj_internal.h"
#include "prim.h"

namespace gj {

constexpr int kCqWaves = 4;          // waves per workgroup
constexpr uint32_t kCqCap = 1024;    // entries of L per wave
constexpr uint32_t kCqChunk = 16;    // edges claimed at a time

// LDS written by some lanes of a wave and read by others
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool lds_contains(const uint32_t* a, uint32_t n0, uint32_t x) {
  uint32_t lo = 0, n = n0;
  while (n > 0) {
    uint32_t half = n >> 1;
    if (a[lo + half] < x) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo < n0 && a[lo] == x;
}

// last i in [0, n] with w[i] <= q (w ascending, w[0] = 0 <= q)
__device__ __forceinline__ uint32_t lds_owner(const uint32_t* w, uint32_t n, uint32_t q) {
  uint32_t lo = 0, hi = n + 1;  // w[lo] <= q < w[hi] (w[n + 1] taken as infinite)
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (w[mid] <= q)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Inequalities of the query (symmetry breaking, Sec. 5.4): the value bound at
// position j must exceed (above[j]) or stay below (below[j]) the values of
// the prefix columns whose bits are set.
struct EdgeIneq {
  uint32_t above[4], below[4];
};

__device__ __forceinline__ bool ineq3(const EdgeIneq& q, int j, uint32_t v, uint32_t c0, uint32_t c1, uint32_t c2) {
  const uint32_t a = q.above[j], b = q.below[j];
  if (!(a | b)) return true;
  bool ok = true;
  if (a & 1) ok = ok && v > c0;
  if (a & 2) ok = ok && v > c1;
  if (a & 4) ok = ok && v > c2;
  if (b & 1) ok = ok && v < c0;
  if (b & 2) ok = ok && v < c1;
  if (b & 4) ok = ok && v < c2;
  return ok;
}

// The values [lb, ub) the inequalities allow at position j given prefix
// columns c0, c1, c2 (ids are below 2^32 - 1, so ub = 2^32 - 1 bounds
// nothing and c + 1 does not wrap).
__device__ __forceinline__ void ineq_range3(const EdgeIneq& q, int j, uint32_t c0, uint32_t c1, uint32_t c2,
                                            uint32_t& lb, uint32_t& ub) {
  const uint32_t a = q.above[j], b = q.below[j];
  lb = 0;
  ub = 0xFFFFFFFFu;
  if (a & 1) lb = max(lb, c0 + 1);
  if (a & 2) lb = max(lb, c1 + 1);
  if (a & 4) lb = max(lb, c2 + 1);
  if (b & 1) ub = min(ub, c0);
  if (b & 2) ub = min(ub, c1);
  if (b & 4) ub = min(ub, c2);
}

// first i in [0, n) with a[i] >= x (a sorted, in LDS), else n
__device__ __forceinline__ uint32_t lds_first_ge(const uint32_t* a, uint32_t n, uint32_t x) {
  uint32_t lo = 0;
  while (n > 0) {
    const uint32_t half = n >> 1;
    if (a[lo + half] < x) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

// With inequalities on a3 (INEQ): S and out(a2) are both sorted, so the
// values a3 may take form one range of each, found by binary search per a2;
// a2's work is the smaller range, and rel records which side it walks and
// where that range starts (bit 31 set: out(a2) from its row start + the low
// bits, probing S; clear: S from that index, probing out(a2)).  Counters
// stay those of the whole sets (the depth-first evaluation's).
__device__ __forceinline__ uint32_t a3_range(const uint32_t* __restrict__ col, uint32_t b2, uint32_t d2,
                                             const uint32_t* S, uint32_t nS, uint32_t lb, uint32_t ub,
                                             uint32_t& rel) {
  if (lb >= ub) {
    rel = 0;
    return 0;
  }
  const uint32_t rl = lower_bound_u32(col, b2, b2 + d2, lb);
  const uint32_t rh = ub == 0xFFFFFFFFu ? b2 + d2 : lower_bound_u32(col, rl, b2 + d2, ub);
  const uint32_t sl = lds_first_ge(S, nS, lb);
  const uint32_t sh = ub == 0xFFFFFFFFu ? nS : sl + lds_first_ge(S + sl, nS - sl, ub);
  if (rh - rl < sh - sl) {
    rel = 0x80000000u | (rl - b2);
    return rh - rl;
  }
  rel = sl;
  return sh - sl;
}

// x in out(v) = col[b, b + d): v's table in the membership index (hd/hs, the
// version's forward direction; null when there is none) where the row has
// one, else a binary search of the row.
__device__ __forceinline__ bool row_member(const uint32_t* __restrict__ col, const uint64_t* __restrict__ hd,
                                           const uint32_t* __restrict__ hs, uint32_t v, uint32_t b, uint32_t d,
                                           uint32_t x) {
  const uint64_t desc = hd ? hd[v] : 0ull;
  return desc ? hash_member(hs, desc, x) : contains_u32(col, b, b + d, x);
}

// SHAPE 0, the transitive 4-clique: S = L = out(a0) & out(a1) and a2 ranges
// over L.  SHAPE 1, the diamond edge(a0,a1), edge(a0,a2), edge(a1,a3),
// edge(a2,a3): S = out(a1) and a2 ranges over out(a0).  Either way a3 ranges
// over S & out(a2), and S sits in the wave's LDS share.
template <int SHAPE, bool INEQ>
__global__ void __launch_bounds__(kCqWaves * 64) k_edge4(const uint32_t* __restrict__ rp,
                                                         const uint32_t* __restrict__ col,
                                                         const uint32_t* __restrict__ row, uint64_t m,
                                                         unsigned long long* __restrict__ claim,
                                                         uint32_t* __restrict__ ovf,
                                                         unsigned long long* __restrict__ acc, EdgeIneq iq,
                                                         const uint64_t* __restrict__ hd,
                                                         const uint32_t* __restrict__ hs) {
  __shared__ uint32_t Ls[kCqWaves][kCqCap];
  __shared__ uint32_t Ws[kCqWaves][kCqCap + 1];
  __shared__ uint32_t Rs[kCqWaves][INEQ ? kCqCap : 1];  // per a2: the side and start of its a3 range
  const int lane = lane_id();
  uint32_t* S = Ls[wave_id()];
  uint32_t* Wp = Ws[wave_id()];
  uint32_t* Rel = Rs[wave_id()];
  uint64_t matches = 0, pre2 = 0, pre3 = 0, ext2 = 0, ext3 = 0;
  for (;;) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(claim, (unsigned long long)kCqChunk);
    base = shfl_u64(base, 0);
    if (base >= m) break;
    uint64_t end = base + kCqChunk < m ? base + kCqChunk : m;
    for (uint64_t e = base; e < end; ++e) {
      const uint32_t x0 = row[e], x1 = col[e];
      if (!ineq3(iq, 1, x1, x0, 0, 0)) continue;  // the seed is not in P_2
      const uint32_t b0 = rp[x0], d0 = rp[x0 + 1] - b0, b1 = rp[x1], d1 = rp[x1 + 1] - b1;
      const uint32_t d01 = d0 < d1 ? d0 : d1;
      wave_lds_sync();  // the previous edge's reads of S are done
      uint32_t nS = 0;
      if (SHAPE == 0) {
        // L = out(x0) & out(x1): the shorter list proposes, in order
        const uint32_t sb = d0 <= d1 ? b0 : b1, gb = d0 <= d1 ? b1 : b0, gd = d0 <= d1 ? d1 : d0;
        const uint32_t gv = d0 <= d1 ? x1 : x0;  // the longer row's vertex
        for (uint32_t t = 0; t < d01; t += 64) {
          uint32_t i = t + lane;
          uint32_t x = 0;
          bool hit = false;
          if (i < d01) {
            x = col[sb + i];
            hit = row_member(col, hd, hs, gv, gb, gd, x);
          }
          uint64_t bal = __ballot(hit);
          uint32_t pos = nS + (uint32_t)__popcll(bal & lanemask_lt());
          if (hit && pos < kCqCap) S[pos] = x;
          nS += (uint32_t)__popcll(bal);
        }
      } else {
        nS = d1;  // S = out(x1)
        if (nS <= kCqCap)
          for (uint32_t i = lane; i < d1; i += 64) S[i] = col[b1 + i];
      }
      if (nS > kCqCap) {  // does not fit: the depth-first path takes this seed
        if (lane == 0) ovf[atomicAdd(claim + 1, 1ull)] = (uint32_t)e;
        continue;
      }
      // the a2 list: L in LDS, or out(x0) in memory; a2 failing an
      // inequality gets no work (S stays whole: a3 may take such values)
      const uint32_t na2 = SHAPE == 0 ? nS : d0;
      if (lane == 0) {
        ext2 += SHAPE == 0 ? d01 : d0;
        pre2 += 1;
      }
      if (na2 == 0) continue;
      wave_lds_sync();
      for (uint32_t c0 = 0; c0 < na2; c0 += kCqCap) {  // a2 in chunks of the offsets' LDS share
        const uint32_t cn = na2 - c0 < kCqCap ? na2 - c0 : kCqCap;
        // work of each a2: min(d2, |S|) probes; exclusive offsets in Wp
        uint32_t run = 0;
        for (uint32_t t = 0; t < cn; t += 64) {
          uint32_t i = t + lane;
          uint32_t w = 0;
          if (i < cn) {
            uint32_t a2 = SHAPE == 0 ? S[c0 + i] : col[b0 + c0 + i];
            if (ineq3(iq, 2, a2, x0, x1, 0)) {
              uint32_t b2 = rp[a2], d2 = rp[a2 + 1] - b2;
              if (INEQ) {
                uint32_t lb, ub, rel;
                ineq_range3(iq, 3, x0, x1, a2, lb, ub);
                w = a3_range(col, b2, d2, S, nS, lb, ub, rel);
                Rel[i] = rel;
              } else {
                w = d2 < nS ? d2 : nS;
              }
              uint32_t lim = SHAPE == 0 ? d01 : d1;  // count-minimisation of the last stage
              ext3 += d2 < lim ? d2 : lim;
              pre3 += 1;
            }
          }
          uint32_t incl = wave_incl_scan(w);
          if (i < cn) Wp[i] = run + incl - w;
          run += __shfl(incl, 63, 64);
        }
        wave_lds_sync();  // Wp's readers below may run ahead of this chunk's writers
        if (lane == 0) Wp[cn] = run;
        wave_lds_sync();
        for (uint32_t q0 = 0; q0 < run; q0 += 64) {
          uint32_t q = q0 + lane;
          bool found = false;
          if (q < run) {
            uint32_t i = lds_owner(Wp, cn, q);  // i < cn: Wp[cn] = run > q
            uint32_t t = q - Wp[i];
            uint32_t a2 = SHAPE == 0 ? S[c0 + i] : col[b0 + c0 + i];
            uint32_t b2 = rp[a2], d2 = rp[a2 + 1] - b2;
            if (INEQ) {
              const uint32_t rel = Rel[i];
              const bool row_side = (rel >> 31) != 0;
              uint32_t a3 = row_side ? col[b2 + (rel & 0x7FFFFFFFu) + t] : S[rel + t];
              found = row_side ? lds_contains(S, nS, a3) : row_member(col, hd, hs, a2, b2, d2, a3);
              found = found && ineq3(iq, 3, a3, x0, x1, a2);
            } else {
              uint32_t a3 = d2 < nS ? col[b2 + t] : S[t];  // t < d2, or t < nS
              found = d2 < nS ? lds_contains(S, nS, a3) : row_member(col, hd, hs, a2, b2, d2, a3);
              found = found && ineq3(iq, 3, a3, x0, x1, a2);
            }
          }
          matches += found ? 1 : 0;
        }
        wave_lds_sync();  // this chunk's reads of Wp are done
      }
    }
  }
  matches = wave_sum(matches);
  ext3 = wave_sum(ext3);
  ext2 = wave_sum(ext2);
  pre3 = wave_sum(pre3);
  pre2 = wave_sum(pre2);
  if (lane == 0) {
    if (matches) atomicAdd(acc + 0, (unsigned long long)matches);
    if (pre3) atomicAdd(acc + 1, (unsigned long long)pre3);
    if (ext2) atomicAdd(acc + 2, (unsigned long long)ext2);
    if (ext3) atomicAdd(acc + 3, (unsigned long long)ext3);
    if (pre2) atomicAdd(acc + 4, (unsigned long long)pre2);
  }
}

// The seeds whose fixed set outgrew a wave's share, again with a whole
// workgroup per seed: 16,384 entries of S (64 KiB of LDS), compaction and
// offsets by workgroup scans, the probes spread over 256 lanes.  Seeds
// beyond that are appended to ovf for the depth-first path.
constexpr uint32_t kCqCapWg = 16384;
constexpr uint32_t kCqOffWg = 1024;

template <int SHAPE, bool INEQ>
__global__ void __launch_bounds__(kBlock) k_edge4_wg(const uint32_t* __restrict__ rp,
                                                     const uint32_t* __restrict__ col,
                                                     const uint32_t* __restrict__ row, const uint32_t* __restrict__ ids,
                                                     uint64_t m, unsigned long long* __restrict__ claim,
                                                     uint32_t* __restrict__ ovf, unsigned long long* __restrict__ acc,
                                                     EdgeIneq iq, const uint64_t* __restrict__ hd,
                                                     const uint32_t* __restrict__ hs) {
  __shared__ uint32_t S[kCqCapWg];
  __shared__ uint32_t Wp[kCqOffWg + 1];
  __shared__ uint32_t Rel[INEQ ? kCqOffWg : 1];  // per a2: the side and start of its a3 range
  __shared__ unsigned long long next;
  const uint32_t tid = threadIdx.x;
  uint64_t matches = 0, pre2 = 0, pre3 = 0, ext2 = 0, ext3 = 0;
  for (;;) {
    __syncthreads();  // the previous seed's reads of S and Wp are done
    if (tid == 0) next = atomicAdd(claim, 1ull);
    __syncthreads();
    const unsigned long long k = next;
    if (k >= m) break;
    const uint64_t e = ids[k];
    const uint32_t x0 = row[e], x1 = col[e];
    if (!ineq3(iq, 1, x1, x0, 0, 0)) continue;
    const uint32_t b0 = rp[x0], d0 = rp[x0 + 1] - b0, b1 = rp[x1], d1 = rp[x1 + 1] - b1;
    const uint32_t d01 = d0 < d1 ? d0 : d1;
    uint32_t nS = 0;
    if (SHAPE == 0) {
      const uint32_t sb = d0 <= d1 ? b0 : b1, gb = d0 <= d1 ? b1 : b0, gd = d0 <= d1 ? d1 : d0;
      const uint32_t gv = d0 <= d1 ? x1 : x0;  // the longer row's vertex
      for (uint32_t t = 0; t < d01; t += kBlock) {
        uint32_t i = t + tid;
        uint32_t x = 0, hit = 0;
        if (i < d01) {
          x = col[sb + i];
          hit = row_member(col, hd, hs, gv, gb, gd, x) ? 1u : 0u;
        }
        uint32_t tot = 0;
        uint32_t pos = nS + block_excl_scan<kBlock>(hit, tot);
        if (hit && pos < kCqCapWg) S[pos] = x;
        nS += tot;
      }
    } else {
      nS = d1;
      if (nS <= kCqCapWg)
        for (uint32_t i = tid; i < d1; i += kBlock) S[i] = col[b1 + i];
    }
    if (nS > kCqCapWg) {
      if (tid == 0) ovf[atomicAdd(claim + 1, 1ull)] = (uint32_t)e;
      continue;
    }
    const uint32_t na2 = SHAPE == 0 ? nS : d0;
    if (tid == 0) {
      ext2 += SHAPE == 0 ? d01 : d0;
      pre2 += 1;
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < na2; c0 += kCqOffWg) {
      const uint32_t cn = na2 - c0 < kCqOffWg ? na2 - c0 : kCqOffWg;
      uint32_t run = 0;
      for (uint32_t t = 0; t < cn; t += kBlock) {
        uint32_t i = t + tid;
        uint32_t w = 0;
        if (i < cn) {
          uint32_t a2 = SHAPE == 0 ? S[c0 + i] : col[b0 + c0 + i];
          if (ineq3(iq, 2, a2, x0, x1, 0)) {
            uint32_t b2 = rp[a2], d2 = rp[a2 + 1] - b2;
            if (INEQ) {
              uint32_t lb, ub, rel;
              ineq_range3(iq, 3, x0, x1, a2, lb, ub);
              w = a3_range(col, b2, d2, S, nS, lb, ub, rel);
              Rel[i] = rel;
            } else {
              w = d2 < nS ? d2 : nS;
            }
            uint32_t lim = SHAPE == 0 ? d01 : d1;
            ext3 += d2 < lim ? d2 : lim;
            pre3 += 1;
          }
        }
        uint32_t tot = 0;
        uint32_t ex = block_excl_scan<kBlock>(w, tot);
        if (i < cn) Wp[i] = run + ex;
        run += tot;
      }
      if (tid == 0) Wp[cn] = run;
      __syncthreads();
      for (uint32_t q0 = 0; q0 < run; q0 += kBlock) {
        uint32_t q = q0 + tid;
        if (q < run) {
          uint32_t i = lds_owner(Wp, cn, q);  // i < cn: Wp[cn] = run > q
          uint32_t t = q - Wp[i];
          uint32_t a2 = SHAPE == 0 ? S[c0 + i] : col[b0 + c0 + i];
          uint32_t b2 = rp[a2], d2 = rp[a2 + 1] - b2;
          bool found;
          uint32_t a3;
          if (INEQ) {
            const uint32_t rel = Rel[i];
            const bool row_side = (rel >> 31) != 0;
            a3 = row_side ? col[b2 + (rel & 0x7FFFFFFFu) + t] : S[rel + t];
            found = row_side ? lds_contains(S, nS, a3) : row_member(col, hd, hs, a2, b2, d2, a3);
          } else {
            a3 = d2 < nS ? col[b2 + t] : S[t];
            found = d2 < nS ? lds_contains(S, nS, a3) : row_member(col, hd, hs, a2, b2, d2, a3);
          }
          matches += (found && ineq3(iq, 3, a3, x0, x1, a2)) ? 1 : 0;
        }
      }
      __syncthreads();  // this chunk's reads of Wp are done
    }
  }
  uint64_t v[5] = {matches, pre3, ext2, ext3, pre2};
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    uint64_t t = block_sum<kBlock>(v[i]);
    if (tid == 0 && t) atomicAdd(acc + i, (unsigned long long)t);
  }
}

__global__ void k_gather_seeds(const uint32_t* __restrict__ ids, uint64_t k, const uint32_t* __restrict__ row,
                               const uint32_t* __restrict__ col, uint32_t* __restrict__ x0, uint32_t* __restrict__ x1) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gs) {
    x0[i] = row[ids[i]];
    x1[i] = col[ids[i]];
  }
}

void edge4_count(gj_ctx* c, const Version& v, int shape, const uint32_t above[4], const uint32_t below[4],
                 const uint64_t* hd, const uint32_t* hs, KernelTimer& timer, uint64_t out[5], uint32_t*& x0,
                 uint32_t*& x1, uint64_t& n_left) {
  const CsrDir& d = v.d[0];
  // ctr: [0] seed claim, [1] overflow count, [2, 7) counters, [7] second-pass
  // claim, [8] its overflow count
  unsigned long long* ctr = (unsigned long long*)ws_get(c, "cq_ctr", 9 * sizeof(unsigned long long));
  uint32_t* ovf = (uint32_t*)ws_get(c, "cq_ovf", (v.m + 1) * sizeof(uint32_t));
  GJ_HIP(hipMemsetAsync(ctr, 0, 9 * sizeof(unsigned long long), c->stream));
  EdgeIneq iq;
  for (int j = 0; j < 4; ++j) {
    iq.above[j] = above[j];
    iq.below[j] = below[j];
  }
  // inequalities on a3: its ranges in S and out(a2) narrowed per a2 (48 KiB
  // of LDS per workgroup, so 3 per CU)
  const bool ineq = (above[3] | below[3]) != 0;
  unsigned grid = (unsigned)c->num_cus * (ineq ? 3 : 4);  // workgroups of 4 waves, 32 KiB of LDS each without
  timer.start();
  if (v.m && shape == 0 && !ineq)
    k_edge4<0, false><<<grid, kCqWaves * 64, 0, c->stream>>>(d.rp, d.col, d.row, v.m, ctr, ovf, ctr + 2, iq, hd, hs);
  if (v.m && shape == 0 && ineq)
    k_edge4<0, true><<<grid, kCqWaves * 64, 0, c->stream>>>(d.rp, d.col, d.row, v.m, ctr, ovf, ctr + 2, iq, hd, hs);
  if (v.m && shape == 1 && !ineq)
    k_edge4<1, false><<<grid, kCqWaves * 64, 0, c->stream>>>(d.rp, d.col, d.row, v.m, ctr, ovf, ctr + 2, iq, hd, hs);
  if (v.m && shape == 1 && ineq)
    k_edge4<1, true><<<grid, kCqWaves * 64, 0, c->stream>>>(d.rp, d.col, d.row, v.m, ctr, ovf, ctr + 2, iq, hd, hs);
  timer.stop();
  GJ_HIP(hipGetLastError());
  unsigned long long n1 = 0;
  read_bytes(c, &n1, ctr + 1, sizeof(n1));
  const uint32_t* left = ovf;
  // the 4-clique's larger sets: a workgroup per seed (measured slower than
  // the depth-first path for the diamond, whose overflowing seeds go there)
  if (n1 && shape == 0) {
    uint32_t* ovf2 = (uint32_t*)ws_get(c, "cq_ovf2", (n1 + 1) * sizeof(uint32_t));
    unsigned grid2 = (unsigned)c->num_cus * 2;  // 2 workgroups per CU (68 KiB of LDS each, 72 KiB with INEQ)
    timer.start();
    if (ineq)
      k_edge4_wg<0, true><<<grid2, kBlock, 0, c->stream>>>(d.rp, d.col, d.row, ovf, n1, ctr + 7, ovf2, ctr + 2, iq, hd, hs);
    else
      k_edge4_wg<0, false><<<grid2, kBlock, 0, c->stream>>>(d.rp, d.col, d.row, ovf, n1, ctr + 7, ovf2, ctr + 2, iq, hd, hs);
    timer.stop();
    GJ_HIP(hipGetLastError());
    left = ovf2;
  }
  unsigned long long h[9];
  read_bytes(c, h, ctr, sizeof(h));
  n_left = n1 && shape == 0 ? h[8] : h[1];
  for (int i = 0; i < 5; ++i) out[i] = h[2 + i];
  x0 = x1 = nullptr;
  if (n_left) {
    x0 = (uint32_t*)ws_get(c, "cq_x0", n_left * sizeof(uint32_t));
    x1 = (uint32_t*)ws_get(c, "cq_x1", n_left * sizeof(uint32_t));
    k_gather_seeds<<<grid_for(n_left, kBlock, 1u << 14), kBlock, 0, c->stream>>>(left, n_left, d.row, d.col, x0, x1);
    GJ_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------- transitive 5-clique
// The transitive 5-clique binds a2 from L = out(a0) & out(a1), a3 from
// L & out(a2) and a4 from L & out(a2) & out(a3) (Sec. 2.2).  Per seed edge a
// wave keeps L (sorted) in LDS together with L's adjacency as bit masks over
// L's positions, row i holding L & out(L[i]), built with the 4-clique
// kernel's probes (whichever side is smaller).  The matches of the edge are
// then the sum over a2 = L[i] and a3 = L[j] in row i of |row i & row j|,
// popcounts of a few words.  Inequalities between vertex ids become ranges
// of positions in the sorted L.  Counters are the depth-first evaluation's,
// as for the 4-clique; edges with |L| > kC5Cap take a second pass with a
// workgroup per edge (k_clique5_wg), and beyond that the depth-first path.
constexpr int kC5Waves = 4;
constexpr uint32_t kC5Cap = 256;           // entries of L per wave
constexpr uint32_t kC5Words = kC5Cap / 64;  // mask words per row at most

struct EdgeIneq5 {
  uint32_t above[5], below[5];
};

// positions of L (sorted, distinct, n entries) that a value bound at
// position p may take: [lo, hi), from the inequalities against the seed
// values (lt / le: how many entries of L are below / at most x0 and x1) and
// against the values at positions 2 and 3 (L[i2], L[i3])
__device__ __forceinline__ void ineq_range(const EdgeIneq5& q, int p, const uint32_t (&lt)[2],
                                           const uint32_t (&le)[2], uint32_t i2, uint32_t i3, uint32_t n,
                                           uint32_t& lo, uint32_t& hi) {
  lo = 0;
  hi = n;
  const uint32_t a = q.above[p], b = q.below[p];
  if (!(a | b)) return;
  for (int c = 0; c < 2; ++c) {
    if ((a >> c) & 1) lo = le[c] > lo ? le[c] : lo;
    if ((b >> c) & 1) hi = lt[c] < hi ? lt[c] : hi;
  }
  if (a & 4) lo = i2 + 1 > lo ? i2 + 1 : lo;
  if (b & 4) hi = i2 < hi ? i2 : hi;
  if (a & 8) lo = i3 + 1 > lo ? i3 + 1 : lo;
  if (b & 8) hi = i3 < hi ? i3 : hi;
}

// the bits of mask word w (positions 64w .. 64w + 63) inside [lo, hi)
__device__ __forceinline__ uint64_t range_bits(uint32_t w, uint32_t lo, uint32_t hi) {
  const uint32_t base = w * 64;
  if (lo >= hi || hi <= base || lo >= base + 64) return 0;
  const uint32_t a = lo > base ? lo - base : 0, b = hi < base + 64 ? hi - base : 64;
  uint64_t m = b == 64 ? ~0ull : ((1ull << b) - 1);
  return m & ~((1ull << a) - 1);
}

__device__ __forceinline__ uint32_t lds_lower(const uint32_t* a, uint32_t n, uint32_t x) {
  uint32_t lo = 0;
  while (n > 0) {
    uint32_t half = n >> 1;
    if (a[lo + half] < x) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

__global__ void __launch_bounds__(kC5Waves * 64) k_clique5(const uint32_t* __restrict__ rp,
                                                           const uint32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ row, uint64_t m,
                                                           unsigned long long* __restrict__ claim,
                                                           uint32_t* __restrict__ ovf,
                                                           unsigned long long* __restrict__ acc, EdgeIneq5 iq, const uint64_t* __restrict__ hd,
                                                       const uint32_t* __restrict__ hs) {
  __shared__ uint32_t Ls[kC5Waves][kC5Cap];
  __shared__ uint32_t Ds[kC5Waves][kC5Cap];
  __shared__ uint32_t Ws[kC5Waves][kC5Cap + 1];
  __shared__ unsigned long long Ms[kC5Waves][kC5Cap * kC5Words];
  const int lane = lane_id();
  uint32_t* S = Ls[wave_id()];
  uint32_t* D = Ds[wave_id()];
  uint32_t* Wp = Ws[wave_id()];
  unsigned long long* M = Ms[wave_id()];
  uint64_t matches = 0, pre2 = 0, ext2 = 0, pre3 = 0, ext3 = 0, pre4 = 0, ext4 = 0;
  for (;;) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(claim, (unsigned long long)kCqChunk);
    base = shfl_u64(base, 0);
    if (base >= m) break;
    uint64_t end = base + kCqChunk < m ? base + kCqChunk : m;
    for (uint64_t e = base; e < end; ++e) {
      const uint32_t x0 = row[e], x1 = col[e];
      if (((iq.above[1] & 1) && !(x1 > x0)) || ((iq.below[1] & 1) && !(x1 < x0))) continue;
      const uint32_t b0 = rp[x0], d0 = rp[x0 + 1] - b0, b1 = rp[x1], d1 = rp[x1 + 1] - b1;
      const uint32_t d01 = d0 < d1 ? d0 : d1;
      wave_lds_sync();  // the previous edge's reads are done
      // L = out(x0) & out(x1), in order, from the shorter list
      uint32_t nS = 0;
      {
        const uint32_t sb = d0 <= d1 ? b0 : b1, gb = d0 <= d1 ? b1 : b0, gd = d0 <= d1 ? d1 : d0;
        const uint32_t gv = d0 <= d1 ? x1 : x0;  // the longer row's vertex
        for (uint32_t t = 0; t < d01; t += 64) {
          uint32_t i = t + lane;
          uint32_t x = 0;
          bool hit = false;
          if (i < d01) {
            x = col[sb + i];
            hit = row_member(col, hd, hs, gv, gb, gd, x);
          }
          uint64_t bal = __ballot(hit);
          uint32_t pos = nS + (uint32_t)__popcll(bal & lanemask_lt());
          if (hit && pos < kC5Cap) S[pos] = x;
          nS += (uint32_t)__popcll(bal);
        }
      }
      if (nS > kC5Cap) {  // does not fit: the depth-first path takes this seed
        if (lane == 0) ovf[atomicAdd(claim + 1, 1ull)] = (uint32_t)e;
        continue;
      }
      if (lane == 0) {
        ext2 += d01;
        pre2 += 1;
      }
      if (nS == 0) continue;
      wave_lds_sync();
      const uint32_t W = (nS + 63) >> 6;
      uint32_t lt[2], le[2];
      lt[0] = lds_lower(S, nS, x0);
      le[0] = lds_lower(S, nS, x0 + 1);  // ids are below 2^32 - 1
      lt[1] = lds_lower(S, nS, x1);
      le[1] = lds_lower(S, nS, x1 + 1);
      uint32_t lo2, hi2;
      ineq_range(iq, 2, lt, le, 0, 0, nS, lo2, hi2);
      for (uint32_t i = lane; i < nS * W; i += 64) M[i] = 0;
      // degrees of L, and the probes of row i: min(d(L[i]), |L|).  Every row
      // is built: L[i] may serve as a3 even where it fails a2's inequalities
      uint32_t run = 0;
      for (uint32_t t = 0; t < nS; t += 64) {
        uint32_t i = t + lane;
        uint32_t w = 0;
        if (i < nS) {
          uint32_t a2 = S[i];
          uint32_t d2 = rp[a2 + 1] - rp[a2];
          D[i] = d2;
          w = d2 < nS ? d2 : nS;
          if (i >= lo2 && i < hi2) {
            ext3 += d2 < d01 ? d2 : d01;
            pre3 += 1;
          }
        }
        uint32_t incl = wave_incl_scan(w);
        if (i < nS) Wp[i] = run + incl - w;
        run += __shfl(incl, 63, 64);
      }
      wave_lds_sync();
      if (lane == 0) Wp[nS] = run;
      wave_lds_sync();
      // row i of the masks: bit j set when L[j] is in out(L[i])
      for (uint32_t q0 = 0; q0 < run; q0 += 64) {
        uint32_t q = q0 + lane;
        if (q < run) {
          uint32_t i = lds_owner(Wp, nS, q);  // i < nS: Wp[nS] = run > q
          uint32_t t = q - Wp[i];
          uint32_t a2 = S[i], d2 = D[i], b2 = rp[a2];
          uint32_t j;
          bool found;
          if (d2 < nS) {  // t < d2: out(a2)'s values against L
            uint32_t a3 = col[b2 + t];
            j = lds_lower(S, nS, a3);
            found = j < nS && S[j] == a3;
          } else {  // t < nS: L's values against out(a2)
            j = t;
            found = row_member(col, hd, hs, a2, b2, d2, S[t]);
          }
          if (found) atomicOr(&M[i * W + (j >> 6)], 1ull << (j & 63));
        }
      }
      wave_lds_sync();
      // a lane per a2: its a3 in row i, then the a4 of both rows
      for (uint32_t t = 0; t < nS; t += 64) {
        uint32_t i = t + lane;
        if (i >= nS || i < lo2 || i >= hi2) continue;
        const uint32_t d2 = D[i];
        const uint32_t m012 = d2 < d01 ? d2 : d01;
        uint32_t lo3, hi3;
        ineq_range(iq, 3, lt, le, i, 0, nS, lo3, hi3);
        for (uint32_t w = 0; w < W; ++w) {
          uint64_t bits = M[i * W + w] & range_bits(w, lo3, hi3);
          while (bits) {
            const uint32_t j = w * 64 + (uint32_t)__builtin_ctzll(bits);
            bits &= bits - 1;
            pre4 += 1;
            ext4 += D[j] < m012 ? D[j] : m012;
            uint32_t lo4, hi4;
            ineq_range(iq, 4, lt, le, i, j, nS, lo4, hi4);
            for (uint32_t w2 = 0; w2 < W; ++w2)
              matches += (uint64_t)__popcll(M[i * W + w2] & M[j * W + w2] & range_bits(w2, lo4, hi4));
          }
        }
      }
    }
  }
  uint64_t v[7] = {matches, pre2, ext2, pre3, ext3, pre4, ext4};
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    uint64_t t = wave_sum(v[i]);
    if (lane == 0 && t) atomicAdd(acc + i, (unsigned long long)t);
  }
}

// The seeds whose L outgrew a wave's share, again with a whole workgroup per
// seed: up to 704 entries of L (11 mask words per row, 70 KiB of LDS),
// compaction and offsets by workgroup scans, the probes over 256 lanes.
// Seeds beyond that are appended to ovf for the depth-first path.
constexpr uint32_t kC5CapWg = 704;
constexpr uint32_t kC5WordsWg = (kC5CapWg + 63) / 64;

__global__ void __launch_bounds__(kBlock) k_clique5_wg(const uint32_t* __restrict__ rp,
                                                       const uint32_t* __restrict__ col,
                                                       const uint32_t* __restrict__ row,
                                                       const uint32_t* __restrict__ ids, uint64_t m,
                                                       unsigned long long* __restrict__ claim,
                                                       uint32_t* __restrict__ ovf,
                                                       unsigned long long* __restrict__ acc, EdgeIneq5 iq, const uint64_t* __restrict__ hd,
                                                       const uint32_t* __restrict__ hs) {
  __shared__ uint32_t S[kC5CapWg];
  __shared__ uint32_t D[kC5CapWg];
  __shared__ uint32_t Wp[kC5CapWg + 1];
  __shared__ unsigned long long M[kC5CapWg * kC5WordsWg];
  __shared__ unsigned long long next;
  const uint32_t tid = threadIdx.x;
  uint64_t matches = 0, pre2 = 0, ext2 = 0, pre3 = 0, ext3 = 0, pre4 = 0, ext4 = 0;
  for (;;) {
    __syncthreads();  // the previous seed's reads are done
    if (tid == 0) next = atomicAdd(claim, 1ull);
    __syncthreads();
    const unsigned long long k = next;
    if (k >= m) break;
    const uint64_t e = ids[k];
    const uint32_t x0 = row[e], x1 = col[e];
    if (((iq.above[1] & 1) && !(x1 > x0)) || ((iq.below[1] & 1) && !(x1 < x0))) continue;
    const uint32_t b0 = rp[x0], d0 = rp[x0 + 1] - b0, b1 = rp[x1], d1 = rp[x1 + 1] - b1;
    const uint32_t d01 = d0 < d1 ? d0 : d1;
    uint32_t nS = 0;
    {
      const uint32_t sb = d0 <= d1 ? b0 : b1, gb = d0 <= d1 ? b1 : b0, gd = d0 <= d1 ? d1 : d0;
      const uint32_t gv = d0 <= d1 ? x1 : x0;  // the longer row's vertex
      for (uint32_t t = 0; t < d01; t += kBlock) {
        uint32_t i = t + tid;
        uint32_t x = 0, hit = 0;
        if (i < d01) {
          x = col[sb + i];
          hit = row_member(col, hd, hs, gv, gb, gd, x) ? 1u : 0u;
        }
        uint32_t tot = 0;
        uint32_t pos = nS + block_excl_scan<kBlock>(hit, tot);
        if (hit && pos < kC5CapWg) S[pos] = x;
        nS += tot;
      }
    }
    if (nS > kC5CapWg) {
      if (tid == 0) ovf[atomicAdd(claim + 1, 1ull)] = (uint32_t)e;
      continue;
    }
    if (tid == 0) {
      ext2 += d01;
      pre2 += 1;
    }
    if (nS == 0) continue;
    __syncthreads();  // L is complete
    const uint32_t W = (nS + 63) >> 6;
    uint32_t lt[2], le[2];
    lt[0] = lds_lower(S, nS, x0);
    le[0] = lds_lower(S, nS, x0 + 1);
    lt[1] = lds_lower(S, nS, x1);
    le[1] = lds_lower(S, nS, x1 + 1);
    uint32_t lo2, hi2;
    ineq_range(iq, 2, lt, le, 0, 0, nS, lo2, hi2);
    for (uint32_t i = tid; i < nS * W; i += kBlock) M[i] = 0;
    uint32_t run = 0;
    for (uint32_t t = 0; t < nS; t += kBlock) {
      uint32_t i = t + tid;
      uint32_t w = 0;
      if (i < nS) {
        uint32_t a2 = S[i];
        uint32_t d2 = rp[a2 + 1] - rp[a2];
        D[i] = d2;
        w = d2 < nS ? d2 : nS;
        if (i >= lo2 && i < hi2) {
          ext3 += d2 < d01 ? d2 : d01;
          pre3 += 1;
        }
      }
      uint32_t tot = 0;
      uint32_t ex = block_excl_scan<kBlock>(w, tot);
      if (i < nS) Wp[i] = run + ex;
      run += tot;
    }
    if (tid == 0) Wp[nS] = run;
    __syncthreads();  // masks cleared, degrees and offsets written
    for (uint32_t q = tid; q < run; q += kBlock) {
      uint32_t i = lds_owner(Wp, nS, q);  // i < nS: Wp[nS] = run > q
      uint32_t t = q - Wp[i];
      uint32_t a2 = S[i], d2 = D[i], b2 = rp[a2];
      uint32_t j;
      bool found;
      if (d2 < nS) {
        uint32_t a3 = col[b2 + t];
        j = lds_lower(S, nS, a3);
        found = j < nS && S[j] == a3;
      } else {
        j = t;
        found = row_member(col, hd, hs, a2, b2, d2, S[t]);
      }
      if (found) atomicOr(&M[i * W + (j >> 6)], 1ull << (j & 63));
    }
    __syncthreads();  // masks complete
    for (uint32_t i = tid; i < nS; i += kBlock) {
      if (i < lo2 || i >= hi2) continue;
      const uint32_t d2 = D[i];
      const uint32_t m012 = d2 < d01 ? d2 : d01;
      uint32_t lo3, hi3;
      ineq_range(iq, 3, lt, le, i, 0, nS, lo3, hi3);
      for (uint32_t w = 0; w < W; ++w) {
        uint64_t bits = M[i * W + w] & range_bits(w, lo3, hi3);
        while (bits) {
          const uint32_t j = w * 64 + (uint32_t)__builtin_ctzll(bits);
          bits &= bits - 1;
          pre4 += 1;
          ext4 += D[j] < m012 ? D[j] : m012;
          uint32_t lo4, hi4;
          ineq_range(iq, 4, lt, le, i, j, nS, lo4, hi4);
          for (uint32_t w2 = 0; w2 < W; ++w2)
            matches += (uint64_t)__popcll(M[i * W + w2] & M[j * W + w2] & range_bits(w2, lo4, hi4));
        }
      }
    }
  }
  uint64_t v[7] = {matches, pre2, ext2, pre3, ext3, pre4, ext4};
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    uint64_t t = block_sum<kBlock>(v[i]);
    if (tid == 0 && t) atomicAdd(acc + i, (unsigned long long)t);
  }
}

void clique5_count(gj_ctx* c, const Version& v, const uint32_t above[5], const uint32_t below[5],
                   const uint64_t* hd, const uint32_t* hs, KernelTimer& timer, uint64_t out[7], uint32_t*& x0,
                   uint32_t*& x1, uint64_t& n_left) {
  const CsrDir& d = v.d[0];
  // ctr: [0] seed claim, [1] overflow count, [2, 9) counters, [9] second-pass
  // claim, [10] its overflow count
  unsigned long long* ctr = (unsigned long long*)ws_get(c, "c5_ctr", 11 * sizeof(unsigned long long));
  uint32_t* ovf = (uint32_t*)ws_get(c, "c5_ovf", (v.m + 1) * sizeof(uint32_t));
  GJ_HIP(hipMemsetAsync(ctr, 0, 11 * sizeof(unsigned long long), c->stream));
  EdgeIneq5 iq;
  for (int j = 0; j < 5; ++j) {
    iq.above[j] = above[j];
    iq.below[j] = below[j];
  }
  unsigned grid = (unsigned)c->num_cus * 3;  // 3 workgroups of 4 waves per CU (44 KiB of LDS each)
  timer.start();
  if (v.m) k_clique5<<<grid, kC5Waves * 64, 0, c->stream>>>(d.rp, d.col, d.row, v.m, ctr, ovf, ctr + 2, iq, hd, hs);
  timer.stop();
  GJ_HIP(hipGetLastError());
  unsigned long long n1 = 0;
  read_bytes(c, &n1, ctr + 1, sizeof(n1));
  const uint32_t* left = ovf;
  if (n1) {  // larger L: a workgroup per seed
    uint32_t* ovf2 = (uint32_t*)ws_get(c, "c5_ovf2", (n1 + 1) * sizeof(uint32_t));
    unsigned grid2 = (unsigned)c->num_cus * 2;  // 2 workgroups per CU (70 KiB of LDS each)
    timer.start();
    k_clique5_wg<<<grid2, kBlock, 0, c->stream>>>(d.rp, d.col, d.row, ovf, n1, ctr + 9, ovf2, ctr + 2, iq, hd,
                                                  hs);
    timer.stop();
    GJ_HIP(hipGetLastError());
    left = ovf2;
  }
  unsigned long long h[11];
  read_bytes(c, h, ctr, sizeof(h));
  n_left = n1 ? h[10] : h[1];
  for (int i = 0; i < 7; ++i) out[i] = h[2 + i];
  x0 = x1 = nullptr;
  if (n_left) {
    x0 = (uint32_t*)ws_get(c, "c5_x0", n_left * sizeof(uint32_t));
    x1 = (uint32_t*)ws_get(c, "c5_x1", n_left * sizeof(uint32_t));
    k_gather_seeds<<<grid_for(n_left, kBlock, 1u << 14), kBlock, 0, c->stream>>>(left, n_left, d.row, d.col, x0, x1);
    GJ_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------- diamond by 2-path counts
// The diamond's matches from a0 are the pairs (a1, a2) of out(a0) with a
// common out-neighbour a3, counted per a3: with k(a3) the number of 2-paths
// a0 -> a1 -> a3, a0 contributes the sum of k(a3)^2 (a1 = a2 included, as
// the join allows).  One workgroup per a0 counts its 2-path endpoints with
// atomics in a private dense array of n counters, noting each endpoint at its
// first visit in a private list, then takes each listed endpoint's count
// with an exchange to zero, which leaves the array clear (one atomic per
// distinct endpoint instead of a second walk of every 2-path).  The
// counters are the depth-first evaluation's: extensions[2] = prefixes[3] =
// sum of d0^2 (a2 is proposed from out(a0) alone), extensions[3] = the sum
// over (a1, a2) in out(a0)^2 of min(d(a1), d(a2)), from tiles of the
// neighbours' degrees in LDS.
constexpr uint32_t kDgTile = 4096;  // degrees per LDS tile
constexpr uint32_t kDgOff = 1024;   // a1 per offsets chunk

__global__ void __launch_bounds__(kBlock) k_diamond2p(const uint32_t* __restrict__ rp,
                                                      const uint32_t* __restrict__ col, uint32_t n,
                                                      unsigned int* __restrict__ cnt_all, uint32_t* __restrict__ list_all,
                                                      uint64_t cnt_stride, unsigned long long* __restrict__ claim,
                                                      unsigned long long* __restrict__ acc) {
  __shared__ uint32_t DA[kDgTile], DB[kDgTile];
  __shared__ uint32_t Wp[kDgOff + 1];
  __shared__ unsigned long long next;
  __shared__ uint32_t s_nl;  // endpoints listed for this a0
  unsigned int* cnt = cnt_all + (uint64_t)blockIdx.x * cnt_stride;
  uint32_t* list = list_all + (uint64_t)blockIdx.x * cnt_stride;
  const uint32_t tid = threadIdx.x;
  const int lane = lane_id();
  uint64_t matches = 0, sq = 0, ext3 = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      next = atomicAdd(claim, 1ull);
      s_nl = 0;
    }
    __syncthreads();
    const unsigned long long a0 = next;
    if (a0 >= n) break;
    const uint32_t b0 = rp[a0], d0 = rp[a0 + 1] - b0;
    if (d0 == 0) continue;
    if (tid == 0) sq += (uint64_t)d0 * d0;
    // extensions[3]: sum over ordered pairs of min(degree), in tiles
    for (uint32_t ta = 0; ta < d0; ta += kDgTile) {
      const uint32_t na = d0 - ta < kDgTile ? d0 - ta : kDgTile;
      __syncthreads();
      for (uint32_t i = tid; i < na; i += kBlock) {
        uint32_t v = col[b0 + ta + i];
        DA[i] = rp[v + 1] - rp[v];
      }
      for (uint32_t tb = 0; tb < d0; tb += kDgTile) {
        const uint32_t nb = d0 - tb < kDgTile ? d0 - tb : kDgTile;
        __syncthreads();
        for (uint32_t i = tid; i < nb; i += kBlock) {
          uint32_t v = col[b0 + tb + i];
          DB[i] = rp[v + 1] - rp[v];
        }
        __syncthreads();
        for (uint32_t i = tid; i < na; i += kBlock) {
          const uint32_t x = DA[i];
          uint64_t s = 0;
          for (uint32_t j = 0; j < nb; ++j) {
            uint32_t y = DB[j];
            s += y < x ? y : x;
          }
          ext3 += s;
        }
      }
    }
    // the 2-paths: count their endpoints, listing each at its first visit
    for (uint32_t c0 = 0; c0 < d0; c0 += kDgOff) {
      const uint32_t cn = d0 - c0 < kDgOff ? d0 - c0 : kDgOff;
      uint32_t run = 0;
      for (uint32_t t = 0; t < cn; t += kBlock) {
        uint32_t i = t + tid, w = 0;
        if (i < cn) {
          uint32_t a1 = col[b0 + c0 + i];
          w = rp[a1 + 1] - rp[a1];
        }
        uint32_t tot = 0;
        uint32_t ex = block_excl_scan<kBlock>(w, tot);
        if (i < cn) Wp[i] = run + ex;
        run += tot;
      }
      if (tid == 0) Wp[cn] = run;
      __syncthreads();
      for (uint32_t q0 = 0; q0 < run; q0 += kBlock) {  // the whole wave takes every step
        const uint32_t q = q0 + tid;
        uint32_t a3 = 0;
        bool first = false;
        if (q < run) {
          uint32_t i = lds_owner(Wp, cn, q);  // i < cn: Wp[cn] = run > q
          uint32_t a1 = col[b0 + c0 + i];
          a3 = col[rp[a1] + (q - Wp[i])];
          first = atomicAdd(cnt + a3, 1u) == 0u;
        }
        const uint64_t fm = __ballot(first);
        if (fm) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&s_nl, (uint32_t)__popcll(fm));
          base = __shfl(base, 0, 64);
          if (first) list[base + (uint32_t)__popcll(fm & lanemask_lt())] = a3;
        }
      }
      __syncthreads();
    }
    // every count and list entry of this a0 is in before any is taken back
    __threadfence();
    __syncthreads();
    const uint32_t nl = s_nl;
    for (uint32_t i = tid; i < nl; i += kBlock) {
      const uint64_t k = atomicExch(cnt + list[i], 0u);
      matches += k * k;
    }
  }
  uint64_t v[3] = {matches, sq, ext3};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    uint64_t t = block_sum<kBlock>(v[i]);
    if (tid == 0 && t) atomicAdd(acc + i, (unsigned long long)t);
  }
}

void diamond2p_count(gj_ctx* c, const Version& v, uint32_t n, KernelTimer& timer, uint64_t out[3]) {
  const CsrDir& d = v.d[0];
  // one dense counter array and one endpoint list per workgroup, at most
  // 16 GiB in all
  uint64_t per = ((uint64_t)n + 63) / 64 * 64;
  uint64_t wgs = std::min<uint64_t>((uint64_t)c->num_cus * 2, std::max<uint64_t>(1, (16ull << 30) / (per * 8)));
  unsigned int* cnt = (unsigned int*)ws_get(c, "dg_cnt", wgs * per * sizeof(unsigned int));
  uint32_t* list = (uint32_t*)ws_get(c, "dg_list", wgs * per * sizeof(uint32_t));
  unsigned long long* ctr = (unsigned long long*)ws_get(c, "dg_ctr", 4 * sizeof(unsigned long long));
  GJ_HIP(hipMemsetAsync(cnt, 0, wgs * per * sizeof(unsigned int), c->stream));
  GJ_HIP(hipMemsetAsync(ctr, 0, 4 * sizeof(unsigned long long), c->stream));
  timer.start();
  k_diamond2p<<<(unsigned)wgs, kBlock, 0, c->stream>>>(d.rp, d.col, n, cnt, list, per, ctr, ctr + 1);
  timer.stop();
  GJ_HIP(hipGetLastError());
  unsigned long long h[4];
  read_bytes(c, h, ctr, sizeof(h));
  for (int i = 0; i < 3; ++i) out[i] = h[1 + i];
}

// ---------------------------------------------------------------- 4-cycle by 2-path counts
// The 4-cycle edge(a0,a1), edge(a1,a2), edge(a2,a3), edge(a3,a0): the
// matches from a0 pair each forward 2-path a0 -> a1 -> a2 with each backward
// one a2 -> a3 -> a0 of the same a2, so a0 contributes the sum over a2 of
// k(a2) k'(a2) (forward times backward 2-path counts).  One workgroup per a0
// adds the forward 2-paths' endpoints into its private counters (listing
// each endpoint at its first visit), walks the backward 2-paths (through
// the reverse index) summing the counters they reach, and clears the listed
// endpoints.  Counters as the
// depth-first evaluation: extensions[2] = prefixes[3] = the forward 2-paths
// (a2 is proposed from out(a1) alone), extensions[3] = the sum over them of
// min(|out(a2)|, |in(a0)|).

// Calls f(a1, a2) for every 2-path a0 -> a1 -> a2 with a1 in col1[b0, b0 + d0)
// and a2 in the row of a1 in (rp2, col2), over the workgroup.
template <class F>
__device__ __forceinline__ void walk_2paths(const uint32_t* __restrict__ col1, uint32_t b0, uint32_t d0,
                                            const uint32_t* __restrict__ rp2, const uint32_t* __restrict__ col2,
                                            uint32_t* Wp, F f) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t c0 = 0; c0 < d0; c0 += kDgOff) {
    const uint32_t cn = d0 - c0 < kDgOff ? d0 - c0 : kDgOff;
    uint32_t run = 0;
    for (uint32_t t = 0; t < cn; t += kBlock) {
      uint32_t i = t + tid, w = 0;
      if (i < cn) {
        uint32_t a1 = col1[b0 + c0 + i];
        w = rp2[a1 + 1] - rp2[a1];
      }
      uint32_t tot = 0;
      uint32_t ex = block_excl_scan<kBlock>(w, tot);
      if (i < cn) Wp[i] = run + ex;
      run += tot;
    }
    if (tid == 0) Wp[cn] = run;
    __syncthreads();
    for (uint32_t q = tid; q < run; q += kBlock) {
      uint32_t i = lds_owner(Wp, cn, q);  // i < cn: Wp[cn] = run > q
      uint32_t a1 = col1[b0 + c0 + i];
      f(a1, col2[rp2[a1] + (q - Wp[i])]);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_cycle4_2p(const uint32_t* __restrict__ rpf,
                                                      const uint32_t* __restrict__ colf,
                                                      const uint32_t* __restrict__ rpr,
                                                      const uint32_t* __restrict__ colr, uint32_t n,
                                                      unsigned int* __restrict__ cnt_all, uint32_t* __restrict__ list_all,
                                                      uint64_t cnt_stride, unsigned long long* __restrict__ claim,
                                                      unsigned long long* __restrict__ acc) {
  __shared__ uint32_t Wp[kDgOff + 1];
  __shared__ unsigned long long next;
  __shared__ uint32_t s_nl;  // forward endpoints listed for this a0
  unsigned int* cnt = cnt_all + (uint64_t)blockIdx.x * cnt_stride;
  uint32_t* list = list_all + (uint64_t)blockIdx.x * cnt_stride;
  const uint32_t tid = threadIdx.x;
  uint64_t matches = 0, paths = 0, ext3 = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      next = atomicAdd(claim, 1ull);
      s_nl = 0;
    }
    __syncthreads();
    const unsigned long long a0 = next;
    if (a0 >= n) break;
    const uint32_t bo = rpf[a0], dout = rpf[a0 + 1] - bo, bi = rpr[a0], din = rpr[a0 + 1] - bi;
    if (dout == 0) continue;
    walk_2paths(colf, bo, dout, rpf, colf, Wp, [&](uint32_t, uint32_t a2) {
      if (atomicAdd(cnt + a2, 1u) == 0u) list[atomicAdd(&s_nl, 1u)] = a2;  // first visit: listed
      uint32_t d2 = rpf[a2 + 1] - rpf[a2];
      ext3 += d2 < din ? d2 : din;
      paths += 1;
    });
    __threadfence();
    __syncthreads();
    if (din)
      walk_2paths(colr, bi, din, rpr, colr, Wp, [&](uint32_t, uint32_t a2) {
        matches += __hip_atomic_load(cnt + a2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // at L2
      });
    __syncthreads();
    // clear the listed endpoints (one store each instead of a third walk)
    const uint32_t nl = s_nl;
    for (uint32_t i = tid; i < nl; i += kBlock)
      __hip_atomic_store(cnt + list[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    __syncthreads();
  }
  uint64_t v[3] = {matches, paths, ext3};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    uint64_t t = block_sum<kBlock>(v[i]);
    if (tid == 0 && t) atomicAdd(acc + i, (unsigned long long)t);
  }
}

void cycle4_2p_count(gj_ctx* c, const Version& v, uint32_t n, KernelTimer& timer, uint64_t out[3]) {
  uint64_t per = ((uint64_t)n + 63) / 64 * 64;
  // one counter array and one endpoint list per workgroup, at most 16 GiB in all
  uint64_t wgs = std::min<uint64_t>((uint64_t)c->num_cus * 2, std::max<uint64_t>(1, (16ull << 30) / (per * 8)));
  unsigned int* cnt = (unsigned int*)ws_get(c, "dg_cnt", wgs * per * sizeof(unsigned int));
  uint32_t* list = (uint32_t*)ws_get(c, "dg_list", wgs * per * sizeof(uint32_t));
  unsigned long long* ctr = (unsigned long long*)ws_get(c, "dg_ctr", 4 * sizeof(unsigned long long));
  GJ_HIP(hipMemsetAsync(cnt, 0, wgs * per * sizeof(unsigned int), c->stream));
  GJ_HIP(hipMemsetAsync(ctr, 0, 4 * sizeof(unsigned long long), c->stream));
  timer.start();
  k_cycle4_2p<<<(unsigned)wgs, kBlock, 0, c->stream>>>(v.d[0].rp, v.d[0].col, v.d[1].rp, v.d[1].col, n, cnt, list,
                                                        per, ctr, ctr + 1);
  timer.stop();
  GJ_HIP(hipGetLastError());
  unsigned long long h[4];
  read_bytes(c, h, ctr, sizeof(h));
  for (int i = 0; i < 3; ++i) out[i] = h[1 + i];
}

}  // namespace gj
