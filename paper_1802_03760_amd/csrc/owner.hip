// Owner-grouped intersection for the first extension stage of an
// edge-seeded query with two binding atoms, one on each seed attribute:
// count over seed edges (x0, x1) of |LA(x0) ∩ LB(x1)|.  Triangle counting is
// this stage (LA = out(a1), LB = out(a2)); so is the cyclic triangle.
//
// Count-minimisation (Sec. 3.1) makes the smaller of the two sets propose and
// the larger one check.  Here every seed edge is assigned to the owner of its
// larger set -- x0 when |LB(x1)| <= |LA(x0)| (ties: atom order), else x1 -- and
// all edges of one owner are processed together: a workgroup loads the
// owner's set once into an LDS hash table and streams the proposing sets of
// its partners through it with coalesced reads.  The paper's extension-index
// property of O(1) membership tests (Sec. 2.2) is what the LDS table
// provides; proposals per edge stay min(|LA|, |LB|), so the candidate count
// equals the count-minimisation total.
//
// Owner units (v, r): r = 0 holds the edges (v, x1) (partners from the seed
// index row of v, probe set LA(v)); r = 1 holds the edges (x0, v) (partners
// from the transposed seed index row of v, probe set LB(v)).  A unit's work
// is split into tasks of partner ranges; persistent workgroups take tasks
// from a device counter in owner-id order (hubs first on R-MAT ids), which is
// the (prefix, range) balancing of Sec. 3.4 applied within the GPU.  Probe
// sets larger than half the table are processed in id-range segments.  Edges
// whose larger set is below kDMin go to a per-edge merge in the same launch.
#include <algorithm>

#include "gj_internal.h"

#include "owner.h"
#include "prim.h"

namespace gj {

constexpr int kOwnNT = 1024;
constexpr int kLogSlots = 14;
constexpr uint32_t kSlots = 1u << kLogSlots;  // 64 KiB table
constexpr uint32_t kSegMax = kSlots / 2;      // load factor <= 1/2
constexpr uint32_t kDMin = 64;
constexpr uint32_t kLong = 64;  // proposing sets streamed by a whole wave
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

struct UnitLists {
  const uint32_t *prp, *padj;  // probe set
  const uint32_t *srp, *sadj;  // partners
  const uint32_t *qrp, *qadj;  // proposing sets of the partners
};

__device__ __forceinline__ UnitLists unit_lists(const OwnerArgs& a, uint32_t r) {
  UnitLists L;
  if (r == 0) {
    L.prp = a.rpA; L.padj = a.adjA;
    L.srp = a.rpS0; L.sadj = a.adjS0;
    L.qrp = a.rpB; L.qadj = a.adjB;
  } else {
    L.prp = a.rpB; L.padj = a.adjB;
    L.srp = a.rpS1; L.sadj = a.adjS1;
    L.qrp = a.rpA; L.qadj = a.adjA;
  }
  return L;
}

// r = 0 owns partners whose set is not larger; r = 1 only strictly smaller
__device__ __forceinline__ bool owned(uint32_t r, uint32_t s, uint32_t D) { return r == 0 ? s <= D : s < D; }

// ---------------------------------------------------------------- planning
// Per index entry (owner v = row, partner u = column) of role r: the number of
// proposals the entry contributes to unit (v, r), zero when the unit does not
// own the edge or its probe set is below kDMin.  A scan of these gives each
// unit's work and the work offset of each of its partners.
__global__ void k_owner_vals(OwnerArgs a, uint32_t r, const uint32_t* __restrict__ row,
                             const uint32_t* __restrict__ col, uint64_t m, uint32_t* __restrict__ vals) {
  UnitLists L = unit_lists(a, r);
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gs) {
    uint32_t v = row[e], u = col[e];
    uint32_t D = L.prp[v + 1] - L.prp[v];
    uint32_t s = L.qrp[u + 1] - L.qrp[u];
    vals[e] = (D >= kDMin && owned(r, s, D)) ? s : 0u;
  }
}

// task count of every unit: work / task size, at most one task per partner
__global__ void k_owner_units(OwnerArgs a, const uint64_t* __restrict__ wscan0, const uint64_t* __restrict__ wscan1,
                              uint64_t tw_min, uint32_t* __restrict__ ntasks,
                              unsigned long long* __restrict__ nsplit) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < 2ull * a.n; u += gs) {
    uint32_t v = (uint32_t)(u >> 1), r = (uint32_t)(u & 1);
    UnitLists L = unit_lists(a, r);
    const uint64_t* ws = r ? wscan1 : wscan0;
    uint32_t ps = L.srp[v], pe = L.srp[v + 1];
    uint64_t w = ws[pe] - ws[ps];
    uint32_t nt = 0;
    if (w) {
      uint32_t D = L.prp[v + 1] - L.prp[v];
      uint64_t nseg = (D + kSegMax - 1) / kSegMax;
      uint64_t tw = tw_min > 8ull * D * nseg ? tw_min : 8ull * D * nseg;
      uint64_t k = (w + tw - 1) / tw;
      uint64_t P = pe - ps;
      nt = (uint32_t)(k < P ? k : P);
    }
    ntasks[u] = nt;
    if (nt > 1) atomicAdd(nsplit, 1ull);
  }
}

// task = (unit, partner range); boundaries split the unit's work evenly
__global__ void k_owner_tasks(OwnerArgs a, const uint64_t* __restrict__ wscan0, const uint64_t* __restrict__ wscan1,
                              const uint32_t* __restrict__ ntasks, const uint64_t* __restrict__ toff,
                              uint32_t* __restrict__ tasks) {
  uint64_t gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < 2ull * a.n; u += gs) {
    uint32_t nt = ntasks[u];
    if (!nt) continue;
    uint32_t v = (uint32_t)(u >> 1), r = (uint32_t)(u & 1);
    UnitLists L = unit_lists(a, r);
    const uint64_t* ws = r ? wscan1 : wscan0;
    uint32_t ps = L.srp[v], pe = L.srp[v + 1];
    uint64_t w0 = ws[ps], W = ws[pe] - w0;
    uint64_t base = toff[u];
    uint32_t prev = 0;
    for (uint32_t k = 0; k < nt; ++k) {
      uint32_t next = pe - ps;
      if (k + 1 < nt) {
        // first partner whose work offset reaches the k+1-th share
        uint64_t target = w0 + W * (k + 1) / nt;
        uint32_t lo = ps, len = pe - ps;
        while (len > 0) {
          uint32_t half = len >> 1;
          if (ws[lo + half] < target) {
            lo += half + 1;
            len -= half + 1;
          } else {
            len = half;
          }
        }
        next = lo - ps;
        if (next < prev) next = prev;
      }
      tasks[3 * (base + k) + 0] = (uint32_t)u;
      tasks[3 * (base + k) + 1] = prev;
      tasks[3 * (base + k) + 2] = next;
      prev = next;
    }
  }
}

// ---------------------------------------------------------------- LDS hash
// Open addressing over buckets of four 32-bit slots, probed bucket by bucket
// (one 16-byte LDS read each).  Insertion claims the first empty slot of the
// first bucket with room, so the filled slots of a bucket are a prefix and a
// bucket with an empty last slot ends an unsuccessful search.
__device__ __forceinline__ uint32_t bucket_of(uint32_t x, int shift) { return (x * 0x9E3779B1u) >> shift; }

__device__ __forceinline__ void insert(uint32_t* H, uint32_t x, int shift, uint32_t bmask) {
  uint32_t b = bucket_of(x, shift);
  for (;;) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (atomicCAS(&H[4 * b + k], kEmpty, x) == kEmpty) return;
    b = (b + 1) & bmask;
  }
}

// continues an unsuccessful search after bucket b
__device__ __noinline__ bool probe_from(const uint32_t* H, uint32_t x, uint32_t b, uint32_t bmask) {
  const uint4* B = reinterpret_cast<const uint4*>(H);
  for (;;) {
    b = (b + 1) & bmask;
    uint4 q = B[b];
    if (q.x == x || q.y == x || q.z == x || q.w == x) return true;
    if (q.w == kEmpty) return false;
  }
}

__device__ __forceinline__ bool probe(const uint32_t* H, uint32_t x, int shift, uint32_t bmask) {
  const uint4* B = reinterpret_cast<const uint4*>(H);
  uint32_t b = bucket_of(x, shift);
  uint4 q = B[b];
  if (min(min(q.x ^ x, q.y ^ x), min(q.z ^ x, q.w ^ x)) == 0u) return true;
  if (q.w == kEmpty) return false;
  return probe_from(H, x, b, bmask);
}

// first i in [lo, hi) with a[i] >= x (hi if none), searching forward from lo
// by doubling steps first: cheap when the answer lies near lo
__device__ __forceinline__ uint32_t gallop_lb(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi, uint32_t x) {
  uint64_t step = 1, b = lo;
  while (b < hi && a[b] < x) {
    lo = (uint32_t)b + 1;
    b = lo + step;
    step <<= 1;
  }
  return lower_bound_u32(a, lo, b < hi ? (uint32_t)b : hi, x);
}

// ---------------------------------------------------------------- main kernel
// Per task: the owner's probe set goes into the LDS table (segment by
// segment), then its partners are taken kOwnNT at a time.  Partners whose
// proposing set has at least kLong elements are streamed by one wave each
// (stream_probe); shorter ones are concatenated and walked in 64-element
// windows.

// Buffer resource word 3 for gfx9-family raw buffers (32-bit dwords, no
// swizzle); loads at or past num_records bytes return zero.
constexpr int kBufWord3 = 0x00020000;

// One wave streams one proposing set through the table: U coalesced loads per
// step (raw-buffer loads off the wave-uniform base of the set, so addressing
// is one offset per step), issued one step ahead so that they are in flight
// while the previous step probes; then U first-bucket reads, and a
// membership test as a minimum of slot-xor-value (zero iff present), which
// keeps the test to a few full-rate instructions.  Values whose first bucket
// is full and lacks them walk on to later buckets behind one wave-uniform
// branch.
template <int U>
__device__ __forceinline__ uint32_t stream_probe(const uint32_t* __restrict__ set, uint32_t s, const uint32_t* H,
                                                 int shift, uint32_t mask) {
  const uint4* B = reinterpret_cast<const uint4*>(H);
  const uint32_t lane = (uint32_t)lane_id();
  // the wave's proposing set (wave-uniform base and size) as a raw buffer
  __amdgpu_buffer_rsrc_t R = __builtin_amdgcn_make_buffer_rsrc((void*)set, (short)0, (int)(s * 4u), kBufWord3);
  uint32_t hits = 0;
  uint32_t xn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) xn[u] = __builtin_amdgcn_raw_buffer_load_b32(R, lane * 4u + 256u * u, 0, 0);
  for (uint32_t i = lane; i < s; i += 64 * U) {
    uint32_t x[U], b[U];
    bool ok[U];
    uint4 q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = i + 64 * u < s;
      x[u] = xn[u];
    }
    // next step's loads in flight while this one probes (zero past the end)
#pragma unroll
    for (int u = 0; u < U; ++u) xn[u] = __builtin_amdgcn_raw_buffer_load_b32(R, (i + 64u * U) * 4u + 256u * u, 0, 0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      b[u] = bucket_of(x[u], shift);
      q[u] = B[b[u]];
    }
    uint32_t pend = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bool hit = min(min(q[u].x ^ x[u], q[u].y ^ x[u]), min(q[u].z ^ x[u], q[u].w ^ x[u])) == 0u;
      hits += (ok[u] & hit) ? 1u : 0u;
      pend |= (ok[u] & !hit & (q[u].w != kEmpty)) ? (1u << u) : 0u;
    }
    // a full first bucket without the value: walk on (one wave-uniform branch)
    if (__ballot(pend != 0)) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        bool more = (pend >> u) & 1u;
        uint32_t bb = b[u];
        while (__ballot(more)) {
          if (more) {
            bb = (bb + 1) & mask;
            uint4 r = B[bb];
            bool hit = min(min(r.x ^ x[u], r.y ^ x[u]), min(r.z ^ x[u], r.w ^ x[u])) == 0u;
            hits += hit ? 1u : 0u;
            more = !hit & (r.w != kEmpty);
          }
        }
      }
    }
  }
  return hits;
}

// SIGNED: seed edges carry signs (a.sg0, a.sg1), acc[2] gets the signed sum
template <bool SIGNED>
__global__ void __launch_bounds__(kOwnNT) __attribute__((amdgpu_waves_per_eu(8))) k_owner_count(OwnerArgs a, const uint32_t* __restrict__ tasks,
                                                        uint32_t ntask, unsigned int* __restrict__ counter,
                                                        const uint32_t* __restrict__ seed_row,
                                                        const uint32_t* __restrict__ seed_col, uint64_t E,
                                                        unsigned long long* __restrict__ acc) {
  __shared__ __attribute__((aligned(16))) uint32_t H[kSlots];
  __shared__ uint32_t pst[kOwnNT];       // start of each partner's proposing set
  __shared__ uint32_t pval[kOwnNT + 1];  // long: size; short: offset in the short space
  __shared__ uint16_t wstart[kOwnNT];    // short window -> set holding its first element
  __shared__ int8_t psg[kOwnNT];         // sign of each partner's seed edge
  __shared__ uint32_t s_task, s_long;
  __shared__ uint32_t s_scan[kOwnNT / 64 + 1];
  __shared__ uint64_t s_sum[kOwnNT / 64 + 1];
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  constexpr int nwaves = kOwnNT / 64;
  uint64_t hits = 0, ext = 0;
  int64_t shits = 0;  // hits times the sign of their seed edge

  for (;;) {
    if (tid == 0) s_task = atomicAdd(counter, 1u);
    __syncthreads();
    uint32_t t = s_task;
    __syncthreads();
    if (t >= ntask) break;
    uint32_t unit = tasks[3 * (uint64_t)t], plo = tasks[3 * (uint64_t)t + 1], phi = tasks[3 * (uint64_t)t + 2];
    uint32_t v = unit >> 1, r = unit & 1;
    UnitLists L = unit_lists(a, r);
    uint32_t Lb = L.prp[v], D = L.prp[v + 1] - Lb;
    uint32_t Sb = L.srp[v];
    uint32_t nseg = (D + kSegMax - 1) / kSegMax;
    // partners kOwnNT at a time; per chunk, the owner's set segment by
    // segment (the table is built once when the set is one segment)
    for (uint32_t c = plo; c < phi; c += kOwnNT) {
      uint32_t i = c + tid;
      uint32_t qb = 0, s_full = 0;
      int8_t sg = 1;
      if (i < phi) {
        if (SIGNED) sg = (r ? a.sg1 : a.sg0)[Sb + i];
        uint32_t u = L.sadj[Sb + i];
        qb = L.qrp[u];
        s_full = L.qrp[u + 1] - qb;
        if (!owned(r, s_full, D)) s_full = 0;
        ext += s_full;
      }
      uint32_t cur = qb;  // first element of the proposing set not yet given to a segment
      for (uint32_t seg = 0; seg < nseg; ++seg) {
        uint32_t e0 = seg * kSegMax, e1 = min(D, e0 + kSegMax), cnt = e1 - e0;
        // slots: power of two >= 8 * cnt (load <= 1/8) up to the table size
        int lg = 6;
        while ((1u << lg) < 8 * cnt && lg < kLogSlots) ++lg;
        uint32_t slots = 1u << lg, mask = (slots >> 2) - 1;  // mask over buckets
        int shift = 32 - (lg - 2);
        if (nseg > 1 || c == plo) {
          for (uint32_t k = tid; k < slots; k += kOwnNT) H[k] = kEmpty;
          __syncthreads();
          for (uint32_t k = tid; k < cnt; k += kOwnNT) insert(H, L.padj[Lb + e0 + k], shift, mask);
          __syncthreads();
        }
        // this segment takes the proposing elements up to its largest value
        // (those below its smallest are in no segment and simply miss)
        uint32_t st = cur, s = 0;
        if (s_full) {
          uint32_t end = qb + s_full;
          // vertex ids are below 2^32 - 1, so hi_s + 1 does not wrap
          uint32_t b1 = seg + 1 == nseg ? end : gallop_lb(L.qadj, cur, end, L.padj[Lb + e1 - 1] + 1);
          s = b1 - cur;
          cur = b1;
        }
        // one scan: long-partner count in the high half, short sizes in the low half
        bool is_long = s >= kLong;
        uint32_t total;
        uint32_t pre = block_scan_lean<kOwnNT>(is_long ? (1u << 16) : s, total, s_scan);
        uint32_t nlong = total >> 16, short_total = total & 0xFFFFu;
        uint32_t kl = pre >> 16;
        if (is_long) {
          pst[kl] = st;
          pval[kl] = s;
          if (SIGNED) psg[kl] = sg;
        } else {
          uint32_t j = nlong + ((uint32_t)tid - kl);
          uint32_t off = pre & 0xFFFFu;
          pst[j] = st;
          pval[j] = off;
          if (SIGNED) psg[j] = sg;
          // the windows of 64 short elements that start inside this set
          for (uint32_t w = (off + 63) >> 6; (w << 6) < off + s; ++w) wstart[w] = (uint16_t)j;
        }
        if (tid == 0) {
          pval[kOwnNT] = short_total;
          s_long = 0;
        }
        __syncthreads();
        // long partners: one wave each, taken dynamically
        for (;;) {
          uint32_t k = 0;
          if (lane == 0) k = atomicAdd(&s_long, 1u);
          k = __shfl(k, 0, 64);
          if (k >= nlong) break;
          // one wave per partner: its set's start and size are wave-uniform
          uint32_t st_k = __builtin_amdgcn_readfirstlane(pst[k]);
          uint32_t s_k = __builtin_amdgcn_readfirstlane(pval[k]);
          // loads per step by set size: fewer wasted lanes on short sets
          uint32_t h;
          if (s_k <= 128)
            h = stream_probe<2>(L.qadj + st_k, s_k, H, shift, mask);
          else if (s_k <= 192)
            h = stream_probe<3>(L.qadj + st_k, s_k, H, shift, mask);
          else
            h = stream_probe<4>(L.qadj + st_k, s_k, H, shift, mask);
          hits += h;
          if (SIGNED) shits += (int64_t)psg[k] * h;
        }
        // short partners: 64-element windows over their concatenation; a
        // lane starts from the set holding its window's first element
        for (uint32_t g0 = (uint32_t)wave * 64; g0 < short_total; g0 += nwaves * 64) {
          uint32_t g = g0 + lane;
          if (g < short_total) {
            uint32_t p = wstart[g0 >> 6];
            while (pval[p + 1] <= g) ++p;
            uint32_t x = L.qadj[pst[p] + (g - pval[p])];
            bool hit = probe(H, x, shift, mask);
            hits += hit ? 1 : 0;
            if (SIGNED) shits += hit ? psg[p] : 0;
          }
        }
        __syncthreads();
      }
    }
  }

  // Edges whose larger set is small (below kDMin = 64 values): each wave
  // scans 64 seed edges at a time, and the small ones among them are
  // intersected by the whole wave, up to four at once: each set in one
  // coalesced load, then every value of LA(x0) looked up among the values of
  // LB(x1) held in registers, through shuffles.
  for (uint64_t e0 = ((uint64_t)blockIdx.x * nwaves + wave) * 64; e0 < E;
       e0 += (uint64_t)gridDim.x * nwaves * 64) {
    uint64_t e = e0 + lane;
    uint32_t la = 0, da = 0, lb = 0, db = 0;
    bool small = false;
    if (e < E) {
      uint32_t x0 = seed_row[e], x1 = seed_col[e];
      la = a.rpA[x0];
      da = a.rpA[x0 + 1] - la;
      lb = a.rpB[x1];
      db = a.rpB[x1 + 1] - lb;
      small = (da > db ? da : db) < kDMin;
    }
    if (small) ext += da < db ? da : db;
    uint64_t m = __ballot(small);
    while (m) {
      constexpr int kG = 4;
      int src[kG];
#pragma unroll
      for (int t = 0; t < kG; ++t) {
        src[t] = m ? __ffsll((unsigned long long)m) - 1 : -1;
        m &= m ? m - 1 : 0;
      }
      uint32_t va[kG], vb[kG], na[kG];
#pragma unroll
      for (int t = 0; t < kG; ++t) {
        va[t] = vb[t] = 0xFFFFFFFFu;
        na[t] = 0;
        if (src[t] >= 0) {
          uint32_t lat = __shfl(la, src[t], 64), dat = __shfl(da, src[t], 64);
          uint32_t lbt = __shfl(lb, src[t], 64), dbt = __shfl(db, src[t], 64);
          na[t] = dat;
          if ((uint32_t)lane < dat) va[t] = a.adjA[lat + lane];
          if ((uint32_t)lane < dbt) vb[t] = a.adjB[lbt + lane];
        }
      }
#pragma unroll
      for (int t = 0; t < kG; ++t) {
        if (src[t] < 0) continue;
        // pos = number of (padded) values of LB below va, at most 63
        uint32_t pos = 0;
#pragma unroll
        for (uint32_t step = 32; step >= 1; step >>= 1) {
          uint32_t y = (uint32_t)__shfl((int)vb[t], (int)(pos + step - 1), 64);
          if (y < va[t]) pos += step;
        }
        uint32_t at = (uint32_t)__shfl((int)vb[t], (int)pos, 64);
        uint32_t eh = (uint32_t)__popcll(__ballot((uint32_t)lane < na[t] && at == va[t]));
        if (lane == 0) {
          hits += eh;
          if (SIGNED) shits += (int64_t)a.sg0[e0 + src[t]] * eh;
        }
      }
    }
  }

  uint64_t th = block_sum_lean<kOwnNT>(hits, s_sum);
  uint64_t te = block_sum_lean<kOwnNT>(ext, s_sum);
  if (tid == 0) {
    atomicAdd(acc, (unsigned long long)th);
    atomicAdd(acc + 1, (unsigned long long)te);
  }
  if (SIGNED) {
    uint64_t ts = block_sum_lean<kOwnNT>((uint64_t)shits, s_sum);  // two's complement: the signed sum
    if (tid == 0) atomicAdd(acc + 2, (unsigned long long)ts);
  }
}

// ---------------------------------------------------------------- host
void owner_count(gj_ctx* c, const OwnerArgs& a, const uint32_t* seed_row, const uint32_t* seed_col,
                 const uint32_t* t_row, const uint32_t* t_col, uint64_t E, KernelTimer& timer, uint64_t& matches,
                 uint64_t& extensions, int64_t* wsum, OwnerPlan* plan, uint64_t gen, gj_ctx* pc) {
  uint64_t units = 2ull * a.n;
  // acc: matches, extensions, signed sum, units split into several tasks
  unsigned long long* acc = (unsigned long long*)ws_get(c, "own_acc", 4 * sizeof(unsigned long long));
  unsigned int* counter = (unsigned int*)ws_get(c, "own_ctr", sizeof(unsigned int));
  GJ_HIP(hipMemsetAsync(acc, 0, 4 * sizeof(unsigned long long), c->stream));
  GJ_HIP(hipMemsetAsync(counter, 0, sizeof(unsigned int), c->stream));
  const uint64_t tw_min = c->owner_task_min;
  const uint32_t* key[4] = {a.rpA, a.rpB, a.rpS0, a.rpS1};
  const bool reuse = plan && plan->tasks && plan->gen == gen && plan->tw == tw_min &&
                     std::equal(key, key + 4, plan->key);
  uint64_t nt = 0, split = 0;
  const uint32_t* tasks = nullptr;
  if (reuse) {
    nt = plan->nt;
    split = plan->split_units;
    tasks = plan->tasks;
  } else {
    uint32_t* ntasks = (uint32_t*)ws_get(c, "own_nt", (units + 1) * sizeof(uint32_t));
    uint64_t* toff = (uint64_t*)ws_get(c, "own_toff", (units + 1) * sizeof(uint64_t));
    uint32_t* vals = (uint32_t*)ws_get(c, "own_vals", (E + 1) * sizeof(uint32_t));
    uint64_t* wscan0 = (uint64_t*)ws_get(c, "own_ws0", (E + 1) * sizeof(uint64_t));
    uint64_t* wscan1 = (uint64_t*)ws_get(c, "own_ws1", (E + 1) * sizeof(uint64_t));
    unsigned ge = grid_for(E, kBlock, 1u << 16);
    if (E) k_owner_vals<<<ge, kBlock, 0, c->stream>>>(a, 0, seed_row, seed_col, E, vals);
    scan_u32_to_u64(c, vals, wscan0, E);
    if (E) k_owner_vals<<<ge, kBlock, 0, c->stream>>>(a, 1, t_row, t_col, E, vals);
    scan_u32_to_u64(c, vals, wscan1, E);
    k_owner_units<<<grid_for(units, kBlock, 1u << 16), kBlock, 0, c->stream>>>(a, wscan0, wscan1, tw_min, ntasks,
                                                                               acc + 3);
    scan_u32_to_u64(c, ntasks, toff, units);
    uint64_t h2[2];
    read_u64s(c, {toff + units, (const uint64_t*)(acc + 3)}, h2);
    nt = h2[0];
    split = h2[1];
    GJ_CHECK(nt < (1ull << 32), GJ_EUNSUPPORTED, "too many owner tasks");
    uint32_t* tw = nullptr;
    if (plan) {
      // the plan is kept with the version: allocated through the graph's context
      if (plan->cap < 3 * nt + 3) {
        plan->gen = ~0ull;
        dev_free(pc, plan->tasks);
        plan->tasks = nullptr;
        plan->cap = 0;
        plan->tasks = (uint32_t*)dev_alloc(pc, (3 * nt + 3) * sizeof(uint32_t));
        plan->cap = 3 * nt + 3;
      }
      tw = plan->tasks;
    } else {
      tw = (uint32_t*)ws_get(c, "own_tasks", (3 * nt + 3) * sizeof(uint32_t));
    }
    k_owner_tasks<<<grid_for(units, kBlock, 1u << 16), kBlock, 0, c->stream>>>(a, wscan0, wscan1, ntasks, toff, tw);
    GJ_HIP(hipGetLastError());
    tasks = tw;
    if (plan) {
      plan->nt = nt;
      plan->split_units = split;
      plan->tw = tw_min;
      std::copy(key, key + 4, plan->key);
      plan->gen = gen;
    }
  }
  unsigned grid = (unsigned)c->num_cus * 2;
  timer.start();
  GJ_CHECK((a.sg0 == nullptr) == (a.sg1 == nullptr), GJ_EINVAL, "owner kernel: signs for one order only");
  if (a.sg0)
    k_owner_count<true><<<grid, kOwnNT, 0, c->stream>>>(a, tasks, (uint32_t)nt, counter, seed_row, seed_col, E, acc);
  else
    k_owner_count<false><<<grid, kOwnNT, 0, c->stream>>>(a, tasks, (uint32_t)nt, counter, seed_row, seed_col, E, acc);
  timer.stop();
  GJ_HIP(hipGetLastError());
  unsigned long long h[3];
  read_bytes(c, h, acc, sizeof(h));
  c->owner_tasks = nt;
  c->owner_split_units = split;
  matches = h[0];
  extensions = h[1];
  if (wsum) *wsum = a.sg0 ? (int64_t)h[2] : (int64_t)h[0];
}

}  // namespace gj
