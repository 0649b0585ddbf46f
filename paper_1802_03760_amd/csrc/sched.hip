// Seed-work estimates: how much Generic Join work each seed edge of a count
// request will cause, so that the server can cut requests into chunks of
// bounded work and order them by remaining work.
//
// Per seed (x0, x1): 1 for the seed itself, plus c3 = the count-min of the
// third attribute (the minimum over its binding atoms of the extension-set
// size, Sec. 2.2), which is exactly the number of level-3 extensions the seed
// proposes; for a fourth attribute c3 * u4, where u4 is the smallest
// extension set among the atoms binding it through a seed attribute (an upper
// bound of each level-4 count-min), or a default fan-out when none does;
// every further attribute multiplies by the default fan-out.  The scheduler
// rescales the estimate of each request by the work its finished chunks
// actually did.
#include <cstring>

#include "prim.h"
#include "sched.h"

namespace gj {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kMaxBlocks = 1024;  // estimate blocks per request
constexpr uint32_t kFan = 16;          // default fan-out of a level
constexpr uint32_t kFanCap = 256;      // cap of the level-4 bound

struct WorkDesc {
  const uint32_t* row;
  const uint32_t* col;
  uint64_t lo, len, out_off;
  uint32_t bs, nb;
  int m, k3, k4;
  int col3[kMaxBind];
  const uint32_t* rp3[kMaxBind];
  int col4[kMaxBind];
  const uint32_t* rp4[kMaxBind];
};

__global__ void __launch_bounds__(kThreads) k_seed_work(const WorkDesc* __restrict__ D, uint64_t* __restrict__ out) {
  const WorkDesc& d = D[blockIdx.y];
  uint32_t b = blockIdx.x;
  if (b >= d.nb) return;  // uniform over the workgroup
  uint64_t s = (uint64_t)b * d.bs;
  uint64_t e = s + d.bs < d.len ? s + d.bs : d.len;
  uint64_t acc = 0;
  for (uint64_t i = s + threadIdx.x; i < e; i += kThreads) {
    uint32_t x0 = d.row[d.lo + i], x1 = d.col[d.lo + i];
    uint64_t w = 1;
    if (d.m >= 3) {
      uint32_t c3 = d.k3 ? 0xffffffffu : 0u;
      for (int a = 0; a < d.k3; ++a) {
        uint32_t v = d.col3[a] ? x1 : x0;
        uint32_t deg = d.rp3[a][v + 1] - d.rp3[a][v];
        c3 = deg < c3 ? deg : c3;
      }
      w += c3;
      if (d.m >= 4) {
        uint32_t u = kFan;
        if (d.k4) {
          u = 0xffffffffu;
          for (int a = 0; a < d.k4; ++a) {
            uint32_t v = d.col4[a] ? x1 : x0;
            uint32_t deg = d.rp4[a][v + 1] - d.rp4[a][v];
            u = deg < u ? deg : u;
          }
        }
        uint64_t deep = (uint64_t)c3 * (u < kFanCap ? u : kFanCap);
        for (int j = 5; j <= d.m; ++j) deep *= kFan;
        w += deep;
      }
    }
    acc += w;
  }
  acc = block_sum<kThreads>(acc);
  if (threadIdx.x == 0) out[d.out_off + b] = acc;
}

}  // namespace

void seed_work(gj_ctx* c, const std::vector<WorkReq>& reqs, std::vector<uint64_t>& out, std::vector<uint64_t>& off) {
  size_t n = reqs.size();
  off.assign(n + 1, 0);
  out.clear();
  if (!n) return;
  GJ_CHECK(n <= 65535, GJ_EINVAL, "too many requests to estimate at once");
  std::vector<WorkDesc> h(n);
  uint32_t max_nb = 0;
  for (size_t i = 0; i < n; ++i) {
    const WorkReq& r = reqs[i];
    const PlanH& P = *r.P;
    WorkDesc& d = h[i];
    memset(&d, 0, sizeof(d));
    GJ_CHECK(r.bs >= 1, GJ_EINVAL, "estimate block of zero seeds");
    int dir = P.seed_fwd ? 0 : 1;
    d.row = r.v->d[dir].row;
    d.col = r.v->d[dir].col;
    d.lo = r.lo;
    d.len = r.len;
    d.bs = r.bs;
    uint64_t nb = (r.len + r.bs - 1) / r.bs;
    GJ_CHECK(nb <= kMaxBlocks, GJ_EINVAL, "estimate blocks per request exceed the limit");
    d.nb = (uint32_t)nb;
    d.m = P.m;
    if (P.m >= 3) {
      for (const BindH& bd : P.bind[2]) {
        if (d.k3 == kMaxBind) break;
        d.col3[d.k3] = bd.col;
        d.rp3[d.k3] = r.v->d[bd.dir].rp;
        ++d.k3;
      }
    }
    if (P.m >= 4) {
      for (const BindH& bd : P.bind[3]) {
        if (bd.col > 1 || d.k4 == kMaxBind) continue;
        d.col4[d.k4] = bd.col;
        d.rp4[d.k4] = r.v->d[bd.dir].rp;
        ++d.k4;
      }
    }
    d.out_off = off[i];
    off[i + 1] = off[i] + nb;
    if (d.nb > max_nb) max_nb = d.nb;
  }
  out.assign(off[n], 0);
  if (!max_nb) return;
  WorkDesc* dd = (WorkDesc*)ws_get(c, "sw_desc", n * sizeof(WorkDesc));
  uint64_t* dout = (uint64_t*)ws_get(c, "sw_out", off[n] * sizeof(uint64_t));
  GJ_HIP(hipMemcpyAsync(dd, h.data(), n * sizeof(WorkDesc), hipMemcpyHostToDevice, c->stream));
  k_seed_work<<<dim3(max_nb, (unsigned)n), kThreads, 0, c->stream>>>(dd, dout);
  GJ_HIP(hipGetLastError());
  GJ_HIP(hipMemcpyAsync(out.data(), dout, off[n] * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
  GJ_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace gj
