// Allocation-free count: gj_run's COUNT mode on the depth-first path, with
// every workspace buffer a piece of one file-scope device array instead of a
// device allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array is resolved to its device address once per device (when a
// context is created on it): in host code the array's name is only a host
// stand-in, so every use goes through the resolved pointer.  Each device
// holds its own copy until the process ends.  Calls on one device share it;
// a per-device lock keeps them from overlapping (a call returns after its
// results are read, so its kernels are done when the lock is released).
#include <mutex>

#include "engine.h"
#include "gj_internal.h"

namespace gj {

constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static std::mutex g_init_mu;
static void* g_scratch[kMaxDevices];
static std::mutex g_dev_mu[kMaxDevices];

uint64_t scratch_bytes() { return kScratchBytes; }

// Device address of this device's scratch (the current device is made
// `device` while it is resolved).
void* scratch_ptr(int device) {
  GJ_CHECK(device >= 0 && device < kMaxDevices, GJ_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (!g_scratch[device]) {
    int prev = 0;
    GJ_HIP(hipGetDevice(&prev));
    GJ_HIP(hipSetDevice(device));
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    GJ_CHECK(e == hipSuccess && p, GJ_EDEVICE,
             std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

void scratch_lock(int device, bool lock) {
  if (lock)
    g_dev_mu[device].lock();
  else
    g_dev_mu[device].unlock();
}

// The context's options and arena while the allocation-free count runs;
// restored on every exit.
struct NoallocScope {
  gj_ctx* c;
  uint64_t frontier_cap, seed_chunk;
  int factorise;
  NoallocScope(gj_ctx* c_, uint64_t fcap) : c(c_) {
    frontier_cap = c->frontier_cap;
    seed_chunk = c->seed_chunk;
    factorise = c->factorise;
    c->frontier_cap = fcap;
    c->seed_chunk = fcap;
    c->factorise = 0;
    c->arena.on = true;
    c->arena.base = (uint8_t*)scratch_ptr(c->device);
    c->arena.size = kScratchBytes;
    c->arena.used = 0;
    c->arena.named.clear();
  }
  ~NoallocScope() {
    c->arena.on = false;
    c->arena.named.clear();
    c->frontier_cap = frontier_cap;
    c->seed_chunk = seed_chunk;
    c->factorise = factorise;
  }
};

}  // namespace gj

extern "C" gj_status gj_count_noalloc(gj_ctx* c, const gj_graph* g, const gj_query* q, uint64_t seed_lo,
                                      uint64_t seed_hi, uint64_t frontier_cap, gj_stats* stats) {
  if (!c || !g || !q) return GJ_EINVAL;
  gj_stats st{};
  gj_status s;
  try {
    GJ_HIP(hipSetDevice(c->device));
    gj::PlanH P = gj::make_plan(q, q->order, -1);
    GJ_CHECK(!g->lsm.on, GJ_EINVAL,
             "the graph has rows appended by log-structured updates; a static read (gj_run, gj_graph_info "
             "with degrees) merges them first, which allocates");
    // the largest batch bound whose buffers fit the scratch
    uint64_t fit = 0;
    for (uint64_t b = 64; b <= (1ull << 24); b <<= 1)
      if (gj::runner_scratch_bytes(P.m, b, b) <= gj::kScratchBytes) fit = b;
    uint64_t fcap = frontier_cap ? frontier_cap : fit;
    GJ_CHECK(fcap >= 64 && fcap <= fit, GJ_EINVAL,
             "frontier_cap " + std::to_string(frontier_cap) + " outside [64, " + std::to_string(fit) +
                 "] (the largest bound whose frontiers fit the " + std::to_string(gj::kScratchBytes) +
                 "-byte scratch for a query of " + std::to_string(P.m) + " attributes)");
    gj::scratch_lock(c->device, true);
    struct Unlock {
      int d;
      ~Unlock() { gj::scratch_lock(d, false); }
    } unlock{c->device};
    gj::NoallocScope scope(c, fcap);
    gj::scan_reserve(c, fcap + 1);
    const gj::Version& v = g->ver[g->cur];
    gj::Views V{&v, &v, -1};
    if (P.ntri) {
      GJ_CHECK(g->tri.rp && g->tri.version == g->version && g->tri.slot == g->cur, GJ_EINVAL,
               "no triangle index for the graph's current version (gj_graph_index_triangles)");
      V.tri = &g->tri;
    }
    int dir = P.seed_fwd ? 0 : 1;
    uint64_t hi = std::min<uint64_t>(seed_hi, v.m), lo = std::min<uint64_t>(seed_lo, hi);
    gj::Runner R(c, P, V, false, false, fcap);
    R.seed(v.d[dir].row + lo, v.d[dir].col + lo, nullptr, hi - lo);
    uint64_t matches = 0;
    int64_t ws = 0;
    R.finish(matches, ws);
    R.st.matches = matches;
    st = R.st;
    c->err.clear();
    s = GJ_OK;
  } catch (const gj::Error& e) {
    c->err = e.msg;
    s = e.code;
  } catch (...) {
    c->err = "unexpected failure";
    s = GJ_EDEVICE;
  }
  if (stats) *stats = st;
  return s;
}
