// C ABI of libgj.so (declared in include/gj.h): argument checks, device
// memory, error reporting.  The computation lives in the other sources.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>

#include "batch.h"
#include "engine.h"
#include "gj_internal.h"
#include "sched.h"

namespace gj {

void* dev_alloc(gj_ctx* c, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  GJ_CHECK(!c->arena.on, GJ_EUNSUPPORTED, "device allocation requested inside the allocation-free path");
  if (c->alloc.alloc) {
    p = c->alloc.alloc(c->alloc.user, bytes, (void*)c->stream);
    if (!p) throw Error{GJ_ENOMEM, "allocator returned no memory for " + std::to_string(bytes) + " bytes"};
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{GJ_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  return p;
}

void dev_free(gj_ctx* c, void* p) {
  if (!p) return;
  if (c->alloc.alloc) {
    // the device is done with p before the allocator may hand it out again
    (void)hipStreamSynchronize(c->stream);
    c->alloc.free(c->alloc.user, p, (void*)c->stream);
    return;
  }
  (void)hipFree(p);
}

// Named grow-only workspace buffers owned by the context (or, inside the
// allocation-free path, named pieces of its scratch, reserved once per call).
void* ws_get(gj_ctx* c, const std::string& name, size_t bytes) {
  if (c->arena.on) {
    gj_ctx::Arena& A = c->arena;
    auto it = A.named.find(name);
    if (it != A.named.end()) {
      GJ_CHECK(bytes <= it->second.bytes, GJ_EUNSUPPORTED,
               "scratch piece " + name + " outgrew its reservation");
      return it->second.p;
    }
    uint64_t at = (A.used + kArenaAlign - 1) & ~(kArenaAlign - 1);
    GJ_CHECK(at + bytes <= A.size, GJ_EUNSUPPORTED,
             "the " + std::to_string(A.size) + "-byte scratch cannot hold piece " + name);
    A.used = at + bytes;
    A.named[name] = DevBuf{A.base + at, bytes};
    return A.base + at;
  }
  DevBuf& b = c->ws[name];
  if (bytes <= b.bytes && b.p) return b.p;
  size_t want = bytes + bytes / 8 + 256;
  if (b.p && b.bytes <= kWsRetireMax) {
    // A small buffer that grows is retired, not freed: freeing synchronises
    // the device (every stream, other threads' included), which would stall
    // a server's other lanes behind this context's growth.  Growth at least
    // doubles, so the retired buffers of a name total at most its final
    // size; they are freed with the context.
    want = std::max<size_t>(want, 2 * b.bytes);
    void* np = dev_alloc(c, want);
    c->ws_retired.push_back(b.p);
    b.p = np;
    b.bytes = want;
    return b.p;
  }
  if (b.p) {
    GJ_HIP(hipStreamSynchronize(c->stream));
    dev_free(c, b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  b.p = dev_alloc(c, want);
  b.bytes = want;
  return b.p;
}

void read_bytes(gj_ctx* c, void* host, const void* dptr, size_t bytes) {
  if (bytes <= 4096) {
    GJ_HIP(hipMemcpyAsync(c->pinned, dptr, bytes, hipMemcpyDeviceToHost, c->stream));
    GJ_HIP(hipStreamSynchronize(c->stream));
    memcpy(host, c->pinned, bytes);
  } else {
    GJ_HIP(hipMemcpyAsync(host, dptr, bytes, hipMemcpyDeviceToHost, c->stream));
    GJ_HIP(hipStreamSynchronize(c->stream));
  }
}

void read_u64s(gj_ctx* c, std::initializer_list<const uint64_t*> ptrs, uint64_t* host) {
  GJ_CHECK(ptrs.size() * sizeof(uint64_t) <= 4096, GJ_EINVAL, "too many values to read");
  uint64_t* st = (uint64_t*)c->pinned;
  size_t i = 0;
  for (const uint64_t* p : ptrs)
    GJ_HIP(hipMemcpyAsync(st + i++, p, sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
  GJ_HIP(hipStreamSynchronize(c->stream));
  memcpy(host, st, ptrs.size() * sizeof(uint64_t));
}

void KernelTimer::start() {
  if (c_->arena.on) return;  // the allocation-free path creates no events (launches still counted)
  if (c_->events.size() < 2 * (n_ + 1)) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      GJ_HIP(hipEventCreate(&e));
      c_->events.push_back(e);
    }
  }
  GJ_HIP(hipEventRecord(c_->events[2 * n_], c_->stream));
}

void KernelTimer::stop() {
  if (!c_->arena.on) GJ_HIP(hipEventRecord(c_->events[2 * n_ + 1], c_->stream));
  ++n_;
}

double KernelTimer::total_ms() {
  GJ_HIP(hipStreamSynchronize(c_->stream));
  if (c_->arena.on) return 0.0;
  double t = 0;
  for (size_t i = 0; i < n_; ++i) {
    float ms = 0;
    GJ_HIP(hipEventElapsedTime(&ms, c_->events[2 * i], c_->events[2 * i + 1]));
    t += ms;
  }
  return t;
}

void read_u32s(gj_ctx* c, std::initializer_list<const uint32_t*> ptrs, uint32_t* host) {
  GJ_CHECK(ptrs.size() * sizeof(uint32_t) <= 4096, GJ_EINVAL, "too many values to read");
  uint32_t* st = (uint32_t*)c->pinned;
  size_t i = 0;
  for (const uint32_t* p : ptrs)
    GJ_HIP(hipMemcpyAsync(st + i++, p, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  GJ_HIP(hipStreamSynchronize(c->stream));
  memcpy(host, st, ptrs.size() * sizeof(uint32_t));
}

uint64_t read_u64(gj_ctx* c, const void* dptr) {
  uint64_t v = 0;
  read_bytes(c, &v, dptr, sizeof(v));
  return v;
}

}  // namespace gj

using gj::Error;

template <class F>
static gj_status guarded(gj_ctx* c, F&& f) {
  try {
    if (c) {
      hipError_t e = hipSetDevice(c->device);
      if (e != hipSuccess) throw Error{GJ_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e)};
    }
    f();
    if (c) c->err.clear();
    return GJ_OK;
  } catch (const Error& e) {
    if (c) c->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return GJ_ENOMEM;
  } catch (...) {
    if (c) c->err = "unexpected failure";
    return GJ_EDEVICE;
  }
}

extern "C" {

gj_status gj_ctx_create(int device, void* hip_stream, const gj_allocator* allocator, gj_ctx** out) {
  if (!out) return GJ_EINVAL;
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free)) return GJ_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GJ_EDEVICE;
  gj_ctx* c = new (std::nothrow) gj_ctx();
  if (!c) return GJ_ENOMEM;
  c->device = device;
  if (allocator) c->alloc = *allocator;
  gj_status s = guarded(c, [&] {
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      GJ_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    GJ_HIP(hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault));
    (void)gj::scratch_ptr(device);  // the allocation-free entry point's scratch on this device
    hipDeviceProp_t prop;
    GJ_HIP(hipGetDeviceProperties(&prop, device));
    c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  });
  if (s != GJ_OK) {
    gj_ctx_destroy(c);
    return s;
  }
  *out = c;
  return GJ_OK;
}

void gj_ctx_destroy(gj_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  gj::batch_destroy(c);
  for (auto& kv : c->ws) gj::dev_free(c, kv.second.p);
  for (void* p : c->ws_retired) gj::dev_free(c, p);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* gj_last_error(const gj_ctx* c) { return c ? c->err.c_str() : "null context"; }

gj_status gj_ctx_set_option(gj_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return GJ_EINVAL;
  return guarded(c, [&] {
    std::string k(key);
    if (k == "frontier_cap") {
      GJ_CHECK(value >= 64 && value <= (1ll << 34), GJ_EINVAL, "frontier_cap out of range");
      c->frontier_cap = (uint64_t)value;
    } else if (k == "seed_chunk") {
      GJ_CHECK(value >= 1 && value <= (1ll << 32), GJ_EINVAL, "seed_chunk out of range");
      c->seed_chunk = (uint64_t)value;
    } else if (k == "strategy") {
      GJ_CHECK(value >= 0 && value <= 2, GJ_EINVAL, "strategy out of range");
      c->strategy = (int)value;
    } else if (k == "delta_owner_min") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "delta_owner_min must be >= 0");
      c->delta_owner_min = (uint64_t)value;
    } else if (k == "delta_lane_min") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "delta_lane_min must be >= 0");
      c->delta_lane_min = (uint64_t)value;
    } else if (k == "owner_task_min") {
      GJ_CHECK(value >= 1 && value <= (1ll << 40), GJ_EINVAL, "owner_task_min out of range");
      c->owner_task_min = (uint64_t)value;
    } else if (k == "hash_index") {
      GJ_CHECK(value >= 0 && value <= 2, GJ_EINVAL, "hash_index must be 0, 1 or 2");
      c->hash_index = (int)value;
    } else if (k == "hash_min_degree") {
      GJ_CHECK(value >= 1 && value <= (1ll << 31), GJ_EINVAL, "hash_min_degree out of range");
      c->hash_min_degree = (uint32_t)value;
    } else if (k == "hash_build_work") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "hash_build_work must be >= 0");
      c->hash_build_work = (uint64_t)value;
    } else if (k == "delta_fused") {
      GJ_CHECK(value == 0 || value == 1, GJ_EINVAL, "delta_fused must be 0 or 1");
      c->delta_fused = (int)value;
    } else if (k == "batch_heavy") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "batch_heavy must be >= 0");
      c->batch_heavy = (uint64_t)value;
    } else if (k == "propose_u") {
      GJ_CHECK(value == 1 || value == 2 || value == 4, GJ_EINVAL, "propose_u must be 1, 2 or 4");
      c->propose_u = (int)value;
    } else if (k == "factorise") {
      GJ_CHECK(value == 0 || value == 1, GJ_EINVAL, "factorise must be 0 or 1");
      c->factorise = (int)value;
    } else if (k == "lsm_updates") {
      GJ_CHECK(value == 0 || value == 1, GJ_EINVAL, "lsm_updates must be 0 or 1");
      c->lsm_updates = (int)value;
    } else if (k == "lsm_max_patch") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "lsm_max_patch must be >= 0");
      c->lsm_max_patch = (uint64_t)value;
    } else if (k == "lsm_fold_min") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "lsm_fold_min must be >= 0");
      c->lsm_fold_min = (uint64_t)value;
    } else if (k == "batch_cap") {
      GJ_CHECK(value >= 64 && value <= (1ll << 32), GJ_EINVAL, "batch_cap out of range");
      c->batch_cap = (uint64_t)value;
    } else if (k == "batch_lin") {
      GJ_CHECK(value >= 0 && value <= 4096, GJ_EINVAL, "batch_lin out of range");
      c->batch_lin = (uint32_t)value;
    } else if (k == "batch_claim_words") {
      GJ_CHECK(value >= 1 && value <= 4096, GJ_EINVAL, "batch_claim_words out of range");
      c->batch_claim_words = (uint32_t)value;
    } else if (k == "run_big") {
      GJ_CHECK(value == 0 || value == 1, GJ_EINVAL, "run_big must be 0 or 1");
      c->run_big = (int)value;
    } else if (k == "batch_run") {
      GJ_CHECK(value == 0 || value == 1, GJ_EINVAL, "batch_run must be 0 or 1");
      c->batch_run = (int)value;
    } else if (k == "run_stage") {
      GJ_CHECK(value == 0 || value == 1, GJ_EINVAL, "run_stage must be 0 or 1");
      c->run_stage = (int)value;
    } else if (k == "run_ratio") {
      GJ_CHECK(value >= 0 && value <= 64, GJ_EINVAL, "run_ratio out of range");
      c->run_ratio = (uint32_t)value;
    } else if (k == "run_min_work") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "run_min_work must be >= 0");
      c->run_min_work = (uint64_t)value;
    } else if (k == "run_task_work") {
      GJ_CHECK(value >= 1 && value <= (1ll << 40), GJ_EINVAL, "run_task_work out of range");
      c->run_task_work = (uint64_t)value;
    } else if (k == "run_reuse") {
      GJ_CHECK(value >= 1 && value <= 1024, GJ_EINVAL, "run_reuse out of range");
      c->run_reuse = (uint32_t)value;
    } else if (k == "run_min_tasks") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "run_min_tasks must be >= 0");
      c->run_min_tasks = (uint64_t)value;
    } else if (k == "run_stage_min") {
      GJ_CHECK(value >= 0, GJ_EINVAL, "run_stage_min must be >= 0");
      c->run_stage_min = (uint64_t)value;
    } else if (k == "batch_waves_per_cu") {
      GJ_CHECK(value >= 4 && value <= 128 && value % 4 == 0, GJ_EINVAL, "batch_waves_per_cu out of range");
      c->batch_waves_per_cu = (uint32_t)value;
    } else {
      throw Error{GJ_EINVAL, "unknown option " + k};
    }
  });
}

gj_status gj_ctx_get_option(gj_ctx* c, const char* key, int64_t* value) {
  if (!c || !key || !value) return GJ_EINVAL;
  return guarded(c, [&] {
    std::string k(key);
    if (k == "frontier_cap") *value = (int64_t)c->frontier_cap;
    else if (k == "seed_chunk") *value = (int64_t)c->seed_chunk;
    else if (k == "strategy") *value = c->strategy;
    else if (k == "batch_cap") *value = (int64_t)c->batch_cap;
    else if (k == "batch_lin") *value = c->batch_lin;
    else if (k == "batch_waves_per_cu") *value = c->batch_waves_per_cu;
    else if (k == "batch_claim_words") *value = c->batch_claim_words;
    else if (k == "batch_run") *value = c->batch_run;
    else if (k == "run_big") *value = c->run_big;
    else if (k == "batch_fallbacks") *value = (int64_t)c->batch_fallbacks;
    else if (k == "delta_fused") *value = c->delta_fused;
    else if (k == "delta_owner_min") *value = (int64_t)c->delta_owner_min;
    else if (k == "delta_lane_min") *value = (int64_t)c->delta_lane_min;
    else if (k == "factorise") *value = c->factorise;
    else if (k == "propose_u") *value = c->propose_u;
    else if (k == "batch_heavy") *value = (int64_t)c->batch_heavy;
    else if (k == "lsm_updates") *value = c->lsm_updates;
    else if (k == "lsm_max_patch") *value = (int64_t)c->lsm_max_patch;
    else if (k == "lsm_compactions") *value = (int64_t)c->lsm_compactions;
    else if (k == "lsm_folds") *value = (int64_t)c->lsm_folds;
    else if (k == "lsm_fold_min") *value = (int64_t)c->lsm_fold_min;
    else if (k == "owner_task_min") *value = (int64_t)c->owner_task_min;
    else if (k == "hash_index") *value = c->hash_index;
    else if (k == "hash_min_degree") *value = c->hash_min_degree;
    else if (k == "hash_build_work") *value = (int64_t)c->hash_build_work;
    else if (k == "hash_builds") *value = (int64_t)c->hash_builds;
    else if (k == "run_stage") *value = c->run_stage;
    else if (k == "run_ratio") *value = c->run_ratio;
    else if (k == "run_min_work") *value = (int64_t)c->run_min_work;
    else if (k == "run_task_work") *value = (int64_t)c->run_task_work;
    else if (k == "run_stage_min") *value = (int64_t)c->run_stage_min;
    else if (k == "run_tasks") *value = (int64_t)c->run_tasks;
    else if (k == "run_tasks_big") *value = (int64_t)c->run_tasks_big;
    else if (k == "run_declined") *value = (int64_t)c->run_declined;
    else if (k == "run_min_tasks") *value = (int64_t)c->run_min_tasks;
    else if (k == "run_reuse") *value = c->run_reuse;
    else if (k == "run_w_staged" || k == "run_w_large" || k == "run_w_light" || k == "run_units" ||
             k == "run_builds" || k == "run_build_elems") {
      static const char* names[] = {"run_w_staged", "run_w_large", "run_w_light", "run_units", "run_builds",
                                    "run_build_elems"};
      uint64_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (c->run_stats) gj::read_bytes(c, h, c->run_stats, sizeof(h));
      for (int i = 0; i < 6; ++i)
        if (k == names[i]) *value = (int64_t)h[i];
    }
    else if (k == "owner_tasks") *value = (int64_t)c->owner_tasks;
    else if (k == "owner_split_units") *value = (int64_t)c->owner_split_units;
    else throw Error{GJ_EINVAL, "unknown option " + k};
  });
}

gj_status gj_graph_build(gj_ctx* c, const uint32_t* src, const uint32_t* dst, uint64_t m, uint32_t nv,
                         uint32_t flags, gj_graph** out) {
  if (!c || !out) return GJ_EINVAL;
  *out = nullptr;
  gj_graph* g = nullptr;
  gj_status s = guarded(c, [&] {
    GJ_CHECK((flags & ~(GJ_INPUT_DEVICE | GJ_BUILD_UNDIRECTED | GJ_BUILD_DEGREE_ORDER)) == 0, GJ_EINVAL,
             "unknown or unsupported graph flags");
    GJ_CHECK(nv > 0, GJ_EINVAL, "num_vertices must be positive");
    GJ_CHECK(m < (1ull << 32), GJ_EUNSUPPORTED, "graphs of 2^32 edges or more are not supported");
    bool sym = (flags & (GJ_BUILD_UNDIRECTED | GJ_BUILD_DEGREE_ORDER)) != 0;
    GJ_CHECK(!sym || m < (1ull << 31), GJ_EUNSUPPORTED,
             "undirected builds of 2^31 input edges or more are not supported");
    GJ_CHECK(m == 0 || (src && dst), GJ_EINVAL, "null edge arrays");
    g = new gj_graph();
    g->ctx = c;
    g->n = nv;
    const uint32_t *ds = src, *dd = dst;
    if (!(flags & GJ_INPUT_DEVICE) && m) {
      uint32_t* s2 = (uint32_t*)gj::ws_get(c, "in_src", m * sizeof(uint32_t));
      uint32_t* d2 = (uint32_t*)gj::ws_get(c, "in_dst", m * sizeof(uint32_t));
      GJ_HIP(hipMemcpyAsync(s2, src, m * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
      GJ_HIP(hipMemcpyAsync(d2, dst, m * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
      ds = s2;
      dd = d2;
    }
    if (sym)
      gj::graph_build_sym(c, g, ds, dd, m, (flags & GJ_BUILD_DEGREE_ORDER) != 0,
                          (flags & GJ_BUILD_UNDIRECTED) != 0);
    else
      gj::graph_build(c, g, ds, dd, m);
    GJ_HIP(hipStreamSynchronize(c->stream));
  });
  if (s != GJ_OK) {
    gj_graph_destroy(g);
    return s;
  }
  *out = g;
  return GJ_OK;
}

gj_status gj_graph_info(const gj_graph* g, uint64_t* edges, uint32_t* vertices, uint32_t* max_out,
                        uint32_t* max_in, uint64_t* version) {
  if (!g) return GJ_EINVAL;
  if (max_out || max_in) {
    gj_status s = gj::settle(g->ctx, g);
    if (s != GJ_OK) return s;
  }
  const gj::Version& v = g->ver[g->cur];
  if (edges) *edges = g->lsm.on ? g->lsm.m : v.m;
  if (vertices) *vertices = g->n;
  if (max_out) *max_out = v.max_deg[0];
  if (max_in) *max_in = v.max_deg[1];
  if (version) *version = g->version;
  return GJ_OK;
}

gj_status gj_graph_csr(const gj_graph* g, int reverse, const uint32_t** row_ptr, const uint32_t** col,
                       const uint32_t** row) {
  if (!g || (reverse != 0 && reverse != 1)) return GJ_EINVAL;
  gj_status s = gj::settle(g->ctx, g);
  if (s != GJ_OK) return s;
  const gj::CsrDir& d = g->ver[g->cur].d[reverse];
  if (row_ptr) *row_ptr = d.rp;
  if (col) *col = d.col;
  if (row) *row = d.row;
  return GJ_OK;
}

void gj_graph_destroy(gj_graph* g) {
  if (!g) return;
  if (g->ctx) {
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
  }
  for (auto& v : g->ver) {
    gj::hash_free(g->ctx, v);
    gj::dev_free(g->ctx, v.plan.tasks);
    v.plan = gj::OwnerPlan{};
    gj::version_free(g->ctx, v);
  }
  gj::lsm_free(g);
  gj::tri_index_free(g);
  gj::dev_free(g->ctx, g->old_of_new);
  delete g;
}

gj_status gj_graph_index_triangles(gj_ctx* c, gj_graph* g, uint64_t* num_triangles) {
  if (!c || !g) return GJ_EINVAL;
  return guarded(c, [&] {
    gj::graph_compact(c, g);
    gj::tri_index_build(c, g);
    if (num_triangles) *num_triangles = g->tri.size;
  });
}

gj_status gj_graph_vertex_ids(const gj_graph* g, uint32_t* old_of_new, int out_on_device) {
  if (!g || !old_of_new) return GJ_EINVAL;
  gj_ctx* c = g->ctx;
  return guarded(c, [&] {
    uint64_t bytes = (uint64_t)g->n * sizeof(uint32_t);
    if (g->old_of_new) {
      GJ_HIP(hipMemcpyAsync(old_of_new, g->old_of_new, bytes,
                            out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
      GJ_HIP(hipStreamSynchronize(c->stream));
    } else if (!out_on_device) {
      for (uint32_t i = 0; i < g->n; ++i) old_of_new[i] = i;
    } else {
      std::vector<uint32_t> id(g->n);
      for (uint32_t i = 0; i < g->n; ++i) id[i] = i;
      GJ_HIP(hipMemcpyAsync(old_of_new, id.data(), bytes, hipMemcpyHostToDevice, c->stream));
      GJ_HIP(hipStreamSynchronize(c->stream));
    }
  });
}

gj_status gj_query_register(gj_ctx* c, uint32_t num_attrs, const gj_atom* atoms, uint32_t num_atoms,
                            const uint8_t* order, gj_query** out) {
  return gj_query_register_ex(c, num_attrs, atoms, num_atoms, order, nullptr, 0, out);
}

gj_status gj_query_register_ex(gj_ctx* c, uint32_t num_attrs, const gj_atom* atoms, uint32_t num_atoms,
                               const uint8_t* order, const gj_less* less, uint32_t num_less, gj_query** out) {
  return gj_query_register_rel(c, num_attrs, atoms, num_atoms, nullptr, 0, order, less, num_less, out);
}

gj_status gj_query_register_rel(gj_ctx* c, uint32_t num_attrs, const gj_atom* atoms, uint32_t num_atoms,
                                const gj_tri_atom* tris, uint32_t num_tris, const uint8_t* order, const gj_less* less,
                                uint32_t num_less, gj_query** out) {
  if (!c || !out) return GJ_EINVAL;
  *out = nullptr;
  gj_query* q = nullptr;
  gj_status s = guarded(c, [&] {
    GJ_CHECK(num_attrs >= 2 && num_attrs <= GJ_MAX_ATTRS, GJ_EINVAL, "num_attrs must be in [2, 8]");
    GJ_CHECK(num_atoms >= 1 && num_atoms + num_tris <= GJ_MAX_ATOMS, GJ_EINVAL,
             "num_atoms must be >= 1 and num_atoms + num_tris at most 16");
    GJ_CHECK(tris || num_tris == 0, GJ_EINVAL, "null ternary atoms");
    GJ_CHECK(atoms && order, GJ_EINVAL, "null atoms or order");
    int m = (int)num_attrs;
    std::vector<int> seen(m, 0), pos(m);
    for (int j = 0; j < m; ++j) {
      GJ_CHECK(order[j] < m && !seen[order[j]], GJ_EINVAL, "order is not a permutation of the attributes");
      seen[order[j]] = 1;
      pos[order[j]] = j;
    }
    for (uint32_t i = 0; i < num_atoms; ++i) {
      GJ_CHECK(atoms[i].src_attr < m && atoms[i].dst_attr < m, GJ_EINVAL, "atom attribute out of range");
      GJ_CHECK(atoms[i].src_attr != atoms[i].dst_attr, GJ_EINVAL, "atom over one attribute twice");
    }
    for (uint32_t i = 0; i < num_tris; ++i) {
      const gj_tri_atom& t = tris[i];
      GJ_CHECK(t.x_attr < m && t.y_attr < m && t.z_attr < m, GJ_EINVAL, "ternary atom attribute out of range");
      GJ_CHECK(t.x_attr != t.y_attr && t.x_attr != t.z_attr && t.y_attr != t.z_attr, GJ_EINVAL,
               "ternary atom over one attribute twice");
      GJ_CHECK(pos[t.z_attr] > pos[t.x_attr] && pos[t.z_attr] > pos[t.y_attr], GJ_EINVAL,
               "a ternary atom's third attribute must come after the other two in the order");
    }
    GJ_CHECK(num_less <= GJ_MAX_LESS, GJ_EINVAL, "more than 28 inequalities");
    GJ_CHECK(less || num_less == 0, GJ_EINVAL, "null inequalities");
    for (uint32_t i = 0; i < num_less; ++i) {
      GJ_CHECK(less[i].lo_attr < m && less[i].hi_attr < m, GJ_EINVAL, "inequality attribute out of range");
      GJ_CHECK(less[i].lo_attr != less[i].hi_attr, GJ_EINVAL, "inequality over one attribute twice");
    }
    for (int j = 1; j < m; ++j) {
      bool any = false;
      for (uint32_t i = 0; i < num_atoms; ++i)
        if (std::max(pos[atoms[i].src_attr], pos[atoms[i].dst_attr]) == j) any = true;
      for (uint32_t i = 0; i < num_tris && j >= 2; ++i)
        if (pos[tris[i].z_attr] == j) any = true;
      GJ_CHECK(any, GJ_EINVAL,
               j == 1 ? "no atom over the first two attributes of the order"
                      : "an attribute has no atom to an earlier attribute of the order");
    }
    q = new gj_query();
    q->m = m;
    q->atoms.assign(atoms, atoms + num_atoms);
    q->order.assign(order, order + m);
    if (num_less) q->less.assign(less, less + num_less);
    if (num_tris) q->tris.assign(tris, tris + num_tris);
    // plan limits are checked here so that run time never fails on them
    gj::PlanHCheck(q);
  });
  if (s != GJ_OK) {
    delete q;
    return s;
  }
  *out = q;
  return GJ_OK;
}

void gj_query_destroy(gj_query* q) { delete q; }

gj_status gj_run(gj_ctx* c, const gj_graph* g, const gj_query* q, int mode, uint64_t seed_lo, uint64_t seed_hi,
                 uint32_t* out, uint64_t out_cap_rows, int out_on_device, gj_stats* stats) {
  if (!c || !g || !q) return GJ_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  gj_stats st{};
  bool overflow = false;
  gj_status s = guarded(c, [&] {
    GJ_CHECK(mode == GJ_MODE_COUNT || mode == GJ_MODE_ENUMERATE, GJ_EINVAL, "mode must be COUNT or ENUMERATE");
    GJ_CHECK(mode == GJ_MODE_COUNT || out || out_cap_rows == 0, GJ_EINVAL, "null output buffer");
    gj::graph_compact(c, const_cast<gj_graph*>(g));  // static runs read plain CSR
    gj::run_static(c, g, q, mode, seed_lo, seed_hi, out, out_cap_rows, out_on_device, &st, overflow);
  });
  st.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  if (s == GJ_OK && overflow) {
    c->err = "output buffer too small";
    return GJ_EOVERFLOW;
  }
  return s;
}

gj_status gj_apply_updates(gj_ctx* c, gj_graph* g, const uint32_t* src, const uint32_t* dst, const int8_t* sign,
                           uint64_t b, int on_device, const gj_query* const* qs, uint32_t nq, int64_t* count_delta,
                           uint32_t* const* delta_rows, int8_t* const* delta_sign, const uint64_t* cap,
                           uint64_t* n_delta, gj_stats* stats) {
  if (!c || !g) return GJ_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  bool overflow = false;
  gj_status s = guarded(c, [&] {
    GJ_CHECK(b == 0 || (src && dst && sign), GJ_EINVAL, "null batch arrays");
    GJ_CHECK(nq == 0 || qs, GJ_EINVAL, "null query list");
    for (uint32_t i = 0; i < nq; ++i) GJ_CHECK(qs[i], GJ_EINVAL, "null query");
    for (uint32_t i = 0; i < nq; ++i)
      GJ_CHECK(qs[i]->tris.empty(), GJ_EUNSUPPORTED, "delta queries with ternary atoms are not supported");
    uint64_t before = g->version;
    gj::apply_updates(c, g, src, dst, sign, b, on_device, qs, nq, count_delta, delta_rows, delta_sign, cap,
                      n_delta, stats, overflow);
    if (g->version != before) gj::tri_index_free(g);  // the relation changed
  });
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    for (uint32_t i = 0; i < nq; ++i) stats[i].ms = ms;
  if (s == GJ_OK && overflow) {
    c->err = "delta output buffer too small";
    return GJ_EOVERFLOW;
  }
  return s;
}

}  // extern "C"

namespace gj {
static void count_fused(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs,
                        const uint64_t* seed_lo, const uint64_t* seed_hi, uint64_t* counts, gj_stats* stats,
                        const Version* ver);

// Counts of nreq requests on version `ver` (null: current): requests of large
// estimated work on the depth-first path, the others in one fused run.
void count_batch(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* seed_lo,
                 const uint64_t* seed_hi, uint64_t* counts, gj_stats* stats, const Version* ver) {
  for (uint32_t i = 0; i < nreq; ++i) GJ_CHECK(qs[i], GJ_EINVAL, "null query");
  for (uint32_t i = 0; i < nreq; ++i)
    GJ_CHECK(qs[i]->tris.empty(), GJ_EUNSUPPORTED, "ternary atoms run only through gj_run");
  if (nreq == 0) return;
  if (c->batch_heavy && nreq > 1) {
    // A request estimated at batch_heavy work or more fills the device alone,
    // and the depth-first kernels serve it faster per candidate than the fused
    // ones: it runs there, the rest stay fused.  Counts and counters are the
    // same either way.
    const Version& v = ver ? *ver : g->ver[g->cur];
    std::vector<PlanH> plans;
    plans.reserve(nreq);
    std::vector<WorkReq> wr;
    std::vector<uint32_t> est_of;
    for (uint32_t i = 0; i < nreq; ++i) {
      plans.push_back(make_plan(qs[i], qs[i]->order, -1));
      uint64_t h = std::min<uint64_t>(seed_hi[i], v.m), l = std::min<uint64_t>(seed_lo[i], h);
      if (h == l) continue;
      wr.push_back(WorkReq{&plans.back(), &v, l, h - l, (uint32_t)std::min<uint64_t>(h - l, 0xffffffffu)});
      est_of.push_back(i);
    }
    std::vector<uint64_t> out, off;
    if (!wr.empty()) seed_work(c, wr, out, off);
    std::vector<char> heavy(nreq, 0);
    uint32_t nh = 0;
    for (size_t k = 0; k < est_of.size(); ++k) {
      uint64_t e = 0;
      for (uint64_t b = off[k]; b < off[k + 1]; ++b) e += out[b];
      if (e >= c->batch_heavy) {
        heavy[est_of[k]] = 1;
        ++nh;
      }
    }
    if (nh) {
      std::vector<const gj_query*> lq;
      std::vector<uint64_t> llo, lhi, lc;
      std::vector<uint32_t> li;
      for (uint32_t i = 0; i < nreq; ++i)
        if (!heavy[i]) {
          li.push_back(i);
          lq.push_back(qs[i]);
          llo.push_back(seed_lo[i]);
          lhi.push_back(seed_hi[i]);
        }
      lc.assign(li.size() + 1, 0);
      std::vector<gj_stats> ls(li.size() + 1);
      if (!li.empty())
        count_fused(c, g, (uint32_t)li.size(), lq.data(), llo.data(), lhi.data(), lc.data(), ls.data(), ver);
      for (size_t k = 0; k < li.size(); ++k) {
        counts[li[k]] = lc[k];
        if (stats) stats[li[k]] = ls[k];
      }
      for (uint32_t i = 0; i < nreq; ++i)
        if (heavy[i]) {
          gj_stats st{};
          bool ov = false;
          run_static(c, g, qs[i], GJ_MODE_COUNT, seed_lo[i], seed_hi[i], nullptr, 0, 1, &st, ov, ver);
          counts[i] = st.matches;
          if (stats) stats[i] = st;
        }
      return;
    }
  }
  hash_note_work(c, g, ver ? *ver : g->ver[g->cur], 0);
  count_fused(c, g, nreq, qs, seed_lo, seed_hi, counts, stats, ver);
  if (stats) {
    uint64_t W = 0;
    for (uint32_t i = 0; i < nreq; ++i)
      for (int j = 3; j <= GJ_MAX_ATTRS; ++j) W += stats[i].extensions[j];
    hash_note_work(c, g, ver ? *ver : g->ver[g->cur], W);
  }
}

// One fused run, or depth-first runs if a level outgrew the batch capacity.
static void count_fused(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs,
                        const uint64_t* seed_lo, const uint64_t* seed_hi, uint64_t* counts, gj_stats* stats,
                        const Version* ver) {
  if (!c->batch) c->batch = new BatchExec();
  bool overflow = false;
  c->batch->run(c, g, nreq, qs, seed_lo, seed_hi, counts, stats, overflow, ver);
  if (overflow) {
    // a level outgrew its capacity: depth-first path, bounded frontiers
    ++c->batch_fallbacks;
    for (uint32_t i = 0; i < nreq; ++i) {
      gj_stats st{};
      bool ov = false;
      run_static(c, g, qs[i], GJ_MODE_COUNT, seed_lo[i], seed_hi[i], nullptr, 0, 1, &st, ov, ver);
      counts[i] = st.matches;
      if (stats) stats[i] = st;
    }
  }
}
gj_status count_on_versions(gj_ctx* c, const gj_graph* g, const Version* const* vers, uint32_t nreq,
                            const gj_query* const* qs, const uint64_t* seed_lo, const uint64_t* seed_hi,
                            uint64_t* counts, gj_stats* stats) {
  return guarded(c, [&] {
    for (uint32_t i = 0; i < nreq; ++i) GJ_CHECK(qs[i] && vers[i], GJ_EINVAL, "null query or version");
    for (uint32_t i = 0; i < nreq; ++i)
      if (i == 0 || vers[i] != vers[i - 1]) hash_note_work(c, g, *vers[i], 0);
    if (nreq == 1) {
      // alone: the depth-first path, no fused-level overhead
      gj_stats st{};
      bool ov = false;
      run_static(c, g, qs[0], GJ_MODE_COUNT, seed_lo[0], seed_hi[0], nullptr, 0, 1, &st, ov, vers[0]);
      counts[0] = st.matches;
      if (stats) stats[0] = st;
      return;
    }
    if (!c->batch) c->batch = new BatchExec();
    std::vector<ReqSpec> specs;
    specs.reserve(nreq);
    for (uint32_t i = 0; i < nreq; ++i) {
      const Version& v = *vers[i];
      ReqSpec r{make_plan(qs[i], qs[i]->order, -1), Views{&v, &v, -1}};
      int dir = r.P.seed_fwd ? 0 : 1;
      uint64_t h = std::min<uint64_t>(seed_hi[i], v.m), l = std::min<uint64_t>(seed_lo[i], h);
      r.row = v.d[dir].row;
      r.col = v.d[dir].col;
      r.lo = l;
      r.len = h - l;
      specs.push_back(std::move(r));
    }
    bool overflow = false;
    c->batch->run_specs(c, specs, counts, nullptr, stats, overflow);
    if (overflow) {
      ++c->batch_fallbacks;
      for (uint32_t i = 0; i < nreq; ++i) {
        gj_stats st{};
        bool ov = false;
        run_static(c, g, qs[i], GJ_MODE_COUNT, seed_lo[i], seed_hi[i], nullptr, 0, 1, &st, ov, vers[i]);
        counts[i] = st.matches;
        if (stats) stats[i] = st;
      }
    }
  });
}

gj_status update_into(gj_ctx* c, gj_graph* g, const uint32_t* src, const uint32_t* dst, const int8_t* sign,
                      uint64_t b, const gj_query* const* qs, uint32_t nq, int64_t* count_delta, int target,
                      const std::vector<gj_ctx*>* lanes) {
  return guarded(c, [&] {
    bool overflow = false;
    apply_updates(c, g, src, dst, sign, b, 0, qs, nq, count_delta, nullptr, nullptr, nullptr, nullptr, nullptr,
                  overflow, target, lanes);
  });
}

gj_status reserve_version(gj_ctx* c, gj_graph* g, int b, uint64_t cap) {
  return guarded(c, [&] {
    GJ_CHECK(b >= 0 && b < kMaxVersions && b != g->cur, GJ_EINVAL, "bad version slot");
    Version& v = g->ver[b];
    version_alloc(c, v, g->n, cap);
    ++v.gen;
    // write the slot once now (a fill kernel), so that whatever the first
    // access to fresh device memory costs is paid here, not by an update
    for (int d = 0; d < 2; ++d) {
      GJ_HIP(hipMemsetAsync(v.d[d].rp, 0, ((uint64_t)g->n + 1) * sizeof(uint32_t), c->stream));
      GJ_HIP(hipMemsetAsync(v.d[d].col, 0, v.cap * sizeof(uint32_t), c->stream));
      GJ_HIP(hipMemsetAsync(v.d[d].row, 0, v.cap * sizeof(uint32_t), c->stream));
    }
    GJ_HIP(hipStreamSynchronize(c->stream));
  });
}

void copy_options(gj_ctx* dst, const gj_ctx* src) {
  dst->frontier_cap = src->frontier_cap;
  dst->seed_chunk = src->seed_chunk;
  dst->strategy = src->strategy;
  dst->batch_lin = src->batch_lin;
  dst->batch_waves_per_cu = src->batch_waves_per_cu;
  dst->batch_claim_words = src->batch_claim_words;
  dst->batch_run = src->batch_run;
  dst->run_big = src->run_big;
  dst->batch_cap = src->batch_cap;
  dst->delta_fused = src->delta_fused;
  dst->delta_owner_min = src->delta_owner_min;
  dst->delta_lane_min = src->delta_lane_min;
  dst->owner_task_min = src->owner_task_min;
  dst->hash_index = src->hash_index;
  dst->hash_min_degree = src->hash_min_degree;
  dst->hash_build_work = src->hash_build_work;
  dst->factorise = src->factorise;
  dst->propose_u = src->propose_u;
  dst->batch_heavy = src->batch_heavy;
  dst->lsm_updates = src->lsm_updates;
  dst->lsm_max_patch = src->lsm_max_patch;
  dst->lsm_fold_min = src->lsm_fold_min;
  dst->run_stage = src->run_stage;
  dst->run_ratio = src->run_ratio;
  dst->run_min_work = src->run_min_work;
  dst->run_task_work = src->run_task_work;
  dst->run_stage_min = src->run_stage_min;
  dst->run_min_tasks = src->run_min_tasks;
  dst->run_reuse = src->run_reuse;
}

gj_status settle(gj_ctx* c, const gj_graph* g) {
  if (!g->lsm.on) return GJ_OK;
  return guarded(c, [&] { graph_compact(c, const_cast<gj_graph*>(g)); });
}

}  // namespace gj

extern "C" {

gj_status gj_run_batch(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs,
                       const uint64_t* seed_lo, const uint64_t* seed_hi, uint64_t* counts, gj_stats* stats) {
  if (!c || !g || (nreq && (!qs || !seed_lo || !seed_hi || !counts))) return GJ_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  return guarded(c, [&] {
    gj::graph_compact(c, const_cast<gj_graph*>(g));
    gj::count_batch(c, g, nreq, qs, seed_lo, seed_hi, counts, stats, nullptr);
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
      for (uint32_t i = 0; i < nreq; ++i) stats[i].ms = ms;
  });
}

gj_status gj_autotune(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs,
                      const uint64_t* seed_lo, const uint64_t* seed_hi, const char* cache_path,
                      gj_tuning* out) {
  if (!c || !g || !nreq || !qs || !seed_lo || !seed_hi) return GJ_EINVAL;
  return guarded(c, [&] {
    gj::graph_compact(c, const_cast<gj_graph*>(g));
    gj::autotune(c, g, nreq, qs, seed_lo, seed_hi, cache_path, out);
  });
}

gj_status gj_last_delta(gj_ctx* c, uint32_t q, uint32_t* rows, int8_t* signs, uint64_t cap, int on_device,
                        uint64_t* n) {
  if (!c || !n) return GJ_EINVAL;
  bool overflow = false;
  gj_status s = guarded(c, [&] {
    GJ_CHECK(q < c->last_delta.size() && c->last_delta[q].kept, GJ_EINVAL,
             "no delta rows kept for this query position");
    const gj_ctx::LastDelta& ld = c->last_delta[q];
    *n = ld.n;
    if (ld.n > cap) {
      overflow = true;
      return;
    }
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (rows && ld.n) GJ_HIP(hipMemcpyAsync(rows, ld.rows, ld.n * ld.m * sizeof(uint32_t), kind, c->stream));
    if (signs && ld.n) GJ_HIP(hipMemcpyAsync(signs, ld.signs, ld.n, kind, c->stream));
    GJ_HIP(hipStreamSynchronize(c->stream));
  });
  if (s == GJ_OK && overflow) {
    c->err = "buffer too small for the kept delta rows";
    return GJ_EOVERFLOW;
  }
  return s;
}

}  // extern "C"
