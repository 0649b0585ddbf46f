// Request server: owns a graph while it lives, keeps its indexes resident,
// and serves count requests and update batches from two threads that overlap
// on the device.
//
// Updates are applied in arrival order on the caller's context (and stream),
// each producing the next version with its count deltas from the fused delta
// queries.  A count request sees exactly the updates that arrived before it
// and none after (logical sequencing as in Sec. 4.3): it is tagged at submit
// time with the number of updates ahead of it, its "state", and runs on an
// internal second context and stream against the resident version that holds
// that state.  The graph keeps two versions (an update reads the current one
// and writes the spare), so counts of the state just before an update run
// concurrently with it; an update only waits while a count still needs the
// state held by the spare it is about to overwrite.
//
// Count requests whose state is resident are admitted in arrival order, up to
// max_batch of them and a frontier-memory budget, all on one version, and run
// as one fused pipeline; requests that arrive meanwhile join the next batch as
// soon as the count stream is free (continuous batching).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "engine.h"
#include "gj_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  int kind = 0;  // GJ_REQ_COUNT or GJ_REQ_UPDATE
  const gj_query* q = nullptr;
  uint64_t lo = 0, hi = 0;
  uint64_t state = 0;  // count: updates submitted before it
  std::vector<uint32_t> src, dst;
  std::vector<int8_t> sign;
  std::vector<const gj_query*> qs;
  int64_t submit_ns = 0;
};

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  double idx = p / 100.0 * (double)(v.size() - 1);
  size_t lo = (size_t)idx;
  size_t hi = std::min(lo + 1, v.size() - 1);
  double f = idx - (double)lo;
  return v[lo] * (1.0 - f) + v[hi] * f;
}

constexpr uint64_t kNone = ~0ull;

}  // namespace

struct gj_server {
  gj_ctx* ctx = nullptr;   // updates: the caller's context
  gj_ctx* cctx = nullptr;  // counts: internal context with its own stream
  gj_graph* g = nullptr;
  uint32_t max_batch = 64;
  uint64_t mem_budget = 0;
  std::mutex mu;
  std::condition_variable cv_count, cv_update, cv_done;
  std::deque<Req> counts, updates;
  std::unordered_map<uint64_t, gj_server_result> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread count_worker, update_worker;
  // version bookkeeping (under mu): state u = the graph after the first u
  // update requests; buffer b of the graph holds states [lo[b], hi[b]]
  uint64_t submitted_updates = 0, applied = 0;
  int cur = 0;
  uint64_t lo[2] = {0, 1}, hi[2] = {0, 0};
  uint64_t version_no[2] = {0, 0};
  uint64_t inflight_state = kNone;  // smallest state of the running count batch
  std::vector<double> lat_count, lat_update;
  uint64_t batches = 0, batched = 0;
};

namespace gj {

// Frontier-memory estimate of a count request: its seeds times the average
// degree once per later attribute (bytes per prefix of each level), the
// admission test of the server.  An underestimate is harmless: a level that
// outgrows the batch capacity reruns on the bounded depth-first path.
static uint64_t estimate_bytes(uint32_t n, uint64_t m, const Req& r) {
  double avg = n ? (double)m / (double)n : 1.0;
  if (avg < 1.0) avg = 1.0;
  uint64_t hi = std::min<uint64_t>(r.hi, m), lo = std::min<uint64_t>(r.lo, hi);
  double prefixes = (double)(hi - lo), total = 0;
  for (int j = 2; j < r.q->m; ++j) {
    total += prefixes * (4.0 * j + 14.0);
    prefixes *= avg;
  }
  return (uint64_t)std::min(total, 1e18);
}

static int buffer_of(const gj_server* s, uint64_t state) {
  for (int b = 0; b < 2; ++b)
    if (s->lo[b] <= state && state <= s->hi[b]) return b;
  return -1;
}

static void finish(gj_server* s, std::vector<Req>& reqs, std::vector<gj_server_result>& out, int64_t start) {
  int64_t done = now_ns();
  for (size_t i = 0; i < reqs.size(); ++i) {
    gj_server_result& res = out[i];
    res.submit_ns = reqs[i].submit_ns;
    res.start_ns = start;
    res.done_ns = done;
    double ms = (double)(done - reqs[i].submit_ns) * 1e-6;
    (res.kind == GJ_REQ_UPDATE ? s->lat_update : s->lat_count).push_back(ms);
    s->results[reqs[i].ticket] = res;
  }
}

static void count_loop(gj_server* s) {
  (void)hipSetDevice(s->cctx->device);
  for (;;) {
    std::vector<Req> batch;
    Version ver;
    uint64_t vno = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_count.wait(lk, [&] {
        return (s->stop && s->counts.empty()) || (!s->counts.empty() && s->counts.front().state <= s->applied);
      });
      if (s->counts.empty()) break;  // stop requested and drained
      int b = buffer_of(s, s->counts.front().state);
      if (b < 0) {
        // unreachable by construction: updates wait for the counts of the
        // state they overwrite; fail the request rather than read freed memory
        Req r = std::move(s->counts.front());
        s->counts.pop_front();
        gj_server_result res;
        memset(&res, 0, sizeof(res));
        res.kind = GJ_REQ_COUNT;
        res.status = GJ_EDEVICE;
        std::vector<Req> one;
        one.push_back(std::move(r));
        std::vector<gj_server_result> out(1, res);
        finish(s, one, out, now_ns());
        lk.unlock();
        s->cv_done.notify_all();
        continue;
      }
      ver = s->g->ver[b];
      vno = s->version_no[b];
      uint64_t est = 0;
      while (!s->counts.empty() && batch.size() < s->max_batch) {
        const Req& r = s->counts.front();
        if (r.state > s->applied || r.state < s->lo[b] || r.state > s->hi[b]) break;
        uint64_t e = estimate_bytes(s->g->n, ver.m, r);
        if (!batch.empty() && s->mem_budget && est + e > s->mem_budget) break;
        est += e;
        batch.push_back(std::move(s->counts.front()));
        s->counts.pop_front();
      }
      s->inflight_state = batch.front().state;
    }
    int64_t start = now_ns();
    std::vector<const gj_query*> qs;
    std::vector<uint64_t> lo, hi, cnt(batch.size());
    for (auto& r : batch) {
      qs.push_back(r.q);
      lo.push_back(r.lo);
      hi.push_back(r.hi);
    }
    gj_status st = count_on_version(s->cctx, s->g, &ver, (uint32_t)batch.size(), qs.data(), lo.data(), hi.data(),
                                    cnt.data());
    std::vector<gj_server_result> out(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
      memset(&out[i], 0, sizeof(gj_server_result));
      out[i].kind = GJ_REQ_COUNT;
      out[i].status = st;
      out[i].count = cnt[i];
      out[i].batch_size = (uint32_t)batch.size();
      out[i].version = vno;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      finish(s, batch, out, start);
      ++s->batches;
      s->batched += batch.size();
      s->inflight_state = kNone;
    }
    s->cv_update.notify_all();
    s->cv_done.notify_all();
  }
}

static void update_loop(gj_server* s) {
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    std::vector<Req> one;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // the spare buffer may be overwritten once no queued or running count
      // needs a state older than the current buffer's
      auto spare_free = [&] {
        uint64_t need = s->inflight_state;
        if (!s->counts.empty()) need = std::min(need, s->counts.front().state);
        return need == kNone || need >= s->lo[s->cur];
      };
      s->cv_update.wait(lk, [&] { return (s->stop && s->updates.empty()) || (!s->updates.empty() && spare_free()); });
      if (s->updates.empty()) break;
      one.push_back(std::move(s->updates.front()));
      s->updates.pop_front();
    }
    Req& r = one[0];
    int64_t start = now_ns();
    std::vector<gj_server_result> out(1);
    gj_server_result& res = out[0];
    memset(&res, 0, sizeof(res));
    res.kind = GJ_REQ_UPDATE;
    res.nq = (uint32_t)r.qs.size();
    int64_t cd[GJ_SERVER_MAX_QUERIES] = {0};
    gj_status st = gj_apply_updates(s->ctx, s->g, r.src.data(), r.dst.data(), r.sign.data(), r.src.size(), 0,
                                    r.qs.data(), (uint32_t)r.qs.size(), cd, nullptr, nullptr, nullptr, nullptr,
                                    nullptr);
    res.status = st;
    for (uint32_t i = 0; i < res.nq; ++i) res.count_delta[i] = cd[i];
    res.batch_size = 1;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      uint64_t u = ++s->applied;
      if (s->g->cur != s->cur) {
        // the update wrote the spare buffer, which now holds state u alone
        s->cur = s->g->cur;
        s->lo[s->cur] = s->hi[s->cur] = u;
        s->version_no[s->cur] = s->g->version;
      } else {
        // nothing changed (all no-ops, or the batch was rejected)
        s->hi[s->cur] = u;
      }
      res.version = s->version_no[s->cur];
      finish(s, one, out, start);
    }
    s->cv_count.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace gj

extern "C" {

gj_status gj_server_create(gj_ctx* ctx, gj_graph* g, uint32_t max_batch, uint64_t mem_budget_bytes,
                           gj_server** out) {
  if (!ctx || !g || !out || max_batch == 0) return GJ_EINVAL;
  gj_server* s = new (std::nothrow) gj_server();
  if (!s) return GJ_ENOMEM;
  s->ctx = ctx;
  s->g = g;
  s->max_batch = max_batch;
  s->mem_budget = mem_budget_bytes;
  gj_status st = gj_ctx_create(ctx->device, nullptr, &s->cctx);
  if (st != GJ_OK) {
    delete s;
    return st;
  }
  gj::copy_options(s->cctx, ctx);
  s->cur = g->cur;
  s->lo[s->cur] = 0;
  s->hi[s->cur] = 0;
  s->lo[1 - s->cur] = 1;  // empty range
  s->hi[1 - s->cur] = 0;
  s->version_no[s->cur] = g->version;
  try {
    s->count_worker = std::thread(gj::count_loop, s);
    s->update_worker = std::thread(gj::update_loop, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_count.notify_all();
    s->cv_update.notify_all();
    if (s->count_worker.joinable()) s->count_worker.join();
    gj_ctx_destroy(s->cctx);
    delete s;
    return GJ_ENOMEM;
  }
  *out = s;
  return GJ_OK;
}

static gj_status enqueue_req(gj_server* s, Req&& r, uint64_t* ticket) {
  bool update = r.kind == GJ_REQ_UPDATE;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return GJ_EBUSY;
    r.ticket = s->next_ticket++;
    r.submit_ns = now_ns();
    *ticket = r.ticket;
    if (update) {
      ++s->submitted_updates;
      s->updates.push_back(std::move(r));
    } else {
      r.state = s->submitted_updates;
      s->counts.push_back(std::move(r));
    }
  }
  (update ? s->cv_update : s->cv_count).notify_one();
  return GJ_OK;
}

gj_status gj_server_submit_count(gj_server* s, const gj_query* q, uint64_t seed_lo, uint64_t seed_hi,
                                 uint64_t* ticket) {
  if (!s || !q || !ticket) return GJ_EINVAL;
  Req r;
  r.kind = GJ_REQ_COUNT;
  r.q = q;
  r.lo = seed_lo;
  r.hi = seed_hi;
  return enqueue_req(s, std::move(r), ticket);
}

gj_status gj_server_submit_update(gj_server* s, const uint32_t* src, const uint32_t* dst, const int8_t* sign,
                                  uint64_t b, const gj_query* const* qs, uint32_t nq, uint64_t* ticket) {
  if (!s || !ticket || (b && (!src || !dst || !sign)) || nq > GJ_SERVER_MAX_QUERIES || (nq && !qs))
    return GJ_EINVAL;
  Req r;
  r.kind = GJ_REQ_UPDATE;
  r.src.assign(src, src + b);
  r.dst.assign(dst, dst + b);
  r.sign.assign(sign, sign + b);
  r.qs.assign(qs, qs + nq);
  return enqueue_req(s, std::move(r), ticket);
}

gj_status gj_server_wait(gj_server* s, uint64_t ticket, int64_t timeout_ms, gj_server_result* out) {
  if (!s || !out) return GJ_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return GJ_EINVAL;
  auto ready = [&] { return s->results.count(ticket) != 0; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return GJ_EBUSY;
  }
  *out = s->results[ticket];
  s->results.erase(ticket);
  return GJ_OK;
}

gj_status gj_server_get_stats(gj_server* s, gj_server_stats* out) {
  if (!s || !out) return GJ_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof(*out));
  out->completed_counts = s->lat_count.size();
  out->completed_updates = s->lat_update.size();
  out->count_batches = s->batches;
  out->mean_count_batch = s->batches ? (double)s->batched / (double)s->batches : 0.0;
  out->count_p50_ms = percentile(s->lat_count, 50);
  out->count_p99_ms = percentile(s->lat_count, 99);
  out->update_p50_ms = percentile(s->lat_update, 50);
  out->update_p99_ms = percentile(s->lat_update, 99);
  return GJ_OK;
}

void gj_server_destroy(gj_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_count.notify_all();
  s->cv_update.notify_all();
  if (s->count_worker.joinable()) s->count_worker.join();
  if (s->update_worker.joinable()) s->update_worker.join();
  gj_ctx_destroy(s->cctx);
  delete s;
}

}  // extern "C"
