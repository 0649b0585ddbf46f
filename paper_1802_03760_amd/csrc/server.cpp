// Request server: one worker thread owns a context and a graph, keeps the
// indexes resident, and serves count requests and update batches.
//
// Updates are applied in arrival order, each as one new version (its count
// deltas from the fused delta queries).  Count requests see the version that
// is current when they reach the head of the queue, i.e. every update that
// arrived before them and none that arrived after (logical sequencing as in
// Sec. 4.3).  Count requests waiting at the head are admitted together, up
// to max_batch of them and a frontier-memory budget, and run as one fused
// pipeline; requests that arrive meanwhile join the next batch as soon as the
// device is free (continuous batching).
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

}  // namespace

struct gj_server {
  gj_ctx* ctx = nullptr;
  gj_graph* g = nullptr;
  uint32_t max_batch = 64;
  uint64_t mem_budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> queue;
  std::unordered_map<uint64_t, gj_server_result> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::vector<double> lat_count, lat_update;
  uint64_t batches = 0, batched = 0, fallbacks = 0;
};

namespace gj {

// Frontier-memory estimate of a count request: its seeds times the average
// degree once per later attribute (bytes per prefix of each level), the
// admission test of the server.  An underestimate is harmless: a level that
// outgrows the batch capacity reruns on the bounded depth-first path.
static uint64_t estimate_bytes(const gj_graph* g, const Req& r) {
  const Version& v = g->ver[g->cur];
  double avg = g->n ? (double)v.m / (double)g->n : 1.0;
  if (avg < 1.0) avg = 1.0;
  uint64_t hi = std::min<uint64_t>(r.hi, v.m), lo = std::min<uint64_t>(r.lo, hi);
  double prefixes = (double)(hi - lo), total = 0;
  for (int j = 2; j < r.q->m; ++j) {
    total += prefixes * (4.0 * j + 14.0);
    prefixes *= avg;
  }
  return (uint64_t)std::min(total, 1e18);
}

static void serve_loop(gj_server* s) {
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    std::vector<Req> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) break;  // stop requested and drained
      if (s->queue.front().kind == GJ_REQ_UPDATE) {
        batch.push_back(std::move(s->queue.front()));
        s->queue.pop_front();
      } else {
        uint64_t est = 0;
        while (!s->queue.empty() && s->queue.front().kind == GJ_REQ_COUNT && batch.size() < s->max_batch) {
          uint64_t e = estimate_bytes(s->g, s->queue.front());
          if (!batch.empty() && s->mem_budget && est + e > s->mem_budget) break;
          est += e;
          batch.push_back(std::move(s->queue.front()));
          s->queue.pop_front();
        }
      }
    }
    int64_t start = now_ns();
    std::vector<gj_server_result> out(batch.size());
    if (batch[0].kind == GJ_REQ_UPDATE) {
      Req& r = batch[0];
      gj_server_result& res = out[0];
      memset(&res, 0, sizeof(res));
      res.kind = GJ_REQ_UPDATE;
      res.nq = (uint32_t)r.qs.size();
      int64_t cd[GJ_SERVER_MAX_QUERIES] = {0};
      gj_status st = gj_apply_updates(s->ctx, s->g, r.src.data(), r.dst.data(), r.sign.data(), r.src.size(), 0,
                                      r.qs.data(), (uint32_t)r.qs.size(), cd, nullptr, nullptr, nullptr,
                                      nullptr, nullptr);
      res.status = st;
      for (uint32_t i = 0; i < res.nq; ++i) res.count_delta[i] = cd[i];
      res.batch_size = 1;
    } else {
      std::vector<const gj_query*> qs;
      std::vector<uint64_t> lo, hi, cnt(batch.size());
      for (auto& r : batch) {
        qs.push_back(r.q);
        lo.push_back(r.lo);
        hi.push_back(r.hi);
      }
      gj_status st;
      if (batch.size() == 1) {
        // alone in the queue: the depth-first path, no fused-level overhead
        gj_stats one{};
        st = gj_run(s->ctx, s->g, qs[0], GJ_MODE_COUNT, lo[0], hi[0], nullptr, 0, 0, &one);
        cnt[0] = one.matches;
      } else {
        st = gj_run_batch(s->ctx, s->g, (uint32_t)batch.size(), qs.data(), lo.data(), hi.data(), cnt.data(),
                          nullptr);
      }
      for (size_t i = 0; i < batch.size(); ++i) {
        memset(&out[i], 0, sizeof(gj_server_result));
        out[i].kind = GJ_REQ_COUNT;
        out[i].status = st;
        out[i].count = cnt[i];
        out[i].batch_size = (uint32_t)batch.size();
      }
    }
    int64_t done = now_ns();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (size_t i = 0; i < batch.size(); ++i) {
        gj_server_result& res = out[i];
        res.version = s->g->version;
        res.submit_ns = batch[i].submit_ns;
        res.start_ns = start;
        res.done_ns = done;
        double ms = (double)(done - batch[i].submit_ns) * 1e-6;
        (res.kind == GJ_REQ_UPDATE ? s->lat_update : s->lat_count).push_back(ms);
        s->results[batch[i].ticket] = res;
      }
      if (batch[0].kind == GJ_REQ_COUNT) {
        ++s->batches;
        s->batched += batch.size();
      }
    }
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
  s->worker = std::thread(gj::serve_loop, s);
  *out = s;
  return GJ_OK;
}

static gj_status enqueue_req(gj_server* s, Req&& r, uint64_t* ticket) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return GJ_EBUSY;
    r.ticket = s->next_ticket++;
    r.submit_ns = now_ns();
    *ticket = r.ticket;
    s->queue.push_back(std::move(r));
  }
  s->cv_work.notify_one();
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
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  delete s;
}

}  // extern "C"
