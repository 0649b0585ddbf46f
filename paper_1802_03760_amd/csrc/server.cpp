// Request server: owns a graph while it lives, keeps its indexes resident,
// and serves count requests and update batches from two threads that overlap
// on the device.
//
// Versions.  Updates are applied in arrival order on the caller's context
// (and stream), each producing the next version with its count deltas from
// the fused delta queries.  A count request sees exactly the updates that
// arrived before it and none after (logical sequencing as in Sec. 4.3): it
// is tagged at submit time with the number of updates ahead of it, its
// "state", and reads the resident version slot that holds that state.  The
// graph keeps up to kMaxVersions slots; an update writes a slot that no
// queued or running count needs, so counts of older states keep running while
// updates proceed, and an update waits only when every other slot is needed.
//
// Counts (continuous batching).  A request joins at the first iteration
// after its state is resident; its remaining work is estimated from its seeds
// (seed-work estimates, rescaled by the work its finished chunks did).  Light
// requests (at most an eighth of the per-iteration budget) run whole,
// shortest first, together in one fused pipeline per iteration on an internal
// context and stream.  Heavy requests are cut into chunks of about
// heavy_work estimated work that run on the depth-first path on a few more
// contexts and streams ("lanes"), each lane taking the oldest heavy request no
// other lane is running; so light requests never wait behind heavy ones and
// a heavy request can pass a heavier one.  Requests whose version slot an
// update waits for go first.  While an update batch is on the device no new
// heavy chunk starts (update priority); light iterations go on.  With a
// budget of zero, requests run whole, in arrival order, up to max_batch per
// iteration.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "engine.h"
#include "gj_internal.h"
#include "sched.h"

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

constexpr uint32_t kEstBlocks = 1024;  // estimate blocks per request

// A count request admitted to the scheduler (owned by the count thread).
struct Active {
  Req r;
  int slot = -1;             // version slot holding its state
  gj::PlanH plan;
  uint64_t lo = 0, hi = 0;   // seed slice, clamped to the version's edges
  uint64_t next = 0;         // first seed not yet run (block aligned)
  uint32_t bs = 1;           // seeds per estimate block
  std::vector<uint64_t> cum; // cum[i] = estimated work of the first i blocks
  double est_done = 0, work_done = 0;
  uint64_t count = 0;
  int64_t start_ns = 0;
  gj_status status = GJ_OK;
  int inflight = 0;          // chunks of it heavy lanes are running

  uint64_t nblocks() const { return cum.empty() ? 0 : cum.size() - 1; }
  uint64_t block_of(uint64_t seed) const { return (seed - lo) / bs; }
  double ratio() const { return est_done > 0 ? std::max(work_done / est_done, 1e-3) : 1.0; }
  double remaining() const {
    if (next >= hi) return 0;
    return (double)(cum[nblocks()] - cum[block_of(next)]) * ratio();
  }
};

}  // namespace

struct gj_server {
  gj_ctx* ctx = nullptr;   // updates: the caller's context
  gj_ctx* cctx = nullptr;  // light counts: internal context with its own stream
  std::vector<gj_ctx*> hctx;  // heavy lanes: one context and stream each
  std::vector<gj_ctx*> uctx;  // delta lanes of the update thread: one context and stream each
  gj_graph* g = nullptr;
  uint32_t max_batch = 64;
  uint64_t mem_budget = 0;
  uint64_t iter_work = 1ull << 24;  // estimated work per light iteration (0: whole requests)
  int nslots = 4;                   // version slots the server may use
  bool started = false;             // a request was submitted
  std::mutex mu;
  std::condition_variable cv_count, cv_heavy, cv_update, cv_done;
  std::deque<Req> counts, updates;
  std::unordered_map<uint64_t, gj_server_result> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread count_worker, update_worker;
  std::vector<std::thread> heavy_workers;
  std::vector<std::unique_ptr<Active>> heavy;  // heavy requests, arrival order (under mu)
  bool light_done = false;                     // the light thread has exited
  bool light_warm = false;                     // the light lane's fused pipeline is built
  int heavy_lanes = 3;                         // heavy requests run concurrently
  int update_lanes = 2;                        // contexts beside ctx that run an update's dQ_i
  uint64_t heavy_work = 0;                     // estimated work per heavy chunk (0: 64 x iter_work)
  // version bookkeeping (under mu): state u = the graph after the first u
  // update requests; slot b holds states [lo[b], hi[b]] (empty if lo > hi)
  uint64_t submitted_updates = 0, applied = 0;
  int cur = 0;
  uint64_t lo[kMaxVersions] = {}, hi[kMaxVersions] = {};
  uint64_t version_no[kMaxVersions] = {};
  std::map<uint64_t, uint32_t> pending;  // states of queued and admitted counts
  int want = -1;                          // slot an update waits for
  bool updating = false;                  // an update batch is on the device
  bool update_priority = true;            // no new heavy chunk meanwhile
  std::vector<double> lat_count, lat_update;
  uint64_t batches = 0, batched = 0;
};

namespace gj {

// Frontier-memory estimate of a chunk: its seeds times the average degree
// once per later attribute (bytes per prefix of each level), the admission
// test of the server.  An underestimate is harmless: a level that outgrows
// the batch capacity reruns on the bounded depth-first path.
static uint64_t estimate_bytes(uint32_t n, uint64_t m, int qm, uint64_t seeds) {
  double avg = n ? (double)m / (double)n : 1.0;
  if (avg < 1.0) avg = 1.0;
  double prefixes = (double)seeds, total = 0;
  for (int j = 2; j < qm; ++j) {
    total += prefixes * (4.0 * j + 14.0);
    prefixes *= avg;
  }
  return (uint64_t)std::min(total, 1e18);
}

static int slot_of(const gj_server* s, uint64_t state) {
  for (int b = 0; b < kMaxVersions; ++b)
    if (s->lo[b] <= state && state <= s->hi[b]) return b;
  return -1;
}

static bool needed(const gj_server* s, int b) {
  if (s->lo[b] > s->hi[b]) return false;
  auto it = s->pending.lower_bound(s->lo[b]);
  return it != s->pending.end() && it->first <= s->hi[b];
}

// Slot for the next update: not current, needed by no count; an allocated
// slot first (empty, else the oldest), a new one otherwise.  -1: none free.
static int pick_target(const gj_server* s) {
  int best = -1;
  uint64_t best_key = ~0ull;
  for (int b = 0; b < s->nslots; ++b) {
    if (b == s->cur || needed(s, b)) continue;
    bool alloc = s->g->ver[b].cap > 0;
    bool empty = s->lo[b] > s->hi[b];
    uint64_t key = alloc ? (empty ? 0 : 1 + s->hi[b]) : ~0ull - 1;
    if (key < best_key) {
      best_key = key;
      best = b;
    }
  }
  return best;
}

// The needed slot with the oldest states (what a waiting update needs freed).
static int oldest_needed(const gj_server* s) {
  int best = -1;
  for (int b = 0; b < s->nslots; ++b)
    if (b != s->cur && needed(s, b) && (best < 0 || s->hi[b] < s->hi[best])) best = b;
  return best;
}

static void release(gj_server* s, uint64_t state) {
  auto it = s->pending.find(state);
  if (it != s->pending.end() && --it->second == 0) s->pending.erase(it);
}

// Records a finished request (under mu).
static void record(gj_server* s, const Req& r, gj_server_result& res) {
  res.submit_ns = r.submit_ns;
  double ms = (double)(res.done_ns - r.submit_ns) * 1e-6;
  (res.kind == GJ_REQ_UPDATE ? s->lat_update : s->lat_count).push_back(ms);
  s->results[r.ticket] = res;
}

static gj_server_result count_result(const Active& a, uint64_t version, uint32_t batch, int64_t done) {
  gj_server_result res;
  memset(&res, 0, sizeof(res));
  res.kind = GJ_REQ_COUNT;
  res.status = a.status;
  res.count = a.count;
  res.version = version;
  res.batch_size = batch;
  res.start_ns = a.start_ns ? a.start_ns : done;
  res.done_ns = done;
  return res;
}

// Seed slices, plans and (with a work budget) seed-work estimates of newly
// admitted requests.
static void prepare(gj_server* s, std::vector<Active*>& fresh, const Version* vers, uint64_t iter_work) {
  std::vector<WorkReq> wr;
  std::vector<Active*> est;
  for (Active* a : fresh) {
    if (a->slot < 0) {
      a->status = GJ_EDEVICE;  // unreachable: the slot of a pending state is kept
      a->next = a->hi = a->lo = 0;
      continue;
    }
    const Version& v = vers[a->slot];
    a->hi = std::min<uint64_t>(a->r.hi, v.m);
    a->lo = std::min<uint64_t>(a->r.lo, a->hi);
    a->next = a->lo;
    uint64_t len = a->hi - a->lo;
    try {
      a->plan = make_plan(a->r.q, a->r.q->order, -1);
    } catch (const Error& e) {
      a->status = e.code;
      a->next = a->hi;
      continue;
    }
    if (!iter_work || !len) {
      a->bs = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(len, 0xffffffffu));
      a->cum = {0, len};
      continue;
    }
    a->bs = (uint32_t)((len + kEstBlocks - 1) / kEstBlocks);
    wr.push_back(WorkReq{&a->plan, &v, a->lo, len, a->bs});
    est.push_back(a);
  }
  if (est.empty()) return;
  std::vector<uint64_t> out, off;
  gj_status st = GJ_OK;
  try {
    seed_work(s->cctx, wr, out, off);
  } catch (const Error& e) {
    st = e.code;
  } catch (...) {
    st = GJ_EDEVICE;
  }
  for (size_t i = 0; i < est.size(); ++i) {
    Active* a = est[i];
    if (st != GJ_OK) {
      // no estimates: run the request whole
      a->bs = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(a->hi - a->lo, 0xffffffffu));
      a->cum = {0, a->hi - a->lo};
      continue;
    }
    a->cum.assign(off[i + 1] - off[i] + 1, 0);
    for (uint64_t k = off[i]; k < off[i + 1]; ++k) a->cum[k - off[i] + 1] = a->cum[k - off[i]] + out[k];
  }
}

struct Chunk {
  Active* a;
  uint64_t b0, b1;  // estimate blocks [b0, b1)
  uint64_t lo, hi;  // seeds
};

// Next chunk of a: whole blocks while the rescaled estimate stays within
// allow (at least one block).
static Chunk take(Active* a, double allow, double& used) {
  uint64_t nb = a->nblocks(), b0 = a->block_of(a->next), b1 = b0 + 1;
  double r = a->ratio();
  while (b1 < nb && (double)(a->cum[b1 + 1] - a->cum[b0]) * r <= allow) ++b1;
  used = (double)(a->cum[b1] - a->cum[b0]) * r;
  uint64_t hi = std::min<uint64_t>(a->lo + b1 * (uint64_t)a->bs, a->hi);
  return Chunk{a, b0, b1, a->next, hi};
}

// Runs chunks on context c (one alone: depth-first; more: one fused
// pipeline) and advances their requests.
static void run_chunks(gj_server* s, gj_ctx* c, std::vector<Chunk>& cs, const Version* vers) {
  uint32_t n = (uint32_t)cs.size();
  if (!n) return;
  std::vector<const gj_query*> qs(n);
  std::vector<const Version*> cv(n);
  std::vector<uint64_t> lo(n), hi(n), cnt(n, 0);
  std::vector<gj_stats> st(n);
  int64_t t_run = now_ns();
  for (uint32_t i = 0; i < n; ++i) {
    qs[i] = cs[i].a->r.q;
    cv[i] = &vers[cs[i].a->slot];
    lo[i] = cs[i].lo;
    hi[i] = cs[i].hi;
    if (!cs[i].a->start_ns) cs[i].a->start_ns = t_run;
  }
  gj_status status = count_on_versions(c, s->g, cv.data(), n, qs.data(), lo.data(), hi.data(), cnt.data(), st.data());
  for (uint32_t i = 0; i < n; ++i) {
    Active* a = cs[i].a;
    if (status != GJ_OK) {
      a->status = status;
      a->next = a->hi;
      continue;
    }
    a->count += cnt[i];
    double work = (double)st[i].prefixes[2];
    for (int j = 0; j <= GJ_MAX_ATTRS; ++j) work += (double)st[i].extensions[j];
    a->est_done += (double)(a->cum[cs[i].b1] - a->cum[cs[i].b0]);
    a->work_done += work;
    a->next = cs[i].hi;
  }
}

// Records the finished requests of `list` (under mu) and drops them.
static void retire(gj_server* s, std::vector<std::unique_ptr<Active>>& list, const uint64_t* vno, uint32_t nc) {
  int64_t done = now_ns();
  for (auto& a : list) {
    if (a->next < a->hi) continue;
    gj_server_result res = count_result(*a, a->slot >= 0 ? vno[a->slot] : 0, nc, done);
    record(s, a->r, res);
    release(s, a->r.state);
  }
  if (nc) {
    ++s->batches;
    s->batched += nc;
  }
  list.erase(std::remove_if(list.begin(), list.end(),
                            [](const std::unique_ptr<Active>& a) { return a->next >= a->hi; }),
             list.end());
}

// Snapshot (under mu) of the version slots that requests of `list` read:
// slots of pending states, which no update writes meanwhile.
static void snapshot(const gj_server* s, const std::vector<std::unique_ptr<Active>>& list, Version* vers,
                     uint64_t* vno) {
  bool used[kMaxVersions] = {};
  for (auto& a : list)
    if (a->slot >= 0) used[a->slot] = true;
  for (int b = 0; b < kMaxVersions; ++b) {
    if (used[b]) vers[b] = s->g->ver[b];
    vno[b] = s->version_no[b];
  }
}

// Light thread: admission, estimates, and the fused iterations of light
// requests; heavy requests go to the heavy thread.
// Builds the light lane's fused pipeline before any request: a batch of two
// empty 4-clique slices allocates and captures it (level arrays, run
// buffers), so that the first light iteration does not pay for device
// allocations of several GB while the other lanes run.  Larger queries
// rebuild it later.  Best effort: a failure leaves the build to the first
// iteration.
// Builds c's fused pipeline for queries of up to m attributes (3 or 4) with
// a batch of two empty slices.
static void warm_pipeline(gj_server* s, gj_ctx* c, uint32_t m) {
  const gj_atom atoms[6] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}, {2, 3}};
  const uint8_t order[4] = {0, 1, 2, 3};
  gj_query* q = nullptr;
  if (gj_query_register(c, m, atoms, m == 3 ? 3 : 6, order, &q) == GJ_OK) {
    Version v = s->g->ver[s->cur];
    const Version* vs[2] = {&v, &v};
    const gj_query* qs[2] = {q, q};
    uint64_t lo[2] = {0, 0}, hi[2] = {0, 0}, cnt[2] = {0, 0};
    gj_stats st[2];
    (void)count_on_versions(c, s->g, vs, 2, qs, lo, hi, cnt, st);
    (void)hipStreamSynchronize(c->stream);
    gj_query_destroy(q);
  }
}

static void warm_light(gj_server* s) {
  warm_pipeline(s, s->cctx, 4);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->light_warm = true;
  }
  s->cv_update.notify_all();
}

static void count_loop(gj_server* s) {
  (void)hipSetDevice(s->cctx->device);
  warm_light(s);
  std::vector<std::unique_ptr<Active>> active;  // arrival order
  Version vers[kMaxVersions];
  for (;;) {
    std::vector<Active*> fresh;
    uint64_t vno[kMaxVersions] = {};
    int want;
    uint64_t iter_work;
    uint32_t max_batch;
    uint64_t mem_budget;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // (light iterations keep running while an update is on the device:
      // they are short, and holding them would put every count behind
      // every update)
      s->cv_count.wait(lk, [&] {
        return !active.empty() || (s->stop && s->counts.empty()) ||
               (!s->counts.empty() && s->counts.front().state <= s->applied);
      });
      if (active.empty() && s->counts.empty()) break;  // stop requested and drained
      while (!s->counts.empty() && s->counts.front().state <= s->applied) {
        std::unique_ptr<Active> a(new Active());
        a->r = std::move(s->counts.front());
        s->counts.pop_front();
        a->slot = slot_of(s, a->r.state);
        fresh.push_back(a.get());
        active.push_back(std::move(a));
      }
      snapshot(s, active, vers, vno);
      want = s->want;
      iter_work = s->iter_work;
      max_batch = s->max_batch;
      mem_budget = s->mem_budget;
    }
    prepare(s, fresh, vers, iter_work);
    const double W = (double)iter_work;
    std::vector<std::unique_ptr<Active>> heavy;
    if (iter_work) {
      // newly estimated requests above an eighth of the budget are heavy
      for (auto& a : active)
        if (a->next == a->lo && a->next < a->hi && a->remaining() > W / 8) heavy.push_back(std::move(a));
      active.erase(std::remove(active.begin(), active.end(), nullptr), active.end());
    }
    // light requests whole: shortest first (the ones an update waits for
    // first), within the budget, max_batch and the memory budget
    std::vector<Active*> light;
    for (auto& a : active)
      if (a->next < a->hi) light.push_back(a.get());
    if (iter_work) {
      std::stable_sort(light.begin(), light.end(),
                       [](const Active* x, const Active* y) { return x->remaining() < y->remaining(); });
      if (want >= 0)
        std::stable_partition(light.begin(), light.end(), [&](const Active* a) { return a->slot == want; });
    }
    std::vector<Chunk> chunks;
    uint64_t mem = 0;
    double left = iter_work ? W : 1e300;
    for (Active* a : light) {
      if (chunks.size() >= max_batch || (left <= 0 && !chunks.empty())) break;
      Chunk c{a, a->block_of(a->next), a->nblocks(), a->next, a->hi};
      uint64_t e = estimate_bytes(s->g->n, vers[a->slot].m, a->plan.m, c.hi - c.lo);
      if (!chunks.empty() && mem_budget && mem + e > mem_budget) break;
      mem += e;
      chunks.push_back(c);
      left -= a->remaining();
    }
    run_chunks(s, s->cctx, chunks, vers);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      retire(s, active, vno, (uint32_t)chunks.size());
      for (auto& h : heavy) s->heavy.push_back(std::move(h));
    }
    if (!heavy.empty()) s->cv_heavy.notify_all();
    s->cv_update.notify_all();
    s->cv_done.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->light_done = true;
  }
  s->cv_heavy.notify_all();
}

// Heavy lane `lane`: claims the next chunk of about heavy_work estimated
// work of the oldest heavy request with seeds left (one whose version slot an
// update waits for first) and runs it on the depth-first path.  Every free
// lane claims chunks of that request until all its seeds are claimed, so the
// oldest heavy request is served by all lanes at once (the stalls of one
// lane's host-driven stages are filled by the others'); lanes run
// concurrently with each other and with the light iterations.  Counts and
// work are added under the lock; the request finishes when its last chunk
// returns.
static void heavy_loop(gj_server* s, int lane) {
  gj_ctx* c = s->hctx[lane];
  (void)hipSetDevice(c->device);
  Version vers[kMaxVersions];
  for (;;) {
    uint64_t vno[kMaxVersions] = {};
    Active* pick = nullptr;
    Chunk ch{};
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_heavy.wait(lk, [&] {
        if (s->updating && s->update_priority) return false;  // updates first
        pick = nullptr;
        for (auto& a : s->heavy) {
          if (a->next >= a->hi) continue;  // every seed claimed
          if (!pick) pick = a.get();
          if (a->slot == s->want) {
            pick = a.get();
            break;
          }
        }
        return pick != nullptr || (s->light_done && s->heavy.empty());
      });
      if (!pick) break;  // the light thread has exited and every heavy request is done
      double W = (double)(s->heavy_work ? s->heavy_work : 64 * std::max<uint64_t>(s->iter_work, 1));
      double used = 0;
      ch = take(pick, W, used);
      pick->next = ch.hi;  // claimed
      ++pick->inflight;
      if (!pick->start_ns) pick->start_ns = now_ns();
      vers[pick->slot] = s->g->ver[pick->slot];
      for (int b = 0; b < kMaxVersions; ++b) vno[b] = s->version_no[b];
    }
    const gj_query* q = pick->r.q;
    const Version* cv = &vers[pick->slot];
    uint64_t cnt = 0;
    gj_stats st{};
    gj_status status = count_on_versions(c, s->g, &cv, 1, &q, &ch.lo, &ch.hi, &cnt, &st);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      --pick->inflight;
      if (status != GJ_OK) {
        pick->status = status;
        pick->next = pick->hi;
      } else {
        pick->count += cnt;
        double work = (double)st.prefixes[2];
        for (int j = 0; j <= GJ_MAX_ATTRS; ++j) work += (double)st.extensions[j];
        pick->est_done += (double)(pick->cum[ch.b1] - pick->cum[ch.b0]);
        pick->work_done += work;
      }
      if (pick->next >= pick->hi && pick->inflight == 0) {
        gj_server_result res = count_result(*pick, vno[pick->slot], 1, now_ns());
        record(s, pick->r, res);
        release(s, pick->r.state);
        s->heavy.erase(std::remove_if(s->heavy.begin(), s->heavy.end(),
                                      [&](const std::unique_ptr<Active>& a) { return a.get() == pick; }),
                       s->heavy.end());
      }
      ++s->batches;
      ++s->batched;
    }
    s->cv_heavy.notify_all();
    s->cv_update.notify_all();
    s->cv_done.notify_all();
  }
}

static void update_loop(gj_server* s) {
  (void)hipSetDevice(s->ctx->device);
  // Once the first request fixes the number of slots, allocate the spare
  // slots up front (sized like the current version plus growth room) so that
  // no update pays for their allocation.
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // the light lane's pipeline is built before the first update is served,
    // so a caller that waits for an update has the server warm
    s->cv_update.wait(lk, [&] { return (s->started && s->light_warm) || s->stop; });
  }
  // the fused pipeline of the count-only delta queries, likewise, before the
  // first update needs it (without the run kernels, which signed delta
  // seeds never take)
  if (s->ctx->delta_fused) {
    const int br = s->ctx->batch_run;
    s->ctx->batch_run = 0;
    warm_pipeline(s, s->ctx, 3);
    s->ctx->batch_run = br;
  }
  {
    const Version& cv = s->g->ver[s->g->cur];
    uint64_t cap = cv.m + cv.m / 16 + (1ull << 20);
    for (int b = 0; b < s->nslots; ++b)
      if (b != s->g->cur && s->g->ver[b].cap == 0) (void)reserve_version(s->ctx, s->g, b, cap);
  }
  for (;;) {
    Req r;
    int target = -1;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_update.wait(lk, [&] {
        if (s->updates.empty()) return s->stop;
        target = pick_target(s);
        s->want = target < 0 ? oldest_needed(s) : -1;
        return target >= 0;
      });
      if (s->updates.empty()) break;
      r = std::move(s->updates.front());
      s->updates.pop_front();
      s->updating = true;
    }
    int64_t start = now_ns();
    gj_server_result res;
    memset(&res, 0, sizeof(res));
    res.kind = GJ_REQ_UPDATE;
    res.nq = (uint32_t)r.qs.size();
    int64_t cd[GJ_SERVER_MAX_QUERIES] = {0};
    res.status = update_into(s->ctx, s->g, r.src.data(), r.dst.data(), r.sign.data(), r.src.size(), r.qs.data(),
                             (uint32_t)r.qs.size(), cd, target, &s->uctx);
    for (uint32_t i = 0; i < res.nq; ++i) res.count_delta[i] = cd[i];
    res.batch_size = 1;
    res.start_ns = start;
    res.done_ns = now_ns();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->updating = false;
      uint64_t u = ++s->applied;
      if (s->g->cur == target) {
        // the update wrote the target slot, which now holds state u alone
        s->cur = target;
        s->lo[target] = s->hi[target] = u;
        s->version_no[target] = s->g->version;
      } else {
        // nothing changed (all no-ops, or the batch was rejected); the target
        // slot held no state anyone needs
        s->hi[s->cur] = u;
        s->lo[target] = 1;
        s->hi[target] = 0;
      }
      res.version = s->version_no[s->cur];
      record(s, r, res);
    }
    s->cv_count.notify_all();
    s->cv_heavy.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace gj

// Serves everything queued, stops the threads, frees the contexts and s.
static void shutdown(gj_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_count.notify_all();
  s->cv_heavy.notify_all();
  s->cv_update.notify_all();
  if (s->count_worker.joinable()) s->count_worker.join();
  for (auto& t : s->heavy_workers)
    if (t.joinable()) t.join();
  if (s->update_worker.joinable()) s->update_worker.join();
  gj_ctx_destroy(s->cctx);
  for (gj_ctx* c : s->hctx) gj_ctx_destroy(c);
  for (gj_ctx* c : s->uctx) gj_ctx_destroy(c);
  delete s;
}

extern "C" {

gj_status gj_server_create(gj_ctx* ctx, gj_graph* g, uint32_t max_batch, uint64_t mem_budget_bytes,
                           gj_server** out) {
  if (!ctx || !g || !out || max_batch == 0) return GJ_EINVAL;
  if (g->lsm.on) {
    // the server rotates plain version slots: merge rows appended by
    // log-structured updates first
    gj_status cs = gj::settle(ctx, g);
    if (cs != GJ_OK) return cs;
  }
  gj_server* s = new (std::nothrow) gj_server();
  if (!s) return GJ_ENOMEM;
  s->ctx = ctx;
  s->g = g;
  s->max_batch = max_batch;
  s->mem_budget = mem_budget_bytes;
  gj_status st = gj_ctx_create(ctx->device, nullptr, ctx->alloc.alloc ? &ctx->alloc : nullptr, &s->cctx);
  if (st != GJ_OK) {
    delete s;
    return st;
  }
  gj::copy_options(s->cctx, ctx);
  s->cctx->hash_build = ctx->hash_index >= 2;  // the server reads indexes built elsewhere unless asked
  // The light lane's fused iterations stage runs in the small shape only: a
  // large-shape workgroup needs a whole CU's LDS, which the heavy lanes'
  // kernels rarely leave free, and waiting for one stalled the iteration
  // (and work queued behind it) for seconds.
  s->cctx->run_big = 0;
  // Its iterations are bounded by iteration_work, so levels of 2^24
  // prefixes suffice (an overflow reruns the iteration depth-first); the
  // pipeline's buffers scale with this capacity, and every GB of them costs
  // about 0.1 s to allocate.
  s->cctx->batch_cap = std::min<uint64_t>(s->cctx->batch_cap, 1ull << 24);
  s->cur = g->cur;
  for (int b = 0; b < kMaxVersions; ++b) {
    s->lo[b] = 1;  // empty
    s->hi[b] = 0;
  }
  s->lo[s->cur] = s->hi[s->cur] = 0;
  s->version_no[s->cur] = g->version;
  if (s->cur >= s->nslots) s->nslots = s->cur + 1;
  try {
    s->count_worker = std::thread(gj::count_loop, s);
    s->update_worker = std::thread(gj::update_loop, s);
  } catch (...) {
    shutdown(s);
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
    if (!s->started) {
      // options are fixed from here: start the heavy lanes (their streams are
      // created now, so that only the lanes in use take hardware queues)
      for (int l = 0; l < s->heavy_lanes; ++l) {
        gj_ctx* c = nullptr;
        gj_status st = gj_ctx_create(s->ctx->device, nullptr, s->ctx->alloc.alloc ? &s->ctx->alloc : nullptr, &c);
        if (st != GJ_OK) break;
        gj::copy_options(c, s->ctx);
        c->hash_build = s->ctx->hash_index >= 2;
        s->hctx.push_back(c);
      }
      if (s->hctx.empty()) return GJ_EDEVICE;
      for (int l = 0; l < s->update_lanes; ++l) {
        gj_ctx* c = nullptr;
        if (gj_ctx_create(s->ctx->device, nullptr, s->ctx->alloc.alloc ? &s->ctx->alloc : nullptr, &c) != GJ_OK)
          break;  // fewer lanes: the updates still run
        gj::copy_options(c, s->ctx);
        c->hash_build = false;
        s->uctx.push_back(c);
      }
      try {
        for (int l = 0; l < (int)s->hctx.size(); ++l) s->heavy_workers.emplace_back(gj::heavy_loop, s, l);
      } catch (...) {
        if (s->heavy_workers.empty()) return GJ_ENOMEM;
      }
      s->started = true;
      s->cv_update.notify_all();
    }
    if (update) {
      ++s->submitted_updates;
      s->updates.push_back(std::move(r));
    } else {
      r.state = s->submitted_updates;
      ++s->pending[r.state];
      s->counts.push_back(std::move(r));
    }
  }
  (update ? s->cv_update : s->cv_count).notify_one();
  return GJ_OK;
}

gj_status gj_server_submit_count(gj_server* s, const gj_query* q, uint64_t seed_lo, uint64_t seed_hi,
                                 uint64_t* ticket) {
  if (!s || !q || !ticket) return GJ_EINVAL;
  if (!q->tris.empty()) return GJ_EUNSUPPORTED;  // ternary atoms run only through gj_run
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
  for (uint32_t i = 0; i < nq; ++i)
    if (!qs[i] || !qs[i]->tris.empty()) return qs[i] ? GJ_EUNSUPPORTED : GJ_EINVAL;
  Req r;
  r.kind = GJ_REQ_UPDATE;
  r.src.assign(src, src + b);
  r.dst.assign(dst, dst + b);
  r.sign.assign(sign, sign + b);
  r.qs.assign(qs, qs + nq);
  return enqueue_req(s, std::move(r), ticket);
}

gj_status gj_server_set_option(gj_server* s, const char* key, int64_t value) {
  if (!s || !key) return GJ_EINVAL;
  std::string k(key);
  std::lock_guard<std::mutex> lk(s->mu);
  if (k == "iteration_work") {
    if (value < 0) return GJ_EINVAL;
    s->iter_work = (uint64_t)value;
  } else if (k == "versions") {
    if (value < 2 || value > kMaxVersions || value <= s->cur) return GJ_EINVAL;
    if (s->started) return GJ_EBUSY;
    s->nslots = (int)value;
  } else if (k == "heavy_lanes") {
    if (value < 1 || value > 4) return GJ_EINVAL;
    if (s->started) return GJ_EBUSY;
    s->heavy_lanes = (int)value;
  } else if (k == "update_lanes") {
    if (value < 0 || value > 4) return GJ_EINVAL;
    if (s->started) return GJ_EBUSY;
    s->update_lanes = (int)value;
  } else if (k == "heavy_work") {
    if (value < 0) return GJ_EINVAL;
    s->heavy_work = (uint64_t)value;
  } else if (k == "update_priority") {
    if (value != 0 && value != 1) return GJ_EINVAL;
    s->update_priority = value != 0;
  } else if (k == "max_batch") {
    if (value < 1 || value > (1 << 16)) return GJ_EINVAL;
    s->max_batch = (uint32_t)value;
  } else {
    return GJ_EINVAL;
  }
  return GJ_OK;
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
  if (s) shutdown(s);
}

}  // extern "C"
