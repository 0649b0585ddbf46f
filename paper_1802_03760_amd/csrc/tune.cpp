// Autotuner of gj_run_batch: searches its parameters on the caller's own
// batch -- the membership test (per-row hash tables or searches), the
// linear-search threshold, the persistent grid (waves per CU), the candidate
// chunk a wave claims at a time, the work bound from which a request leaves
// the fused pipeline for the depth-first path, the depth-first propose
// kernel's lockstep width, and the intersection strategy of the last stages
// (grouped by prefix runs in the fused pipeline or not, and the size ratio
// at which a run streams a prefix's set rather than probing it) -- keeps the
// fastest, and caches the choice in a
// small JSON file keyed by the graph and the query set.  Every configuration
// must produce the same counts; a difference is reported as a device error.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <vector>

#include "batch.h"
#include "gj_internal.h"

namespace gj {

static std::string tune_key(const gj_graph* g, uint32_t nreq, const gj_query* const* qs) {
  // graph size + an FNV-1a hash of the queries (atoms and orders)
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t x) {
    for (int i = 0; i < 8; ++i) {
      h ^= (x >> (8 * i)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  for (uint32_t i = 0; i < nreq; ++i) {
    mix((uint64_t)qs[i]->m);
    for (auto& a : qs[i]->atoms) mix(((uint64_t)a.src_attr << 8) | a.dst_attr);
    for (int o : qs[i]->order) mix((uint64_t)o);
  }
  std::ostringstream k;
  k << "n" << g->n << "_e" << g->ver[g->cur].m << "_r" << nreq << "_q" << std::hex << h;
  return k.str();
}

// The tuned parameters, in the order they are searched.
struct Params {
  uint32_t lin, waves, claim, hash, propose_u;
  uint64_t heavy;
  uint32_t batch_run, run_ratio;
};

static bool same(const Params& a, const Params& b) {
  return a.lin == b.lin && a.waves == b.waves && a.claim == b.claim && a.hash == b.hash &&
         a.propose_u == b.propose_u && a.heavy == b.heavy && a.batch_run == b.batch_run &&
         a.run_ratio == b.run_ratio;
}

static Params current(const gj_ctx* c) {
  return Params{c->batch_lin, c->batch_waves_per_cu, c->batch_claim_words, (uint32_t)(c->hash_index ? 1 : 0),
                (uint32_t)c->propose_u, c->batch_heavy, (uint32_t)c->batch_run, c->run_ratio};
}

static void apply(gj_ctx* c, const Params& p) {
  c->batch_lin = p.lin;
  c->batch_waves_per_cu = p.waves;
  c->batch_claim_words = p.claim;
  c->hash_index = p.hash ? (c->hash_index ? c->hash_index : 1) : 0;
  c->propose_u = (int)p.propose_u;
  c->batch_heavy = p.heavy;
  c->batch_run = (int)p.batch_run;
  c->run_ratio = p.run_ratio;
}

// one entry per line: "key": [lin, waves, claim, hash, propose_u, heavy,
// batch_run, run_ratio], (entries of the first six only keep the defaults
// of the last two)
static std::map<std::string, Params> read_cache(const char* path) {
  std::map<std::string, Params> m;
  if (!path) return m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    size_t a = line.find('"'), b = line.find('"', a + 1), l = line.find('[', b), r = line.find(']', l);
    if (a == std::string::npos || b == std::string::npos || l == std::string::npos || r == std::string::npos)
      continue;
    unsigned lin = 0, waves = 0, claim = 0, hash = 0, pu = 0, brun = 1, ratio = 2;
    unsigned long long heavy = 0;
    const int got = sscanf(line.c_str() + l + 1, "%u , %u , %u , %u , %u , %llu , %u , %u", &lin, &waves, &claim,
                           &hash, &pu, &heavy, &brun, &ratio);
    if (got == 6 || got == 8)
      m[line.substr(a + 1, b - a - 1)] = Params{lin, waves, claim, hash, pu, heavy, brun, ratio};
  }
  return m;
}

static void write_cache(const char* path, const std::map<std::string, Params>& m) {
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (auto& kv : m) {
    const Params& p = kv.second;
    f << "  \"" << kv.first << "\": [" << p.lin << ", " << p.waves << ", " << p.claim << ", " << p.hash << ", "
      << p.propose_u << ", " << p.heavy << ", " << p.batch_run << ", " << p.run_ratio << "]"
      << (++i < m.size() ? "," : "") << "\n";
  }
  f << "}\n";
}

static void report(gj_tuning* out, const Params& p, double ms, int tried, int cached) {
  if (!out) return;
  out->batch_lin = p.lin;
  out->batch_waves_per_cu = p.waves;
  out->batch_claim_words = p.claim;
  out->hash_index = p.hash;
  out->propose_u = p.propose_u;
  out->batch_heavy = p.heavy;
  out->batch_run = p.batch_run;
  out->run_ratio = p.run_ratio;
  out->best_ms = ms;
  out->configs_tried = tried;
  out->from_cache = cached;
}

// Coordinate descent over the parameters of gj_run_batch on the caller's own
// batch: each parameter in turn takes each of its candidate values with the
// others held at their best so far, and keeps the fastest (wall time of the
// whole call, best of two after a warm-up that also builds what the
// configuration needs: captured pipeline, membership index).  Every
// configuration must give the same counts.
void autotune(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* lo,
              const uint64_t* hi, const char* cache_path, gj_tuning* out) {
  std::string key = tune_key(g, nreq, qs);
  auto cache = read_cache(cache_path);
  auto it = cache.find(key);
  if (it != cache.end()) {
    apply(c, it->second);
    report(out, it->second, -1, 0, 1);
    return;
  }
  std::vector<uint64_t> ref(nreq), cnt(nreq);
  std::vector<gj_stats> st(nreq);
  // configurations with the membership index have it from their warm-up on
  const uint64_t build_work = c->hash_build_work;
  struct Restore {
    gj_ctx* c;
    uint64_t w;
    ~Restore() { c->hash_build_work = w; }
  } restore{c, build_work};
  c->hash_build_work = 0;
  bool have_ref = false;
  int tried = 0;
  auto time_one = [&](const Params& p) {
    apply(c, p);
    count_batch(c, g, nreq, qs, lo, hi, cnt.data(), st.data(), nullptr);  // warm-up
    double t = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      GJ_HIP(hipStreamSynchronize(c->stream));
      auto t0 = std::chrono::steady_clock::now();
      count_batch(c, g, nreq, qs, lo, hi, cnt.data(), st.data(), nullptr);
      GJ_HIP(hipStreamSynchronize(c->stream));
      t = std::min(t, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    if (!have_ref) {
      ref = cnt;
      have_ref = true;
    }
    GJ_CHECK(cnt == ref, GJ_EDEVICE, "autotune: configurations disagree on the counts");
    ++tried;
    return t;
  };
  Params best = current(c);
  double best_ms = time_one(best);
  auto sweep = [&](auto field, std::initializer_list<uint64_t> values) {
    Params base = best;
    for (uint64_t v : values) {
      Params p = base;
      field(p, v);
      if (same(p, base)) continue;
      double t = time_one(p);
      if (t < best_ms) {
        best_ms = t;
        best = p;
      }
    }
  };
  sweep([](Params& p, uint64_t v) { p.hash = (uint32_t)v; }, {0, 1});
  sweep([](Params& p, uint64_t v) { p.lin = (uint32_t)v; }, {0, 8, 32, 128});
  sweep([](Params& p, uint64_t v) { p.waves = (uint32_t)v; }, {16, 32, 64});
  sweep([](Params& p, uint64_t v) { p.claim = (uint32_t)v; }, {4, 16, 64});
  sweep([](Params& p, uint64_t v) { p.heavy = v; }, {0, 1ull << 22, 1ull << 24, 1ull << 26});
  sweep([](Params& p, uint64_t v) { p.propose_u = (uint32_t)v; }, {1, 2, 4});
  sweep([](Params& p, uint64_t v) { p.batch_run = (uint32_t)v; }, {0, 1});
  sweep([](Params& p, uint64_t v) { p.run_ratio = (uint32_t)v; }, {1, 2, 8});
  apply(c, best);
  if (cache_path) {
    cache[key] = best;
    write_cache(cache_path, cache);
  }
  report(out, best, best_ms, tried, 0);
}

}  // namespace gj
