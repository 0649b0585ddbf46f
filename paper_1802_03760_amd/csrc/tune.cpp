// Autotuner of the batched executor: times every candidate configuration on
// the caller's own batch, keeps the fastest, and caches the choice in a small
// JSON file keyed by the graph and the query set.  Every configuration must
// produce the same counts; a difference is reported as a device error.
#include <algorithm>
#include <cstdio>
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

static std::map<std::string, std::pair<uint32_t, uint32_t>> read_cache(const char* path) {
  std::map<std::string, std::pair<uint32_t, uint32_t>> m;
  if (!path) return m;
  std::ifstream f(path);
  std::string line;
  // one entry per line: "key": [lin, waves],
  while (std::getline(f, line)) {
    size_t a = line.find('"'), b = line.find('"', a + 1), l = line.find('[', b), r = line.find(']', l);
    if (a == std::string::npos || b == std::string::npos || l == std::string::npos || r == std::string::npos)
      continue;
    unsigned lin = 0, waves = 0;
    if (sscanf(line.c_str() + l + 1, "%u , %u", &lin, &waves) == 2)
      m[line.substr(a + 1, b - a - 1)] = {lin, waves};
  }
  return m;
}

static void write_cache(const char* path, const std::map<std::string, std::pair<uint32_t, uint32_t>>& m) {
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (auto& kv : m) {
    f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
      << (++i < m.size() ? "," : "") << "\n";
  }
  f << "}\n";
}

void autotune(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* lo,
              const uint64_t* hi, const char* cache_path, gj_tuning* out) {
  std::string key = tune_key(g, nreq, qs);
  auto cache = read_cache(cache_path);
  auto it = cache.find(key);
  if (it != cache.end()) {
    c->batch_lin = it->second.first;
    c->batch_waves_per_cu = it->second.second;
    if (out) {
      out->batch_lin = c->batch_lin;
      out->batch_waves_per_cu = c->batch_waves_per_cu;
      out->best_ms = -1;
      out->configs_tried = 0;
      out->from_cache = 1;
    }
    return;
  }
  if (!c->batch) c->batch = new BatchExec();
  const uint32_t lins[] = {0, 8, 32, 128};
  const uint32_t waves[] = {16, 32, 64};
  std::vector<uint64_t> ref(nreq), cnt(nreq);
  std::vector<gj_stats> st(nreq);
  double best = 1e300;
  uint32_t best_lin = c->batch_lin, best_w = c->batch_waves_per_cu;
  bool have_ref = false;
  int tried = 0;
  for (uint32_t w : waves) {
    for (uint32_t l : lins) {
      c->batch_lin = l;
      c->batch_waves_per_cu = w;
      bool ov = false;
      c->batch->run(c, g, nreq, qs, lo, hi, cnt.data(), st.data(), ov);  // warm-up / capture
      GJ_CHECK(!ov, GJ_EUNSUPPORTED, "autotune: batch exceeds the frontier capacity");
      double t = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        c->batch->run(c, g, nreq, qs, lo, hi, cnt.data(), st.data(), ov);
        t = std::min(t, st[0].kernel_ms);
      }
      if (!have_ref) {
        ref = cnt;
        have_ref = true;
      }
      GJ_CHECK(cnt == ref, GJ_EDEVICE, "autotune: configurations disagree on the counts");
      ++tried;
      if (t < best) {
        best = t;
        best_lin = l;
        best_w = w;
      }
    }
  }
  c->batch_lin = best_lin;
  c->batch_waves_per_cu = best_w;
  if (cache_path) {
    cache[key] = {best_lin, best_w};
    write_cache(cache_path, cache);
  }
  if (out) {
    out->batch_lin = best_lin;
    out->batch_waves_per_cu = best_w;
    out->best_ms = best;
    out->configs_tried = tried;
    out->from_cache = 0;
  }
}

}  // namespace gj
