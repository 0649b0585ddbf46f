// Internal declarations shared by the HIP sources of libgj.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gj.h"

namespace gj {
class BatchExec;

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kMaxBind = 8;       // binding atoms per stage handled by the kernels

// ---------------------------------------------------------------- errors
struct Error {
  gj_status code;
  std::string msg;
};

#define GJ_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      throw ::gj::Error{GJ_EDEVICE, std::string(#call) + ": " +             \
                                        hipGetErrorString(e_)};             \
  } while (0)

#define GJ_CHECK(cond, code, msg)                      \
  do {                                                 \
    if (!(cond)) throw ::gj::Error{(code), (msg)};     \
  } while (0)

// ---------------------------------------------------------------- device structs
// One stage P_j -> P_{j+1}: the atoms binding the new attribute.  For binding
// atom a the extension set of prefix p is adj[a][rp[a][v] .. rp[a][v+1]) with
// v = prefix column col[a] of p.  Binding atoms are in atom-index order so
// that count-minimisation ties resolve to the lowest atom.
struct StageDesc {
  int j;                 // bound columns
  int k;                 // binding atoms (1..kMaxBind)
  uint32_t above, below;  // inequalities: the new value exceeds / stays below these columns
  int col[kMaxBind];
  const uint32_t* rp[kMaxBind];
  const uint32_t* adj[kMaxBind];
  // ternary bindings (col2[a] >= 0): the set of the pair (col, col2) is
  // tcol[trp[e] .. trp[e+1]) with e the position of that pair in the forward
  // CSR (erp, ecol); empty when the pair is no edge
  int ntri;
  int col2[kMaxBind];
  const uint64_t* trp;
  const uint32_t* tcol;
  const uint32_t* erp;
  const uint32_t* ecol;
  // rows rewritten by log-structured updates (row_range in prim.h); null:
  // every row of the atom's version is rp[v] .. rp[v + 1]
  const uint64_t* pm[kMaxBind];
  // membership index of the atom's version and direction (hash.hip), or
  // null: hd[a][v] describes row v's table in hs[a] (0: no table)
  const uint64_t* hd[kMaxBind];
  const uint32_t* hs[kMaxBind];
  // Per-prefix records written by count-minimisation (the prefix's count and
  // proposing index of Sec. 3.1, with where its sets live), or null: the
  // stage kernels then resolve every candidate's rows from the frontier.
  // pl[p]: start of the proposing atom's row in adj[mini[p]];
  // ent[a * es + p] for the other atoms: the row's table descriptor (as
  // hd), or kEntRange | length << 32 | start when it has none.  Binary atoms
  // only (no ternary binding in the stage), rows below 2^31 entries.
  uint32_t* pl;
  uint64_t* ent;
  uint64_t es;
};

constexpr uint64_t kEntRange = 1ull << 63;

// Membership filters of the seed pairs (atoms over the first two attributes
// other than the seed atom): keep (x0, x1) iff x[val] is in adj[rp[x[key]]..].
struct SeedFilter {
  int n;
  uint32_t above, below;  // bit 0: x1 must exceed / stay below x0 (inequalities)
  int key[kMaxBind];
  int val[kMaxBind];
  const uint32_t* rp[kMaxBind];
  const uint32_t* adj[kMaxBind];
  const uint64_t* pm[kMaxBind];
};

// Column permutation for final rows: value of prefix column c goes to
// attribute attr[c] of a row of m values.
struct RowMap {
  int m;
  int attr[GJ_MAX_ATTRS];
};

// ---------------------------------------------------------------- host structs
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct CsrDir {
  uint32_t* rp = nullptr;   // n + 1
  uint32_t* col = nullptr;  // cap
  uint32_t* row = nullptr;  // cap
};

// Membership index of one direction (hash.hip): per row a table of 2^b
// four-slot buckets; desc[v] = first bucket << 8 | b, 0 for rows without one.
struct HashDir {
  uint64_t* desc = nullptr;
  uint32_t* slots = nullptr;
  uint64_t buckets_cap = 0;
};

// The owner-grouped kernel's plan of a static count over one version: its
// tasks (owner unit, partner range), a function of the version's degrees,
// kept while gen matches the version's and the key (row-pointer arrays of the
// atoms and seed indexes, the minimum task work) is the same.
struct OwnerPlan {
  uint32_t* tasks = nullptr;  // 3 x nt, device, allocated through the graph's context
  uint64_t cap = 0;           // u32 entries allocated
  uint64_t nt = 0, split_units = 0;
  uint64_t gen = ~0ull, tw = 0;
  const uint32_t* key[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct Version {
  CsrDir d[2];  // 0 forward, 1 reverse
  uint64_t m = 0, cap = 0;
  uint32_t max_deg[2] = {0, 0};
  // contents generation, advanced whenever the slot is written; the index
  // h is valid while hash_gen == gen
  uint64_t gen = 0;
  uint64_t hash_gen = ~0ull;
  uint32_t hash_min = 0;  // the least row size with a table in h
  HashDir h[2];
  // candidates proposed by static reads of the contents of generation
  // work_gen (decides when an index pays for its build)
  uint64_t probe_work = 0, work_gen = ~0ull;
  // Views written by a log-structured update only (never a graph's slot):
  // per direction and vertex, the row as arena offset | length << 32 when the
  // update path has rewritten it into the tail of col, ~0 when it is still
  // rp[v] .. rp[v + 1]; null when no row is rewritten.
  const uint64_t* pmap[2] = {nullptr, nullptr};
  // only the graph's own slots fill it (copies of a Version never do)
  OwnerPlan plan;
};

// Log-structured updates (the multi-version index of Sec. 4.3): between two
// compactions the current version is the compacted slot ver[cur] plus the
// rows an update has rewritten, appended to the slack of that slot's column
// arrays past m and found through one of two per-vertex maps (one for the
// current version, the other written for the next, so that the old and the
// new version of a batch are both readable while its delta queries run).
struct LsmState {
  bool on = false;      // some row is rewritten: the current version is ver[cur] + map[cur_map]
  int cur_map = 0;
  uint64_t* map[2][2] = {};  // [buffer][direction], n entries each, ~0 = row in the compacted slot
  uint32_t* keys[2] = {};    // [direction]: vertices with a map entry since the last compaction
  uint64_t nkeys[2] = {0, 0};
  uint64_t used[2] = {0, 0};  // arena entries appended per direction
  uint64_t m = 0;             // edges of the current version
};

// The triangle relation of one version, keyed by forward edge position.
struct TriIndex {
  uint64_t* rp = nullptr;   // m + 1
  uint32_t* col = nullptr;  // size
  uint64_t size = 0;
  uint64_t version = ~0ull;  // graph version it was built for
  int slot = -1;
};

}  // namespace gj

struct gj_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  gj_allocator alloc{};     // device memory source (alloc == null: hipMalloc / hipFree)
  std::string err;
  uint64_t frontier_cap = 1ull << 25;
  uint64_t seed_chunk = 1ull << 25;
  int strategy = 0;
  int num_cus = 256;
  std::map<std::string, gj::DevBuf> ws;
  // workspace buffers replaced by larger ones (ws_get), kept until the
  // context is destroyed
  std::vector<void*> ws_retired;
  // While `on`, ws_get hands out named pieces of [base, base + size) (the
  // allocation-free entry point's scratch) and dev_alloc refuses to run.
  struct Arena {
    bool on = false;
    uint8_t* base = nullptr;
    uint64_t size = 0, used = 0;
    std::map<std::string, gj::DevBuf> named;
  } arena;
  void* pinned = nullptr;  // small pinned host staging (4 KiB)
  std::vector<hipEvent_t> events;  // pool for kernel timing (pairs)
  // consolidated delta rows of the last gj_apply_updates, per query position
  struct LastDelta {
    bool kept = false;
    int m = 0;
    uint64_t n = 0;
    uint32_t* rows = nullptr;
    int8_t* signs = nullptr;
  };
  std::vector<LastDelta> last_delta;
  // batched executor and its tuned parameters
  gj::BatchExec* batch = nullptr;
  uint32_t batch_lin = 8;           // linear search below this extension-set size
  uint32_t batch_waves_per_cu = 32; // resident waves per CU of the persistent grids
  uint32_t batch_claim_words = 16;  // words of 64 candidates a wave of the fused propose claims at a time
  uint64_t batch_cap = 1ull << 27;  // prefixes per level of the batched pipeline
  int batch_run = 1;                 // the batched pipeline's last stages take the run kernels where they apply
  uint64_t batch_fallbacks = 0;     // batches rerun depth-first after a level overflow
  int delta_fused = 1;              // count-only delta queries through the fused pipeline
  uint64_t delta_owner_min = 1ull << 17;  // changes from which triangle-shaped deltas use the owner kernel
  uint64_t delta_lane_min = 1024;  // changes from which a server's updates run their dQ_i on its delta lanes
  int factorise = 0;  // gj_run counts: trailing independent attributes as products
  uint64_t batch_heavy = 1ull << 24;  // gj_run_batch: estimated work from which a request runs depth-first
  int propose_u = 4;  // candidates per lane tested in lockstep by the generic propose kernel (1, 2, 4)
  int lsm_updates = 0;  // gj_apply_updates: append rewritten rows instead of rewriting both indexes
  uint64_t lsm_max_patch = 0;  // arena entries per direction before a compaction (0: the slot's slack)
  uint64_t lsm_fold_min = 8192;  // batches of at least this many changes fold without sizing their rows
  uint64_t lsm_compactions = 0;  // compactions run on this context
  uint64_t lsm_folds = 0;  // batches written as a new version while appended rows were pending
  uint64_t owner_task_min = 1ull << 20;  // least proposals per owner task (owner-grouped kernel)
  int hash_index = 1;      // 0: rows are searched; 1, 2: membership indexes are used where built
  bool hash_build = true;  // this context builds missing indexes on static reads
  uint32_t hash_min_degree = 32;  // rows of at least this many entries get a table
  uint64_t hash_build_work = 64;  // build once reads of a version proposed this many candidates per edge
  uint64_t hash_builds = 0;       // membership indexes built by this context
  int run_stage = 1;               // last-stage counts grouped by prefix runs where they apply
  uint32_t run_ratio = 2;          // stream a new set through S's table up to this many times |S|
  uint64_t run_min_work = 256;     // least count-minimised candidates of a staged run
  uint64_t run_task_work = 1ull << 15;  // candidates per task of a staged run beyond its build
  uint64_t run_stage_min = 1ull << 22;  // least candidates of a stage taken by the run kernels
  uint32_t run_reuse = 4;          // staged runs: candidates >= this x the shared set bound
  int run_big = 1;                 // 0: shared sets beyond the small shape's table are not staged
  uint64_t run_min_tasks = 256;    // fewer staged tasks in a stage: the per-candidate kernel takes it
  uint64_t run_tasks = 0;          // tasks of the run kernels on this context
  uint64_t run_tasks_big = 0;      // of those, tasks of the large-set shape
  uint64_t run_declined = 0;       // stages planned by runs but left to the per-candidate kernel
  // device sums over the context's life (run.hip): count-minimised
  // candidates of planned runs that were staged, whose shared set exceeds
  // the tables, with too little work to repay a build; then the counting
  // kernels' units (values tested), builds, and the values builds streamed
  unsigned long long* run_stats = nullptr;
  uint64_t owner_tasks = 0;        // tasks of the last owner-grouped launch
  uint64_t owner_split_units = 0;  // owner units of that launch cut into more than one task
};

// Resident versions of a graph: ver[cur] is current; an update reads it and
// writes another slot (allocated on first use), which then becomes current.
// Two slots serve the plain update path; a server may rotate through more so
// that counts of older versions keep running while updates proceed.
constexpr int kMaxVersions = 8;

struct gj_graph {
  gj_ctx* ctx = nullptr;
  uint32_t n = 0;
  uint32_t* old_of_new = nullptr;  // device, n entries: renamed by degree, else null
  gj::TriIndex tri;
  gj::Version ver[kMaxVersions];
  int cur = 0;
  uint64_t version = 0;
  gj::LsmState lsm;
  std::mutex hash_mu;  // one build of a version's membership index at a time
};

struct gj_query {
  int m = 0;
  std::vector<gj_atom> atoms;
  std::vector<int> order;
  std::vector<gj_less> less;  // value(lo_attr) < value(hi_attr)
  std::vector<gj_tri_atom> tris;
};

namespace gj {

// ---------------------------------------------------------------- host helpers
// Times the hot kernels of one call with HIP events on the context stream.
class KernelTimer {
 public:
  explicit KernelTimer(gj_ctx* c) : c_(c) {}
  void start();
  void stop();
  // synchronises the stream; returns summed milliseconds of the recorded pairs
  double total_ms();
  uint64_t launches() const { return n_; }

 private:
  gj_ctx* c_;
  size_t n_ = 0;
};

// workspace buffers up to this size are retired rather than freed when they grow
constexpr size_t kWsRetireMax = 256ull << 20;
void* ws_get(gj_ctx* c, const std::string& name, size_t bytes);
// Device memory through the context's allocator (hipMalloc / hipFree without
// one).  dev_alloc throws GJ_ENOMEM on failure; dev_free(c, null) is a no-op.
void dev_free(gj_ctx* c, void* p);
void* dev_alloc(gj_ctx* c, size_t bytes);

// Device memory owned by one scope, freed on every exit (errors included).
class DevMem {
 public:
  DevMem() = default;
  DevMem(gj_ctx* c, size_t bytes) : c_(c), p_(dev_alloc(c, bytes)) {}
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : c_(o.c_), p_(o.p_) { o.p_ = nullptr; }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      reset();
      c_ = o.c_;
      p_ = o.p_;
      o.p_ = nullptr;
    }
    return *this;
  }
  ~DevMem() { reset(); }
  void reset() {
    if (p_) dev_free(c_, p_);
    p_ = nullptr;
  }
  template <class T>
  T* as() const {
    return (T*)p_;
  }
  void* get() const { return p_; }
  void* release() {
    void* p = p_;
    p_ = nullptr;
    return p;
  }

 private:
  gj_ctx* c_ = nullptr;
  void* p_ = nullptr;
};
uint64_t read_u64(gj_ctx* c, const void* dptr);
void read_bytes(gj_ctx* c, void* host, const void* dptr, size_t bytes);
// several device words, one synchronisation
void read_u64s(gj_ctx* c, std::initializer_list<const uint64_t*> ptrs, uint64_t* host);
void read_u32s(gj_ctx* c, std::initializer_list<const uint32_t*> ptrs, uint32_t* host);

inline unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap = 1u << 20) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// hash.hip: the membership index of version v (both directions), built if
// this context builds indexes and v's is missing or stale; freed with v
void hash_ensure(gj_ctx* c, const gj_graph* g, const Version& v);
// adds W proposed candidates to v's account and builds its index (as
// hash_ensure) once the account reaches hash_build_work x its edges;
// returns whether v's index is usable now
bool hash_note_work(gj_ctx* c, const gj_graph* g, const Version& v, uint64_t W);
void hash_free(gj_ctx* c, Version& v);

// scan.hip: workspace bytes of the scans of up to n items, and their
// reservation (so that later scans of at most n items take no new buffer)
uint64_t scan_scratch_bytes(uint64_t n);
void scan_reserve(gj_ctx* c, uint64_t n);
// engine.hip: workspace bytes of a count-only, unweighted Runner (query of m
// attributes, P_2 batches of seed_cap seeds, frontiers of fcap prefixes),
// scans included, in pieces aligned as the arena aligns them
uint64_t runner_scratch_bytes(int m, uint64_t seed_cap, uint64_t fcap);
// noalloc.hip: the scratch array of this device (resolved once per device)
// and the lock that keeps calls on one device from overlapping on it
void* scratch_ptr(int device);
uint64_t scratch_bytes();
void scratch_lock(int device, bool lock);
constexpr uint64_t kArenaAlign = 256;

// scan.hip: exclusive scans; out has n + 1 entries (out[n] = total)
void scan_u32_to_u64(gj_ctx* c, const uint32_t* in, uint64_t* out, uint64_t n);
void scan_u64(gj_ctx* c, const uint64_t* in, uint64_t* out, uint64_t n);
void scan_u32(gj_ctx* c, const uint32_t* in, uint32_t* out, uint64_t n);

// sort.hip: stable LSD radix sorts; return the buffer holding the result
uint64_t* sort_u64(gj_ctx* c, uint64_t* keys, uint64_t* alt, uint64_t n, int lo_bits, int hi_bits);
// sorts (key, val) pairs by key; key/val and alt buffers swap.  Equal keys
// keep their input order above 2048 pairs and are ordered by val below (one
// workgroup sorts those), so callers must not rely on the order among equal
// keys.
void sort_kv_u64(gj_ctx* c, uint64_t*& key, uint32_t*& val, uint64_t*& key_alt, uint32_t*& val_alt,
                 uint64_t n, int lo_bits, int hi_bits);
void sort_kv_u32(gj_ctx* c, uint32_t*& key, uint32_t*& val, uint32_t*& key_alt,
                 uint32_t*& val_alt, uint64_t n, int bits);

// graph.hip
void graph_build(gj_ctx* c, gj_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m);
// The input read as undirected: its symmetric edge set (both directions of
// every distinct pair), or with degree_order the vertices renamed by ascending
// (degree, id) and each pair kept once from the lower new id to the higher
// (both directions when `undirected`).  Sets g->old_of_new when renaming.
void graph_build_sym(gj_ctx* c, gj_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                     bool degree_order, bool undirected);
void version_alloc(gj_ctx* c, Version& v, uint32_t n, uint64_t cap);
void version_free(gj_ctx* c, Version& v);
// Log-structured updates: merge the rewritten rows into a compacted slot
// (no-op when none are); release the maps.
void graph_compact(gj_ctx* c, gj_graph* g);
void lsm_free(gj_graph* g);
// graph_compact for readers that need the current version as one plain CSR
// (the relation is unchanged); errors as a status
gj_status settle(gj_ctx* c, const gj_graph* g);

// stage.hip
void launch_seed(gj_ctx* c, const uint32_t* x0, const uint32_t* x1, const int8_t* w, uint64_t cnt,
                 const SeedFilter& f, uint32_t* flags, uint64_t* off, uint32_t* F, uint64_t stride,
                 int8_t* Fw);
void launch_count_min(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const StageDesc& d,
                      uint32_t* minc, uint8_t* mini);
// The new values of the survivors of [w0, w1) only, at out[obase + pos].
void launch_emit_values(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off,
                        const uint8_t* mini, const StageDesc& d, uint64_t w0, uint64_t w1, const uint64_t* mask,
                        const uint64_t* woff, uint32_t* out, uint64_t obase, uint64_t ocap);
// clique.hip: the transitive 4-clique (shape 0) or the diamond (shape 1) over
// every forward edge of v, grouped by seed edge, with the plan's inequality
// masks of positions 1..3.  out = {matches, prefixes[3], extensions[2],
// extensions[3], prefixes[2]} of the seeds it finished; the n_left others
// (their fixed set too large for LDS) are left as seed pairs (x0[i], x1[i]) in
// context workspace for the depth-first path.
// hd/hs: the version's forward membership index (row tables for the probes
// of rows in memory), or null.
void edge4_count(gj_ctx* c, const Version& v, int shape, const uint32_t above[4], const uint32_t below[4],
                 const uint64_t* hd, const uint32_t* hs, KernelTimer& timer, uint64_t out[5], uint32_t*& x0,
                 uint32_t*& x1, uint64_t& n_left);
// clique.hip: the diamond over every forward edge of v by 2-path counts (no
// inequalities): out = {matches, prefixes[3] = extensions[2], extensions[3]}.
void diamond2p_count(gj_ctx* c, const Version& v, uint32_t n, KernelTimer& timer, uint64_t out[3]);
// the transitive 5-clique by seed edge (forward CSR): out = matches,
// prefixes[2], extensions[2], prefixes[3], extensions[3], prefixes[4],
// extensions[4] of the seeds it took; the others (x0, x1: n_left pairs, in
// workspace) are left to the depth-first path
void clique5_count(gj_ctx* c, const Version& v, const uint32_t above[5], const uint32_t below[5],
                   const uint64_t* hd, const uint32_t* hs, KernelTimer& timer, uint64_t out[7], uint32_t*& x0,
                   uint32_t*& x1, uint64_t& n_left);
// clique.hip: the 4-cycle a0 -> a1 -> a2 -> a3 -> a0 by forward and backward
// 2-path counts (no inequalities): out = {matches, prefixes[3] =
// extensions[2], extensions[3]}.
void cycle4_2p_count(gj_ctx* c, const Version& v, uint32_t n, KernelTimer& timer, uint64_t out[3]);
// tri.hip: the triangle relation of the graph's current version (replaces
// g->tri); frees it
void tri_index_build(gj_ctx* c, gj_graph* g);
void tri_index_free(gj_graph* g);
// Sum over the n prefixes of the product of T per-prefix counts
// cnt[t * stride + p], added to acc[0].
void launch_factor_sum(gj_ctx* c, const uint32_t* cnt, uint64_t stride, uint64_t n, int T,
                       unsigned long long* acc);
void launch_propose(gj_ctx* c, int mode, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off,
                    const uint8_t* mini, const StageDesc& d, uint64_t w0, uint64_t w1, uint64_t* mask,
                    uint32_t* wcnt, const int8_t* wt, unsigned long long* acc);
void launch_emit(gj_ctx* c, bool final_rows, const uint32_t* F, uint64_t stride, uint64_t n, const uint64_t* off,
                 const uint8_t* mini, const StageDesc& d, uint64_t w0, uint64_t w1, const uint64_t* mask,
                 const uint64_t* woff, const int8_t* wt, uint32_t* G, uint64_t gstride, int8_t* Gw,
                 const RowMap& map, uint64_t obase, uint64_t ocap);
void launch_rows_from_frontier(gj_ctx* c, const uint32_t* F, uint64_t stride, uint64_t n, const int8_t* wt,
                               const RowMap& map, uint32_t* rows, int8_t* osign, uint64_t obase, uint64_t ocap,
                               unsigned long long* acc);

// rows.hip: sort rows (and optional signs) ascending; consolidate signed rows
void sort_rows(gj_ctx* c, uint32_t* rows, int8_t* signs, uint64_t nrows, int m, uint32_t nverts);
uint64_t consolidate_rows(gj_ctx* c, const uint32_t* rows, const int8_t* signs, uint64_t nrows, int m,
                          uint32_t* out_rows, int8_t* out_signs, uint64_t cap, int64_t* sum);
int bits_for(uint32_t n);
// Row pointers and largest degrees of both directions: computed here from the
// rows, or (from_update) already written by the update, the degrees into the
// "maxdeg" workspace.  Reads the degrees back to the host.
void version_finish(gj_ctx* c, Version& v, uint32_t n, bool from_update);

// api.hip: counts of nreq requests on version ver (null: current), fused
void count_batch(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* seed_lo,
                 const uint64_t* seed_hi, uint64_t* counts, gj_stats* stats, const Version* ver);

// api.hip: counts of nreq requests, request i on version vers[i], as a status
// (one request alone: the depth-first path; more: one fused pipeline)
gj_status count_on_versions(gj_ctx* c, const gj_graph* g, const Version* const* vers, uint32_t nreq,
                            const gj_query* const* qs, const uint64_t* seed_lo, const uint64_t* seed_hi,
                            uint64_t* counts, gj_stats* stats);
// api.hip: an update batch from host arrays written into version slot
// `target`, count deltas only, as a status
gj_status update_into(gj_ctx* c, gj_graph* g, const uint32_t* src, const uint32_t* dst, const int8_t* sign,
                      uint64_t b, const gj_query* const* qs, uint32_t nq, int64_t* count_delta, int target,
                      const std::vector<gj_ctx*>* lanes = nullptr);
// api.hip: allocate version slot b with room for cap edges, as a status
gj_status reserve_version(gj_ctx* c, gj_graph* g, int b, uint64_t cap);
// api.hip: copy the tunable options of one context to another
void copy_options(gj_ctx* dst, const gj_ctx* src);

// tune.cpp
void autotune(gj_ctx* c, const gj_graph* g, uint32_t nreq, const gj_query* const* qs, const uint64_t* lo,
              const uint64_t* hi, const char* cache_path, gj_tuning* out);

// engine.hip
// ver: the graph version to read (null: the current one)
void run_static(gj_ctx* c, const gj_graph* g, const gj_query* q, int mode, uint64_t lo,
                uint64_t hi, uint32_t* out, uint64_t cap, int out_on_device, gj_stats* st,
                bool& overflow, const Version* ver = nullptr);
// target: the version slot to write (-1: slot 1 - cur for cur < 2, else 0)
// lanes: other contexts on the device on which the count-only dQ_i of a
// batch of at least delta_lane_min changes run side by side (null: none)
void apply_updates(gj_ctx* c, gj_graph* g, const uint32_t* src, const uint32_t* dst,
                   const int8_t* sign, uint64_t b, int on_device, const gj_query* const* qs,
                   uint32_t nq, int64_t* count_delta, uint32_t* const* rows,
                   int8_t* const* signs, const uint64_t* cap, uint64_t* n_delta,
                   gj_stats* stats, bool& overflow, int target = -1,
                   const std::vector<gj_ctx*>* lanes = nullptr);

}  // namespace gj
