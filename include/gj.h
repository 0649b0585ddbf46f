/*
 * gj.h -- C ABI of the MI355X Generic Join library (libgj.so).
 *
 * Evaluates subgraph queries as multiway self-joins of one edge relation with
 * Generic Join, and maintains their results under edge insertions and
 * deletions with delta queries.  Paper: Ammar, McSherry, Salihoglu,
 * Joglekar, "Distributed Evaluation of Subgraph Queries Using Worst-case
 * Optimal Low-Memory Dataflows" (VLDB 2018).
 *
 * Conventions for every call:
 *  - Returns gj_status; nothing throws across the ABI.  On failure a message
 *    is available from gj_last_error() of the context.
 *  - Inputs are copied (host or device pointers, as each call states);
 *    handles are owned by the library; output buffers are owned by the caller.
 *  - One context per host thread.  Work is issued on the context's HIP
 *    stream; calls return after their results are in the caller's buffers.
 *  - Vertex ids are uint32 < num_vertices; edges per graph < 2^32.
 *  - Counts are exact unsigned 64-bit integers.
 */
#ifndef GJ_H
#define GJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GJ_OK = 0,
  GJ_EINVAL = 1,       /* invalid argument, query or update batch */
  GJ_ENOMEM = 2,       /* device allocation failed */
  GJ_EDEVICE = 3,      /* HIP runtime error */
  GJ_EOVERFLOW = 4,    /* output buffer too small; required size reported */
  GJ_EUNSUPPORTED = 5, /* outside the supported limits */
  GJ_EBUSY = 6         /* resource in use */
} gj_status;

#define GJ_MAX_ATTRS 8
#define GJ_MAX_ATOMS 16

typedef struct gj_ctx gj_ctx;
typedef struct gj_graph gj_graph;
typedef struct gj_query gj_query;

/* Source of the library's device memory (graph indexes, frontiers,
 * workspace).  alloc returns `bytes` of device memory on the current device,
 * or NULL when none is left (the call then fails with GJ_ENOMEM); `stream`
 * is the hipStream_t of the context that asks.  free returns a block from
 * alloc; the library calls it only after that stream has finished with the
 * block.  Both may be called from the threads of a server (gj_server_*) on
 * the context, and from several contexts at once when they share the
 * allocator.  `user` is passed through. */
typedef struct {
  void* (*alloc)(void* user, size_t bytes, void* stream);
  void (*free)(void* user, void* ptr, void* stream);
  void* user;
} gj_allocator;

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * issue work on (NULL: the library creates its own).  `allocator` (copied;
 * its callbacks must stay valid until the context and everything built on it
 * are destroyed) supplies every device allocation of the context, its
 * graphs and its servers; NULL uses hipMalloc / hipFree.  Internal buffers
 * are owned by the context and reused across calls.  Errors: GJ_EDEVICE for
 * a bad device, GJ_EINVAL for an allocator without both callbacks. */
gj_status gj_ctx_create(int device, void* hip_stream, const gj_allocator* allocator, gj_ctx** out);
/* Releases the context.  Servers and graphs built on it must be destroyed
 * first: gj_graph_destroy waits on the context's stream. */
void gj_ctx_destroy(gj_ctx* ctx);

/* Message of the last failed call on `ctx`; owned by ctx, valid until the
 * next call.  Never NULL. */
const char* gj_last_error(const gj_ctx* ctx);

/* Tuning options (integers).  Keys:
 *   "frontier_cap"  max prefixes held per stage buffer and max candidates
 *                   proposed per batch (the batch bound B of Sec. 3.1.2);
 *                   default 2^25, minimum 64
 *   "seed_chunk"    max seed edges per P_2 batch (default 2^25)
 *   "strategy"      intersection kernel choice: 0 auto, 1 generic
 *                   per-candidate search only, 2 owner-grouped LDS kernel
 *                   where applicable
 *   "batch_lin"     gj_run_batch: linear instead of binary search in
 *                   extension sets of at most this size (default 8)
 *   "batch_waves_per_cu"  gj_run_batch: resident waves per CU of its
 *                   persistent grids, a multiple of 4 in [4, 128] (default 32)
 *   "batch_claim_words"  gj_run_batch: words of 64 candidates a wave of the
 *                   fused propose kernel claims from the device counter at a
 *                   time, 1..4096 (default 16)
 *   "batch_cap"     gj_run_batch: prefixes per level (default 2^27)
 *   "batch_run"     gj_run_batch: 1 (default) lets the fused pipeline's last
 *                   stage of a static count take the run kernels of
 *                   "run_stage" (with its run_ratio, run_min_work,
 *                   run_reuse and run_task_work; levels of at most 2^25
 *                   prefixes; the context's run_* sums count their work);
 *                   0 keeps the per-candidate kernel there.  Counts and
 *                   counters are the same either way
 *   "batch_heavy"   gj_run_batch: requests whose estimated work (the
 *                   server's seed-work estimate) reaches this run on the
 *                   depth-first path, the rest fused (default 2^24; 0: all
 *                   fused)
 *   "delta_fused"   gj_apply_updates: 1 (default) runs the delta queries of
 *                   every query that asks for counts only as one fused
 *                   pipeline (as gj_run_batch, with signed seeds); 0 runs
 *                   each dQ_i on the depth-first path
 *   "delta_lane_min"  a server's updates: batches with at least this many
 *                   distinct changes (default 1024, >= 0) run their
 *                   count-only dQ_i on the server's delta lanes (see
 *                   gj_server_create)
 *   "delta_owner_min"  gj_apply_updates: batches with at least this many
 *                   distinct changes (default 2^17, >= 0) run the count-only
 *                   delta queries of three-attribute queries whose every
 *                   dQ_i binds the last attribute by one atom on each seed
 *                   attribute (the triangle shapes) on the owner-grouped
 *                   kernel, unless "strategy" is 1
 *   "owner_task_min"  owner-grouped kernel: least proposals per task; a
 *                   unit (an owner's set and its partners) with more work is
 *                   cut into tasks of partner ranges of at least this many
 *                   proposals and at least 8 x the owner's set size (default
 *                   2^20, >= 1)
 *   "hash_index"    membership tests of the generic propose kernels
 *                   (Sec. 2.2: O(1) membership in an extension set): 1
 *                   (default) gives a graph version a per-row open-addressing
 *                   table (four-slot buckets at load <= 1/2) for every row of
 *                   at least "hash_min_degree" entries in both directions
 *                   (about 12 bytes per such entry and direction, plus 8 per
 *                   vertex; kept until the version is rewritten or the graph
 *                   destroyed) once the static reads of that version
 *                   (gj_run, gj_run_batch, gj_autotune) have proposed
 *                   "hash_build_work" candidates per edge, and then probes it
 *                   instead of searching the row; the server and delta
 *                   queries use tables built this way but build none; 2 also
 *                   lets the server build them; 0 searches every row.
 *                   Results are the same either way
 *   "hash_min_degree"  rows of at least this many entries get a table
 *                   (default 32, >= 1)
 *   "hash_build_work"  candidates per edge that static reads of a version
 *                   propose before its tables are built (default 64; 0: at
 *                   the first read that tests membership)
 *   "propose_u"     candidates per lane whose membership searches the
 *                   generic propose kernel runs in lockstep: 1, 2 or 4
 *                   (default 4; at most 2 in stages with ternary atoms)
 *   "factorise"     gj_run counts: 1 counts a trailing run of at least two
 *                   attributes that share no atom and no inequality as the
 *                   product of their extension counts per prefix before the
 *                   run (factorisation, Sec. 5.4): the same count, without
 *                   enumerating the run's prefixes.  Counters then cover that
 *                   work: prefixes inside the run are 0, extensions[t] sums
 *                   the smallest set of position t over the prefixes where
 *                   the run starts.  0 (default) enumerates
 *   "lsm_updates"   gj_apply_updates: 1 keeps the index log-structured
 *                   (the multi-version index of Sec. 4.3): a batch rewrites
 *                   only the rows it touches, appended past the current
 *                   version's edges in the slack of its column arrays and
 *                   found through a per-vertex map, instead of writing a new
 *                   version of both indexes.  A batch whose rewritten rows
 *                   do not fit the rest of the slack, or exceed an eighth of
 *                   the edges (2^16 entries at least) in a direction, is
 *                   written as a new version of both indexes that takes the
 *                   appended rows in too (counter "lsm_folds").  Any call
 *                   that reads the graph other than gj_apply_updates merges
 *                   appended rows into one CSR first (a compaction, into
 *                   another version slot; counter "lsm_compactions"):
 *                   gj_run, gj_run_batch, gj_autotune, gj_graph_csr,
 *                   gj_graph_info with max_out or max_in,
 *                   gj_graph_index_triangles, gj_server_create.  Results
 *                   are the same either way.  0 (default) writes every
 *                   batch as a new version of both indexes
 *   "lsm_fold_min"  with lsm_updates: a batch of at least this many distinct
 *                   changes (default 8192; 0: every batch) is written as a
 *                   new version of both indexes without first sizing the rows
 *                   it touches (such a batch touches most heavy rows)
 *   "lsm_max_patch" with lsm_updates: at most this many appended entries
 *                   per direction (0, default: the slot's slack; a
 *                   compaction leaves m / 2 + 2^22 entries of it, and
 *                   reallocates the slot when less than half of that is
 *                   left)
 *   "run_stage"     1 (default): the last stage of a static count on the
 *                   depth-first path (gj_run, the server's heavy lanes,
 *                   gj_run_batch's heavy requests), when its binary atoms split
 *                   into at least one reading an earlier column and at most
 *                   one reading the last bound column, is counted grouped
 *                   by prefix runs: consecutive prefixes that agree on the
 *                   columns the earlier atoms read share those atoms'
 *                   extension sets, so one workgroup intersects them once
 *                   into an LDS hash table (at most 24,576 values) and counts
 *                   every prefix of the run against it (O(1) membership,
 *                   Sec. 2.2).  Runs with a larger shared set, or too little
 *                   work, stay with the per-candidate kernel.  0 always
 *                   uses the per-candidate kernel; "strategy" 1 does too.
 *                   Counts and counters are the same either way
 *   "run_ratio"     run_stage: a prefix's own set is streamed through the
 *                   table when it holds at most this many times the shared
 *                   set's values, else the shared values are looked up in
 *                   it (0..64, default 2)
 *   "run_min_work"  run_stage: least count-minimised candidates of a run
 *                   for it to be staged (default 256, >= 0)
 *   "run_reuse"     run_stage: a staged run also has at least this many
 *                   times as many candidates as its smallest shared set
 *                   holds values (default 4, 1..1024)
 *   "run_big"       run_stage: 1 (default) stages shared sets of up to
 *                   24,576 values in the large workgroup shape (a whole CU's
 *                   LDS); 0 stages only those of up to 4,096 (the server's
 *                   light lane, whose kernels share the device with other
 *                   lanes)
 *   "run_task_work" run_stage: a run's prefixes are cut into tasks of about
 *                   this many candidates plus 8 per value the build reads
 *                   (default 2^15, >= 1)
 *   "run_stage_min" run_stage: least count-minimised candidates of a stage
 *                   for it to take the run kernels (default 2^22, >= 0;
 *                   a smaller stage takes the per-candidate kernel, which
 *                   finishes it in about the time planning the runs takes)
 *   "run_min_tasks" run_stage: a stage whose staged runs make fewer tasks
 *                   than this (default 256, >= 0) is left whole to the
 *                   per-candidate kernel (a workgroup works through a task
 *                   alone, so a few tasks cannot occupy the device)
 * Returns GJ_EINVAL for an unknown key or out-of-range value. */
gj_status gj_ctx_set_option(gj_ctx* ctx, const char* key, int64_t value);

/* Reads an option (keys above, plus "batch_cap", the counters
 * "lsm_compactions" and "lsm_folds" of this context (see "lsm_updates"),
 * the counter "batch_fallbacks" (gj_run_batch calls that fell back to the
 * depth-first path), "hash_builds" (membership indexes this context built),
 * and of the last owner-grouped launch on this context
 * "owner_tasks" (its tasks) and "owner_split_units" (units cut into more
 * than one task), and of the run kernels (see "run_stage") on this context
 * "run_tasks", "run_tasks_big" (of them, tasks of the large-set shape),
 * "run_declined" (stages planned by runs but left to the per-candidate
 * kernel),
 * "run_w_staged", "run_w_large", "run_w_light" (count-minimised candidates
 * of runs staged, with a shared set above the tables, with too little
 * work), "run_units" (values tested), "run_builds" and "run_build_elems"
 * (shared sets built, and the values they streamed)). */
gj_status gj_ctx_get_option(gj_ctx* ctx, const char* key, int64_t* value);

/* ---------------------------------------------------------------- graphs */

#define GJ_INPUT_DEVICE 1u /* src/dst are device pointers (default: host) */
#define GJ_KEEP_LOOPS 2u   /* not supported: self-loops are always dropped */
/* The input edges are read as undirected: every distinct pair {u, v}, u != v,
 * is stored in both directions. */
#define GJ_BUILD_UNDIRECTED 4u
/* Symmetry breaking's input transform (Sec. 5.4): the input is read as
 * undirected, vertices get new ids in ascending order of (number of distinct
 * neighbours, old id), and each pair is stored once, from its lower new id
 * to its higher (both directions with GJ_BUILD_UNDIRECTED).  A clique query
 * over this graph finds each undirected clique once.  gj_graph_vertex_ids
 * gives the old id of every new one. */
#define GJ_BUILD_DEGREE_ORDER 8u

/* Builds the forward (out-neighbour) and reverse (in-neighbour) indices of
 * the edge relation (one physical copy each, Sec. 4.1): CSR rows sorted
 * ascending, repeated edges collapsed, self-loops dropped.
 * src, dst: m vertex ids each (host memory unless GJ_INPUT_DEVICE).
 * Errors: GJ_EINVAL for an id >= num_vertices, num_vertices == 0 or an
 * unknown flag; GJ_EUNSUPPORTED if m >= 2^32, or m >= 2^31 with
 * GJ_BUILD_UNDIRECTED or GJ_BUILD_DEGREE_ORDER. */
gj_status gj_graph_build(gj_ctx* ctx, const uint32_t* src, const uint32_t* dst,
                         uint64_t m, uint32_t num_vertices, uint32_t flags,
                         gj_graph** out);

/* Sizes of the current version.  Any pointer may be NULL.  Asking for
 * max_out or max_in merges rows appended by log-structured updates first
 * (option "lsm_updates"; errors as gj_apply_updates, on g's context). */
gj_status gj_graph_info(const gj_graph* g, uint64_t* edges, uint32_t* vertices,
                        uint32_t* max_out, uint32_t* max_in, uint64_t* version);

/* Device pointers of the current version's index (valid until the next
 * gj_apply_updates or gj_graph_destroy, or a call that merges rows appended
 * by log-structured updates): reverse = 0 forward, 1 reverse.  Merges such
 * rows first (on g's context).
 * row_ptr has vertices+1 entries, col and row have `edges` entries; row[e] is
 * the row (source for forward, destination for reverse) of entry e. */
gj_status gj_graph_csr(const gj_graph* g, int reverse, const uint32_t** row_ptr,
                       const uint32_t** col, const uint32_t** row);

/* Waits for the context's stream, then frees every version.  Before the
 * context is destroyed, and after any server on the graph. */
void gj_graph_destroy(gj_graph* g);

/* Materialises the triangle relation of g's current version for ternary
 * atoms (Sec. 5.4): for every edge (x, y) the sorted list out(x) & out(y),
 * as a CSR over forward edge positions with 64-bit row pointers (8 B per
 * edge + 4 B per triangle of device memory).  *num_triangles (may be NULL)
 * receives the relation's size.  Kept until gj_graph_destroy or the next
 * gj_apply_updates that changes the graph, which drops it. */
gj_status gj_graph_index_triangles(gj_ctx* ctx, gj_graph* g, uint64_t* num_triangles);

/* Old vertex id of every vertex id of g (num_vertices entries written to
 * old_of_new, a host or device array as out_on_device says): the renaming of
 * GJ_BUILD_DEGREE_ORDER, else the identity.  Match rows and update batches
 * use the graph's own ids. */
gj_status gj_graph_vertex_ids(const gj_graph* g, uint32_t* old_of_new, int out_on_device);

/* ---------------------------------------------------------------- queries */

/* atom = edge(a_src, a_dst) (Sec. 1.1: one atom per query edge) */
typedef struct {
  uint8_t src_attr, dst_attr;
} gj_atom;

/* Registers Q(a_0..a_{m-1}) := edge(...), ... with a global attribute order
 * (Sec. 2.2).  order is a permutation of 0..num_attrs-1.  P_2 is seeded from
 * the edges of the lowest-index atom over order[0], order[1] (Sec. 4.2).
 * Errors (GJ_EINVAL): num_attrs outside [2, 8]; num_atoms outside [1, 16];
 * an atom over one attribute twice or outside the attributes; order not a
 * permutation; no atom over order[0], order[1]; a later attribute with no
 * atom to an earlier one. */
gj_status gj_query_register(gj_ctx* ctx, uint32_t num_attrs, const gj_atom* atoms,
                            uint32_t num_atoms, const uint8_t* order, gj_query** out);

/* Inequality a_lo < a_hi between attribute values (symmetry breaking,
 * Sec. 5.4). */
typedef struct {
  uint8_t lo_attr, hi_attr;
} gj_less;
#define GJ_MAX_LESS 28

/* Ternary atom tri(a_x, a_y, a_z) over the triangle relation of the graph
 * (x -> y, x -> z and y -> z are edges; Sec. 5.4).  It binds a_z, which the
 * order must place after a_x and a_y; its extension set for a prefix is the
 * list of third vertices of the pair (x, y), read from the graph's triangle
 * index (gj_graph_index_triangles). */
typedef struct {
  uint8_t x_attr, y_attr, z_attr;
} gj_tri_atom;

/* gj_query_register plus inequalities every match must satisfy (less may be
 * NULL when num_less is 0).  Each is a filter on the prefixes, applied when
 * the later of its two attributes is bound (to the seed pair if both are the
 * first two); extension counters are those of the query without them.  With
 * one inequality per automorphism-equivalent pair of adjacent attributes, an
 * undirected (symmetric) graph yields each subgraph once instead of |Aut|
 * times.  Errors (GJ_EINVAL) as gj_query_register, and: num_less above
 * GJ_MAX_LESS, an attribute out of range, lo_attr == hi_attr. */
gj_status gj_query_register_ex(gj_ctx* ctx, uint32_t num_attrs, const gj_atom* atoms,
                               uint32_t num_atoms, const uint8_t* order, const gj_less* less,
                               uint32_t num_less, gj_query** out);

/* gj_query_register_ex plus ternary atoms (tris may be NULL when num_tris is
 * 0).  num_atoms + num_tris is at most GJ_MAX_ATOMS; P_2 is still seeded
 * from a binary atom over order[0], order[1].  A query with ternary atoms
 * runs only through gj_run, on a graph whose triangle index is current
 * (else GJ_EINVAL); gj_run_batch, the server and gj_apply_updates reject it
 * (GJ_EUNSUPPORTED).  Errors (GJ_EINVAL) as gj_query_register_ex, and: a
 * ternary atom over an attribute twice or out of range, or whose third
 * attribute is not after the other two in the order. */
gj_status gj_query_register_rel(gj_ctx* ctx, uint32_t num_attrs, const gj_atom* atoms,
                                uint32_t num_atoms, const gj_tri_atom* tris, uint32_t num_tris,
                                const uint8_t* order, const gj_less* less, uint32_t num_less,
                                gj_query** out);
void gj_query_destroy(gj_query* q);

/* Per-call counters.  prefixes[j] = |P_j| (j >= 2; prefixes[m] = matches),
 * extensions[j] = sum over p in P_j of the smallest extension-set size
 * (count-minimisation, Sec. 3.1), i.e. candidates proposed at stage j. */
typedef struct {
  uint64_t matches;
  uint64_t prefixes[GJ_MAX_ATTRS + 1];
  uint64_t extensions[GJ_MAX_ATTRS + 1];
  uint64_t noop_inserts;   /* gj_apply_updates: insertions of present edges */
  uint64_t noop_deletes;   /* gj_apply_updates: deletions of absent edges */
  uint64_t raw_emissions;  /* gj_apply_updates: signed rows before consolidation */
  uint64_t kernel_launches;/* launches of the propose+intersect kernels */
  double kernel_ms;        /* their summed device time (HIP events on the context stream) */
  double ms;               /* wall time of the call */
} gj_stats;

#define GJ_MODE_COUNT 0
#define GJ_MODE_ENUMERATE 1

/* Runs Generic Join (Sec. 2.2) in the edge-seeded form (Sec. 4.2) over seed
 * edges [seed_lo, seed_hi) of the seed atom's index (forward when the seed
 * atom is edge(order[0], order[1]), else reverse; clamped to the edge
 * count; 0, UINT64_MAX = all).
 * mode COUNT: stats->matches only (out may be NULL).
 * mode ENUMERATE: writes the matches to `out` as rows of num_attrs uint32,
 * columns in attribute-index order, rows sorted ascending (unsigned
 * lexicographic); `out` is device memory if out_on_device, else host.  If
 * more than out_cap_rows rows match, returns GJ_EOVERFLOW with
 * stats->matches = the required row count (buffer contents unspecified).
 * stats may be NULL. */
gj_status gj_run(gj_ctx* ctx, const gj_graph* g, const gj_query* q, int mode,
                 uint64_t seed_lo, uint64_t seed_hi, uint32_t* out,
                 uint64_t out_cap_rows, int out_on_device, gj_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): gj_run in
 * COUNT mode over seed edges [seed_lo, seed_hi) (clamped as gj_run), on the
 * depth-first per-candidate path, with every workspace buffer (frontiers,
 * minimum counts, scans, ballots, counters) taken from one static 64 MiB
 * device array per GPU instead of an allocation; no hipMalloc, hipFree or
 * allocating call is made.  frontier_cap is the batch bound B (Sec. 3.1.2):
 * prefixes per frontier and proposals per batch; 0 takes the largest power
 * of two whose buffers fit the array for this query (2^21 prefixes for two
 * attributes, 2^20 for three or four, 2^19 for five or six, 2^18 for seven
 * or eight); a larger value, or one below 64, is rejected with
 * GJ_EINVAL and a message naming the maximum.  Counts and counters equal
 * gj_run's (options "factorise" and "strategy" are ignored: it always
 * enumerates on the generic kernels; stats->kernel_ms is 0, no timing
 * events are created).  The array is shared by every call on that GPU and
 * keeps the last call's contents; calls on one GPU are serialised by a lock
 * in the library (a call returns once its kernels are done), so overlapping
 * calls wait rather than race.  Errors: GJ_EINVAL for a graph with rows
 * appended by log-structured updates that no static read has merged yet
 * (merging allocates), or without the triangle index a ternary atom needs. */
gj_status gj_count_noalloc(gj_ctx* ctx, const gj_graph* g, const gj_query* q, uint64_t seed_lo,
                           uint64_t seed_hi, uint64_t frontier_cap, gj_stats* stats);

/* Applies one signed update batch (sign +1 insert, -1 delete; host memory
 * unless on_device) as a new version of the graph, and returns for each of
 * the nq queries the change of its result (Delta-GJ, Sec. 3.3.1: the signed
 * union of the delta queries dQ_i, consolidated).
 * Batch normalisation: self-loops dropped; repeated rows collapse; inserting
 * a present edge / deleting an absent one is a no-op (counted in stats).
 * Errors (graph unchanged): GJ_EINVAL for an id >= num_vertices, a sign
 * other than +-1, or one edge both inserted and deleted in the batch.
 * count_delta[q]: signed change of the match count.
 * delta_rows / delta_sign (either array or any entry may be NULL: counts
 * only): per query, up to cap[q] rows of num_attrs uint32 in attribute order,
 * sorted ascending, with sign +1 (new match) or -1 (lost match); host memory
 * unless on_device.  n_delta[q] = number of consolidated rows; if it exceeds
 * cap[q] the call still applies the batch and returns GJ_EOVERFLOW.
 * stats may be NULL or an array of nq. */
gj_status gj_apply_updates(gj_ctx* ctx, gj_graph* g, const uint32_t* src,
                           const uint32_t* dst, const int8_t* sign, uint64_t b,
                           int on_device, const gj_query* const* qs, uint32_t nq,
                           int64_t* count_delta, uint32_t* const* delta_rows,
                           int8_t* const* delta_sign, const uint64_t* cap,
                           uint64_t* n_delta, gj_stats* stats);

/* ---------------------------------------------------------------- batches */

/* Counts nreq requests (query qs[i] over seed edges [seed_lo[i], seed_hi[i])
 * of its seed atom, as gj_run) on the current version in one fused pipeline:
 * every level of every request shares one count-minimisation, scan and
 * propose+intersect launch, with sizes kept in device memory, captured once
 * as a hipGraph and replayed (the synchronous dataflow primitive of
 * Sec. 3.1.1 over all requests).  counts[i] and stats[i] (stats may be NULL)
 * equal what gj_run(COUNT) returns for request i.  A level larger than
 * "batch_cap" prefixes makes the call fall back to one depth-first gj_run
 * per request (same results, bounded memory). */
gj_status gj_run_batch(gj_ctx* ctx, const gj_graph* g, uint32_t nreq, const gj_query* const* qs,
                       const uint64_t* seed_lo, const uint64_t* seed_hi, uint64_t* counts,
                       gj_stats* stats);

typedef struct {
  uint32_t batch_lin;          /* linear search below this extension-set size */
  uint32_t batch_waves_per_cu; /* waves per CU of the persistent grids */
  uint32_t batch_claim_words;  /* words of 64 candidates a fused-propose wave claims at a time */
  uint32_t hash_index;         /* membership tests: 1 per-row hash tables, 0 row searches */
  uint32_t propose_u;          /* lockstep width of the depth-first propose kernel */
  uint64_t batch_heavy;        /* work bound from which a request runs depth-first (0: all fused) */
  double best_ms;              /* wall time of the chosen configuration (-1: cached) */
  int configs_tried;
  int from_cache;
  uint32_t batch_run;          /* last stages grouped by prefix runs in the fused pipeline (0 or 1) */
  uint32_t run_ratio;          /* runs stream a prefix's set up to this many times the shared set */
} gj_tuning;

/* Tunes gj_run_batch on this batch by coordinate descent: the options
 * "hash_index" (0 or 1), "batch_lin" (0, 8, 32, 128), "batch_waves_per_cu"
 * (16, 32, 64), "batch_claim_words" (4, 16, 64), "batch_heavy" (0, 2^22,
 * 2^24, 2^26), "propose_u" (1, 2, 4), and the intersection strategy of the
 * last stages, "batch_run" (0, 1) and "run_ratio" (1, 2, 8), in turn, each value timed (wall time
 * of the whole call, best of two after a warm-up) with the others at their
 * best so far.  Keeps the fastest in ctx and, if cache_path is not NULL,
 * records it in that JSON file keyed by graph size and query set (a cached
 * key is reused without timing).  All configurations must agree on the
 * counts (else GJ_EDEVICE).  out may be NULL. */
gj_status gj_autotune(gj_ctx* ctx, const gj_graph* g, uint32_t nreq, const gj_query* const* qs,
                      const uint64_t* seed_lo, const uint64_t* seed_hi, const char* cache_path,
                      gj_tuning* out);

/* ---------------------------------------------------------------- serving */

/* A request server: worker threads that own ctx and g (make no other call on
 * them while the server exists) and serve count requests and update batches,
 * overlapped on the device.
 *
 * Updates are applied in arrival order on ctx and its stream, one version
 * each (count deltas through the fused delta queries).  A count request sees
 * every update submitted before it and none submitted after (the logical
 * sequencing of Sec. 4.3): it reads the resident version that holds that
 * state.  The server rotates the graph through up to "versions" resident
 * versions (default 4, each the size of the graph's indexes, allocated on
 * first use and kept until gj_graph_destroy), so counts of older versions run
 * while updates build newer ones; an update waits only while every other
 * version is still needed by a queued or running count.
 *
 * Counts run on contexts with their own streams that the server creates on
 * ctx's device (with ctx's options) -- one for light requests, and
 * "heavy_lanes" more (default 3, created at the first request) -- as
 * continuous batching: a request joins as soon as its version is resident;
 * its work is estimated from its seed edges (the exact level-3 extension
 * count per seed, times a bound for deeper levels, rescaled by what its
 * finished chunks did).  Light requests (at most iteration_work / 8
 * estimated extensions; iteration_work defaults to 2^24) run whole, shortest
 * first, up to max_batch and iteration_work per iteration and while their
 * estimated frontier memory (seed edges x average degree per later attribute
 * x bytes per prefix) stays within mem_budget_bytes (0: no limit), in one
 * fused pipeline per iteration (a request alone runs the depth-first path).
 * Heavy requests are cut into chunks of about "heavy_work" estimated
 * extensions (0, the default: 64 x iteration_work, so that a chunk's last
 * stage is large enough for the kernels that group prefix runs, see
 * "run_stage") that the heavy lanes run
 * concurrently on the depth-first path, each lane taking the oldest heavy
 * request no other lane is running.  Requests whose version an update waits
 * for go first; with "update_priority" (default 1) no new heavy chunk starts
 * while an update batch is on the device (light iterations go on).  Updates
 * run on ctx; the count-only delta queries of a batch with at least ctx's
 * "delta_lane_min" distinct changes run depth-first side by side on ctx and
 * "update_lanes" more contexts (default 2, created at the first request),
 * one host thread each; smaller batches take ctx alone.  With iteration_work
 * 0 requests run whole, in arrival order, in the fused pipeline.  Results
 * equal gj_run / gj_apply_updates issued alone in submission order.
 * Start-up: the light context's fused pipeline (levels of at most 2^24
 * prefixes, last stages grouped by runs in the small shape only, see
 * "run_big") is built as soon as the server is created, and ctx's delta
 * pipeline before the first update is served, so a caller that submits and
 * waits for an empty update batch before timing has every large allocation
 * behind it.
 * gj_server_create returns GJ_EDEVICE / GJ_ENOMEM if the light context or
 * the threads cannot be created; the first submit returns GJ_EDEVICE if no
 * heavy lane can be created. */
typedef struct gj_server gj_server;

#define GJ_REQ_COUNT 0
#define GJ_REQ_UPDATE 1
#define GJ_SERVER_MAX_QUERIES 16

typedef struct {
  int kind;          /* GJ_REQ_COUNT or GJ_REQ_UPDATE */
  gj_status status;  /* status of the underlying gj_run_batch / gj_apply_updates */
  uint64_t count;    /* count request: matches */
  uint32_t nq;       /* update: number of queries */
  int64_t count_delta[GJ_SERVER_MAX_QUERIES]; /* update: change of each query's count */
  uint64_t version;  /* graph version the request read (count) or left (update) */
  uint32_t batch_size; /* chunks in the step (fused iteration or heavy chunk) that finished it */
  int64_t submit_ns, start_ns, done_ns; /* steady-clock timestamps */
} gj_server_result;

typedef struct {
  uint64_t completed_counts, completed_updates;
  uint64_t count_batches;   /* scheduler steps: fused iterations and heavy chunks */
  double mean_count_batch;  /* chunks per step */
  double count_p50_ms, count_p99_ms;   /* submit -> done */
  double update_p50_ms, update_p99_ms;
} gj_server_stats;

gj_status gj_server_create(gj_ctx* ctx, gj_graph* g, uint32_t max_batch, uint64_t mem_budget_bytes,
                           gj_server** out);
/* Server options: "iteration_work" (>= 0), "heavy_work" (>= 0),
 * "update_priority" (0 or 1; 0 is experimental: under a mixed load of heavy
 * counts and updates it has stalled served requests for seconds),
 * "max_batch" (1..65536) at any time;
 * "versions" (2..8), "heavy_lanes" (1..4) and "update_lanes" (0..4) before
 * the first request, else GJ_EBUSY.  GJ_EINVAL for an unknown key or a value
 * out of range. */
gj_status gj_server_set_option(gj_server* s, const char* key, int64_t value);
/* Queues a count of query q over seed edges [seed_lo, seed_hi) (as gj_run);
 * *ticket identifies the result.  The query must outlive the request. */
gj_status gj_server_submit_count(gj_server* s, const gj_query* q, uint64_t seed_lo, uint64_t seed_hi,
                                 uint64_t* ticket);
/* Queues an update batch (host arrays, copied) and the queries (at most
 * GJ_SERVER_MAX_QUERIES) whose count deltas to report. */
gj_status gj_server_submit_update(gj_server* s, const uint32_t* src, const uint32_t* dst, const int8_t* sign,
                                  uint64_t b, const gj_query* const* qs, uint32_t nq, uint64_t* ticket);
/* Waits for a result (timeout_ms < 0: no limit; GJ_EBUSY on timeout).  A
 * result is returned once. */
gj_status gj_server_wait(gj_server* s, uint64_t ticket, int64_t timeout_ms, gj_server_result* out);
gj_status gj_server_get_stats(gj_server* s, gj_server_stats* out);
/* Serves everything queued, then stops the workers and frees the server's
 * own contexts.  Before its context, its graph or a query of its requests is
 * destroyed. */
void gj_server_destroy(gj_server* s);

/* Copies the consolidated delta rows of query number q (its position in the
 * qs list) of the most recent gj_apply_updates on ctx that requested rows
 * (non-NULL delta_rows or delta_sign for q): up to cap rows and signs, in
 * the layout gj_apply_updates uses, device memory if on_device else host.
 * *n receives the row count.  Lets a caller that got GJ_EOVERFLOW fetch the
 * rows without re-applying the batch.  The rows stay available until the
 * next gj_apply_updates on ctx.  Errors: GJ_EINVAL if q has no kept rows;
 * GJ_EOVERFLOW if *n > cap (nothing copied). */
gj_status gj_last_delta(gj_ctx* ctx, uint32_t q, uint32_t* rows, int8_t* signs,
                        uint64_t cap, int on_device, uint64_t* n);

/* ---------------------------------------------------------------- calibration */

/* Bandwidth peaks of ctx's device as measured by microbenchmark kernels, the
 * reference beside the published peaks when kernels are reported against
 * their roofline: *copy_gbs, a device-to-device copy of 2 GiB (bytes read +
 * written per second, 16-byte vector accesses; takes 4 GiB of device memory
 * through ctx's allocator for the call); *lds_gbs, 16-byte LDS reads at
 * conflict-free addresses by every lane of every CU.  Best of five timed
 * launches each.  Either pointer may be NULL to skip that measurement. */
gj_status gj_measure_peaks(gj_ctx* ctx, double* copy_gbs, double* lds_gbs);

#ifdef __cplusplus
}
#endif

#endif /* GJ_H */
