/*
 * Seeded synthetic inputs for the subgraph-query workloads: R-MAT and
 * Erdos-Renyi edge lists and signed update batches.
 *
 * This file holds input generation only.  It performs no part of the join
 * (no dedupe, no indexing, no intersection): both the GPU library and the CPU
 * oracle receive the raw arrays produced here and normalise them on their own.
 *
 * Randomness is counter based.  The value number n of stream `key` is the
 * (n+1)-th output of SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) started from state `key`:
 * x = key + (n+1) * 0x9E3779B97F4A7C15, followed by the published
 * variant-13 finaliser.  Any draw can therefore be recomputed on its own.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

uint64_t synth_splitmix64(uint64_t key, uint64_t n) {
  uint64_t z = key + (n + 1) * GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Stream keys derived from a user seed and a stream tag. */
static uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return synth_splitmix64(seed ^ 0xD1B54A32D192ED03ULL, tag);
}

/* Quadrant thresholds as 32-bit fixed point: a draw u (uniform u32) picks
 * quadrant 0 if u < ta, 1 if u < tab, 2 if u < tabc, else 3. */
typedef struct { uint32_t ta, tab, tabc; } rmat_thr;

static rmat_thr make_thr(double a, double b, double c) {
  rmat_thr t;
  double s = 4294967296.0;
  double x;
  x = a * s;             t.ta   = x >= s ? 0xFFFFFFFFu : (uint32_t)x;
  x = (a + b) * s;       t.tab  = x >= s ? 0xFFFFFFFFu : (uint32_t)x;
  x = (a + b + c) * s;   t.tabc = x >= s ? 0xFFFFFFFFu : (uint32_t)x;
  return t;
}

/* One R-MAT draw number k of stream `key`: `scale` quadrant choices from the
 * most significant bit down.  Quadrant 1 (b) sets the destination bit,
 * quadrant 2 (c) the source bit, quadrant 3 (d) both.  Two levels use one
 * 64-bit value (its high and low 32-bit halves). */
static void rmat_one(uint64_t key, uint64_t k, int scale, rmat_thr t,
                     uint32_t* s_out, uint32_t* d_out) {
  uint32_t s = 0, d = 0;
  for (int l = 0; l < scale; l += 2) {
    uint64_t z = synth_splitmix64(key, k * 32u + (uint64_t)(l >> 1));
    for (int h = 0; h < 2 && l + h < scale; ++h) {
      uint32_t u = h == 0 ? (uint32_t)(z >> 32) : (uint32_t)z;
      uint32_t bit = 1u << (scale - 1 - (l + h));
      if (u < t.ta) {
      } else if (u < t.tab) {
        d |= bit;
      } else if (u < t.tabc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
  }
  *s_out = s;
  *d_out = d;
}

typedef struct {
  uint64_t key, lo, hi;
  int scale;
  rmat_thr t;
  uint32_t *src, *dst;
} rmat_job;

static void* rmat_worker(void* p) {
  rmat_job* j = (rmat_job*)p;
  for (uint64_t k = j->lo; k < j->hi; ++k)
    rmat_one(j->key, k, j->scale, j->t, &j->src[k - j->lo], &j->dst[k - j->lo]);
  return NULL;
}

/* Raw R-MAT draws [first, first+count) of stream (seed, tag 0).  Duplicates
 * and self-loops are kept: removing them is the consumer's job. */
void synth_rmat(int scale, uint64_t first, uint64_t count, double a, double b,
                double c, uint64_t seed, int threads, uint32_t* src,
                uint32_t* dst) {
  if (threads < 1) threads = 1;
  if (threads > 64) threads = 64;
  rmat_thr t = make_thr(a, b, c);
  uint64_t key = stream_key(seed, 0);
  pthread_t th[64];
  rmat_job jobs[64];
  uint64_t per = (count + threads - 1) / threads;
  int used = 0;
  for (int i = 0; i < threads; ++i) {
    uint64_t lo = (uint64_t)i * per, hi = lo + per;
    if (lo >= count) break;
    if (hi > count) hi = count;
    jobs[i].key = key;
    jobs[i].lo = first + lo;
    jobs[i].hi = first + hi;
    jobs[i].scale = scale;
    jobs[i].t = t;
    jobs[i].src = src + lo;
    jobs[i].dst = dst + lo;
    pthread_create(&th[i], NULL, rmat_worker, &jobs[i]);
    ++used;
  }
  for (int i = 0; i < used; ++i) pthread_join(th[i], NULL);
}

/* ---- open-addressing set of u64 keys (generator bookkeeping only) ---- */
typedef struct { uint64_t* slot; uint64_t mask; } u64set;

static int set_init(u64set* s, uint64_t expect) {
  uint64_t cap = 16;
  while (cap < expect * 2 + 16) cap <<= 1;
  s->slot = (uint64_t*)malloc(cap * sizeof(uint64_t));
  if (!s->slot) return -1;
  memset(s->slot, 0xFF, cap * sizeof(uint64_t));
  s->mask = cap - 1;
  return 0;
}
/* returns 1 if inserted, 0 if already present; key must not be ~0 */
static int set_add(u64set* s, uint64_t key) {
  uint64_t h = synth_splitmix64(0x5EED, key) & s->mask;
  while (s->slot[h] != ~0ULL) {
    if (s->slot[h] == key) return 0;
    h = (h + 1) & s->mask;
  }
  s->slot[h] = key;
  return 1;
}
static int set_has(const u64set* s, uint64_t key) {
  uint64_t h = synth_splitmix64(0x5EED, key) & s->mask;
  while (s->slot[h] != ~0ULL) {
    if (s->slot[h] == key) return 1;
    h = (h + 1) & s->mask;
  }
  return 0;
}

/* Erdos-Renyi style digraph: `m` distinct ordered pairs (u, v), u != v, each
 * endpoint uniform in [0, n) (multiply-high of a 32-bit half), drawn in
 * sequence from stream (seed, tag 1); repeats and self-loops are redrawn.
 * Returns the number of draws consumed, or 0 on failure. */
uint64_t synth_er(uint32_t n, uint64_t m, uint64_t seed, uint32_t* src,
                  uint32_t* dst) {
  if (n < 2 || m > (uint64_t)n * (n - 1)) return 0;
  u64set s;
  if (set_init(&s, m)) return 0;
  uint64_t key = stream_key(seed, 1), got = 0, k = 0;
  while (got < m) {
    uint64_t z = synth_splitmix64(key, k++);
    uint32_t u = (uint32_t)(((z >> 32) * (uint64_t)n) >> 32);
    uint32_t v = (uint32_t)(((z & 0xFFFFFFFFULL) * (uint64_t)n) >> 32);
    if (u == v) continue;
    if (!set_add(&s, ((uint64_t)u << 32) | v)) continue;
    src[got] = u;
    dst[got] = v;
    ++got;
  }
  free(s.slot);
  return k;
}

/* Size of update batch number `k` of stream (seed, tag 2): log-uniform in
 * [lo, hi], i.e. floor(lo * exp(U * ln((hi + 1) / lo))) clamped to [lo, hi]. */
uint64_t synth_batch_size(uint64_t seed, uint64_t k, uint64_t lo, uint64_t hi) {
  uint64_t z = synth_splitmix64(stream_key(seed, 2), k);
  double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  double s = floor((double)lo * exp(u * log(((double)hi + 1.0) / (double)lo)));
  if (s < (double)lo) s = (double)lo;
  if (s > (double)hi) s = (double)hi;
  return (uint64_t)s;
}

/* Update batch number `k` with `size` operations (stream (seed, tag 3+k)).
 * Each operation is a deletion with probability del_frac, else an insertion.
 * A deletion re-derives a uniformly chosen base R-MAT draw (index in
 * [0, base_draws) of the base stream base_seed); an insertion is a fresh R-MAT
 * draw of stream (seed, tag 0) at index k * 2^32 + 64 * i + r, where r counts
 * redraws after a self-loop (at most 64 tries, then the operation is dropped).  Within the batch, repeated operations collapse and an insertion
 * equal to one of the batch's deletions is dropped, so the batch never both
 * inserts and deletes one edge.  Writes at most `size` rows and returns the
 * number written.  Whether an operation changes the graph (a deletion of an
 * absent edge, an insertion of a present one) is left to the consumer. */
uint64_t synth_update_batch(int scale, double a, double b, double c,
                            uint64_t base_seed, uint64_t base_draws,
                            uint64_t seed, uint64_t k, uint64_t size,
                            double del_frac, uint32_t* src, uint32_t* dst,
                            int8_t* sign) {
  rmat_thr t = make_thr(a, b, c);
  uint64_t base_key = stream_key(base_seed, 0);
  uint64_t ins_key = stream_key(seed, 0);
  uint64_t op_key = stream_key(seed, 3 + k);
  uint32_t del_thr;
  {
    double x = del_frac * 4294967296.0;
    del_thr = x >= 4294967296.0 ? 0xFFFFFFFFu : (uint32_t)x;
  }
  u64set dels, ins;
  if (set_init(&dels, size) || set_init(&ins, size)) return 0;
  /* first pass: decide kinds, collect deletions */
  uint8_t* kind = (uint8_t*)malloc(size ? size : 1);
  uint32_t* us = (uint32_t*)malloc((size ? size : 1) * sizeof(uint32_t));
  uint32_t* vs = (uint32_t*)malloc((size ? size : 1) * sizeof(uint32_t));
  uint64_t ctr = 0;
  for (uint64_t i = 0; i < size; ++i) {
    uint64_t z = synth_splitmix64(op_key, ctr++);
    int is_del = (uint32_t)(z >> 32) < del_thr;
    uint32_t u = 0, v = 0;
    int ok = 0;
    if (is_del) {
      for (int tries = 0; tries < 64 && !ok; ++tries) {
        uint64_t r = synth_splitmix64(op_key, ctr++);
        uint64_t idx = (uint64_t)(((unsigned __int128)r * base_draws) >> 64);
        rmat_one(base_key, idx, scale, t, &u, &v);
        ok = u != v;
      }
      if (ok) set_add(&dels, ((uint64_t)u << 32) | v);
    } else {
      for (uint64_t sub = 0; sub < 64 && !ok; ++sub) {
        rmat_one(ins_key, (k << 32) + i * 64 + sub, scale, t, &u, &v);
        ok = u != v;
      }
    }
    /* 0 = insert, 1 = delete, 2 = no loop-free draw found: dropped */
    kind[i] = ok ? (uint8_t)is_del : 2;
    us[i] = u;
    vs[i] = v;
  }
  uint64_t out = 0;
  u64set seen_del;
  set_init(&seen_del, size);
  for (uint64_t i = 0; i < size; ++i) {
    uint64_t key = ((uint64_t)us[i] << 32) | vs[i];
    if (kind[i] == 2) continue;
    if (kind[i]) {
      if (!set_add(&seen_del, key)) continue;
      src[out] = us[i]; dst[out] = vs[i]; sign[out] = -1; ++out;
    } else {
      if (set_has(&dels, key)) continue;
      if (!set_add(&ins, key)) continue;
      src[out] = us[i]; dst[out] = vs[i]; sign[out] = 1; ++out;
    }
  }
  free(kind); free(us); free(vs);
  free(dels.slot); free(ins.slot); free(seen_del.slot);
  return out;
}
