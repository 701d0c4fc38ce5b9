/*
 * Seeded synthetic workload generators: RMAT and Erdos-Renyi edge lists,
 * a seeded bijective vertex relabelling, and a seeded source picker.
 *
 * This module holds no BFS arithmetic. It is the single source of inputs for
 * both the GPU path and the CPU oracle, so that neither feeds the other.
 *
 * RMAT follows the paper's workload description (Section VI-A, "Reporting"):
 * scale N, 2^N vertices, edge factor 16, quadrant probabilities
 * A,B,C,D = 0.57,0.19,0.19,0.05, vertex IDs relabelled by a deterministic
 * hash after generation. The Graph500 generator itself is not reproduced:
 * this is plain recursive quadrant selection with fixed probabilities and no
 * per-level noise. Each (edge, level) pair takes one 32-bit uniform draw from
 * a counter-based SplitMix64 stream (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): the k-th output of a
 * SplitMix64 stream with state s is mix(s + (k+1)*gamma), so any draw can be
 * computed from its counter alone and generation parallelises trivially.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

/* SplitMix64 output function (the published finaliser). */
uint64_t inp_splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* k-th output (k >= 0) of the SplitMix64 stream whose initial state is seed. */
uint64_t inp_splitmix64_at(uint64_t seed, uint64_t k) {
  return inp_splitmix64_mix(seed + (k + 1) * GAMMA);
}

static int pick_threads(int nthreads) {
  if (nthreads > 0) return nthreads > 64 ? 64 : nthreads;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  if (c < 1) c = 1;
  if (c > 16) c = 16;
  return (int)c;
}

typedef struct {
  int scale;
  int64_t lo, hi;
  uint32_t t1, t2, t3;
  uint64_t seed;
  int32_t *src, *dst;
} rmat_job;

static void *rmat_worker(void *arg) {
  rmat_job *j = (rmat_job *)arg;
  const int N = j->scale;
  for (int64_t e = j->lo; e < j->hi; ++e) {
    uint32_t u = 0, v = 0;
    const uint64_t base = (uint64_t)e * 64u;
    for (int i = 0; i < N; ++i) {
      uint32_t r = (uint32_t)(inp_splitmix64_at(j->seed, base + (uint64_t)i) >> 32);
      uint32_t rb, cb;
      if (r < j->t1) { rb = 0; cb = 0; }
      else if (r < j->t2) { rb = 0; cb = 1; }
      else if (r < j->t3) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      u |= rb << (N - 1 - i);
      v |= cb << (N - 1 - i);
    }
    j->src[e] = (int32_t)u;
    j->dst[e] = (int32_t)v;
  }
  return NULL;
}

/*
 * RMAT edge list: num_edges directed pairs over [0, 2^scale), before
 * relabelling. Quadrant thresholds are floor(p * 2^32) of the cumulative
 * probabilities a, a+b, a+b+c. Returns 0, or -1 on a bad argument.
 */
int inp_rmat(int scale, int64_t num_edges, double a, double b, double c,
             uint64_t seed, int32_t *src, int32_t *dst, int nthreads) {
  if (scale < 1 || scale > 31 || num_edges < 0 || !src || !dst) return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  const double two32 = 4294967296.0;
  double c1 = a * two32, c2 = (a + b) * two32, c3 = (a + b + c) * two32;
  uint32_t t1 = c1 >= two32 ? 0xFFFFFFFFu : (uint32_t)c1;
  uint32_t t2 = c2 >= two32 ? 0xFFFFFFFFu : (uint32_t)c2;
  uint32_t t3 = c3 >= two32 ? 0xFFFFFFFFu : (uint32_t)c3;
  int T = pick_threads(nthreads);
  pthread_t th[64];
  rmat_job jobs[64];
  for (int t = 0; t < T; ++t) {
    jobs[t].scale = scale;
    jobs[t].lo = num_edges * t / T;
    jobs[t].hi = num_edges * (t + 1) / T;
    jobs[t].t1 = t1; jobs[t].t2 = t2; jobs[t].t3 = t3;
    jobs[t].seed = seed;
    jobs[t].src = src; jobs[t].dst = dst;
    pthread_create(&th[t], NULL, rmat_worker, &jobs[t]);
  }
  for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
  return 0;
}

/*
 * Seeded bijection on N-bit integers, used as the "deterministic hashing"
 * relabelling of vertex IDs. Each round is a bijection of [0, 2^N):
 * multiply by an odd constant mod 2^N, xor with a right shift of itself,
 * add a constant mod 2^N.
 */
typedef struct { uint64_t mul[4], add[4]; int shift; uint64_t mask; } perm_key;

static void perm_init(perm_key *k, int bits, uint64_t seed) {
  k->mask = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1ULL);
  k->shift = bits / 2 > 0 ? bits / 2 : 1;
  for (int r = 0; r < 4; ++r) {
    k->mul[r] = (inp_splitmix64_at(seed, (uint64_t)(2 * r)) | 1ULL) & k->mask;
    if (k->mul[r] == 0) k->mul[r] = 1;
    k->add[r] = inp_splitmix64_at(seed, (uint64_t)(2 * r + 1)) & k->mask;
  }
}

static inline uint64_t perm_apply(const perm_key *k, uint64_t x) {
  for (int r = 0; r < 4; ++r) {
    x = (x * k->mul[r]) & k->mask;
    x ^= x >> k->shift;
    x = (x + k->add[r]) & k->mask;
  }
  return x;
}

uint64_t inp_perm_value(int bits, uint64_t seed, uint64_t x) {
  perm_key k;
  perm_init(&k, bits, seed);
  return perm_apply(&k, x);
}

typedef struct { const perm_key *k; int64_t lo, hi; int32_t *src, *dst; } perm_job;

static void *perm_worker(void *arg) {
  perm_job *j = (perm_job *)arg;
  for (int64_t e = j->lo; e < j->hi; ++e) {
    j->src[e] = (int32_t)perm_apply(j->k, (uint32_t)j->src[e]);
    j->dst[e] = (int32_t)perm_apply(j->k, (uint32_t)j->dst[e]);
  }
  return NULL;
}

/* Relabel both endpoints of every edge in place through the N-bit bijection. */
int inp_permute(int bits, uint64_t seed, int32_t *src, int32_t *dst,
                int64_t num_edges, int nthreads) {
  if (bits < 1 || bits > 31 || num_edges < 0 || !src || !dst) return -1;
  perm_key k;
  perm_init(&k, bits, seed);
  int T = pick_threads(nthreads);
  pthread_t th[64];
  perm_job jobs[64];
  for (int t = 0; t < T; ++t) {
    jobs[t].k = &k;
    jobs[t].lo = num_edges * t / T;
    jobs[t].hi = num_edges * (t + 1) / T;
    jobs[t].src = src; jobs[t].dst = dst;
    pthread_create(&th[t], NULL, perm_worker, &jobs[t]);
  }
  for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
  return 0;
}

typedef struct { int32_t n; int64_t lo, hi; uint64_t seed; int32_t *src, *dst; } er_job;

static void *er_worker(void *arg) {
  er_job *j = (er_job *)arg;
  for (int64_t e = j->lo; e < j->hi; ++e) {
    uint64_t r = inp_splitmix64_at(j->seed, (uint64_t)e);
    uint64_t hi32 = r >> 32, lo32 = r & 0xFFFFFFFFULL;
    j->src[e] = (int32_t)((hi32 * (uint64_t)j->n) >> 32);
    j->dst[e] = (int32_t)((lo32 * (uint64_t)j->n) >> 32);
  }
  return NULL;
}

/*
 * Erdos-Renyi style edge list: num_pairs uniform (u, v) pairs drawn with
 * replacement over [0, n). Each pair uses one 64-bit draw; the high and low
 * 32-bit halves are scaled to [0, n) by a multiply-high.
 */
int inp_er(int32_t n, int64_t num_pairs, uint64_t seed, int32_t *src,
           int32_t *dst, int nthreads) {
  if (n < 1 || num_pairs < 0 || !src || !dst) return -1;
  int T = pick_threads(nthreads);
  pthread_t th[64];
  er_job jobs[64];
  for (int t = 0; t < T; ++t) {
    jobs[t].n = n;
    jobs[t].lo = num_pairs * t / T;
    jobs[t].hi = num_pairs * (t + 1) / T;
    jobs[t].seed = seed;
    jobs[t].src = src; jobs[t].dst = dst;
    pthread_create(&th[t], NULL, er_worker, &jobs[t]);
  }
  for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
  return 0;
}

/*
 * Seeded source picker: k distinct vertices, each an endpoint of at least one
 * pair (u, v) with u != v in the raw edge list (so it has degree >= 1 in the
 * simple symmetric graph). Candidates are scaled SplitMix64 draws, taken in
 * stream order and rejected if unsuitable or already chosen. Returns the
 * number of sources written (less than k only if too few vertices qualify),
 * or -1 on a bad argument / allocation failure.
 */
int64_t inp_pick_sources(const int32_t *src, const int32_t *dst, int64_t num_edges,
                         int32_t n, int64_t k, uint64_t seed, int32_t *out) {
  if (n < 1 || k < 0 || num_edges < 0 || !out || (num_edges > 0 && (!src || !dst)))
    return -1;
  uint8_t *ok = (uint8_t *)calloc((size_t)n, 1);
  if (!ok) return -1;
  int64_t eligible = 0;
  for (int64_t e = 0; e < num_edges; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v || u < 0 || v < 0 || u >= n || v >= n) continue;
    if (!ok[u]) { ok[u] = 1; ++eligible; }
    if (!ok[v]) { ok[v] = 1; ++eligible; }
  }
  int64_t want = k < eligible ? k : eligible, got = 0;
  const uint64_t max_draws = 64ULL * (uint64_t)n + 4096ULL;
  for (uint64_t j = 0; got < want && j < max_draws; ++j) {
    uint64_t r = inp_splitmix64_at(seed, j) >> 32;
    int32_t v = (int32_t)((r * (uint64_t)n) >> 32);
    if (ok[v] == 1) { ok[v] = 2; out[got++] = v; }
  }
  /* Draw budget spent (only when nearly every eligible vertex is wanted):
     take the remaining eligible vertices in ascending order. */
  for (int32_t v = 0; got < want && v < n; ++v)
    if (ok[v] == 1) { ok[v] = 2; out[got++] = v; }
  free(ok);
  return got;
}

/*
 * The same picker from a degree array: vertex v is eligible iff deg[v] > 0,
 * which for the simple symmetric graph of an edge list is exactly "endpoint
 * of a pair u != v", so both pickers return the same sources.
 */
int64_t inp_pick_sources_deg(const int32_t *deg, int32_t n, int64_t k, uint64_t seed,
                             int32_t *out) {
  if (n < 1 || k < 0 || !deg || !out) return -1;
  uint8_t *ok = (uint8_t *)calloc((size_t)n, 1);
  if (!ok) return -1;
  int64_t eligible = 0;
  for (int32_t v = 0; v < n; ++v)
    if (deg[v] > 0) { ok[v] = 1; ++eligible; }
  int64_t want = k < eligible ? k : eligible, got = 0;
  const uint64_t max_draws = 64ULL * (uint64_t)n + 4096ULL;
  for (uint64_t j = 0; got < want && j < max_draws; ++j) {
    uint64_t r = inp_splitmix64_at(seed, j) >> 32;
    int32_t v = (int32_t)((r * (uint64_t)n) >> 32);
    if (ok[v] == 1) { ok[v] = 2; out[got++] = v; }
  }
  for (int32_t v = 0; got < want && v < n; ++v)
    if (ok[v] == 1) { ok[v] = 2; out[got++] = v; }
  free(ok);
  return got;
}
