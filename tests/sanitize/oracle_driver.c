/*
 * Calls every entry point of the CPU oracle on small random graphs (with
 * self-loops, duplicates and isolated vertices) so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer can check the oracle's
 * memory accesses and arithmetic. Exits 0 when every call succeeds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_graph or_graph;
typedef struct or_work_graph or_work_graph;
int or_graph_build(const int32_t *, const int32_t *, int64_t, int32_t, or_graph **);
void or_graph_free(or_graph *);
int or_bfs(const or_graph *, int32_t, int32_t *, int32_t *);
int or_apsp(int32_t, const int32_t *, const int32_t *, int64_t, int32_t *);
int or_components(int32_t, const int32_t *, const int32_t *, int64_t, int32_t *);
int or_check_bfs(const or_graph *, int32_t, const int32_t *, const int32_t *, const int32_t *,
                 int64_t *);
int or_split_stats(const or_graph *, int64_t, void *);
int or_delegate_ids(const or_graph *, int64_t, int32_t *);
int or_split_rows(const or_graph *, int64_t, const int32_t *, int64_t *, int32_t *, int64_t *,
                  int32_t *, int64_t *, int32_t *, int64_t *, int32_t *);
int or_do_replay(const or_graph *, int64_t, const int32_t *, const double *, const double *, int,
                 void *, int);
int or_do_replay4(const or_graph *, int64_t, const int32_t *, const double *, const double *,
                  int, void *, int);
int or_work_prepare(const or_graph *, int64_t, or_work_graph **);
void or_work_free(or_work_graph *);
int or_do_work(const or_work_graph *, const int32_t *, const double *, const double *, void *,
               int);
int or_work_bytes(const void *, int, int64_t, int, double *, int64_t *);
int or_ms_work(const or_graph *, const int32_t *, int32_t, int32_t, int32_t *, void *, int,
               double *);
int or_pagerank(const or_graph *, double, int32_t, double *);

static uint64_t state = 0x1234567;
static uint32_t next(void) {
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(state >> 33);
}

#define CHECK(x)                                              \
  do {                                                        \
    if ((x) < 0) {                                            \
      fprintf(stderr, "%s failed at line %d\n", #x, __LINE__); \
      return 1;                                               \
    }                                                         \
  } while (0)

int main(void) {
  static unsigned char levels[4096 * 512];   /* large enough for any level record array */
  for (int round = 0; round < 6; ++round) {
    const int32_t n = 40 + round * 37;
    const int64_t g = 3 * n;
    int32_t *src = malloc(g * sizeof(int32_t)), *dst = malloc(g * sizeof(int32_t));
    for (int64_t e = 0; e < g; ++e) {
      src[e] = (int32_t)(next() % (uint32_t)n);
      dst[e] = (e % 7 == 0) ? src[e] : (int32_t)(next() % (uint32_t)(n / 2 + 1));
    }
    or_graph *G = NULL;
    CHECK(or_graph_build(src, dst, g, n, &G));
    int32_t *depth = malloc(n * sizeof(int32_t)), *parent = malloc(n * sizeof(int32_t));
    int32_t *label = malloc(n * sizeof(int32_t)), *dist = malloc((size_t)n * n * sizeof(int32_t));
    CHECK(or_components(n, src, dst, g, label));
    CHECK(or_apsp(n, src, dst, g, dist));
    for (int32_t s = 0; s < n; s += 7) {
      int64_t bad = 0;
      CHECK(or_bfs(G, s, depth, parent));
      if (or_check_bfs(G, s, depth, parent, label, &bad) != 0) return 2;
      for (int64_t th = 0; th <= 8; th += 4) {
        const double f0[4] = {0.5, 0.05, 1e-7, 1e-3}, f1[4] = {0.0, 0.1, 0.0, 0.5};
        CHECK(or_do_replay(G, th, depth, f0, f1, s & 1, levels, 4096));
        CHECK(or_do_replay4(G, th, depth, f0, f1, s & 1, levels, 4096));
        or_work_graph *W = NULL;
        CHECK(or_work_prepare(G, th, &W));
        const int nl = or_do_work(W, depth, f0, f1, levels, 4096);
        CHECK(nl);
        double bytes[7];
        int64_t launches[7];
        CHECK(or_work_bytes(levels, nl, n, 8, bytes, launches));
        or_work_free(W);
      }
    }
    unsigned char st[128];
    int32_t *did = malloc(n * sizeof(int32_t));
    CHECK(or_split_stats(G, 3, st));
    CHECK(or_delegate_ids(G, 3, did));
    {
      const int64_t m = 2 * g;
      int64_t *o1 = calloc(n + 1, 8), *o2 = calloc(n + 1, 8), *o3 = calloc(n + 1, 8),
              *o4 = calloc(n + 1, 8);
      int32_t *c1 = calloc(m + 1, 4), *c2 = calloc(m + 1, 4), *c3 = calloc(m + 1, 4),
              *c4 = calloc(m + 1, 4);
      CHECK(or_split_rows(G, 3, did, o1, c1, o2, c2, o3, c3, o4, c4));
      free(o1); free(o2); free(o3); free(o4); free(c1); free(c2); free(c3); free(c4);
    }
    int32_t ms_src[130];
    for (int i = 0; i < 130; ++i) ms_src[i] = (int32_t)(next() % (uint32_t)n);
    int32_t *msd = malloc((size_t)130 * n * sizeof(int32_t));
    double b = 0;
    CHECK(or_ms_work(G, ms_src, 130, 20, msd, levels, 4096, &b));
    double *rank = malloc(n * sizeof(double));
    CHECK(or_pagerank(G, 0.85, 25, rank));
    double sum = 0;
    for (int32_t v = 0; v < n; ++v) sum += rank[v];
    if (fabs(sum - 1.0) > 1e-9) return 3;
    free(rank); free(msd); free(did); free(depth); free(parent); free(label); free(dist);
    free(src); free(dst);
    or_graph_free(G);
  }
  printf("oracle driver ok\n");
  return 0;
}
