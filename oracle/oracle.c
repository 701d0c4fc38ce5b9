/*
 * CPU oracle for degree-separated, direction-optimized BFS.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link,
 * load or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code with the GPU library: it
 * builds its own adjacency, runs its own search and computes its own
 * statistics from the paper's definitions, written plainly and slowly.
 *
 * What it computes, and the passage each part follows:
 *  - G: the simple symmetric graph of an edge list. The paper assumes a
 *    symmetric graph (Section II-A, "graph") built by edge doubling
 *    (Section VI-A, "Reporting"); self-loops and duplicate edges are dropped
 *    (the paper is silent on both; simple-graph reading).
 *  - BFS depth = hop distance from the source (Section VI-A: the
 *    implementation outputs hop distances), found by a serial FIFO search.
 *    Direction optimization only changes the work, never the result
 *    (Section IV-B), so every GPU mode must reproduce exactly these depths.
 *  - parent: any neighbour one level shallower is valid; results are checked
 *    by invariants, not by equality (several trees are correct).
 *  - Degree separation (Section II-A "delegates"/"normal vertices",
 *    Section III-A): a vertex is a delegate iff its out-degree exceeds TH;
 *    delegates are renumbered 0..d-1 in ascending vertex ID (Fig. 2 caption).
 *  - The four edge classes nn, nd, dn, dd (Section II-A, Section IV) and the
 *    source list / masks used by the backward kernels (Section IV-B).
 *  - The direction decision of Section IV-B: forward workload FV (sum of
 *    neighbour-list lengths of the frontier), backward workload
 *    BV = |U|(q+s)/q, switch forward->backward when FV > factor0*BV and
 *    backward->forward when FV < factor1*BV, replayed level by level from
 *    the oracle's own depths.
 *  - Brute-force all-pairs shortest paths (Floyd-Warshall) and union-find
 *    components, built straight from the edge list, to pin the search.
 *  - The work model of a search (or_do_work, or_work_bytes): per level, the
 *    schedule of Section IV-B and the edges, candidates, scanned entries and
 *    candidate-set bytes of every visit, from the oracle's own level sets;
 *    this is the m' + d*b work bound of Section IV-B at p = 1, turned into
 *    the bytes the method must move.
 *
 * Parity status: every function here is pinned by tests against closed
 * forms, brute force or hand-derived values: the search by closed forms and
 * Floyd-Warshall, the exact-BV option by a brute-force expectation over
 * frontier subsets, the work model by hand-derived searches (one where the
 * stored row order changes the scan), closed forms of an all-forward search
 * and the per-level replay.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct or_graph {
  int32_t n;
  int64_t m;   /* directed edges (each undirected edge counted twice) */
  int64_t *off;
  int32_t *col;
} or_graph;

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2 };

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Adjacency of the simple symmetric graph: both directions of every pair with
 * u != v, rows sorted ascending, duplicates removed. Returns OR_OK or an error
 * (endpoint outside [0, n), allocation failure).
 */
int or_graph_build(const int32_t *src, const int32_t *dst, int64_t g, int32_t n,
                   or_graph **out) {
  if (!out || n < 1 || g < 0 || (g > 0 && (!src || !dst))) return OR_EINVAL;
  *out = NULL;
  for (int64_t e = 0; e < g; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return OR_EINVAL;

  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return OR_ENOMEM;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < g; ++e) {
    if (src[e] == dst[e]) continue;
    __atomic_fetch_add(&cnt[src[e]], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&cnt[dst[e]], 1, __ATOMIC_RELAXED);
  }
  int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!start) { free(cnt); return OR_ENOMEM; }
  start[0] = 0;
  for (int32_t v = 0; v < n; ++v) start[v + 1] = start[v] + cnt[v];
  int64_t total = start[n];
  int32_t *tmp = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  if (!tmp) { free(cnt); free(start); return OR_ENOMEM; }
  memset(cnt, 0, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < g; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    int64_t pu = __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
    int64_t pv = __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    tmp[start[u] + pu] = v;
    tmp[start[v] + pv] = u;
  }
  /* sort and de-duplicate each row in place; cnt[v] becomes the unique degree */
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t v = 0; v < n; ++v) {
    int32_t *row = tmp + start[v];
    int64_t len = start[v + 1] - start[v];
    if (len > 64) {
      qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
    } else {
      for (int64_t i = 1; i < len; ++i) {   /* insertion sort for short rows */
        int32_t x = row[i];
        int64_t j = i - 1;
        while (j >= 0 && row[j] > x) { row[j + 1] = row[j]; --j; }
        row[j + 1] = x;
      }
    }
    int64_t k = 0;
    for (int64_t i = 0; i < len; ++i)
      if (k == 0 || row[i] != row[k - 1]) row[k++] = row[i];
    cnt[v] = k;
  }
  or_graph *G = (or_graph *)calloc(1, sizeof(or_graph));
  int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!G || !off) { free(G); free(off); free(cnt); free(start); free(tmp); return OR_ENOMEM; }
  off[0] = 0;
  for (int32_t v = 0; v < n; ++v) off[v + 1] = off[v] + cnt[v];
  int64_t m = off[n];
  int32_t *col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!col) { free(G); free(off); free(cnt); free(start); free(tmp); return OR_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t v = 0; v < n; ++v)
    memcpy(col + off[v], tmp + start[v], (size_t)cnt[v] * sizeof(int32_t));
  free(cnt); free(start); free(tmp);
  G->n = n; G->m = m; G->off = off; G->col = col;
  *out = G;
  return OR_OK;
}

void or_graph_free(or_graph *G) {
  if (!G) return;
  free(G->off); free(G->col); free(G);
}
int32_t or_graph_n(const or_graph *G) { return G->n; }
int64_t or_graph_m(const or_graph *G) { return G->m; }
const int64_t *or_graph_off(const or_graph *G) { return G->off; }
const int32_t *or_graph_col(const or_graph *G) { return G->col; }

/*
 * Serial FIFO BFS from s: depth = hop distance (-1 if unreachable),
 * parent = the vertex that first discovered it (s for s, -1 if unreachable).
 * parent may be NULL.
 */
int or_bfs(const or_graph *G, int32_t s, int32_t *depth, int32_t *parent) {
  if (!G || !depth || s < 0 || s >= G->n) return OR_EINVAL;
  const int32_t n = G->n;
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!queue) return OR_ENOMEM;
  for (int32_t v = 0; v < n; ++v) depth[v] = -1;
  if (parent)
    for (int32_t v = 0; v < n; ++v) parent[v] = -1;
  int64_t head = 0, tail = 0;
  depth[s] = 0;
  if (parent) parent[s] = s;
  queue[tail++] = s;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t i = G->off[u]; i < G->off[u + 1]; ++i) {
      int32_t v = G->col[i];
      if (depth[v] < 0) {
        depth[v] = depth[u] + 1;
        if (parent) parent[v] = u;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return OR_OK;
}

/*
 * Brute force: Floyd-Warshall all-pairs hop distances on the simple symmetric
 * graph of the raw pairs, built straight from the edge list (no CSR), for
 * n <= 1024. dist is n*n row-major, -1 where unreachable.
 */
int or_apsp(int32_t n, const int32_t *src, const int32_t *dst, int64_t g, int32_t *dist) {
  if (n < 1 || n > 1024 || !dist || g < 0) return OR_EINVAL;
  const int32_t INF = 1 << 29;
  for (int64_t i = 0; i < (int64_t)n * n; ++i) dist[i] = INF;
  for (int32_t i = 0; i < n; ++i) dist[(int64_t)i * n + i] = 0;
  for (int64_t e = 0; e < g; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) return OR_EINVAL;
    if (u == v) continue;
    dist[(int64_t)u * n + v] = 1;
    dist[(int64_t)v * n + u] = 1;
  }
  for (int32_t k = 0; k < n; ++k)
    for (int32_t i = 0; i < n; ++i) {
      int32_t dik = dist[(int64_t)i * n + k];
      if (dik >= INF) continue;
      for (int32_t j = 0; j < n; ++j) {
        int32_t c = dik + dist[(int64_t)k * n + j];
        if (c < dist[(int64_t)i * n + j]) dist[(int64_t)i * n + j] = c;
      }
    }
  for (int64_t i = 0; i < (int64_t)n * n; ++i)
    if (dist[i] >= INF) dist[i] = -1;
  return OR_OK;
}

static int32_t uf_find(int32_t *p, int32_t x) {
  while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
  return x;
}

/*
 * Connected components by union-find over the raw pairs (no CSR).
 * label[v] = smallest vertex ID in v's component.
 */
int or_components(int32_t n, const int32_t *src, const int32_t *dst, int64_t g, int32_t *label) {
  if (n < 1 || !label || g < 0) return OR_EINVAL;
  int32_t *p = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!p) return OR_ENOMEM;
  for (int32_t v = 0; v < n; ++v) p[v] = v;
  for (int64_t e = 0; e < g; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) { free(p); return OR_EINVAL; }
    int32_t a = uf_find(p, u), b = uf_find(p, v);
    if (a == b) continue;
    if (a < b) p[b] = a; else p[a] = b;   /* root is always the smaller ID */
  }
  for (int32_t v = 0; v < n; ++v) label[v] = uf_find(p, v);
  free(p);
  return OR_OK;
}

static int has_edge(const or_graph *G, int32_t u, int32_t v) {
  int64_t lo = G->off[u], hi = G->off[u + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (G->col[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo < G->off[u + 1] && G->col[lo] == v;
}

/*
 * Invariants of a BFS result from s (checked on every run):
 *  1  depth[s] == 0 (and parent[s] == s when parents are given);
 *  2  every reached v != s has {parent[v], v} in E and
 *     depth[parent[v]] == depth[v] - 1;
 *  3  every edge {u, v} has both ends unreached or |depth[u]-depth[v]| <= 1;
 *  4  the reached set equals the component of s (label from or_components);
 *  5  unreached vertices carry depth -1 and parent -1; no depth below -1.
 * 1-4 together force depth[v] == dist(s, v). Returns 0 when all hold, else
 * the number of the first failed invariant; *bad gets the offending vertex.
 * parent and label may be NULL (their checks are skipped).
 */
int or_check_bfs(const or_graph *G, int32_t s, const int32_t *depth, const int32_t *parent,
                 const int32_t *label, int64_t *bad) {
  const int32_t n = G->n;
  int64_t dummy;
  if (!bad) bad = &dummy;
  *bad = -1;
  if (s < 0 || s >= n || !depth) return OR_EINVAL;
  if (depth[s] != 0 || (parent && parent[s] != s)) { *bad = s; return 1; }
  if (parent) {
    for (int32_t v = 0; v < n; ++v) {
      if (v == s || depth[v] < 0) continue;
      int32_t p = parent[v];
      if (p < 0 || p >= n || !has_edge(G, p, v) || depth[p] != depth[v] - 1) {
        *bad = v;
        return 2;
      }
    }
  }
  for (int32_t u = 0; u < n; ++u) {
    for (int64_t i = G->off[u]; i < G->off[u + 1]; ++i) {
      int32_t v = G->col[i];
      int32_t du = depth[u], dv = depth[v];
      if (du < 0 && dv < 0) continue;
      if (du < 0 || dv < 0 || du - dv > 1 || dv - du > 1) { *bad = u; return 3; }
    }
  }
  if (label) {
    for (int32_t v = 0; v < n; ++v) {
      int same = label[v] == label[s];
      if (same != (depth[v] >= 0)) { *bad = v; return 4; }
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    if (depth[v] < -1) { *bad = v; return 5; }
    if (depth[v] == -1 && parent && parent[v] != -1) { *bad = v; return 5; }
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Degree separation (Section II-A, Section III-A, Fig. 2 caption).        */
/* ---------------------------------------------------------------------- */

static inline int64_t or_deg(const or_graph *G, int32_t v) { return G->off[v + 1] - G->off[v]; }

typedef struct {
  int64_t n, m, d;
  int64_t e_nn, e_nd, e_dn, e_dd;
  int64_t n_ndsrc, n_ddsrc, n_dnsrc;
  int64_t max_deg;
} or_split_stats_t;

/*
 * Counts of the degree-separated layout at threshold TH: d = #{v: deg v > TH};
 * e_xy = directed edges u->v with class(u) = x, class(v) = y (n = normal,
 * d = delegate); ndsrc = normals with >= 1 delegate neighbour; ddsrc /
 * dnsrc = delegates with >= 1 delegate / normal neighbour (Section IV-B).
 */
int or_split_stats(const or_graph *G, int64_t TH, or_split_stats_t *st) {
  if (!G || !st) return OR_EINVAL;
  memset(st, 0, sizeof(*st));
  st->n = G->n;
  st->m = G->m;
  for (int32_t u = 0; u < G->n; ++u) {
    int64_t du = or_deg(G, u);
    if (du > st->max_deg) st->max_deg = du;
    int u_del = du > TH;
    if (u_del) st->d++;
    int64_t to_del = 0, to_norm = 0;
    for (int64_t i = G->off[u]; i < G->off[u + 1]; ++i) {
      int v_del = or_deg(G, G->col[i]) > TH;
      if (v_del) to_del++; else to_norm++;
    }
    if (u_del) {
      st->e_dd += to_del; st->e_dn += to_norm;
      if (to_del) st->n_ddsrc++;
      if (to_norm) st->n_dnsrc++;
    } else {
      st->e_nd += to_del; st->e_nn += to_norm;
      if (to_del) st->n_ndsrc++;
    }
  }
  return OR_OK;
}

/* Delegate IDs: did[v] = rank of v among delegates in ascending ID, else -1. */
int or_delegate_ids(const or_graph *G, int64_t TH, int32_t *did) {
  if (!G || !did) return OR_EINVAL;
  int32_t next = 0;
  for (int32_t v = 0; v < G->n; ++v) did[v] = or_deg(G, v) > TH ? next++ : -1;
  return OR_OK;
}

/*
 * The four subgraphs as separate CSRs, rows in ascending neighbour order:
 *   nn: rows 0..n-1 (empty for delegates), columns = vertex IDs of normals
 *   nd: rows 0..n-1 (empty for delegates), columns = delegate IDs
 *   dn: rows 0..d-1 (delegate IDs), columns = vertex IDs of normals
 *   dd: rows 0..d-1, columns = delegate IDs
 * Offsets arrays have n+1 or d+1 entries; column arrays are sized by the
 * e_xy counts of or_split_stats.
 */
int or_split_rows(const or_graph *G, int64_t TH, const int32_t *did,
                  int64_t *nn_off, int32_t *nn_col, int64_t *nd_off, int32_t *nd_col,
                  int64_t *dn_off, int32_t *dn_col, int64_t *dd_off, int32_t *dd_col) {
  if (!G || !did) return OR_EINVAL;
  int64_t a = 0, b = 0, c = 0, e = 0;
  int32_t k = 0;
  nn_off[0] = nd_off[0] = 0;
  dn_off[0] = dd_off[0] = 0;
  for (int32_t u = 0; u < G->n; ++u) {
    int u_del = or_deg(G, u) > TH;
    for (int64_t i = G->off[u]; i < G->off[u + 1]; ++i) {
      int32_t v = G->col[i];
      int v_del = or_deg(G, v) > TH;
      if (!u_del && !v_del) nn_col[a++] = v;
      else if (!u_del && v_del) nd_col[b++] = did[v];
      else if (u_del && !v_del) dn_col[c++] = v;
      else dd_col[e++] = did[v];
    }
    nn_off[u + 1] = a;
    nd_off[u + 1] = b;
    if (u_del) { dn_off[k + 1] = c; dd_off[k + 1] = e; ++k; }
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Direction decision replay (Section IV-B).                               */
/* ---------------------------------------------------------------------- */

/*
 * One term of the backward workload: the expected number of parents checked
 * before the first visited one, when each of od potential parents is visited
 * with probability a, i.e. the sum over i < od of (1-a)^i, in closed form
 * (1 - (1-a)^od) / a.
 */
double or_bv_term(double a, int64_t od) {
  if (od <= 0) return 0.0;
  if (a >= 1.0) return 1.0;
  return (1.0 - pow(1.0 - a, (double)od)) / a;
}

/* The paper's approximation of BV for large od: |U| (q + s) / q. */
double or_bv_approx(int64_t U, int64_t q, int64_t s) {
  if (q <= 0 || U <= 0) return 0.0;
  return (double)U * ((double)q + (double)s) / (double)q;
}

enum { K_DD = 0, K_DN = 1, K_ND = 2, K_NN = 3 };

typedef struct {
  int64_t q[3], s[3], U[3], FV[3];   /* per DO kernel dd, dn, nd */
  double BV[3];
  int32_t dir[3];                    /* direction used at this level: 0 fwd, 1 bwd */
  int64_t FV_nn, q_nn;               /* nn is always forward */
  int64_t frontier_normal, frontier_delegate;
} or_level_t;

/* One level of the schedule with nn under the direction decision too. */
typedef struct {
  int64_t q[4], s[4], U[4], FV[4];   /* dd, dn, nd, nn */
  double BV[4];
  int32_t dir[4];
  int64_t frontier_normal, frontier_delegate;
} or_level4_t;

/*
 * Replays the direction schedule of one search from the oracle's own depths,
 * for the kernels dd, dn, nd and nn. At level L (frontier = vertices at depth
 * L; visited = depth in [0, L]):
 *   dd: FV = sum of dd degrees of frontier delegates, q = frontier delegates
 *       with a dd edge, U = ddsrc minus visited, s = |U|;
 *   dn: FV = sum of dn degrees of frontier delegates, q = frontier delegates
 *       with a dn edge, U = ndsrc minus visited, s = |dnsrc minus visited|;
 *   nd: FV = sum of nd degrees of frontier normals, q = frontier normals
 *       with an nd edge, U = dnsrc minus visited, s = |ndsrc minus visited|;
 *   nn: FV = sum of nn degrees of frontier normals, q = frontier normals
 *       with an nn edge, U = normals with an nn edge minus visited, s = |U|
 *       (nn is symmetric at one GPU, like dd).
 * Section IV-B keeps nn forward (across GPUs nn is not symmetric); a factor0
 * of +infinity for nn reproduces that. If q == 0 the kernel has nothing to
 * do and keeps its direction; otherwise forward switches to backward when
 * FV > factor0*BV and backward switches to forward when FV < factor1*BV. BV
 * is |U|(q+s)/q (bv_exact == 0) or the sum of or_bv_term over U with od = the
 * degree in the reversed subgraph (bv_exact == 1). Writes at most max_levels
 * records; returns the number of levels with a non-empty frontier, or a
 * negative error.
 */
int or_do_replay4(const or_graph *G, int64_t TH, const int32_t *depth, const double *factor0,
                  const double *factor1, int bv_exact, or_level4_t *out, int max_levels) {
  if (!G || !depth || !factor0 || !factor1) return OR_EINVAL;
  const int32_t n = G->n;
  int32_t maxd = -1;
  for (int32_t v = 0; v < n; ++v) if (depth[v] > maxd) maxd = depth[v];
  int32_t dir[4] = {0, 0, 0, 0};
  int levels = maxd + 1;
  for (int32_t L = 0; L <= maxd; ++L) {
    or_level4_t r;
    memset(&r, 0, sizeof(r));
    double bvx[4] = {0, 0, 0, 0};
    for (int32_t v = 0; v < n; ++v) {
      int64_t dv = or_deg(G, v);
      int del = dv > TH;
      int64_t to_del = 0, to_norm = 0;
      for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i) {
        if (or_deg(G, G->col[i]) > TH) to_del++; else to_norm++;
      }
      int in_frontier = depth[v] == L;
      int unvisited = depth[v] < 0 || depth[v] > L;
      if (del) {
        if (in_frontier) {
          r.frontier_delegate++;
          r.FV[K_DD] += to_del;
          r.FV[K_DN] += to_norm;
          if (to_del) r.q[K_DD]++;
          if (to_norm) r.q[K_DN]++;
        }
        if (unvisited) {
          if (to_del) { r.U[K_DD]++; r.s[K_DD]++; }
          if (to_norm) { r.U[K_ND]++; r.s[K_DN]++; }
        }
      } else {
        if (in_frontier) {
          r.frontier_normal++;
          r.FV[K_ND] += to_del;
          r.FV[K_NN] += to_norm;
          if (to_del) r.q[K_ND]++;
          if (to_norm) r.q[K_NN]++;
        }
        if (unvisited && to_del) { r.U[K_DN]++; r.s[K_ND]++; }
        if (unvisited && to_norm) { r.U[K_NN]++; r.s[K_NN]++; }
      }
    }
    if (bv_exact) {
      for (int k = 0; k < 4; ++k) {
        if (r.q[k] == 0) continue;
        double a = (double)r.q[k] / ((double)r.q[k] + (double)r.s[k]);
        for (int32_t v = 0; v < n; ++v) {
          int64_t dv = or_deg(G, v);
          int del = dv > TH;
          if (!(depth[v] < 0 || depth[v] > L)) continue;
          int64_t to_del = 0, to_norm = 0;
          for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i) {
            if (or_deg(G, G->col[i]) > TH) to_del++; else to_norm++;
          }
          /* od(u) = degree of u in the reversed subgraph the backward kernel scans */
          if (k == K_DD && del && to_del) bvx[k] += or_bv_term(a, to_del);
          if (k == K_DN && !del && to_del) bvx[k] += or_bv_term(a, to_del);
          if (k == K_ND && del && to_norm) bvx[k] += or_bv_term(a, to_norm);
          if (k == K_NN && !del && to_norm) bvx[k] += or_bv_term(a, to_norm);
        }
      }
    }
    for (int k = 0; k < 4; ++k) {
      r.BV[k] = bv_exact ? bvx[k] : or_bv_approx(r.U[k], r.q[k], r.s[k]);
      if (r.q[k] > 0) {
        if (dir[k] == 0 && (double)r.FV[k] > factor0[k] * r.BV[k]) dir[k] = 1;
        else if (dir[k] == 1 && (double)r.FV[k] < factor1[k] * r.BV[k]) dir[k] = 0;
      }
      r.dir[k] = dir[k];
    }
    if (out && L < max_levels) out[L] = r;
  }
  return levels;
}

/*
 * The schedule of Section IV-B itself: dd, dn and nd under the decision, nn
 * always forward (or_do_replay4 with nn's factor0 at +infinity).
 */
int or_do_replay(const or_graph *G, int64_t TH, const int32_t *depth, const double *factor0,
                 const double *factor1, int bv_exact, or_level_t *out, int max_levels) {
  if (!G || !depth || !factor0 || !factor1) return OR_EINVAL;
  const double f0[4] = {factor0[0], factor0[1], factor0[2], INFINITY};
  const double f1[4] = {factor1[0], factor1[1], factor1[2], 0.0};
  or_level4_t *r4 = NULL;
  if (out && max_levels > 0) {
    r4 = (or_level4_t *)malloc((size_t)max_levels * sizeof(or_level4_t));
    if (!r4) return OR_ENOMEM;
  }
  int nl = or_do_replay4(G, TH, depth, f0, f1, bv_exact, r4, out ? max_levels : 0);
  for (int L = 0; r4 && L < nl && L < max_levels; ++L) {
    or_level_t *o = &out[L];
    for (int k = 0; k < 3; ++k) {
      o->q[k] = r4[L].q[k]; o->s[k] = r4[L].s[k]; o->U[k] = r4[L].U[k];
      o->FV[k] = r4[L].FV[k]; o->BV[k] = r4[L].BV[k]; o->dir[k] = r4[L].dir[k];
    }
    o->FV_nn = r4[L].FV[K_NN];
    o->q_nn = r4[L].q[K_NN];
    o->frontier_normal = r4[L].frontier_normal;
    o->frontier_delegate = r4[L].frontier_delegate;
  }
  free(r4);
  return nl;
}

/* ---------------------------------------------------------------------- */
/* Work model of one search: the bytes the method must move (algorithmic   */
/* bytes), level by level, for the schedule of Section IV-B.               */
/* ---------------------------------------------------------------------- */

/*
 * Log-scale degree bucket: eight buckets per power of two, from the position
 * of the leading one bit and the three bits below it, capped at 255.
 */
static int32_t or_deg_bucket(int64_t x) {
  if (x <= 1) return 0;
  int lg = 63 - __builtin_clzll((unsigned long long)x);
  int64_t frac = lg >= 3 ? (x >> (lg - 3)) & 7 : (x << (3 - lg)) & 7;
  int64_t b = (int64_t)lg * 8 + frac;
  return (int32_t)(b < 255 ? b : 255);
}

/*
 * The rows a backward scan reads, in the order it reads them (the paper fixes
 * only which edges each subgraph holds, Table I; the order inside a row is
 * the layout's choice, and a scan that stops at the first frontier neighbour
 * inspects a number of entries that depends on it):
 *   normal v:   its delegate neighbours (the nd part), by decreasing degree,
 *               ties by ascending ID;
 *   delegate u: its delegate neighbours (dd part), by decreasing degree
 *               bucket, ties by ascending ID, then its normal neighbours
 *               (dn part), ascending.
 * brow[v] .. brow[v+1] is the row; bmid[v] ends a delegate's dd part.
 */
typedef struct or_work_graph {
  const or_graph *G;
  int64_t TH;
  int32_t n;
  uint8_t *del;            /* 1 iff delegate (degree > TH) */
  int64_t *to_del, *to_norm;
  int64_t *brow, *bmid;
  int32_t *bcol;
  int64_t n_ndsrc, n_ddsrc, n_dnsrc, d;
} or_work_graph;

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

static int64_t or_max_deg(const or_graph *G) {
  int64_t mx = 0;
  for (int32_t v = 0; v < G->n; ++v) if (or_deg(G, v) > mx) mx = or_deg(G, v);
  return mx;
}

void or_work_free(or_work_graph *W) {
  if (!W) return;
  free(W->del); free(W->to_del); free(W->to_norm); free(W->brow); free(W->bmid); free(W->bcol);
  free(W);
}

int or_work_prepare(const or_graph *G, int64_t TH, or_work_graph **out) {
  if (!G || !out) return OR_EINVAL;
  *out = NULL;
  const int32_t n = G->n;
  or_work_graph *W = (or_work_graph *)calloc(1, sizeof(or_work_graph));
  if (!W) return OR_ENOMEM;
  W->G = G; W->TH = TH; W->n = n;
  W->del = (uint8_t *)malloc((size_t)n);
  W->to_del = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  W->to_norm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  W->brow = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  W->bmid = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  if (!W->del || !W->to_del || !W->to_norm || !W->brow || !W->bmid) {
    or_work_free(W);
    return OR_ENOMEM;
  }
  for (int32_t v = 0; v < n; ++v) W->del[v] = or_deg(G, v) > TH;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; ++v) {
    int64_t a = 0, b = 0;
    for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i) {
      if (W->del[G->col[i]]) a++; else b++;
    }
    W->to_del[v] = a;
    W->to_norm[v] = b;
  }
  for (int32_t v = 0; v < n; ++v) {
    if (W->del[v]) {
      W->d++;
      if (W->to_del[v]) W->n_ddsrc++;
      if (W->to_norm[v]) W->n_dnsrc++;
    } else if (W->to_del[v]) {
      W->n_ndsrc++;
    }
  }
  W->brow[0] = 0;
  for (int32_t v = 0; v < n; ++v)
    W->brow[v + 1] = W->brow[v] + (W->del[v] ? or_deg(G, v) : W->to_del[v]);
  W->bcol = (int32_t *)malloc((size_t)(W->brow[n] > 0 ? W->brow[n] : 1) * sizeof(int32_t));
  if (!W->bcol) { or_work_free(W); return OR_ENOMEM; }
  /* sort keys: the rank (decreasing degree, or decreasing degree bucket) in
     the high 32 bits, the vertex ID in the low 32 */
  const int64_t maxdeg = or_max_deg(G);
  int failed = 0;
#pragma omp parallel
  {
    uint64_t *key = (uint64_t *)malloc((size_t)(maxdeg > 0 ? maxdeg : 1) * sizeof(uint64_t));
    if (!key) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) {
      if (!key) continue;
      int32_t *row = W->bcol + W->brow[v];
      int64_t k = 0;
      for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i) {
        int32_t u = G->col[i];
        if (!W->del[u]) continue;
        uint64_t rank = W->del[v] ? (uint64_t)(255 - or_deg_bucket(or_deg(G, u)))
                                  : (uint64_t)(INT32_MAX - or_deg(G, u));
        key[k++] = (rank << 32) | (uint32_t)u;
      }
      qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
      for (int64_t i = 0; i < k; ++i) row[i] = (int32_t)(key[i] & 0xffffffffu);
      W->bmid[v] = W->brow[v] + k;
      if (W->del[v])   /* dn part: ascending, as the CSR row already is */
        for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i)
          if (!W->del[G->col[i]]) row[k++] = G->col[i];
    }
    free(key);
  }
  if (failed) { or_work_free(W); return OR_ENOMEM; }
  *out = W;
  return OR_OK;
}

/* Per level of one search: the schedule and the work of every visit. */
typedef struct {
  int64_t q[3], s[3], U[3], FV[3];   /* dd, dn, nd: the decision's inputs */
  double BV[3];
  int32_t dir[3];                    /* direction used (0 forward, 1 backward) */
  int32_t runs[5];                   /* visits with work: nd fwd, dd fwd, dn fwd, dn bwd, dd/nd bwd */
  int64_t f_norm, f_deleg;           /* frontier vertices with >= 1 edge */
  int64_t e_nn, e_nd, e_dd, e_dn;    /* edges expanded forward, per subgraph */
  int64_t c_dn, e_bu_dn;             /* backward dn: candidates, entries inspected */
  int64_t c_dd, e_bu_dd, c_nd, e_bu_nd;  /* backward dd / nd */
  int64_t c_deleg;                   /* delegate candidates of the backward dd/nd visit */
  int64_t s_dn, s_dd, s_nd;          /* candidate-set bytes scanned */
  int64_t cl_nn, cl_nd, cl_dd, cl_dn, cl_bu_dn, cl_bu_deleg;  /* first reached, by visit */
} or_work_level_t;

/*
 * The work of one search whose depths are `depth`, at threshold TH, with the
 * direction factors of Section IV-B (BV = |U|(q+s)/q). The decision's inputs
 * are the per-kernel definitions of or_do_replay, summed here from per-depth
 * histograms (every vertex is in exactly one level's frontier, and "not
 * visited at level L" is "total minus visited up to L"), so the schedule is
 * the same one in O(n + m) per search.
 *
 * Within a level the visits run in the order: nn forward (always, Section
 * IV-B), nd forward, dd and dn forward, dn backward, dd and nd backward (one
 * pass over the delegate candidates: the dd part first, then the dn part if
 * the dd part has no frontier neighbour). A vertex is first reached by the
 * first visit in that order that can reach it, and a backward visit's
 * candidates are the vertices of its source set not visited before the level
 * and not reached earlier in the level. A forward visit reads each edge of
 * its frontier's rows; a backward scan reads a candidate's row in stored
 * order up to and including its first frontier neighbour (the whole row if
 * there is none).
 *
 * Bytes (per level; the 8 bytes of output per vertex are counted where the
 * vertex is first reached, and by the initialization for unreached vertices):
 *   offsets 16 per frontier vertex with an edge, and 16 per backward
 *   candidate; 4 per edge expanded or entry inspected; candidate sets
 *   4|ndsrc| + n/8 (dn) and 2 d/8 (dd, nd) per backward visit that runs.
 * Returns the number of levels (max depth + 1) or a negative error.
 */
int or_do_work(const or_work_graph *W, const int32_t *depth, const double *factor0,
               const double *factor1, or_work_level_t *out, int max_levels) {
  if (!W || !depth || !factor0 || !factor1) return OR_EINVAL;
  const or_graph *G = W->G;
  const int32_t n = W->n;
  int32_t maxd = -1;
  for (int32_t v = 0; v < n; ++v) if (depth[v] > maxd) maxd = depth[v];
  const int32_t NL = maxd + 1;
  if (NL <= 0) return 0;
  /* per-depth histograms of the decision's inputs */
  int64_t *H = (int64_t *)calloc((size_t)NL * 12, sizeof(int64_t));
  if (!H) return OR_ENOMEM;
  enum { FVDD, FVDN, QDD, QDN, FVND, FVNN, QND, QNN, VDD, VDN, VND, FN };
  for (int32_t v = 0; v < n; ++v) {
    int32_t L = depth[v];
    if (L < 0) continue;
    int64_t *h = H + (size_t)L * 12;
    int64_t a = W->to_del[v], b = W->to_norm[v];
    if (W->del[v]) {
      h[FVDD] += a; h[FVDN] += b; h[QDD] += a > 0; h[QDN] += b > 0;
      h[VDD] += a > 0; h[VDN] += b > 0;
    } else {
      h[FVND] += a; h[FVNN] += b; h[QND] += a > 0; h[QNN] += b > 0;
      h[VND] += a > 0;
    }
  }
  int32_t dir[3] = {0, 0, 0};
  int64_t vis_dd = 0, vis_dn = 0, vis_nd = 0;   /* visited up to this level */
  for (int32_t L = 0; L < NL; ++L) {
    const int64_t *h = H + (size_t)L * 12;
    or_work_level_t r;
    memset(&r, 0, sizeof(r));
    vis_dd += h[VDD]; vis_dn += h[VDN]; vis_nd += h[VND];
    r.q[K_DD] = h[QDD]; r.q[K_DN] = h[QDN]; r.q[K_ND] = h[QND];
    r.FV[K_DD] = h[FVDD]; r.FV[K_DN] = h[FVDN]; r.FV[K_ND] = h[FVND];
    /* dd: U = ddsrc unvisited, s = |U|; dn: U = ndsrc unvisited, s = dnsrc
       unvisited; nd: U = dnsrc unvisited, s = ndsrc unvisited */
    r.U[K_DD] = W->n_ddsrc - vis_dd; r.s[K_DD] = r.U[K_DD];
    r.U[K_DN] = W->n_ndsrc - vis_nd; r.s[K_DN] = W->n_dnsrc - vis_dn;
    r.U[K_ND] = W->n_dnsrc - vis_dn; r.s[K_ND] = W->n_ndsrc - vis_nd;
    for (int k = 0; k < 3; ++k) {
      r.BV[k] = or_bv_approx(r.U[k], r.q[k], r.s[k]);
      if (r.q[k] > 0) {
        if (dir[k] == 0 && (double)r.FV[k] > factor0[k] * r.BV[k]) dir[k] = 1;
        else if (dir[k] == 1 && (double)r.FV[k] < factor1[k] * r.BV[k]) dir[k] = 0;
      }
      r.dir[k] = dir[k];
    }
    const int nd_fwd = dir[K_ND] == 0 && r.q[K_ND] > 0;
    const int dd_fwd = dir[K_DD] == 0 && r.q[K_DD] > 0;
    const int dn_fwd = dir[K_DN] == 0 && r.q[K_DN] > 0;
    const int dn_bwd = dir[K_DN] == 1 && r.q[K_DN] > 0 && r.U[K_DN] > 0;
    const int dd_bwd = dir[K_DD] == 1 && r.q[K_DD] > 0 && r.U[K_DD] > 0;
    const int nd_bwd = dir[K_ND] == 1 && r.q[K_ND] > 0 && r.U[K_ND] > 0;
    r.runs[0] = nd_fwd; r.runs[1] = dd_fwd; r.runs[2] = dn_fwd; r.runs[3] = dn_bwd;
    r.runs[4] = dd_bwd || nd_bwd;
    r.e_nn = h[FVNN];
    if (nd_fwd) r.e_nd = h[FVND];
    if (dd_fwd) r.e_dd = h[FVDD];
    if (dn_fwd) r.e_dn = h[FVDN];
    for (int32_t v = 0; v < n; ++v) {
      if (depth[v] != L) continue;
      if (W->del[v]) r.f_deleg += or_deg(G, v) > 0;
      else r.f_norm += or_deg(G, v) > 0;
    }
    /* first reach of every vertex at depth L + 1, and the backward scans */
    if (dn_bwd) r.s_dn = 4 * W->n_ndsrc + ((int64_t)n + 7) / 8;
    if (dd_bwd) r.s_dd = 2 * ((W->d + 7) / 8);
    if (nd_bwd) r.s_nd = 2 * ((W->d + 7) / 8);
    for (int32_t v = 0; v < n; ++v) {
      const int32_t dv = depth[v];
      if (dv >= 0 && dv <= L) continue;   /* visited before this level */
      int from_norm = 0, from_del = 0;     /* has a frontier neighbour of that class */
      if (dv == L + 1) {
        for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i) {
          int32_t u = G->col[i];
          if (depth[u] != L) continue;
          if (W->del[u]) from_del = 1; else from_norm = 1;
        }
      }
      if (!W->del[v]) {
        if (from_norm) { r.cl_nn++; continue; }          /* nn forward */
        if (dn_fwd && from_del) { r.cl_dn++; continue; }
        if (dn_bwd && W->to_del[v] > 0) {
          r.c_dn++;
          int64_t k = 0, hit = 0;
          for (int64_t i = W->brow[v]; i < W->brow[v + 1]; ++i) {
            ++k;
            if (depth[W->bcol[i]] == L) { hit = 1; break; }
          }
          r.e_bu_dn += k;
          if (hit) r.cl_bu_dn++;
        }
      } else {
        if (nd_fwd && from_norm) { r.cl_nd++; continue; }
        if (dd_fwd && from_del) { r.cl_dd++; continue; }
        const int scan_dd = dd_bwd && W->to_del[v] > 0, scan_dn = nd_bwd && W->to_norm[v] > 0;
        if (!scan_dd && !scan_dn) continue;
        r.c_deleg++;
        int hit = 0;
        if (scan_dd) {
          r.c_dd++;
          int64_t k = 0;
          for (int64_t i = W->brow[v]; i < W->bmid[v]; ++i) {
            ++k;
            if (depth[W->bcol[i]] == L) { hit = 1; break; }
          }
          r.e_bu_dd += k;
        }
        if (!hit && scan_dn) {
          r.c_nd++;
          int64_t k = 0;
          for (int64_t i = W->bmid[v]; i < W->brow[v + 1]; ++i) {
            ++k;
            if (depth[W->bcol[i]] == L) { hit = 1; break; }
          }
          r.e_bu_nd += k;
        }
        if (hit) r.cl_bu_deleg++;
      }
    }
    if (out && L < max_levels) out[L] = r;
  }
  free(H);
  return NL;
}

/*
 * Algorithmic bytes of a search from its work levels, per visit:
 *   [0] initialization: out_bytes per vertex never reached and for the source;
 *   [1] normal frontier (previsit and nn forward): 16 per frontier normal with
 *       an edge, 4 per nn edge, out_bytes per vertex first reached;
 *   [2] delegate frontier previsit: 16 per frontier delegate with an edge;
 *   [3] nd forward, [4] dd and dn forward: 4 per edge, out_bytes per vertex
 *       first reached;
 *   [5] dn backward, [6] dd and nd backward: 16 per candidate, 4 per entry
 *       inspected, the candidate-set bytes, out_bytes per vertex first reached.
 * out_bytes = 8 with parents (depth + parent), 4 without. launches[k] counts
 * the levels on which visit k had work (for [0], 1).
 */
int or_work_bytes(const or_work_level_t *lv, int nl, int64_t n, int out_bytes, double *bytes,
                  int64_t *launches) {
  if (!lv || nl < 0 || !bytes || !launches) return OR_EINVAL;
  for (int k = 0; k < 7; ++k) { bytes[k] = 0.0; launches[k] = 0; }
  const double ob = (double)out_bytes;
  int64_t reached = 1;
  for (int L = 0; L < nl; ++L) {
    const or_work_level_t *r = &lv[L];
    reached += r->cl_nn + r->cl_nd + r->cl_dd + r->cl_dn + r->cl_bu_dn + r->cl_bu_deleg;
    bytes[1] += 16.0 * r->f_norm + 4.0 * r->e_nn + ob * r->cl_nn;
    bytes[2] += 16.0 * r->f_deleg;
    bytes[3] += 4.0 * r->e_nd + ob * r->cl_nd;
    bytes[4] += 4.0 * (r->e_dd + r->e_dn) + ob * (r->cl_dd + r->cl_dn);
    bytes[5] += 16.0 * r->c_dn + 4.0 * r->e_bu_dn + (double)r->s_dn + ob * r->cl_bu_dn;
    bytes[6] += 16.0 * r->c_deleg + 4.0 * (r->e_bu_dd + r->e_bu_nd) + (double)(r->s_dd + r->s_nd) +
                ob * r->cl_bu_deleg;
    launches[1] += 1;
    launches[2] += 1;
    launches[3] += r->runs[0];
    launches[4] += r->runs[1] || r->runs[2];
    launches[5] += r->runs[3];
    launches[6] += r->runs[4];
  }
  bytes[0] = ob * (double)(n - reached + 1);
  launches[0] = 1;
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Work model of bit-parallel multi-source BFS (one batch).                */
/* ---------------------------------------------------------------------- */

/*
 * Bit-parallel multi-source BFS (Then et al., "The More the Merrier", PVLDB
 * 8(4), 2014; not in the paper): k <= 64 W sources are the lanes of W 64-bit
 * words per vertex. At level L, F[v] = the lanes first reaching v at depth L,
 * seen[v] = the lanes reaching v at depth <= L, live = the lanes with a
 * non-empty F. The next level is next[w] = (OR of F[u] over neighbours u)
 * and not seen[w]. A level runs top-down when its active vertices (F != 0)
 * number at most n * permille / 1000 (integer division), else bottom-up:
 *   top-down:  each active vertex reads its row: E = sum of their degrees,
 *              V = active vertices;
 *   bottom-up: each vertex with wanted = live and not seen[w] non-empty reads
 *              its row in stored order, ORing F of the entries, until the
 *              OR covers wanted (the whole row if it never does):
 *              E = entries read, V = such vertices.
 * Rows are read in stored order: neighbours by decreasing degree bucket,
 * ties by ascending ID (or_deg_bucket). Bytes of a level: 4 E (columns) +
 * 8 W E (lane sets of the entries) + 24 W V (seen, frontier and next of the
 * vertices) + 16 V (their row offsets); of the batch: the levels plus
 * 4 k n for the depth rows. depth (k x n, may be NULL) receives every lane's
 * hop distances (-1 unreached). Returns the number of levels run, or a
 * negative error.
 */
typedef struct {
  int64_t active, e, v;   /* active vertices; entries read; vertices processed */
  int32_t bottom_up;
  int32_t pad;
} or_ms_level_t;

int or_ms_work(const or_graph *G, const int32_t *sources, int32_t k, int32_t permille,
               int32_t *depth, or_ms_level_t *out, int max_levels, double *bytes) {
  if (!G || !sources || k < 1 || k > 256 || permille < 0 || permille > 1000 || !bytes)
    return OR_EINVAL;
  const int32_t n = G->n;
  const int W = (k + 63) / 64;
  for (int32_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= n) return OR_EINVAL;
  uint64_t *seen = (uint64_t *)calloc((size_t)n * W, sizeof(uint64_t));
  uint64_t *F = (uint64_t *)calloc((size_t)n * W, sizeof(uint64_t));
  uint64_t *nx = (uint64_t *)calloc((size_t)n * W, sizeof(uint64_t));
  int64_t *row = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int32_t *col = (int32_t *)malloc((size_t)(G->m > 0 ? G->m : 1) * sizeof(int32_t));
  if (!seen || !F || !nx || !row || !col) {
    free(seen); free(F); free(nx); free(row); free(col);
    return OR_ENOMEM;
  }
  /* rows in stored order */
  for (int32_t v = 0; v <= n; ++v) row[v] = G->off[v];
  int64_t maxdeg = or_max_deg(G);
  int failed = 0;
#pragma omp parallel
  {
    uint64_t *key = (uint64_t *)malloc((size_t)(maxdeg > 0 ? maxdeg : 1) * sizeof(uint64_t));
    if (!key) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) {
      if (!key) continue;
      int64_t len = G->off[v + 1] - G->off[v];
      for (int64_t i = 0; i < len; ++i) {
        int32_t u = G->col[G->off[v] + i];
        key[i] = ((uint64_t)(255 - or_deg_bucket(or_deg(G, u))) << 32) | (uint32_t)u;
      }
      qsort(key, (size_t)len, sizeof(uint64_t), cmp_u64);
      for (int64_t i = 0; i < len; ++i) col[G->off[v] + i] = (int32_t)(key[i] & 0xffffffffu);
    }
    free(key);
  }
  if (failed) {
    free(seen); free(F); free(nx); free(row); free(col);
    return OR_ENOMEM;
  }
  if (depth)
    for (int64_t i = 0; i < (int64_t)k * n; ++i) depth[i] = -1;
  for (int32_t i = 0; i < k; ++i) {
    int32_t s = sources[i];
    F[(size_t)s * W + i / 64] |= 1ull << (i % 64);
    seen[(size_t)s * W + i / 64] |= 1ull << (i % 64);
    if (depth) depth[(size_t)i * n + s] = 0;
  }
  const int64_t threshold = (int64_t)n * permille / 1000;
  double total = 4.0 * k * n;
  int L = 0;
  while (1) {
    uint64_t live[4] = {0, 0, 0, 0};
    int64_t active = 0;
    for (int32_t v = 0; v < n; ++v) {
      int any = 0;
      for (int w = 0; w < W; ++w) {
        live[w] |= F[(size_t)v * W + w];
        any |= F[(size_t)v * W + w] != 0;
      }
      active += any;
    }
    if (active == 0) break;
    const int bu = active > threshold;
    int64_t E = 0, V = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : E, V)
    for (int32_t x = 0; x < n; ++x) {
      uint64_t want[4], acc[4] = {0, 0, 0, 0};
      int wanted = 0;
      for (int w = 0; w < W; ++w) {
        want[w] = live[w] & ~seen[(size_t)x * W + w];
        wanted |= want[w] != 0;
      }
      /* top-down: an active vertex reads its whole row */
      if (!bu) {
        int act = 0;
        for (int w = 0; w < W; ++w) act |= F[(size_t)x * W + w] != 0;
        if (act) { E += row[x + 1] - row[x]; V += 1; }
      }
      int64_t read = 0;
      if (wanted) {
        for (int64_t i = row[x]; i < row[x + 1]; ++i) {
          int32_t u = col[i];
          int covered = 1;
          for (int w = 0; w < W; ++w) {
            acc[w] |= F[(size_t)u * W + w];
            covered &= (acc[w] & want[w]) == want[w];
          }
          ++read;
          if (covered) break;
        }
        if (bu) { E += read; V += 1; }
      }
      for (int w = 0; w < W; ++w) nx[(size_t)x * W + w] = acc[w] & want[w];
    }
    if (out && L < max_levels) {
      out[L].active = active;
      out[L].e = E;
      out[L].v = V;
      out[L].bottom_up = bu;
      out[L].pad = 0;
    }
    total += 4.0 * E + 8.0 * W * E + 24.0 * W * V + 16.0 * V;
    for (int32_t v = 0; v < n; ++v)
      for (int w = 0; w < W; ++w) {
        uint64_t b = nx[(size_t)v * W + w];
        seen[(size_t)v * W + w] |= b;
        F[(size_t)v * W + w] = b;
        if (depth)
          while (b) {
            int lane = w * 64 + __builtin_ctzll(b);
            b &= b - 1;
            depth[(size_t)lane * n + v] = L + 1;
          }
      }
    ++L;
  }
  *bytes = total;
  free(seen); free(F); free(nx); free(row); free(col);
  return L;
}

/* ---------------------------------------------------------------------- */
/* PageRank on the simple symmetric graph (another algorithm on the        */
/* degree-separated layout: delegates then hold multi-bit state, the       */
/* paper's future work, Sections VI-D and VII).                            */
/* ---------------------------------------------------------------------- */

/*
 * Power iteration in FP64, `iterations` steps from the uniform vector:
 *   D_t = sum of r_t[u] over vertices of degree 0 (their rank is spread
 *         uniformly);
 *   r_{t+1}[v] = (1 - alpha) / n + alpha * (D_t / n + sum over neighbours u
 *                of r_t[u] / deg(u)).
 * The sum over a vertex's neighbours is taken in ascending neighbour order.
 * rank receives r after the last step. Returns 0 or a negative error.
 */
int or_pagerank(const or_graph *G, double alpha, int32_t iterations, double *rank) {
  if (!G || !rank || iterations < 0 || !(alpha >= 0.0 && alpha <= 1.0)) return OR_EINVAL;
  const int32_t n = G->n;
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *c = (double *)malloc((size_t)n * sizeof(double));
  if (!r || !c) { free(r); free(c); return OR_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) r[v] = 1.0 / (double)n;
  for (int32_t t = 0; t < iterations; ++t) {
    double D = 0.0;
    for (int32_t u = 0; u < n; ++u) {
      int64_t du = or_deg(G, u);
      if (du == 0) { D += r[u]; c[u] = 0.0; }
      else c[u] = r[u] / (double)du;
    }
    for (int32_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int64_t i = G->off[v]; i < G->off[v + 1]; ++i) s += c[G->col[i]];
      r[v] = (1.0 - alpha) / (double)n + alpha * (D / (double)n + s);
    }
  }
  memcpy(rank, r, (size_t)n * sizeof(double));
  free(r);
  free(c);
  return OR_OK;
}
