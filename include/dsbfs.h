/*
 * dsbfs: degree-separated, direction-optimized breadth-first search for one
 * AMD Instinct MI355X (gfx950).
 *
 * The method is that of Pan, Pearce and Owens, "Scalable Breadth-First Search
 * on a GPU Cluster" (arXiv 1803.03922), for one GPU's share of the graph:
 * vertices are separated by degree into delegates (degree > TH) and normal
 * vertices (Section III-A), edges are stored as four subgraphs nn, nd, dn, dd
 * with 32-bit local IDs (Section III-C, Table I), and each BFS level chooses
 * top-down or bottom-up traversal per subgraph from a workload comparison
 * (Section IV-B). On top of it: bit-parallel multi-source BFS (64 sources per
 * batch as lanes of a 64-bit mask per vertex) and a continuous-batching query
 * server.
 *
 * Conventions for every function below:
 *  - Every function returns a dsbfs_status: 0 on success, a negative code on
 *    failure. No function throws or aborts across this boundary. The message
 *    of the last failure on the calling thread is dsbfs_last_error().
 *  - Vertex IDs are int32 in [0, n) with n <= 2^31 - 1; edge counts are int64.
 *  - "stream" is a hipStream_t passed as void* (NULL = the legacy default
 *    stream). Device work of a call is ordered on that stream. Calls that
 *    return results on the host synchronize the stream before returning.
 *  - Device pointers are plain device (HBM) addresses, host pointers are
 *    plain host addresses; no framework types cross this boundary.
 *  - A graph is immutable after creation: concurrent searches on one graph
 *    with distinct workspaces and streams are safe. A workspace is used by
 *    one call at a time.
 */
#ifndef DSBFS_H
#define DSBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dsbfs_status;

enum {
  DSBFS_OK = 0,
  DSBFS_ERR_INVALID_ARG = -1,   /* bad pointer, size, vertex ID or option */
  DSBFS_ERR_RANGE = -2,         /* a size does not fit the layout's integer widths */
  DSBFS_ERR_OUT_OF_MEMORY = -3, /* the allocator returned NULL */
  DSBFS_ERR_BUDGET = -4,        /* server admission refused: HBM budget exhausted */
  DSBFS_ERR_HIP = -5,           /* a HIP runtime call failed (message kept) */
  DSBFS_ERR_NOT_READY = -6,     /* server wait timed out */
  DSBFS_ERR_DEVICE = -7         /* a kernel reported an internal failure */
};

/*
 * Device memory provider. alloc returns a device pointer of at least `bytes`
 * bytes usable on `stream`, or NULL; free releases one. Passing NULL for the
 * allocator everywhere below means hipMalloc / hipFree. The library keeps the
 * pointer it was given for the lifetime of the objects created with it.
 */
typedef struct dsbfs_allocator {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*free)(void *ctx, void *ptr, void *stream);
} dsbfs_allocator;

/* Options of graph construction. */
typedef struct dsbfs_build_opts {
  int32_t threshold;       /* TH >= 0: a vertex is a delegate iff degree > TH
                              (Section II-A, "delegates"; Section III-A) */
  int32_t edges_on_device; /* 1: src/dst are device pointers; 0: host pointers */
  int32_t keep_plain_csr;  /* 1: keep the plain CSR too (needed by mode 0 and by
                              multi-source BFS); 0: free it after the split */
  int32_t skip_nn_copy;    /* 0 (default): build the compact copy of the nn
                              parts that the forward nn visit reads (arrays 18
                              and 19 of dsbfs_graph_export, 4 n + 8 e_nn bytes);
                              1: do not, and read the packed offsets and rows */
} dsbfs_build_opts;

/* Sizes of a built graph. Degrees are counted after symmetrization,
   self-loop removal and de-duplication. */
typedef struct dsbfs_graph_stats {
  int64_t n;          /* vertices */
  int64_t m_dir;      /* directed edges (twice the undirected simple edges) */
  int64_t d;          /* delegates */
  int64_t e_nn, e_nd, e_dn, e_dd; /* directed edges per class (Section II-A) */
  int64_t n_ndsrc;    /* normal vertices with a delegate neighbour (Section IV-B) */
  int64_t n_ddsrc;    /* delegates with a delegate neighbour */
  int64_t n_dnsrc;    /* delegates with a normal neighbour */
  int64_t max_degree;
  int64_t bytes_layout; /* device bytes of the degree-separated layout */
  int64_t bytes_plain;  /* device bytes of the plain CSR (0 if not kept) */
  int32_t threshold;
  int32_t reserved;
  int64_t n_nnsrc;      /* normal vertices with a normal neighbour */
} dsbfs_graph_stats;

/*
 * Direction-switch factors printed in Section VI-B for (dd, dn, nd), tuned
 * there for the paper's layout and GPUs. The library's defaults differ (see
 * dsbfs_run_opts.factor0); pass these to reproduce the paper's schedule.
 */
#define DSBFS_PAPER_FACTOR0_DD 0.5
#define DSBFS_PAPER_FACTOR0_DN 0.05
#define DSBFS_PAPER_FACTOR0_ND 1e-7

/* Per-search options. */
typedef struct dsbfs_run_opts {
  int32_t mode;         /* 0: plain top-down BFS on the plain CSR;
                           1: degree-separated direction-optimized BFS */
  int32_t want_parent;  /* 1: write parent[] as well as depth[] */
  double factor0[3];    /* forward->backward switch factors for dd, dn, nd
                           (Section IV-B). Defaults 0.02, 0.001, 1e-6: a joint
                           sweep on this layout (rows ordered by decreasing
                           neighbour degree, so bottom-up finds a parent
                           sooner than the paper's BV model assumes) on
                           RMAT scale 26, TH 32. The paper's values are the
                           DSBFS_PAPER_FACTOR0_* constants. */
  double factor1[3];    /* backward->forward switch factors; default 0 */
  int32_t forced;       /* direction schedule: 0 heuristic (Section IV-B);
                           1 always forward; 2 backward wherever possible from
                           level 1 on; 3 seeded random per level and kernel.
                           Depths never depend on it (Section IV-B). */
  int32_t profile;      /* 1: time every kernel launch with HIP events on the
                           call's stream and report per-kernel totals in stats */
  uint64_t forced_seed; /* seed of schedule 3 */
  int32_t nn_do;        /* 1: nn under the direction decision too, with its own
                           bottom-up visit (a variant: Section IV-B keeps nn
                           forward because across GPUs nn is not symmetric; at
                           one GPU it is). The normal previsit then only counts
                           and a separate pass expands nn forward. Default 0. */
  int32_t reserved;
  double factor0_nn;    /* nn's forward->backward factor when nn_do (default 1e-3) */
  double factor1_nn;    /* nn's backward->forward factor when nn_do (default 0) */
} dsbfs_run_opts;

/* Fills *o with the defaults listed above (mode 1, parents on). */
dsbfs_status dsbfs_run_opts_default(dsbfs_run_opts *o);

/* One BFS level of a mode-1 search: the inputs of the direction decision
   (Section IV-B) for the three kernels with direction optimization, indexed
   dd = 0, dn = 1, nd = 2, and the work the level's kernels did. */
typedef struct dsbfs_level_stats {
  int64_t q[3];      /* frontier vertices with an edge in that subgraph */
  int64_t s[3];      /* unvisited sources in the forward subgraph */
  int64_t U[3];      /* unvisited sources of the reversed subgraph */
  int64_t FV[3];     /* forward workload: frontier neighbour-list lengths */
  double BV[3];      /* backward workload |U|(q+s)/q */
  int32_t dir[3];    /* direction taken: 0 forward, 1 backward */
  int32_t reserved;
  int64_t FV_nn, q_nn;               /* nn's workload and frontier */
  int64_t frontier_normal, frontier_delegate;
  double kernel_ms[11]; /* profile = 1 only: HIP-event time of each kernel of
                           this level (indexed DSBFS_K_*), 0 when it had no
                           work; all 0 without profiling */
  int64_t U_nn, s_nn;   /* nn_do: unvisited normals with an nn edge (both) */
  double BV_nn;         /* nn_do: nn's backward workload */
  int32_t dir_nn;       /* direction nn took (always 0 without nn_do) */
  int32_t reserved2;
} dsbfs_level_stats;

/* Kernels of a search, for per-kernel profiles. */
enum {
  DSBFS_K_INIT = 0,        /* depth/parent fill and bitmap clear */
  DSBFS_K_PREV_NORMAL = 1, /* previsit of the normal queue fused with its
                              top-down nn visit (with nn_do: previsit only) */
  DSBFS_K_PREV_DELEG = 2,  /* previsit of the delegate frontier mask */
  DSBFS_K_TD_NORMAL = 3,   /* top-down nd from the normal queue */
  DSBFS_K_TD_DELEG = 4,    /* top-down dd and/or dn from the delegate frontier */
  DSBFS_K_BU_NORMAL = 5,   /* bottom-up dn over the nd source list */
  DSBFS_K_BU_DELEG = 6,    /* bottom-up dd and/or nd over unvisited delegates */
  DSBFS_K_CLOSE = 7,       /* level close */
  DSBFS_K_PLAIN = 8,       /* mode 0: length, scan and expansion of one level */
  DSBFS_K_TD_NN = 9,       /* nn_do: top-down nn from the normal queue */
  DSBFS_K_BU_NN = 10,      /* nn_do: bottom-up nn over normals with an nn edge */
  DSBFS_NUM_KERNELS = 11
};

/* Per-kernel totals of one search. bytes is the algorithmic HBM traffic of the
   work the kernel did, from counts the kernel itself keeps: 4 B per queue or
   list entry read or written, 16 B per pair of 64-bit row offsets, 4 B per
   adjacency entry read, 4 B per depth (+4 B per parent) written or filled,
   4 B per delegate ID translated; bitmaps (at most n/8 bytes, cache
   resident) are not counted. */
typedef struct dsbfs_kernel_profile {
  double ms;          /* sum of HIP-event durations of its launches (profile=1) */
  int64_t launches;
  int64_t bytes;      /* algorithmic bytes over all its launches */
  int64_t edges;      /* adjacency entries it read */
} dsbfs_kernel_profile;

/* Summary of one search. levels[] is caller memory of `capacity` records;
   the first min(num_levels, capacity) are filled (mode 1 only). */
typedef struct dsbfs_run_stats {
  int32_t num_levels;   /* levels with a non-empty frontier */
  int32_t capacity;
  dsbfs_level_stats *levels;
  int64_t reached;      /* vertices with depth >= 0 */
  int64_t edges_cc;     /* undirected simple edges in the source's component */
  dsbfs_kernel_profile kernels[DSBFS_NUM_KERNELS];
} dsbfs_run_stats;

typedef struct dsbfs_graph dsbfs_graph;
typedef struct dsbfs_workspace dsbfs_workspace;
typedef struct dsbfs_server dsbfs_server;

/*
 * Builds the graph on the device from an edge list of num_edges pairs
 * (src[i], dst[i]): the simple symmetric graph on [0, num_vertices) (the
 * paper assumes a symmetric graph made by edge doubling, Section II-A and
 * Section VI-A; self-loops and duplicates are dropped), then the degree
 * separation at opts->threshold: delegate IDs in ascending vertex ID
 * (Fig. 2 caption), the four subgraphs nn/nd/dn/dd (Section III-C), the nd
 * source list and the dd/dn source masks (Section IV-B).
 * Ownership: the caller keeps src/dst (copied); the graph owns its device
 * memory, taken from `alloc` (NULL = hipMalloc). Synchronizes `stream`.
 * Errors: INVALID_ARG (null pointer, num_vertices < 1, num_edges < 0, an
 * endpoint outside [0, n), threshold < 0), RANGE (a row too long for the
 * packed offsets), OUT_OF_MEMORY, HIP.
 */
dsbfs_status dsbfs_graph_create(const int32_t *src, const int32_t *dst, int64_t num_edges,
                                int32_t num_vertices, const dsbfs_build_opts *opts,
                                const dsbfs_allocator *alloc, void *stream, dsbfs_graph **out);

/* Sizes of a graph (host struct). */
dsbfs_status dsbfs_graph_stats_get(const dsbfs_graph *g, dsbfs_graph_stats *out);

/*
 * Copies one array of the device layout to host memory, for inspection and
 * tests. `which`: 0 degree int32[n]; 1 delegate ID int32[n] (-1 for normal);
 * 2 vertex of each delegate int32[d]; 3 normal row offsets uint64[n+1];
 * 4 normal columns int32[]; 5 delegate row offsets uint64[d+1]; 6 delegate
 * columns int32[]; 7 nd source list int32[n_ndsrc]; 8 dd source mask
 * uint32[ceil(d/32)]; 9 dn source mask uint32[ceil(d/32)]; 10 plain CSR
 * offsets int64[n+1]; 11 plain CSR columns int32[m_dir] (each row ordered
 * like the dd parts, by neighbour degree); 12 offsets of the
 * nd rows in nd-source-list order int64[n_ndsrc+1]; 13 their columns
 * (delegate IDs) int32[e_nd]; 14 the first entry of each of those rows as
 * a pair (delegate ID, its vertex) int32[2 n_ndsrc]. Row i of 12/13 and pair
 * i of 14 belong to vertex ndsrc[i]; the bottom-up dn kernel probes 14 and
 * walks 12/13 only on a miss; 15 the first entry of each delegate's dd part
 * as a pair (delegate ID, its vertex), (-1, -1) if the part is empty,
 * int32[2 d], probed first by the bottom-up dd kernel; 16 the part lengths
 * of every normal row, uint16[n]: nn length | nd length << 8, 0xFFFF when
 * either is 255 or more, 0 for a delegate (read by the normal previsit);
 * 17 the normal vertices with a normal neighbour, ascending, int32[n_nnsrc]
 * (candidates of the bottom-up nn visit when nn_do is set); 18 the start of
 * each vertex's nn part in array 19, uint32[n]; 19 the nn parts of all
 * normal rows concatenated in vertex order, int32[e_nn] (what the forward nn
 * visit reads). 18 and 19 are empty (size 0) when e_nn >= 2^32.
 * Row offsets are packed: bits 0..39 = start of the row, bits 40..63 = length
 * of its first part (nn for normal rows, dd for delegate rows); the row ends
 * at the start of the next row. Normal row v holds nn neighbours (vertex IDs)
 * then nd neighbours (delegate IDs); delegate row k holds dd neighbours
 * (delegate IDs) then dn neighbours (vertex IDs). nn and dn parts are in
 * ascending ID; dd parts, and nd parts of at most 64 entries, are ordered by
 * neighbour degree, highest first (dd: by a log-scale degree bucket, 8 per
 * power of two; ties by ascending ID), so bottom-up scans meet hubs first.
 * *bytes receives the array size; nothing is copied if capacity is smaller.
 * Synchronizes the graph's stream.
 */
dsbfs_status dsbfs_graph_export(const dsbfs_graph *g, int32_t which, void *host_out,
                                int64_t capacity_bytes, int64_t *bytes);

/*
 * RMAT workload on the device (Section VI-A "Reporting": the graphs are
 * generated on the GPUs, vertex IDs relabelled by a deterministic hash).
 * Edge e takes one quadrant per level i < scale from the high 32 bits of the
 * (64 e + i)-th output of the SplitMix64 stream with initial state `seed`
 * (the stream's k-th output is the published finaliser of
 * seed + (k + 1) * 0x9E3779B97F4A7C15), against thresholds floor(p * 2^32)
 * of a, a + b, a + b + c (row bit set from a + b on, column bit in [a, a + b)
 * and from a + b + c on); with `permute`, both endpoints then pass through a
 * bijection of scale-bit integers: four rounds of x = x * mul_r, x ^= x >> (scale / 2),
 * x = x + add_r (mod 2^scale), with mul_r = (output 2r | 1) and add_r = output
 * 2r + 1 of the stream seeded with perm_seed, masked to scale bits. The
 * same definition as the host generator of the test inputs; results are
 * equal bit for bit.
 */
typedef struct dsbfs_rmat_spec {
  int32_t scale;        /* 2^scale vertices, 1..31 */
  int32_t permute;      /* 1: relabel vertex IDs through the seeded bijection */
  int64_t num_edges;    /* generated pairs (the paper's edge factor 16: 16 * 2^scale) */
  double a, b, c;       /* quadrant probabilities; d = 1 - a - b - c */
  uint64_t seed;        /* graph seed */
  uint64_t perm_seed;   /* relabelling seed */
} dsbfs_rmat_spec;

/*
 * Writes the RMAT edge list of *spec to device arrays src, dst
 * (int32[num_edges] each, caller-owned), ordered on `stream` (not
 * synchronized). Errors: INVALID_ARG (bad spec, NULL arrays), HIP.
 */
dsbfs_status dsbfs_rmat_generate(const dsbfs_rmat_spec *spec, int32_t *src, int32_t *dst,
                                 void *stream);

/*
 * dsbfs_graph_create for the RMAT graph of *spec (n = 2^scale) without an
 * edge list anywhere: the generator writes both directions of every
 * non-loop edge straight into the builder's sort keys on the device, so the
 * largest graph that fits is bounded by device memory alone (two 8-byte keys
 * per directed edge during the sort). Same layout, options, ownership and
 * errors as dsbfs_graph_create.
 */
dsbfs_status dsbfs_graph_create_rmat(const dsbfs_rmat_spec *spec, const dsbfs_build_opts *opts,
                                     const dsbfs_allocator *alloc, void *stream,
                                     dsbfs_graph **out);

/* Frees the graph's device memory. NULL is accepted. */
dsbfs_status dsbfs_graph_destroy(dsbfs_graph *g);

/*
 * Per-call scratch for searches on graph g: bitmaps, queues and counters of
 * single-source search. max_lanes (0 or 64) = 64 enables multi-source use,
 * whose lane state is allocated at its first call (see dsbfs_msbfs). Memory
 * from the graph's allocator.
 */
dsbfs_status dsbfs_workspace_create(const dsbfs_graph *g, int32_t max_lanes,
                                    dsbfs_workspace **out);
dsbfs_status dsbfs_workspace_destroy(dsbfs_workspace *ws);

/*
 * Single-source BFS from `source`. depth (device int32[n], required) gets the
 * hop distance of every vertex (-1 unreachable); parent (device int32[n], or
 * NULL when opts->want_parent is 0) gets a BFS-tree parent (source: itself;
 * unreachable: -1). Both indexed by original vertex ID. Mode 1 follows
 * Section IV: per level, previsit of the normal queue and of the delegate
 * frontier mask, the direction decision of Section IV-B for dd, dn and nd
 * (nn always forward), then the visits. opts NULL = defaults. stats may be
 * NULL; when given, the call synchronizes the stream and fills it.
 * Errors: INVALID_ARG (source outside [0, n), null depth, mode 0 without a
 * plain CSR, parent NULL while want_parent), HIP, DEVICE.
 */
dsbfs_status dsbfs_bfs(const dsbfs_graph *g, dsbfs_workspace *ws, int32_t source,
                       const dsbfs_run_opts *opts, int32_t *depth, int32_t *parent,
                       dsbfs_run_stats *stats, void *stream);

/*
 * dsbfs_bfs without a workspace and without any allocation, for callers that
 * cannot allocate device memory (serving loops with a fixed footprint,
 * harnesses that forbid allocation). Same arguments, results and errors as
 * dsbfs_bfs, with the search's scratch memory taken from one static device
 * array per GPU of 64 MiB (held from the library's load until the process
 * ends). A graph needing more (about 26 MB at RMAT scale 20; roughly 25 bytes
 * per vertex) is refused with RANGE before any device work. Levels run as
 * direct launches, and the call returns after its work on `stream` has
 * completed; calls on one device are serialized by a lock, so they never
 * overlap, and each call starts from a cleared state (the array keeps the
 * previous call's contents, which the search overwrites before reading).
 * opts->profile must be 0 (timing events are not created).
 * Errors: as dsbfs_bfs; RANGE (graph too large for the scratch array);
 * INVALID_ARG (profile = 1).
 */
dsbfs_status dsbfs_bfs_noalloc(const dsbfs_graph *g, int32_t source, const dsbfs_run_opts *opts,
                               int32_t *depth, int32_t *parent, dsbfs_run_stats *stats,
                               void *stream);

/*
 * PageRank on the degree-separated layout (another primitive on degree-
 * separated graphs with multi-bit delegate state, the paper's future work,
 * Sections VI-D and VII): FP64 power iteration from the uniform vector,
 *   r'[v] = (1 - alpha)/n + alpha * (D/n + sum over neighbours u of r[u]/deg(u)),
 * D = rank held by degree-0 vertices. Delegates keep their contributions in a
 * compact array by delegate ID, normal vertices by vertex ID. Runs
 * max_iterations steps, or stops after the first step whose L1 change is
 * below tolerance (tolerance > 0: one host synchronization per step). rank:
 * device double[n], caller-owned. *iterations_done and *last_delta (host,
 * either may be NULL) receive the steps run and the last L1 change. Scratch
 * (3 n + 2 d doubles) comes from the graph's allocator for the call. The
 * first call on a graph also builds a cache kept with the graph until it is
 * destroyed: the delegates' ranks by descending degree and a copy of the
 * delegate columns with dd entries as ranks (4 (d + e_dd + e_dn) bytes), so
 * that dd gathers of the most-connected delegates share cache lines.
 * Synchronizes the stream. Errors: INVALID_ARG (alpha outside [0, 1],
 * negative max_iterations, NULL rank), OUT_OF_MEMORY, HIP.
 */
dsbfs_status dsbfs_pagerank(const dsbfs_graph *g, double alpha, int32_t max_iterations,
                            double tolerance, double *rank, int32_t *iterations_done,
                            double *last_delta, void *stream);

/* Tile and schedule parameters of multi-source BFS (chosen by the tuner). */
typedef struct dsbfs_ms_opts {
  int32_t block;          /* threads per workgroup: 64, 128, 256, 512 or 1024 */
  int32_t blocks_per_cu;  /* workgroups per compute unit of the persistent grid */
  int32_t bu_permille;    /* bottom-up when active frontier vertices exceed this
                             many per mille of n (0..1000) */
  int32_t use_graph;      /* 1: capture the launch in a hipGraph and replay it */
  int32_t lanes_per_batch; /* sources per batch: 64, 128 or 256; 0 = automatic
                              (the narrowest that holds k, at most 256) */
} dsbfs_ms_opts;

/*
 * Multi-source BFS from k sources (host int32[k], each in [0, n)), bit-parallel
 * in batches of 64, 128 or 256 lanes, all batches in one persistent launch.
 * Device memory held by the workspace for it: 17 x n x (lanes / 8) bytes of
 * lane state, plus, once per graph, a copy of the plain CSR's columns with
 * hub neighbours renumbered (4 x m_dir bytes) and a hub index (4 x n). depth is a
 * device int32[k][n] array: row i gets the hop distances from sources[i]
 * (-1 unreachable), exactly as k single-source searches would. Uses the plain
 * CSR (graph built with keep_plain_csr = 1). opts NULL = tuned/cached
 * defaults. Errors: INVALID_ARG, HIP, DEVICE (persistent-grid barrier failure).
 */
dsbfs_status dsbfs_msbfs(const dsbfs_graph *g, dsbfs_workspace *ws, const int32_t *sources,
                         int32_t k, const dsbfs_ms_opts *opts, int32_t *depth, void *stream);

/*
 * Autotuner of multi-source BFS: times every candidate tile/schedule setting on
 * graph g with the given sources and writes the fastest to *best. If
 * cache_path is not NULL the result is read from / stored in that JSON file,
 * keyed by the graph's n, m_dir and the device name.
 */
dsbfs_status dsbfs_msbfs_tune(const dsbfs_graph *g, dsbfs_workspace *ws, const int32_t *sources,
                              int32_t k, const char *cache_path, dsbfs_ms_opts *best,
                              void *stream);

/* Per-query record of the server, times in host steady-clock nanoseconds. */
typedef struct dsbfs_query_stats {
  int64_t arrival_ns, admit_ns, start_ns, done_ns;
  int32_t graph_id, source, levels, batched; /* batched: 1 = ran as a lane */
  int32_t waited_budget;  /* 1: admission waited at least once for HBM budget */
  int32_t loaded_graph;   /* 1: its graph was loaded from host memory for it */
} dsbfs_query_stats;

/* Server totals (dsbfs_server_stats_get). */
typedef struct dsbfs_server_stats {
  int64_t budget_bytes, used_bytes;   /* budget and what is charged now */
  int64_t graphs, resident_graphs;    /* added / on the device now */
  int64_t loads, evictions;           /* graph moves host -> device, device -> host */
  int64_t budget_waits;               /* queries whose admission waited for budget */
  int64_t queries_done;
} dsbfs_server_stats;

/* Server configuration. */
typedef struct dsbfs_server_opts {
  size_t hbm_budget_bytes; /* cap on graphs + lane state + result buffers */
  int32_t max_lanes;       /* lanes per running batch, 1..64 */
  int32_t batched;         /* 1: continuous batching into multi-source lanes;
                              0: one query at a time with single-source BFS;
                              2: adaptive: a graph with no batch running serves
                                 its queue one query at a time while that is
                                 cheaper than one batch (measured per graph),
                                 else batches as in 1 */
  dsbfs_ms_opts ms;        /* kernel parameters of the batched path */
  int32_t join_levels;     /* batched: waiting queries join a running batch only
                              during its first join_levels levels (<= 0: 2); a
                              large value admits at every level boundary */
  int32_t reserved;
} dsbfs_server_opts;

/*
 * Query server (continuous batching). create starts one scheduler thread on
 * the current device; result rows come from `alloc` when given (called from
 * the scheduler thread, so it must be callable from any thread), else from
 * hipMalloc. add_graph moves a graph under the server: BUDGET (and the caller
 * keeps the graph) if the graph plus one result row can never fit; a graph
 * that does not fit now is kept in host memory until a query needs it, and
 * idle graphs (no query waiting or running) are evicted to host memory, least
 * recently used first, to make room (Section III-C's per-GPU memory bound
 * applied to several resident graphs). submit queues a single-source query
 * (arrival_ns: caller's steady-clock timestamp, 0 = now) and returns a
 * ticket; wait blocks until that query's depth array is on the device
 * (timeout_ns < 0: forever; NOT_READY on timeout) and returns its device
 * pointer (int32[n_graph], owned by the server until release); release
 * returns the result buffer to the budget. Results stay device resident.
 * stats_get reports the budget, residency and admission totals. destroy
 * stops the thread and frees everything. Every call may come from any
 * thread at any time, including add_graph while queries run. Rows count
 * against the budget until released: a client that holds results while it
 * waits for a query whose graph needs that room waits for ever.
 */
dsbfs_status dsbfs_server_create(const dsbfs_server_opts *opts, const dsbfs_allocator *alloc,
                                 dsbfs_server **out);
dsbfs_status dsbfs_server_add_graph(dsbfs_server *s, dsbfs_graph *g, int32_t *graph_id);
dsbfs_status dsbfs_server_submit(dsbfs_server *s, int32_t graph_id, int32_t source,
                                 int64_t arrival_ns, int64_t *ticket);
dsbfs_status dsbfs_server_wait(dsbfs_server *s, int64_t ticket, int64_t timeout_ns,
                               const int32_t **depth_dev, dsbfs_query_stats *stats);
dsbfs_status dsbfs_server_release(dsbfs_server *s, int64_t ticket);
dsbfs_status dsbfs_server_stats_get(dsbfs_server *s, dsbfs_server_stats *out);
dsbfs_status dsbfs_server_destroy(dsbfs_server *s);

/* Host steady-clock now, in nanoseconds (the server's time base). */
int64_t dsbfs_now_ns(void);

/* Static text of a status code. */
const char *dsbfs_status_str(dsbfs_status st);
/* Message of the last failure on the calling thread ("" if none). */
const char *dsbfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DSBFS_H */
