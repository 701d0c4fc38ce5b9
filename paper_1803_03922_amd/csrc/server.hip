// Query server with continuous batching.
//
// Several graphs stay resident on the device. Clients submit single-source
// queries; one scheduler thread serves them:
//   batched mode: each graph runs a cohort of up to 64 lanes, a multi-source
//     BFS advanced one level at a time. At every level boundary the lanes
//     whose frontier ran empty complete their queries, and waiting queries
//     take free lanes (their lane bits are cleared, their result rows filled
//     with -1, their sources seeded) while the cohort is in its first
//     kJoinLevels levels, or start the next cohort once it has drained. So
//     requests that arrive while others are running join work already on
//     the GPU, while the lanes of a cohort stay within a few levels of each
//     other. Each cohort
//     advances on its own stream and at its own pace: one whose level has
//     finished is relaunched at once, so the levels of different cohorts and
//     graphs overlap on the device and a small graph never waits for a
//     large one.
//   plain mode: one query at a time, single-source direction-optimized BFS.
//   adaptive mode: batched, except that a graph with no batch running serves
//     a short queue one query at a time with single-source DOBFS. A batch is
//     opened once serving the waiting queries one by one would take longer
//     than one batch: queue length x (measured time of one single-source
//     search) >= (measured time of one batched level) x (measured levels per
//     query). Both times are running averages kept per graph.
// Admission is bounded by an HBM budget: a resident graph's layout and lane
// state, and every result row (int32[n]) while it is held or cached. A graph
// that does not fit when it is added, or whose queries wait while idle graphs
// hold the budget, is kept in host memory: idle graphs (no query waiting or
// running) are evicted, least recently used first, and a graph is loaded back
// when a query needs it. A query waits for budget, and one that can never fit
// is refused. Results stay on the device until the client releases them.
// Result rows come from the caller's allocator when one is given (called from
// the scheduler thread), else from hipMalloc; frees of rows dropped to make
// room run outside the lock that clients take.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace dsbfs {

int ms_level(const Graph *g, Workspace *ws, uint64_t live, int64_t active, int32_t bu_permille,
             int32_t L, unsigned long long *ctl, hipStream_t s);
void ms_level_flush(const Graph *g, Workspace *ws, const LaneFlush &f, unsigned long long *ctl,
                    unsigned long long *next_ctl, unsigned long long *host_ctl, hipStream_t s);
int ms_level_ring();
size_t ms_state_bytes(const Workspace *ws);
void ms_level_prepare(const Graph *g, Workspace *ws, hipStream_t s);
void ms_level_recycle(const Graph *g, Workspace *ws, int32_t L, uint64_t clear, uint64_t seed_mask,
                      const SeedList &seeds, hipStream_t s);
Workspace *workspace_create(const Graph *g, int32_t max_lanes);
void workspace_destroy(Workspace *ws);
void graph_destroy(Graph *G);
void bfs_run(const Graph *g, Workspace *ws, int32_t source, const dsbfs_run_opts *o,
             int32_t *depth, int32_t *parent, dsbfs_run_stats *stats, hipStream_t s);
void run_opts_default(dsbfs_run_opts *o);

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

namespace {

size_t buf_bytes(const DevBuf &b) { return b.p ? b.bytes : 0; }

size_t graph_footprint(const Graph *g) {
  return buf_bytes(g->deg) + buf_bytes(g->did) + buf_bytes(g->vid_of) + buf_bytes(g->noff) +
         buf_bytes(g->ncol) + buf_bytes(g->doff) + buf_bytes(g->dcol) + buf_bytes(g->ndsrc) +
         buf_bytes(g->ddsrc_mask) + buf_bytes(g->dnsrc_mask) + buf_bytes(g->nds_off) +
         buf_bytes(g->nds_col) + buf_bytes(g->nds_first) + buf_bytes(g->dd_first) +
         buf_bytes(g->nlen) + buf_bytes(g->nnsrc) + buf_bytes(g->nnoff) + buf_bytes(g->nncol) +
         buf_bytes(g->pr_rank) + buf_bytes(g->pr_col) +
         buf_bytes(g->poff) +
         buf_bytes(g->pcol);
}

size_t workspace_footprint(const Workspace *w) {
  return buf_bytes(w->Vn) + buf_bytes(w->Fn) + buf_bytes(w->Vd) + buf_bytes(w->Fd) +
         buf_bytes(w->Cd) + buf_bytes(w->q0) + buf_bytes(w->q1) + buf_bytes(w->dlist) +
         buf_bytes(w->dcand) + buf_bytes(w->dlen) + buf_bytes(w->dscan) + buf_bytes(w->c0) +
         buf_bytes(w->c1) + buf_bytes(w->ctr) + buf_bytes(w->scan_tmp) + buf_bytes(w->dctl) +
         buf_bytes(w->dtiles) + ms_state_bytes(w);
}

enum QState { Q_PENDING = 0, Q_RUNNING = 1, Q_DONE = 2, Q_RELEASED = 3 };

struct Query {
  int64_t ticket = 0;
  int32_t gid = 0, source = 0;
  int64_t arrival = 0, admit = 0, start = 0, done = 0;
  int32_t levels = 0, batched = 0;
  int32_t waited_budget = 0, loaded_graph = 0;
  int32_t *res = nullptr;
  QState state = Q_PENDING;
};

// One batch of up to 64 lanes on one graph: its lane state, stream and
// level bookkeeping. Lanes of a cohort start within a few levels of each
// other, so its bottom-up levels keep their early exit.
struct Cohort {
  Workspace *ws = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr, ev0 = nullptr;
  Query *lane[64] = {};
  int32_t start_level[64] = {};
  int32_t from[64] = {};  // first level of each lane whose depths are not yet written
  uint64_t used = 0, live = 0, new_lanes = 0;
  int64_t active = 0;
  int32_t L = 0;
  int32_t batch_start = 0;  // level at which the running batch began
  // control blocks of the levels, alternating by level parity (4 words each),
  // and the host copy of the last finished level's
  unsigned long long *ctl_dev = nullptr, *ctl_host = nullptr;
  SeedList seeds{};  // sources of the lanes admitted for the next level
  bool launched = false;
};
// Cohorts per graph. With two, a query that misses the join window of the
// running cohort starts the other at once; measured on the served mix (RMAT
// 18-24 + ER 2^22), two half-full cohorts repeat each other's bottom-up scans
// and both p50 and p99 latency came out higher than with one.
constexpr int kCohorts = 1;

// A graph's device buffers saved in host memory while it is evicted.
struct Saved {
  DevBuf *buf;
  size_t bytes;
  std::vector<char> host;
};

struct GState {
  Graph *g = nullptr;
  Cohort co[kCohorts];
  std::deque<Query *> pending;
  std::vector<int32_t *> free_bufs;
  size_t bytes = 0;            // layout + lane state while resident
  size_t layout_bytes = 0;
  bool resident = true;
  std::vector<Saved> saved;    // device buffers kept on the host while evicted
  int64_t last_use = 0;        // last admission (eviction order)
  // adaptive mode: cost model and the query served alone this round
  double t_single_ms = 0, t_level_ms = 0, levels_per_query = 0;
  Query *single = nullptr;
  bool running() const {
    for (const Cohort &c : co)
      if (c.used) return true;
    return false;
  }
  bool in_flight() const {
    for (const Cohort &c : co)
      if (c.launched) return true;
    return false;
  }
};

// running average with weight 1/4 for the newest sample (first sample taken as is)
void ema(double &avg, double x) { avg = avg > 0 ? 0.75 * avg + 0.25 * x : x; }

// The device buffers of a graph's layout.
std::vector<DevBuf *> graph_bufs(Graph *g) {
  return {&g->deg, &g->did, &g->vid_of, &g->noff, &g->ncol, &g->doff, &g->dcol, &g->ndsrc,
          &g->ddsrc_mask, &g->dnsrc_mask, &g->nds_off, &g->nds_col, &g->nds_first, &g->dd_first,
          &g->nlen, &g->nnsrc, &g->nnoff, &g->nncol, &g->pr_rank, &g->pr_col, &g->poff,
          &g->pcol};
}

void cohort_init(Cohort &c, Graph *g, bool batched);
void cohort_free(Cohort &c);

constexpr int kMaxGraphs = 256;

}  // namespace

constexpr int32_t kJoinLevels = 2;

struct Server {
  dsbfs_server_opts o{};
  int32_t join_levels = kJoinLevels;
  int device = 0;
  Alloc al;                       // result rows: the caller's allocator, else hipMalloc
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  // Graphs are never removed while the server runs: the scheduler reads the
  // count once per pass and the entries below it without the lock.
  GState *graphs[kMaxGraphs] = {};
  std::atomic<int32_t> ngraphs{0};
  std::unordered_map<int64_t, Query *> queries;
  int64_t next_ticket = 1;
  size_t used_bytes = 0;
  int64_t loads = 0, evictions = 0, budget_waits = 0, done_count = 0;
  std::vector<int32_t *> drop;    // rows to free outside the lock
  bool stop = false;
  std::string thread_error;
  std::thread th;

  size_t row_bytes(const GState *G) const { return size_t(G->g->n) * 4; }

  int32_t *alloc_row(size_t bytes) {
    void *p = nullptr;
    try {
      p = al.get(bytes, nullptr);
    } catch (const Error &) {
      return nullptr;
    }
    return static_cast<int32_t *>(p);
  }

  // Frees rows dropped to make room (scheduler thread, lock not held).
  void free_dropped() {
    std::vector<int32_t *> d;
    {
      std::lock_guard<std::mutex> lk(mu);
      d.swap(drop);
    }
    for (int32_t *p : d) al.put(p, nullptr);
  }

  // Gets a result row for G within the budget, leaving `keep` bytes of it
  // free (caller holds mu). A cached row of G is reused (it is charged
  // already); cached rows of other graphs dropped to make room are freed
  // later, outside the lock.
  int32_t *take_row(GState *G, size_t keep) {
    const size_t need = row_bytes(G);
    const bool cached = !G->free_bufs.empty();
    const size_t add = cached ? 0 : need;  // what taking the row adds to the charge
    if (used_bytes + add + keep > o.hbm_budget_bytes) {
      const int32_t ng = ngraphs.load(std::memory_order_acquire);
      for (int32_t i = 0; i < ng; ++i) {
        GState *H = graphs[i];
        const size_t spare = (H == G && cached) ? 1 : 0;  // the row about to be reused
        while (H->free_bufs.size() > spare && used_bytes + add + keep > o.hbm_budget_bytes) {
          drop.push_back(H->free_bufs.back());
          H->free_bufs.pop_back();
          used_bytes -= row_bytes(H);
        }
      }
      if (used_bytes + add + keep > o.hbm_budget_bytes) return nullptr;
    }
    if (cached) {
      int32_t *p = G->free_bufs.back();
      G->free_bufs.pop_back();
      return p;
    }
    int32_t *p = alloc_row(need);
    if (!p) return nullptr;
    used_bytes += need;
    return p;
  }

  // The oldest waiting query over the resident graphs, and the bytes of its
  // row (caller holds mu). A younger query is admitted only while that row
  // would still fit: when the budget binds, memory freed by releases then
  // goes to the oldest query instead of to later arrivals on graphs with
  // smaller rows, which would otherwise starve it.
  Query *oldest = nullptr;
  size_t oldest_bytes = 0;
  void pick_oldest() {
    oldest = nullptr;
    oldest_bytes = 0;
    const int32_t ng = ngraphs.load(std::memory_order_acquire);
    for (int32_t i = 0; i < ng; ++i) {
      GState *H = graphs[i];
      if (!H->resident || H->pending.empty()) continue;
      Query *q = H->pending.front();
      if (!oldest || q->arrival < oldest->arrival) {
        oldest = q;
        oldest_bytes = row_bytes(H);
      }
    }
  }
  size_t keep_for(const Query *q) const { return q == oldest ? 0 : oldest_bytes; }
  // after admitting q: the next oldest is reserved for
  void admitted(const Query *q) {
    if (q == oldest) pick_oldest();
  }

  // A query that found no budget for its row or its graph (counted once).
  void budget_wait(Query *q) {
    if (!q->waited_budget) {
      q->waited_budget = 1;
      ++budget_waits;
    }
  }

  bool idle(const GState *G) const {
    return G->resident && !G->running() && !G->in_flight() && !G->single && G->pending.empty();
  }

  // Graph residency (scheduler thread). evict: an idle graph's layout goes
  // to host memory and its lane state and cached rows are freed. load: the
  // reverse, for a graph with waiting queries, after evicting idle graphs
  // (least recently used first) until it fits. Returns false when it cannot
  // fit yet (queries of other graphs hold the budget).
  void evict(GState *G) {
    for (Cohort &c : G->co) cohort_free(c);
    std::vector<int32_t *> rows;
    {
      std::lock_guard<std::mutex> lk(mu);
      rows.swap(G->free_bufs);
      for (size_t i = 0; i < rows.size(); ++i) used_bytes -= row_bytes(G);
      used_bytes -= G->bytes;
      G->resident = false;
      ++evictions;
    }
    for (int32_t *p : rows) al.put(p, nullptr);
    for (DevBuf *b : graph_bufs(G->g)) {
      if (!b->p) continue;
      Saved sv{b, b->bytes, std::vector<char>(b->bytes)};
      HIPCHK(hipMemcpy(sv.host.data(), b->p, b->bytes, hipMemcpyDeviceToHost));
      b->reset();
      G->saved.push_back(std::move(sv));
    }
  }

  bool make_resident(GState *G) {
    const size_t need = G->bytes;  // layout + lane state
    while (true) {
      GState *victim = nullptr;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (used_bytes + need + row_bytes(G) <= o.hbm_budget_bytes) {
          used_bytes += need;   // reserved before the copies
          break;
        }
        const int32_t ng = ngraphs.load(std::memory_order_acquire);
        for (int32_t i = 0; i < ng; ++i) {
          GState *H = graphs[i];
          if (H != G && idle(H) && (!victim || H->last_use < victim->last_use)) victim = H;
        }
        if (!victim) {
          if (!G->pending.empty()) budget_wait(G->pending.front());
          return false;
        }
      }
      evict(victim);
    }
    for (Saved &sv : G->saved) {
      sv.buf->alloc(&G->g->al, sv.bytes, nullptr);
      HIPCHK(hipMemcpy(sv.buf->p, sv.host.data(), sv.bytes, hipMemcpyHostToDevice));
    }
    G->saved.clear();
    const int nco = o.batched ? kCohorts : 1;
    for (int i = 0; i < nco; ++i) cohort_init(G->co[i], G->g, o.batched != 0);
    std::lock_guard<std::mutex> lk(mu);
    G->resident = true;
    ++loads;
    for (Query *q : G->pending) q->loaded_graph = 1;
    return true;
  }

  // Loads the graphs that have waiting queries but are on the host.
  void ensure_resident() {
    const int32_t ng = ngraphs.load(std::memory_order_acquire);
    for (int32_t i = 0; i < ng; ++i) {
      GState *G = graphs[i];
      bool want;
      {
        std::lock_guard<std::mutex> lk(mu);
        want = !G->resident && !G->pending.empty();
      }
      if (want) make_resident(G);
    }
  }

  void finish(Query *q, GState *G, int64_t t) {
    q->done = t;
    q->state = Q_DONE;
    ++done_count;
    (void)G;
  }

  bool has_work() const {
    const int32_t ng = ngraphs.load(std::memory_order_acquire);
    for (int32_t i = 0; i < ng; ++i)
      if (graphs[i]->running() || !graphs[i]->pending.empty()) return true;
    return false;
  }

  // Adaptive mode: should G (no batch running) serve its head query alone?
  bool serve_alone(const GState *G) const {
    if (G->t_single_ms <= 0) return true;  // nothing measured yet: a single search measures it
    // until a batched level has been timed, assume a batch costs 8 single searches
    const double batch_ms = G->t_level_ms > 0 && G->levels_per_query > 0
                                ? G->t_level_ms * G->levels_per_query
                                : 8.0 * G->t_single_ms;
    return double(G->pending.size()) * G->t_single_ms < batch_ms;
  }

  // Admits waiting queries of G (caller holds mu): in adaptive mode the head
  // query alone when that is cheaper, else into free lanes of a cohort at a
  // level boundary, preferring a running cohort still within its first
  // kJoinLevels levels, then an idle one. A query that joined a batch later
  // would have a tiny frontier while the batch's bottom-up levels cover the
  // graph, and every unseen vertex would scan its whole row for its bit.
  void admit(GState *G, uint64_t lane_cap, bool adaptive, int64_t t) {
    for (Cohort &c : G->co)
      if (!c.launched) c.new_lanes = 0;
    if (G->pending.empty() || !G->resident) return;
    G->last_use = t;
    if (adaptive && !G->running() && !G->in_flight() && serve_alone(G)) {
      Query *q = G->pending.front();
      int32_t *row = take_row(G, keep_for(q));
      if (!row) {  // budget: wait for releases
        budget_wait(q);
        return;
      }
      G->pending.pop_front();
      admitted(q);
      q->res = row;
      q->admit = q->start = t;
      q->state = Q_RUNNING;
      q->batched = 0;
      G->single = q;
      return;
    }
    for (int pass = 0; pass < 2 && !G->pending.empty(); ++pass) {
      for (Cohort &c : G->co) {
        if (c.launched || G->pending.empty()) continue;
        const bool joinable = c.used && c.L - c.batch_start < join_levels;
        if (pass == 0 ? !joinable : c.used != 0) continue;
        if (!c.used) c.batch_start = c.L;
        uint64_t free = ~c.used & lane_cap;
        bool no_budget = false;
        while (free && !G->pending.empty()) {
          Query *q = G->pending.front();
          int32_t *row = take_row(G, keep_for(q));
          if (!row) {  // budget: the rest waits for releases
            budget_wait(q);
            no_budget = true;
            break;
          }
          G->pending.pop_front();
          admitted(q);
          const int i = __builtin_ctzll(free);
          free &= free - 1;
          q->res = row;
          q->admit = q->start = t;
          q->state = Q_RUNNING;
          q->batched = 1;
          c.lane[i] = q;
          c.start_level[i] = c.L;
          c.from[i] = c.L;
          c.seeds.src[i] = q->source;
          c.new_lanes |= 1ull << i;
        }
        c.used |= c.new_lanes;  // the lanes admitted so far run in any case
        if (no_budget) return;
      }
    }
  }

  // Rows of the lanes in `lanes` from their first unwritten level up to the
  // current level c.L (final: only those whose frontier ran empty this level).
  static LaneFlush lane_flush(const Cohort &c, uint64_t lanes, int final) {
    LaneFlush f{};
    f.lanes = lanes;
    f.final = final;
    f.jhi = c.L;
    f.jlo = c.L;
    for (uint64_t m = lanes; m; m &= m - 1) f.jlo = std::min(f.jlo, c.from[__builtin_ctzll(m)]);
    for (int i = 0; i < 64; ++i) {
      f.res[i] = c.lane[i] ? c.lane[i]->res : nullptr;
      f.start[i] = c.start_level[i];
    }
    for (int o = 0; o <= f.jhi - f.jlo; ++o)
      for (uint64_t m = lanes; m; m &= m - 1) {
        const int i = __builtin_ctzll(m);
        if (c.from[i] <= f.jlo + o) f.valid[o] |= 1ull << i;
      }
    return f;
  }

  // Enqueues one multi-source level of cohort c of G on its stream, then the
  // rows of the lanes it completes.
  void launch_level(GState *G, Cohort &c) {
    unsigned long long *const ctl = c.ctl_dev + 4 * (c.L & 1);
    unsigned long long *const next_ctl = c.ctl_dev + 4 * ((c.L + 1) & 1);
    HIPCHK(hipEventRecord(c.ev0, c.stream));
    // this level's next frontier overwrites ring level L + 1 - ring: lanes
    // whose rows still need it are written up to level L first
    uint64_t wrap = 0;
    for (uint64_t m = c.used & ~c.new_lanes; m; m &= m - 1) {
      const int i = __builtin_ctzll(m);
      if (c.from[i] <= c.L + 1 - ms_level_ring()) wrap |= 1ull << i;
    }
    if (wrap) {
      ms_level_flush(G->g, c.ws, lane_flush(c, wrap, 0), ctl, nullptr, nullptr, c.stream);
      for (uint64_t m = wrap; m; m &= m - 1) c.from[__builtin_ctzll(m)] = c.L + 1;
    }
    if (c.new_lanes) {
      ms_level_recycle(G->g, c.ws, c.L, c.new_lanes, c.new_lanes, c.seeds, c.stream);
      c.live |= c.new_lanes;
      c.active += __builtin_popcountll(c.new_lanes);
      c.new_lanes = 0;
    }
    ms_level(G->g, c.ws, c.live, c.active, o.ms.bu_permille, c.L, ctl, c.stream);
    // rows of the lanes this level completes; publishes the level's counts to
    // c.ctl_host and clears the next level's control block
    ms_level_flush(G->g, c.ws, lane_flush(c, c.used, 1), ctl, next_ctl, c.ctl_host, c.stream);
    HIPCHK(hipEventRecord(c.ev, c.stream));
    c.launched = true;
  }

  // Level of cohort c done on the device: complete the lanes whose frontier
  // ran empty.
  void complete_level(GState *G, Cohort &c) {
    const int64_t t = now_ns();
    float level_ms = 0;
    HIPCHK(hipEventElapsedTime(&level_ms, c.ev0, c.ev));
    ema(G->t_level_ms, double(level_ms));
    const uint64_t alive = c.ctl_host[1];
    std::lock_guard<std::mutex> lk(mu);
    uint64_t fin = c.used & ~alive;
    while (fin) {
      const int i = __builtin_ctzll(fin);
      fin &= fin - 1;
      Query *q = c.lane[i];
      q->levels = c.L + 1 - c.start_level[i];
      ema(G->levels_per_query, double(q->levels));
      finish(q, G, t);
      c.lane[i] = nullptr;
      c.used &= ~(1ull << i);
    }
    c.live = alive & c.used;
    c.active = int64_t(c.ctl_host[0]);
    c.L += 1;
    c.launched = false;
  }

  // Every cohort of every graph advances on its own: one whose level finished
  // is admitted into and relaunched at once, without waiting for the others.
  void loop_batched() {
    const uint64_t lane_cap = o.max_lanes >= 64 ? ~0ull : ((1ull << o.max_lanes) - 1ull);
    const bool adaptive = o.batched == 2;
    dsbfs_run_opts ro{};
    run_opts_default(&ro);
    ro.want_parent = 0;
    while (true) {
      const int32_t ng = ngraphs.load(std::memory_order_acquire);
      bool in_flight = false;
      for (int32_t i = 0; i < ng; ++i) in_flight = in_flight || graphs[i]->in_flight();
      {
        std::unique_lock<std::mutex> lk(mu);
        if (!in_flight) cv_work.wait(lk, [&] { return stop || has_work(); });
        if (stop) return;
      }
      ensure_resident();
      {
        std::lock_guard<std::mutex> lk(mu);
        const int64_t t = now_ns();
        pick_oldest();
        for (int32_t i = 0; i < ng; ++i)
          if (!graphs[i]->single) admit(graphs[i], lane_cap, adaptive, t);
      }
      free_dropped();
      bool started = false;
      for (int32_t i = 0; i < ng; ++i)
        for (Cohort &c : graphs[i]->co)
          if (!c.launched && c.used) {
            launch_level(graphs[i], c);
            started = true;
          }
      // queries served alone run while the levels of other graphs are in
      // flight (on the first cohort's workspace, idle when one is chosen)
      bool progressed = false;
      for (int32_t i = 0; i < ng; ++i) {
        GState *G = graphs[i];
        Query *q = G->single;
        if (!q) continue;
        Cohort &c = G->co[0];
        dsbfs_run_stats rs{};
        const int64_t t0 = now_ns();
        bfs_run(G->g, c.ws, q->source, &ro, q->res, nullptr, &rs, c.stream);
        HIPCHK(hipStreamSynchronize(c.stream));
        const int64_t t = now_ns();
        ema(G->t_single_ms, double(t - t0) * 1e-6);
        ema(G->levels_per_query, double(rs.num_levels));
        std::lock_guard<std::mutex> lk(mu);
        q->levels = rs.num_levels;
        finish(q, G, t);
        G->single = nullptr;
        progressed = true;
      }
      for (int32_t i = 0; i < ng; ++i)
        for (Cohort &c : graphs[i]->co) {
          if (!c.launched) continue;
          const hipError_t e = hipEventQuery(c.ev);
          if (e == hipErrorNotReady) continue;
          HIPCHK(e);
          complete_level(graphs[i], c);
          progressed = true;
        }
      if (progressed) {
        cv_done.notify_all();
        continue;
      }
      in_flight = false;
      for (int32_t i = 0; i < ng; ++i) in_flight = in_flight || graphs[i]->in_flight();
      if (in_flight) {
        if (!started) std::this_thread::sleep_for(std::chrono::microseconds(20));
      } else {
        // waiting queries but no budget for their rows: wait for a release
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::milliseconds(1));
      }
    }
  }

  void loop_plain() {
    dsbfs_run_opts ro{};
    run_opts_default(&ro);
    ro.want_parent = 0;
    while (true) {
      Query *q = nullptr;
      GState *G = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || has_work(); });
        if (stop) return;
      }
      ensure_resident();
      {
        std::unique_lock<std::mutex> lk(mu);
        // oldest waiting query over the resident graphs
        const int32_t ng = ngraphs.load(std::memory_order_acquire);
        for (int32_t i = 0; i < ng; ++i) {
          GState *H = graphs[i];
          if (H->resident && !H->pending.empty() &&
              (!q || H->pending.front()->arrival < q->arrival)) {
            q = H->pending.front();
            G = H;
          }
        }
        if (!q) {   // every waiting query's graph is on the host and cannot fit yet
          cv_done.wait_for(lk, std::chrono::milliseconds(1));
          continue;
        }
        int32_t *row = take_row(G, 0);  // q is the oldest waiting query
        if (!row) {
          budget_wait(q);
          lk.unlock();
          free_dropped();
          lk.lock();
          cv_done.wait_for(lk, std::chrono::milliseconds(1));
          continue;
        }
        G->pending.pop_front();
        G->last_use = now_ns();
        q->res = row;
        q->admit = q->start = now_ns();
        q->state = Q_RUNNING;
      }
      free_dropped();
      bfs_run(G->g, G->co[0].ws, q->source, &ro, q->res, nullptr, nullptr, G->co[0].stream);
      HIPCHK(hipStreamSynchronize(G->co[0].stream));
      {
        std::lock_guard<std::mutex> lk(mu);
        finish(q, G, now_ns());
      }
      cv_done.notify_all();
    }
  }

  void run() {
    try {
      HIPCHK(hipSetDevice(device));
      if (o.batched) loop_batched();
      else loop_plain();
    } catch (const Error &e) {
      std::lock_guard<std::mutex> lk(mu);
      thread_error = e.msg;
      stop = true;
      cv_done.notify_all();
    }
  }
};

Server *server_create(const dsbfs_server_opts *o, const dsbfs_allocator *alloc) {
  if (o->max_lanes < 1 || o->max_lanes > 64)
    fail(DSBFS_ERR_INVALID_ARG, "max_lanes must be in [1, 64]");
  if (o->batched < 0 || o->batched > 2)
    fail(DSBFS_ERR_INVALID_ARG, "batched must be 0 (plain), 1 (batched) or 2 (adaptive)");
  if (o->ms.bu_permille < 0 || o->ms.bu_permille > 1000)
    fail(DSBFS_ERR_INVALID_ARG, "ms.bu_permille must be in [0, 1000]");
  if (alloc && (!alloc->alloc || !alloc->free))
    fail(DSBFS_ERR_INVALID_ARG, "allocator needs both alloc and free");
  Server *S = new Server();
  S->o = *o;
  S->join_levels = o->join_levels > 0 ? o->join_levels : kJoinLevels;
  if (alloc) {
    S->al.a = *alloc;
    S->al.custom = true;
  }
  HIPCHK(hipGetDevice(&S->device));
  S->th = std::thread([S] { S->run(); });
  return S;
}

namespace {

// Lane state, stream, events and small control buffers of one cohort.
void cohort_init(Cohort &c, Graph *g, bool batched) {
  HIPCHK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreate(&c.ev));
  HIPCHK(hipEventCreate(&c.ev0));
  c.ws = workspace_create(g, 64);
  if (batched) ms_level_prepare(g, c.ws, c.stream);
  HIPCHK(hipMalloc(reinterpret_cast<void **>(&c.ctl_dev), 8 * sizeof(unsigned long long)));
  HIPCHK(hipMemsetAsync(c.ctl_dev, 0, 8 * sizeof(unsigned long long), c.stream));
  HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&c.ctl_host), 4 * sizeof(unsigned long long),
                       hipHostMallocDefault));
  HIPCHK(hipStreamSynchronize(c.stream));
}

void cohort_free(Cohort &c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (c.ws) workspace_destroy(c.ws);
  if (c.ctl_dev) (void)hipFree(c.ctl_dev);
  if (c.ctl_host) (void)hipHostFree(c.ctl_host);
  if (c.ev) (void)hipEventDestroy(c.ev);
  if (c.ev0) (void)hipEventDestroy(c.ev0);
  if (c.stream) (void)hipStreamDestroy(c.stream);
  c = Cohort();
}

}  // namespace

void server_add_graph(Server *S, Graph *g, int32_t *id) {
  if (!g->pcol.p && g->m > 0 && S->o.batched)
    fail(DSBFS_ERR_INVALID_ARG, "batched serving needs graphs built with keep_plain_csr");
  GState *G = new GState();
  try {
    G->g = g;
    // the plain server needs one search workspace; batched modes one per cohort
    const int nco = S->o.batched ? kCohorts : 1;
    G->layout_bytes = graph_footprint(g);
    G->bytes = G->layout_bytes;
    for (int i = 0; i < nco; ++i) {
      cohort_init(G->co[i], g, S->o.batched != 0);
      G->bytes += workspace_footprint(G->co[i].ws);
    }
    bool fits;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->ngraphs.load() >= kMaxGraphs) fail(DSBFS_ERR_INVALID_ARG, "too many graphs");
      if (G->bytes + S->row_bytes(G) > S->o.hbm_budget_bytes)
        fail(DSBFS_ERR_BUDGET, "graph and one result row can never fit the HBM budget");
      fits = S->used_bytes + G->bytes <= S->o.hbm_budget_bytes;
      if (fits) S->used_bytes += G->bytes;
    }
    if (!fits) {
      // not visible to the scheduler yet: keep it on the host until a query needs it
      for (Cohort &c : G->co) cohort_free(c);
      for (DevBuf *b : graph_bufs(g)) {
        if (!b->p) continue;
        Saved sv{b, b->bytes, std::vector<char>(b->bytes)};
        HIPCHK(hipMemcpy(sv.host.data(), b->p, b->bytes, hipMemcpyDeviceToHost));
        b->reset();
        G->saved.push_back(std::move(sv));
      }
      G->resident = false;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t i = S->ngraphs.load();
    S->graphs[i] = G;
    *id = i;
    S->ngraphs.store(i + 1, std::memory_order_release);
  } catch (...) {
    for (Cohort &c : G->co) cohort_free(c);
    delete G;
    throw;
  }
}

void server_submit(Server *S, int32_t gid, int32_t source, int64_t arrival, int64_t *ticket) {
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->thread_error.empty()) fail(DSBFS_ERR_HIP, "server stopped: " + S->thread_error);
  if (gid < 0 || gid >= S->ngraphs.load()) fail(DSBFS_ERR_INVALID_ARG, "unknown graph id");
  GState *G = S->graphs[gid];
  if (source < 0 || source >= G->g->n) fail(DSBFS_ERR_INVALID_ARG, "source outside [0, n)");
  Query *q = new Query();
  q->ticket = S->next_ticket++;
  q->gid = gid;
  q->source = source;
  q->arrival = arrival > 0 ? arrival : now_ns();
  S->queries[q->ticket] = q;
  G->pending.push_back(q);
  *ticket = q->ticket;
  S->cv_work.notify_one();
}

dsbfs_status server_wait(Server *S, int64_t ticket, int64_t timeout_ns, const int32_t **depth,
                         dsbfs_query_stats *st) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->queries.find(ticket);
  if (it == S->queries.end()) fail(DSBFS_ERR_INVALID_ARG, "unknown ticket");
  Query *q = it->second;
  auto ready = [&] { return q->state >= Q_DONE || !S->thread_error.empty(); };
  if (timeout_ns < 0) S->cv_done.wait(lk, ready);
  else if (!S->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready))
    return DSBFS_ERR_NOT_READY;
  if (q->state < Q_DONE) fail(DSBFS_ERR_HIP, "server stopped: " + S->thread_error);
  if (q->state == Q_RELEASED) fail(DSBFS_ERR_INVALID_ARG, "ticket already released");
  if (depth) *depth = q->res;
  if (st) {
    st->arrival_ns = q->arrival;
    st->admit_ns = q->admit;
    st->start_ns = q->start;
    st->done_ns = q->done;
    st->graph_id = q->gid;
    st->source = q->source;
    st->levels = q->levels;
    st->batched = q->batched;
    st->waited_budget = q->waited_budget;
    st->loaded_graph = q->loaded_graph;
  }
  return DSBFS_OK;
}

void server_stats(Server *S, dsbfs_server_stats *st) {
  std::lock_guard<std::mutex> lk(S->mu);
  *st = dsbfs_server_stats{};
  st->budget_bytes = int64_t(S->o.hbm_budget_bytes);
  st->used_bytes = int64_t(S->used_bytes);
  const int32_t ng = S->ngraphs.load();
  st->graphs = ng;
  for (int32_t i = 0; i < ng; ++i) st->resident_graphs += S->graphs[i]->resident;
  st->loads = S->loads;
  st->evictions = S->evictions;
  st->budget_waits = S->budget_waits;
  st->queries_done = S->done_count;
}

void server_release(Server *S, int64_t ticket) {
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->queries.find(ticket);
  if (it == S->queries.end()) fail(DSBFS_ERR_INVALID_ARG, "unknown ticket");
  Query *q = it->second;
  if (q->state != Q_DONE) fail(DSBFS_ERR_INVALID_ARG, "query not done (or already released)");
  S->graphs[q->gid]->free_bufs.push_back(q->res);
  q->res = nullptr;
  q->state = Q_RELEASED;
  S->queries.erase(it);
  delete q;
  S->cv_work.notify_one();
}

void server_destroy(Server *S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  if (S->th.joinable()) S->th.join();
  for (auto &kv : S->queries) {
    if (kv.second->res) S->al.put(kv.second->res, nullptr);
    delete kv.second;
  }
  for (int32_t *p : S->drop) S->al.put(p, nullptr);
  const int32_t ng = S->ngraphs.load();
  for (int32_t i = 0; i < ng; ++i) {
    GState *G = S->graphs[i];
    for (Cohort &c : G->co) cohort_free(c);
    for (int32_t *p : G->free_bufs) S->al.put(p, nullptr);
    graph_destroy(G->g);
    delete G;
  }
  delete S;
}

}  // namespace dsbfs
