// extern "C" entry points of libdsbfs.so: argument checks, exception-to-status
// translation, thread-local error messages, allocator plumbing.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <string>

#include "internal.hpp"

namespace dsbfs {

static thread_local std::string g_last_error;

void fail(dsbfs_status st, const std::string &msg) { throw Error{st, msg}; }

void hip_check(hipError_t e, const char *what, const char *file, int line) {
  if (e == hipSuccess) return;
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  if (e == hipErrorOutOfMemory) throw Error{DSBFS_ERR_OUT_OF_MEMORY, buf};
  throw Error{DSBFS_ERR_HIP, buf};
}

void *Alloc::get(size_t bytes, hipStream_t s) const {
  void *p = nullptr;
  if (custom) {
    p = a.alloc(a.ctx, bytes, s);
    if (!p) fail(DSBFS_ERR_OUT_OF_MEMORY, "allocator returned NULL for " + std::to_string(bytes) +
                                              " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(DSBFS_ERR_OUT_OF_MEMORY, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
  }
  return p;
}

void Alloc::put(void *p, hipStream_t s) const {
  if (!p) return;
  if (custom) a.free(a.ctx, p, s);
  else (void)hipFree(p);
}

// defined in the other translation units
Graph *graph_create(const int32_t *src, const int32_t *dst, int64_t g, int32_t n,
                    const dsbfs_build_opts *opts, const dsbfs_allocator *alloc, hipStream_t s,
                    const dsbfs_rmat_spec *rmat);
void rmat_generate(const dsbfs_rmat_spec *sp, int32_t *src, int32_t *dst, hipStream_t s);
void pagerank_run(const Graph *g, double alpha, int32_t max_iter, double tol, double *rank,
                  int32_t *iters_done, double *last_delta, hipStream_t s);
void graph_destroy(Graph *G);
Workspace *workspace_create(const Graph *g, int32_t max_lanes);
void workspace_destroy(Workspace *ws);
void run_opts_default(dsbfs_run_opts *o);
void bfs_run(const Graph *g, Workspace *ws, int32_t source, const dsbfs_run_opts *o,
             int32_t *depth, int32_t *parent, dsbfs_run_stats *stats, hipStream_t s);
void bfs_run_noalloc(const Graph *g, int32_t source, const dsbfs_run_opts *o, int32_t *depth,
                     int32_t *parent, dsbfs_run_stats *stats, hipStream_t s);
void graph_export(const Graph *g, int32_t which, void *host_out, int64_t cap, int64_t *bytes);
void msbfs_run(const Graph *g, Workspace *ws, const int32_t *sources, int32_t k,
               const dsbfs_ms_opts *o, int32_t *depth, hipStream_t s);
void msbfs_tune(const Graph *g, Workspace *ws, const int32_t *sources, int32_t k,
                const char *cache_path, dsbfs_ms_opts *best, hipStream_t s);
struct Server;
Server *server_create(const dsbfs_server_opts *o, const dsbfs_allocator *alloc);
void server_add_graph(Server *S, Graph *g, int32_t *id);
void server_submit(Server *S, int32_t gid, int32_t source, int64_t arrival, int64_t *ticket);
dsbfs_status server_wait(Server *S, int64_t ticket, int64_t timeout_ns, const int32_t **depth,
                         dsbfs_query_stats *st);
void server_release(Server *S, int64_t ticket);
void server_stats(Server *S, dsbfs_server_stats *st);
void server_destroy(Server *S);
int64_t now_ns();

template <class F> static dsbfs_status guard(F &&f) {
  try {
    g_last_error.clear();
    f();
    return DSBFS_OK;
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return DSBFS_ERR_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return DSBFS_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown internal error";
    return DSBFS_ERR_HIP;
  }
}

}  // namespace dsbfs

using namespace dsbfs;

struct dsbfs_graph {
  Graph *g;
};
struct dsbfs_workspace {
  Workspace *w;
};
struct dsbfs_server {
  Server *s;
};

extern "C" {

dsbfs_status dsbfs_run_opts_default(dsbfs_run_opts *o) {
  return guard([&] {
    if (!o) fail(DSBFS_ERR_INVALID_ARG, "opts must not be NULL");
    run_opts_default(o);
  });
}

dsbfs_status dsbfs_graph_create(const int32_t *src, const int32_t *dst, int64_t num_edges,
                                int32_t num_vertices, const dsbfs_build_opts *opts,
                                const dsbfs_allocator *alloc, void *stream, dsbfs_graph **out) {
  return guard([&] {
    if (!out) fail(DSBFS_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    Graph *g = graph_create(src, dst, num_edges, num_vertices, opts, alloc,
                            static_cast<hipStream_t>(stream), nullptr);
    *out = new dsbfs_graph{g};
  });
}

dsbfs_status dsbfs_graph_create_rmat(const dsbfs_rmat_spec *spec, const dsbfs_build_opts *opts,
                                     const dsbfs_allocator *alloc, void *stream,
                                     dsbfs_graph **out) {
  return guard([&] {
    if (!out || !spec) fail(DSBFS_ERR_INVALID_ARG, "spec and out must not be NULL");
    *out = nullptr;
    Graph *g = graph_create(nullptr, nullptr, 0, 0, opts, alloc,
                            static_cast<hipStream_t>(stream), spec);
    *out = new dsbfs_graph{g};
  });
}

dsbfs_status dsbfs_rmat_generate(const dsbfs_rmat_spec *spec, int32_t *src, int32_t *dst,
                                 void *stream) {
  return guard([&] { rmat_generate(spec, src, dst, static_cast<hipStream_t>(stream)); });
}

dsbfs_status dsbfs_graph_stats_get(const dsbfs_graph *g, dsbfs_graph_stats *out) {
  return guard([&] {
    if (!g || !out) fail(DSBFS_ERR_INVALID_ARG, "graph and out must not be NULL");
    *out = g->g->st;
  });
}

dsbfs_status dsbfs_graph_export(const dsbfs_graph *g, int32_t which, void *host_out,
                                int64_t capacity_bytes, int64_t *bytes) {
  return guard([&] {
    if (!g || !bytes) fail(DSBFS_ERR_INVALID_ARG, "graph and bytes must not be NULL");
    graph_export(g->g, which, host_out, capacity_bytes, bytes);
  });
}

dsbfs_status dsbfs_graph_destroy(dsbfs_graph *g) {
  return guard([&] {
    if (!g) return;
    graph_destroy(g->g);
    delete g;
  });
}

dsbfs_status dsbfs_workspace_create(const dsbfs_graph *g, int32_t max_lanes,
                                    dsbfs_workspace **out) {
  return guard([&] {
    if (!g || !out) fail(DSBFS_ERR_INVALID_ARG, "graph and out must not be NULL");
    *out = nullptr;
    Workspace *w = workspace_create(g->g, max_lanes);
    *out = new dsbfs_workspace{w};
  });
}

dsbfs_status dsbfs_workspace_destroy(dsbfs_workspace *ws) {
  return guard([&] {
    if (!ws) return;
    workspace_destroy(ws->w);
    delete ws;
  });
}

dsbfs_status dsbfs_bfs(const dsbfs_graph *g, dsbfs_workspace *ws, int32_t source,
                       const dsbfs_run_opts *opts, int32_t *depth, int32_t *parent,
                       dsbfs_run_stats *stats, void *stream) {
  return guard([&] {
    if (!g || !ws) fail(DSBFS_ERR_INVALID_ARG, "graph and workspace must not be NULL");
    bfs_run(g->g, ws->w, source, opts, depth, parent, stats, static_cast<hipStream_t>(stream));
  });
}

dsbfs_status dsbfs_bfs_noalloc(const dsbfs_graph *g, int32_t source, const dsbfs_run_opts *opts,
                               int32_t *depth, int32_t *parent, dsbfs_run_stats *stats,
                               void *stream) {
  return guard([&] {
    if (!g) fail(DSBFS_ERR_INVALID_ARG, "graph must not be NULL");
    bfs_run_noalloc(g->g, source, opts, depth, parent, stats, static_cast<hipStream_t>(stream));
  });
}

dsbfs_status dsbfs_pagerank(const dsbfs_graph *g, double alpha, int32_t max_iterations,
                            double tolerance, double *rank, int32_t *iterations_done,
                            double *last_delta, void *stream) {
  return guard([&] {
    if (!g) fail(DSBFS_ERR_INVALID_ARG, "graph must not be NULL");
    pagerank_run(g->g, alpha, max_iterations, tolerance, rank, iterations_done, last_delta,
                 static_cast<hipStream_t>(stream));
  });
}

dsbfs_status dsbfs_msbfs(const dsbfs_graph *g, dsbfs_workspace *ws, const int32_t *sources,
                         int32_t k, const dsbfs_ms_opts *opts, int32_t *depth, void *stream) {
  return guard([&] {
    if (!g || !ws) fail(DSBFS_ERR_INVALID_ARG, "graph and workspace must not be NULL");
    msbfs_run(g->g, ws->w, sources, k, opts, depth, static_cast<hipStream_t>(stream));
  });
}

dsbfs_status dsbfs_msbfs_tune(const dsbfs_graph *g, dsbfs_workspace *ws, const int32_t *sources,
                              int32_t k, const char *cache_path, dsbfs_ms_opts *best,
                              void *stream) {
  return guard([&] {
    if (!g || !ws || !best) fail(DSBFS_ERR_INVALID_ARG, "graph, workspace, best must be given");
    msbfs_tune(g->g, ws->w, sources, k, cache_path, best, static_cast<hipStream_t>(stream));
  });
}

dsbfs_status dsbfs_server_create(const dsbfs_server_opts *opts, const dsbfs_allocator *alloc,
                                 dsbfs_server **out) {
  return guard([&] {
    if (!opts || !out) fail(DSBFS_ERR_INVALID_ARG, "opts and out must not be NULL");
    *out = nullptr;
    Server *s = server_create(opts, alloc);
    *out = new dsbfs_server{s};
  });
}

dsbfs_status dsbfs_server_add_graph(dsbfs_server *s, dsbfs_graph *g, int32_t *graph_id) {
  return guard([&] {
    if (!s || !g || !graph_id) fail(DSBFS_ERR_INVALID_ARG, "server, graph, id must be given");
    server_add_graph(s->s, g->g, graph_id);
    g->g = nullptr;  // ownership moved to the server
    delete g;
  });
}

dsbfs_status dsbfs_server_submit(dsbfs_server *s, int32_t graph_id, int32_t source,
                                 int64_t arrival_ns, int64_t *ticket) {
  return guard([&] {
    if (!s || !ticket) fail(DSBFS_ERR_INVALID_ARG, "server and ticket must not be NULL");
    server_submit(s->s, graph_id, source, arrival_ns, ticket);
  });
}

dsbfs_status dsbfs_server_wait(dsbfs_server *s, int64_t ticket, int64_t timeout_ns,
                               const int32_t **depth_dev, dsbfs_query_stats *stats) {
  dsbfs_status st = DSBFS_OK;
  dsbfs_status g = guard([&] {
    if (!s) fail(DSBFS_ERR_INVALID_ARG, "server must not be NULL");
    st = server_wait(s->s, ticket, timeout_ns, depth_dev, stats);
  });
  return g != DSBFS_OK ? g : st;
}

dsbfs_status dsbfs_server_release(dsbfs_server *s, int64_t ticket) {
  return guard([&] {
    if (!s) fail(DSBFS_ERR_INVALID_ARG, "server must not be NULL");
    server_release(s->s, ticket);
  });
}

dsbfs_status dsbfs_server_stats_get(dsbfs_server *s, dsbfs_server_stats *out) {
  return guard([&] {
    if (!s || !out) fail(DSBFS_ERR_INVALID_ARG, "server and out must not be NULL");
    server_stats(s->s, out);
  });
}

dsbfs_status dsbfs_server_destroy(dsbfs_server *s) {
  return guard([&] {
    if (!s) return;
    server_destroy(s->s);
    delete s;
  });
}

int64_t dsbfs_now_ns(void) { return now_ns(); }

const char *dsbfs_status_str(dsbfs_status st) {
  switch (st) {
    case DSBFS_OK: return "ok";
    case DSBFS_ERR_INVALID_ARG: return "invalid argument";
    case DSBFS_ERR_RANGE: return "out of range";
    case DSBFS_ERR_OUT_OF_MEMORY: return "out of memory";
    case DSBFS_ERR_BUDGET: return "HBM budget exhausted";
    case DSBFS_ERR_HIP: return "HIP runtime error";
    case DSBFS_ERR_NOT_READY: return "not ready";
    case DSBFS_ERR_DEVICE: return "device-side failure";
    default: return "unknown status";
  }
}

const char *dsbfs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
