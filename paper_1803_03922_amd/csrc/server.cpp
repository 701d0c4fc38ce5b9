#include <chrono>
#include "internal.hpp"
namespace dsbfs {
struct Server {};
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}
Server *server_create(const dsbfs_server_opts *, const dsbfs_allocator *) {
  fail(DSBFS_ERR_INVALID_ARG, "server is not available in this build");
}
void server_add_graph(Server *, Graph *, int32_t *) {}
void server_submit(Server *, int32_t, int32_t, int64_t, int64_t *) {}
dsbfs_status server_wait(Server *, int64_t, int64_t, const int32_t **, dsbfs_query_stats *) {
  return DSBFS_ERR_INVALID_ARG;
}
void server_release(Server *, int64_t) {}
void server_destroy(Server *) {}
}  // namespace dsbfs
