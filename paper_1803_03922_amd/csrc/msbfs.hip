#include "internal.hpp"
namespace dsbfs {
void msbfs_run(const Graph *, Workspace *, const int32_t *, int32_t, const dsbfs_ms_opts *,
               int32_t *, hipStream_t) {
  fail(DSBFS_ERR_INVALID_ARG, "multi-source BFS is not available in this build");
}
void msbfs_tune(const Graph *, Workspace *, const int32_t *, int32_t, const char *,
                dsbfs_ms_opts *, hipStream_t) {
  fail(DSBFS_ERR_INVALID_ARG, "multi-source BFS is not available in this build");
}
}  // namespace dsbfs
