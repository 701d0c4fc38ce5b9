// Plain copy kernel of known size: 1 GiB read and 1 GiB written per
// dispatch. Profiling it with the FETCH_SIZE and WRITE_SIZE counters gives
// the factor that turns those counters into bytes on this device; the same
// factor then scales the counters of the search kernels.
#include <hip/hip_runtime.h>
#include <cstdio>

__global__ void copy_calib_kernel(const int4 *a, int4 *b, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    b[i] = a[i];
}

__global__ void fill_calib_kernel(int4 *a, size_t n, int v) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    a[i] = make_int4(v, v, v, v);
}

static int check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
  }
  return 0;
}

int main() {
  const size_t bytes = size_t(1) << 30;
  const size_t n = bytes / sizeof(int4);
  int4 *a = nullptr, *b = nullptr;
  if (check(hipMalloc(&a, bytes), "hipMalloc") || check(hipMalloc(&b, bytes), "hipMalloc"))
    return 1;
  hipLaunchKernelGGL(fill_calib_kernel, dim3(4096), dim3(256), 0, 0, a, n, 1);
  if (check(hipGetLastError(), "fill")) return 1;
  for (int r = 0; r < 3; ++r) {
    hipLaunchKernelGGL(copy_calib_kernel, dim3(4096), dim3(256), 0, 0, a, b, n);
    if (check(hipGetLastError(), "copy")) return 1;
  }
  if (check(hipDeviceSynchronize(), "sync")) return 1;
  std::printf("copy_calib: 3 dispatches of %zu bytes read + %zu bytes written\n", bytes, bytes);
  (void)hipFree(a);
  (void)hipFree(b);
  return 0;
}
