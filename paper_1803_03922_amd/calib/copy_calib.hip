// Kernels of known traffic for calibrating the HBM counters (FETCH_SIZE,
// WRITE_SIZE) on this device:
//   copy_calib_kernel:    1 GiB read and 1 GiB written per dispatch, streaming;
//   gather_calib_kernel:  2^24 reads of 4 bytes, each in its own 128-byte line
//                         of a 4 GiB array (lines visited in a scattered
//                         order), plus 4 bytes written per thread;
//   scatter_calib_kernel: 2^24 writes of 4 bytes, each in its own 128-byte
//                         line, scattered the same way.
// Profiling each with one counter per run gives the factor that turns the
// counters into bytes for streaming traffic, and what one scattered 4-byte
// access costs in counted traffic.
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

// Line of access i: an odd multiplier mod 2^lines_log2 is a bijection, so the
// 2^24 accesses of a dispatch touch 2^24 distinct lines.
__device__ __forceinline__ size_t scattered_line(size_t i, int lines_log2) {
  return (i * 0x9E3779B1ull) & ((size_t(1) << lines_log2) - 1);
}

__global__ void gather_calib_kernel(const int *a, int *out, size_t reads, int lines_log2) {
  int s = 0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < reads;
       i += size_t(gridDim.x) * blockDim.x)
    s += a[scattered_line(i, lines_log2) * 32];   // 32 ints = one 128-byte line
  out[blockIdx.x * size_t(blockDim.x) + threadIdx.x] = s;
}

__global__ void scatter_calib_kernel(int *a, size_t writes, int lines_log2, int v) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < writes;
       i += size_t(gridDim.x) * blockDim.x)
    a[scattered_line(i, lines_log2) * 32] = v;
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

  // scattered accesses over a 4 GiB array: 2^25 lines of 128 bytes
  const int lines_log2 = 25;
  const size_t big = (size_t(1) << lines_log2) * 128;
  const size_t accesses = size_t(1) << 24;
  const int grid = 4096, block = 256;
  int *g = nullptr, *out = nullptr;
  if (check(hipMalloc(&g, big), "hipMalloc") ||
      check(hipMalloc(&out, size_t(grid) * block * sizeof(int)), "hipMalloc"))
    return 1;
  hipLaunchKernelGGL(fill_calib_kernel, dim3(4096), dim3(256), 0, 0, reinterpret_cast<int4 *>(g),
                     big / sizeof(int4), 2);
  if (check(hipGetLastError(), "fill")) return 1;
  // each dispatch timed with events on the null stream: the rate of scattered
  // single-word accesses, the ceiling of a kernel made of them
  hipEvent_t ev[7];
  for (auto &e : ev)
    if (check(hipEventCreate(&e), "hipEventCreate")) return 1;
  if (check(hipEventRecord(ev[0], 0), "hipEventRecord")) return 1;
  for (int r = 0; r < 3; ++r) {
    hipLaunchKernelGGL(gather_calib_kernel, dim3(grid), dim3(block), 0, 0, g, out, accesses,
                       lines_log2);
    if (check(hipGetLastError(), "gather")) return 1;
    if (check(hipEventRecord(ev[1 + r], 0), "hipEventRecord")) return 1;
  }
  for (int r = 0; r < 3; ++r) {
    hipLaunchKernelGGL(scatter_calib_kernel, dim3(grid), dim3(block), 0, 0, g, accesses,
                       lines_log2, r);
    if (check(hipGetLastError(), "scatter")) return 1;
    if (check(hipEventRecord(ev[4 + r], 0), "hipEventRecord")) return 1;
  }
  if (check(hipDeviceSynchronize(), "sync")) return 1;
  float ms[6];
  for (int r = 0; r < 6; ++r)
    if (check(hipEventElapsedTime(&ms[r], ev[r], ev[r + 1]), "hipEventElapsedTime")) return 1;
  std::printf("gather_calib: 3 dispatches of %zu scattered 4-byte reads (+ %zu bytes written); "
              "ms %.4f %.4f %.4f; last: %.2f G reads/s\n",
              accesses, size_t(grid) * block * sizeof(int), ms[0], ms[1], ms[2],
              accesses / (ms[2] * 1e-3) / 1e9);
  std::printf("scatter_calib: 3 dispatches of %zu scattered 4-byte writes; ms %.4f %.4f %.4f; "
              "last: %.2f G writes/s\n",
              accesses, ms[3], ms[4], ms[5], accesses / (ms[5] * 1e-3) / 1e9);
  for (auto &e : ev) (void)hipEventDestroy(e);
  (void)hipFree(g);
  (void)hipFree(out);
  return 0;
}
