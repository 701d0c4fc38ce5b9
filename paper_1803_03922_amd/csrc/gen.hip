// Device-side RMAT generation (the paper's workload generator runs on the
// GPUs too, Section VI-A "Reporting").
//
// Same definition as the host generator of the seeded inputs: scale N, 2^N
// vertices, each edge e picks one quadrant per level i (0..N-1) from the
// high 32 bits of the (64 e + i)-th output of a counter-based SplitMix64
// stream (Steele, Lea, Flood, OOPSLA 2014), against thresholds
// floor(p * 2^32) of the cumulative probabilities a, a+b, a+b+c; then both
// endpoints go through a seeded bijection of N-bit integers (four rounds of
// multiply by an odd constant, xor with a right shift by N/2, add a
// constant), the "deterministic hashing" of vertex IDs. Integer arithmetic
// only, so the device and host edge lists are equal bit for bit.
#include "internal.hpp"

namespace dsbfs {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// k-th output (k >= 0) of the SplitMix64 stream with initial state seed.
__host__ __device__ inline uint64_t sm64_at(uint64_t seed, uint64_t k) {
  return sm64_mix(seed + (k + 1) * kGamma);
}

struct PermKey {
  uint64_t mul[4], add[4], mask;
  int shift;
  int on;
};

PermKey perm_key(int bits, uint64_t seed, bool on) {
  PermKey k{};
  k.on = on;
  k.mask = (uint64_t(1) << bits) - 1;
  k.shift = bits / 2 > 0 ? bits / 2 : 1;
  for (int r = 0; r < 4; ++r) {
    k.mul[r] = (sm64_at(seed, uint64_t(2 * r)) | 1ULL) & k.mask;
    if (k.mul[r] == 0) k.mul[r] = 1;
    k.add[r] = sm64_at(seed, uint64_t(2 * r + 1)) & k.mask;
  }
  return k;
}

__device__ __forceinline__ uint32_t perm_apply(const PermKey &k, uint32_t x0) {
  if (!k.on) return x0;
  uint64_t x = x0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    x = (x * k.mul[r]) & k.mask;
    x ^= x >> k.shift;
    x = (x + k.add[r]) & k.mask;
  }
  return uint32_t(x);
}

struct RmatArgs {
  int N;
  int64_t g;
  uint32_t t1, t2, t3;
  uint64_t seed;
  PermKey perm;
};

__device__ __forceinline__ void rmat_edge(const RmatArgs &a, int64_t e, uint32_t &u,
                                          uint32_t &v) {
  u = 0;
  v = 0;
  const uint64_t base = uint64_t(e) * 64u;
  for (int i = 0; i < a.N; ++i) {
    const uint32_t r = uint32_t(sm64_at(a.seed, base + uint64_t(i)) >> 32);
    const uint32_t rb = r >= a.t2, cb = (r >= a.t1 && r < a.t2) || r >= a.t3;
    u |= rb << (a.N - 1 - i);
    v |= cb << (a.N - 1 - i);
  }
  u = perm_apply(a.perm, u);
  v = perm_apply(a.perm, v);
}

__global__ void k_rmat_edges(RmatArgs a, int32_t *src, int32_t *dst) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < a.g;
       e += int64_t(gridDim.x) * blockDim.x) {
    uint32_t u, v;
    rmat_edge(a, e, u, v);
    src[e] = int32_t(u);
    dst[e] = int32_t(v);
  }
}

// Both directions of every edge that is not a self-loop, as (row << B) | col
// keys, appended in wave order (the builder sorts them).
__global__ void k_rmat_keys(RmatArgs a, int B, uint64_t *keys, unsigned long long *cursor) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e0 = int64_t(blockIdx.x) * blockDim.x; e0 < a.g; e0 += stride) {
    const int64_t e = e0 + threadIdx.x;
    uint32_t u = 0, v = 0;
    bool keep = false;
    if (e < a.g) {
      rmat_edge(a, e, u, v);
      keep = u != v;
    }
    const int64_t pos = wave_append(keep, cursor);
    if (keep) {
      keys[2 * pos] = (uint64_t(u) << B) | uint64_t(v);
      keys[2 * pos + 1] = (uint64_t(v) << B) | uint64_t(u);
    }
  }
}

RmatArgs rmat_args(const dsbfs_rmat_spec *sp) {
  if (!sp) fail(DSBFS_ERR_INVALID_ARG, "RMAT spec must not be NULL");
  if (sp->scale < 1 || sp->scale > 31) fail(DSBFS_ERR_INVALID_ARG, "scale must be in [1, 31]");
  if (sp->num_edges < 0) fail(DSBFS_ERR_INVALID_ARG, "num_edges must be >= 0");
  if (!(sp->a >= 0 && sp->b >= 0 && sp->c >= 0 && sp->a + sp->b + sp->c <= 1.0))
    fail(DSBFS_ERR_INVALID_ARG, "quadrant probabilities must be >= 0 with a + b + c <= 1");
  const double two32 = 4294967296.0;
  const double c1 = sp->a * two32, c2 = (sp->a + sp->b) * two32,
               c3 = (sp->a + sp->b + sp->c) * two32;
  RmatArgs a{};
  a.N = sp->scale;
  a.g = sp->num_edges;
  a.t1 = c1 >= two32 ? 0xFFFFFFFFu : uint32_t(c1);
  a.t2 = c2 >= two32 ? 0xFFFFFFFFu : uint32_t(c2);
  a.t3 = c3 >= two32 ? 0xFFFFFFFFu : uint32_t(c3);
  a.seed = sp->seed;
  a.perm = perm_key(sp->scale, sp->perm_seed, sp->permute != 0);
  return a;
}

}  // namespace

void rmat_generate(const dsbfs_rmat_spec *sp, int32_t *src, int32_t *dst, hipStream_t s) {
  const RmatArgs a = rmat_args(sp);
  if (a.g > 0 && (!src || !dst)) fail(DSBFS_ERR_INVALID_ARG, "src/dst must not be NULL");
  if (a.g == 0) return;
  hipLaunchKernelGGL(k_rmat_edges, dim3(grid_for(a.g, 256, 65536)), dim3(256), 0, s, a, src, dst);
  HIPCHK(hipGetLastError());
}

int64_t rmat_pack_keys(const dsbfs_rmat_spec *sp, int B, uint64_t *keys, unsigned long long *cursor,
                       hipStream_t s) {
  const RmatArgs a = rmat_args(sp);
  if (a.g == 0) return 0;
  HIPCHK(hipMemsetAsync(cursor, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_rmat_keys, dim3(grid_for(a.g, 256, 65536)), dim3(256), 0, s, a, B, keys,
                     cursor);
  HIPCHK(hipGetLastError());
  return 2 * int64_t(d2h_scalar(reinterpret_cast<const uint64_t *>(cursor), s));
}

}  // namespace dsbfs
