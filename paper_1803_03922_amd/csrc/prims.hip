// Device-wide primitives for the graph builder and the search drivers:
// exclusive scan, order-preserving compaction and LSD radix sort of 64-bit
// keys. Tiles are wave64-native: block-level scans are built from wave
// shuffles plus one LDS slot per wave, and the radix scatter ranks keys inside
// a wave by digit matching with 8 ballots (stable, no LDS key staging).
#include "internal.hpp"

namespace dsbfs {

namespace {

constexpr int kBS = 256;             // threads per block of scans/compactions
constexpr int kItems = 8;            // consecutive items per thread
constexpr int64_t kTile = kBS * kItems;
constexpr int kNW = kBS / kWave;

constexpr int kRadixBS = 256;
constexpr int kRadixRounds = 32;     // rounds of kRadixBS keys per tile
constexpr int64_t kRadixTile = int64_t(kRadixBS) * kRadixRounds;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline int64_t ntiles(int64_t N, int64_t tile) { return (N + tile - 1) / tile; }

// Exclusive scan of one value per thread over the block; *total = block sum.
__device__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t *total) {
  const int tid = threadIdx.x, w = tid / kWave, l = tid % kWave;
  int64_t incl = wave_incl_scan(v);
  if (l == kWave - 1) sh[w] = incl;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int i = 0; i < kNW; ++i) {
      int64_t t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[kNW] = run;
  }
  __syncthreads();
  int64_t r = sh[w] + incl - v;
  *total = sh[kNW];
  __syncthreads();
  return r;
}

__device__ int64_t block_sum(int64_t v, int64_t *sh) {
  int64_t t;
  block_excl_scan(v, sh, &t);
  return t;
}

template <class T>
__global__ void __launch_bounds__(kBS) k_scan_reduce(const T *in, int64_t N, int64_t *bsum) {
  __shared__ int64_t sh[kNW + 1];
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(threadIdx.x) * kItems;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (base + k < N) s += static_cast<int64_t>(in[base + k]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

template <class T>
__global__ void __launch_bounds__(kBS) k_scan_down(const T *in, int64_t *out, int64_t N,
                                                    const int64_t *bscan) {
  __shared__ int64_t sh[kNW + 1];
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(threadIdx.x) * kItems;
  T v[kItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = base + k < N ? in[base + k] : T(0);
    s += static_cast<int64_t>(v[k]);
  }
  int64_t total;
  int64_t pre = block_excl_scan(s, sh, &total);
  const int64_t boff = bscan ? bscan[blockIdx.x] : 0;
  pre += boff;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (base + k < N) out[base + k] = pre;
    pre += static_cast<int64_t>(v[k]);
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[N] = boff + total;
}

template <class T>
void scan_impl(const T *in, int64_t *out, int64_t N, void *tmp, hipStream_t s) {
  const int64_t nb = ntiles(N, kTile);
  if (N == 0) {
    HIPCHK(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    return;
  }
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_down<T>, dim3(1), dim3(kBS), 0, s, in, out, N,
                       static_cast<const int64_t *>(nullptr));
    HIPCHK(hipGetLastError());
    return;
  }
  char *t = static_cast<char *>(tmp);
  int64_t *bsum = reinterpret_cast<int64_t *>(t);
  t += align256(size_t(nb) * 8);
  int64_t *bscan = reinterpret_cast<int64_t *>(t);
  t += align256(size_t(nb + 1) * 8);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(unsigned(nb)), dim3(kBS), 0, s, in, N, bsum);
  HIPCHK(hipGetLastError());
  scan_impl<int64_t>(bsum, bscan, nb, t, s);
  hipLaunchKernelGGL(k_scan_down<T>, dim3(unsigned(nb)), dim3(kBS), 0, s, in, out, N,
                     static_cast<const int64_t *>(bscan));
  HIPCHK(hipGetLastError());
}

// ---- compaction -----------------------------------------------------------

struct FlagPred {
  const uint8_t *f;
  __device__ bool operator()(int64_t i) const { return f[i] != 0; }
};
struct FlagOut {
  int32_t *out;
  __device__ void operator()(int64_t pos, int64_t i) const { out[pos] = static_cast<int32_t>(i); }
};
struct UniqPred {
  const uint64_t *k;
  __device__ bool operator()(int64_t i) const { return i == 0 || k[i] != k[i - 1]; }
};
struct UniqOut {
  const uint64_t *k;
  uint64_t *out;
  __device__ void operator()(int64_t pos, int64_t i) const { out[pos] = k[i]; }
};

template <class P>
__global__ void __launch_bounds__(kBS) k_compact_count(P pred, int64_t N, int64_t *bsum) {
  __shared__ int64_t sh[kNW + 1];
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(threadIdx.x) * kItems;
  int64_t c = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (base + k < N && pred(base + k)) ++c;
  c = block_sum(c, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = c;
}

template <class P, class O>
__global__ void __launch_bounds__(kBS) k_compact_write(P pred, O out, int64_t N,
                                                        const int64_t *bscan, int64_t *count) {
  __shared__ int64_t sh[kNW + 1];
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(threadIdx.x) * kItems;
  bool keep[kItems];
  int64_t c = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    keep[k] = base + k < N && pred(base + k);
    c += keep[k];
  }
  int64_t total;
  int64_t pos = block_excl_scan(c, sh, &total);
  const int64_t boff = bscan ? bscan[blockIdx.x] : 0;
  pos += boff;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (keep[k]) out(pos++, base + k);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count = boff + total;
}

template <class P, class O>
void compact_impl(P pred, O out, int64_t N, int64_t *count, void *tmp, hipStream_t s) {
  if (N == 0) {
    HIPCHK(hipMemsetAsync(count, 0, sizeof(int64_t), s));
    return;
  }
  const int64_t nb = ntiles(N, kTile);
  if (nb == 1) {
    hipLaunchKernelGGL((k_compact_write<P, O>), dim3(1), dim3(kBS), 0, s, pred, out, N,
                       static_cast<const int64_t *>(nullptr), count);
    HIPCHK(hipGetLastError());
    return;
  }
  char *t = static_cast<char *>(tmp);
  int64_t *bsum = reinterpret_cast<int64_t *>(t);
  t += align256(size_t(nb) * 8);
  int64_t *bscan = reinterpret_cast<int64_t *>(t);
  t += align256(size_t(nb + 1) * 8);
  hipLaunchKernelGGL((k_compact_count<P>), dim3(unsigned(nb)), dim3(kBS), 0, s, pred, N, bsum);
  HIPCHK(hipGetLastError());
  scan_impl<int64_t>(bsum, bscan, nb, t, s);
  hipLaunchKernelGGL((k_compact_write<P, O>), dim3(unsigned(nb)), dim3(kBS), 0, s, pred, out, N,
                     static_cast<const int64_t *>(bscan), count);
  HIPCHK(hipGetLastError());
}

// ---- radix sort -----------------------------------------------------------

__global__ void __launch_bounds__(kRadixBS) k_radix_hist(const uint64_t *keys, int64_t N,
                                                          int shift, int64_t nb,
                                                          int64_t *ghist) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t tile = int64_t(blockIdx.x) * kRadixTile;
  for (int r = 0; r < kRadixRounds; ++r) {
    int64_t i = tile + int64_t(r) * kRadixBS + threadIdx.x;
    if (i < N) atomicAdd(&hist[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  ghist[int64_t(threadIdx.x) * nb + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter of one tile: keys are taken in rounds of 256 (thread order =
// key order); inside a wave, lanes with equal digits are matched with 8
// ballots, so the rank of a key among equal digits of its wave is a popcount;
// across waves and rounds the running per-digit offsets live in LDS.
__global__ void __launch_bounds__(kRadixBS) k_radix_scatter(const uint64_t *keys, uint64_t *out,
                                                             int64_t N, int shift, int64_t nb,
                                                             const int64_t *gscan) {
  __shared__ int wcnt[kRadixBS / kWave][256];
  __shared__ int64_t base[256];
  __shared__ int rtot[256];
  const int tid = threadIdx.x, w = tid / kWave;
  base[tid] = gscan[int64_t(tid) * nb + blockIdx.x];
  const int64_t tile = int64_t(blockIdx.x) * kRadixTile;
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t rb = tile + int64_t(r) * kRadixBS;
    if (rb >= N) break;  // uniform across the block
    const int64_t i = rb + tid;
    const bool active = i < N;
    const uint64_t key = active ? keys[i] : 0;
    const uint32_t dig = static_cast<uint32_t>((key >> shift) & 255u);
    uint64_t m = __ballot(active);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      m &= bit ? bal : ~bal;
    }
    const uint32_t rank = lanes_below(m);
#pragma unroll
    for (int k = 0; k < kRadixBS / kWave; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    if (active && rank == 0) wcnt[w][dig] = __popcll(m);
    __syncthreads();
    {
      int run = 0;
#pragma unroll
      for (int k = 0; k < kRadixBS / kWave; ++k) {
        int c = wcnt[k][tid];
        wcnt[k][tid] = run;
        run += c;
      }
      rtot[tid] = run;
    }
    __syncthreads();
    if (active) out[base[dig] + wcnt[w][dig] + rank] = key;
    __syncthreads();
    base[tid] += rtot[tid];
    __syncthreads();
  }
}

}  // namespace

size_t scan_tmp_bytes(int64_t N) {
  const int64_t nb = ntiles(N, kTile);
  if (nb <= 1) return 256;
  return align256(size_t(nb) * 8) + align256(size_t(nb + 1) * 8) + scan_tmp_bytes(nb);
}

void scan_excl_i32_to_i64(const int32_t *in, int64_t *out, int64_t N, void *tmp, hipStream_t s) {
  scan_impl<int32_t>(in, out, N, tmp, s);
}
void scan_excl_i64(const int64_t *in, int64_t *out, int64_t N, void *tmp, hipStream_t s) {
  scan_impl<int64_t>(in, out, N, tmp, s);
}

size_t compact_tmp_bytes(int64_t N) { return scan_tmp_bytes(N); }

void compact_flags_u8(const uint8_t *flag, int64_t N, int32_t *out, int64_t *count, void *tmp,
                      hipStream_t s) {
  compact_impl(FlagPred{flag}, FlagOut{out}, N, count, tmp, s);
}

void unique_sorted_u64(const uint64_t *keys, int64_t N, uint64_t *out, int64_t *count, void *tmp,
                       hipStream_t s) {
  compact_impl(UniqPred{keys}, UniqOut{keys, out}, N, count, tmp, s);
}

size_t radix_tmp_bytes(int64_t N) {
  const int64_t nb = ntiles(N, kRadixTile);
  const int64_t H = 256 * (nb > 0 ? nb : 1);
  return align256(size_t(H) * 8) + align256(size_t(H + 1) * 8) + scan_tmp_bytes(H);
}

void radix_sort_u64(uint64_t *keys, uint64_t *alt, int64_t N, int key_bits, void *tmp,
                    hipStream_t s) {
  radix_sort_u64_bits(keys, alt, N, 0, key_bits, tmp, s);
}

void radix_sort_u64_bits(uint64_t *keys, uint64_t *alt, int64_t N, int lo_bit, int hi_bit,
                         void *tmp, hipStream_t s) {
  if (N <= 1 || hi_bit <= lo_bit) return;
  const int64_t nb = ntiles(N, kRadixTile);
  const int64_t H = 256 * nb;
  char *t = static_cast<char *>(tmp);
  int64_t *ghist = reinterpret_cast<int64_t *>(t);
  t += align256(size_t(H) * 8);
  int64_t *gscan = reinterpret_cast<int64_t *>(t);
  t += align256(size_t(H + 1) * 8);
  uint64_t *src = keys, *dst = alt;
  for (int shift = lo_bit; shift < hi_bit; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(unsigned(nb)), dim3(kRadixBS), 0, s, src, N, shift, nb,
                       ghist);
    HIPCHK(hipGetLastError());
    scan_impl<int64_t>(ghist, gscan, H, t, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(unsigned(nb)), dim3(kRadixBS), 0, s, src, dst, N,
                       shift, nb, gscan);
    HIPCHK(hipGetLastError());
    uint64_t *x = src;
    src = dst;
    dst = x;
  }
  if (src != keys)
    HIPCHK(hipMemcpyAsync(keys, src, size_t(N) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
}

}  // namespace dsbfs
