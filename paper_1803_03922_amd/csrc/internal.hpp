// Internal declarations of the dsbfs HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dsbfs.h"

namespace dsbfs {

constexpr int kWave = 64;
constexpr uint64_t kOffMask = (1ull << 40) - 1;  // packed row offset: start in bits 0..39
constexpr int kOffShift = 40;                    // length of the first part in bits 40..63
constexpr int64_t kMaxFirstPart = (1ll << 24) - 1;

// ---------------------------------------------------------------------------
// Errors: internal code throws dsbfs::Error; the C-ABI layer catches it.
// ---------------------------------------------------------------------------
struct Error {
  dsbfs_status status;
  std::string msg;
};

[[noreturn]] void fail(dsbfs_status st, const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPCHK(x) ::dsbfs::hip_check((x), #x, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// Device memory through the caller's allocator (or hipMalloc).
// ---------------------------------------------------------------------------
struct Alloc {
  dsbfs_allocator a{};
  bool custom = false;
  void *get(size_t bytes, hipStream_t s) const;
  void put(void *p, hipStream_t s) const;
};

// Owning device buffer bound to an allocator.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  const Alloc *al = nullptr;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      reset();
      p = o.p; bytes = o.bytes; al = o.al; s = o.s;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { reset(); }
  void alloc(const Alloc *a, size_t nbytes, hipStream_t st) {
    reset();
    al = a; s = st; bytes = nbytes;
    p = a->get(nbytes < 256 ? 256 : nbytes, st);
  }
  void reset() {
    if (p && al) al->put(p, s);
    p = nullptr; bytes = 0;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// Graph: the degree-separated layout (Section III-C) plus the plain CSR.
//   Normal rows  (n rows, indexed by vertex ID; empty for delegates):
//     [ nn neighbours (vertex IDs) | nd neighbours (delegate IDs) ]
//   Delegate rows (d rows, indexed by delegate ID):
//     [ dd neighbours (delegate IDs) | dn neighbours (vertex IDs) ]
//   noff/doff are packed: start (bits 0..39) | first-part length << 40.
// ---------------------------------------------------------------------------
constexpr uint16_t kLenWide = 0xFFFF;

struct Graph {
  Alloc al;
  hipStream_t stream = nullptr;
  int device = 0;
  int32_t n = 0, d = 0, TH = 0;
  int64_t m = 0;
  dsbfs_graph_stats st{};
  DevBuf deg, did, vid_of, noff, ncol, doff, dcol, ndsrc, ddsrc_mask, dnsrc_mask;
  // nd rows again, in nd-source-list order (row i = nd part of ndsrc[i]), so
  // bottom-up passes over the source list stream them: int64 [n_ndsrc+1],
  // int32 [e_nd] delegate IDs.
  DevBuf nds_off, nds_col, nds_first;
  DevBuf dd_first;  // per delegate: (first dd neighbour, its vertex), or (-1, -1)
  // per vertex, uint16: nn length | nd length << 8 of a normal row (0 for a
  // delegate), kLenWide when either is 255 or more (read noff instead); the
  // normal previsit reads these 2 bytes instead of two 8-byte row offsets
  DevBuf nlen;
  DevBuf nnsrc;     // normal vertices with a normal neighbour, ascending (nn_do bottom-up)
  // nn parts again, concatenated in vertex order (int32 [e_nn] vertex IDs),
  // and the start of each vertex's part (uint32 [n]): a forward nn visit
  // reads 4 bytes per frontier vertex and a column array of 4 bytes per nn
  // edge, where most parts are one or two entries, instead of the 8-byte
  // packed offset and a line of the full row. Not built (null) when
  // e_nn >= 2^32; the kernels then read noff and ncol.
  DevBuf nnoff, nncol;
  DevBuf poff, pcol;  // plain CSR: int64 offsets [n+1], int32 columns [m]
  // PageRank's gather-friendly copy, built by its first call and kept with
  // the graph: pr_rank[k] = rank of delegate k by descending degree (ties by
  // ID), and pr_col = dcol with every dd entry replaced by that rank, so the
  // contributions of the most-gathered delegates sit together (int32 [d],
  // int32 [e_dd + e_dn]).
  mutable DevBuf pr_rank, pr_col;
  mutable std::mutex pr_mu;
  int32_t dwords() const { return (d + 31) / 32; }
  int32_t nwords() const { return (n + 31) / 32; }
};

// Per-level counters of a single-source search (device; accumulated with
// wave-aggregated atomics). Two copies alternate between levels.
struct LevelCtr {
  // Tails of the next normal queue (bits 0..31: the queue length of the next
  // level) and of the next bottom-up normal candidate list (bits 32..63), in
  // one word: the bottom-up normal pass appends to both and reserves both
  // with one atomic. Neither count reaches 2^31, so no carry crosses.
  unsigned long long qn_nc;
  unsigned long long nd_list;   // frontier delegates of this level (length of dlist)
  unsigned long long nd_cand;   // unvisited delegates with a dd or dn edge (length of dcand)
  unsigned long long fv_nn, q_nn, fv_nd, q_nd;  // normal previsit
  unsigned long long fv_dd, q_dd, fv_dn, q_dn;  // delegate previsit
  // Work units per kernel (index DSBFS_K_*), slot meanings in bfs.hip.
  unsigned long long units[DSBFS_NUM_KERNELS][4];
};

__host__ __device__ inline int64_t lc_qn(const LevelCtr *c) {
  return int64_t(c->qn_nc & 0xffffffffull);
}
__host__ __device__ inline int64_t lc_nc(const LevelCtr *c) { return int64_t(c->qn_nc >> 32); }

// Scratch of one search at a time (single-source and multi-source).
struct Workspace {
  const Graph *g = nullptr;
  int32_t max_lanes = 0;
  // uint32 bitmaps: visited / frontier normals; visited at level start,
  // frontier, and claimed (visited or found this level) delegates
  DevBuf Vn, Fn, Vd, Fd, Cd;
  DevBuf q0, q1;               // normal queues, int32[n]
  DevBuf dlist, dcand, dlen;   // int32[d]
  DevBuf dscan;                // int64[max(n, d) + 1]: prefix of top-down lengths
  DevBuf c0, c1;               // bottom-up normal candidates, int32[n_ndsrc]
  DevBuf ctr;                  // LevelCtr[2]
  DevBuf scan_tmp;
  LevelCtr *hctr = nullptr;    // pinned host copy of ctr
  std::vector<hipEvent_t> events;  // profiling event pool
  // device-side level control of degree-separated DOBFS (bfs.hip)
  DevBuf dctl;                 // control block of the search in progress
  DevBuf dtiles;               // tile sums and their scan (delegate-frontier prefix sum)
  void *hstat = nullptr;       // pinned ring of per-level status records
  void *lvl = nullptr;         // captured level graphs
  hipEvent_t lev_ev[3] = {};   // completion of recent levels
  // multi-source lane state
  void *ms_state = nullptr;           // launch state of multi-source BFS (msbfs.hip)
  // borrowed: every buffer points into memory the workspace does not own (the
  // allocation-free search's static scratch); hstat is then device memory,
  // read by copies, and hctr a host buffer of the caller's frame
  bool borrowed = false;
  ~Workspace();
};

// Per-lane result rows of a level-at-a-time multi-source step (server).
// Sources of the lanes admitted at one level (by value: no copy per level).
struct SeedList {
  int32_t src[64];
};

// Rows written by one flush of the server's level ring (see k_lv_flush).
struct LaneFlush {
  int32_t *res[64];    // result row of each lane (int32[n]) or NULL if the lane is idle
  int32_t start[64];   // level at which each lane's source had depth 0
  uint64_t valid[16];  // per level jlo + o: the lanes whose unwritten levels include it
  uint64_t lanes;      // lanes considered
  int32_t jlo, jhi;    // levels [jlo, jhi], jhi - jlo < 16
  int32_t final;       // 1: only lanes whose frontier ran empty; write -1 where unreached
};

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of mask in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

template <class T> __device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Cross-lane moves through DPP (data-parallel primitives: a VALU operand
// modifier, no LDS round trip, unlike ds_bpermute behind __shfl). Lanes whose
// source is outside the row / wave, or whose row is masked off, read `old`.
constexpr int kDppRowShr = 0x110;   // + n (1..15): lane l reads l - n within its 16-lane row
constexpr int kDppWaveShl1 = 0x130; // lane l reads l + 1
constexpr int kDppWaveShr1 = 0x138; // lane l reads l - 1
constexpr int kDppBcast15 = 0x142;  // rows 1..3 read lane 15 of the previous row
constexpr int kDppBcast31 = 0x143;  // rows 2..3 read lane 31
template <int Ctrl, int RowMask = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(old), int(v), Ctrl, RowMask, 0xf, false));
}

// Lane `src` (wave-uniform) of v, through a scalar register.
__device__ __forceinline__ int32_t lane_read(int32_t v, int src) {
  return __builtin_amdgcn_readlane(v, src);
}
__device__ __forceinline__ int64_t lane_read(int64_t v, int src) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(uint64_t(v))), src));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(uint64_t(v) >> 32)), src));
  return int64_t((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ unsigned long long lane_read(unsigned long long v, int src) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), src));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), src));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// OR of a 64-bit value over the wave, returned to every lane (DPP inclusive
// OR-scan of each half, then lane 63 through a scalar register). The whole
// wave must be active.
__device__ __forceinline__ uint32_t wave_or_dpp_u32(uint32_t x) {
  x |= dpp_u32<kDppRowShr + 1>(0u, x);
  x |= dpp_u32<kDppRowShr + 2>(0u, x);
  x |= dpp_u32<kDppRowShr + 4>(0u, x);
  x |= dpp_u32<kDppRowShr + 8>(0u, x);
  x |= dpp_u32<kDppBcast15, 0xa>(0u, x);
  x |= dpp_u32<kDppBcast31, 0xc>(0u, x);
  return uint32_t(__builtin_amdgcn_readlane(int(x), kWave - 1));
}
__device__ __forceinline__ uint64_t wave_or_all(uint64_t x) {
  const uint32_t lo = wave_or_dpp_u32(uint32_t(x));
  const uint32_t hi = wave_or_dpp_u32(uint32_t(x >> 32));
  return (uint64_t(hi) << 32) | lo;
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <class T> __device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = lane_id();
  for (int o = 1; o < kWave; o <<= 1) {
    T t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}
// 32-bit version with DPP: Hillis-Steele inside each 16-lane row, then the
// row totals carried across rows by two broadcasts.
template <> __device__ __forceinline__ int32_t wave_incl_scan<int32_t>(int32_t v) {
  uint32_t x = uint32_t(v);
  x += dpp_u32<kDppRowShr + 1>(0u, x);
  x += dpp_u32<kDppRowShr + 2>(0u, x);
  x += dpp_u32<kDppRowShr + 4>(0u, x);
  x += dpp_u32<kDppRowShr + 8>(0u, x);
  x += dpp_u32<kDppBcast15, 0xa>(0u, x);
  x += dpp_u32<kDppBcast31, 0xc>(0u, x);
  return int32_t(x);
}

// Wave-aggregated append: every lane with `want` gets a distinct slot of
// *counter (returned), one atomic per wave. Lanes without `want` get -1.
__device__ __forceinline__ int64_t wave_append(bool want, unsigned long long *counter) {
  uint64_t m = __ballot(want);
  if (m == 0) return -1;
  int leader = __ffsll(static_cast<long long>(m)) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, static_cast<unsigned long long>(__popcll(m)));
  base = lane_read(base, leader);
  return want ? static_cast<int64_t>(base + lanes_below(m)) : -1;
}

__device__ __forceinline__ bool bit_test(const uint32_t *bm, uint32_t v) {
  return (bm[v >> 5] >> (v & 31)) & 1u;
}
// Test-and-set: true iff this call changed the bit from 0 to 1.
__device__ __forceinline__ bool bit_claim(uint32_t *bm, uint32_t v) {
  const uint32_t b = 1u << (v & 31);
  if (__hip_atomic_load(&bm[v >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & b) return false;
  return !(atomicOr(&bm[v >> 5], b) & b);
}

// Wave-cooperative bitmap update for lanes whose bits tend to share words
// (vertices visited in ascending order). Adjacent lanes with the same word
// form a run; a segmented OR-scan combines the run's bits and the run's last
// lane issues the one atomicOr. Atomics on one word from many lanes of one
// instruction serialize in the cache, so this is several times faster than a
// per-lane atomicOr on ascending patterns. Must be called by the whole wave.
//   claim: returns true for exactly one lane per bit that was 0 before the
//   call (a bit wanted by several lanes of one run goes to the lowest lane).
struct WaveBits {
  uint32_t word, bit, incl, old;
  bool want, head;
  // valid: v is a vertex (its word joins a run even without a bit, so the
  // runs of an ascending list are not cut by lanes that want nothing)
  __device__ __forceinline__ void run(uint32_t *bm, uint32_t v, bool valid, bool w,
                                      bool need_old) {
    const int l = lane_id();
    want = valid && w;
    word = valid ? (v >> 5) : 0xffffffffu;
    bit = want ? (1u << (v & 31)) : 0u;
    // neighbours' words (lane 0 / lane 63 read a value no word can take)
    const uint32_t prev_word = dpp_u32<kDppWaveShr1>(0xfffffffeu, word);
    const uint32_t next_word = dpp_u32<kDppWaveShl1>(0xfffffffeu, word);
    head = l == 0 || prev_word != word;
    const bool tail = l == kWave - 1 || next_word != word;
    // segmented inclusive OR-scan (incl = OR of the bits from the run's head
    // to this lane) with DPP; f marks that a head lies within the span so far
    incl = bit;
    uint32_t f = head ? 1u : 0u, t, tf;
#define DSBFS_SEG_STEP(CTRL, MASK)              \
    t = dpp_u32<CTRL, MASK>(0u, incl);           \
    tf = dpp_u32<CTRL, MASK>(0u, f);             \
    if (!f) incl |= t;                           \
    f |= tf;
    DSBFS_SEG_STEP(kDppRowShr + 1, 0xf)
    DSBFS_SEG_STEP(kDppRowShr + 2, 0xf)
    DSBFS_SEG_STEP(kDppRowShr + 4, 0xf)
    DSBFS_SEG_STEP(kDppRowShr + 8, 0xf)
    DSBFS_SEG_STEP(kDppBcast15, 0xa)
    DSBFS_SEG_STEP(kDppBcast31, 0xc)
#undef DSBFS_SEG_STEP
    old = 0;
    if (tail && word != 0xffffffffu && incl) old = atomicOr(&bm[word], incl);
    if (need_old) {
      // the run's tail is the first tail lane at or after this lane
      const uint64_t tails = __ballot(tail);
      const int tp = l + __builtin_ctzll(tails >> l);
      old = uint32_t(__shfl(int(old), tp, kWave));
    }
  }
  // true iff this lane set its bit first (bit was 0 and no lower lane of the run wanted it)
  __device__ __forceinline__ bool won() const {
    const uint32_t before = dpp_u32<kDppWaveShr1>(0u, incl);
    const uint32_t excl = head ? 0u : before;
    return want && !(old & bit) && !(excl & bit);
  }
};

__device__ __forceinline__ bool wave_bit_claim(uint32_t *bm, uint32_t v, bool valid, bool want) {
  WaveBits wb;
  wb.run(bm, v, valid, want, true);
  return wb.won();
}

__device__ __forceinline__ void wave_bit_set(uint32_t *bm, uint32_t v, bool valid, bool want) {
  WaveBits wb;
  wb.run(bm, v, valid, want, false);
}

// Orders LDS traffic of one wave around a point where lanes read what other
// lanes of the same wave wrote.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-level append buffer in LDS for grid-stride kernels: lanes reserve
// slots with one LDS atomic per wave; the block writes the buffer out with a
// single global atomic per flush, coalesced. Device-scope atomics on one
// global counter serialize across the chip, so kernels never do one per wave.
// Appends beyond the buffer (only possible if one iteration produces more
// than `cap - margin` entries) fall back to a wave-aggregated global append.
struct BlockAppend {
  int32_t *buf;              // LDS, cap entries
  int *count;                // LDS
  unsigned long long *base;  // LDS
  int cap;
  unsigned long long *gcount;
  int32_t *gout;
  int shift = 0;  // the 32-bit half of *gcount that counts this list (0 or 32)

  // Reserves n entries of the list: the old count of its half of *gcount.
  __device__ unsigned long long reserve(unsigned long long n) const {
    return (atomicAdd(gcount, n << shift) >> shift) & 0xffffffffull;
  }

  __device__ void init() {
    if (threadIdx.x == 0) *count = 0;
  }
  // Called by every lane of a wave (wave-uniform).
  __device__ void push(bool want, int32_t v) {
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    const int leader = __ffsll(static_cast<long long>(m)) - 1;
    int p = 0;
    if (lane_id() == leader) p = atomicAdd(count, __popcll(m));
    p = lane_read(p, leader);
    const int pos = p + int(lanes_below(m));
    const bool over = want && pos >= cap;
    if (want && !over) buf[pos] = v;
    const uint64_t mo = __ballot(over);
    if (mo) {
      const int lo = __ffsll(static_cast<long long>(mo)) - 1;
      unsigned long long b = 0;
      if (lane_id() == lo) b = reserve(__popcll(mo));
      b = lane_read(b, lo);
      if (over) gout[b + lanes_below(mo)] = v;
    }
  }
  // Block-uniform: writes the buffer out if it holds more than cap - margin.
  __device__ void maybe_flush(int margin) {
    __syncthreads();
    if (*count > cap - margin) flush();
  }
  // Block-uniform.
  __device__ void flush() {
    __syncthreads();
    const int c = min(*count, cap);
    if (threadIdx.x == 0) *base = c ? reserve((unsigned long long)c) : 0ull;
    __syncthreads();
    const unsigned long long b = *base;
    for (int i = threadIdx.x; i < c; i += blockDim.x) gout[b + i] = buf[i];
    __syncthreads();
    if (threadIdx.x == 0) *count = 0;
    __syncthreads();
  }
};

// Writes out two append buffers that count in the two halves of one word
// (q: bits 0..31, c: bits 32..63) with a single atomic (block-uniform).
__device__ inline void flush_pair(BlockAppend &q, BlockAppend &c) {
  __syncthreads();
  const int nq = min(*q.count, q.cap), nc = min(*c.count, c.cap);
  if (threadIdx.x == 0) {
    unsigned long long b = 0;
    if (nq || nc)
      b = atomicAdd(q.gcount, (static_cast<unsigned long long>(nc) << 32) |
                                  static_cast<unsigned long long>(nq));
    *q.base = b & 0xffffffffull;
    *c.base = b >> 32;
  }
  __syncthreads();
  const unsigned long long bq = *q.base, bc = *c.base;
  for (int i = threadIdx.x; i < nq; i += blockDim.x) q.gout[bq + i] = q.buf[i];
  for (int i = threadIdx.x; i < nc; i += blockDim.x) c.gout[bc + i] = c.buf[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    *q.count = 0;
    *c.count = 0;
  }
  __syncthreads();
}

// Sums four per-thread counts over the block and adds them to dst[0..3] with
// one global atomic each (block-uniform call; sh holds 4 * waves entries).
__device__ __forceinline__ void block_add4(unsigned long long *dst, unsigned long long a,
                                           unsigned long long b, unsigned long long c,
                                           unsigned long long d, unsigned long long *sh) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  d = wave_sum(d);
  if (lane_id() == 0) {
    sh[w] = a;
    sh[nw + w] = b;
    sh[2 * nw + w] = c;
    sh[3 * nw + w] = d;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long t = 0;
    for (int i = 0; i < nw; ++i) t += sh[threadIdx.x * nw + i];
    if (t) atomicAdd(&dst[threadIdx.x], t);
  }
  __syncthreads();
}

__device__ __forceinline__ int64_t row_start(uint64_t w) { return static_cast<int64_t>(w & kOffMask); }
__device__ __forceinline__ int64_t row_first(uint64_t w) { return static_cast<int64_t>(w >> kOffShift); }

inline int grid_for(int64_t items, int per_block, int cap = 65536) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

// ---------------------------------------------------------------------------
// Device-wide primitives (prims.hip).
// ---------------------------------------------------------------------------
// out[i] = sum of in[0..i), i in [0, N]; out has N+1 entries. tmp is scratch
// of scan_tmp_bytes(N) bytes.
size_t scan_tmp_bytes(int64_t N);
void scan_excl_i32_to_i64(const int32_t *in, int64_t *out, int64_t N, void *tmp, hipStream_t s);
void scan_excl_i64(const int64_t *in, int64_t *out, int64_t N, void *tmp, hipStream_t s);

// LSD radix sort of N uint64 keys over bits [0, key_bits). Result lands in
// keys (alt is scratch of N keys). hist_tmp is radix_tmp_bytes(N) bytes.
size_t radix_tmp_bytes(int64_t N);
void radix_sort_u64(uint64_t *keys, uint64_t *alt, int64_t N, int key_bits, void *hist_tmp,
                    hipStream_t s);
// Stable sort on bits [lo_bit, hi_bit) only (keys already ordered below lo_bit
// keep that order among equal sort fields).
void radix_sort_u64_bits(uint64_t *keys, uint64_t *alt, int64_t N, int lo_bit, int hi_bit,
                         void *hist_tmp, hipStream_t s);

// Order-preserving compaction of indices i in [0, N) with flag[i] != 0 into
// out; *count (device) gets the number kept. tmp: compact_tmp_bytes(N).
size_t compact_tmp_bytes(int64_t N);
void compact_flags_u8(const uint8_t *flag, int64_t N, int32_t *out, int64_t *count, void *tmp,
                      hipStream_t s);
// Keeps keys[i] where i == 0 or keys[i] != keys[i-1] (sorted input -> unique).
void unique_sorted_u64(const uint64_t *keys, int64_t N, uint64_t *out, int64_t *count, void *tmp,
                       hipStream_t s);

// Host helpers.
template <class T> T d2h_scalar(const T *dptr, hipStream_t s) {
  T v{};
  HIPCHK(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

}  // namespace dsbfs
