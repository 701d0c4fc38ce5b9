// Single-source BFS on one GPU.
//
// Mode 1 is the paper's degree-separated direction-optimized BFS at p = 1
// (Section IV): the normal frontier is a compacted queue, the delegate
// frontier a bitmask (Section IV-A). Each level runs
//   previsit  - normal queue: nn/nd workloads, normal frontier bitmap;
//               delegate mask: frontier list, dd/dn workloads, bottom-up
//               candidate list (Section IV, "previsit");
//   decision  - per kernel dd, dn, nd: FV vs BV = |U|(q+s)/q with factor0 /
//               factor1 (Section IV-B); nn is always top-down;
//   visits    - top-down: normal queue over nn (+nd), delegate list over dd
//               and/or dn with merge-path style load balance over the
//               frontier's prefix sum; bottom-up: dn via the nd rows of the nd
//               source list, dd and nd via the delegate rows of unvisited
//               delegates, each stopping at the first frontier parent;
//   close     - Fd = Cd & ~Vd, Vd = Cd, clear the normal frontier bitmap.
// Exactly-once discovery comes from atomic test-and-set on the claimed
// bitmaps (normals: Vn; delegates: Cd = visited or found this level), so
// queues hold no duplicates and depth/parent are written once per vertex.
// The normal previsit and the nn top-down visit share one pass over the
// queue: nn is always top-down, and its claims change none of the decision's
// inputs (those come from the frontier and from running counts).
//
// Mode 0 is plain top-down BFS over the plain CSR (the paper's "BFS" beside
// "DOBFS", Section VI-C), with the same load-balanced expansion.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace dsbfs {

void msbfs_release(Workspace *ws);

void level_graphs_release(Workspace *ws);

Workspace::~Workspace() {
  msbfs_release(this);
  level_graphs_release(this);
  if (hctr && !borrowed) (void)hipHostFree(hctr);
  if (hstat && !borrowed) (void)hipHostFree(hstat);
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  for (hipEvent_t e : lev_ev)
    if (e) (void)hipEventDestroy(e);
}

namespace {

constexpr int kBS = 256;
constexpr int kNW = kBS / kWave;

// Search state of degree-separated DOBFS on the device. One small kernel per
// level (k_decide) makes the direction decision and writes the level's plan
// here; every other kernel of the level reads its flag and returns at once
// when it has no work, so the levels run back to back without a host round
// trip (the host only learns, a level or two later, that the search ended).
struct DevCtl {
  double f0[4], f1[4];     // direction-switch factors (dd, dn, nd, nn)
  uint64_t forced_seed;
  int32_t forced;
  int32_t done;            // the frontier is empty: every later kernel returns
  int32_t level;           // level in progress
  int32_t level1;          // depth this level writes (level + 1)
  int32_t dir[4];          // current direction per kernel (0 forward, 1 backward)
  int32_t nn_do;           // nn under the direction decision (else always forward)
  int32_t nn_td, nn_bu;    // plan of this level for nn (nn_do only)
  int32_t cand_state;      // -1: the next bottom-up normal pass scans the whole nd source list
  int32_t nc_pending;      // the previous pass compacted a candidate list of unknown length
  int32_t mark_fn;         // this level marks the normal frontier bitmap
  int32_t nd_td, dd_td, dn_td, dn_bu, dd_bu, nd_bu;  // plan of this level
  int32_t bulk_fn, clear_fn, cin_sel, cout_sel;
  int64_t nwords;
  int64_t rem[4];          // unvisited: delegates with a dd edge, with a dn edge, nd-list
                           // normals, normals with an nn edge
  int64_t nc;              // candidates of the next bottom-up normal pass
  int64_t qn, fdn;         // frontier sizes of this level
  unsigned long long deg_sum;                         // sum of frontier degrees so far
  unsigned long long units[DSBFS_NUM_KERNELS][6];     // work units per kernel so far
};

// What the host learns of each level, written by k_decide into pinned host
// memory (a ring of 4 slots, slot = level & 3).
struct LevelStatus {
  int32_t done, level;
  int32_t plan[10];  // nd_td, dd_td, dn_td, dn_bu (runs), dd_bu, nd_bu, bulk_fn, mark_fn,
                     // nn_td (separate pass), nn_bu
  dsbfs_level_stats rec;
};
constexpr int kStatusSlots = 4;

// Whether this level marks the normal frontier bitmap Fn. Fn is read only by
// a bottom-up nd visit (which needs an unvisited delegate with a dn edge left
// after this level's frontier: rem[1] - q_dn > 0) and, with nn_do, by a
// bottom-up nn visit. The delegate previsit runs first, so q_dn is known to
// the normal previsit and to the decision alike.
__device__ __forceinline__ int level_marks_fn(const DevCtl *c, int64_t q_dn) {
  return c->mark_fn && (c->rem[1] - q_dn > 0 || (c->nn_do && c->rem[3] > 0));
}

// Bytes of one of the two tile arrays of the delegate-frontier prefix sum.
inline size_t dtiles_half(int64_t d) {
  const size_t nb = size_t((d + kBS * 8 - 1) / (kBS * 8)) + 1;
  return (nb * 8 + 255) / 256 * 256;
}

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Backward workload estimate |U|(q+s)/q (Section IV-B), 0 when q or |U| is 0.
__host__ __device__ inline double bv_estimate(int64_t U, int64_t q, int64_t s) {
  if (q <= 0 || U <= 0) return 0.0;
  return double(U) * (double(q) + double(s)) / double(q);
}

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
__global__ void k_init(int32_t *depth, int32_t *parent, int32_t n, uint32_t *Vn, uint32_t *Fn,
                       int32_t nwords, uint32_t *Vd, uint32_t *Fd, uint32_t *Cd, int32_t dwords) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t v = t0; v < n; v += stride) {
    depth[v] = -1;
    if (parent) parent[v] = -1;
  }
  for (int64_t w = t0; w < nwords; w += stride) {
    Vn[w] = 0;
    Fn[w] = 0;
  }
  for (int64_t w = t0; w < dwords; w += stride) {
    Vd[w] = 0;
    Fd[w] = 0;
    Cd[w] = 0;
  }
}

// Seeds the source: a delegate enters the delegate frontier mask, a normal
// vertex the normal queue. prev's queue tail becomes the level-0 queue
// length (no bottom-up candidates yet).
__global__ void k_seed(int32_t s, const int32_t *did, int32_t *depth, int32_t *parent,
                       uint32_t *Vn, uint32_t *Vd, uint32_t *Fd, uint32_t *Cd, int32_t *Q,
                       LevelCtr *prev, int mode) {
  depth[s] = 0;
  if (parent) parent[s] = s;
  const int32_t k = mode == 1 ? did[s] : -1;
  if (k >= 0) {
    Vd[k >> 5] |= 1u << (k & 31);
    Fd[k >> 5] |= 1u << (k & 31);
    Cd[k >> 5] |= 1u << (k & 31);
    prev->qn_nc = 0;
  } else {
    Vn[s >> 5] |= 1u << (s & 31);
    Q[0] = s;
    prev->qn_nc = 1;
  }
}

// ---------------------------------------------------------------------------
// previsit
// ---------------------------------------------------------------------------
// All per-level kernels are grid-stride loops over a bounded grid (a few
// workgroups per CU) and publish counters and queue entries once per block:
// device-scope atomics on one address serialize chip-wide, so one per wave
// over a multi-million-entry frontier would dominate the level.
constexpr int kQCap = 1536;  // LDS append buffer entries per queue per block

// Exclusive scan over the block of one int per thread; *total = block sum.
__device__ __forceinline__ int block_excl_scan_i32(int v, int *sh, int *total) {
  const int w = threadIdx.x / kWave, l = lane_id();
  const int incl = wave_incl_scan(v);
  if (l == kWave - 1) sh[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int i = 0; i < kNW; ++i) {
    const int t = sh[i];
    before += i < w ? t : 0;
    all += t;
  }
  *total = all;
  __syncthreads();
  return before + incl - v;
}

// One thread per mask word: frontier delegates -> dlist, with their dd/dn
// workloads. Positions come from a block scan plus one global atomic per block.
__global__ void __launch_bounds__(kBS) k_prev_deleg(const uint32_t *Fd, int32_t dwords,
                                                    const uint64_t *doff, int32_t *dlist,
                                                    LevelCtr *cur, const DevCtl *c) {
  if (c->done) return;
  // The frontier list feeds only the forward dd/dn visit. Under the
  // heuristic schedule, once dd and dn both go backward with no switch back
  // (factor1 = 0) none can follow: the list is not written.
  const bool want_list = !(c->forced == 0 && c->dir[0] == 1 && c->dir[1] == 1 &&
                           c->f1[0] == 0.0 && c->f1[1] == 0.0);
  __shared__ int shf[kNW];
  __shared__ unsigned long long base;
  __shared__ unsigned long long sh[4 * kNW];
  unsigned long long fv_dd = 0, q_dd = 0, fv_dn = 0, q_dn = 0;
  for (int64_t w0 = int64_t(blockIdx.x) * blockDim.x; w0 < dwords;
       w0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t w = w0 + threadIdx.x;
    uint32_t f = w < dwords ? Fd[w] : 0u;
    int tf;
    const int ef = block_excl_scan_i32(__popc(f), shf, &tf);
    if (threadIdx.x == 0) base = tf ? atomicAdd(&cur->nd_list, (unsigned long long)tf) : 0ull;
    __syncthreads();
    unsigned long long pf = base + ef;
    while (f) {
      const int b = __ffs(f) - 1;
      f &= f - 1;
      const int32_t k = int32_t(w * 32 + b);
      if (want_list) dlist[pf] = k;
      ++pf;
      const uint64_t x0 = doff[k], x1 = doff[k + 1];
      const int64_t dd = row_first(x0), dn = row_start(x1) - row_start(x0) - dd;
      fv_dd += dd;
      q_dd += dd > 0;
      fv_dn += dn;
      q_dn += dn > 0;
    }
    __syncthreads();
  }
  block_add4(&cur->fv_dd, fv_dd, q_dd, fv_dn, q_dn, sh);
}

// Unclaimed delegates (not visited and not claimed earlier in this level)
// with an edge in a subgraph scanned bottom-up this level (dd part if dd_bu,
// dn part if nd_bu) -> dcand, ascending.
__global__ void __launch_bounds__(kBS) k_dcand(const uint32_t *Cd, const uint32_t *ddm,
                                               const uint32_t *dnm, int32_t dwords,
                                               const DevCtl *ctl, int32_t *dcand, LevelCtr *cur) {
  if (ctl->done || !(ctl->dd_bu || ctl->nd_bu)) return;
  const int dd_bu = ctl->dd_bu, nd_bu = ctl->nd_bu;
  __shared__ int shc[kNW];
  __shared__ unsigned long long base;
  for (int64_t w0 = int64_t(blockIdx.x) * blockDim.x; w0 < dwords;
       w0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t w = w0 + threadIdx.x;
    uint32_t c = 0;
    if (w < dwords) c = ~Cd[w] & ((dd_bu ? ddm[w] : 0u) | (nd_bu ? dnm[w] : 0u));
    int tc;
    const int ec = block_excl_scan_i32(__popc(c), shc, &tc);
    if (threadIdx.x == 0) base = tc ? atomicAdd(&cur->nd_cand, (unsigned long long)tc) : 0ull;
    __syncthreads();
    unsigned long long pc = base + ec;
    while (c) {
      const int b = __ffs(c) - 1;
      c &= c - 1;
      dcand[pc++] = int32_t(w * 32 + b);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// visits
// ---------------------------------------------------------------------------
struct Out {
  int32_t *depth;
  int32_t *parent;
  int32_t level1;  // depth written by this level (L + 1)
  __device__ __forceinline__ void put(int32_t v, int32_t p) const {
    depth[v] = level1;
    if (parent) parent[v] = p;
  }
};

// Largest index lo in [0, 64) with ex[lo] <= e (ex non-decreasing, ex[0] = 0).
__device__ __forceinline__ int owner64(const int32_t *ex, int32_t e) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    const int c = lo + step;
    if (ex[c] <= e) lo = c;
  }
  return lo;
}

// Wave-balanced top-down expansion of one part of the rows of the normal
// queue: each wave owns 64 queue entries per step; their part lengths are
// prefix-summed across the wave and the wave walks the concatenated edge
// range 64 edges at a time, so lanes stay busy whatever the mix of degrees
// (all are <= TH). `part` 0 = nn (claims normals, enqueues them), 1 = nd
// (claims delegates in Cd).
template <int part>
__device__ __forceinline__ void expand_normal_rows(int32_t u, int32_t len, int64_t beg,
                                                   int32_t (&s_excl)[kWave],
                                                   int32_t (&s_u)[kWave],
                                                   int64_t (&s_beg)[kWave], const int32_t *ncol,
                                                   const int32_t *vid_of, const Out &out,
                                                   uint32_t *Vn, uint32_t *Cd, BlockAppend &qa,
                                                   unsigned long long &edges,
                                                   unsigned long long &claimed) {
  const int l = lane_id();
  const int32_t incl = wave_incl_scan(len);
  const int32_t T = lane_read(incl, kWave - 1);
  wave_sync();
  s_excl[l] = incl - len;
  s_u[l] = u;
  s_beg[l] = beg;
  wave_sync();
  if (l == 0) edges += T;
  for (int32_t e0 = 0; e0 < T; e0 += kWave) {
    const int32_t e = e0 + l;
    bool won = false;
    int32_t v = 0;
    if (e < T) {
      const int lo = owner64(s_excl, e);
      v = ncol[s_beg[lo] + (e - s_excl[lo])];
      if (part == 0) {
        won = bit_claim(Vn, uint32_t(v));
        if (won) {
          out.put(v, s_u[lo]);
          ++claimed;
        }
      } else if (bit_claim(Cd, uint32_t(v))) {
        out.put(vid_of[v], s_u[lo]);
        ++claimed;
      }
    }
    if (part == 0) qa.push(won, v);
  }
}

// One pass over the normal queue: previsit (nn/nd workloads and counts of
// the frontier, normal frontier bitmap Fn) fused with the nn top-down visit.
// Fn is only read by a bottom-up nd visit; mark_fn = 0 when none can happen
// (no unvisited delegate has a dn edge).
__global__ void __launch_bounds__(kBS) k_normal_level(const int32_t *Q, const LevelCtr *prev,
                                                      const uint64_t *noff, const uint16_t *nlen,
                                                      const int32_t *ncol, const uint32_t *nnoff,
                                                      const int32_t *nncol,
                                                      Out out, uint32_t *Vn, uint32_t *Fn,
                                                      const DevCtl *c, int32_t *Qnext,
                                                      LevelCtr *cur) {
  if (c->done) return;
  const int64_t qn = lc_qn(prev);
  // blocks past the queue have nothing to add (a short queue leaves most of
  // the grid idle: skip its LDS set-up and block reductions)
  if (int64_t(blockIdx.x) * blockDim.x >= qn) return;
  const int mark_fn = level_marks_fn(c, int64_t(cur->q_dn));
  // with nn under the direction decision this pass only counts (and marks
  // Fn); nn is expanded after the decision, forward or backward
  const int expand = !c->nn_do;
  out.level1 = c->level1;
  __shared__ int32_t s_excl[kNW][kWave];
  __shared__ int32_t s_u[kNW][kWave];
  __shared__ int64_t s_beg[kNW][kWave];
  __shared__ int32_t qbuf[kQCap];
  __shared__ int qcount;
  __shared__ unsigned long long qbase;
  __shared__ unsigned long long sh[4 * kNW];
  BlockAppend qa{qbuf, &qcount, &qbase, kQCap, &cur->qn_nc, Qnext};
  qa.init();
  const int w = threadIdx.x / kWave;
  unsigned long long fv_nn = 0, q_nn = 0, fv_nd = 0, q_nd = 0, edges = 0, claimed = 0;
  for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < qn;
       b0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    int32_t u = 0, nn = 0;
    int64_t beg = 0;
    if (i < qn) {
      u = Q[i];
      // part lengths from 2 bytes per vertex; where the nn part starts only
      // for rows with nn edges (most normal rows have none), from the compact
      // nn copy when there is one
      const uint32_t lw = nlen[u];
      int64_t nd;
      if (lw == kLenWide) {
        const uint64_t w0 = noff[u], w1 = noff[u + 1];
        nn = int32_t(row_first(w0));
        nd = row_start(w1) - row_start(w0) - nn;
        beg = nnoff ? int64_t(nnoff[u]) : row_start(w0);
      } else {
        nn = int32_t(lw & 0xFFu);
        nd = int64_t(lw >> 8);
        if (nn > 0 && expand) beg = nnoff ? int64_t(nnoff[u]) : row_start(noff[u]);
      }
      fv_nn += nn;
      q_nn += nn > 0;
      fv_nd += nd;
      q_nd += nd > 0;
    }
    // queues filled by the bottom-up pass are in ascending order: mark word by word
    if (mark_fn) wave_bit_set(Fn, uint32_t(u), i < qn, true);
    expand_normal_rows<0>(u, expand ? nn : 0, beg, s_excl[w], s_u[w], s_beg[w],
                          nnoff ? nncol : ncol, nullptr, out, Vn, nullptr, qa, edges, claimed);
    qa.maybe_flush(kBS * 2);
  }
  qa.flush();
  block_add4(&cur->fv_nn, fv_nn, q_nn, fv_nd, q_nd, sh);
  // units: queue entries (counted on the host), nn edges, normals claimed
  block_add4(cur->units[DSBFS_K_PREV_NORMAL], 0, edges, claimed, 0, sh);
}

// Top-down nn from the normal queue, after the direction decision (nn_do,
// levels where nn goes forward): the expansion k_normal_level fuses into the
// previsit otherwise.
__global__ void __launch_bounds__(kBS) k_td_nn(const int32_t *Q, const DevCtl *c,
                                               const uint64_t *noff, const uint16_t *nlen,
                                               const int32_t *ncol, const uint32_t *nnoff,
                                               const int32_t *nncol, Out out, uint32_t *Vn,
                                               int32_t *Qnext, LevelCtr *cur) {
  if (c->done || !c->nn_td) return;
  const int64_t qn = c->qn;
  if (int64_t(blockIdx.x) * blockDim.x >= qn) return;
  out.level1 = c->level1;
  __shared__ int32_t s_excl[kNW][kWave];
  __shared__ int32_t s_u[kNW][kWave];
  __shared__ int64_t s_beg[kNW][kWave];
  __shared__ int32_t qbuf[kQCap];
  __shared__ int qcount;
  __shared__ unsigned long long qbase;
  __shared__ unsigned long long sh[4 * kNW];
  BlockAppend qa{qbuf, &qcount, &qbase, kQCap, &cur->qn_nc, Qnext};
  qa.init();
  const int w = threadIdx.x / kWave;
  unsigned long long edges = 0, claimed = 0;
  for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < qn;
       b0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    int32_t u = 0, nn = 0;
    int64_t beg = 0;
    if (i < qn) {
      u = Q[i];
      const uint32_t lw = nlen[u];
      if (lw == kLenWide) {
        const uint64_t w0 = noff[u];
        nn = int32_t(row_first(w0));
        beg = nnoff ? int64_t(nnoff[u]) : row_start(w0);
      } else {
        nn = int32_t(lw & 0xFFu);
        if (nn > 0) beg = nnoff ? int64_t(nnoff[u]) : row_start(noff[u]);
      }
    }
    expand_normal_rows<0>(u, nn, beg, s_excl[w], s_u[w], s_beg[w], nnoff ? nncol : ncol, nullptr,
                          out, Vn, nullptr, qa, edges, claimed);
    qa.maybe_flush(kBS * 2);
  }
  qa.flush();
  // units: queue entries (counted by the decision), nn edges, normals claimed
  block_add4(cur->units[DSBFS_K_TD_NN], 0, edges, claimed, 0, sh);
}

// Bottom-up nn (nn_do, levels where nn goes backward): every normal vertex
// with an nn edge that is still unvisited scans its nn part (ascending IDs)
// for a vertex of the level's normal frontier (bitmap Fn, marked by the
// previsit), stopping at the first; the rows of a wave's 64 candidates are
// walked together, 64 entries per step, as in k_bu_normal. A candidate is
// one lane's and no other kernel claims normals while this one runs, so
// claims set bits without reading them back.
__global__ void __launch_bounds__(kBS) k_bu_nn(const DevCtl *c, const int32_t *nnsrc,
                                               int64_t nsrc, const uint64_t *noff,
                                               const uint16_t *nlen, const int32_t *ncol,
                                               const uint32_t *Fn, Out out, uint32_t *Vn,
                                               int32_t *Qnext, LevelCtr *cur) {
  if (c->done || !c->nn_bu) return;
  out.level1 = c->level1;
  __shared__ int32_t s_excl[kNW][kWave];
  __shared__ int32_t s_found[kNW][kWave];
  __shared__ int64_t s_beg[kNW][kWave];
  __shared__ int32_t qbuf[kQCap];
  __shared__ int qcount;
  __shared__ unsigned long long qbase;
  __shared__ unsigned long long sh[4 * kNW];
  BlockAppend qa{qbuf, &qcount, &qbase, kQCap, &cur->qn_nc, Qnext};
  qa.init();
  const int w = threadIdx.x / kWave, l = lane_id();
  constexpr int32_t kNone = 0x7fffffff;
  unsigned long long reads = 0, scanned = 0, edges = 0, claimed = 0;
  for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < nsrc;
       b0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    const bool ok = i < nsrc;
    int32_t v = 0, len = 0;
    int64_t beg = 0;
    if (ok) {
      v = nnsrc[i];
      ++reads;
      if (!bit_test(Vn, uint32_t(v))) {
        ++scanned;
        const uint32_t lw = nlen[v];
        const uint64_t w0 = noff[v];
        beg = row_start(w0);
        len = lw == kLenWide ? int32_t(row_first(w0)) : int32_t(lw & 0xFFu);
      }
    }
    const int32_t incl = wave_incl_scan(len);
    const int32_t T = lane_read(incl, kWave - 1);
    wave_sync();
    s_excl[w][l] = incl - len;
    s_beg[w][l] = beg;
    s_found[w][l] = kNone;
    wave_sync();
    uint64_t remaining = __ballot(len > 0);
    for (int32_t e0 = 0; e0 < T && remaining; e0 += kWave) {
      const int32_t e = e0 + l;
      if (e < T) {
        const int lo = owner64(s_excl[w], e);
        if (s_found[w][lo] == kNone) {
          const int32_t x = ncol[s_beg[w][lo] + (e - s_excl[w][lo])];
          ++edges;
          if (bit_test(Fn, uint32_t(x))) atomicMin(&s_found[w][lo], e);
        }
      }
      wave_sync();
      remaining = __ballot(len > 0 && s_found[w][l] == kNone);
    }
    const int32_t fe = s_found[w][l];
    const bool won = ok && len > 0 && fe != kNone;
    wave_bit_set(Vn, uint32_t(v), ok, won);
    if (won) {
      out.put(v, ncol[beg + (fe - (incl - len))]);
      ++claimed;
    }
    qa.push(won, v);
    qa.maybe_flush(kBS);
  }
  qa.flush();
  // units: list entries read, unvisited scanned, edges inspected, claimed
  block_add4(cur->units[DSBFS_K_BU_NN], reads, scanned, edges, claimed, sh);
}

// Top-down nd from the normal queue (only on levels where nd goes forward).
__global__ void __launch_bounds__(kBS) k_td_nd(const int32_t *Q, const DevCtl *c,
                                               const uint64_t *noff, const int32_t *ncol,
                                               const int32_t *vid_of, Out out, uint32_t *Cd,
                                               LevelCtr *cur) {
  if (c->done || !c->nd_td) return;
  const int64_t qn = c->qn;
  out.level1 = c->level1;
  __shared__ int32_t s_excl[kNW][kWave];
  __shared__ int32_t s_u[kNW][kWave];
  __shared__ int64_t s_beg[kNW][kWave];
  __shared__ unsigned long long sh[4 * kNW];
  const int w = threadIdx.x / kWave;
  BlockAppend none{nullptr, nullptr, nullptr, 0, nullptr, nullptr};
  unsigned long long edges = 0, claimed = 0;
  for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < qn;
       b0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    int32_t u = 0, len = 0;
    int64_t beg = 0;
    if (i < qn) {
      u = Q[i];
      const uint64_t w0 = noff[u], w1 = noff[u + 1];
      beg = row_start(w0) + row_first(w0);
      len = int32_t(row_start(w1) - beg);
    }
    expand_normal_rows<1>(u, len, beg, s_excl[w], s_u[w], s_beg[w], ncol, vid_of, out, nullptr,
                          Cd, none, edges, claimed);
  }
  // units: -, edges, -, delegates claimed
  block_add4(cur->units[DSBFS_K_TD_NORMAL], 0, edges, 0, claimed, sh);
}

// Largest idx in [0, cnt) with pre[idx] <= e (pre non-decreasing, pre[0] = 0).
__device__ __forceinline__ int64_t seg_search(const int64_t *pre, int64_t cnt, int64_t e) {
  int64_t lo = 0, hi = cnt - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Top-down from the delegate frontier over dd and/or dn. Delegate degrees span
// a wide range, so the work is balanced over edges: the frontier's selected
// row parts, concatenated, are cut into one contiguous range per block, and a
// block takes 256 consecutive edges per step, one per lane. Lanes of a wave
// mostly share a row, so the row lookups broadcast and the column reads
// coalesce. Each wave finds the row of its first edge once by binary search
// in the prefix sum of the part lengths and walks forward from there.
__global__ void __launch_bounds__(kBS) k_td_deleg(const int32_t *dlist, const int64_t *dscan,
                                                  const LevelCtr *curc, const uint64_t *doff,
                                                  const int32_t *dcol, const int32_t *vid_of,
                                                  const DevCtl *c, Out out, uint32_t *Vn,
                                                  uint32_t *Cd, int32_t *Qnext, LevelCtr *cur) {
  if (c->done || !(c->dd_td || c->dn_td)) return;
  const int dd_td = c->dd_td;
  out.level1 = c->level1;
  __shared__ int32_t qbuf[kQCap];
  __shared__ int qcount;
  __shared__ unsigned long long qbase;
  __shared__ unsigned long long sh[4 * kNW];
  BlockAppend qa{qbuf, &qcount, &qbase, kQCap, &cur->qn_nc, Qnext};
  qa.init();
  const int64_t nd = int64_t(curc->nd_list);
  const int64_t E = dscan[nd];
  const int w = threadIdx.x / kWave;
  unsigned long long cl_n = 0, cl_d = 0, edges = 0;
  // block range [bs, be), a multiple of the block width long
  const int64_t per = (E + gridDim.x - 1) / gridDim.x;
  const int64_t bchunk = (per + kBS - 1) / kBS * kBS;
  const int64_t bs = int64_t(blockIdx.x) * bchunk, be = min(bs + bchunk, E);
  int64_t idx = 0;  // row of the wave's first edge in the current step
  if (bs + w * kWave < be) idx = seg_search(dscan, nd, bs + w * kWave);
  for (int64_t b0 = bs; b0 < be; b0 += kBS) {
    const int64_t e = b0 + threadIdx.x;
    const bool valid = e < be;
    int64_t my = idx;
    int32_t x = 0, pk = 0;
    bool is_dd = false;
    if (valid) {
      while (dscan[my + 1] <= e) ++my;
      const int32_t k = dlist[my];
      const int64_t j = e - dscan[my];
      const uint64_t w0 = doff[k];
      const int64_t beg = row_start(w0), dd = row_first(w0);
      is_dd = dd_td && j < dd;
      x = dcol[dd_td ? beg + j : beg + dd + j];
      pk = vid_of[k];
      ++edges;
    }
    // the next step's first edge lies at or after this step's last one
    idx = lane_read(my, kWave - 1);
    // claims: a cheap visited test first (most edges lead to vertices already
    // claimed), then one atomic per run of lanes sharing a bitmap word
    const bool want_d = valid && is_dd && !bit_test(Cd, uint32_t(x));
    const bool want_n = valid && !is_dd && !bit_test(Vn, uint32_t(x));
    const bool won_d = wave_bit_claim(Cd, uint32_t(x), valid && is_dd, want_d);
    const bool won_n = wave_bit_claim(Vn, uint32_t(x), valid && !is_dd, want_n);
    if (won_d) {
      out.put(vid_of[x], pk);
      ++cl_d;
    }
    if (won_n) {
      out.put(x, pk);
      ++cl_n;
    }
    qa.push(won_n, x);
    qa.maybe_flush(kBS);
  }
  qa.flush();
  // units: -, edges, normals claimed, delegates claimed
  block_add4(cur->units[DSBFS_K_TD_DELEG], 0, edges, cl_n, cl_d, sh);
}

// Bottom-up dn (destination: normal vertices). Candidates are positions in
// the nd source list; row p of the source-list-ordered nd copy holds the
// delegate neighbours of ndsrc[p]. Each wave takes 64 candidates, drops the
// visited ones, and walks the concatenation of the remaining rows 64 entries
// at a time (consecutive candidates have consecutive rows, so the first pass
// over the whole list streams them); the first entry of a row found in the
// frontier mask Fd is kept with an LDS atomicMin, and the wave stops as soon
// as every remaining candidate has one. Candidates still unvisited are
// compacted (as positions) for the next bottom-up level.
__global__ void __launch_bounds__(kBS) k_bu_normal(const DevCtl *c, int32_t *c0, int32_t *c1,
                                                   const int32_t *ndsrc, const int64_t *nds_off,
                                                   const int32_t *nds_col, const int2 *nds_first,
                                                   const int32_t *vid_of, const uint32_t *Fd,
                                                   Out out, uint32_t *Vn, int32_t *Qnext,
                                                   LevelCtr *cur) {
  if (c->done || !c->dn_bu) return;
  // first pass: every position of the nd source list (dense); later passes:
  // the positions the previous pass left unvisited
  const int dense = c->cin_sel < 0;
  const int32_t *cin = c->cin_sel == 0 ? c0 : c1;
  int32_t *cout = c->cout_sel == 0 ? c0 : c1;
  const int64_t nc = c->nc;
  out.level1 = c->level1;
  __shared__ int32_t s_excl[kNW][kWave];
  __shared__ int32_t s_found[kNW][kWave];
  __shared__ int64_t s_beg[kNW][kWave];
  __shared__ int32_t qbuf[kQCap], cbuf[kQCap];
  __shared__ int qcount, ccount;
  __shared__ unsigned long long qbase, cbase;
  __shared__ unsigned long long sh[4 * kNW];
  BlockAppend qa{qbuf, &qcount, &qbase, kQCap, &cur->qn_nc, Qnext};
  BlockAppend ca{cbuf, &ccount, &cbase, kQCap, &cur->qn_nc, cout, 32};
  qa.init();
  ca.init();
  const int w = threadIdx.x / kWave, l = lane_id();
  constexpr int32_t kNone = 0x7fffffff;
  unsigned long long reads = 0, scanned = 0, edges = 0, claimed = 0;
  for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < nc;
       b0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    const bool ok = i < nc;
    int32_t pos = 0, v = 0, len = 0;
    int64_t beg = 0;
    bool visited = true;
    int32_t hit0 = -1;  // delegate found at the first entry of the row
    int32_t pk0 = 0;  // vertex of the row's first delegate (its parent if it is a hit)
    if (ok) {
      pos = dense ? int32_t(i) : cin[i];
      // The loads are ordered to keep the chain of dependent accesses short:
      // the vertex and its row bounds both depend on pos only; the row's
      // first entry (rows in the list are never empty) does not wait for the
      // visited test, and the parent candidate is fetched beside the
      // frontier test.
      v = ndsrc[pos];
      // Rows start with their highest-degree delegate, the likeliest to be in
      // the frontier: a hit there skips the wave's walk for this row. The
      // first entry and its vertex come from a dense array (8 bytes per
      // candidate, read in list order); its frontier bit is tested whether
      // or not the candidate turns out to be visited, so that the loads
      // overlap the visited test instead of following it.
      const int2 f = nds_first[pos];
      const int32_t k0 = f.x;
      pk0 = f.y;
      const bool f0 = bit_test(Fd, uint32_t(k0));
      ++reads;
      visited = bit_test(Vn, uint32_t(v));
      hit0 = (!visited && f0) ? k0 : -1;
      scanned += !visited;
      edges += !visited;
      if (!visited && !f0) {
        // a miss: the rest of the row is walked below
        beg = nds_off[pos] + 1;
        len = int32_t(nds_off[pos + 1] - beg);
      }
    }
    const int32_t incl = wave_incl_scan(len);
    const int32_t T = lane_read(incl, kWave - 1);
    wave_sync();
    s_excl[w][l] = incl - len;
    s_beg[w][l] = beg;
    s_found[w][l] = kNone;
    wave_sync();
    uint64_t remaining = __ballot(len > 0);
    for (int32_t e0 = 0; e0 < T && remaining; e0 += kWave) {
      const int32_t e = e0 + l;
      if (e < T) {
        const int lo = owner64(s_excl[w], e);
        // a row whose parent an earlier step found is not read further: a
        // scan stops at its first frontier neighbour (Section IV-B)
        if (s_found[w][lo] == kNone) {
          const int32_t x = nds_col[s_beg[w][lo] + (e - s_excl[w][lo])];
          ++edges;
          if (bit_test(Fd, uint32_t(x))) atomicMin(&s_found[w][lo], e);
        }
      }
      wave_sync();
      remaining = __ballot(len > 0 && s_found[w][l] == kNone);
    }
    const int32_t fe = s_found[w][l];
    const bool found = hit0 >= 0 || (len > 0 && fe != kNone);
    // A vertex is the candidate of one lane only, and no other kernel claims
    // normal vertices while this one runs (the level's nn visit is complete),
    // so a found candidate is this lane's: its bit is set without waiting for
    // the atomic's old value. Candidates are ascending: set word by word.
    const bool won = ok && found;
    wave_bit_set(Vn, uint32_t(v), ok, won);
    if (won) {
      out.put(v, hit0 >= 0 ? pk0 : vid_of[nds_col[beg + (fe - (incl - len))]]);
      ++claimed;
    }
    qa.push(won, v);
    ca.push(ok && !visited && !found, pos);
    __syncthreads();
    if (qcount > kQCap - kBS || ccount > kQCap - kBS) flush_pair(qa, ca);
  }
  flush_pair(qa, ca);
  // units: list entries read, unvisited scanned, edges inspected, claimed
  block_add4(cur->units[DSBFS_K_BU_NORMAL], reads, scanned, edges, claimed, sh);
}

// Bottom-up dd and/or nd (destination: delegates). One unvisited delegate
// per lane: it first tests the first entry of its scanned range (dd parts
// start with their highest-degree neighbour, the likeliest to be in the
// frontier); the rows that miss are then walked together, 64 entries per step
// over their concatenation (prefix sums across the wave), until each has a
// hit or ends. dd entries are tested against Fd, dn entries against the
// normal frontier bitmap Fn. Candidates are ascending, so claims go word by
// word.
__global__ void __launch_bounds__(kBS) k_bu_deleg(const int32_t *dcand, const LevelCtr *curc,
                                                  const uint64_t *doff, const int32_t *dcol,
                                                  const int2 *dd_first, const uint32_t *Fd,
                                                  const uint32_t *Fn,
                                                  const int32_t *vid_of, const DevCtl *c,
                                                  Out out, uint32_t *Cd, LevelCtr *cur) {
  if (c->done || !(c->dd_bu || c->nd_bu)) return;
  const int dd_bu = c->dd_bu, nd_bu = c->nd_bu;
  out.level1 = c->level1;
  __shared__ int32_t s_excl[kNW][kWave];
  __shared__ int32_t s_found[kNW][kWave];
  __shared__ int64_t s_beg[kNW][kWave];
  __shared__ int64_t s_mid[kNW][kWave];
  __shared__ unsigned long long sh[4 * kNW];
  const int64_t nc = int64_t(curc->nd_cand);
  const int w = threadIdx.x / kWave, l = lane_id();
  constexpr int32_t kNone = 0x7fffffff;
  unsigned long long cands = 0, edges = 0, claimed = 0;
  for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < nc;
       b0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    const bool ok = i < nc;
    int32_t k = 0, len = 0, vk = 0, px = 0;
    int64_t p = 0, mid = 0, hit = -1;
    if (ok) {
      k = dcand[i];
      const uint64_t w0 = doff[k], w1 = doff[k + 1];
      vk = vid_of[k];                    // fetched beside the row bounds,
      const int2 f = dd_first[k];        // as is the dense first dd entry
      const int64_t beg = row_start(w0);
      mid = beg + row_first(w0);
      p = dd_bu ? beg : mid;
      const int64_t hi = nd_bu ? row_start(w1) : mid;
      if (p < hi) {
        ++cands;
        const bool in_dd = p < mid;
        const int32_t x = in_dd ? f.x : dcol[p];
        ++edges;
        px = in_dd ? f.y : x;  // the parent if this entry is a hit
        if (in_dd ? bit_test(Fd, uint32_t(x)) : bit_test(Fn, uint32_t(x))) hit = p;
        else ++p;
        // delegate degrees are below 2^24, so 64 rows sum below 2^31
        if (hit < 0) len = int32_t(hi - p);
      }
    }
    const bool probe_hit = hit >= 0;
    const int32_t incl = wave_incl_scan(len);
    const int32_t T = lane_read(incl, kWave - 1);
    if (T > 0) {
      wave_sync();
      s_excl[w][l] = incl - len;
      s_beg[w][l] = p;
      s_mid[w][l] = mid;
      s_found[w][l] = kNone;
      wave_sync();
      uint64_t remaining = __ballot(len > 0);
      for (int32_t e0 = 0; e0 < T && remaining; e0 += kWave) {
        const int32_t e = e0 + l;
        if (e < T) {
          const int lo = owner64(s_excl[w], e);
          if (s_found[w][lo] == kNone) {
            const int64_t q = s_beg[w][lo] + (e - s_excl[w][lo]);
            const int32_t x = dcol[q];
            ++edges;
            if (q < s_mid[w][lo] ? bit_test(Fd, uint32_t(x)) : bit_test(Fn, uint32_t(x)))
              atomicMin(&s_found[w][lo], e);
          }
        }
        wave_sync();
        remaining = __ballot(len > 0 && s_found[w][l] == kNone);
      }
      const int32_t fe = s_found[w][l];
      if (len > 0 && fe != kNone) hit = p + (fe - (incl - len));
      wave_sync();
    }
    // each candidate delegate is one lane's, and no other kernel claims
    // delegates while this one runs: set the bit without reading it back
    const bool won = ok && hit >= 0;
    wave_bit_set(Cd, uint32_t(k), ok, won);
    if (won) {
      int32_t par = px;
      if (!probe_hit) {
        const int32_t x = dcol[hit];
        par = hit < mid ? vid_of[x] : x;
      }
      out.put(vk, par);
      ++claimed;
    }
  }
  // units: candidates scanned, edges inspected, claimed
  block_add4(cur->units[DSBFS_K_BU_DELEG], cands, edges, claimed, 0, sh);
}

// Level close: the next delegate frontier is what was claimed this level
// (Fd = Cd & ~Vd, Vd = Cd); the normal frontier bitmap is cleared either
// word by word under this level's queue (small levels) or, when the host has
// cleared it in bulk, not at all (clear_fn = 0).
__global__ void k_close(uint32_t *Vd, uint32_t *Fd, const uint32_t *Cd, int32_t dwords,
                        uint32_t *Fn, int64_t nwords, const int32_t *Q, DevCtl *c,
                        LevelCtr *next) {
  if (c->done) return;
  const int clear_fn = c->clear_fn, bulk_fn = c->bulk_fn;
  const int64_t qn = c->qn;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t w = t0; w < dwords; w += stride) {
    const uint32_t cw = Cd[w];
    Fd[w] = cw & ~Vd[w];
    Vd[w] = cw;
  }
  if (bulk_fn) {
    for (int64_t w = t0; w < nwords; w += stride) Fn[w] = 0;
  } else if (clear_fn) {
    for (int64_t i = t0; i < qn; i += stride) Fn[Q[i] >> 5] = 0;
  }
  // Open the next level: clear its counters (this level's "previous" ones,
  // which nothing reads after the decision) and fix its depth and whether it
  // marks the normal frontier bitmap (only read by a bottom-up nd visit,
  // impossible once no unvisited delegate has a dn edge).
  if (blockIdx.x == 0) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(next);
    for (int i = threadIdx.x; i < int(sizeof(LevelCtr) / 8); i += blockDim.x) w[i] = 0;
    if (threadIdx.x == 0) {
      c->level += 1;
      c->level1 = c->level + 1;
      c->mark_fn = c->rem[1] > 0 || (c->nn_do && c->rem[3] > 0);
    }
  }
}

// ---------------------------------------------------------------------------
// level control on the device
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(DevCtl *c, DevCtl init) { *c = init; }

// The decision itself (one thread), into the level's status record.
__device__ void decide_level(DevCtl *__restrict__ c, const LevelCtr *__restrict__ cur,
                             const LevelCtr *__restrict__ prev, LevelStatus *st) {
  const int32_t L = c->level;
  const int64_t qn = lc_qn(prev), fdn = int64_t(cur->nd_list);
  c->units[DSBFS_K_PREV_NORMAL][0] += qn;
  c->units[DSBFS_K_PREV_DELEG][0] += fdn;
  c->deg_sum += cur->fv_nn + cur->fv_nd + cur->fv_dd + cur->fv_dn;
  if (c->nc_pending) {
    // length of the candidate list the previous bottom-up normal pass compacted
    c->nc = lc_nc(prev);
    c->units[DSBFS_K_BU_NORMAL][4] += lc_nc(prev);
    c->nc_pending = 0;
  }
  if (qn == 0 && fdn == 0) {
    c->done = 1;
    st->level = L;
    st->done = 1;
    return;
  }
  const int64_t q[3] = {int64_t(cur->q_dd), int64_t(cur->q_dn), int64_t(cur->q_nd)};
  const int64_t FV[3] = {int64_t(cur->fv_dd), int64_t(cur->fv_dn), int64_t(cur->fv_nd)};
  // what the normal previsit of this level did (before the counts move on)
  c->mark_fn = level_marks_fn(c, q[1]);
  c->rem[0] -= q[0];
  c->rem[1] -= q[1];
  c->rem[2] -= q[2];
  const int64_t q_nn = int64_t(cur->q_nn), fv_nn = int64_t(cur->fv_nn);
  c->rem[3] -= q_nn;
  const int64_t U[3] = {c->rem[0], c->rem[2], c->rem[1]};
  const int64_t S[3] = {c->rem[0], c->rem[1], c->rem[2]};
  double BV[3];
  auto choose = [&](int k, int64_t qk, int64_t fvk, double bvk) {
    int d = c->dir[k];
    if (c->forced == 1) d = 0;
    else if (c->forced == 2) d = L >= 1 ? 1 : 0;
    else if (c->forced == 3)
      d = int(mix64(c->forced_seed + uint64_t(L) * 3 + k + (k == 3 ? 0x5bd1e995ull : 0)) & 1);
    else if (qk > 0) {
      if (d == 0 && double(fvk) > c->f0[k] * bvk) d = 1;
      else if (d == 1 && double(fvk) < c->f1[k] * bvk) d = 0;
    }
    c->dir[k] = d;
  };
  for (int k = 0; k < 3; ++k) {
    BV[k] = bv_estimate(U[k], q[k], S[k]);
    choose(k, q[k], FV[k], BV[k]);
    st->rec.q[k] = q[k];
    st->rec.s[k] = S[k];
    st->rec.U[k] = U[k];
    st->rec.FV[k] = FV[k];
    st->rec.BV[k] = BV[k];
    st->rec.dir[k] = c->dir[k];
  }
  // nn (nn_do only): U = s = unvisited normals with an nn edge (symmetric)
  const double BV_nn = c->nn_do ? bv_estimate(c->rem[3], q_nn, c->rem[3]) : 0.0;
  if (c->nn_do) choose(3, q_nn, fv_nn, BV_nn);
  st->rec.U_nn = c->nn_do ? c->rem[3] : 0;
  st->rec.s_nn = st->rec.U_nn;
  st->rec.BV_nn = BV_nn;
  st->rec.dir_nn = c->nn_do ? c->dir[3] : 0;
  st->rec.FV_nn = fv_nn;
  st->rec.q_nn = q_nn;
  st->rec.frontier_normal = qn;
  st->rec.frontier_delegate = fdn;
  const int nn_td = c->nn_do && c->dir[3] == 0 && q_nn > 0;
  const int nn_bu = c->nn_do && c->dir[3] == 1 && q_nn > 0 && c->rem[3] > 0;
  // without nn_do, nn went top-down inside k_normal_level already
  const int dd_td = c->dir[0] == 0 && q[0] > 0, dn_td = c->dir[1] == 0 && q[1] > 0;
  const int nd_td = c->dir[2] == 0 && q[2] > 0;
  const int dd_bu = c->dir[0] == 1 && q[0] > 0 && U[0] > 0;
  const int dn_bu = c->dir[1] == 1 && q[1] > 0 && U[1] > 0 && c->nc > 0;
  const int nd_bu = c->dir[2] == 1 && q[2] > 0 && U[2] > 0;
  // large levels clear the normal frontier bitmap with one streaming fill
  // instead of one scattered store per queue entry
  const int bulk_fn = c->mark_fn && qn * 16 > c->nwords;
  c->nd_td = nd_td;
  c->dd_td = dd_td;
  c->dn_td = dn_td;
  c->dn_bu = dn_bu;
  c->dd_bu = dd_bu;
  c->nd_bu = nd_bu;
  c->nn_td = nn_td;
  c->nn_bu = nn_bu;
  c->bulk_fn = bulk_fn;
  c->clear_fn = c->mark_fn && !bulk_fn;
  c->qn = qn;
  c->fdn = fdn;
  if (dn_bu) {
    c->cin_sel = c->cand_state;
    c->cout_sel = c->cand_state < 0 ? 0 : (c->cand_state ^ 1);
    c->cand_state = c->cout_sel;
    c->nc_pending = 1;
  }
  if (nd_td) c->units[DSBFS_K_TD_NORMAL][0] += qn;
  if (nn_td) c->units[DSBFS_K_TD_NN][0] += qn;
  if (dd_td || dn_td) c->units[DSBFS_K_TD_DELEG][0] += fdn;
  c->units[DSBFS_K_CLOSE][0] += bulk_fn ? c->nwords / 4 : qn;
  const int plan[10] = {nd_td, dd_td, dn_td, dn_bu, dd_bu, nd_bu, bulk_fn, c->mark_fn, nn_td,
                        nn_bu};
  for (int i = 0; i < 10; ++i) st->plan[i] = plan[i];
  st->level = L;
  st->done = 0;
}

// Direction decision of Section IV-B for dd, dn, nd (indices 0, 1, 2) from
// this level's previsit counts, in FP64 with the same expression as the
// oracle's replay, and the plan of the rest of the level. One wave: the work
// units are summed by 36 lanes, the decision is made by lane 0 into an LDS
// record, and the record goes to pinned host memory one word per lane.
__global__ void k_decide(DevCtl *c, const LevelCtr *cur, const LevelCtr *prev,
                         LevelStatus *hs) {
  if (c->done) return;
  __shared__ LevelStatus rec;
  __shared__ int32_t slot;
  const int t = threadIdx.x;
  // the previous level's kernels are complete: their work units
  if (t < DSBFS_NUM_KERNELS * 4) c->units[t / 4][t % 4] += prev->units[t / 4][t % 4];
  __syncthreads();
  if (t == 0) {
    decide_level(c, cur, prev, &rec);
    slot = rec.level & (kStatusSlots - 1);
  }
  __syncthreads();
  const uint32_t *from = reinterpret_cast<const uint32_t *>(&rec);
  uint32_t *to = reinterpret_cast<uint32_t *>(hs + slot);
  for (int i = t; i < int(sizeof(LevelStatus) / 4); i += blockDim.x) to[i] = from[i];
}

// Exclusive prefix sum of the top-down row lengths of the frontier delegates
// (count on the device): tile sums, a scan of the tile sums in one block, and
// the per-tile scans. Grids cover every delegate; tiles past the count return.
constexpr int kScanItems = 8, kScanTile = kBS * kScanItems;

__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t *sh, int64_t *total) {
  const int w = threadIdx.x / kWave, l = lane_id(), nw = blockDim.x / kWave;
  const int64_t incl = wave_incl_scan(v);
  if (l == kWave - 1) sh[w] = incl;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    before += i < w ? sh[i] : 0;
    all += sh[i];
  }
  *total = all;
  __syncthreads();
  return before + incl - v;
}

// First pass: the top-down length of each frontier delegate's row (dd part
// if dd goes forward, dn part if dn does) and the sum of each tile.
__global__ void __launch_bounds__(kBS) k_dscan_reduce(const int32_t *dlist, const uint64_t *doff,
                                                      const LevelCtr *cur, const DevCtl *c,
                                                      int32_t *len, int64_t *bsum) {
  if (c->done || !(c->dd_td || c->dn_td)) return;
  __shared__ int64_t sh[kNW];
  const int dd_td = c->dd_td, dn_td = c->dn_td;
  const int64_t N = int64_t(cur->nd_list);
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  if (base >= N) return;
  int64_t x = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + int64_t(threadIdx.x) * kScanItems + k;
    if (i < N) {
      const int32_t kd = dlist[i];
      const uint64_t w0 = doff[kd], w1 = doff[kd + 1];
      const int64_t dd = row_first(w0), dn = row_start(w1) - row_start(w0) - dd;
      const int32_t l = int32_t((dd_td ? dd : 0) + (dn_td ? dn : 0));
      len[i] = l;
      x += l;
    }
  }
  int64_t tot;
  (void)block_excl_scan_i64(x, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_dscan_top(const int64_t *bsum, int64_t *bscan,
                                                    int64_t *out, const LevelCtr *cur,
                                                    const DevCtl *c) {
  if (c->done || !(c->dd_td || c->dn_td)) return;
  __shared__ int64_t sh[1024 / kWave];
  const int64_t N = int64_t(cur->nd_list);
  const int64_t nb = (N + kScanTile - 1) / kScanTile;
  int64_t carry = 0;
  for (int64_t i0 = 0; i0 < nb; i0 += blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const int64_t x = i < nb ? bsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan_i64(x, sh, &tot);
    if (i < nb) bscan[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) out[N] = carry;
}

__global__ void __launch_bounds__(kBS) k_dscan_down(const int32_t *len, int64_t *out,
                                                    const LevelCtr *cur, const DevCtl *c,
                                                    const int64_t *bscan) {
  if (c->done || !(c->dd_td || c->dn_td)) return;
  __shared__ int64_t sh[kNW];
  const int64_t N = int64_t(cur->nd_list);
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  if (base >= N) return;
  const int64_t t0 = base + int64_t(threadIdx.x) * kScanItems;
  int64_t x = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (t0 + k < N) x += len[t0 + k];
  int64_t tot;
  int64_t run = bscan[blockIdx.x] + block_excl_scan_i64(x, sh, &tot);
  for (int k = 0; k < kScanItems; ++k)
    if (t0 + k < N) {
      out[t0 + k] = run;
      run += len[t0 + k];
    }
}

// ---------------------------------------------------------------------------
// plain top-down (mode 0)
// ---------------------------------------------------------------------------
// Runs of consecutive edges per thread in the plain top-down expansion.
constexpr int kRun = 4;

__global__ void k_plain_len(const int32_t *Q, const LevelCtr *prev, const int64_t *poff,
                            int32_t *len) {
  const int64_t qn = lc_qn(prev);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < qn;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t u = Q[i];
    len[i] = int32_t(poff[u + 1] - poff[u]);
  }
}

__global__ void __launch_bounds__(kBS) k_plain_expand(const int32_t *Q, const LevelCtr *prev,
                                                      const int64_t *scan, const int64_t *poff,
                                                      const int32_t *pcol, Out out, uint32_t *Vn,
                                                      int32_t *Qnext, LevelCtr *cur) {
  __shared__ int32_t qbuf[kQCap];
  __shared__ int qcount;
  __shared__ unsigned long long qbase;
  __shared__ unsigned long long sh[4 * kNW];
  BlockAppend qa{qbuf, &qcount, &qbase, kQCap, &cur->qn_nc, Qnext};
  qa.init();
  const int64_t qn = lc_qn(prev);
  const int64_t E = scan[qn];
  const int64_t nruns = (E + kRun - 1) / kRun;
  unsigned long long claimed = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t r0 = int64_t(blockIdx.x) * blockDim.x; r0 < nruns; r0 += stride) {
    const int64_t r = r0 + threadIdx.x;
    int64_t e = r * kRun;
    const int64_t eend = min(e + kRun, E);
    int64_t idx = r < nruns ? seg_search(scan, qn, e) : 0;
    for (int t = 0; t < kRun; ++t, ++e) {
      bool won = false;
      int32_t v = 0;
      if (r < nruns && e < eend) {
        while (scan[idx + 1] <= e) ++idx;
        const int32_t u = Q[idx];
        v = pcol[poff[u] + (e - scan[idx])];
        won = bit_claim(Vn, uint32_t(v));
        if (won) {
          out.put(v, u);
          ++claimed;
        }
      }
      qa.push(won, v);
    }
    qa.maybe_flush(kBS * kRun + kBS);
  }
  qa.flush();
  unsigned long long entries = 0, edges = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    entries = (unsigned long long)qn;
    edges = (unsigned long long)E;
  }
  // units: queue entries, edges, claimed
  block_add4(cur->units[DSBFS_K_PLAIN], entries, edges, claimed, 0, sh);
}


// Number of resident waves worth of blocks for grid-stride kernels.
int stride_grid() { return 256 * 8; }

}  // namespace

Workspace *workspace_create(const Graph *g, int32_t max_lanes) {
  if (max_lanes != 0 && max_lanes != 64)
    fail(DSBFS_ERR_INVALID_ARG, "max_lanes must be 0 or 64");
  Workspace *ws = new Workspace();
  try {
    ws->g = g;
    ws->max_lanes = max_lanes;
    const Alloc *al = &g->al;
    hipStream_t s = g->stream;
    const int64_t n = g->n, d = g->d;
    ws->Vn.alloc(al, size_t(g->nwords()) * 4, s);
    ws->Fn.alloc(al, size_t(g->nwords()) * 4, s);
    ws->Vd.alloc(al, size_t(g->dwords()) * 4, s);
    ws->Fd.alloc(al, size_t(g->dwords()) * 4, s);
    ws->Cd.alloc(al, size_t(g->dwords()) * 4, s);
    ws->q0.alloc(al, size_t(n) * 4, s);
    ws->q1.alloc(al, size_t(n) * 4, s);
    ws->dlist.alloc(al, size_t(d) * 4, s);
    ws->dcand.alloc(al, size_t(d) * 4, s);
    ws->dlen.alloc(al, size_t(std::max(n, d)) * 4, s);
    ws->dscan.alloc(al, size_t(std::max(n, d) + 1) * 8, s);
    ws->c0.alloc(al, size_t(g->st.n_ndsrc) * 4, s);
    ws->c1.alloc(al, size_t(g->st.n_ndsrc) * 4, s);
    ws->ctr.alloc(al, 2 * sizeof(LevelCtr), s);
    ws->scan_tmp.alloc(al, scan_tmp_bytes(std::max(n, d)), s);
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&ws->hctr), 2 * sizeof(LevelCtr),
                         hipHostMallocDefault));
    ws->dctl.alloc(al, sizeof(DevCtl), s);
    ws->dtiles.alloc(al, 2 * dtiles_half(d), s);
    HIPCHK(hipHostMalloc(&ws->hstat, kStatusSlots * sizeof(LevelStatus), hipHostMallocDefault));
    std::memset(ws->hstat, 0, kStatusSlots * sizeof(LevelStatus));
    for (hipEvent_t &e : ws->lev_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return ws;
  } catch (...) {
    delete ws;
    throw;
  }
}

void workspace_destroy(Workspace *ws) { delete ws; }

static dsbfs_run_opts default_opts() {
  dsbfs_run_opts o{};
  o.mode = 1;
  o.want_parent = 1;
  // tuned for this layout (see the header); the paper's are DSBFS_PAPER_FACTOR0_*
  o.factor0[0] = 0.02;
  o.factor0[1] = 0.001;
  o.factor0[2] = 1e-6;
  o.factor1[0] = o.factor1[1] = o.factor1[2] = 0.0;
  o.forced = 0;
  o.forced_seed = 0;
  o.nn_do = 0;
  o.factor0_nn = 1e-3;
  o.factor1_nn = 0.0;
  return o;
}

void run_opts_default(dsbfs_run_opts *o) { *o = default_opts(); }


// Per-kernel launch counts, unit totals and (optionally) HIP-event timing.
struct Prof {
  bool on = false;
  hipStream_t s = nullptr;
  Workspace *ws = nullptr;
  size_t next = 0;
  struct Span { int k, b, e, level; };
  int level = -1;  // level whose kernels are being launched (-1: init)
  std::vector<Span> spans;
  int64_t launches[DSBFS_NUM_KERNELS] = {};
  double units[DSBFS_NUM_KERNELS][6] = {};

  hipEvent_t ev() {
    if (next == ws->events.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ws->events.push_back(e);
    }
    return ws->events[next++];
  }
  int begin() {
    if (!on) return -1;
    const int i = int(next);
    HIPCHK(hipEventRecord(ev(), s));
    return i;
  }
  void end(int k, int b) {
    ++launches[k];
    if (!on) return;
    const int i = int(next);
    HIPCHK(hipEventRecord(ev(), s));
    spans.push_back({k, b, i, level});
  }
  void add_level(const LevelCtr &c) {
    for (int k = 0; k < DSBFS_NUM_KERNELS; ++k)
      for (int j = 0; j < 4; ++j) units[k][j] += double(c.units[k][j]);
  }
};

namespace {

// The kernels of one level of degree-separated DOBFS (queue parity p: the
// level reads Q[p] and ctr[p ^ 1], writes Q[p ^ 1] and ctr[p]). Every kernel
// reads the plan from the control block, so the same sequence serves every
// level and can be captured once.
struct LevelLaunch {
  const Graph *g;
  Workspace *ws;
  Out out;
  DevCtl *c;
  LevelCtr *ctr;
  int32_t *Q[2], *C[2];
  uint32_t *Vn, *Fn, *Vd, *Fd, *Cd;
  LevelStatus *hs;
  int64_t *bsum, *bscan;
  bool nn_do;  // nn under the direction decision: its own forward and backward passes

  // skip: kernels left out because they cannot have work (captured level
  // variants): bit 0 the forward nd visit, bit 1 the forward dd/dn visit and
  // its prefix sum. Direct launches pass 0.
  void enqueue(int p, hipStream_t s, Prof *P, int skip = 0) const {
    const int32_t n = g->n, d = g->d;
    LevelCtr *cur = ctr + p, *prev = ctr + (p ^ 1);
    const int SG = stride_grid();
    auto begin = [&]() { return P ? P->begin() : -1; };
    auto end = [&](int k, int b) {
      if (P) P->end(k, b);
    };
    // the delegate previsit first: the normal previsit reads its frontier
    // count (whether Fn is needed this level)
    int b = -1;
    if (d > 0) {
      b = begin();
      hipLaunchKernelGGL(k_prev_deleg, dim3(grid_for(g->dwords(), kBS, 4096)), dim3(kBS), 0, s,
                         Fd, g->dwords(), g->doff.as<uint64_t>(), ws->dlist.as<int32_t>(), cur,
                         static_cast<const DevCtl *>(c));
      HIPCHK(hipGetLastError());
      end(DSBFS_K_PREV_DELEG, b);
    }
    b = begin();
    hipLaunchKernelGGL(k_normal_level, dim3(SG), dim3(kBS), 0, s, Q[p], prev,
                       g->noff.as<uint64_t>(), g->nlen.as<uint16_t>(), g->ncol.as<int32_t>(),
                       static_cast<const uint32_t *>(g->nnoff.as<uint32_t>()),
                       static_cast<const int32_t *>(g->nncol.as<int32_t>()), out, Vn, Fn,
                       static_cast<const DevCtl *>(c), Q[p ^ 1], cur);
    HIPCHK(hipGetLastError());
    end(DSBFS_K_PREV_NORMAL, b);
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(kWave), 0, s, c, static_cast<const LevelCtr *>(cur),
                       static_cast<const LevelCtr *>(prev), hs);
    HIPCHK(hipGetLastError());
    if (nn_do) {
      b = begin();
      hipLaunchKernelGGL(k_td_nn, dim3(SG), dim3(kBS), 0, s, static_cast<const int32_t *>(Q[p]),
                         static_cast<const DevCtl *>(c), g->noff.as<uint64_t>(),
                         g->nlen.as<uint16_t>(), g->ncol.as<int32_t>(),
                         static_cast<const uint32_t *>(g->nnoff.as<uint32_t>()),
                         static_cast<const int32_t *>(g->nncol.as<int32_t>()), out, Vn, Q[p ^ 1],
                         cur);
      HIPCHK(hipGetLastError());
      end(DSBFS_K_TD_NN, b);
    }
    if (d > 0 && !(skip & 1)) {
      b = begin();
      hipLaunchKernelGGL(k_td_nd, dim3(SG), dim3(kBS), 0, s, static_cast<const int32_t *>(Q[p]),
                         static_cast<const DevCtl *>(c), g->noff.as<uint64_t>(),
                         g->ncol.as<int32_t>(), g->vid_of.as<int32_t>(), out, Cd, cur);
      HIPCHK(hipGetLastError());
      end(DSBFS_K_TD_NORMAL, b);
    }
    if (d > 0 && !(skip & 2)) {
      b = begin();
      const unsigned nb = unsigned((int64_t(d) + kScanTile - 1) / kScanTile);
      hipLaunchKernelGGL(k_dscan_reduce, dim3(nb), dim3(kBS), 0, s,
                         static_cast<const int32_t *>(ws->dlist.as<int32_t>()),
                         g->doff.as<uint64_t>(), static_cast<const LevelCtr *>(cur),
                         static_cast<const DevCtl *>(c), ws->dlen.as<int32_t>(), bsum);
      hipLaunchKernelGGL(k_dscan_top, dim3(1), dim3(1024), 0, s, static_cast<const int64_t *>(bsum),
                         bscan, ws->dscan.as<int64_t>(), static_cast<const LevelCtr *>(cur),
                         static_cast<const DevCtl *>(c));
      hipLaunchKernelGGL(k_dscan_down, dim3(nb), dim3(kBS), 0, s, ws->dlen.as<int32_t>(),
                         ws->dscan.as<int64_t>(), static_cast<const LevelCtr *>(cur),
                         static_cast<const DevCtl *>(c), static_cast<const int64_t *>(bscan));
      hipLaunchKernelGGL(k_td_deleg, dim3(SG), dim3(kBS), 0, s, ws->dlist.as<int32_t>(),
                         ws->dscan.as<int64_t>(), static_cast<const LevelCtr *>(cur),
                         g->doff.as<uint64_t>(), g->dcol.as<int32_t>(), g->vid_of.as<int32_t>(),
                         static_cast<const DevCtl *>(c), out, Vn, Cd, Q[p ^ 1], cur);
      HIPCHK(hipGetLastError());
      end(DSBFS_K_TD_DELEG, b);
    }
    // bottom-up nn (nn_do): after every forward visit of the level, before
    // the bottom-up dn visit (which then sees its claims as visited)
    if (nn_do && g->st.n_nnsrc > 0) {
      b = begin();
      hipLaunchKernelGGL(k_bu_nn, dim3(SG), dim3(kBS), 0, s, static_cast<const DevCtl *>(c),
                         g->nnsrc.as<int32_t>(), g->st.n_nnsrc, g->noff.as<uint64_t>(),
                         g->nlen.as<uint16_t>(), g->ncol.as<int32_t>(),
                         static_cast<const uint32_t *>(Fn), out, Vn, Q[p ^ 1], cur);
      HIPCHK(hipGetLastError());
      end(DSBFS_K_BU_NN, b);
    }
    if (d > 0) {
      if (g->st.n_ndsrc > 0 && !(skip & 4)) {
        b = begin();
        hipLaunchKernelGGL(k_bu_normal, dim3(SG), dim3(kBS), 0, s, static_cast<const DevCtl *>(c),
                           C[0], C[1], g->ndsrc.as<int32_t>(), g->nds_off.as<int64_t>(),
                           g->nds_col.as<int32_t>(), g->nds_first.as<int2>(),
                           g->vid_of.as<int32_t>(), static_cast<const uint32_t *>(Fd), out, Vn,
                           Q[p ^ 1], cur);
        HIPCHK(hipGetLastError());
        end(DSBFS_K_BU_NORMAL, b);
      }
      if (!(skip & 8)) {
      b = begin();
      hipLaunchKernelGGL(k_dcand, dim3(grid_for(g->dwords(), kBS, 4096)), dim3(kBS), 0, s,
                         static_cast<const uint32_t *>(Cd), g->ddsrc_mask.as<uint32_t>(),
                         g->dnsrc_mask.as<uint32_t>(), g->dwords(), static_cast<const DevCtl *>(c),
                         ws->dcand.as<int32_t>(), cur);
      hipLaunchKernelGGL(k_bu_deleg, dim3(SG), dim3(kBS), 0, s, ws->dcand.as<int32_t>(),
                         static_cast<const LevelCtr *>(cur), g->doff.as<uint64_t>(),
                         g->dcol.as<int32_t>(), g->dd_first.as<int2>(),
                         static_cast<const uint32_t *>(Fd), static_cast<const uint32_t *>(Fn),
                         g->vid_of.as<int32_t>(), static_cast<const DevCtl *>(c), out, Cd, cur);
      HIPCHK(hipGetLastError());
      end(DSBFS_K_BU_DELEG, b);
      }
    }
    b = begin();
    hipLaunchKernelGGL(k_close, dim3(grid_for(std::max<int64_t>(n, g->dwords()), kBS, 4096)),
                       dim3(kBS), 0, s, Vd, Fd, static_cast<const uint32_t *>(Cd), g->dwords(), Fn,
                       int64_t(g->nwords()), static_cast<const int32_t *>(Q[p]), c, prev);
    HIPCHK(hipGetLastError());
    end(DSBFS_K_CLOSE, b);
  }
};

LevelLaunch level_launch(const Graph *g, Workspace *ws, const Out &out, bool nn_do) {
  LevelLaunch ll{};
  ll.nn_do = nn_do;
  ll.g = g;
  ll.ws = ws;
  ll.out = out;
  ll.c = ws->dctl.as<DevCtl>();
  ll.ctr = ws->ctr.as<LevelCtr>();
  ll.Q[0] = ws->q0.as<int32_t>();
  ll.Q[1] = ws->q1.as<int32_t>();
  ll.C[0] = ws->c0.as<int32_t>();
  ll.C[1] = ws->c1.as<int32_t>();
  ll.Vn = ws->Vn.as<uint32_t>();
  ll.Fn = ws->Fn.as<uint32_t>();
  ll.Vd = ws->Vd.as<uint32_t>();
  ll.Fd = ws->Fd.as<uint32_t>();
  ll.Cd = ws->Cd.as<uint32_t>();
  ll.hs = static_cast<LevelStatus *>(ws->hstat);
  // tile sums and their scan of the delegate-frontier prefix sum
  const size_t half = dtiles_half(g->d);
  ll.bsum = ws->dtiles.as<int64_t>();
  ll.bscan = reinterpret_cast<int64_t *>(ws->dtiles.as<char>() + half);
  return ll;
}

// Captured level graphs per workspace, for the depth / parent buffers they
// were captured with: one per queue parity and skip variant (see
// LevelLaunch::enqueue), each captured when first needed.
constexpr int kLevelVariants = 16;
struct LevelGraphs {
  int32_t *depth = nullptr, *parent = nullptr;
  bool nn_do = false;
  int64_t searches = 0;  // searches run on these graphs
  hipGraph_t graph[kLevelVariants][2] = {};
  hipGraphExec_t exec[kLevelVariants][2] = {};
};

}  // namespace

void level_graphs_release(Workspace *ws) {
  auto *lg = static_cast<LevelGraphs *>(ws->lvl);
  if (!lg) return;
  for (int v = 0; v < kLevelVariants; ++v)
    for (int i = 0; i < 2; ++i) {
      if (lg->exec[v][i]) (void)hipGraphExecDestroy(lg->exec[v][i]);
      if (lg->graph[v][i]) (void)hipGraphDestroy(lg->graph[v][i]);
    }
  delete lg;
  ws->lvl = nullptr;
}

namespace {

// The level graphs of this workspace for ll's buffers (recaptured when they
// change); variant v of parity p is captured on first use.
LevelGraphs &level_graphs(Workspace *ws, const LevelLaunch &ll) {
  auto *lg = static_cast<LevelGraphs *>(ws->lvl);
  if (lg && lg->depth == ll.out.depth && lg->parent == ll.out.parent && lg->nn_do == ll.nn_do)
    return *lg;
  level_graphs_release(ws);
  lg = new LevelGraphs();
  ws->lvl = lg;
  lg->depth = ll.out.depth;
  lg->parent = ll.out.parent;
  lg->nn_do = ll.nn_do;
  return *lg;
}

hipGraphExec_t level_exec(Workspace *ws, LevelGraphs &lg, const LevelLaunch &ll, int v, int p) {
  if (lg.exec[v][p]) return lg.exec[v][p];
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  try {
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      ll.enqueue(p, cs, nullptr, v);
    } catch (...) {
      hipGraph_t gr = nullptr;
      (void)hipStreamEndCapture(cs, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    HIPCHK(hipStreamEndCapture(cs, &lg.graph[v][p]));
    HIPCHK(hipGraphInstantiate(&lg.exec[v][p], lg.graph[v][p], nullptr, nullptr, 0));
  } catch (...) {
    (void)hipStreamDestroy(cs);
    level_graphs_release(ws);
    throw;
  }
  (void)hipStreamDestroy(cs);
  return lg.exec[v][p];
}

}  // namespace

void bfs_run(const Graph *g, Workspace *ws, int32_t source, const dsbfs_run_opts *opts_in,
             int32_t *depth, int32_t *parent, dsbfs_run_stats *stats, hipStream_t s) {
  if (!ws || ws->g != g) fail(DSBFS_ERR_INVALID_ARG, "workspace does not belong to this graph");
  if (source < 0 || source >= g->n) fail(DSBFS_ERR_INVALID_ARG, "source outside [0, n)");
  if (!depth) fail(DSBFS_ERR_INVALID_ARG, "depth must not be NULL");
  const dsbfs_run_opts o = opts_in ? *opts_in : default_opts();
  if (o.mode != 0 && o.mode != 1) fail(DSBFS_ERR_INVALID_ARG, "mode must be 0 or 1");
  if (o.want_parent && !parent) fail(DSBFS_ERR_INVALID_ARG, "parent is NULL but want_parent");
  if (o.mode == 0 && !g->pcol.p && g->m > 0)
    fail(DSBFS_ERR_INVALID_ARG, "mode 0 needs the plain CSR (keep_plain_csr)");
  if (o.forced < 0 || o.forced > 3) fail(DSBFS_ERR_INVALID_ARG, "forced must be 0..3");
  if (o.nn_do != 0 && o.nn_do != 1) fail(DSBFS_ERR_INVALID_ARG, "nn_do must be 0 or 1");
  int32_t *par = o.want_parent ? parent : nullptr;

  const int32_t n = g->n, d = g->d;
  uint32_t *Vn = ws->Vn.as<uint32_t>(), *Fn = ws->Fn.as<uint32_t>();
  uint32_t *Vd = ws->Vd.as<uint32_t>(), *Fd = ws->Fd.as<uint32_t>(), *Cd = ws->Cd.as<uint32_t>();
  int32_t *Q[2] = {ws->q0.as<int32_t>(), ws->q1.as<int32_t>()};
  LevelCtr *ctr = ws->ctr.as<LevelCtr>();
  LevelCtr *h = ws->hctr;
  const int SG = stride_grid();
  Prof P;
  P.on = o.profile != 0 && stats != nullptr;
  P.s = s;
  P.ws = ws;

  int b = P.begin();
  hipLaunchKernelGGL(k_init, dim3(grid_for(std::max(n, 1), kBS, 4096)), dim3(kBS), 0, s, depth,
                     par, n, Vn, Fn, g->nwords(), Vd, Fd, Cd, g->dwords());
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(ctr, 0, 2 * sizeof(LevelCtr), s));
  // level L uses ctr[L & 1]; the seed plays the part of "level -1" (ctr[1]).
  hipLaunchKernelGGL(k_seed, dim3(1), dim3(1), 0, s, source, g->did.as<int32_t>(), depth, par,
                     Vn, Vd, Fd, Cd, Q[0], ctr + 1, o.mode);
  HIPCHK(hipGetLastError());
  P.end(DSBFS_K_INIT, b);
  P.units[DSBFS_K_INIT][0] = n;

  std::vector<dsbfs_level_stats> rec;
  double deg_sum = 0;  // sum of degrees over all frontiers = over reached vertices
  int qi = 0;  // Q[qi] is the current queue
  Out out{depth, par, 0};

  if (o.mode == 0) {
    for (int32_t L = 0;; ++L) {
      LevelCtr *cur = ctr + (L & 1), *prev = ctr + ((L + 1) & 1);
      // the previous level's queue length is the only input of this level
      HIPCHK(hipMemcpyAsync(h, prev, sizeof(LevelCtr), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      P.add_level(*h);
      const int64_t qn = lc_qn(h);
      if (qn == 0) break;
      HIPCHK(hipMemsetAsync(cur, 0, sizeof(LevelCtr), s));
      out.level1 = L + 1;
      b = P.begin();
      hipLaunchKernelGGL(k_plain_len, dim3(grid_for(qn, kBS, 8192)), dim3(kBS), 0, s, Q[qi], prev,
                         g->poff.as<int64_t>(), ws->dlen.as<int32_t>());
      HIPCHK(hipGetLastError());
      scan_excl_i32_to_i64(ws->dlen.as<int32_t>(), ws->dscan.as<int64_t>(), qn, ws->scan_tmp.p, s);
      hipLaunchKernelGGL(k_plain_expand, dim3(SG), dim3(kBS), 0, s, Q[qi], prev,
                         ws->dscan.as<int64_t>(), g->poff.as<int64_t>(), g->pcol.as<int32_t>(),
                         out, Vn, Q[qi ^ 1], cur);
      HIPCHK(hipGetLastError());
      P.end(DSBFS_K_PLAIN, b);
      qi ^= 1;
      dsbfs_level_stats r{};
      r.frontier_normal = qn;
      rec.push_back(r);
    }
  } else {
    // Degree-separated DOBFS with the level control on the device.
    DevCtl *c = ws->dctl.as<DevCtl>();
    DevCtl init{};
    for (int k = 0; k < 3; ++k) {
      init.f0[k] = o.factor0[k];
      init.f1[k] = o.factor1[k];
    }
    init.f0[3] = o.factor0_nn;
    init.f1[3] = o.factor1_nn;
    init.nn_do = o.nn_do;
    init.forced = o.forced;
    init.forced_seed = o.forced_seed;
    init.level = 0;  // level 0 is open: counters cleared above, depth 1 next
    init.level1 = 1;
    init.mark_fn = g->st.n_dnsrc > 0 || (o.nn_do && g->st.n_nnsrc > 0);
    init.cand_state = -1;
    init.nwords = g->nwords();
    init.rem[0] = g->st.n_ddsrc;
    init.rem[1] = g->st.n_dnsrc;
    init.rem[2] = g->st.n_ndsrc;
    init.rem[3] = g->st.n_nnsrc;
    init.nc = g->st.n_ndsrc;
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, s, c, init);
    HIPCHK(hipGetLastError());
    LevelStatus *hs = static_cast<LevelStatus *>(ws->hstat);
    const LevelLaunch ll = level_launch(g, ws, out, o.nn_do != 0);
    std::vector<LevelStatus> seen;
    if (ws->borrowed) {
      // allocation-free search: direct launches (no captured graphs, no
      // events), and the level's status record copied from device memory
      // after each level
      for (int32_t L = 0;; ++L) {
        ll.enqueue(L & 1, s, nullptr);
        LevelStatus st;
        HIPCHK(hipMemcpyAsync(&st, hs + (L & (kStatusSlots - 1)), sizeof(LevelStatus),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (st.done) break;
        seen.push_back(st);
      }
    } else if (P.on) {
      // direct launches with an event around each kernel and one stream
      // synchronization per level, so that only kernels with work are counted
      for (int32_t L = 0;; ++L) {
        const size_t sp0 = P.spans.size();
        P.level = L;
        ll.enqueue(L & 1, s, &P);
        HIPCHK(hipStreamSynchronize(s));
        const LevelStatus st = hs[L & (kStatusSlots - 1)];
        const int32_t ran[DSBFS_NUM_KERNELS] = {
            0, 1, d > 0, !st.done && st.plan[0], !st.done && (st.plan[1] || st.plan[2]),
            !st.done && st.plan[3], !st.done && (st.plan[4] || st.plan[5]), !st.done, 0,
            !st.done && st.plan[8], !st.done && st.plan[9]};
        std::vector<Prof::Span> keep;
        for (size_t i = sp0; i < P.spans.size(); ++i) {
          if (ran[P.spans[i].k]) keep.push_back(P.spans[i]);
          else --P.launches[P.spans[i].k];
        }
        P.spans.resize(sp0);
        P.spans.insert(P.spans.end(), keep.begin(), keep.end());
        if (st.done) break;
        seen.push_back(st);
      }
    } else {
      // one captured graph per level; the host stays one level ahead and
      // stops once a finished level reports an empty frontier (the level
      // already queued behind it returns at once). One level ahead hides the
      // host's wait and launch behind the level in flight; two would add a
      // second graph of no-op kernels at the end of every search.
      //
      // The level the host launches next leaves out kernels that cannot have
      // work, from the latest status it has seen (two levels earlier):
      // - under the heuristic schedule with factor1 = 0 a subgraph that went
      //   backward never switches back (FV < 0 * BV never holds), so its
      //   forward kernels could only return at once;
      // - the counts U of unvisited vertices a bottom-up visit scans never
      //   grow, and a bottom-up visit needs U > 0 (any schedule).
      //
      // Variants run only on graphs kept from an earlier search: a caller
      // that passes new output buffers on every call (the query server's
      // result rows) would otherwise capture several graphs per search.
      LevelGraphs &lg = level_graphs(ws, ll);
      const bool variants = lg.searches > 0;
      const bool monotone = o.forced == 0 && o.factor1[0] == 0.0 && o.factor1[1] == 0.0 &&
                            o.factor1[2] == 0.0;
      int variant = 0;
      for (int32_t L = 0;; ++L) {
        HIPCHK(hipGraphLaunch(level_exec(ws, lg, ll, variant, L & 1), s));
        HIPCHK(hipEventRecord(ws->lev_ev[L % 3], s));
        if (L >= 1) {
          HIPCHK(hipEventSynchronize(ws->lev_ev[(L - 1) % 3]));
          const LevelStatus &st = hs[(L - 1) & (kStatusSlots - 1)];
          if (st.done) break;
          seen.push_back(st);
          if (!variants) continue;
          variant = (st.rec.U[1] == 0 ? 4 : 0) | (st.rec.U[0] == 0 && st.rec.U[2] == 0 ? 8 : 0);
          if (monotone)
            variant |= (st.rec.dir[2] == 1 ? 1 : 0) |
                       (st.rec.dir[0] == 1 && st.rec.dir[1] == 1 ? 2 : 0);
        }
      }
      ++lg.searches;
    }
    for (const LevelStatus &st : seen) {
      rec.push_back(st.rec);
      if (!P.on) {
        const int32_t *pl = st.plan;
        ++P.launches[DSBFS_K_PREV_NORMAL];
        if (d > 0) ++P.launches[DSBFS_K_PREV_DELEG];
        if (pl[0]) ++P.launches[DSBFS_K_TD_NORMAL];
        if (pl[1] || pl[2]) ++P.launches[DSBFS_K_TD_DELEG];
        if (pl[3]) ++P.launches[DSBFS_K_BU_NORMAL];
        if (pl[4] || pl[5]) ++P.launches[DSBFS_K_BU_DELEG];
        if (pl[8]) ++P.launches[DSBFS_K_TD_NN];
        if (pl[9]) ++P.launches[DSBFS_K_BU_NN];
        ++P.launches[DSBFS_K_CLOSE];
      }
    }
    if (!P.on) {
      // the level that found the frontier empty ran its previsit (as did the
      // levels queued behind it, which return at once and are not counted)
      ++P.launches[DSBFS_K_PREV_NORMAL];
      if (d > 0) ++P.launches[DSBFS_K_PREV_DELEG];
    }
    if (stats) {
      DevCtl hc{};
      HIPCHK(hipMemcpyAsync(&hc, c, sizeof(DevCtl), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int k = 0; k < DSBFS_NUM_KERNELS; ++k) {
        if (k == DSBFS_K_INIT) continue;
        for (int j = 0; j < 6; ++j) P.units[k][j] = double(hc.units[k][j]);
      }
      deg_sum = double(hc.deg_sum);
    }
  }

  if (stats) {
    HIPCHK(hipStreamSynchronize(s));
    stats->num_levels = int32_t(rec.size());
    for (int32_t i = 0; i < stats->num_levels && i < stats->capacity && stats->levels; ++i) {
      stats->levels[i] = rec[i];
      for (double &t : stats->levels[i].kernel_ms) t = 0.0;  // filled from the spans below
    }
    // Every reached vertex sits in exactly one level's frontier, whose previsit
    // (or plain expansion) summed its full degree; each vertex but the source
    // was claimed exactly once. So the component's size and edge count come
    // from the level counters without another pass over depth[].
    const auto &Uc = P.units;
    const double claims = Uc[DSBFS_K_PREV_NORMAL][2] + Uc[DSBFS_K_TD_NORMAL][3] +
                          Uc[DSBFS_K_TD_DELEG][2] + Uc[DSBFS_K_TD_DELEG][3] +
                          Uc[DSBFS_K_BU_NORMAL][3] + Uc[DSBFS_K_BU_DELEG][2] +
                          Uc[DSBFS_K_PLAIN][2] + Uc[DSBFS_K_TD_NN][2] + Uc[DSBFS_K_BU_NN][3];
    stats->reached = 1 + int64_t(claims);
    if (o.mode == 0) deg_sum = Uc[DSBFS_K_PLAIN][1];
    stats->edges_cc = int64_t(deg_sum / 2);

    // Algorithmic bytes per kernel from its unit counts (see dsbfs.h).
    const double out_b = o.want_parent ? 8.0 : 4.0;  // depth (+ parent) per vertex
    const auto &U = P.units;
    double bytes[DSBFS_NUM_KERNELS] = {};
    double edges[DSBFS_NUM_KERNELS] = {};
    bytes[DSBFS_K_INIT] = U[DSBFS_K_INIT][0] * out_b;
    bytes[DSBFS_K_PREV_NORMAL] = U[DSBFS_K_PREV_NORMAL][0] * (4 + 16) +
                                 U[DSBFS_K_PREV_NORMAL][1] * 4 +
                                 U[DSBFS_K_PREV_NORMAL][2] * (out_b + 4);
    edges[DSBFS_K_PREV_NORMAL] = U[DSBFS_K_PREV_NORMAL][1];
    bytes[DSBFS_K_PREV_DELEG] = U[DSBFS_K_PREV_DELEG][0] * (4 + 16);
    bytes[DSBFS_K_TD_NORMAL] = U[DSBFS_K_TD_NORMAL][0] * (4 + 16) + U[DSBFS_K_TD_NORMAL][1] * 4 +
                               U[DSBFS_K_TD_NORMAL][3] * (out_b + 4);
    edges[DSBFS_K_TD_NORMAL] = U[DSBFS_K_TD_NORMAL][1];
    bytes[DSBFS_K_TD_DELEG] = U[DSBFS_K_TD_DELEG][0] * (4 + 16) + U[DSBFS_K_TD_DELEG][1] * 4 +
                              U[DSBFS_K_TD_DELEG][2] * (out_b + 4 + 4) +
                              U[DSBFS_K_TD_DELEG][3] * (out_b + 4 + 4);
    edges[DSBFS_K_TD_DELEG] = U[DSBFS_K_TD_DELEG][1];
    bytes[DSBFS_K_BU_NORMAL] = U[DSBFS_K_BU_NORMAL][0] * 4 + U[DSBFS_K_BU_NORMAL][1] * 16 +
                               U[DSBFS_K_BU_NORMAL][2] * 4 +
                               U[DSBFS_K_BU_NORMAL][3] * (out_b + 4 + 4) +
                               U[DSBFS_K_BU_NORMAL][4] * 4;
    edges[DSBFS_K_BU_NORMAL] = U[DSBFS_K_BU_NORMAL][2];
    bytes[DSBFS_K_BU_DELEG] = U[DSBFS_K_BU_DELEG][0] * (4 + 4 + 16) +
                              U[DSBFS_K_BU_DELEG][1] * 4 + U[DSBFS_K_BU_DELEG][2] * (out_b + 4 + 4);
    edges[DSBFS_K_BU_DELEG] = U[DSBFS_K_BU_DELEG][1];
    bytes[DSBFS_K_CLOSE] = U[DSBFS_K_CLOSE][0] * 4;
    bytes[DSBFS_K_PLAIN] = U[DSBFS_K_PLAIN][0] * (4 + 16) + U[DSBFS_K_PLAIN][1] * 4 +
                           U[DSBFS_K_PLAIN][2] * (out_b + 4);
    edges[DSBFS_K_PLAIN] = U[DSBFS_K_PLAIN][1];
    bytes[DSBFS_K_TD_NN] = U[DSBFS_K_TD_NN][0] * (4 + 16) + U[DSBFS_K_TD_NN][1] * 4 +
                           U[DSBFS_K_TD_NN][2] * (out_b + 4);
    edges[DSBFS_K_TD_NN] = U[DSBFS_K_TD_NN][1];
    bytes[DSBFS_K_BU_NN] = U[DSBFS_K_BU_NN][0] * 4 + U[DSBFS_K_BU_NN][1] * 16 +
                           U[DSBFS_K_BU_NN][2] * 4 + U[DSBFS_K_BU_NN][3] * (out_b + 4 + 4);
    edges[DSBFS_K_BU_NN] = U[DSBFS_K_BU_NN][2];
    double ms[DSBFS_NUM_KERNELS] = {};
    for (const Prof::Span &sp : P.spans) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ws->events[sp.b], ws->events[sp.e]));
      ms[sp.k] += double(t);
      if (sp.level >= 0 && sp.level < stats->num_levels && sp.level < stats->capacity &&
          stats->levels)
        stats->levels[sp.level].kernel_ms[sp.k] += double(t);
    }
    for (int k = 0; k < DSBFS_NUM_KERNELS; ++k) {
      stats->kernels[k].ms = ms[k];
      stats->kernels[k].launches = P.launches[k];
      stats->kernels[k].bytes = int64_t(bytes[k]);
      stats->kernels[k].edges = int64_t(edges[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Allocation-free single-source search
// ---------------------------------------------------------------------------
// For callers that cannot allocate device memory: the search's scratch (the
// workspace's bitmaps, queues, candidate lists, counters, control block and
// level status ring) is carved out of one file-scope device array. Each GPU
// holds its own copy of the array, at its own address, from the library's
// load until the process ends; host code never uses the array's name as an
// address, only the device address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct ScratchSlot {
  std::mutex mu;         // one search at a time per device
  void *ptr = nullptr;   // device address of `scratch` on this device
};

ScratchSlot &scratch_slot(int dev) {
  static ScratchSlot slots[kMaxDevices];
  return slots[dev];
}

inline size_t round256(size_t b) { return ((b < 256 ? 256 : b) + 255) / 256 * 256; }

}  // namespace

size_t noalloc_scratch_bytes(const Graph *g) {
  const int64_t n = g->n, d = g->d, nm = std::max(n, d);
  size_t t = 0;
  t += 2 * round256(size_t(g->nwords()) * 4);          // Vn, Fn
  t += 3 * round256(size_t(g->dwords()) * 4);          // Vd, Fd, Cd
  t += 2 * round256(size_t(n) * 4);                    // q0, q1
  t += 2 * round256(size_t(d) * 4);                    // dlist, dcand
  t += round256(size_t(nm) * 4);                       // dlen
  t += round256(size_t(nm + 1) * 8);                   // dscan
  t += 2 * round256(size_t(g->st.n_ndsrc) * 4);        // c0, c1
  t += round256(2 * sizeof(LevelCtr));                 // ctr
  t += round256(scan_tmp_bytes(nm));                   // scan_tmp
  t += round256(sizeof(DevCtl));                       // dctl
  t += round256(2 * dtiles_half(d));                   // dtiles
  t += round256(kStatusSlots * sizeof(LevelStatus));   // status ring
  return t;
}

void bfs_run_noalloc(const Graph *g, int32_t source, const dsbfs_run_opts *opts, int32_t *depth,
                     int32_t *parent, dsbfs_run_stats *stats, hipStream_t s) {
  if (!g) fail(DSBFS_ERR_INVALID_ARG, "graph must not be NULL");
  if (opts && opts->profile)
    fail(DSBFS_ERR_INVALID_ARG, "profile = 1 needs timing events; the allocation-free search "
                                "does not create them");
  const size_t need = noalloc_scratch_bytes(g);
  if (need > kScratchBytes)
    fail(DSBFS_ERR_RANGE, "graph needs " + std::to_string(need) +
                              " bytes of search scratch; the allocation-free search holds " +
                              std::to_string(kScratchBytes) + " (use a workspace)");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(DSBFS_ERR_INVALID_ARG, "device index out of range");
  ScratchSlot &sl = scratch_slot(dev);
  std::lock_guard<std::mutex> lock(sl.mu);
  if (!sl.ptr) {
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(DSBFS_ERR_HIP, "hipGetSymbolAddress returned NULL for the search scratch");
    sl.ptr = ptr;
  }
  char *base = static_cast<char *>(sl.ptr);
  size_t off = 0;
  auto carve = [&](DevBuf &b, size_t bytes) {
    b.p = base + off;
    b.bytes = round256(bytes);
    b.al = nullptr;   // not owned: nothing is freed
    b.s = s;
    off += b.bytes;
  };
  const int64_t n = g->n, d = g->d, nm = std::max(n, d);
  Workspace ws;
  ws.g = g;
  ws.borrowed = true;
  carve(ws.Vn, size_t(g->nwords()) * 4);
  carve(ws.Fn, size_t(g->nwords()) * 4);
  carve(ws.Vd, size_t(g->dwords()) * 4);
  carve(ws.Fd, size_t(g->dwords()) * 4);
  carve(ws.Cd, size_t(g->dwords()) * 4);
  carve(ws.q0, size_t(n) * 4);
  carve(ws.q1, size_t(n) * 4);
  carve(ws.dlist, size_t(d) * 4);
  carve(ws.dcand, size_t(d) * 4);
  carve(ws.dlen, size_t(nm) * 4);
  carve(ws.dscan, size_t(nm + 1) * 8);
  carve(ws.c0, size_t(g->st.n_ndsrc) * 4);
  carve(ws.c1, size_t(g->st.n_ndsrc) * 4);
  carve(ws.ctr, 2 * sizeof(LevelCtr));
  carve(ws.scan_tmp, scan_tmp_bytes(nm));
  carve(ws.dctl, sizeof(DevCtl));
  carve(ws.dtiles, 2 * dtiles_half(d));
  DevBuf ring;
  carve(ring, kStatusSlots * sizeof(LevelStatus));
  if (off != need) fail(DSBFS_ERR_HIP, "allocation-free scratch layout mismatch");
  LevelCtr hctr[2];
  ws.hctr = hctr;
  ws.hstat = ring.p;
  bfs_run(g, &ws, source, opts, depth, parent, stats, s);
  // the next call reuses the array: this one's work must be complete
  HIPCHK(hipStreamSynchronize(s));
}

}  // namespace dsbfs
