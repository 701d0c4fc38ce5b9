// Bit-parallel multi-source BFS: 64 x W sources per batch (W = 1, 2 or 4) as
// the lanes of W 64-bit words per vertex (seen, and a ring of per-level lane
// sets that serves as frontier and as depth record), all batches in one
// persistent launch.
//
// Not in the paper: the batched form follows the bit-parallel multi-source
// BFS of Then et al., "The More the Merrier" (PVLDB 8(4), 2014). Each lane's
// depths are exactly those of a single-source BFS from that lane's source.
//
// Per level of a batch:
//   top-down  (few frontier vertices): every vertex v with frontier[v] != 0
//             ORs frontier[v] & ~seen[w] into next[w] of each neighbour w,
//             then a close pass folds next into seen;
//   bottom-up (otherwise): every vertex w with unseen lanes ORs frontier[v]
//             of its neighbours until all of its unseen lanes are covered,
//             and closes itself on the spot (writes next[w], seen[w]).
// Depths are written from the ring once per batch (earlier only if the search
// runs longer than the ring holds). Levels and batches are separated by a grid
// barrier inside one kernel whose grid fits the chip (occupancy-checked); the
// barrier's wait is bounded, so a grid that is not fully resident ends with an
// error flag instead of a hang. The launch can be captured once into a
// hipGraph and replayed.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>

#include "internal.hpp"

namespace dsbfs {

namespace {

// Arrival counters of the grid barrier, one per 128-byte line so that the
// groups' atomics do not meet on one address.
constexpr int kBarGroups = 32;
struct alignas(128) BarSlot {
  unsigned long long count;  // 64-bit: never wraps within a launch
  unsigned long long pad[15];
};

// A batch runs 64 x W sources as the bits of W 64-bit words per vertex.
constexpr int kMaxWords = 4;

struct MsCtl {
  BarSlot grp[kBarGroups];     // arrivals per block group (monotonic)
  BarSlot top;                 // groups complete (monotonic)
  unsigned int err;            // 1: a barrier wait timed out
  unsigned int pad;
  unsigned long long td_count;   // frontier vertices listed for a top-down level
  unsigned long long active[3];  // vertices with a non-empty next mask, per level (rolling)
  unsigned long long alive[3][kMaxWords];  // lanes with a non-empty next frontier (rolling)
  unsigned long long levels;     // levels run, summed over batches
  unsigned long long edges;      // adjacency entries read, summed over batches
};

struct MsArgs {
  const int64_t *off;
  const int32_t *col;
  int32_t n;
  const int32_t *sources;  // device copy, k entries
  int32_t k;
  int32_t *depth;          // [k][n]
  void *seen;              // LaneSet<W>[n]
  void *ring;              // kRing slots of LaneSet<W>[n]: lanes first reaching each vertex at level j
  int32_t *tdlist;         // frontier vertices of a top-down level, n entries
  int64_t *tdscan;         // prefix of their degrees, n + 1 entries
  const int32_t *hubs;     // vertices of degree > kHub, scanned by whole waves bottom-up
  int64_t nhubs;
  // Hub frontier cache (bottom-up reads): col2 is col with every hub
  // neighbour h replaced by n + (its index in hubs); hot holds two slots of
  // nhubs lane sets, slot L & 1 a copy of level L's frontier of the hubs.
  // col2 == col and hot == nullptr when the cache is off.
  const int32_t *col2;
  const int32_t *hub_idx;  // index in hubs of each vertex, -1 if not a hub
  void *hot;
  MsCtl *ctl;
  int64_t bu_threshold;    // bottom-up when active vertices exceed this
  long long timeout_ticks; // bound of one barrier wait (wall clock ticks)
};

__device__ __forceinline__ long long wall_ticks() { return wall_clock64(); }

// Grid-wide barrier in two levels: block b counts its arrival on group
// b % kBarGroups; the group's last arrival counts on `top`, and everyone waits
// for `top` to reach the epoch's target. Counters only grow (the launch starts
// them at zero), so an arrival's ticket names its epoch and nothing is reset.
// Fences on both sides make every plain store before the barrier visible to
// every block after it; the wait itself polls with relaxed loads, since an
// acquiring load per poll would invalidate the L2 under the blocks still at
// work. Returns false (everywhere) once any wait has exceeded the bound.
__device__ bool grid_sync(MsCtl *ctl, long long timeout_ticks) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned long long G = gridDim.x;
    const unsigned long long grp = blockIdx.x % kBarGroups;
    const unsigned long long gsize = G / kBarGroups + (grp < G % kBarGroups ? 1u : 0u);
    const unsigned long long ngroups = G < kBarGroups ? G : kBarGroups;
    const unsigned long long ticket = atomicAdd(&ctl->grp[grp].count, 1ull);
    const unsigned long long target = (ticket / gsize + 1u) * ngroups;
    if (ticket % gsize == gsize - 1u) {
      __threadfence();
      atomicAdd(&ctl->top.count, 1ull);
    }
    const long long t0 = wall_ticks();
    while (__hip_atomic_load(&ctl->top.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           target) {
      if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      if (wall_ticks() - t0 > timeout_ticks) {
        atomicOr(&ctl->err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
    ok = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  return ok;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long *sh) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  return t;
}

// The lanes of one vertex: W 64-bit words, lane i in bit i % 64 of word i / 64.
template <int W>
struct alignas(W == 1 ? 8 : 16) LaneSet {
  uint64_t w[W];
};

template <int W>
__device__ __forceinline__ bool lanes_any(const LaneSet<W> &x) {
  uint64_t o = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) o |= x.w[j];
  return o != 0;
}

// Ring of per-level lane sets: slot j % kRing holds, for every vertex, the
// lanes that first reach it at level j. That array is level j's frontier and
// also the record from which depths are written, so depths are stored once
// per batch in one dense pass (or when the ring is about to wrap) instead of
// one masked store per level.
constexpr int kRing = 16;

template <int W>
__device__ __forceinline__ LaneSet<W> *ring_slot(const MsArgs &a, int32_t j) {
  return static_cast<LaneSet<W> *>(a.ring) + int64_t(j & (kRing - 1)) * a.n;
}

// Writes depth j for the lanes of ring levels [f, t) (t - f < kRing) and, when
// `final`, -1 for the lanes that never reached the vertex. A wave takes 64
// consecutive vertices and stores one 256-byte row segment per batch lane.
// mask[j]: the batch's lanes in word j.
template <int W>
__device__ void flush_depth(const MsArgs &a, int64_t row0, const uint64_t *mask, int32_t f,
                            int32_t t, bool final, int64_t tid, int64_t nthreads,
                            int64_t nv_iter) {
  const int32_t n = a.n;
  const LaneSet<W> *seen = static_cast<const LaneSet<W> *>(a.seen);
  for (int64_t it = 0; it < nv_iter; ++it) {
    const int64_t v = tid + it * nthreads;
    const bool valid = v < n;
    // bit b of a lane's level offset j - f, as four lane sets
    LaneSet<W> q0{}, q1{}, q2{}, q3{}, got{}, miss{};
    if (valid) {
      for (int32_t j = f; j < t; ++j) {
        const LaneSet<W> m = ring_slot<W>(a, j)[v];
        const int32_t o = j - f;
#pragma unroll
        for (int x = 0; x < W; ++x) {
          got.w[x] |= m.w[x];
          q0.w[x] |= (o & 1) ? m.w[x] : 0ull;
          q1.w[x] |= (o & 2) ? m.w[x] : 0ull;
          q2.w[x] |= (o & 4) ? m.w[x] : 0ull;
          q3.w[x] |= (o & 8) ? m.w[x] : 0ull;
        }
      }
      if (final) {
        const LaneSet<W> sv = seen[v];
#pragma unroll
        for (int x = 0; x < W; ++x) miss.w[x] = ~sv.w[x] & mask[x];
      }
    }
#pragma unroll
    for (int x = 0; x < W; ++x) {
      const uint64_t wr = got.w[x] | miss.w[x];
      uint64_t all = wave_or_all(wr);
      while (all) {
        const int i = __ffsll(static_cast<long long>(all)) - 1;
        all &= all - 1;
        if ((wr >> i) & 1ull) {
          const int32_t d = ((miss.w[x] >> i) & 1ull)
                                ? -1
                                : f + int32_t((q0.w[x] >> i) & 1ull) +
                                      (int32_t((q1.w[x] >> i) & 1ull) << 1) +
                                      (int32_t((q2.w[x] >> i) & 1ull) << 2) +
                                      (int32_t((q3.w[x] >> i) & 1ull) << 3);
          a.depth[(row0 + 64 * x + i) * int64_t(n) + v] = d;
        }
      }
    }
  }
}

constexpr int kHub = 64;

__device__ __forceinline__ uint64_t wave_or(uint64_t x) { return wave_or_all(x); }

// LDS rows of one wave for the bottom-up walk (64 vertices).
template <int W>
struct BuRows {
  int32_t ex[kWave];           // exclusive prefix of the row lengths
  int64_t beg[kWave];          // row starts
  LaneSet<W> want[kWave];      // lanes each vertex still needs
  unsigned long long acc[kWave][W];  // lanes found so far
};

// Bottom-up for the 64 vertices of a wave (one per lane; lanes with nothing
// wanted take no part): the rows are prefix-summed across the wave and walked
// 64 entries at a time, so consecutive vertices' rows are read coalesced and
// 64 frontier sets are in flight per step. Each vertex's frontier OR collects
// in LDS; the walk stops once every vertex's wanted lanes are covered. Called
// by every lane of the wave; returns the lanes found for this lane's vertex.
// The frontier set of neighbour entry c: fcur[c], or hcur[c - nlim] for an
// entry that names a hub slot (c >= nlim).
template <int W>
__device__ __forceinline__ LaneSet<W> front_of(const LaneSet<W> *fcur, const LaneSet<W> *hcur,
                                               int32_t nlim, int32_t c) {
  return c >= nlim ? hcur[c - nlim] : fcur[c];
}

template <int W>
__device__ LaneSet<W> bu_wave(const int64_t *off, const int32_t *col, const LaneSet<W> *fcur,
                              const LaneSet<W> *hcur, int32_t nlim, int64_t w,
                              const LaneSet<W> &want, BuRows<W> &r,
                              unsigned long long &edges) {
  const int l = lane_id();
  int32_t len = 0;
  int64_t beg = 0;
  if (lanes_any(want)) {
    beg = off[w];
    len = int32_t(off[w + 1] - beg);
  }
  const int32_t incl = wave_incl_scan(len);
  const int32_t T = lane_read(incl, kWave - 1);
  wave_sync();
  r.ex[l] = incl - len;
  r.beg[l] = beg;
  r.want[l] = want;
#pragma unroll
  for (int x = 0; x < W; ++x) r.acc[l][x] = 0;
  wave_sync();
  auto covered = [&](int o, const LaneSet<W> &wl) {
    bool c = true;
#pragma unroll
    for (int x = 0; x < W; ++x) c = c && (r.acc[o][x] & wl.w[x]) == wl.w[x];
    return c;
  };
  uint64_t pend = __ballot(len > 0);
  for (int32_t e0 = 0; e0 < T && pend; e0 += kWave) {
    const int32_t e = e0 + l;
    if (e < T) {
      int o = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        const int c = o + step;
        if (r.ex[c] <= e) o = c;
      }
      const LaneSet<W> wl = r.want[o];
      if (!covered(o, wl)) {
        const LaneSet<W> m = front_of<W>(fcur, hcur, nlim, col[r.beg[o] + (e - r.ex[o])]);
        ++edges;
#pragma unroll
        for (int x = 0; x < W; ++x) {
          const uint64_t y = m.w[x] & wl.w[x];
          if (y) atomicOr(&r.acc[o][x], (unsigned long long)y);
        }
      }
    }
    wave_sync();
    pend = __ballot(len > 0 && !covered(l, want));
  }
  LaneSet<W> res;
#pragma unroll
  for (int x = 0; x < W; ++x) res.w[x] = r.acc[l][x] & want.w[x];
  wave_sync();
  return res;
}

template <int W>
__global__ void __launch_bounds__(1024) k_msbfs(MsArgs a) {
  // per wave: bottom-up rows, or a top-down level's window of the degree scan
  __shared__ union {
    BuRows<W> rows[16];
    int64_t win[16][kWave + 1];
  } s_u;
  __shared__ unsigned long long sh[16];
  constexpr int kLanes = 64 * W;
  const int32_t n = a.n;
  LaneSet<W> *const seen = static_cast<LaneSet<W> *>(a.seen);
  LaneSet<W> *const hot = static_cast<LaneSet<W> *>(a.hot);
  const int32_t nlim = hot ? n : INT32_MAX;  // col2 entries >= nlim name hub slots
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nthreads = int64_t(gridDim.x) * blockDim.x;
  const int64_t nv_iter = (int64_t(n) + nthreads - 1) / nthreads;
  const int nbatch = (a.k + kLanes - 1) / kLanes;
  const int64_t wid = tid / kWave, nwaves = nthreads / kWave;
  const int l = lane_id();
  unsigned long long edges = 0;
  for (int b = 0; b < nbatch; ++b) {
    const int lanes = min(kLanes, a.k - b * kLanes);
    uint64_t mask[W];
#pragma unroll
    for (int x = 0; x < W; ++x) {
      const int in = lanes - 64 * x;
      mask[x] = in >= 64 ? ~0ull : (in > 0 ? (1ull << in) - 1ull : 0ull);
    }
    const int64_t row0 = int64_t(b) * kLanes;
    // reset lane state: seen, level 0 (the sources) and level 1 (a top-down
    // first level ORs into it)
    LaneSet<W> *const lv0 = ring_slot<W>(a, 0), *const lv1 = ring_slot<W>(a, 1);
    for (int64_t v = tid; v < n; v += nthreads) {
      seen[v] = LaneSet<W>{};
      lv0[v] = LaneSet<W>{};
      lv1[v] = LaneSet<W>{};
    }
    if (hot)
      for (int64_t h = tid; h < a.nhubs; h += nthreads) hot[h] = LaneSet<W>{};
    if (blockIdx.x == 0 && threadIdx.x < 3) {
      a.ctl->active[threadIdx.x] = 0;
#pragma unroll
      for (int x = 0; x < kMaxWords; ++x) a.ctl->alive[threadIdx.x][x] = 0;
    }
    if (!grid_sync(a.ctl, a.timeout_ticks)) return;
    // seed the sources of this batch (duplicates share a vertex: OR the lanes)
    if (tid < lanes) {
      const int32_t s = a.sources[row0 + tid];
      const int x = int(tid) >> 6;
      const unsigned long long bit = 1ull << (tid & 63);
      atomicOr(reinterpret_cast<unsigned long long *>(&seen[s].w[x]), bit);
      atomicOr(reinterpret_cast<unsigned long long *>(&lv0[s].w[x]), bit);
      if (hot && a.hub_idx[s] >= 0)
        atomicOr(reinterpret_cast<unsigned long long *>(&hot[a.hub_idx[s]].w[x]), bit);
    }
    if (!grid_sync(a.ctl, a.timeout_ticks)) return;
    int64_t active = lanes;
    int32_t flushed = 0;  // levels [0, flushed) have their depths written
    // Lanes whose frontier is empty are finished: no vertex waits for them.
    LaneSet<W> live;
#pragma unroll
    for (int x = 0; x < W; ++x) live.w[x] = mask[x];
    int32_t L = 0;
    for (;; ++L) {
      // slot L + 2 is cleared at the end of this level and slot L + 1 written
      // during it: the levels they held must have their depths out first
      if (L + 2 - kRing >= flushed) {
        flush_depth<W>(a, row0, mask, flushed, L + 1, false, tid, nthreads, nv_iter);
        flushed = L + 1;
        if (!grid_sync(a.ctl, a.timeout_ticks)) return;
      }
      LaneSet<W> *const fcur = ring_slot<W>(a, L), *const fnext = ring_slot<W>(a, L + 1);
      // hub copies of this level's frontier (read) and of the next (written)
      LaneSet<W> *const hcur = hot ? hot + (L & 1) * a.nhubs : nullptr;
      LaneSet<W> *const hnext = hot ? hot + ((L + 1) & 1) * a.nhubs : nullptr;
      // the rolling count slot level L + 1 adds into; every block read it
      // (for level L - 2) before the barrier that ended level L - 1
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl->active[(L + 2) % 3] = 0;
#pragma unroll
        for (int x = 0; x < W; ++x) a.ctl->alive[(L + 2) % 3][x] = 0;
      }
      unsigned long long act = 0;
      LaneSet<W> lor{};
      if (active <= a.bu_threshold) {
        // top-down, edge-parallel: (1) list the frontier vertices that have
        // edges, (2) one block prefix-sums their degrees, (3) every wave takes
        // a contiguous share of the concatenated rows. fnext is all zero here.
        for (int64_t v0 = int64_t(blockIdx.x) * blockDim.x; v0 < n; v0 += nthreads) {
          const int64_t v = v0 + threadIdx.x;
          const bool f = v < n && lanes_any(fcur[v]) && a.off[v + 1] > a.off[v];
          const int64_t pos = wave_append(f, &a.ctl->td_count);
          if (f) a.tdlist[pos] = int32_t(v);
        }
        if (!grid_sync(a.ctl, a.timeout_ticks)) return;
        const int64_t cnt = int64_t(__hip_atomic_load(&a.ctl->td_count, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
        if (blockIdx.x == 0) {
          unsigned long long carry = 0;
          for (int64_t i0 = 0; i0 < cnt; i0 += blockDim.x) {
            const int64_t i = i0 + threadIdx.x;
            unsigned long long dg = 0;
            if (i < cnt) {
              const int32_t v = a.tdlist[i];
              dg = (unsigned long long)(a.off[v + 1] - a.off[v]);
            }
            const unsigned long long incl = wave_incl_scan(dg);
            if (lane_id() == kWave - 1) sh[threadIdx.x / kWave] = incl;
            __syncthreads();
            unsigned long long before = 0, tot = 0;
            for (int j = 0; j < int(blockDim.x / kWave); ++j) {
              before += j < int(threadIdx.x / kWave) ? sh[j] : 0ull;
              tot += sh[j];
            }
            if (i < cnt) a.tdscan[i] = int64_t(carry + before + incl - dg);
            carry += tot;
            __syncthreads();
          }
          if (threadIdx.x == 0) a.tdscan[cnt] = int64_t(carry);
        }
        if (!grid_sync(a.ctl, a.timeout_ticks)) return;
        const int64_t E = a.tdscan[cnt];
        // wave share: [eb, ee), a multiple of 64 edges. Every listed row has
        // an edge, so 64 consecutive edges belong to at most 64 consecutive
        // list entries: a step stages the scan values of the 65 entries from
        // its first edge's owner in LDS, finds each edge's owner among the
        // first 64, and the first edge of the next step's owner with the 65th.
        const int64_t share = ((E + nwaves - 1) / nwaves + kWave - 1) / kWave * kWave;
        const int64_t eb = wid * share, ee = min(E, eb + share);
        if (eb < ee) {
          int64_t own = 0, hi = cnt - 1;  // owner of eb: last i with tdscan[i] <= eb
          while (own < hi) {
            const int64_t mid = (own + hi + 1) >> 1;
            if (a.tdscan[mid] <= eb) own = mid;
            else hi = mid - 1;
          }
          int64_t *const win = s_u.win[threadIdx.x / kWave];
          for (int64_t e0 = eb; e0 < ee; e0 += kWave) {
            win[l] = own + l < cnt ? a.tdscan[own + l] : INT64_MAX;
            if (l == 0) win[kWave] = own + kWave < cnt ? a.tdscan[own + kWave] : INT64_MAX;
            wave_sync();
            const int64_t e = e0 + l;
            int o = 0;
            if (e < ee) {
#pragma unroll
              for (int step = 32; step > 0; step >>= 1) {
                const int c = o + step;
                if (win[c] <= e) o = c;
              }
              const int32_t v = a.tdlist[own + o];
              const int32_t w = a.col[a.off[v] + (e - win[o])];
              ++edges;
              // lanes already in next (a possibly stale read: the atomic
              // decides) need no atomic
              const LaneSet<W> fv = fcur[v], sw = seen[w], nx = fnext[w];
#pragma unroll
              for (int x = 0; x < W; ++x) {
                const uint64_t m = fv.w[x] & ~sw.w[x] & ~nx.w[x];
                if (m) atomicOr(reinterpret_cast<unsigned long long *>(&fnext[w].w[x]), m);
              }
            }
            // owner of e0 + 64: the owner of this step's last edge, or the
            // entry after it when that row ended at e0 + 63 (a partial step
            // is the last one)
            const int o63 = lane_read(o, kWave - 1);
            own += o63 + (e0 + kWave >= win[o63 + 1] ? 1 : 0);
            wave_sync();
          }
        }
        if (!grid_sync(a.ctl, a.timeout_ticks)) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->td_count = 0;
        // close: fold next into seen (the scatter only set lanes that were
        // unseen, and seen did not change during it, so next is all new)
        for (int64_t v = tid; v < n; v += nthreads) {
          const LaneSet<W> nw = fnext[v];
          if (lanes_any(nw)) {
            LaneSet<W> s1 = seen[v];
#pragma unroll
            for (int x = 0; x < W; ++x) {
              s1.w[x] |= nw.w[x];
              lor.w[x] |= nw.w[x];
            }
            seen[v] = s1;
            ++act;
          }
        }
        if (hot)
          for (int64_t h = tid; h < a.nhubs; h += nthreads) hnext[h] = fnext[a.hubs[h]];
      } else {
        // bottom-up with the close fused in: w is only written by the thread
        // (or, for a hub, the wave) that scans it. Vertices of degree <= kHub:
        // one thread each; hubs: one wave each, 64 neighbours per step.
        BuRows<W> &rows = s_u.rows[threadIdx.x / kWave];
        for (int64_t it = 0; it < nv_iter; ++it) {
          const int64_t w = tid + it * nthreads;
          bool valid = w < n;
          LaneSet<W> s0{}, want{};
          if (valid) {
            if (a.off[w + 1] - a.off[w] > kHub) {
              valid = false;  // the hub pass below owns it
            } else {
              s0 = seen[w];
#pragma unroll
              for (int x = 0; x < W; ++x) want.w[x] = ~s0.w[x] & live.w[x];
            }
          }
          const LaneSet<W> nw = bu_wave<W>(a.off, a.col2, fcur, hcur, nlim, w, want, rows, edges);
          if (valid) {
            const bool any = lanes_any(nw);
            if (any) {
              LaneSet<W> s1;
#pragma unroll
              for (int x = 0; x < W; ++x) s1.w[x] = s0.w[x] | nw.w[x];
              seen[w] = s1;
            }
            fnext[w] = nw;
            act += any;
#pragma unroll
            for (int x = 0; x < W; ++x) lor.w[x] |= nw.w[x];
          }
        }
        // hubs, 64 per wave step: each lane screens one and closes it if it
        // wants nothing (most hubs in late levels); the wave then scans the
        // rows of the others one at a time
        for (int64_t h0 = wid * kWave; h0 < a.nhubs; h0 += nwaves * kWave) {
          const int64_t hl = h0 + l;
          bool need = false;
          if (hl < a.nhubs) {
            const int32_t wl = a.hubs[hl];
            const LaneSet<W> sl = seen[wl];
            LaneSet<W> wantl;
#pragma unroll
            for (int x = 0; x < W; ++x) wantl.w[x] = ~sl.w[x] & live.w[x];
            need = lanes_any(wantl);
            if (!need) {
              fnext[wl] = LaneSet<W>{};
              if (hot) hnext[hl] = LaneSet<W>{};
            }
          }
          for (uint64_t todo = __ballot(need); todo; todo &= todo - 1) {
            const int64_t h = h0 + __builtin_ctzll(todo);
            const int32_t w = a.hubs[h];
            const LaneSet<W> s0 = seen[w];
            LaneSet<W> want, acc{};
#pragma unroll
            for (int x = 0; x < W; ++x) want.w[x] = ~s0.w[x] & live.w[x];
            {
              const int64_t p1 = a.off[w + 1];
              for (int64_t p = a.off[w]; p < p1; p += kWave) {
                LaneSet<W> y{};
                if (p + l < p1) y = front_of<W>(fcur, hcur, nlim, a.col2[p + l]);
                bool done = true;
#pragma unroll
                for (int x = 0; x < W; ++x) {
                  acc.w[x] |= wave_or(y.w[x]);
                  done = done && (acc.w[x] & want.w[x]) == want.w[x];
                }
                if (l == 0) edges += uint64_t(min<int64_t>(kWave, p1 - p));
                if (done) break;
              }
            }
            LaneSet<W> nw;
#pragma unroll
            for (int x = 0; x < W; ++x) nw.w[x] = acc.w[x] & want.w[x];
            if (l == 0) {
              const bool any = lanes_any(nw);
              if (any) {
                LaneSet<W> s1;
#pragma unroll
                for (int x = 0; x < W; ++x) s1.w[x] = s0.w[x] | nw.w[x];
                seen[w] = s1;
              }
              fnext[w] = nw;
              if (hot) hnext[h] = nw;
              act += any;
#pragma unroll
              for (int x = 0; x < W; ++x) lor.w[x] |= nw.w[x];
            }
          }
        }
      }
      const unsigned long long bact = block_sum_u64(act, sh);
      if (threadIdx.x == 0 && bact) atomicAdd(&a.ctl->active[(L + 1) % 3], bact);
#pragma unroll
      for (int x = 0; x < W; ++x) {
        const uint64_t o = wave_or(lor.w[x]);
        if (l == 0 && o) atomicOr(&a.ctl->alive[(L + 1) % 3][x], (unsigned long long)o);
      }
      if (!grid_sync(a.ctl, a.timeout_ticks)) return;
      active = int64_t(__hip_atomic_load(&a.ctl->active[(L + 1) % 3], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT));
#pragma unroll
      for (int x = 0; x < W; ++x)
        live.w[x] = __hip_atomic_load(&a.ctl->alive[(L + 1) % 3][x], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.ctl->levels, 1ull);
      if (active == 0) break;
      // a top-down level L + 1 ORs into slot L + 2, which must start at zero
      // (its scatter comes two barriers after this); a bottom-up level
      // overwrites every entry itself
      if (active <= a.bu_threshold) {
        LaneSet<W> *const after = ring_slot<W>(a, L + 2);
        for (int64_t v = tid; v < n; v += nthreads) after[v] = LaneSet<W>{};
      }
    }
    // depths of the levels not yet written, and -1 for lanes never seen
    flush_depth<W>(a, row0, mask, flushed, L + 1, true, tid, nthreads, nv_iter);
    if (!grid_sync(a.ctl, a.timeout_ticks)) return;
  }
  const unsigned long long be = block_sum_u64(edges, sh);
  if (threadIdx.x == 0 && be) atomicAdd(&a.ctl->edges, be);
}

__global__ void k_hub_index(const int32_t *hubs, int64_t nhubs, int32_t *hub_idx) {
  for (int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; h < nhubs;
       h += int64_t(gridDim.x) * blockDim.x)
    hub_idx[hubs[h]] = int32_t(h);
}

__global__ void k_col_remap(const int32_t *col, int64_t m, const int32_t *hub_idx, int32_t n,
                            int32_t *col2) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int32_t c = col[e];
    const int32_t h = hub_idx[c];
    col2[e] = h >= 0 ? n + h : c;
  }
}

__global__ void k_flag_hub(const int64_t *off, int32_t n, uint8_t *flag) {
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x)
    flag[v] = off[v + 1] - off[v] > kHub;
}

int device_cus() {
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus;
}

std::string device_name() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t p;
  HIPCHK(hipGetDeviceProperties(&p, dev));
  return std::string(p.gcnArchName);
}

dsbfs_ms_opts default_ms_opts() {
  dsbfs_ms_opts o{};
  o.block = 1024;
  o.blocks_per_cu = 1;
  o.bu_permille = 2;
  o.use_graph = 1;
  o.lanes_per_batch = 0;
  return o;
}

// 64-bit words per vertex for k sources: the narrowest batch that holds them
// all, at most kMaxWords (the frontier set of a vertex is read whole per edge,
// so a wider batch costs little more per edge and needs fewer batches).
int ms_words(const dsbfs_ms_opts &o, int32_t k) {
  if (o.lanes_per_batch) return o.lanes_per_batch / 64;
  return k <= 64 ? 1 : (k <= 128 ? 2 : kMaxWords);
}

const void *ms_kernel(int words) {
  switch (words) {
    case 1: return reinterpret_cast<const void *>(&k_msbfs<1>);
    case 2: return reinterpret_cast<const void *>(&k_msbfs<2>);
    default: return reinterpret_cast<const void *>(&k_msbfs<4>);
  }
}

void check_ms_opts(const dsbfs_ms_opts &o) {
  if (o.block != 64 && o.block != 128 && o.block != 256 && o.block != 512 && o.block != 1024)
    fail(DSBFS_ERR_INVALID_ARG, "ms block must be 64, 128, 256, 512 or 1024");
  if (o.blocks_per_cu < 1 || o.blocks_per_cu > 32)
    fail(DSBFS_ERR_INVALID_ARG, "ms blocks_per_cu must be in [1, 32]");
  if (o.bu_permille < 0 || o.bu_permille > 1000)
    fail(DSBFS_ERR_INVALID_ARG, "ms bu_permille must be in [0, 1000]");
  if (o.lanes_per_batch != 0 && o.lanes_per_batch != 64 && o.lanes_per_batch != 128 &&
      o.lanes_per_batch != 256)
    fail(DSBFS_ERR_INVALID_ARG, "ms lanes_per_batch must be 0 (automatic), 64, 128 or 256");
}

// The graph captured for one (workspace, launch configuration, k, depth).
struct MsGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct MsState {
  DevBuf ctl, srcs, hubs;
  DevBuf ring, seen;  // kRing x n and n lane sets of `words` words each
  DevBuf hub_idx, col2, hot;  // hub frontier cache (see MsArgs)
  DevBuf lvring, lvseen;       // level-at-a-time use: kRing x n and n lane masks
  int words = 0;
  int64_t nhubs = -1;  // -1: hub list not built yet
  int32_t cap_k = 0;
  std::map<std::string, MsGraph> graphs;
  ~MsState() {
    for (auto &kv : graphs) {
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
  }
};

}  // namespace

void msbfs_release(Workspace *ws) {
  delete reinterpret_cast<MsState *>(ws->ms_state);
  ws->ms_state = nullptr;
}

static void msbfs_launch(const Graph *g, Workspace *ws, const int32_t *sources, int32_t k,
                         const dsbfs_ms_opts &o, int32_t *depth, hipStream_t s,
                         unsigned long long *levels_out, unsigned long long *edges_out) {
  if (!ws || ws->g != g) fail(DSBFS_ERR_INVALID_ARG, "workspace does not belong to this graph");
  if (ws->max_lanes != 64) fail(DSBFS_ERR_INVALID_ARG, "workspace was created without lanes");
  if (!g->pcol.p && g->m > 0) fail(DSBFS_ERR_INVALID_ARG, "multi-source BFS needs the plain CSR");
  if (k < 1 || !sources || !depth) fail(DSBFS_ERR_INVALID_ARG, "need k >= 1 sources and depth");
  for (int32_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) fail(DSBFS_ERR_INVALID_ARG, "source outside [0, n)");
  check_ms_opts(o);
  if (!ws->ms_state) ws->ms_state = new MsState();
  MsState *st = reinterpret_cast<MsState *>(ws->ms_state);
  const Alloc *al = &g->al;
  if (!st->ctl.p) st->ctl.alloc(al, sizeof(MsCtl), s);
  if (st->nhubs < 0) {
    // vertices whose rows a whole wave scans in bottom-up levels
    DevBuf flag, tmp, cnt;
    flag.alloc(al, size_t(g->n), s);
    tmp.alloc(al, compact_tmp_bytes(g->n), s);
    cnt.alloc(al, 8, s);
    st->hubs.alloc(al, size_t(g->n) * 4, s);
    hipLaunchKernelGGL(k_flag_hub, dim3(grid_for(g->n, 256, 8192)), dim3(256), 0, s,
                       g->poff.as<int64_t>(), g->n, flag.as<uint8_t>());
    HIPCHK(hipGetLastError());
    compact_flags_u8(flag.as<uint8_t>(), g->n, st->hubs.as<int32_t>(), cnt.as<int64_t>(), tmp.p,
                     s);
    st->nhubs = d2h_scalar(cnt.as<int64_t>(), s);
  }
  // hub frontier cache: the remapped columns once per graph (while hub slot
  // numbers n + h fit int32)
  if (st->nhubs > 0 && !st->col2.p && int64_t(g->n) + st->nhubs < int64_t(INT32_MAX)) {
    st->hub_idx.alloc(al, size_t(g->n) * 4, s);
    HIPCHK(hipMemsetAsync(st->hub_idx.p, 0xff, size_t(g->n) * 4, s));
    hipLaunchKernelGGL(k_hub_index, dim3(grid_for(st->nhubs, 256, 8192)), dim3(256), 0, s,
                       st->hubs.as<int32_t>(), st->nhubs, st->hub_idx.as<int32_t>());
    st->col2.alloc(al, size_t(g->m) * 4, s);
    hipLaunchKernelGGL(k_col_remap, dim3(grid_for(g->m, 256, 8192)), dim3(256), 0, s,
                       g->pcol.as<int32_t>(), g->m, st->hub_idx.as<int32_t>(), g->n,
                       st->col2.as<int32_t>());
    HIPCHK(hipGetLastError());
  }
  const int words = ms_words(o, k);
  const bool grow_lanes = st->words < words;
  if (grow_lanes) {
    st->ring.alloc(al, size_t(kRing) * size_t(g->n) * 8 * words, s);
    st->seen.alloc(al, size_t(g->n) * 8 * words, s);
    if (st->col2.p) st->hot.alloc(al, size_t(2) * size_t(st->nhubs) * 8 * words, s);
    st->words = words;
  }
  if (st->cap_k < k || grow_lanes) {
    if (st->cap_k < k) st->srcs.alloc(al, size_t(k) * 4, s);
    st->cap_k = std::max(st->cap_k, k);
    // captured graphs hold the old pointer
    for (auto &kv : st->graphs) {
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    st->graphs.clear();
  }
  HIPCHK(hipMemcpyAsync(st->srcs.p, sources, size_t(k) * 4, hipMemcpyHostToDevice, s));
  const void *kern = ms_kernel(words);
  int occ = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, o.block, 0));
  if (occ < 1) fail(DSBFS_ERR_INVALID_ARG, "ms block size does not fit a compute unit");
  const int per_cu = std::min(o.blocks_per_cu, occ);
  const int grid = device_cus() * per_cu;

  MsArgs a{};
  a.off = g->poff.as<int64_t>();
  a.col = g->pcol.as<int32_t>();
  a.n = g->n;
  a.sources = st->srcs.as<int32_t>();
  a.k = k;
  a.depth = depth;
  a.seen = st->seen.p;
  a.ring = st->ring.p;
  a.tdlist = ws->dlen.as<int32_t>();    // int32[max(n, d)]
  a.tdscan = ws->dscan.as<int64_t>();   // int64[max(n, d) + 1]
  a.hubs = st->hubs.as<int32_t>();
  a.nhubs = st->nhubs;
  a.col2 = st->col2.p ? st->col2.as<int32_t>() : a.col;
  a.hub_idx = st->col2.p ? st->hub_idx.as<int32_t>() : nullptr;
  a.hot = st->col2.p ? st->hot.p : nullptr;
  a.ctl = st->ctl.as<MsCtl>();
  a.bu_threshold = int64_t(g->n) * o.bu_permille / 1000;
  a.timeout_ticks = 100000000ll * 20;  // 20 s of the 100 MHz wall clock per barrier wait

  // control block cleared by a kernel-free copy of zeros from the host
  static const MsCtl zero{};
  HIPCHK(hipMemcpyAsync(st->ctl.p, &zero, sizeof(MsCtl), hipMemcpyHostToDevice, s));
  if (o.use_graph) {
    char key[160];
    std::snprintf(key, sizeof(key), "%d/%d/%d/%d/%d/%p", o.block, grid, k, o.bu_permille, words,
                  static_cast<void *>(depth));
    MsGraph &mg = st->graphs[key];
    if (!mg.exec) {
      hipStream_t cs;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        // captured as a cooperative launch, so the runtime still checks that
        // the whole grid is co-resident when the graph is replayed
        void *args[] = {&a};
        e = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(o.block), args, 0, cs);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &gr);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) {
          mg.graph = gr;
          e = hipGraphInstantiate(&mg.exec, gr, nullptr, nullptr, 0);
        } else if (gr) {
          (void)hipGraphDestroy(gr);
        }
      }
      (void)hipStreamDestroy(cs);
      HIPCHK(e);
    }
    HIPCHK(hipGraphLaunch(mg.exec, s));
  } else {
    void *args[] = {&a};
    HIPCHK(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(o.block), args, 0, s));
  }
  MsCtl h{};
  HIPCHK(hipMemcpyAsync(&h, st->ctl.p, sizeof(MsCtl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h.err) fail(DSBFS_ERR_DEVICE, "multi-source BFS: a grid barrier wait timed out");
  if (levels_out) *levels_out = h.levels;
  if (edges_out) *edges_out = h.edges;
}

static const dsbfs_ms_opts *tuned_or_default(const Graph *g, dsbfs_ms_opts *buf) {
  *buf = default_ms_opts();
  (void)g;
  return buf;
}

void msbfs_run(const Graph *g, Workspace *ws, const int32_t *sources, int32_t k,
               const dsbfs_ms_opts *opts, int32_t *depth, hipStream_t s) {
  dsbfs_ms_opts buf;
  const dsbfs_ms_opts &o = opts ? *opts : *tuned_or_default(g, &buf);
  msbfs_launch(g, ws, sources, k, o, depth, s, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate (block, blocks per CU, switch threshold) settings
// on the caller's sources and keeps the fastest; results are cached in a
// small JSON file keyed by device, n and m.
// ---------------------------------------------------------------------------
static std::string tune_key(const Graph *g) {
  std::ostringstream os;
  os << device_name() << ":n" << g->n << ":m" << g->m;
  return os.str();
}

static bool cache_lookup(const char *path, const std::string &key, dsbfs_ms_opts *o) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    // one entry per line: {"key": "...", "block": B, "blocks_per_cu": C, "bu_permille": P, "use_graph": G}
    const std::string tag = "\"key\": \"" + key + "\"";
    if (line.find(tag) == std::string::npos) continue;
    auto num = [&](const char *name, int32_t *dst) {
      const std::string t = std::string("\"") + name + "\": ";
      size_t p = line.find(t);
      if (p == std::string::npos) return false;
      *dst = std::atoi(line.c_str() + p + t.size());
      return true;
    };
    dsbfs_ms_opts r{};
    if (num("block", &r.block) && num("blocks_per_cu", &r.blocks_per_cu) &&
        num("bu_permille", &r.bu_permille) && num("use_graph", &r.use_graph)) {
      check_ms_opts(r);
      *o = r;
      return true;
    }
  }
  return false;
}

static void cache_store(const char *path, const std::string &key, const dsbfs_ms_opts &o,
                        double ms) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  if (!f) fail(DSBFS_ERR_INVALID_ARG, std::string("cannot write tuner cache ") + path);
  f << "{\"key\": \"" << key << "\", \"block\": " << o.block << ", \"blocks_per_cu\": "
    << o.blocks_per_cu << ", \"bu_permille\": " << o.bu_permille << ", \"use_graph\": "
    << o.use_graph << ", \"ms\": " << ms << "}\n";
}

void msbfs_tune(const Graph *g, Workspace *ws, const int32_t *sources, int32_t k,
                const char *cache_path, dsbfs_ms_opts *best, hipStream_t s) {
  const std::string key = tune_key(g);
  if (cache_lookup(cache_path, key, best)) return;
  if (k < 1) fail(DSBFS_ERR_INVALID_ARG, "tuning needs at least one source");
  // up to one full batch of the widest lane set, so the candidates run at the
  // lane width the full launch will use
  const int32_t kt = std::min<int32_t>(k, 64 * kMaxWords);
  DevBuf out;
  out.alloc(&g->al, size_t(kt) * size_t(g->n) * 4, s);
  double best_ms = 1e30;
  dsbfs_ms_opts bo = default_ms_opts();
  const int blocks[] = {256, 512, 1024};
  const int percu[] = {1, 2, 4, 8};
  const int thr[] = {0, 1, 5, 20};
  for (int b : blocks)
    for (int c : percu) {
      int occ = 0;
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, ms_kernel(ms_words(default_ms_opts(), kt)), b, 0));
      if (c > occ || b * c > 2048) continue;
      for (int t : thr) {
        dsbfs_ms_opts o{};
        o.block = b;
        o.blocks_per_cu = c;
        o.bu_permille = t;
        o.use_graph = 0;
        msbfs_launch(g, ws, sources, kt, o, out.as<int32_t>(), s, nullptr, nullptr);  // warm
        const auto t0 = std::chrono::steady_clock::now();
        msbfs_launch(g, ws, sources, kt, o, out.as<int32_t>(), s, nullptr, nullptr);
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
        if (ms < best_ms) {
          best_ms = ms;
          bo = o;
        }
      }
    }
  bo.use_graph = 1;
  *best = bo;
  cache_store(cache_path, key, bo, best_ms);
}

}  // namespace dsbfs

// ---------------------------------------------------------------------------
// Level-at-a-time multi-source BFS for the query server: lanes join and leave
// at level boundaries (continuous batching), so each lane has its own result
// row and its own start level, and the host decides between levels. As in the
// persistent kernel, a ring of kRing per-level lane masks is the frontier and
// the depth record: a lane's row is written in one dense pass when its
// frontier runs empty (or, for the levels about to be overwritten, when the
// ring wraps).
// ---------------------------------------------------------------------------
namespace dsbfs {

struct MsLevel {
  const int64_t *off;
  const int32_t *col;
  int32_t n;
  uint64_t *seen, *fcur, *fnext;
  uint64_t *ring;           // kRing slots of n masks; fcur / fnext are two of them
  int32_t *tdlist;
  int64_t *tdscan;
  const int32_t *hubs;
  int64_t nhubs;
  unsigned long long *ctl;  // [0] active, [1] alive, [2] td_count, [3] edges
  uint64_t live;
};

namespace {

__device__ __forceinline__ void lv_flush(const MsLevel &a, unsigned long long act, uint64_t lor,
                                         unsigned long long edges) {
  act = wave_sum(act);
  edges = wave_sum(edges);
  lor = wave_or_all(lor);
  if (lane_id() == 0) {
    if (act) atomicAdd(&a.ctl[0], act);
    if (lor) atomicOr(&a.ctl[1], (unsigned long long)lor);
    if (edges) atomicAdd(&a.ctl[3], edges);
  }
}

// Clears the lanes in `clear` (recycled lanes) from seen and from the current
// and next frontier. Their bits in older ring slots stay: a lane's rows only
// ever read levels from its start on.
__global__ void k_lv_recycle(MsLevel a, uint64_t clear) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    a.seen[v] &= ~clear;
    a.fcur[v] &= ~clear;
    a.fnext[v] &= ~clear;
  }
}

// Seeds lane i at source src.src[i] for every lane in `mask` (its depth 0 is
// written from the ring with the rest of its row).
__global__ void k_lv_seed(MsLevel a, uint64_t mask, SeedList src) {
  const int i = threadIdx.x;
  if (i < 64 && ((mask >> i) & 1ull)) {
    const int32_t s = src.src[i];
    atomicOr(reinterpret_cast<unsigned long long *>(&a.seen[s]), 1ull << i);
    atomicOr(reinterpret_cast<unsigned long long *>(&a.fcur[s]), 1ull << i);
  }
}

// Also, when publish is set (once per level, after the level's kernels):
// block 0 copies the level's control block to host_ctl (pinned host memory,
// read by the host once the stream passes this kernel) and clears
// next_ctl, the control block of the next level.
// Writes the result rows of a set of lanes from ring levels [f.jlo, f.jhi]
// (fewer than kRing): depth j - start[i] where lane i's bit is in level j's
// mask and f.valid[j - jlo] admits lane i (levels before a lane's start or
// already written are excluded), and, when `final`, -1 where the lane never
// arrived. final: the set is f.lanes minus the lanes still alive after the
// level just run (ctl[1]), i.e. the lanes that completed; else f.lanes.
__global__ void k_lv_flush(MsLevel a, LaneFlush f, unsigned long long *next_ctl,
                           unsigned long long *host_ctl) {
  if (host_ctl && blockIdx.x == 0 && threadIdx.x < 4) {
    host_ctl[threadIdx.x] = a.ctl[threadIdx.x];
    next_ctl[threadIdx.x] = 0;
  }
  uint64_t set = f.lanes;
  if (f.final) set &= ~a.ctl[1];
  if (!set) return;
  const int64_t nthreads = int64_t(gridDim.x) * blockDim.x;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t iters = (int64_t(a.n) + nthreads - 1) / nthreads;
  const int32_t nlev = f.jhi - f.jlo + 1;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t v = tid + it * nthreads;
    const bool valid = v < a.n;
    uint64_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, got = 0, miss = 0;
    if (valid) {
      for (int32_t o = 0; o < nlev; ++o) {
        const int32_t j = f.jlo + o;
        const uint64_t m = a.ring[int64_t(j & (kRing - 1)) * a.n + v] & f.valid[o] & set;
        got |= m;
        q0 |= (o & 1) ? m : 0ull;
        q1 |= (o & 2) ? m : 0ull;
        q2 |= (o & 4) ? m : 0ull;
        q3 |= (o & 8) ? m : 0ull;
      }
      if (f.final) miss = ~a.seen[v] & set;
    }
    const uint64_t wr = got | miss;
    uint64_t all = wave_or_all(wr);
    while (all) {
      const int i = __ffsll(static_cast<long long>(all)) - 1;
      all &= all - 1;
      if ((wr >> i) & 1ull) {
        const int32_t d = ((miss >> i) & 1ull)
                              ? -1
                              : f.jlo + int32_t((q0 >> i) & 1ull) +
                                    (int32_t((q1 >> i) & 1ull) << 1) +
                                    (int32_t((q2 >> i) & 1ull) << 2) +
                                    (int32_t((q3 >> i) & 1ull) << 3) - f.start[i];
        f.res[i][v] = d;
      }
    }
  }
}

// Lists the frontier vertices of a top-down level and clears next (the
// scatter ORs into it; a later kernel, so the clear is complete by then).
__global__ void k_lv_td_list(MsLevel a) {
  for (int64_t v0 = int64_t(blockIdx.x) * blockDim.x; v0 < a.n;
       v0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t v = v0 + threadIdx.x;
    const bool f = v < a.n && a.fcur[v] != 0;
    if (v < a.n) a.fnext[v] = 0;
    const int64_t pos = wave_append(f, &a.ctl[2]);
    if (f) a.tdlist[pos] = int32_t(v);
  }
}

__global__ void __launch_bounds__(1024) k_lv_td_scan(MsLevel a) {
  __shared__ unsigned long long sh[16];
  const int64_t cnt = int64_t(a.ctl[2]);
  unsigned long long carry = 0;
  for (int64_t i0 = 0; i0 < cnt; i0 += blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    unsigned long long dg = 0;
    if (i < cnt) {
      const int32_t v = a.tdlist[i];
      dg = (unsigned long long)(a.off[v + 1] - a.off[v]);
    }
    const unsigned long long incl = wave_incl_scan(dg);
    if (lane_id() == kWave - 1) sh[threadIdx.x / kWave] = incl;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
    for (int j = 0; j < int(blockDim.x / kWave); ++j) {
      before += j < int(threadIdx.x / kWave) ? sh[j] : 0ull;
      tot += sh[j];
    }
    if (i < cnt) a.tdscan[i] = int64_t(carry + before + incl - dg);
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) a.tdscan[cnt] = int64_t(carry);
}

__global__ void k_lv_td_expand(MsLevel a) {
  const int64_t cnt = int64_t(a.ctl[2]);
  const int64_t E = a.tdscan[cnt];
  unsigned long long edges = 0;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < E;
       e += int64_t(gridDim.x) * blockDim.x) {
    int64_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (a.tdscan[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int32_t v = a.tdlist[lo];
    const int32_t w = a.col[a.off[v] + (e - a.tdscan[lo])];
    ++edges;
    // lanes already in next (a possibly stale read: the atomic decides) need
    // no atomic
    const uint64_t m = a.fcur[v] & ~a.seen[w] & ~a.fnext[w];
    if (m) atomicOr(reinterpret_cast<unsigned long long *>(&a.fnext[w]), m);
  }
  lv_flush(a, 0, 0, edges);
}

// Close of a top-down level: fold next into seen (the scatter only set lanes
// that were unseen, and seen did not change during it, so next is all new).
__global__ void k_lv_td_close(MsLevel a) {
  const int64_t nthreads = int64_t(gridDim.x) * blockDim.x;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t iters = (int64_t(a.n) + nthreads - 1) / nthreads;
  unsigned long long act = 0;
  uint64_t lor = 0;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t v = tid + it * nthreads;
    if (v < a.n) {
      const uint64_t nw = a.fnext[v];
      if (nw) {
        a.seen[v] |= nw;
        ++act;
        lor |= nw;
      }
    }
  }
  lv_flush(a, act, lor, 0);
}

__global__ void __launch_bounds__(256) k_lv_bu(MsLevel a) {
  __shared__ BuRows<1> s_rows[4];
  const int64_t nthreads = int64_t(gridDim.x) * blockDim.x;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t iters = (int64_t(a.n) + nthreads - 1) / nthreads;
  const int l = lane_id(), wv = threadIdx.x / kWave;
  unsigned long long act = 0, edges = 0;
  uint64_t lor = 0;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t w = tid + it * nthreads;
    bool valid = w < a.n;
    uint64_t s0 = 0, want = 0;
    if (valid) {
      if (a.off[w + 1] - a.off[w] > kHub) {
        valid = false;
      } else {
        s0 = a.seen[w];
        want = ~s0 & a.live;
      }
    }
    const uint64_t nw =
        bu_wave<1>(a.off, a.col, reinterpret_cast<const LaneSet<1> *>(a.fcur), nullptr,
                   INT32_MAX, w, LaneSet<1>{{want}}, s_rows[wv], edges)
            .w[0];
    if (valid) {
      if (nw) a.seen[w] = s0 | nw;
      a.fnext[w] = nw;
      act += nw != 0;
      lor |= nw;
    }
  }
  const int64_t wid = tid / kWave, nwaves = nthreads / kWave;
  // hubs, 64 per wave step: lanes close those that want nothing, the wave
  // scans the rows of the others one at a time
  for (int64_t h0 = wid * kWave; h0 < a.nhubs; h0 += nwaves * kWave) {
    const int64_t hl = h0 + l;
    bool need = false;
    if (hl < a.nhubs) {
      const int32_t wl = a.hubs[hl];
      need = (~a.seen[wl] & a.live) != 0;
      if (!need) a.fnext[wl] = 0;
    }
    for (uint64_t todo = __ballot(need); todo; todo &= todo - 1) {
      const int32_t w = a.hubs[h0 + __builtin_ctzll(todo)];
      const uint64_t s0 = a.seen[w];
      const uint64_t want = ~s0 & a.live;
      uint64_t nw = 0;
      {
        const int64_t p1 = a.off[w + 1];
        uint64_t acc = 0;
        for (int64_t p = a.off[w]; p < p1; p += kWave) {
          const uint64_t x = p + l < p1 ? a.fcur[a.col[p + l]] : 0ull;
          acc |= wave_or(x);
          if (l == 0) edges += uint64_t(min<int64_t>(kWave, p1 - p));
          if ((acc & want) == want) break;
        }
        nw = acc & want;
      }
      if (l == 0) {
        if (nw) a.seen[w] = s0 | nw;
        a.fnext[w] = nw;
        act += nw != 0;
        lor |= nw;
      }
    }
  }
  lv_flush(a, act, lor, edges);
}

}  // namespace

// Host side of one level for the server. ws must have 64 lanes. `live` are
// the lanes with a non-empty frontier; L is the level (ring slot L is its
// frontier, slot L + 1 receives the next). After the call (asynchronous on s)
// ctl[0] holds the next frontier's vertex count, ctl[1] its lanes. Returns
// the direction used (0 top-down, 1 up).
static MsLevel level_args(const Graph *g, Workspace *ws, int32_t L, unsigned long long *ctl) {
  MsState *st = reinterpret_cast<MsState *>(ws->ms_state);
  MsLevel a{};
  a.off = g->poff.as<int64_t>();
  a.col = g->pcol.as<int32_t>();
  a.n = g->n;
  a.seen = st->lvseen.as<uint64_t>();
  a.ring = st->lvring.as<uint64_t>();
  a.fcur = a.ring + int64_t(L & (kRing - 1)) * g->n;
  a.fnext = a.ring + int64_t((L + 1) & (kRing - 1)) * g->n;
  a.tdlist = ws->dlen.as<int32_t>();
  a.tdscan = ws->dscan.as<int64_t>();
  a.hubs = st->hubs.as<int32_t>();
  a.nhubs = st->nhubs;
  a.ctl = ctl;
  return a;
}

int ms_level(const Graph *g, Workspace *ws, uint64_t live, int64_t active, int32_t bu_permille,
             int32_t L, unsigned long long *ctl, hipStream_t s) {
  MsLevel a = level_args(g, ws, L, ctl);
  a.live = live;
  const int SG = device_cus() * 8;
  // ctl starts at zero: cleared by the previous level's publishing flush (or
  // at set-up)
  const bool td = active <= int64_t(g->n) * bu_permille / 1000;
  if (td) {
    hipLaunchKernelGGL(k_lv_td_list, dim3(grid_for(g->n, 256, SG)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_lv_td_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_lv_td_expand, dim3(SG), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_lv_td_close, dim3(grid_for(g->n, 256, SG)), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_lv_bu, dim3(grid_for(g->n, 256, SG)), dim3(256), 0, s, a);
  }
  HIPCHK(hipGetLastError());
  return td ? 0 : 1;
}

// Writes result rows from the level ring (k_lv_flush); ctl is the level's
// control block (read for `final`). With host_ctl, also publishes ctl there
// and clears next_ctl (see k_lv_flush).
void ms_level_flush(const Graph *g, Workspace *ws, const LaneFlush &f, unsigned long long *ctl,
                    unsigned long long *next_ctl, unsigned long long *host_ctl, hipStream_t s) {
  if (f.jhi - f.jlo >= kRing || f.jhi < f.jlo)
    fail(DSBFS_ERR_DEVICE, "server level flush window outside the ring");
  MsLevel a = level_args(g, ws, f.jhi, ctl);
  const int SG = device_cus() * 8;
  hipLaunchKernelGGL(k_lv_flush, dim3(grid_for(g->n, 256, SG)), dim3(256), 0, s, a, f, next_ctl,
                     host_ctl);
  HIPCHK(hipGetLastError());
}

// Levels a lane may keep unwritten in the ring before its rows must be
// flushed (the ring holds kRing levels; one slot receives the next level).
int ms_level_ring() { return kRing; }

// Device bytes held by the multi-source state of a workspace.
size_t ms_state_bytes(const Workspace *ws) {
  const MsState *st = reinterpret_cast<const MsState *>(ws->ms_state);
  if (!st) return 0;
  const DevBuf *b[] = {&st->ctl, &st->srcs, &st->hubs, &st->ring, &st->seen,
                       &st->hub_idx, &st->col2, &st->hot, &st->lvring, &st->lvseen};
  size_t t = 0;
  for (const DevBuf *x : b) t += x->p ? x->bytes : 0;
  return t;
}

// Prepares a 64-lane workspace for level-at-a-time use (hub list, state).
void ms_level_prepare(const Graph *g, Workspace *ws, hipStream_t s) {
  if (ws->max_lanes != 64) fail(DSBFS_ERR_INVALID_ARG, "workspace was created without lanes");
  if (!g->pcol.p && g->m > 0) fail(DSBFS_ERR_INVALID_ARG, "batched serving needs the plain CSR");
  if (!ws->ms_state) ws->ms_state = new MsState();
  MsState *st = reinterpret_cast<MsState *>(ws->ms_state);
  const Alloc *al = &g->al;
  if (st->nhubs < 0) {
    DevBuf flag, tmp, cnt;
    flag.alloc(al, size_t(g->n), s);
    tmp.alloc(al, compact_tmp_bytes(g->n), s);
    cnt.alloc(al, 8, s);
    st->hubs.alloc(al, size_t(g->n) * 4, s);
    hipLaunchKernelGGL(k_flag_hub, dim3(grid_for(g->n, 256, 8192)), dim3(256), 0, s,
                       g->poff.as<int64_t>(), g->n, flag.as<uint8_t>());
    HIPCHK(hipGetLastError());
    compact_flags_u8(flag.as<uint8_t>(), g->n, st->hubs.as<int32_t>(), cnt.as<int64_t>(), tmp.p,
                     s);
    st->nhubs = d2h_scalar(cnt.as<int64_t>(), s);
  }
  const int64_t n = g->n;
  if (!st->lvring.p) st->lvring.alloc(al, size_t(kRing) * size_t(n) * 8, s);
  if (!st->lvseen.p) st->lvseen.alloc(al, size_t(n) * 8, s);
  HIPCHK(hipMemsetAsync(st->lvseen.p, 0, size_t(n) * 8, s));
  HIPCHK(hipMemsetAsync(st->lvring.p, 0, size_t(kRing) * size_t(n) * 8, s));
}

// Admission at level L: clears the lanes in `clear` and seeds the lanes in
// seed_mask at seeds.src[i].
void ms_level_recycle(const Graph *g, Workspace *ws, int32_t L, uint64_t clear, uint64_t seed_mask,
                      const SeedList &seeds, hipStream_t s) {
  MsLevel a = level_args(g, ws, L, nullptr);
  const int SG = device_cus() * 8;
  if (clear)
    hipLaunchKernelGGL(k_lv_recycle, dim3(grid_for(g->n, 256, SG)), dim3(256), 0, s, a, clear);
  if (seed_mask) hipLaunchKernelGGL(k_lv_seed, dim3(1), dim3(64), 0, s, a, seed_mask, seeds);
  HIPCHK(hipGetLastError());
}

}  // namespace dsbfs
