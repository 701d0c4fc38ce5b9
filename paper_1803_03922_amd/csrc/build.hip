// Graph construction on the device.
//
// Edge list -> simple symmetric graph (edge doubling, Section VI-A; symmetric
// graph assumption, Section II-A; self-loops and duplicates dropped) ->
// plain CSR -> degree separation at TH (Section III-A: delegate iff degree >
// TH; delegates renumbered in ascending vertex ID, Fig. 2 caption) -> the
// four subgraphs (Section III-C) stored as two row sets with packed offsets:
//   normal row v   = [nn neighbours (vertex IDs) | nd neighbours (delegate IDs)]
//   delegate row k = [dd neighbours (delegate IDs) | dn neighbours (vertex IDs)]
// and the source list of nd plus the source masks of dd and dn (Section IV-B).
//
// At one GPU every vertex is local, so nn columns are 32-bit vertex IDs too
// (the paper keeps them 64-bit only because they may be remote), and the
// offsets are 64-bit because one GPU holds more than 2^32 edges at scale 26.
#include <algorithm>

#include "internal.hpp"

namespace dsbfs {

namespace {

constexpr int kBS = 256;

__global__ void k_validate(const int32_t *src, const int32_t *dst, int64_t g, int32_t n,
                           unsigned long long *ctr /* [0] bad, [1] non-loop */) {
  unsigned long long bad = 0, keep = 0;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < g;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int32_t u = src[e], v = dst[e];
    if (u < 0 || u >= n || v < 0 || v >= n) ++bad;
    else if (u != v) ++keep;
  }
  bad = wave_sum(bad);
  keep = wave_sum(keep);
  if (lane_id() == 0) {
    if (bad) atomicAdd(&ctr[0], bad);
    if (keep) atomicAdd(&ctr[1], keep);
  }
}

// Both directions of every non-loop pair as 64-bit keys (u << B) | v.
__global__ void k_pack(const int32_t *src, const int32_t *dst, int64_t g, int B, uint64_t *keys,
                       unsigned long long *cursor) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e0 = int64_t(blockIdx.x) * blockDim.x; e0 < g; e0 += stride) {
    const int64_t e = e0 + threadIdx.x;
    int32_t u = 0, v = 0;
    bool keep = false;
    if (e < g) {
      u = src[e];
      v = dst[e];
      keep = u != v;
    }
    const int64_t pos = wave_append(keep, cursor);
    if (keep) {
      keys[2 * pos] = (uint64_t(uint32_t(u)) << B) | uint64_t(uint32_t(v));
      keys[2 * pos + 1] = (uint64_t(uint32_t(v)) << B) | uint64_t(uint32_t(u));
    }
  }
}

// poff[x] = index of the first key with row >= x, for x in [0, n]: between
// consecutive keys j-1 and j every row in (row[j-1], row[j]] starts at j.
__global__ void k_row_offsets(const uint64_t *keys, int64_t m, int B, int32_t n, int64_t *poff) {
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j <= m;
       j += int64_t(gridDim.x) * blockDim.x) {
    const int64_t prev = j > 0 ? int64_t(keys[j - 1] >> B) : -1;
    const int64_t cur = j < m ? int64_t(keys[j] >> B) : int64_t(n);
    for (int64_t x = prev + 1; x <= cur; ++x) poff[x] = j;
  }
}

__global__ void k_cols_and_degree(const uint64_t *keys, int64_t m, uint64_t vmask,
                                  const int64_t *poff, int32_t n, int32_t *pcol, int32_t *deg) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < m; j += stride)
    pcol[j] = int32_t(keys[j] & vmask);
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += stride)
    deg[v] = int32_t(poff[v + 1] - poff[v]);
}

__global__ void k_flag_gt(const int32_t *deg, int32_t n, int32_t th, uint8_t *flag) {
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x)
    flag[v] = deg[v] > th;
}

__global__ void k_fill_i32(int32_t *p, int64_t N, int32_t val) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = val;
}

__global__ void k_did_scatter(const int32_t *vid_of, int32_t d, int32_t *did) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < d;
       k += int64_t(gridDim.x) * blockDim.x)
    did[vid_of[k]] = int32_t(k);
}

// cnt_del[u] = number of delegate neighbours of u. Edge-parallel over the
// sorted keys; rows are contiguous, so a segmented wave scan by row folds a
// hub's entries into one atomic per wave.
__global__ void k_count_delegate_nbrs(const uint64_t *keys, int64_t m, int B, uint64_t vmask,
                                      const int32_t *did, int32_t *cnt_del) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int l = lane_id();
  for (int64_t j0 = int64_t(blockIdx.x) * blockDim.x; j0 < m; j0 += stride) {
    const int64_t j = j0 + threadIdx.x;
    int64_t u = -1 - l;  // distinct per inactive lane: never merges
    int32_t c = 0;
    if (j < m) {
      const uint64_t k = keys[j];
      u = int64_t(k >> B);
      c = did[int32_t(k & vmask)] >= 0;
    }
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t uo = __shfl_up(u, o, kWave);
      const int32_t co = __shfl_up(c, o, kWave);
      if (l >= o && uo == u) c += co;
    }
    const int64_t un = __shfl_down(u, 1, kWave);
    const bool tail = (l == kWave - 1) || un != u;
    if (j < m && tail && c) atomicAdd(&cnt_del[u], c);
  }
}

__global__ void k_row_lengths(const int32_t *deg, const int32_t *did, const int32_t *vid_of,
                              int32_t n, int32_t d, int32_t *nlen, int32_t *dlen) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += stride)
    nlen[v] = did[v] < 0 ? deg[v] : 0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < d; k += stride)
    dlen[k] = deg[vid_of[k]];
}

__global__ void k_pack_offsets(const int64_t *nstart, const int64_t *dstart, const int32_t *deg,
                               const int32_t *did, const int32_t *vid_of, const int32_t *cnt_del,
                               int32_t n, int32_t d, uint64_t *noff, uint64_t *doff) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v <= n; v += stride) {
    uint64_t first = 0;
    if (v < n && did[v] < 0) first = uint64_t(deg[v] - cnt_del[v]);  // nn part
    noff[v] = uint64_t(nstart[v]) | (first << kOffShift);
  }
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k <= d; k += stride) {
    uint64_t first = k < d ? uint64_t(cnt_del[vid_of[k]]) : 0;      // dd part
    doff[k] = uint64_t(dstart[k]) | (first << kOffShift);
  }
}

// Compact part lengths of the normal rows (see Graph::nlen).
__global__ void k_pack_lens(const int32_t *deg, const int32_t *did, const int32_t *cnt_del,
                            int32_t n, uint16_t *nlen) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += stride) {
    uint16_t x = 0;
    if (did[v] < 0) {
      const int32_t nd = cnt_del[v], nn = deg[v] - nd;
      x = (nn < 255 && nd < 255) ? uint16_t(nn | (nd << 8)) : kLenWide;
    }
    nlen[v] = x;
  }
}

// nn length of every vertex (0 for a delegate): the part sizes of the
// compact nn copy.
__global__ void k_nn_counts(const int32_t *deg, const int32_t *did, const int32_t *cnt_del,
                            int32_t n, int32_t *cnt) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += stride)
    cnt[v] = did[v] < 0 ? deg[v] - cnt_del[v] : 0;
}

// Copies the nn part of every normal row (its first part) to its place in
// the compact nn copy and records where it starts.
__global__ void k_nn_fill(const int64_t *start, const int32_t *cnt, const uint64_t *noff,
                          const int32_t *ncol, int32_t n, uint32_t *nnoff, int32_t *nncol) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t o = start[v];
    nnoff[v] = uint32_t(o);
    const int32_t c = cnt[v];
    if (c > 0) {
      const int64_t b = row_start(noff[v]);
      for (int32_t j = 0; j < c; ++j) nncol[o + j] = ncol[b + j];
    }
  }
}

// Destination of row u in the new layout: (row offsets, columns, is delegate).
struct RowDst {
  uint64_t w;
  int32_t *col;
  bool del;
};

__device__ __forceinline__ RowDst row_dst(int32_t u, const int32_t *did, const uint64_t *noff,
                                          int32_t *ncol, const uint64_t *doff, int32_t *dcol) {
  const int32_t k = did[u];
  if (k >= 0) return RowDst{doff[k], dcol, true};
  return RowDst{noff[u], ncol, false};
}

// Rows with at most kSmallRow entries: one thread walks the row in order.
constexpr int kSmallRow = 64;

__global__ void k_split_small(const int64_t *poff, const int32_t *pcol, const int32_t *did,
                              int32_t n, const uint64_t *noff, int32_t *ncol,
                              const uint64_t *doff, int32_t *dcol) {
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
       u += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = poff[u], e = poff[u + 1];
    if (e - b == 0 || e - b > kSmallRow) continue;
    const RowDst r = row_dst(int32_t(u), did, noff, ncol, doff, dcol);
    int64_t pa = row_start(r.w), pb = pa + row_first(r.w);
    for (int64_t j = b; j < e; ++j) {
      const int32_t v = pcol[j];
      const int32_t kv = did[v];
      const bool v_del = kv >= 0;
      // first part: same class as the row for delegates (dd), opposite-of-delegate
      // for normals (nn); columns of delegate neighbours are delegate IDs.
      const bool first = r.del ? v_del : !v_del;
      const int32_t val = v_del ? kv : v;
      if (first) r.col[pa++] = val;
      else r.col[pb++] = val;
    }
  }
}

// Rows with more than kSmallRow entries: one wave per row, 64 entries per step,
// order kept by ballot ranks.
__global__ void k_split_large(const int32_t *rows, const int64_t *nrows, const int64_t *poff,
                              const int32_t *pcol, const int32_t *did, const uint64_t *noff,
                              int32_t *ncol, const uint64_t *doff, int32_t *dcol) {
  const int64_t R = *nrows;
  const int l = lane_id();
  const int64_t wid = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * blockDim.x / kWave;
  for (int64_t i = wid; i < R; i += nw) {
    const int32_t u = rows[i];
    const int64_t b = poff[u], e = poff[u + 1];
    const RowDst r = row_dst(u, did, noff, ncol, doff, dcol);
    int64_t pa = row_start(r.w), pb = pa + row_first(r.w);
    for (int64_t j0 = b; j0 < e; j0 += kWave) {
      const int64_t j = j0 + l;
      const bool ok = j < e;
      int32_t v = 0, kv = -1;
      if (ok) {
        v = pcol[j];
        kv = did[v];
      }
      const bool v_del = kv >= 0;
      const bool first = r.del ? v_del : !v_del;
      const uint64_t ma = __ballot(ok && first), mb = __ballot(ok && !first);
      const int32_t val = v_del ? kv : v;
      if (ok && first) r.col[pa + lanes_below(ma)] = val;
      if (ok && !first) r.col[pb + lanes_below(mb)] = val;
      pa += __popcll(ma);
      pb += __popcll(mb);
    }
  }
}

__global__ void k_flag_large(const int64_t *poff, int32_t n, uint8_t *flag) {
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
       u += int64_t(gridDim.x) * blockDim.x)
    flag[u] = poff[u + 1] - poff[u] > kSmallRow;
}

__global__ void k_flag_ndsrc(const int32_t *did, const int32_t *cnt_del, int32_t n, uint8_t *flag) {
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
       u += int64_t(gridDim.x) * blockDim.x)
    flag[u] = did[u] < 0 && cnt_del[u] > 0;
}

// Normal vertices with a normal neighbour (bottom-up nn candidates).
__global__ void k_flag_nnsrc(const int32_t *deg, const int32_t *did, const int32_t *cnt_del,
                             int32_t n, uint8_t *flag) {
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
       u += int64_t(gridDim.x) * blockDim.x)
    flag[u] = did[u] < 0 && deg[u] > cnt_del[u];
}

__global__ void k_source_masks(const int32_t *vid_of, const int32_t *deg, const int32_t *cnt_del,
                               int32_t d, uint32_t *ddm, uint32_t *dnm) {
  const int32_t W = (d + 31) / 32;
  for (int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < W;
       w += int64_t(gridDim.x) * blockDim.x) {
    uint32_t a = 0, b = 0;
    for (int i = 0; i < 32; ++i) {
      const int64_t k = w * 32 + i;
      if (k >= d) break;
      const int32_t u = vid_of[k];
      if (cnt_del[u] > 0) a |= 1u << i;
      if (deg[u] - cnt_del[u] > 0) b |= 1u << i;
    }
    ddm[w] = a;
    dnm[w] = b;
  }
}

__global__ void k_nds_len(const int32_t *ndsrc, int64_t cnt, const int32_t *cnt_del,
                          int32_t *len) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x)
    len[i] = cnt_del[ndsrc[i]];
}

// Copies the nd part of row ndsrc[i] to row i of the source-list-ordered copy,
// and its first entry (delegate ID, then that delegate's vertex) to pair i of
// nds_first, the dense array a bottom-up pass probes first.
__global__ void k_nds_fill(const int32_t *ndsrc, int64_t cnt, const uint64_t *noff,
                           const int32_t *ncol, const int32_t *vid_of, const int64_t *nds_off,
                           int32_t *nds_col, int32_t *nds_first) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t v = ndsrc[i];
    const uint64_t w0 = noff[v];
    const int64_t from = row_start(w0) + row_first(w0);
    const int64_t to = nds_off[i], len = nds_off[i + 1] - to;
    for (int64_t j = 0; j < len; ++j) nds_col[to + j] = ncol[from + j];
    // rows of the list are never empty
    nds_first[2 * i] = ncol[from];
    nds_first[2 * i + 1] = vid_of[ncol[from]];
  }
}

// [0] e_nn [1] e_nd [2] e_dn [3] e_dd [4] n_ndsrc [5] n_ddsrc [6] n_dnsrc [7] max degree
__global__ void k_stats(const int32_t *deg, const int32_t *did, const int32_t *cnt_del, int32_t n,
                        unsigned long long *out) {
  unsigned long long a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long mx = 0;
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
       u += int64_t(gridDim.x) * blockDim.x) {
    const unsigned long long dg = deg[u], cd = cnt_del[u], cn = dg - cd;
    if (did[u] < 0) {
      a[0] += cn; a[1] += cd; a[4] += cd > 0; a[7] += cn > 0;
    } else {
      a[2] += cn; a[3] += cd; a[5] += cd > 0; a[6] += cn > 0;
    }
    mx = dg > mx ? dg : mx;
  }
  for (int i = 0; i < 8; ++i) {
    unsigned long long s = wave_sum(a[i]);
    // out[7] is the maximum degree; the count of normals with an nn edge is out[8]
    if (lane_id() == 0 && s) atomicAdd(&out[i < 7 ? i : 8], s);
  }
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long t = __shfl_xor(mx, o, kWave);
    mx = t > mx ? t : mx;
  }
  if (lane_id() == 0) atomicMax(&out[7], mx);
}

int bits_for(int64_t n) {
  int B = 1;
  while ((int64_t(1) << B) < n) ++B;
  return B;
}

// Degree bucket of a vertex on a log scale (8 buckets per power of two), so
// that sorting by bucket orders neighbours by degree with a short key.
__device__ __forceinline__ uint32_t deg_bucket(int32_t deg) {
  if (deg <= 1) return 0;
  const uint32_t lg = 31u - __clz(uint32_t(deg));          // floor(log2)
  const uint32_t frac = lg >= 3 ? (uint32_t(deg) >> (lg - 3)) & 7u : (uint32_t(deg) << (3 - lg)) & 7u;
  const uint32_t b = lg * 8u + frac;
  return b > 255u ? 255u : b;
}

// Keys of every dd entry: (row k, 255 - degree bucket of the neighbour,
// neighbour delegate ID), so one radix sort orders each dd part by
// neighbour degree, highest first (ties by ID). One wave per row.
__global__ void k_dd_keys(const uint64_t *doff, const int32_t *dcol, const int64_t *ddpre,
                          const int32_t *vid_of, const int32_t *deg, int32_t d, int Bd,
                          uint64_t *keys) {
  const int l = lane_id();
  const int64_t wid = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * blockDim.x / kWave;
  for (int64_t k = wid; k < d; k += nw) {
    const uint64_t w = doff[k];
    const int64_t beg = row_start(w), len = row_first(w);
    const int64_t out = ddpre[k];
    for (int64_t j = l; j < len; j += kWave) {
      const int32_t x = dcol[beg + j];
      const uint64_t b = 255u - deg_bucket(deg[vid_of[x]]);
      keys[out + j] = (uint64_t(k) << (Bd + 8)) | (b << Bd) | uint64_t(uint32_t(x));
    }
  }
}

// Writes the sorted dd entries back into their rows.
__global__ void k_dd_back(const uint64_t *keys, int64_t e_dd, const uint64_t *doff,
                          const int64_t *ddpre, int Bd, int32_t *dcol) {
  const uint64_t xmask = (uint64_t(1) << Bd) - 1;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < e_dd;
       j += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t key = keys[j];
    const int64_t k = int64_t(key >> (Bd + 8));
    dcol[row_start(doff[k]) + (j - ddpre[k])] = int32_t(key & xmask);
  }
}

// Keys of every plain-CSR entry: (row, 255 - degree bucket of the
// neighbour, position in the row). Rows are ascending by neighbour ID, so a
// stable sort on the row and bucket bits orders each row by neighbour degree,
// highest first, ties by ascending ID. One wave per row.
__global__ void k_plain_keys(const int64_t *poff, const int32_t *pcol, const int32_t *deg,
                             int32_t n, uint64_t *keys) {
  const int l = lane_id();
  const int64_t wid = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * blockDim.x / kWave;
  for (int64_t v = wid; v < n; v += nw) {
    const int64_t beg = poff[v], len = poff[v + 1] - beg;
    for (int64_t j = l; j < len; j += kWave) {
      const uint64_t b = 255u - deg_bucket(deg[pcol[beg + j]]);
      keys[beg + j] = (uint64_t(v) << 32) | (b << 24) | uint64_t(j);
    }
  }
}

// Rebuilds the columns in key order (each row keeps its range).
__global__ void k_plain_back(const uint64_t *keys, int64_t m, const int64_t *poff,
                             const int32_t *pcol, int32_t *out) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
       e += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t key = keys[e];
    out[e] = pcol[poff[int64_t(key >> 32)] + int64_t(key & 0xffffffu)];
  }
}

// First entry of every dd part (its highest-degree neighbour) and that
// neighbour's vertex, as a dense pair per delegate; (-1, -1) if the part is
// empty. The bottom-up dd visit probes it before walking the row.
__global__ void k_dd_first(const uint64_t *doff, const int32_t *dcol, const int32_t *vid_of,
                           int32_t d, int32_t *out) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < d;
       k += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t w = doff[k];
    const int32_t x = row_first(w) > 0 ? dcol[row_start(w)] : -1;
    out[2 * k] = x;
    out[2 * k + 1] = x >= 0 ? vid_of[x] : -1;
  }
}

__global__ void k_dd_len(const uint64_t *doff, int32_t d, int32_t *len) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < d;
       k += int64_t(gridDim.x) * blockDim.x)
    len[k] = int32_t(row_first(doff[k]));
}

// nd part of every normal row (at most a few dozen entries when TH is small):
// insertion sort by neighbour degree, highest first, ties by delegate ID.
// Parts longer than 64 entries keep ascending ID order.
__global__ void k_nd_sort(const uint64_t *noff, int32_t n, const int32_t *did, int32_t *ncol,
                          const int32_t *vid_of, const int32_t *deg) {
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    if (did[v] >= 0) continue;
    const uint64_t w0 = noff[v], w1 = noff[v + 1];
    const int64_t b = row_start(w0) + row_first(w0), e = row_start(w1);
    if (e - b < 2 || e - b > 64) continue;
    for (int64_t i = b + 1; i < e; ++i) {
      const int32_t x = ncol[i];
      const int32_t dx = deg[vid_of[x]];
      int64_t j = i - 1;
      while (j >= b) {
        const int32_t y = ncol[j];
        const int32_t dy = deg[vid_of[y]];
        if (dy > dx || (dy == dx && y < x)) break;
        ncol[j + 1] = y;
        --j;
      }
      ncol[j + 1] = x;
    }
  }
}

}  // namespace

int64_t rmat_pack_keys(const dsbfs_rmat_spec *sp, int B, uint64_t *keys, unsigned long long *cursor,
                       hipStream_t s);

// Builds the layout from an edge list (src, dst: g pairs), or, with rmat
// set, from the RMAT generator writing the symmetrized keys directly.
Graph *graph_create(const int32_t *src, const int32_t *dst, int64_t g, int32_t n,
                    const dsbfs_build_opts *opts, const dsbfs_allocator *alloc, hipStream_t s,
                    const dsbfs_rmat_spec *rmat) {
  if (rmat) {
    if (rmat->scale < 1 || rmat->scale > 31)
      fail(DSBFS_ERR_INVALID_ARG, "scale must be in [1, 31]");
    if (rmat->scale == 31) fail(DSBFS_ERR_RANGE, "2^31 vertices do not fit int32 IDs");
    n = int32_t(int64_t(1) << rmat->scale);
    g = rmat->num_edges;
    src = dst = nullptr;
  }
  if (n < 1) fail(DSBFS_ERR_INVALID_ARG, "num_vertices must be >= 1");
  if (g < 0) fail(DSBFS_ERR_INVALID_ARG, "num_edges must be >= 0");
  if (g > 0 && !rmat && (!src || !dst)) fail(DSBFS_ERR_INVALID_ARG, "src/dst must not be NULL");
  dsbfs_build_opts o{};
  o.threshold = 32;
  o.keep_plain_csr = 1;
  if (opts) o = *opts;
  if (o.threshold < 0) fail(DSBFS_ERR_INVALID_ARG, "threshold must be >= 0");
  if (o.skip_nn_copy != 0 && o.skip_nn_copy != 1)
    fail(DSBFS_ERR_INVALID_ARG, "skip_nn_copy must be 0 or 1");
  if (g > (int64_t(1) << 38)) fail(DSBFS_ERR_RANGE, "too many edges for the packed offsets");

  Graph *G = new Graph();
  try {
    if (alloc && alloc->alloc && alloc->free) {
      G->al.a = *alloc;
      G->al.custom = true;
    }
    HIPCHK(hipGetDevice(&G->device));
    G->stream = s;
    G->n = n;
    G->TH = o.threshold;
    const Alloc *al = &G->al;
    const int B = bits_for(n);
    const uint64_t vmask = (uint64_t(1) << B) - 1;

    // 1. edges on the device, validated (or generated: step 2)
    DevBuf esrc, edst;
    const int32_t *ds = src, *dd = dst;
    if (!rmat && !o.edges_on_device && g > 0) {
      esrc.alloc(al, size_t(g) * 4, s);
      edst.alloc(al, size_t(g) * 4, s);
      HIPCHK(hipMemcpyAsync(esrc.p, src, size_t(g) * 4, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(edst.p, dst, size_t(g) * 4, hipMemcpyHostToDevice, s));
      ds = esrc.as<int32_t>();
      dd = edst.as<int32_t>();
    }
    DevBuf ctr;
    ctr.alloc(al, 16 * sizeof(unsigned long long), s);
    HIPCHK(hipMemsetAsync(ctr.p, 0, 16 * sizeof(unsigned long long), s));
    unsigned long long *c = ctr.as<unsigned long long>();
    int64_t M2 = 2 * g;   // upper bound for the generator (self-loops are dropped)
    if (!rmat) {
      if (g > 0) {
        hipLaunchKernelGGL(k_validate, dim3(grid_for(g, kBS, 8192)), dim3(kBS), 0, s, ds, dd, g,
                           n, c);
        HIPCHK(hipGetLastError());
      }
      unsigned long long hc[2];
      HIPCHK(hipMemcpyAsync(hc, c, sizeof(hc), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (hc[0]) fail(DSBFS_ERR_INVALID_ARG, "edge endpoint outside [0, num_vertices)");
      M2 = 2 * int64_t(hc[1]);
    }

    // 2. symmetrize into keys, sort, de-duplicate
    DevBuf keys, alt;
    keys.alloc(al, size_t(M2) * 8, s);
    alt.alloc(al, size_t(M2) * 8, s);
    if (rmat) {
      M2 = rmat_pack_keys(rmat, B, keys.as<uint64_t>(), c, s);
    } else if (M2 > 0) {
      HIPCHK(hipMemsetAsync(c, 0, sizeof(unsigned long long), s));
      hipLaunchKernelGGL(k_pack, dim3(grid_for(g, kBS, 8192)), dim3(kBS), 0, s, ds, dd, g, B,
                         keys.as<uint64_t>(), c);
      HIPCHK(hipGetLastError());
    }
    esrc.reset();
    edst.reset();
    int64_t m = 0;
    {
      DevBuf tmp;
      tmp.alloc(al, std::max(radix_tmp_bytes(M2), compact_tmp_bytes(M2)), s);
      radix_sort_u64(keys.as<uint64_t>(), alt.as<uint64_t>(), M2, 2 * B, tmp.p, s);
      int64_t *cnt = reinterpret_cast<int64_t *>(c + 2);
      unique_sorted_u64(keys.as<uint64_t>(), M2, alt.as<uint64_t>(), cnt, tmp.p, s);
      m = d2h_scalar(cnt, s);
    }
    keys.reset();
    G->m = m;
    const uint64_t *uk = alt.as<uint64_t>();

    // 3. plain CSR and degrees
    G->poff.alloc(al, size_t(n + 1) * 8, s);
    G->pcol.alloc(al, size_t(m) * 4, s);
    G->deg.alloc(al, size_t(n) * 4, s);
    hipLaunchKernelGGL(k_row_offsets, dim3(grid_for(m + 1, kBS, 16384)), dim3(kBS), 0, s, uk, m, B,
                       n, G->poff.as<int64_t>());
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_cols_and_degree, dim3(grid_for(std::max<int64_t>(m, n), kBS, 16384)),
                       dim3(kBS), 0, s, uk, m, vmask, G->poff.as<int64_t>(), n,
                       G->pcol.as<int32_t>(), G->deg.as<int32_t>());
    HIPCHK(hipGetLastError());

    // 4. degree separation: delegate iff degree > TH, IDs in ascending vertex ID
    DevBuf flag, tmp;
    flag.alloc(al, size_t(n), s);
    tmp.alloc(al, compact_tmp_bytes(n), s);
    G->vid_of.alloc(al, size_t(n) * 4, s);  // shrunk below once d is known
    G->did.alloc(al, size_t(n) * 4, s);
    hipLaunchKernelGGL(k_flag_gt, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                       G->deg.as<int32_t>(), n, o.threshold, flag.as<uint8_t>());
    HIPCHK(hipGetLastError());
    int64_t *cnt = reinterpret_cast<int64_t *>(c + 2);
    compact_flags_u8(flag.as<uint8_t>(), n, G->vid_of.as<int32_t>(), cnt, tmp.p, s);
    const int64_t d = d2h_scalar(cnt, s);
    G->d = int32_t(d);
    {
      DevBuf v2;
      v2.alloc(al, size_t(d) * 4, s);
      if (d > 0)
        HIPCHK(hipMemcpyAsync(v2.p, G->vid_of.p, size_t(d) * 4, hipMemcpyDeviceToDevice, s));
      G->vid_of = std::move(v2);
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                       G->did.as<int32_t>(), int64_t(n), -1);
    HIPCHK(hipGetLastError());
    if (d > 0) {
      hipLaunchKernelGGL(k_did_scatter, dim3(grid_for(d, kBS, 8192)), dim3(kBS), 0, s,
                         G->vid_of.as<int32_t>(), int32_t(d), G->did.as<int32_t>());
      HIPCHK(hipGetLastError());
    }

    // 5. delegate neighbours per row
    DevBuf cnt_del;
    cnt_del.alloc(al, size_t(n) * 4, s);
    HIPCHK(hipMemsetAsync(cnt_del.p, 0, size_t(n) * 4, s));
    if (m > 0) {
      hipLaunchKernelGGL(k_count_delegate_nbrs, dim3(grid_for(m, kBS, 16384)), dim3(kBS), 0, s,
                         uk, m, B, vmask, G->did.as<int32_t>(), cnt_del.as<int32_t>());
      HIPCHK(hipGetLastError());
    }
    alt.reset();

    // 6. statistics (needed for sizes and the packed-offset range check)
    HIPCHK(hipMemsetAsync(c, 0, 9 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_stats, dim3(grid_for(n, kBS, 4096)), dim3(kBS), 0, s,
                       G->deg.as<int32_t>(), G->did.as<int32_t>(), cnt_del.as<int32_t>(), n, c);
    HIPCHK(hipGetLastError());
    unsigned long long hs[9];
    HIPCHK(hipMemcpyAsync(hs, c, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (int64_t(hs[7]) > kMaxFirstPart)
      fail(DSBFS_ERR_RANGE, "a vertex degree exceeds the packed row-offset limit (2^24-1)");

    // 7. row offsets of the two row sets
    {
      DevBuf nlen, dlen, nstart, dstart, stmp;
      nlen.alloc(al, size_t(n) * 4, s);
      dlen.alloc(al, size_t(d) * 4, s);
      nstart.alloc(al, size_t(n + 1) * 8, s);
      dstart.alloc(al, size_t(d + 1) * 8, s);
      stmp.alloc(al, scan_tmp_bytes(std::max<int64_t>(n, d)), s);
      hipLaunchKernelGGL(k_row_lengths, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                         G->deg.as<int32_t>(), G->did.as<int32_t>(), G->vid_of.as<int32_t>(), n,
                         int32_t(d), nlen.as<int32_t>(), dlen.as<int32_t>());
      HIPCHK(hipGetLastError());
      scan_excl_i32_to_i64(nlen.as<int32_t>(), nstart.as<int64_t>(), n, stmp.p, s);
      scan_excl_i32_to_i64(dlen.as<int32_t>(), dstart.as<int64_t>(), d, stmp.p, s);
      G->noff.alloc(al, size_t(n + 1) * 8, s);
      G->doff.alloc(al, size_t(d + 1) * 8, s);
      hipLaunchKernelGGL(k_pack_offsets, dim3(grid_for(n + 1, kBS, 8192)), dim3(kBS), 0, s,
                         nstart.as<int64_t>(), dstart.as<int64_t>(), G->deg.as<int32_t>(),
                         G->did.as<int32_t>(), G->vid_of.as<int32_t>(), cnt_del.as<int32_t>(), n,
                         int32_t(d), G->noff.as<uint64_t>(), G->doff.as<uint64_t>());
      HIPCHK(hipGetLastError());
      G->nlen.alloc(al, size_t(n) * 2, s);
      hipLaunchKernelGGL(k_pack_lens, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                         G->deg.as<int32_t>(), G->did.as<int32_t>(), cnt_del.as<int32_t>(), n,
                         G->nlen.as<uint16_t>());
      HIPCHK(hipGetLastError());
    }
    const int64_t e_nn = hs[0], e_nd = hs[1], e_dn = hs[2], e_dd = hs[3];
    G->ncol.alloc(al, size_t(e_nn + e_nd) * 4, s);
    G->dcol.alloc(al, size_t(e_dn + e_dd) * 4, s);

    // 8. scatter columns into the split rows
    hipLaunchKernelGGL(k_split_small, dim3(grid_for(n, kBS, 16384)), dim3(kBS), 0, s,
                       G->poff.as<int64_t>(), G->pcol.as<int32_t>(), G->did.as<int32_t>(), n,
                       G->noff.as<uint64_t>(), G->ncol.as<int32_t>(), G->doff.as<uint64_t>(),
                       G->dcol.as<int32_t>());
    HIPCHK(hipGetLastError());
    {
      DevBuf rows;
      rows.alloc(al, size_t(n) * 4, s);
      hipLaunchKernelGGL(k_flag_large, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                         G->poff.as<int64_t>(), n, flag.as<uint8_t>());
      HIPCHK(hipGetLastError());
      compact_flags_u8(flag.as<uint8_t>(), n, rows.as<int32_t>(), cnt, tmp.p, s);
      hipLaunchKernelGGL(k_split_large, dim3(2048), dim3(kBS), 0, s, rows.as<int32_t>(), cnt,
                         G->poff.as<int64_t>(), G->pcol.as<int32_t>(), G->did.as<int32_t>(),
                         G->noff.as<uint64_t>(), G->ncol.as<int32_t>(), G->doff.as<uint64_t>(),
                         G->dcol.as<int32_t>());
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
    }

    // 8a. compact copy of the nn parts (the forward nn visit's rows), while
    //     its 32-bit starts can address it
    if (e_nn < (int64_t(1) << 32) && !o.skip_nn_copy) {
      DevBuf cnt_nn, start, stmp;
      cnt_nn.alloc(al, size_t(n) * 4, s);
      start.alloc(al, size_t(n + 1) * 8, s);
      stmp.alloc(al, scan_tmp_bytes(n), s);
      hipLaunchKernelGGL(k_nn_counts, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                         G->deg.as<int32_t>(), G->did.as<int32_t>(), cnt_del.as<int32_t>(), n,
                         cnt_nn.as<int32_t>());
      HIPCHK(hipGetLastError());
      scan_excl_i32_to_i64(cnt_nn.as<int32_t>(), start.as<int64_t>(), n, stmp.p, s);
      G->nnoff.alloc(al, size_t(n) * 4, s);
      G->nncol.alloc(al, size_t(std::max<int64_t>(e_nn, 1)) * 4, s);
      hipLaunchKernelGGL(k_nn_fill, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                         start.as<int64_t>(), cnt_nn.as<int32_t>(), G->noff.as<uint64_t>(),
                         G->ncol.as<int32_t>(), n, G->nnoff.as<uint32_t>(),
                         G->nncol.as<int32_t>());
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
    }

    // 8b. delegate-neighbour parts ordered by neighbour degree, highest first:
    //     bottom-up scans meet frontier hubs early. (Order inside a part is
    //     free; the four subgraphs are unchanged.)
    if (d > 0 && e_dd > 1) {
      const int Bd = bits_for(d);
      DevBuf ddlen, ddpre, keys, alt2, stmp;
      ddlen.alloc(al, size_t(d) * 4, s);
      ddpre.alloc(al, size_t(d + 1) * 8, s);
      stmp.alloc(al, scan_tmp_bytes(d), s);
      hipLaunchKernelGGL(k_dd_len, dim3(grid_for(d, kBS, 4096)), dim3(kBS), 0, s,
                         G->doff.as<uint64_t>(), int32_t(d), ddlen.as<int32_t>());
      HIPCHK(hipGetLastError());
      scan_excl_i32_to_i64(ddlen.as<int32_t>(), ddpre.as<int64_t>(), d, stmp.p, s);
      keys.alloc(al, size_t(e_dd) * 8, s);
      alt2.alloc(al, size_t(e_dd) * 8, s);
      hipLaunchKernelGGL(k_dd_keys, dim3(4096), dim3(kBS), 0, s, G->doff.as<uint64_t>(),
                         G->dcol.as<int32_t>(), ddpre.as<int64_t>(), G->vid_of.as<int32_t>(),
                         G->deg.as<int32_t>(), int32_t(d), Bd, keys.as<uint64_t>());
      HIPCHK(hipGetLastError());
      {
        DevBuf rtmp;
        rtmp.alloc(al, radix_tmp_bytes(e_dd), s);
        // keys are written row by row with IDs ascending inside a row, so a
        // stable sort on the (row, bucket) fields alone keeps IDs ascending
        // among equal buckets
        radix_sort_u64_bits(keys.as<uint64_t>(), alt2.as<uint64_t>(), e_dd, Bd, 2 * Bd + 8,
                            rtmp.p, s);
      }
      hipLaunchKernelGGL(k_dd_back, dim3(grid_for(e_dd, kBS, 16384)), dim3(kBS), 0, s,
                         keys.as<uint64_t>(), e_dd, G->doff.as<uint64_t>(), ddpre.as<int64_t>(),
                         Bd, G->dcol.as<int32_t>());
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
    }
    G->dd_first.alloc(al, size_t(d) * 8, s);
    if (d > 0) {
      hipLaunchKernelGGL(k_dd_first, dim3(grid_for(d, kBS, 4096)), dim3(kBS), 0, s,
                         G->doff.as<uint64_t>(), G->dcol.as<int32_t>(), G->vid_of.as<int32_t>(),
                         int32_t(d), G->dd_first.as<int32_t>());
      HIPCHK(hipGetLastError());
    }
    if (d > 0 && e_nd > 1) {
      hipLaunchKernelGGL(k_nd_sort, dim3(grid_for(n, kBS, 16384)), dim3(kBS), 0, s,
                         G->noff.as<uint64_t>(), n, G->did.as<int32_t>(), G->ncol.as<int32_t>(),
                         G->vid_of.as<int32_t>(), G->deg.as<int32_t>());
      HIPCHK(hipGetLastError());
    }

    // 9. source list of nd, source masks of dd and dn
    hipLaunchKernelGGL(k_flag_ndsrc, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                       G->did.as<int32_t>(), cnt_del.as<int32_t>(), n, flag.as<uint8_t>());
    HIPCHK(hipGetLastError());
    G->ndsrc.alloc(al, size_t(hs[4]) * 4, s);
    compact_flags_u8(flag.as<uint8_t>(), n, G->ndsrc.as<int32_t>(), cnt, tmp.p, s);
    hipLaunchKernelGGL(k_flag_nnsrc, dim3(grid_for(n, kBS, 8192)), dim3(kBS), 0, s,
                       G->deg.as<int32_t>(), G->did.as<int32_t>(), cnt_del.as<int32_t>(), n,
                       flag.as<uint8_t>());
    HIPCHK(hipGetLastError());
    G->nnsrc.alloc(al, size_t(hs[8]) * 4, s);
    compact_flags_u8(flag.as<uint8_t>(), n, G->nnsrc.as<int32_t>(), cnt, tmp.p, s);
    {
      const int64_t nsrc = int64_t(hs[4]);
      DevBuf len, stmp;
      len.alloc(al, size_t(nsrc) * 4, s);
      stmp.alloc(al, scan_tmp_bytes(nsrc), s);
      G->nds_off.alloc(al, size_t(nsrc + 1) * 8, s);
      G->nds_col.alloc(al, size_t(e_nd) * 4, s);
      G->nds_first.alloc(al, size_t(nsrc) * 8, s);
      if (nsrc > 0) {
        hipLaunchKernelGGL(k_nds_len, dim3(grid_for(nsrc, kBS, 8192)), dim3(kBS), 0, s,
                           G->ndsrc.as<int32_t>(), nsrc, cnt_del.as<int32_t>(),
                           len.as<int32_t>());
        HIPCHK(hipGetLastError());
      }
      scan_excl_i32_to_i64(len.as<int32_t>(), G->nds_off.as<int64_t>(), nsrc, stmp.p, s);
      if (nsrc > 0) {
        hipLaunchKernelGGL(k_nds_fill, dim3(grid_for(nsrc, kBS, 16384)), dim3(kBS), 0, s,
                           G->ndsrc.as<int32_t>(), nsrc, G->noff.as<uint64_t>(),
                           G->ncol.as<int32_t>(), G->vid_of.as<int32_t>(),
                           G->nds_off.as<int64_t>(), G->nds_col.as<int32_t>(),
                           G->nds_first.as<int32_t>());
        HIPCHK(hipGetLastError());
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    G->ddsrc_mask.alloc(al, size_t(G->dwords()) * 4, s);
    G->dnsrc_mask.alloc(al, size_t(G->dwords()) * 4, s);
    if (d > 0) {
      hipLaunchKernelGGL(k_source_masks, dim3(grid_for(G->dwords(), kBS, 4096)), dim3(kBS), 0, s,
                         G->vid_of.as<int32_t>(), G->deg.as<int32_t>(), cnt_del.as<int32_t>(),
                         int32_t(d), G->ddsrc_mask.as<uint32_t>(), G->dnsrc_mask.as<uint32_t>());
      HIPCHK(hipGetLastError());
    }
    if (!o.keep_plain_csr) {
      G->poff.reset();
      G->pcol.reset();
    } else if (m > 1) {
      // Plain rows by neighbour degree, highest first: a bottom-up pass over
      // them (multi-source BFS, the query server) meets hubs first.
      DevBuf keys, alt, rtmp, col2;
      keys.alloc(al, size_t(m) * 8, s);
      alt.alloc(al, size_t(m) * 8, s);
      rtmp.alloc(al, radix_tmp_bytes(m), s);
      hipLaunchKernelGGL(k_plain_keys, dim3(8192), dim3(kBS), 0, s, G->poff.as<int64_t>(),
                         G->pcol.as<int32_t>(), G->deg.as<int32_t>(), n, keys.as<uint64_t>());
      HIPCHK(hipGetLastError());
      radix_sort_u64_bits(keys.as<uint64_t>(), alt.as<uint64_t>(), m, 24, 63, rtmp.p, s);
      alt.reset();
      rtmp.reset();
      col2.alloc(al, size_t(m) * 4, s);
      hipLaunchKernelGGL(k_plain_back, dim3(grid_for(m, kBS, 16384)), dim3(kBS), 0, s,
                         keys.as<uint64_t>(), m, G->poff.as<int64_t>(), G->pcol.as<int32_t>(),
                         col2.as<int32_t>());
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      std::swap(G->pcol, col2);
    }
    HIPCHK(hipStreamSynchronize(s));

    dsbfs_graph_stats &st = G->st;
    std::memset(&st, 0, sizeof(st));
    st.n = n;
    st.m_dir = m;
    st.d = d;
    st.e_nn = e_nn; st.e_nd = e_nd; st.e_dn = e_dn; st.e_dd = e_dd;
    st.n_ndsrc = hs[4]; st.n_ddsrc = hs[5]; st.n_dnsrc = hs[6];
    st.max_degree = hs[7];
    st.n_nnsrc = int64_t(hs[8]);
    st.threshold = o.threshold;
    // the four subgraphs; the source-list-ordered nd copy is reported apart
    st.bytes_layout = int64_t(n + 1) * 8 + int64_t(d + 1) * 8 + 4 * m;
    st.bytes_plain = o.keep_plain_csr ? int64_t(n + 1) * 8 + 4 * m : 0;
    return G;
  } catch (...) {
    delete G;
    throw;
  }
}

void graph_destroy(Graph *G) { delete G; }

void graph_export(const Graph *G, int32_t which, void *host_out, int64_t cap, int64_t *bytes) {
  const DevBuf *b = nullptr;
  int64_t nb = 0;
  const int64_t n = G->n, d = G->d;
  switch (which) {
    case 0: b = &G->deg; nb = n * 4; break;
    case 1: b = &G->did; nb = n * 4; break;
    case 2: b = &G->vid_of; nb = d * 4; break;
    case 3: b = &G->noff; nb = (n + 1) * 8; break;
    case 4: b = &G->ncol; nb = (G->st.e_nn + G->st.e_nd) * 4; break;
    case 5: b = &G->doff; nb = (d + 1) * 8; break;
    case 6: b = &G->dcol; nb = (G->st.e_dn + G->st.e_dd) * 4; break;
    case 7: b = &G->ndsrc; nb = G->st.n_ndsrc * 4; break;
    case 8: b = &G->ddsrc_mask; nb = int64_t(G->dwords()) * 4; break;
    case 9: b = &G->dnsrc_mask; nb = int64_t(G->dwords()) * 4; break;
    case 10: b = &G->poff; nb = G->poff.p ? (n + 1) * 8 : 0; break;
    case 11: b = &G->pcol; nb = G->pcol.p ? G->m * 4 : 0; break;
    case 12: b = &G->nds_off; nb = (G->st.n_ndsrc + 1) * 8; break;
    case 13: b = &G->nds_col; nb = G->st.e_nd * 4; break;
    case 14: b = &G->nds_first; nb = G->st.n_ndsrc * 8; break;
    case 15: b = &G->dd_first; nb = d * 8; break;
    case 16: b = &G->nlen; nb = n * 2; break;
    case 17: b = &G->nnsrc; nb = G->st.n_nnsrc * 4; break;
    case 18: b = &G->nnoff; nb = G->nnoff.p ? n * 4 : 0; break;
    case 19: b = &G->nncol; nb = G->nncol.p ? G->st.e_nn * 4 : 0; break;
    default: fail(DSBFS_ERR_INVALID_ARG, "unknown array index");
  }
  *bytes = nb;
  if (!host_out || cap < nb || nb == 0) return;
  HIPCHK(hipMemcpyAsync(host_out, b->p, size_t(nb), hipMemcpyDeviceToHost, G->stream));
  HIPCHK(hipStreamSynchronize(G->stream));
}

}  // namespace dsbfs
