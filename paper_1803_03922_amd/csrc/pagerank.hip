// PageRank on the degree-separated layout.
//
// The paper names other graph primitives on degree-separated graphs as future
// work, where delegates carry multi-bit state instead of the one-bit masks of
// BFS (Sections VI-D, VII). Here the delegate state is each delegate's rank
// contribution r/deg, kept in a compact array indexed by delegate ID (the
// array that would be replicated across GPUs, as the BFS masks are); normal
// vertices keep theirs in an array indexed by vertex ID. One FP64 power
// iteration step from r to r':
//   D = rank of the degree-0 vertices (spread uniformly),
//   r'[v] = (1 - alpha) / n + alpha * (D / n + sum over neighbours u of
//           r[u] / deg(u)),
// as three kernels: contributions (and D), the pull over normal rows (nn part
// from the normal array, nd part from the delegate array; rows have at most
// TH entries: one thread per row), and the pull over delegate rows (dd part
// from the delegate array, dn part from the normal array; long rows: one wave
// per row). Row sums run in stored row order per thread and in a fixed-shape
// wave reduction; the dangling mass and the L1 change are summed with atomics,
// whose order can move the last bits between runs.
//
// The dd part is 90% of the edges at RMAT 26, and on scale-free graphs most
// of its gathers land on the few highest-degree delegates, which delegate IDs
// (ascending vertex IDs) scatter over the whole contribution array. The
// delegate pull therefore reads its dd entries from a copy of the delegate
// columns in which each dd entry is the neighbour's rank by descending degree,
// and gathers from the contributions stored by that rank: the hot ones share
// lines and stay in the L2, while the columns stream past it (nontemporal
// loads). The values summed and their order are unchanged.
#include "internal.hpp"

namespace dsbfs {

namespace {

constexpr int kPB = 256;

struct PrAcc {
  double dangling;  // rank of degree-0 vertices this step
  double delta;     // L1 change of this step
};

__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Block sum of one double per thread, added to *dst with one atomic.
__device__ __forceinline__ void block_add_f64(double *dst, double x, double *sh) {
  x = wave_sum_f64(x);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < int(blockDim.x) / kWave; ++i) t += sh[i];
    if (t != 0.0) atomicAdd(dst, t);
  }
  __syncthreads();
}

__global__ void k_pr_fill(double *r, int32_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    r[i] = v;
}

// Sort keys of the delegates: (max degree - degree) above the delegate ID,
// so ascending keys are descending degree, ties by ID.
__global__ void k_pr_keys(const int32_t *vid_of, const int32_t *deg, int32_t d, int32_t maxdeg,
                          uint64_t *keys) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < d;
       k += int64_t(gridDim.x) * blockDim.x)
    keys[k] = (uint64_t(uint32_t(maxdeg - deg[vid_of[k]])) << 32) | uint64_t(uint32_t(k));
}

__global__ void k_pr_ranks(const uint64_t *keys, int32_t d, int32_t *rank) {
  for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < d;
       r += int64_t(gridDim.x) * blockDim.x)
    rank[uint32_t(keys[r])] = int32_t(r);
}

// pr_col: the delegate rows with dd entries as ranks, dn entries as they are.
__global__ void __launch_bounds__(kPB) k_pr_cols(const uint64_t *doff, const int32_t *dcol,
                                                 const int32_t *rank, int32_t d, int32_t *pcol) {
  const int l = lane_id();
  const int64_t wid = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * blockDim.x / kWave;
  for (int64_t k = wid; k < d; k += nw) {
    const uint64_t w0 = doff[k], w1 = doff[k + 1];
    const int64_t b = row_start(w0), mid = b + row_first(w0), e = row_start(w1);
    for (int64_t i = b + l; i < e; i += kWave) {
      const int32_t c = dcol[i];
      pcol[i] = i < mid ? rank[c] : c;
    }
  }
}

__global__ void __launch_bounds__(kPB) k_pr_contrib(const double *r, const int32_t *deg,
                                                    const int32_t *did, const int32_t *rank,
                                                    int32_t n, double *cn, double *cd,
                                                    double *cdr, PrAcc *acc) {
  __shared__ double sh[kPB / kWave];
  double dang = 0.0;
  for (int64_t v0 = int64_t(blockIdx.x) * blockDim.x; v0 < n;
       v0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t v = v0 + threadIdx.x;
    if (v < n) {
      const double x = r[v];
      const int32_t dg = deg[v];
      const double c = dg > 0 ? x / double(dg) : 0.0;
      if (dg == 0) dang += x;
      const int32_t k = did[v];
      if (k >= 0) {
        cd[k] = c;
        cdr[rank[k]] = c;
      } else {
        cn[v] = c;
      }
    }
  }
  block_add_f64(&acc->dangling, dang, sh);
}

__device__ __forceinline__ double pr_base(const PrAcc *acc, double alpha, int32_t n) {
  return (1.0 - alpha) / double(n) + alpha * acc->dangling / double(n);
}

// Normal rows: nn part (vertex IDs, normal contributions), then nd part
// (delegate IDs, delegate contributions). A thread sums its row in stored
// order, four entries at a time: four column loads, then four gathers, then
// the four additions. Slots past the row end re-load its last entry and add
// +0.0 (the partial sum is non-negative), as in the delegate pull.
constexpr int kPrRowUnroll = 4;

__global__ void __launch_bounds__(kPB) k_pr_normal(const uint64_t *noff, const int32_t *ncol,
                                                   const int32_t *did, int32_t n,
                                                   const double *cn, const double *cd,
                                                   double alpha, const PrAcc *acc,
                                                   const double *r, double *rn, PrAcc *out) {
  __shared__ double sh[kPB / kWave];
  const double base = pr_base(acc, alpha, n);
  double delta = 0.0;
  for (int64_t v0 = int64_t(blockIdx.x) * blockDim.x; v0 < n;
       v0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t v = v0 + threadIdx.x;
    if (v < n && did[v] < 0) {
      const uint64_t w0 = noff[v], w1 = noff[v + 1];
      const int64_t b = row_start(w0), mid = b + row_first(w0), e = row_start(w1);
      double s = 0.0;
      for (int64_t i0 = b; i0 < e; i0 += kPrRowUnroll) {
        int32_t c[kPrRowUnroll];
        double y[kPrRowUnroll];
#pragma unroll
        for (int u = 0; u < kPrRowUnroll; ++u) c[u] = ncol[i0 + u < e ? i0 + u : e - 1];
#pragma unroll
        for (int u = 0; u < kPrRowUnroll; ++u) {
          const int64_t j = i0 + u;
          const double g = ((j < e ? j : e - 1) < mid ? cn : cd)[c[u]];
          y[u] = j < e ? g : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPrRowUnroll; ++u) s += y[u];
      }
      const double x = base + alpha * s;
      delta += fabs(x - r[v]);
      rn[v] = x;
    }
  }
  block_add_f64(&out->delta, delta, sh);
}

// Delegate rows, one wave per row: dd part (delegate ranks, contributions by
// rank), then dn part (vertex IDs, normal contributions). Each lane takes the
// row's entries l, l + 64, l + 128, ... in that order. Rows longer than a wave
// go eight entries per lane at a time: eight column loads, then eight
// gathers, then the eight additions, so eight gathers are in flight per lane
// instead of one and the sum is the same. A slot past the row end loads the
// row's last entry again (no branch, so no wait between the loads) and adds
// +0.0, which leaves the non-negative partial sum unchanged. Eight costs 80
// VGPRs (6 waves per SIMD) and still beats four at 64 (8 waves per SIMD).
constexpr int kPrUnroll = 8;

__global__ void __launch_bounds__(kPB) k_pr_deleg(const uint64_t *doff, const int32_t *pcol,
                                                  const int32_t *vid_of, int32_t d, int32_t n,
                                                  const double *cn, const double *cdr,
                                                  double alpha, const PrAcc *acc,
                                                  const double *r, double *rn, PrAcc *out) {
  __shared__ double sh[kPB / kWave];
  const double base = pr_base(acc, alpha, n);
  const int l = lane_id();
  const int64_t wid = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = int64_t(gridDim.x) * blockDim.x / kWave;
  double delta = 0.0;
  for (int64_t k = wid; k < d; k += nw) {
    const uint64_t w0 = doff[k], w1 = doff[k + 1];
    const int64_t b = row_start(w0), mid = b + row_first(w0), e = row_start(w1);
    double s = 0.0;
    if (e - b <= kWave) {
      const int64_t i = b + l;
      if (i < e) s = (i < mid ? cdr : cn)[__builtin_nontemporal_load(pcol + i)];
    } else {
      for (int64_t i0 = b + l; i0 < e; i0 += kPrUnroll * kWave) {
        int32_t c[kPrUnroll];
        double x[kPrUnroll];
#pragma unroll
        for (int u = 0; u < kPrUnroll; ++u) {
          const int64_t j = i0 + int64_t(u) * kWave;
          c[u] = __builtin_nontemporal_load(pcol + (j < e ? j : e - 1));
        }
#pragma unroll
        for (int u = 0; u < kPrUnroll; ++u) {
          const int64_t j = i0 + int64_t(u) * kWave;
          const double v = ((j < e ? j : e - 1) < mid ? cdr : cn)[c[u]];
          x[u] = j < e ? v : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPrUnroll; ++u) s += x[u];
      }
    }
    s = wave_sum_f64(s);
    if (l == 0) {
      const int32_t v = vid_of[k];
      const double x = base + alpha * s;
      delta += fabs(x - r[v]);
      rn[v] = x;
    }
  }
  block_add_f64(&out->delta, delta, sh);
}

}  // namespace

void pagerank_run(const Graph *g, double alpha, int32_t max_iter, double tol, double *rank,
                  int32_t *iters_done, double *last_delta, hipStream_t s) {
  if (!rank) fail(DSBFS_ERR_INVALID_ARG, "rank must not be NULL");
  if (!(alpha >= 0.0 && alpha <= 1.0)) fail(DSBFS_ERR_INVALID_ARG, "alpha must be in [0, 1]");
  if (max_iter < 0) fail(DSBFS_ERR_INVALID_ARG, "max_iterations must be >= 0");
  const int32_t n = g->n, d = g->d;
  const Alloc *al = &g->al;
  if (d > 0) {
    std::lock_guard<std::mutex> lk(g->pr_mu);
    if (!g->pr_col.p) {
      DevBuf keys, alt, tmp, rank, pcol;
      keys.alloc(al, size_t(d) * 8, s);
      alt.alloc(al, size_t(d) * 8, s);
      tmp.alloc(al, radix_tmp_bytes(d), s);
      rank.alloc(al, size_t(d) * 4, s);
      const int64_t ecols = g->st.e_dd + g->st.e_dn;
      pcol.alloc(al, size_t(std::max<int64_t>(ecols, 1)) * 4, s);
      const int G0 = grid_for(d, kPB, 8192);
      hipLaunchKernelGGL(k_pr_keys, dim3(G0), dim3(kPB), 0, s, g->vid_of.as<int32_t>(),
                         g->deg.as<int32_t>(), d, int32_t(g->st.max_degree), keys.as<uint64_t>());
      HIPCHK(hipGetLastError());
      // keys start in ascending ID order: a stable sort on the degree field
      // alone leaves ties in ID order
      int db = 0;
      while ((int64_t(1) << db) <= g->st.max_degree) ++db;
      radix_sort_u64_bits(keys.as<uint64_t>(), alt.as<uint64_t>(), d, 32, 32 + db, tmp.p, s);
      hipLaunchKernelGGL(k_pr_ranks, dim3(G0), dim3(kPB), 0, s, keys.as<uint64_t>(), d,
                         rank.as<int32_t>());
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(k_pr_cols, dim3(grid_for(int64_t(d) * kWave, kPB, 8192)), dim3(kPB), 0,
                         s, g->doff.as<uint64_t>(), g->dcol.as<int32_t>(), rank.as<int32_t>(), d,
                         pcol.as<int32_t>());
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      g->pr_rank = std::move(rank);
      g->pr_col = std::move(pcol);
    }
  }
  DevBuf cn, cd, cdr, rb, acc;
  cn.alloc(al, size_t(n) * 8, s);
  cd.alloc(al, size_t(std::max(d, 1)) * 8, s);
  cdr.alloc(al, size_t(std::max(d, 1)) * 8, s);
  rb.alloc(al, size_t(n) * 8, s);
  // two accumulators per step, alternating (one is cleared while the other is read)
  acc.alloc(al, 2 * sizeof(PrAcc), s);
  // the last step must land in `rank`: start in whichever buffer makes it so
  double *buf[2] = {rank, rb.as<double>()};
  int cur = (max_iter % 2 == 0) ? 0 : 1;
  const int G1 = grid_for(n, kPB, 8192);
  hipLaunchKernelGGL(k_pr_fill, dim3(G1), dim3(kPB), 0, s, buf[cur], n, 1.0 / double(n));
  HIPCHK(hipGetLastError());
  PrAcc *A = acc.as<PrAcc>();
  int32_t it = 0;
  double dl = 0.0;
  for (; it < max_iter; ++it) {
    PrAcc *a = A + (it & 1);
    HIPCHK(hipMemsetAsync(a, 0, sizeof(PrAcc), s));
    hipLaunchKernelGGL(k_pr_contrib, dim3(G1), dim3(kPB), 0, s, buf[cur], g->deg.as<int32_t>(),
                       g->did.as<int32_t>(), g->pr_rank.as<int32_t>(), n, cn.as<double>(),
                       cd.as<double>(), cdr.as<double>(), a);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_pr_normal, dim3(G1), dim3(kPB), 0, s, g->noff.as<uint64_t>(),
                       g->ncol.as<int32_t>(), g->did.as<int32_t>(), n, cn.as<double>(),
                       cd.as<double>(), alpha, a, buf[cur], buf[cur ^ 1], a);
    HIPCHK(hipGetLastError());
    if (d > 0) {
      hipLaunchKernelGGL(k_pr_deleg, dim3(grid_for(int64_t(d) * kWave, kPB, 8192)), dim3(kPB), 0,
                         s, g->doff.as<uint64_t>(), g->pr_col.as<int32_t>(),
                         g->vid_of.as<int32_t>(), d, n, cn.as<double>(), cdr.as<double>(), alpha,
                         a, buf[cur], buf[cur ^ 1], a);
      HIPCHK(hipGetLastError());
    }
    cur ^= 1;
    if (tol > 0.0 || it + 1 == max_iter) {
      PrAcc h{};
      HIPCHK(hipMemcpyAsync(&h, a, sizeof(PrAcc), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      dl = h.delta;
      if (tol > 0.0 && dl < tol) {
        ++it;
        break;
      }
    }
  }
  if (buf[cur] != rank)
    HIPCHK(hipMemcpyAsync(rank, buf[cur], size_t(n) * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (iters_done) *iters_done = it;
  if (last_delta) *last_delta = dl;
}

}  // namespace dsbfs
