// Stage 1, kNN search and Eq. 3 (Section 3.2.4 and 4.1.4 of the paper).
//
// One query per lane, lanes taking the queries in cell order (the queries are
// binned by the same counting sort as the data), so that a wavefront's lanes
// walk neighbouring cells and share cache lines.  Each lane grows square rings
// of cells around its query's cell (level L = cells at Chebyshev distance L)
// and keeps its k best candidates in registers, ordered by (squared distance,
// data index), with a fully unrolled insertion (the paper's insert-and-swap
// k-array, initialised to +inf instead of 0 so that it accepts candidates) whose
// comparisons are branch-free (vector compares combined with bitwise operators).
//
// Stop rule.  The paper expands until the block holds k points and then adds
// one more level.  That is not always enough: the block of level L only
// guarantees that points outside it are at least the distance from the query
// to the block's edge, while the k-th candidate found may lie toward a corner,
// up to sqrt(2) times further.  Here a lane stops when it has seen >= k points
// AND the current k-th squared distance is strictly smaller than the squared
// distance from the query to the nearest open side of the block (a side beyond
// which grid cells remain), reduced by a slack that covers float32 binning
// error; or when the block covers the whole grid.  Then no unseen point can
// enter the k best, and the result equals the brute-force definition.
//
// Squared distances are formed in float64 from the float32 inputs, without
// contraction (this file is compiled with -ffp-contract=off), exactly as the
// definition states; r_obs sums the k square roots in ascending order in float64.
#include <float.h>

#include "aidw_internal.h"
#include "knn_core.h"
#include "pair_core.h"

namespace aidw {

namespace {


template <int KMAX, bool PAPER = false>
__global__ __launch_bounds__(256) void k_knn(const GridScalars* __restrict__ gs, const int32_t* __restrict__ cell_start,
                                             const float* __restrict__ sx, const float* __restrict__ sy,
                                             const int32_t* __restrict__ sidx, const float* __restrict__ qx,
                                             const float* __restrict__ qy, const uint32_t* __restrict__ qperm,
                                             const uint32_t* __restrict__ active, int m, int k,
                                             float* __restrict__ r_obs, float* __restrict__ d1sq,
                                             int32_t* __restrict__ nn_idx) {
  // XCD-aware order only when every workgroup has queries (with a device-side count, the live
  // workgroups are the first ones, which the remap would put on one XCD)
  const int blk = active ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int t = blk * blockDim.x + threadIdx.x;
  if (t >= m || (active && (uint32_t)t >= *active) || gs->status != AIDW_OK) return;
  const double slack = slack_cells(gs->ncol, gs->nrow);
  const int q = qperm ? (int)qperm[t] : t;
  const float fx = qx[q], fy = qy[q];
  const knn::View g{gs->minx, gs->miny, gs->inv_cw, gs->ncol, gs->nrow, gs->cwd};
  double bk[KMAX];
  int32_t bi[KMAX];
  knn::search<KMAX, 1, PAPER>(g, cell_start, sx, sy, sidx, fx, fy, k, slack, bk, bi);
  float ro, d1;
  knn::summarise<KMAX>(bk, k, ro, d1);
  r_obs[q] = ro;
  if (d1sq) d1sq[q] = d1;
  if (nn_idx) {
    int32_t* row = nn_idx + (size_t)q * k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
      if (s >= KMAX - k) row[s - (KMAX - k)] = bi[s];
  }
}

// The kNN of 256 binned queries per workgroup with their cells' neighbourhood staged in LDS:
// the queries of a workgroup lie in consecutive cells of one grid row (or two), so the window
// is that column range widened by kWinHalo cells on each side over the rows within kWinHalo of
// theirs (all columns when the queries span two rows).  A window row is one contiguous run of
// the cell-ordered arrays, copied with coalesced loads.  A segment of a ring inside the window
// is read from LDS, any other from global memory; a window of more than kWinCap points is not
// staged (every read goes to global memory, as in k_knn).
constexpr int kWinHalo = 2;
constexpr int kWinCap = 2048;
constexpr int kWinRowsMax = 2 + 2 * kWinHalo;
template <int KMAX>
__global__ __launch_bounds__(256) void k_knn_window(const GridScalars* __restrict__ gs,
                                                    const int32_t* __restrict__ cell_start,
                                                    const float* __restrict__ sx, const float* __restrict__ sy,
                                                    const int32_t* __restrict__ sidx, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const uint32_t* __restrict__ qperm,
                                                    int m, int k, float* __restrict__ r_obs, float* __restrict__ d1sq,
                                                    int32_t* __restrict__ nn_idx) {
  __shared__ float w_x[kWinCap], w_y[kWinCap];
  __shared__ int32_t w_i[kWinCap];
  __shared__ int w_p0[kWinRowsMax], w_base[kWinRowsMax + 1], w_off[kWinRowsMax];
  __shared__ int w_dims[4];  // r0, r1 (r1 < r0: no window), c0, c1
  if (gs->status != AIDW_OK) return;
  const knn::View g{gs->minx, gs->miny, gs->inv_cw, gs->ncol, gs->nrow, gs->cwd};
  const int ncol = g.ncol, nrow = g.nrow;
  const int t0 = xcd_block(blockIdx.x, gridDim.x) * blockDim.x;
  const int t = t0 + threadIdx.x;
  if (threadIdx.x == 0) {
    // the first and last query of the workgroup bound its cells (binned order is cell order)
    const int qa = qperm ? (int)qperm[t0] : t0;
    const int tl = min(m - 1, t0 + (int)blockDim.x - 1);
    const int qb = qperm ? (int)qperm[tl] : tl;
    const int ca = knn::clamp_cell((qx[qa] - g.minx) * g.inv, ncol), ra = knn::clamp_cell((qy[qa] - g.miny) * g.inv, nrow);
    const int cb = knn::clamp_cell((qx[qb] - g.minx) * g.inv, ncol), rb = knn::clamp_cell((qy[qb] - g.miny) * g.inv, nrow);
    int r0 = max(0, min(ra, rb) - kWinHalo), r1 = min(nrow - 1, max(ra, rb) + kWinHalo);
    int c0 = 0, c1 = ncol - 1;
    if (ra == rb) {
      c0 = max(0, min(ca, cb) - kWinHalo);
      c1 = min(ncol - 1, max(ca, cb) + kWinHalo);
    }
    if (r1 - r0 + 1 > kWinRowsMax) r1 = r0 - 1;
    int total = 0;
    for (int r = r0; r <= r1; ++r) {
      const int p0 = cell_start[r * ncol + c0], p1 = cell_start[r * ncol + c1 + 1];
      w_p0[r - r0] = p0;
      w_base[r - r0] = total;
      w_off[r - r0] = total - p0;
      total += p1 - p0;
    }
    if (total > kWinCap) r1 = r0 - 1;
    w_base[r1 >= r0 ? r1 - r0 + 1 : 0] = total;
    w_dims[0] = r0;
    w_dims[1] = r1;
    w_dims[2] = c0;
    w_dims[3] = c1;
  }
  __syncthreads();
  const int r0 = w_dims[0], r1 = w_dims[1];
  const int nrows = r1 >= r0 ? r1 - r0 + 1 : 0;
  for (int r = 0; r < nrows; ++r) {
    const int b0 = w_base[r], len = w_base[r + 1] - b0, p0 = w_p0[r];
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      w_x[b0 + i] = sx[p0 + i];
      w_y[b0 + i] = sy[p0 + i];
      w_i[b0 + i] = sidx[p0 + i];
    }
  }
  __syncthreads();
  if (t >= m) return;
  const knn::Window win{r0, r1, w_dims[2], w_dims[3], w_off, w_x, w_y, w_i};
  const double slack = slack_cells(ncol, nrow);
  const int q = qperm ? (int)qperm[t] : t;
  double bk[KMAX];
  int32_t bi[KMAX];
  knn::search<KMAX, 1, false, true>(g, cell_start, sx, sy, sidx, qx[q], qy[q], k, slack, bk, bi, 0, &win);
  float ro, d1;
  knn::summarise<KMAX>(bk, k, ro, d1);
  r_obs[q] = ro;
  if (d1sq) d1sq[q] = d1;
  if (nn_idx) {
    int32_t* row = nn_idx + (size_t)q * k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
      if (s >= KMAX - k) row[s - (KMAX - k)] = bi[s];
  }
}

// LANES lanes per query (knn::search with LANES > 1), for query sets too small to fill
// the chip with one query per lane: LANES times the wavefronts to hide the gathers'
// latency, and 1 / LANES of the candidates per lane.
template <int KMAX, int LANES>
__global__ __launch_bounds__(256) void k_knn_lanes(const GridScalars* __restrict__ gs, const int32_t* __restrict__ cell_start,
                                              const float* __restrict__ sx, const float* __restrict__ sy,
                                              const int32_t* __restrict__ sidx, const float* __restrict__ qx,
                                              const float* __restrict__ qy, const uint32_t* __restrict__ qperm,
                                              const uint32_t* __restrict__ active, int m, int k,
                                              float* __restrict__ r_obs, float* __restrict__ d1sq,
                                              int32_t* __restrict__ nn_idx, AlphaParams ap,
                                              float* __restrict__ alpha_f) {
  // XCD-aware order only without a device-side count (see k_knn)
  const int blk = active ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int gt = blk * blockDim.x + threadIdx.x;
  const int t = gt / LANES, sub = gt % LANES;
  // the lanes of a query leave together
  if (t >= m || (active && (uint32_t)t >= *active) || gs->status != AIDW_OK) return;
  const double slack = slack_cells(gs->ncol, gs->nrow);
  const int q = qperm ? (int)qperm[t] : t;
  const knn::View g{gs->minx, gs->miny, gs->inv_cw, gs->ncol, gs->nrow, gs->cwd};
  double bk[KMAX];
  int32_t bi[KMAX];
  knn::search<KMAX, LANES>(g, cell_start, sx, sy, sidx, qx[q], qy[q], k, slack, bk, bi, sub);
  float ro, d1;
  knn::merge_lanes<KMAX, LANES>(bk, bi, k, sub, ro, d1, nn_idx ? nn_idx + (size_t)q * k : nullptr);
  if (sub == 0) {
    r_obs[q] = ro;
    if (d1sq) d1sq[q] = d1;
    // Eq. 4-6 from the stored r_obs, as the alpha kernel of the plain path computes them
    if (alpha_f)
      alpha_f[q] =
          (float)pair::level_alpha(pair::fuzzy_mu((double)ro / alpha_r_exp(ap), ap.r_min, ap.r_max), ap.levels);
  }
}

// The per-query brute-force kNN of the earlier GPU AIDW that the paper improves on
// (Section 3.1): every query scans all n data points and keeps its k best in
// registers.  One query per lane; the data index is the same across a wavefront,
// so x, y come through the scalar cache.  Squared distances in float64 and the
// (d2, index) order as in k_knn, so the result is the exact kNN, bit for bit.
template <int KMAX>
__global__ __launch_bounds__(256) void k_knn_brute(const float* __restrict__ x, const float* __restrict__ y, int n,
                                                   const float* __restrict__ qx, const float* __restrict__ qy, int m,
                                                   int k, float* __restrict__ r_obs, float* __restrict__ d1sq,
                                                   int32_t* __restrict__ nn_idx) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = q < m;
  const double px = live ? qx[q] : 0.0, py = live ? qy[q] : 0.0;
  double bk[KMAX];
  int32_t bi[KMAX];
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    const bool pad = s < KMAX - k;
    bk[s] = pad ? -1.0 : INFINITY;
    bi[s] = pad ? -1 : INT32_MAX;
  }
  // points arrive in index order, so a later point with an equal distance never enters
  for (int i = 0; i < n; ++i) {
    const double dx = (double)x[i] - px;
    const double dy = (double)y[i] - py;
    const double d2 = dx * dx + dy * dy;
    if (d2 < bk[KMAX - 1]) {
      bk[KMAX - 1] = d2;
      bi[KMAX - 1] = i;
#pragma unroll
      for (int s = KMAX - 1; s > 0; --s) {
        const bool sw = bk[s] < bk[s - 1];
        const double lo = bk[s], hi = bk[s - 1];
        const int32_t ilo = bi[s], ihi = bi[s - 1];
        bk[s - 1] = sw ? lo : hi;
        bk[s] = sw ? hi : lo;
        bi[s - 1] = sw ? ilo : ihi;
        bi[s] = sw ? ihi : ilo;
      }
    }
  }
  if (!live) return;
  float ro, d1;
  knn::summarise<KMAX>(bk, k, ro, d1);
  r_obs[q] = ro;
  if (d1sq) d1sq[q] = d1;
  if (nn_idx) {
    int32_t* row = nn_idx + (size_t)q * k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
      if (s >= KMAX - k) row[s - (KMAX - k)] = bi[s];
  }
}

}  // namespace

hipError_t launch_knn_brute(const float* x, const float* y, int n, const float* qx, const float* qy, int m, int k,
                            float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((m + 255) / 256), block(256);
#define AIDW_KNNB(K) \
  hipLaunchKernelGGL(k_knn_brute<K>, grid, block, 0, s, x, y, n, qx, qy, m, k, r_obs, d1sq, nn_idx)
  if (k <= 8)
    AIDW_KNNB(8);
  else if (k <= 16)
    AIDW_KNNB(16);
  else if (k <= 32)
    AIDW_KNNB(32);
  else
    AIDW_KNNB(64);
#undef AIDW_KNNB
  return hipGetLastError();
}

hipError_t launch_knn_paper(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                            const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm, int m, int k,
                            float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((m + 255) / 256), block(256);
#define AIDW_KNNP(K)                                                                                                \
  hipLaunchKernelGGL((k_knn<K, true>), grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, nullptr, m, \
                     k, r_obs, d1sq, nn_idx)
  if (k <= 8)
    AIDW_KNNP(8);
  else if (k <= 16)
    AIDW_KNNP(16);
  else if (k <= 32)
    AIDW_KNNP(32);
  else
    AIDW_KNNP(64);
#undef AIDW_KNNP
  return hipGetLastError();
}

hipError_t launch_knn_lanes(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                            const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                            const uint32_t* active, int m, int k, float* r_obs, float* d1sq, int32_t* nn_idx,
                            int lanes, hipStream_t s, const AlphaParams* ap, float* alpha_f) {
  if (m <= 0) return hipSuccess;
  const AlphaParams apv = ap ? *ap : AlphaParams{};
  if (!ap) alpha_f = nullptr;
  if (lanes != 2 && lanes != 4 && lanes != 8) return hipErrorInvalidValue;
  // one workgroup per 256 / lanes queries; with an active count the workgroups beyond it exit at
  // once (a grid-stride loop instead keeps more registers live across the search: measured slower)
  const dim3 grid((int)(((int64_t)m * lanes + 255) / 256)), block(256);
#define AIDW_KNNL(K, LN)                                                                                         \
  hipLaunchKernelGGL((k_knn_lanes<K, LN>), grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, \
                     m, k, r_obs, d1sq, nn_idx, apv, alpha_f)
#define AIDW_KNNL_2(K) AIDW_KNNL(K, 2)
#define AIDW_KNNL_4(K) AIDW_KNNL(K, 4)
#define AIDW_KNNL_8(K) AIDW_KNNL(K, 8)
#define AIDW_KNNL_K(LN) AIDW_FOR_KNN_SLOTS(k, AIDW_KNNL_##LN)
  if (lanes == 2) {
    AIDW_KNNL_K(2);
  } else if (lanes == 4) {
    AIDW_KNNL_K(4);
  } else {
    AIDW_KNNL_K(8);
  }
#undef AIDW_KNNL_K
#undef AIDW_KNNL_8
#undef AIDW_KNNL_4
#undef AIDW_KNNL_2
#undef AIDW_KNNL
  return hipGetLastError();
}

hipError_t launch_knn4(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                       const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                       const uint32_t* active, int m, int k, float* r_obs, float* d1sq, int32_t* nn_idx,
                       hipStream_t s) {
  return launch_knn_lanes(gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, m, k, r_obs, d1sq, nn_idx, 4, s);
}

hipError_t launch_knn_window(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                             const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm, int m, int k,
                             float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((m + 255) / 256), block(256);
#define AIDW_KNNW(K)                                                                                            \
  hipLaunchKernelGGL(k_knn_window<K>, grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, m, k, r_obs, \
                     d1sq, nn_idx)
  AIDW_FOR_KNN_SLOTS(k, AIDW_KNNW)
#undef AIDW_KNNW
  return hipGetLastError();
}

hipError_t launch_knn(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                      const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                      const uint32_t* active, int m, int k, float* r_obs, float* d1sq, int32_t* nn_idx,
                      hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((m + 255) / 256), block(256);
#define AIDW_KNN1(K)                                                                                              \
  hipLaunchKernelGGL(k_knn<K>, grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, m, k, \
                     r_obs, d1sq, nn_idx)
  AIDW_FOR_KNN_SLOTS(k, AIDW_KNN1)
#undef AIDW_KNN1
  return hipGetLastError();
}

}  // namespace aidw
