// Stage 1, kNN search and Eq. 3 (Section 3.2.4 and 4.1.4 of the paper).
//
// One query per lane, lanes taking the queries in cell order (the queries are
// binned by the same counting sort as the data), so that a wavefront's lanes
// walk neighbouring cells and share cache lines.  Each lane grows square rings
// of cells around its query's cell (level L = cells at Chebyshev distance L)
// and keeps its k best candidates in registers, ordered by (squared distance,
// data index), with a fully unrolled insertion (the paper's insert-and-swap
// k-array, initialised to +inf instead of 0 so that it accepts candidates).
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

namespace aidw {

namespace {

__device__ inline int clamp_cell(float t, int nc) {
  if (!(t >= 0.0f)) return 0;  // negative or NaN
  if (t >= 2147483520.0f) return nc - 1;
  const int c = (int)t;
  return c > nc - 1 ? nc - 1 : c;
}

template <int KMAX>
__global__ __launch_bounds__(256) void k_knn(const GridScalars* __restrict__ gs, const int32_t* __restrict__ cell_start,
                                             const float* __restrict__ sx, const float* __restrict__ sy,
                                             const int32_t* __restrict__ sidx, const float* __restrict__ qx,
                                             const float* __restrict__ qy, const uint32_t* __restrict__ qperm,
                                             const uint32_t* __restrict__ active, int m, int k, double slack_cells,
                                             float* __restrict__ r_obs, float* __restrict__ d1sq,
                                             int32_t* __restrict__ nn_idx) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m || (active && (uint32_t)t >= *active)) return;
  const int q = qperm ? (int)qperm[t] : t;
  const float fx = qx[q], fy = qy[q];
  const double px = fx, py = fy;
  const float minx = gs->minx, miny = gs->miny, inv = gs->inv_cw;
  const int ncol = gs->ncol, nrow = gs->nrow;
  const double cwd = gs->cwd;
  const double minxd = minx, minyd = miny;
  const int c0 = clamp_cell((fx - minx) * inv, ncol);
  const int r0 = clamp_cell((fy - miny) * inv, nrow);
  const double slack = slack_cells * cwd;

  // slots [0, KMAX - k) hold a -1 sentinel that no candidate can pass; the k
  // live slots [KMAX - k, KMAX) are kept in ascending (d2, index) order.
  double bk[KMAX];
  int32_t bi[KMAX];
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    const bool pad = s < KMAX - k;
    bk[s] = pad ? -1.0 : INFINITY;
    bi[s] = pad ? -1 : INT32_MAX;
  }
  int count = 0;

  for (int L = 0;; ++L) {
    const int cl = c0 - L, cr = c0 + L, rb = r0 - L, rt = r0 + L;
    const int ca = cl > 0 ? cl : 0;
    const int cb = cr < ncol - 1 ? cr : ncol - 1;
    const int ra = rb + 1 > 0 ? rb + 1 : 0;
    const int re = rt - 1 < nrow - 1 ? rt - 1 : nrow - 1;
    const int nside = re >= ra ? re - ra + 1 : 0;
    // ring L as segments: [0] bottom row, [1] top row (each one contiguous run of
    // points in cell order), then the left / right cell of every row in between.
    const int nseg = L == 0 ? 1 : 2 + 2 * nside;
    for (int sg = 0; sg < nseg; ++sg) {
      int row, a, b;
      bool ok;
      if (L == 0) {
        row = r0;
        a = b = c0;
        ok = true;
      } else if (sg < 2) {
        row = sg == 0 ? rb : rt;
        a = ca;
        b = cb;
        ok = sg == 0 ? rb >= 0 : rt < nrow;
      } else {
        const bool right = (sg - 2) & 1;
        row = ra + ((sg - 2) >> 1);
        a = b = right ? cr : cl;
        ok = right ? cr < ncol : cl >= 0;
      }
      if (!ok) continue;
      const int base = row * ncol;
      const int p0 = cell_start[base + a];
      const int p1 = cell_start[base + b + 1];
      count += p1 - p0;
      for (int p = p0; p < p1; ++p) {
        const double dx = (double)sx[p] - px;
        const double dy = (double)sy[p] - py;
        const double d2 = dx * dx + dy * dy;
        const int32_t id = sidx[p];
        if (d2 < bk[KMAX - 1] || (d2 == bk[KMAX - 1] && id < bi[KMAX - 1])) {
          bk[KMAX - 1] = d2;
          bi[KMAX - 1] = id;
#pragma unroll
          for (int s = KMAX - 1; s > 0; --s) {
            const bool sw = bk[s] < bk[s - 1] || (bk[s] == bk[s - 1] && bi[s] < bi[s - 1]);
            const double lo = bk[s], hi = bk[s - 1];
            const int32_t ilo = bi[s], ihi = bi[s - 1];
            bk[s - 1] = sw ? lo : hi;
            bk[s] = sw ? hi : lo;
            bi[s - 1] = sw ? ilo : ihi;
            bi[s] = sw ? ihi : ilo;
          }
        }
      }
    }
    const bool open_l = cl > 0, open_r = cr < ncol - 1, open_b = rb > 0, open_t = rt < nrow - 1;
    if (!(open_l || open_r || open_b || open_t)) break;  // the block covers the grid
    if (count >= k) {
      double dout = INFINITY;
      if (open_l) dout = fmin(dout, px - (minxd + (double)cl * cwd));
      if (open_r) dout = fmin(dout, (minxd + (double)(cr + 1) * cwd) - px);
      if (open_b) dout = fmin(dout, py - (minyd + (double)rb * cwd));
      if (open_t) dout = fmin(dout, (minyd + (double)(rt + 1) * cwd) - py);
      dout -= slack;
      if (dout > 0.0 && bk[KMAX - 1] < dout * dout) break;
    }
  }

  double sum = 0.0;
  float d1 = 0.0f;
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    if (s >= KMAX - k) sum += sqrt(bk[s]);
    if (s == KMAX - k) d1 = bk[s] == 0.0 ? 0.0f : fmaxf((float)bk[s], FLT_MIN);
  }
  r_obs[q] = (float)(sum / (double)k);
  if (d1sq) d1sq[q] = d1;
  if (nn_idx) {
    int32_t* row = nn_idx + (size_t)q * k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
      if (s >= KMAX - k) row[s - (KMAX - k)] = bi[s];
  }
}

}  // namespace

hipError_t launch_knn(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                      const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                      const uint32_t* active, int m, int k, double slack_cells, float* r_obs, float* d1sq,
                      int32_t* nn_idx, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((m + 255) / 256), block(256);
  if (k <= 8)
    hipLaunchKernelGGL(k_knn<8>, grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, m, k, slack_cells,
                       r_obs, d1sq, nn_idx);
  else if (k <= 16)
    hipLaunchKernelGGL(k_knn<16>, grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, m, k, slack_cells,
                       r_obs, d1sq, nn_idx);
  else if (k <= 32)
    hipLaunchKernelGGL(k_knn<32>, grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, m, k, slack_cells,
                       r_obs, d1sq, nn_idx);
  else
    hipLaunchKernelGGL(k_knn<64>, grid, block, 0, s, gs, cell_start, sx, sy, sidx, qx, qy, qperm, active, m, k, slack_cells,
                       r_obs, d1sq, nn_idx);
  return hipGetLastError();
}

}  // namespace aidw
