// Device code shared by the kNN kernels of the single-job path (knn.hip) and the
// batched path (batch.hip): the exact ring search of Section 3.2.4 / 4.1.4 over
// one job's grid, and the coincident-query mean.  The search rule, the stop rule
// and the (squared distance, index) ordering are described in knn.hip.
#pragma once

#include <float.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aidw {
namespace knn {

// Cell coordinate of a float32 offset t = (x - min) * inv_cw: truncated, clamped
// into [0, nc); negative or NaN -> 0.
__device__ inline int clamp_cell(float t, int nc) {
  if (!(t >= 0.0f)) return 0;
  if (t >= 2147483520.0f) return nc - 1;
  const int c = (int)t;
  return c > nc - 1 ? nc - 1 : c;
}

// One job's grid scalars.  The CSR arrays travel beside it: cell_start indexed
// from the job's first cell, sx, sy, sidx in cell order.
struct View {
  float minx, miny, inv;
  int ncol, nrow;
  double cwd;
};

// The k nearest data points of (fx, fy): on return slots [KMAX - k, KMAX) of
// (bk, bi) hold their squared distances and indices in ascending (d2, index)
// order.  slack_cells covers the float32 binning error, in cells.
//
// LANES > 1: LANES consecutive lanes (sub = 0 .. LANES - 1) search for the same
// query together; each takes every LANES-th candidate of a segment and keeps the
// k best of its own candidates, so the union of the lanes' lists holds the k
// nearest.  The lanes walk the same rings in step and stop together: the global
// k-th distance is at most the largest over the lanes of each lane's
// ceil(k / LANES)-th, and that bound must pass the stop test (a lane with fewer
// candidates contributes +inf, which only delays the stop).  merge_lanes then
// reads the k nearest out in ascending order.
//
// PAPER = true: the paper's stop rule instead (Section 3.2.4 and its Remark):
// grow the level until the block holds >= k points, search one more level, stop.
// Not exact in general; kept to measure that rule.
// The largest over the LANES lanes of a query (an aligned group of LANES consecutive lanes)
// of each lane's ceil(k / LANES)-th best d2 (+inf where a lane holds fewer):
// the group holds at least k candidates at or below it, so the k-th nearest is no larger.
template <int KMAX, int LANES>
__device__ __forceinline__ double group_kth(const double (&bk)[KMAX], int k) {
  const int kq = (k + LANES - 1) / LANES;  // the lane's kq-th best: slot KMAX - k + kq - 1
  double v = bk[KMAX - 1];
#pragma unroll
  for (int s = 0; s < KMAX; ++s)
    if (s == KMAX - k + kq - 1) v = bk[s];
#pragma unroll
  for (int o = 1; o < LANES; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// A copy of part of the grid in LDS: rows [r0, r1], columns [c0, c1] (rows empty when r1 < r0).
// Each of its rows is one contiguous run of the cell-ordered arrays; row r's points sit at
// x[p + off[r - r0]] (and y, idx) for the global position p.  The pointers are generic, so a
// lane reads a segment from LDS or from global memory with the same loads; the pointers stay
// at the arrays' starts and the shift goes into the index, which is in range.
struct Window {
  int r0, r1, c0, c1;
  const int* off;
  const float* x;
  const float* y;
  const int32_t* idx;
};

template <int KMAX, int LANES = 1, bool PAPER = false, bool WIN = false>
__device__ __forceinline__ void search(const View& g, const int32_t* __restrict__ cell_start,
                                       const float* __restrict__ sx, const float* __restrict__ sy,
                                       const int32_t* __restrict__ sidx, float fx, float fy, int k,
                                       double slack_cells, double (&bk)[KMAX], int32_t (&bi)[KMAX], int sub = 0,
                                       const Window* win = nullptr) {
  const double px = fx, py = fy;
  const int ncol = g.ncol, nrow = g.nrow;
  const double cwd = g.cwd;
  const double minxd = g.minx, minyd = g.miny;
  const int c0 = clamp_cell((fx - g.minx) * g.inv, ncol);
  const int r0 = clamp_cell((fy - g.miny) * g.inv, nrow);
  const double slack = slack_cells * cwd;
  // slots [0, KMAX - k) hold a -1 sentinel that no candidate can pass; the k
  // live slots [KMAX - k, KMAX) are kept in ascending (d2, index) order.
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    const bool pad = s < KMAX - k;
    bk[s] = pad ? -1.0 : INFINITY;
    bi[s] = pad ? -1 : INT32_MAX;
  }
  int count = 0;
  // LANES > 1: an upper bound of the query's k-th (d2) over all lanes -- the largest of the
  // lanes' ceil(k / LANES)-th values once every lane holds that many -- refreshed after each
  // segment and never raised; a candidate above it cannot be among the k nearest, so it is
  // not offered (a lane then keeps fewer than k, which the merge allows).
  double bound = INFINITY;
  int final_level = -1;  // PAPER: the level after the one where the block first held >= k points

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
      const float* X = sx;
      const float* Y = sy;
      const int32_t* I = sidx;
      int shift = 0;
      if constexpr (WIN) {
        if (row >= win->r0 && row <= win->r1 && a >= win->c0 && b <= win->c1) {
          shift = win->off[row - win->r0];
          X = win->x;
          Y = win->y;
          I = win->idx;
        }
      }
      for (int p = p0 + sub; p < p1; p += LANES) {
        const double dx = (double)X[p + shift] - px;
        const double dy = (double)Y[p + shift] - py;
        const double d2 = dx * dx + dy * dy;
        const int32_t id = I[p + shift];
        // the comparisons of the (d2, index) order are combined with bitwise operators: each is
        // then one vector compare, where short-circuit forms compile to branches on the exec mask
        const bool take = (d2 < bk[KMAX - 1]) | ((d2 == bk[KMAX - 1]) & (id < bi[KMAX - 1]));
        if ((LANES == 1 || d2 <= bound) && take) {
          bk[KMAX - 1] = d2;
          bi[KMAX - 1] = id;
#pragma unroll
          for (int s = KMAX - 1; s > 0; --s) {
            const bool sw = (bk[s] < bk[s - 1]) | ((bk[s] == bk[s - 1]) & (bi[s] < bi[s - 1]));
            const double lo = bk[s], hi = bk[s - 1];
            const int32_t ilo = bi[s], ihi = bi[s - 1];
            bk[s - 1] = sw ? lo : hi;
            bk[s] = sw ? hi : lo;
            bi[s - 1] = sw ? ilo : ihi;
            bi[s] = sw ? ihi : ilo;
          }
        }
      }
      if constexpr (LANES > 1) {
        // the lanes of a query agree on p0, p1 and count, so this is uniform across them
        if (p1 > p0 && count >= k) bound = fmin(bound, group_kth<KMAX, LANES>(bk, k));
      }
    }
    const bool open_l = cl > 0, open_r = cr < ncol - 1, open_b = rb > 0, open_t = rt < nrow - 1;
    if (!(open_l || open_r || open_b || open_t)) break;  // the block covers the grid
    if constexpr (PAPER) {
      if (final_level < 0 && count >= k) final_level = L + 1;
      if (L == final_level) break;
      continue;
    }
    if (count >= k) {
      double dout = INFINITY;
      if (open_l) dout = fmin(dout, px - (minxd + (double)cl * cwd));
      if (open_r) dout = fmin(dout, (minxd + (double)(cr + 1) * cwd) - px);
      if (open_b) dout = fmin(dout, py - (minyd + (double)rb * cwd));
      if (open_t) dout = fmin(dout, (minyd + (double)(rt + 1) * cwd) - py);
      dout -= slack;
      const double kth = LANES > 1 ? bound : bk[KMAX - 1];
      if (dout > 0.0 && kth < dout * dout) break;
    }
  }

}

// The k nearest over a group of LANES lanes that searched together (search with
// LANES > 1): popped in ascending (d2, index) order, the same order summarise
// uses, so r_obs and d1 are bitwise those of a one-lane search.  Every lane of the
// group returns r_obs and d1; idx (may be null) receives the indices from lane sub 0.
template <int KMAX, int LANES>
__device__ __forceinline__ void merge_lanes(double (&bk)[KMAX], int32_t (&bi)[KMAX], int k, int sub, float& r_obs,
                                            float& d1, int32_t* __restrict__ idx) {
  // move the k live slots to the front: left shift by KMAX - k, one power of two at a time
  const int sh = KMAX - k;
#pragma unroll
  for (int b = 1; b < KMAX; b <<= 1) {
    if (sh & b) {
#pragma unroll
      for (int s = 0; s < KMAX; ++s) {
        bk[s] = s + b < KMAX ? bk[s + b] : INFINITY;
        bi[s] = s + b < KMAX ? bi[s + b] : INT32_MAX;
      }
    }
  }
  double sum = 0.0;
  d1 = 0.0f;
  for (int it = 0; it < k; ++it) {
    double mv = bk[0];
    int32_t mi = bi[0];
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
      const double ov = __shfl_xor(mv, o, 64);
      const int32_t oi = __shfl_xor(mi, o, 64);
      if (ov < mv || (ov == mv && oi < mi)) {
        mv = ov;
        mi = oi;
      }
    }
    if (bk[0] == mv && bi[0] == mi) {  // this lane's head was the smallest: pop it
#pragma unroll
      for (int s = 0; s < KMAX; ++s) {
        bk[s] = s + 1 < KMAX ? bk[s + 1] : INFINITY;
        bi[s] = s + 1 < KMAX ? bi[s + 1] : INT32_MAX;
      }
    }
    sum += sqrt(mv);
    if (it == 0) d1 = mv == 0.0 ? 0.0f : fmaxf((float)mv, FLT_MIN);
    if (idx && sub == 0) idx[it] = mi;
  }
  r_obs = (float)(sum / (double)k);
}

// Eq. 3 from the search result: r_obs = (1/k) sum of the k distances, added in
// ascending order in float64; d1 = the nearest squared distance (0 for a
// coincident query, else at least FLT_MIN so that 1/d1 stays finite).
template <int KMAX>
__device__ __forceinline__ void summarise(const double (&bk)[KMAX], int k, float& r_obs, float& d1) {
  double sum = 0.0;
  d1 = 0.0f;
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    if (s >= KMAX - k) sum += sqrt(bk[s]);
    if (s == KMAX - k) d1 = bk[s] == 0.0 ? 0.0f : fmaxf((float)bk[s], FLT_MIN);
  }
  r_obs = (float)(sum / (double)k);
}

// A coincident query's value: the mean z of the data points at its exact
// position (the limit of Eq. 1).  Those points share the query's cell, which is
// ordered by index, so the float64 sum runs in index order.  Returns false if
// no data point is at (fx, fy).
__device__ inline bool coincident_mean(const View& g, const int32_t* __restrict__ cell_start,
                                       const float* __restrict__ sx, const float* __restrict__ sy,
                                       const int32_t* __restrict__ sidx, const float* __restrict__ z, float fx,
                                       float fy, float& out) {
  const int col = clamp_cell((fx - g.minx) * g.inv, g.ncol);
  const int row = clamp_cell((fy - g.miny) * g.inv, g.nrow);
  const int c = row * g.ncol + col;
  double s = 0.0;
  int hits = 0;
  for (int p = cell_start[c]; p < cell_start[c + 1]; ++p) {
    if (sx[p] == fx && sy[p] == fy) {
      s += (double)z[sidx[p]];
      ++hits;
    }
  }
  if (hits > 0) out = (float)(s / hits);
  return hits > 0;
}

}  // namespace knn
}  // namespace aidw
