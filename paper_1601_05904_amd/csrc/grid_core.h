// Grid scalars from the bounds (Eq. 2, Section 4.1.1), shared by the single-job
// finalize kernel (grid.hip) and the batched one (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aidw_internal.h"

namespace aidw {
namespace gridc {

__device__ inline float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_or(int v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// Min / max / non-finite flag over the bounds partials [begin, end), reduced by a
// workgroup of up to 1024 threads; the result is valid in every thread.
__device__ inline BoundsPartial block_reduce_bounds(const BoundsPartial* __restrict__ partial, int begin, int end) {
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  int bad = 0;
  for (int i = begin + (int)threadIdx.x; i < end; i += blockDim.x) {
    mnx = fminf(mnx, partial[i].minx);
    mny = fminf(mny, partial[i].miny);
    mxx = fmaxf(mxx, partial[i].maxx);
    mxy = fmaxf(mxy, partial[i].maxy);
    bad |= partial[i].nonfinite;
  }
  mnx = wave_min(mnx);
  mny = wave_min(mny);
  mxx = wave_max(mxx);
  mxy = wave_max(mxy);
  bad = wave_or(bad);
  __shared__ BoundsPartial s[16];  // one per wavefront of a block of up to 1024 threads
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s[wave] = BoundsPartial{mnx, mny, mxx, mxy, bad, {0, 0, 0}};
  __syncthreads();
  BoundsPartial r = s[0];
  const int nw = (int)(blockDim.x + 63) >> 6;
  for (int w = 1; w < nw; ++w) {
    r.minx = fminf(r.minx, s[w].minx);
    r.miny = fminf(r.miny, s[w].miny);
    r.maxx = fmaxf(r.maxx, s[w].maxx);
    r.maxy = fmaxf(r.maxy, s[w].maxy);
    r.nonfinite |= s[w].nonfinite;
  }
  return r;
}

// Cells of a grid of side c over a W x H box: (int)((W + c) / c) * (int)((H + c) / c).
__device__ inline double cell_count(double W, double H, double c) { return floor((W + c) / c) * floor((H + c) / c); }

// In float64: A = bounding-box area unless given, r_exp = 1 / (2 sqrt(n / A)),
// cell side = given or sqrt(occ * A / n), nCol = (int)((W + cw) / cw), nRow
// likewise.  cap <= 0: a grid above AIDW_MAX_CELLS cells is AIDW_ECAPACITY.
// cap > 0: the side is enlarged until the grid has at most cap cells (the kNN
// result does not depend on the side, only the search cost does).  A failed
// status comes with safe scalars (one cell) so that later kernels stay in bounds.
__device__ inline GridScalars grid_scalars(float mnx, float mny, float mxx, float mxy, bool nonfinite, int64_t n,
                                           double area_in, double cw_in, double occ, int64_t cap) {
  GridScalars g{};
  g.minx = mnx;
  g.miny = mny;
  g.maxx = mxx;
  g.maxy = mxy;
  g.ncol = g.nrow = 1;
  g.ncells = 1;
  g.cw = g.cwd = 1.0;
  g.inv_cw = 0.0f;
  g.r_exp = 1.0;
  g.status = AIDW_OK;
  if (nonfinite) {
    g.status = AIDW_ENONFINITE;
    return g;
  }
  const double W = (double)mxx - (double)mnx;
  const double H = (double)mxy - (double)mny;
  const double area = area_in > 0 ? area_in : W * H;
  if (!(area > 0) || !isfinite(area)) {
    g.status = AIDW_EDEGENERATE;
    return g;
  }
  double cw = cw_in > 0 ? cw_in : sqrt(occ * area / (double)n);
  if (cap > 0 && !(cell_count(W, H, cw) <= (double)cap)) {
    // 1/c for (W/c + 1)(H/c + 1) = cap, the positive root of W H u^2 + (W + H) u + 1 - cap
    const double a = W * H, b = W + H, cc = 1.0 - (double)cap;
    const double u = a > 0 ? (-b + sqrt(b * b - 4.0 * a * cc)) / (2.0 * a) : (b > 0 ? -cc / b : 1.0);
    double c2 = u > 0 ? fmax(cw, 1.0 / u) : cw;
    for (int it = 0; it < 256 && !(cell_count(W, H, c2) <= (double)cap); ++it) c2 *= 1.0625;
    if (!(cell_count(W, H, c2) <= (double)cap)) c2 = 2.0 * fmax(W, H) + 1.0;  // one cell
    cw = c2;
  }
  const double fc = (W + cw) / cw;
  const double fr = (H + cw) / cw;
  if (!(cw > 0) || !(fc < (double)AIDW_MAX_CELLS) || !(fr < (double)AIDW_MAX_CELLS) ||
      (int64_t)fc * (int64_t)fr > AIDW_MAX_CELLS) {
    g.status = AIDW_ECAPACITY;
    return g;
  }
  g.area = area;
  g.r_exp = 1.0 / (2.0 * sqrt((double)n / area));
  g.ncol = (int32_t)fc;
  g.nrow = (int32_t)fr;
  g.ncells = (int64_t)g.ncol * g.nrow;
  g.cw = cw;
  g.inv_cw = (float)(1.0 / cw);
  g.cwd = 1.0 / (double)g.inv_cw;
  return g;
}

}  // namespace gridc
}  // namespace aidw
