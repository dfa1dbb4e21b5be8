// Device code shared by the pair kernels of the single-job path (interp.hip) and the
// batched path (batch.hip): Eq. 4-6 per query, and the compensated accumulation of
// the Eq. 1 sums over a range of data points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aidw {
namespace pair {

#ifndef AIDW_CHUNK
#define AIDW_CHUNK 8
#endif
constexpr int kThreads = 256;       // queries per workgroup (times Q)
constexpr int kChunk = AIDW_CHUNK;  // data points per scalar fetch
constexpr int kTile = 256;          // data points per float32 partial before the two-sum fold
constexpr int kMaxIntPow = 8;       // integer alpha classes with a dedicated loop

// Eq. 5 as printed: 0 below R_min, 1 above R_max, else 0.5 - 0.5 cos(pi / R_max (R - R_min)).
__device__ inline double fuzzy_mu(double R, double rmin, double rmax) {
  if (R <= rmin) return 0.0;
  if (R >= rmax) return 1.0;
  return 0.5 - 0.5 * cos((M_PI / rmax) * (R - rmin));
}

// Eq. 6: piecewise-linear between the levels at mu = 0.1, 0.3, 0.5, 0.7, 0.9, constant outside.
__device__ inline double level_alpha(double mu, const double* a) {
  if (mu <= 0.1) return a[0];
  if (mu <= 0.3) return a[0] * (1.0 - 5.0 * (mu - 0.1)) + 5.0 * a[1] * (mu - 0.1);
  if (mu <= 0.5) return 5.0 * a[2] * (mu - 0.3) + a[1] * (1.0 - 5.0 * (mu - 0.3));
  if (mu <= 0.7) return a[2] * (1.0 - 5.0 * (mu - 0.5)) + 5.0 * a[3] * (mu - 0.5);
  if (mu <= 0.9) return 5.0 * a[4] * (mu - 0.7) + a[3] * (1.0 - 5.0 * (mu - 0.7));
  return a[4];
}

// Pair-kernel class of an alpha: p when alpha is exactly the integer p in 1..kMaxIntPow, else 0.
__device__ inline uint32_t alpha_class(double alpha) {
  if (alpha >= 1.0 && alpha <= (double)kMaxIntPow && alpha == floor(alpha)) return (uint32_t)alpha;
  return 0u;
}

struct Acc {
  float num_t, den_t;  // current tile
  float num_h, num_l;  // folded: two-sum hi / lo
  float den_h, den_l;
};

__device__ inline void two_sum_fold(float& hi, float& lo, float v) {
  const float s = hi + v;
  const float bp = s - hi;
  const float err = (hi - (s - bp)) + (v - bp);
  hi = s;
  lo += err;
}

// w = r^P by repeated squaring (P known at compile time).
template <int P>
__device__ inline float ipow(float r) {
  if constexpr (P == 1) {
    return r;
  } else if constexpr (P % 2 == 0) {
    const float h = ipow<P / 2>(r);
    return h * h;
  } else {
    return ipow<P - 1>(r) * r;
  }
}

// Scale of a query: s = 2^k, the smallest power of two with s^2 * d1sq >= 1
// (d1sq = the query's nearest squared distance; 1 when d1sq is 0 or not finite).
__device__ inline float pow2_scale(float d1sq) {
  if (!(d1sq > 0.0f) || !(d1sq <= 3.402823466e38f)) return 1.0f;
  int e;
  (void)frexpf(d1sq, &e);       // d1sq = m 2^e, m in [0.5, 1)
  int k = (1 - e + 1) >> 1;     // ceil((1 - e) / 2): m 2^(2k + e) in [1, 4)
  k = k < -64 ? -64 : (k > 64 ? 64 : k);
  return ldexpf(1.0f, k);
}

// Per-lane state of Q queries.  The weight of Eq. 1 is evaluated on the
// query's scaled squared distance t = s^2 d^2 (s = pow2_scale(d1sq)):
//   dx s = fma(x, -s, qx s), dy s likewise, t = fma(dx s, dx s, (dy s)^2),
// which is exactly s^2 times the float32 d^2 = fma(dx, dx, dy dy) because
// scaling by a power of two commutes with rounding; t >= 1 for every data
// point (up to one rounding of d1sq), so the weights w = t^(-alpha/2) stay
// <= ~1 for any alpha, and the common factor s^-alpha cancels between the
// numerator and the denominator.  POW = 0: general alpha, w = 2^(nh log2 t)
// with nh = -alpha/2; POW = p > 0: alpha == p, w = rsq(t)^p.
template <int Q, int POW>
struct Lane {
  float qxs[Q], qys[Q], ns[Q], nh[Q];
  Acc acc[Q];

  __device__ inline void pair(float x, float y, float z) {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const float dx = __builtin_fmaf(x, ns[j], qxs[j]);
      const float dy = __builtin_fmaf(y, ns[j], qys[j]);
      const float t = __builtin_fmaf(dx, dx, dy * dy);
      float w;
      if constexpr (POW == 0)
        w = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(t) * nh[j]);
      else
        w = ipow<POW>(__builtin_amdgcn_rsqf(t));
      acc[j].num_t = __builtin_fmaf(w, z, acc[j].num_t);
      acc[j].den_t += w;
    }
  }
  __device__ inline void fold() {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      two_sum_fold(acc[j].num_h, acc[j].num_l, acc[j].num_t);
      two_sum_fold(acc[j].den_h, acc[j].den_l, acc[j].den_t);
      acc[j].num_t = 0.0f;
      acc[j].den_t = 0.0f;
    }
  }
  // Query j at (fx, fy) with alpha a and nearest squared distance d1 (0: coincident
  // query, whose sums are replaced by the fix-up, so any finite scale serves).
  __device__ inline void set(int j, float fx, float fy, float a, float d1) {
    const float sc = pow2_scale(d1);
    qxs[j] = fx * sc;
    qys[j] = fy * sc;
    ns[j] = -sc;
    nh[j] = -0.5f * a;
    acc[j] = Acc{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  }
  // Unused slot: finite values, result discarded.
  __device__ inline void clear(int j) {
    qxs[j] = 0.0f;
    qys[j] = 0.0f;
    ns[j] = -1.0f;
    nh[j] = 0.0f;
    acc[j] = Acc{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  }
  __device__ inline double num(int j) const { return (double)acc[j].num_h + (double)acc[j].num_l; }
  __device__ inline double den(int j) const { return (double)acc[j].den_h + (double)acc[j].den_l; }
};

// Accumulates the data points [lo, hi) into L, kChunk points per wave-uniform
// fetch, folding the float32 tile sums every kTile points and once at the end.
// x, y, z must stay readable for kChunk points past the last full chunk (the
// prefetch of the chunk after it).
template <int Q, int POW>
__device__ __forceinline__ void pair_range(Lane<Q, POW>& L, const float* __restrict__ x,
                                           const float* __restrict__ y, const float* __restrict__ z, int lo, int hi) {
  const int nfull = hi > lo ? (hi - lo) / kChunk : 0;
  constexpr int kFoldMask = kTile / kChunk - 1;
  // Double-buffered: each iteration fetches the next chunk while it evaluates the
  // current one, and the compiler is left free to place the fetch (pinning it to
  // the top of the loop bunches the scalar work and measured slower).  The copy of
  // the fetched chunk into the working registers stays: two buffers used in turn (no
  // copies) measured ~11 % slower, because scalar loads complete out of order, so the
  // wait before one buffer's use also waits for the fetch just issued into the other.
  if (nfull > 0) {
    float cx[kChunk], cy[kChunk], cz[kChunk];
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
      cx[i] = x[lo + i];
      cy[i] = y[lo + i];
      cz[i] = z[lo + i];
    }
    for (int ci = 0; ci < nfull; ++ci) {
      const int pn = lo + (ci + 1) * kChunk;
      float nx[kChunk], ny[kChunk], nz[kChunk];
#pragma unroll
      for (int i = 0; i < kChunk; ++i) {
        nx[i] = x[pn + i];
        ny[i] = y[pn + i];
        nz[i] = z[pn + i];
      }

#pragma unroll
      for (int i = 0; i < kChunk; ++i) L.pair(cx[i], cy[i], cz[i]);
      if (((ci + 1) & kFoldMask) == 0) L.fold();
#pragma unroll
      for (int i = 0; i < kChunk; ++i) {
        cx[i] = nx[i];
        cy[i] = ny[i];
        cz[i] = nz[i];
      }
    }
  }
  for (int p = lo + nfull * kChunk; p < hi; ++p) L.pair(x[p], y[p], z[p]);
  L.fold();
}

// Zero-padded length of a data array read by pair_range over [0, n).
__host__ __device__ inline int padded_len(int n) { return (n + kChunk - 1) / kChunk * kChunk + kChunk; }

}  // namespace pair
}  // namespace aidw
