// Stage 2: adaptive power (Eq. 2, 4, 5, 6) and the weighted mean of Eq. 1 over
// all n data points (Section 3.3, 4.2 of the paper).
//
// The paper's tiled kernel gives each thread one query and stages blocks of
// data points through shared memory, so that all threads of a block reuse each
// loaded point.  On CDNA the same reuse is available without LDS traffic: the
// data index is the same for every lane of a wavefront, so the compiler
// fetches each chunk of x, y, z once per wavefront with scalar loads into SGPRs
// and every VALU instruction reads the point directly as a scalar operand.
// Each lane holds Q queries, which gives Q independent dependency chains per
// data point.  Per pair (query j, point i) the lane evaluates, in float32,
//     t = (s_j qx - s_j x)^2 + (s_j qy - s_j y)^2,  w = 2^(nh_j * log2 t),
//     num += w z,  den += w,
// with s_j the smallest power of two with s_j^2 d1sq_j >= 1 (d1 = nearest-neighbour
// distance) and nh_j = -alpha_j / 2.  Scaling by a power of two is exact, so t is
// the float32 d^2 times s_j^2: the common factor s_j^-alpha cancels in num / den,
// w stays <= ~1 (no overflow for any alpha) and the argument of log2 stays near 1
// for the dominant near points, where the hardware log2 is most accurate.
// The float32 sums of each tile of kTile points are folded into (hi, lo)
// two-sum pairs; the final num / den is formed in float64.  Splitting the data
// axis (blockIdx.y) gives more wavefronts when m is small; the splits' float64
// partials are then combined in split order by a second kernel.
//
// Integer powers.  With the usual levels most queries have alpha saturated at
// a level (mu <= 0.1 or >= 0.9, Eq. 6), and when that level is an integer p the
// weight is w = (d1 / d)^p = r^p with r = rsq(t): one transcendental and a few
// multiplies instead of log2 + exp2.  A prologue kernel evaluates Eq. 4-6 per
// query and keys each query by its class (p in 1..8 when alpha == p exactly,
// else 0); a sort by key groups the classes, and in the one pair launch a block
// whose queries all share an integer class runs that class's loop, any other
// block the general loop.  Which path a query takes depends only on the inputs,
// so results stay deterministic.
#include <float.h>

#include "aidw_internal.h"
#include "knn_core.h"
#include "pair_core.h"

namespace aidw {

namespace {

using pair::alpha_class;
using pair::fuzzy_mu;
using pair::kChunk;
using pair::kMaxIntPow;
using pair::kThreads;
using pair::Lane;
using pair::level_alpha;

// Eq. 4-6 per query (float64), the query's class key and the identity permutation; a query
// with d1sq = 0 (coincident with a data point) is appended to list (count cleared before).
__global__ __launch_bounds__(256) void k_alpha_class(const float* __restrict__ r_obs, int m, AlphaParams ap,
                                                     float* __restrict__ alpha_f, float* __restrict__ alpha_out,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                     const float* __restrict__ d1sq, uint32_t* __restrict__ count,
                                                     uint32_t* __restrict__ list) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  if (d1sq[q] == 0.0f) list[atomicAdd(count, 1u)] = (uint32_t)q;
  const double R = (double)r_obs[q] / alpha_r_exp(ap);                           // Eq. 4
  const double alpha = level_alpha(fuzzy_mu(R, ap.r_min, ap.r_max), ap.levels);  // Eq. 5, 6
  const float af = (float)alpha;
  alpha_f[q] = af;
  if (alpha_out) alpha_out[q] = af;
  keys[q] = alpha_class(alpha);
  vals[q] = (uint32_t)q;
}

// Eq. 4: the nearest-neighbour statistic R = r_obs / r_exp of each query, capped at clip.
__global__ __launch_bounds__(256) void k_nn_statistic(const float* __restrict__ r_obs, int m, double r_exp,
                                                      double clip, float* __restrict__ R) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const double v = (double)r_obs[q] / r_exp;
  R[q] = (float)(clip > 0.0 ? fmin(v, clip) : v);
}

// The class key of a given alpha, the identity permutation and the coincident-query list (as
// k_alpha_class).
__global__ __launch_bounds__(256) void k_class_keys(const float* __restrict__ alpha_f, int m,
                                                    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    const float* __restrict__ d1sq, uint32_t* __restrict__ count,
                                                    uint32_t* __restrict__ list) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  if (d1sq[q] == 0.0f) list[atomicAdd(count, 1u)] = (uint32_t)q;
  const float a = alpha_f[q];
  uint32_t key = 0;
  if (a >= 1.0f && a <= (float)kMaxIntPow && a == floorf(a)) key = (uint32_t)a;
  keys[q] = key;
  vals[q] = (uint32_t)q;
}

// One block: the Q * kThreads queries at positions pos0 ... of the class order (slot (j,
// thread) -> position -> query perm[position]) against the data range of split blockIdx.y,
// with the power-POW weight (POW = 0: general alpha).
template <int Q, int POW>
__device__ __forceinline__ void interp_block(const float* __restrict__ x, const float* __restrict__ y,
                                             const float* __restrict__ z, int n, int chunk,
                                             const float* __restrict__ qx, const float* __restrict__ qy,
                                             const float* __restrict__ alpha_f, const float* __restrict__ d1sq,
                                             const uint32_t* __restrict__ perm, int m, int pos0,
                                             float* __restrict__ qz, double2* __restrict__ partial) {
  Lane<Q, POW> L;
  const int split = blockIdx.y;
  uint32_t qid[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int pos = pos0 + j * kThreads + threadIdx.x;
    qid[j] = 0xffffffffu;
    if (pos < m) {
      const uint32_t q = perm[pos];
      qid[j] = q;
      L.set(j, qx[q], qy[q], alpha_f[q], d1sq[q]);
    } else {
      L.clear(j);
    }
  }
  const int lo = split * chunk;
  pair::pair_range<Q, POW>(L, x, y, z, lo, min(n, lo + chunk));

#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (qid[j] == 0xffffffffu) continue;
    const double num = L.num(j);
    const double den = L.den(j);
    if (gridDim.y == 1)
      qz[qid[j]] = (float)(num / den);
    else
      partial[(size_t)split * m + qid[j]] = make_double2(num, den);
  }
}

// The pair kernel, one launch for every alpha class: a block whose queries all have the
// integer class p (fast_mask bit p set) runs the power-p loop, any other block (general
// alpha, or a block that spans two classes) the general loop.  Class 0 sorts first, so the
// costlier general blocks are dispatched first.
template <int Q>
__global__ __launch_bounds__(kThreads) void k_interp(const float* __restrict__ x, const float* __restrict__ y,
                                                     const float* __restrict__ z, int n, int chunk,
                                                     const float* __restrict__ qx, const float* __restrict__ qy,
                                                     const float* __restrict__ alpha_f,
                                                     const float* __restrict__ d1sq,
                                                     const uint32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ skeys, int m, uint32_t fast_mask,
                                                     float* __restrict__ qz, double2* __restrict__ partial,
                                                     const GridScalars* __restrict__ gs) {
  if (gs && gs->status != AIDW_OK) return;  // a failed grid build: no result to compute
  const int pos0 = blockIdx.x * kThreads * Q;
  const int posl = min(m, pos0 + kThreads * Q) - 1;
  const uint32_t k0 = skeys[pos0], kl = skeys[posl];
  const uint32_t cls = (k0 == kl && ((fast_mask >> k0) & 1u)) ? k0 : 0u;
  switch (cls) {
#define AIDW_CASE(P)                                                                                        \
  case P:                                                                                                   \
    interp_block<Q, P>(x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, m, pos0, qz, partial);               \
    break;
    AIDW_CASE(1)
    AIDW_CASE(2)
    AIDW_CASE(3)
    AIDW_CASE(4)
    AIDW_CASE(5)
    AIDW_CASE(6)
    AIDW_CASE(7)
    AIDW_CASE(8)
#undef AIDW_CASE
    default:
      interp_block<Q, 0>(x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, m, pos0, qz, partial);
  }
}

// The untiled kernel the paper compares its tiled kernel against (Section 4.2): one
// query per lane, and every lane reads each data point from global memory itself.
// lane_stride is 0 at run time; the compiler cannot prove the address uniform, so the
// loads stay per-lane vector loads instead of the wavefront-shared scalar stream of
// k_interp.  Same per-query state, weight form (general alpha) and tile folds as
// k_interp with one data range, hence the same sums bit for bit.
__global__ __launch_bounds__(kThreads) void k_interp_naive(const float* __restrict__ x, const float* __restrict__ y,
                                                           const float* __restrict__ z, int n,
                                                           const float* __restrict__ qx, const float* __restrict__ qy,
                                                           const float* __restrict__ alpha_f,
                                                           const float* __restrict__ d1sq, int m, int lane_stride,
                                                           float* __restrict__ qz) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  Lane<1, 0> L;
  L.set(0, qx[q], qy[q], alpha_f[q], d1sq[q]);
  const int off = lane_stride * (int)threadIdx.x;
  for (int i = 0; i < n; ++i) {
    L.pair(x[i + off], y[i + off], z[i + off]);
    if (((i + 1) & (pair::kTile - 1)) == 0) L.fold();
  }
  L.fold();
  qz[q] = (float)(L.num(0) / L.den(0));
}

// Copies the data into zero-padded arrays of interp_padded_len(n) points; clears *zero_word
// (may be null) on the way.
__global__ __launch_bounds__(256) void k_pad_copy(const float* __restrict__ x, const float* __restrict__ y,
                                                  const float* __restrict__ z, int n, int npad,
                                                  float* __restrict__ xp, float* __restrict__ yp,
                                                  float* __restrict__ zp, uint32_t* __restrict__ zero_word) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (zero_word && i == 0) *zero_word = 0u;
  if (i >= npad) return;
  const bool in = i < n;
  xp[i] = in ? x[i] : 0.0f;
  yp[i] = in ? y[i] : 0.0f;
  zp[i] = in ? z[i] : 0.0f;
}

__global__ __launch_bounds__(256) void k_combine(const double2* __restrict__ partial, int m, int split,
                                                 float* __restrict__ qz) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  double num = 0.0, den = 0.0;
  for (int s = 0; s < split; ++s) {
    const double2 v = partial[(size_t)s * m + q];
    num += v.x;
    den += v.y;
  }
  qz[q] = (float)(num / den);
}

// Coincident query = mean z of the data points at its exact position (the limit
// of Eq. 1).  Those points share the query's cell; the cell is ordered by index,
// so the sum runs in index order.
__global__ __launch_bounds__(256) void k_fixup_grid(const uint32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ list, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const GridScalars* __restrict__ gs,
                                                    const int32_t* __restrict__ cell_start,
                                                    const float* __restrict__ sx, const float* __restrict__ sy,
                                                    const int32_t* __restrict__ sidx, const float* __restrict__ z,
                                                    float* __restrict__ qz) {
  if (gs->status != AIDW_OK) return;
  const uint32_t cnt = *count;
  const knn::View g{gs->minx, gs->miny, gs->inv_cw, gs->ncol, gs->nrow, gs->cwd};
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += gridDim.x * blockDim.x) {
    const uint32_t q = list[e];
    float v;
    if (knn::coincident_mean(g, cell_start, sx, sy, sidx, z, qx[q], qy[q], v)) qz[q] = v;
  }
}

// Same without a grid: one block per listed query scans all n points; per-thread
// float64 sums in stride order, then a fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_fixup_scan(const uint32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ list, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const float* __restrict__ x,
                                                    const float* __restrict__ y, const float* __restrict__ z, int n,
                                                    float* __restrict__ qz) {
  __shared__ double ss[256];
  __shared__ int sc[256];
  const uint32_t cnt = *count;
  for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
    const uint32_t q = list[e];
    const float fx = qx[q], fy = qy[q];
    double s = 0.0;
    int hits = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      if (x[i] == fx && y[i] == fy) {
        s += (double)z[i];
        ++hits;
      }
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = hits;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        ss[threadIdx.x] += ss[threadIdx.x + w];
        sc[threadIdx.x] += sc[threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0 && sc[0] > 0) qz[q] = (float)(ss[0] / sc[0]);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_alpha_class(const float* r_obs, int m, const AlphaParams& ap, float* alpha_f, float* alpha_out,
                              uint32_t* keys, uint32_t* vals, const float* d1sq, uint32_t* count, uint32_t* list,
                              hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpha_class, dim3((m + 255) / 256), dim3(256), 0, s, r_obs, m, ap, alpha_f, alpha_out, keys,
                     vals, d1sq, count, list);
  return hipGetLastError();
}

hipError_t launch_nn_statistic(const float* r_obs, int m, double r_exp, double clip, float* R, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nn_statistic, dim3((m + 255) / 256), dim3(256), 0, s, r_obs, m, r_exp, clip, R);
  return hipGetLastError();
}

hipError_t launch_class_keys(const float* alpha_f, int m, uint32_t* keys, uint32_t* vals, const float* d1sq,
                             uint32_t* count, uint32_t* list, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_class_keys, dim3((m + 255) / 256), dim3(256), 0, s, alpha_f, m, keys, vals, d1sq, count, list);
  return hipGetLastError();
}

namespace {

template <int Q>
hipError_t launch_q(dim3 grid, hipStream_t s, const float* x, const float* y, const float* z, int n, int chunk,
                    const float* qx, const float* qy, const float* alpha_f, const float* d1sq, const uint32_t* perm,
                    const uint32_t* skeys, int m, uint32_t mask, float* qz, double2* partial,
                    const GridScalars* gs) {
  hipLaunchKernelGGL((k_interp<Q>), grid, dim3(kThreads), 0, s, x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, skeys,
                     m, mask, qz, partial, gs);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_interp(const float* x, const float* y, const float* z, int n, const float* qx, const float* qy,
                         const float* alpha_f, const float* d1sq, const uint32_t* perm, const uint32_t* skeys, int m,
                         uint32_t fast_mask, int q, int split, float* qz, double2* partial, const GridScalars* gs,
                         hipStream_t s) {
  if (m <= 0) return hipSuccess;
  int chunk = (n + split - 1) / split;
  chunk = (chunk + kChunk - 1) / kChunk * kChunk;
  const dim3 grid((m + kThreads * q - 1) / (kThreads * q), split);
  fast_mask &= ((1u << (kMaxIntPow + 1)) - 2u);
  switch (q) {
    case 1: return launch_q<1>(grid, s, x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, skeys, m, fast_mask, qz, partial, gs);
    case 2: return launch_q<2>(grid, s, x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, skeys, m, fast_mask, qz, partial, gs);
    case 4: return launch_q<4>(grid, s, x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, skeys, m, fast_mask, qz, partial, gs);
    case 8: return launch_q<8>(grid, s, x, y, z, n, chunk, qx, qy, alpha_f, d1sq, perm, skeys, m, fast_mask, qz, partial, gs);
    default: return hipErrorInvalidValue;
  }
}

int interp_padded_len(int n) { return pair::padded_len(n); }

hipError_t launch_interp_naive(const float* x, const float* y, const float* z, int n, const float* qx, const float* qy,
                               const float* alpha_f, const float* d1sq, int m, float* qz, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_naive, dim3((m + kThreads - 1) / kThreads), dim3(kThreads), 0, s, x, y, z, n, qx, qy,
                     alpha_f, d1sq, m, 0, qz);
  return hipGetLastError();
}

hipError_t launch_pad_copy(const float* x, const float* y, const float* z, int n, float* xp, float* yp, float* zp,
                           uint32_t* zero_word, hipStream_t s) {
  const int npad = interp_padded_len(n);
  hipLaunchKernelGGL(k_pad_copy, dim3((npad + 255) / 256), dim3(256), 0, s, x, y, z, n, npad, xp, yp, zp, zero_word);
  return hipGetLastError();
}

hipError_t launch_combine(const double2* partial, int m, int split, float* qz, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3((m + 255) / 256), dim3(256), 0, s, partial, m, split, qz);
  return hipGetLastError();
}

hipError_t launch_fixup_grid(const uint32_t* count, const uint32_t* list, const float* qx, const float* qy,
                             const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                             const int32_t* sidx, const float* z, float* qz, hipStream_t s) {
  hipLaunchKernelGGL(k_fixup_grid, dim3(64), dim3(256), 0, s, count, list, qx, qy, gs, cell_start, sx, sy, sidx, z,
                     qz);
  return hipGetLastError();
}

hipError_t launch_fixup_scan(const uint32_t* count, const uint32_t* list, const float* qx, const float* qy,
                             const float* x, const float* y, const float* z, int n, float* qz, hipStream_t s) {
  hipLaunchKernelGGL(k_fixup_scan, dim3(256), dim3(256), 0, s, count, list, qx, qy, x, y, z, n, qz);
  return hipGetLastError();
}

}  // namespace aidw
