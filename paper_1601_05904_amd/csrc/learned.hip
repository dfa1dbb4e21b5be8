// Learned-R form: a small network predicts the nearest-neighbour statistic R of
// Eq. 4 from the grid's occupancy around each query, so that most queries skip
// the kNN search of Section 3.2.4; exact kNN remains the fallback wherever the
// prediction could change alpha (Eq. 5, 6).
//
// Network (27 -> 64 -> 64 -> 1):
//   x  = bf16(features)                     (5 x 5 cell counts / mean occupancy, in-cell offsets)
//   h1 = bf16(gelu(W1 x + b1)),  h2 = bf16(gelu(W2 h1 + b2)),  y = W3 h2 + b3
// with bf16 weights and activations as operands and float32 accumulation, gelu
// the tanh form u / 2 (1 + tanh(sqrt(2 / pi) (u + 0.044715 u^3))).  Inference
// (the learned run's fused front and aidw_mlp_forward) runs the network on the
// matrix cores (see mlp_tile).  Training: per-sample forward and backward in one
// kernel (one sample per lane, v_dot2c_f32_bf16 dot products whose weight pairs,
// the same for every lane, are scalar operands), the weight gradients summed
// over the batch in a fixed order, then Adam on the float32 master weights and a
// repack of the bf16 copies.
#include <float.h>

#include "aidw_internal.h"

namespace aidw {

namespace {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

constexpr int kIn = 27;
constexpr int kInPairs = 14;  // 27 inputs + one zero pad
constexpr int kH = 64;
constexpr int kHPairs = 32;

typedef float float2v_t __attribute__((ext_vector_type(2)));

// float32 -> bfloat16, round to nearest, ties to even (the hardware conversion)
__device__ inline uint32_t bf16_bits(float f) { return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ inline float bf16_round(float f) { return (float)(__bf16)f; }
__device__ inline uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v_t{lo, hi}, bf16x2_t));
}
__device__ inline float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
}

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

__device__ inline float tanh_f(float v) {
  // tanh(v) = 1 - 2 / (exp(2v) + 1); exp overflow gives 1, underflow gives -1
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * v);  // 2 / ln 2
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}
// 0.5 u (1 + tanh(v)), v = c (u + a u^3), evaluated as u - u / (1 + e^(2 v)) (the same
// function): 2 v log2(e) = u (K1 + K2 u^2)
constexpr float kGeluK1 = (float)(2.0 * 0.7978845608028654 * 1.4426950408889634);
constexpr float kGeluK2 = (float)(2.0 * 0.7978845608028654 * 0.044715 * 1.4426950408889634);
__device__ inline float gelu_f(float u) {
  const float z = u * __builtin_fmaf(kGeluK2, u * u, kGeluK1);
  return __builtin_fmaf(-u, __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(z) + 1.0f), u);
}
__device__ inline float gelu_grad_f(float u) {
  const float t = tanh_f(kGeluC * (u + kGeluA * u * u * u));
  return 0.5f * (1.0f + t) + 0.5f * u * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * u * u);
}

__device__ inline int clamp_cell(float t, int nc) {
  if (!(t >= 0.0f)) return 0;
  if (t >= 2147483520.0f) return nc - 1;
  const int c = (int)t;
  return c > nc - 1 ? nc - 1 : c;
}

// ---- features -------------------------------------------------------------------

// Per query: 25 cell counts of the 5 x 5 block around its cell (0 outside the grid)
// times nCells / n, its in-cell offsets, and d1sq: the exact squared distance to its
// nearest data point when that point lies in the surrounding 3 x 3 block of cells
// and nearer than the block's open sides, otherwise a lower bound (the squared
// distance to those sides).  d1sq is exactly 0 iff the query coincides with a point.
__global__ __launch_bounds__(256) void k_features(const GridScalars* __restrict__ gs,
                                                  const int32_t* __restrict__ cell_start,
                                                  const float* __restrict__ sx, const float* __restrict__ sy,
                                                  const float* __restrict__ qx, const float* __restrict__ qy,
                                                  const uint32_t* __restrict__ perm, int m, int64_t n,
                                                  float* __restrict__ feat, float* __restrict__ d1sq) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const double inv_occ = (double)gs->ncells / (double)n;
  const double slack = slack_cells(gs->ncol, gs->nrow);
  const int q = perm ? (int)perm[t] : t;
  const float minx = gs->minx, miny = gs->miny, inv = gs->inv_cw;
  const int ncol = gs->ncol, nrow = gs->nrow;
  const float fx = qx[q], fy = qy[q];
  const float tx = (fx - minx) * inv;
  const float ty = (fy - miny) * inv;
  const int c0 = clamp_cell(tx, ncol), r0 = clamp_cell(ty, nrow);
  float* f = feat + (size_t)t * kIn;
#pragma unroll
  for (int dr = -2; dr <= 2; ++dr) {
    const int r = r0 + dr;
    // the six offsets bounding the row's five cells (clipped to the row)
    int off[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      int c = c0 - 2 + e;
      c = c < 0 ? 0 : (c > ncol ? ncol : c);
      off[e] = (r >= 0 && r < nrow) ? cell_start[r * ncol + c] : 0;
    }
#pragma unroll
    for (int dc = -2; dc <= 2; ++dc) {
      const int c = c0 + dc;
      const int cnt = (c >= 0 && c < ncol) ? off[dc + 3] - off[dc + 2] : 0;
      f[(dr + 2) * 5 + (dc + 2)] = (float)((double)cnt * inv_occ);
    }
  }
  f[25] = tx - (float)c0;
  f[26] = ty - (float)r0;
  if (!d1sq) return;
  // nearest point in the 3 x 3 block
  const double px = fx, py = fy;
  double best = INFINITY;
  const int ca = c0 > 0 ? c0 - 1 : 0, cb = c0 + 1 < ncol ? c0 + 1 : ncol - 1;
  for (int r = r0 - 1; r <= r0 + 1; ++r) {
    if (r < 0 || r >= nrow) continue;
    const int p1 = cell_start[r * ncol + cb + 1];
    for (int p = cell_start[r * ncol + ca]; p < p1; ++p) {
      const double dx = (double)sx[p] - px;
      const double dy = (double)sy[p] - py;
      const double d2 = dx * dx + dy * dy;
      best = d2 < best ? d2 : best;
    }
  }
  const double cwd = gs->cwd, minxd = minx, minyd = miny;
  double dout = INFINITY;
  if (c0 - 1 > 0) dout = fmin(dout, px - (minxd + (double)(c0 - 1) * cwd));
  if (c0 + 1 < ncol - 1) dout = fmin(dout, (minxd + (double)(c0 + 2) * cwd) - px);
  if (r0 - 1 > 0) dout = fmin(dout, py - (minyd + (double)(r0 - 1) * cwd));
  if (r0 + 1 < nrow - 1) dout = fmin(dout, (minyd + (double)(r0 + 2) * cwd) - py);
  dout -= slack * cwd;
  double v;
  if (dout == INFINITY || best < dout * dout)
    v = best;                       // exact nearest distance
  else
    v = dout > 0 ? dout * dout : 0; // lower bound
  d1sq[t] = v == 0.0 ? (best == 0.0 ? 0.0f : FLT_MIN) : fmaxf((float)v, FLT_MIN);
}

// ---- network ------------------------------------------------------------------------

// Layer weights in the kernels' layout: bf16 pairs for the forward, float32 values of
// the rounded weights for the backward.
struct MlpWeights {
  const uint32_t* w1p;  // [64][14]
  const uint32_t* w2p;  // [64][32]
  const uint32_t* w3p;  // [32]
  const float* w2r;     // [64][64]
  const float* w3r;     // [64]
  const float* master;  // float32 parameters (biases are read from here)
};

constexpr int kOffW1 = 0, kOffB1 = 64 * 27, kOffW2 = kOffB1 + 64, kOffB2 = kOffW2 + 64 * 64, kOffW3 = kOffB2 + 64,
              kOffB3 = kOffW3 + 64, kParams = kOffB3 + 1;
static_assert(kParams == AIDW_MLP_PARAMS, "parameter layout");

__device__ inline void load_x(const float* __restrict__ f, uint32_t* xp) {
#pragma unroll
  for (int p = 0; p < kInPairs; ++p) {
    const float lo = f[2 * p];
    const float hi = 2 * p + 1 < kIn ? f[2 * p + 1] : 0.0f;
    xp[p] = pack_bf16(lo, hi);
  }
}

// a1 = W1 x + b1 for one output row
__device__ inline float layer1_row(const MlpWeights& w, const uint32_t* xp, int o) {
  float acc = w.master[kOffB1 + o];
#pragma unroll
  for (int p = 0; p < kInPairs; ++p) acc = dot2(w.w1p[o * kInPairs + p], xp[p], acc);
  return acc;
}
__device__ inline float layer2_row(const MlpWeights& w, const uint32_t* hp, int o) {
  float acc = w.master[kOffB2 + o];
#pragma unroll
  for (int p = 0; p < kHPairs; ++p) acc = dot2(w.w2p[o * kHPairs + p], hp[p], acc);
  return acc;
}
__device__ inline float layer3(const MlpWeights& w, const uint32_t* hp) {
  float acc = w.master[kOffB3];
#pragma unroll
  for (int p = 0; p < kHPairs; ++p) acc = dot2(w.w3p[p], hp[p], acc);
  return acc;
}

// One sample per lane: forward, loss term, and the per-sample backward down to the
// pre-activation gradients; saves the operands of the weight gradients, sample-major.
__global__ __launch_bounds__(64) void k_mlp_train_sample(MlpWeights w, const float* __restrict__ feat,
                                                         const float* __restrict__ target,
                                                         const uint32_t* __restrict__ sel, int B, float two_over_b,
                                                         float* __restrict__ s_x, float* __restrict__ s_h1,
                                                         float* __restrict__ s_h2, float* __restrict__ s_da1,
                                                         float* __restrict__ s_da2, float* __restrict__ s_dy,
                                                         float* __restrict__ s_err2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int j = sel ? (int)sel[b] : b;
  uint32_t xp[kInPairs], h1p[kHPairs], h2p[kHPairs];
  float a1[kH], a2[kH];
  load_x(feat + (size_t)j * kIn, xp);
#pragma unroll
  for (int o = 0; o < kH; o += 2) {
    a1[o] = layer1_row(w, xp, o);
    a1[o + 1] = layer1_row(w, xp, o + 1);
    h1p[o / 2] = pack_bf16(gelu_f(a1[o]), gelu_f(a1[o + 1]));
  }
#pragma unroll
  for (int o = 0; o < kH; o += 2) {
    a2[o] = layer2_row(w, h1p, o);
    a2[o + 1] = layer2_row(w, h1p, o + 1);
    h2p[o / 2] = pack_bf16(gelu_f(a2[o]), gelu_f(a2[o + 1]));
  }
  const float y = layer3(w, h2p);
  const float err = y - target[j];
  const float dy = two_over_b * err;
  s_dy[b] = dy;
  s_err2[b] = err * err;
#pragma unroll
  for (int p = 0; p < kInPairs; ++p) {
    s_x[(size_t)b * 28 + 2 * p] = __uint_as_float(xp[p] << 16);
    s_x[(size_t)b * 28 + 2 * p + 1] = __uint_as_float(xp[p] & 0xFFFF0000u);
  }
#pragma unroll
  for (int p = 0; p < kHPairs; ++p) {
    s_h1[(size_t)b * kH + 2 * p] = __uint_as_float(h1p[p] << 16);
    s_h1[(size_t)b * kH + 2 * p + 1] = __uint_as_float(h1p[p] & 0xFFFF0000u);
    s_h2[(size_t)b * kH + 2 * p] = __uint_as_float(h2p[p] << 16);
    s_h2[(size_t)b * kH + 2 * p + 1] = __uint_as_float(h2p[p] & 0xFFFF0000u);
  }
  // da2 = dy * W3 * gelu'(a2)
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    a2[i] = dy * w.w3r[i] * gelu_grad_f(a2[i]);
    s_da2[(size_t)b * kH + i] = a2[i];
  }
  // da1 = (W2^T da2) * gelu'(a1)
#pragma unroll
  for (int c = 0; c < kH; ++c) {
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < kH; ++i) acc = __builtin_fmaf(w.w2r[i * kH + c], a2[i], acc);
    s_da1[(size_t)b * kH + c] = acc * gelu_grad_f(a1[c]);
  }
}

// Weight gradients: grad[p] = sum over the batch of the parameter's two operands;
// grad[kParams] = mean squared error of the batch.  The batch is cut into
// kGradChunks contiguous chunks (blockIdx.y); each chunk's sum runs in sample
// order, then k_mlp_wgrad_sum adds the chunks in chunk order.
constexpr int kGradChunks = 16;

__global__ __launch_bounds__(256) void k_mlp_wgrad(int B, const float* __restrict__ s_x,
                                                   const float* __restrict__ s_h1, const float* __restrict__ s_h2,
                                                   const float* __restrict__ s_da1, const float* __restrict__ s_da2,
                                                   const float* __restrict__ s_dy, const float* __restrict__ s_err2,
                                                   float* __restrict__ part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kParams) return;
  const int per = (B + kGradChunks - 1) / kGradChunks;
  const int b0 = blockIdx.y * per, b1 = min(B, b0 + per);
  float acc = 0.0f;
  if (p < kOffB1) {
    const int o = p / kIn, i = p % kIn;
    for (int b = b0; b < b1; ++b) acc = __builtin_fmaf(s_da1[(size_t)b * kH + o], s_x[(size_t)b * 28 + i], acc);
  } else if (p < kOffW2) {
    const int o = p - kOffB1;
    for (int b = b0; b < b1; ++b) acc += s_da1[(size_t)b * kH + o];
  } else if (p < kOffB2) {
    const int o = (p - kOffW2) / kH, i = (p - kOffW2) % kH;
    for (int b = b0; b < b1; ++b) acc = __builtin_fmaf(s_da2[(size_t)b * kH + o], s_h1[(size_t)b * kH + i], acc);
  } else if (p < kOffW3) {
    const int o = p - kOffB2;
    for (int b = b0; b < b1; ++b) acc += s_da2[(size_t)b * kH + o];
  } else if (p < kOffB3) {
    const int i = p - kOffW3;
    for (int b = b0; b < b1; ++b) acc = __builtin_fmaf(s_dy[b], s_h2[(size_t)b * kH + i], acc);
  } else if (p == kOffB3) {
    for (int b = b0; b < b1; ++b) acc += s_dy[b];
  } else {
    for (int b = b0; b < b1; ++b) acc += s_err2[b];
  }
  part[(size_t)blockIdx.y * (kParams + 1) + p] = acc;
}

__global__ __launch_bounds__(256) void k_mlp_wgrad_sum(int B, const float* __restrict__ part,
                                                       float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kParams) return;
  float acc = 0.0f;
  for (int c = 0; c < kGradChunks; ++c) acc += part[(size_t)c * (kParams + 1) + p];
  grad[p] = p == kParams ? acc / (float)B : acc;
}

// Adam on the float32 masters.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ master, const float* __restrict__ grad,
                                              float* __restrict__ mom, float* __restrict__ vel, float lr, float b1,
                                              float b2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float g = grad[p];
  const float mm = b1 * mom[p] + (1.0f - b1) * g;
  const float vv = b2 * vel[p] + (1.0f - b2) * g * g;
  mom[p] = mm;
  vel[p] = vv;
  master[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// bf16 copies of the weights in the kernels' layout.
__global__ __launch_bounds__(256) void k_mlp_repack(const float* __restrict__ master, uint32_t* __restrict__ w1p,
                                                    uint32_t* __restrict__ w2p, uint32_t* __restrict__ w3p,
                                                    float* __restrict__ w2r, float* __restrict__ w3r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kH * kInPairs) {
    const int o = t / kInPairs, p = t % kInPairs;
    const float lo = master[kOffW1 + o * kIn + 2 * p];
    const float hi = 2 * p + 1 < kIn ? master[kOffW1 + o * kIn + 2 * p + 1] : 0.0f;
    w1p[t] = pack_bf16(lo, hi);
  }
  if (t < kH * kHPairs) {
    const int o = t / kHPairs, p = t % kHPairs;
    w2p[t] = pack_bf16(master[kOffW2 + o * kH + 2 * p], master[kOffW2 + o * kH + 2 * p + 1]);
  }
  if (t < kHPairs) w3p[t] = pack_bf16(master[kOffW3 + 2 * t], master[kOffW3 + 2 * t + 1]);
  if (t < kH * kH) w2r[t] = bf16_round(master[kOffW2 + t]);
  if (t < kH) w3r[t] = bf16_round(master[kOffW3 + t]);
}

// MFMA operands (see mlp_tile): lane = 16 g + r of tile tt holds 8 bf16 of row 16 tt + r.
//   W1: columns (inputs) 8 g .. 8 g + 7 (zero beyond the 27 inputs);
//   W2, k-step s: columns h(32 s + 8 g + j) = 16 (2 s + j / 4) + 4 g + j % 4.
__global__ __launch_bounds__(256) void k_mlp_repack_mfma(const float* __restrict__ master, uint32_t* __restrict__ w1a,
                                                         uint32_t* __restrict__ w2a, float* __restrict__ b1f,
                                                         float* __restrict__ b2f, float* __restrict__ w3f) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;  // one bf16 pair of an operand
  if (t < 4 * 64 * 4) {  // W1: [tile][lane][pair]
    const int tt = t / 256, lane = (t / 4) % 64, pr = t % 4;
    const int row = 16 * tt + lane % 16, g = lane / 16;
    float v[2];
    for (int e = 0; e < 2; ++e) {
      const int col = 8 * g + 2 * pr + e;
      v[e] = col < kIn ? master[kOffW1 + row * kIn + col] : 0.0f;
    }
    w1a[t] = pack_bf16(v[0], v[1]);
  }
  if (t < 8 * 64 * 4) {  // W2: [tile][step][lane][pair]
    const int ts = t / 256, lane = (t / 4) % 64, pr = t % 4;
    const int tt = ts / 2, st = ts % 2;
    const int row = 16 * tt + lane % 16, g = lane / 16;
    float v[2];
    for (int e = 0; e < 2; ++e) {
      const int j = 2 * pr + e;
      const int h = 16 * (2 * st + j / 4) + 4 * g + j % 4;
      v[e] = master[kOffW2 + row * kH + h];
    }
    w2a[t] = pack_bf16(v[0], v[1]);
  }
  if (t < kH) {
    b1f[t] = master[kOffB1 + t];
    b2f[t] = master[kOffB2 + t];
    w3f[t] = bf16_round(master[kOffW3 + t]);
  }
}

// Loss of batch `step` into epoch_loss[epoch] (a single thread: fixed order).
__global__ void k_accumulate_loss(const float* __restrict__ grad, float* __restrict__ epoch_loss, int epoch,
                                  float scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) epoch_loss[epoch] += grad[kParams] * scale;
}

// ---- learned run: fallback decision -----------------------------------------------------

// Per position t of the binned query order (query q = perm[t]), from the prediction
// r_hat[t] of R: fall back to exact kNN when the prediction could change alpha, else
// take alpha from the rule.
//   rule 0 (literal): fall back when |r_hat - R_min| < delta or |r_hat - R_max| < delta;
//                     other queries use alpha(mu(r_hat)) by Eq. 5, 6.
//   rule 1 (alpha-exact): skip only when r_hat >= r_sat_hi + delta (alpha = alpha_5) or
//                     r_hat <= r_sat_lo - delta (alpha = alpha_1), where mu = 0.9 / 0.1.
//   rule 2 (certified): skip only when a lower bound of r_obs (from the counts of the 5 x 5
//                     block, or the exact distances of the 3 x 3 block) proves R beyond the
//                     point where alpha saturates at alpha_5 (certified_saturated,
//                     certified_by_distances below); the network is not evaluated.
//   rule 3 (certified, then alpha-exact): skip when certified, else as rule 1.
//   rule 4 (network-gated certificate): skip only when certified, as rule 2; the 3 x 3 distance
//                     scan is tried only where the network predicts r_hat >= r_sat_hi - delta
//                     (elsewhere the query goes straight to the exact kNN), so the network
//                     never sets an alpha: every query gets the exact path's.
// Coincident queries (d1 == 0) always fall back.
__device__ inline double fuzzy_mu_l(double R, double rmin, double rmax) {
  if (R <= rmin) return 0.0;
  if (R >= rmax) return 1.0;
  return 0.5 - 0.5 * cos((M_PI / rmax) * (R - rmin));
}
__device__ inline double level_alpha_l(double mu, const double* a) {
  if (mu <= 0.1) return a[0];
  if (mu <= 0.3) return a[0] * (1.0 - 5.0 * (mu - 0.1)) + 5.0 * a[1] * (mu - 0.1);
  if (mu <= 0.5) return 5.0 * a[2] * (mu - 0.3) + a[1] * (1.0 - 5.0 * (mu - 0.3));
  if (mu <= 0.7) return a[2] * (1.0 - 5.0 * (mu - 0.5)) + 5.0 * a[3] * (mu - 0.5);
  if (mu <= 0.9) return 5.0 * a[4] * (mu - 0.7) + a[3] * (1.0 - 5.0 * (mu - 0.7));
  return a[4];
}

// The rule for one query: true = fall back to exact kNN; else *alpha is the rule's alpha.
__device__ inline bool decide_one(double R, float d1, const AlphaParams& ap, int rule, double delta, double r_sat_lo,
                                  double r_sat_hi, double* alpha) {
  *alpha = 0.0;
  if (d1 == 0.0f || !isfinite(R)) return true;
  if (rule == 0) {
    *alpha = level_alpha_l(fuzzy_mu_l(R, ap.r_min, ap.r_max), ap.levels);
    return fabs(R - ap.r_min) < delta || fabs(R - ap.r_max) < delta;
  }
  if (R >= r_sat_hi + delta) {
    *alpha = ap.levels[4];
    return false;
  }
  if (R <= r_sat_lo - delta) {
    *alpha = ap.levels[0];
    return false;
  }
  return true;
}

// Lower bound of Eq. 3 from block counts.  B_L is the block of (2L + 1)^2 cells around the
// query's cell (clipped to the grid) and c_L the number of data points binned into it; every
// point binned outside B_L lies at least D_L from the query, D_L = the distance from the query
// to the nearest side of B_L that has cells beyond it, less the binning slack (no such side:
// the block holds every point).  At most c_L of the query's neighbours lie inside B_L, so its
// j-th nearest distance is >= D_L whenever c_L < j; the k nearest distances sum to at least
// sum over L of D_L * (min(k, c_{L+1}) - min(k, c_L)), with c_3 = k.  True when that sum
// exceeds sum_min (k * r_exp * the R above which alpha = alpha_5, with a relative margin).
__device__ inline double block_side_distance(double px, double py, int c0, int r0, int L, int ncol, int nrow,
                                             double minx, double miny, double cw, double slack) {
  double d = INFINITY;
  if (c0 - L > 0) d = fmin(d, px - (minx + (double)(c0 - L) * cw));
  if (c0 + L < ncol - 1) d = fmin(d, (minx + (double)(c0 + L + 1) * cw) - px);
  if (r0 - L > 0) d = fmin(d, py - (miny + (double)(r0 - L) * cw));
  if (r0 + L < nrow - 1) d = fmin(d, (miny + (double)(r0 + L + 1) * cw) - py);
  return fmax(d - slack * cw, 0.0);
}
__device__ inline bool certified_saturated(double px, double py, int c0, int r0, int ncol, int nrow, double minx,
                                           double miny, double cw, double slack, int c_0, int c_1, int c_2, int k,
                                           double sum_min) {
  const int c[4] = {min(c_0, k), min(c_1, k), min(c_2, k), k};
  double sum = 0.0;
#pragma unroll
  for (int L = 0; L < 3; ++L) {
    const int mult = c[L + 1] - c[L];
    if (mult > 0) sum += (double)mult * block_side_distance(px, py, c0, r0, L, ncol, nrow, minx, miny, cw, slack);
  }
  return sum > sum_min;
}

// Tighter, from the exact distances of the 3 x 3 block: its points nearer than D_1 are all
// the data points within D_1 of the query (v_cnt of them, distances summing to v_sum, the
// largest v_max).  The j-th nearest distance is >= min(s_j, D_1), s_j the j-th smallest
// distance in the 3 x 3 block, and >= D_2 when c_2 < j.  With K = min(k, c_2), the K smallest
// of min(s_j, D_1) sum to v_sum + (K - v_cnt) D_1 when v_cnt < K, and to at least
// v_sum - (v_cnt - K) v_max otherwise (the v_cnt - K left out are each <= v_max); the other
// k - K terms are >= D_2.  The float32 distances are each within 2.2e-7 relative of the exact
// ones and a point within that of D_1 may be counted on either side of it: the sum is lowered
// by (3 v_cnt + k) * 5e-7 * D_1 to cover both.
__device__ inline bool certified_by_distances(double v_sum, int v_cnt, float v_max, int c_2, int k, double d_1,
                                              double d_2, double sum_min) {
  const int kk = min(k, c_2);
  double sum = v_cnt < kk ? v_sum + (double)(kk - v_cnt) * d_1 : v_sum - (double)(v_cnt - kk) * (double)v_max;
  if (k > kk) sum += (double)(k - kk) * d_2;
  return sum - (double)(3 * v_cnt + k) * 5e-7 * d_1 > sum_min;
}

// ---- inference on the matrix cores -----------------------------------------------------
//
// v_mfma_f32_16x16x32_bf16 computes D (16 x 16) = A (16 x 32) B (32 x 16) + C with, for
// lane l = 16 g + r of the wavefront: A row r, columns 8 g .. 8 g + 7; B column r, rows
// 8 g .. 8 g + 7; D column r, rows 4 g .. 4 g + 3.  The network runs transposed on a tile
// of 16 queries, H^T = W X^T, so that lane 16 g + c holds the inputs 8 g .. 8 g + 7 of query
// c (the B operand) and receives hidden units 16 t + 4 g + i (i = 0..3) of query c from
// tile t.  Layer 2 takes those as its B operand directly: its k-step s reads hidden units
// h(32 s + 8 g + j) = 16 (2 s + j / 4) + 4 g + j % 4, the order in which k_mlp_repack_mfma
// stores the columns of W2.  Layer 3 is a float32 dot over each lane's 16 hidden units and
// a sum over the 4 lanes of a query.  Operands are bf16, accumulation float32, as in the
// VALU kernels (the summation order differs).

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// The W1 and W2 operands of a workgroup, staged in LDS (12 KB): [tile][lane] and
// [tile][k-step][lane], one 16-byte operand each.
struct MfmaNet {
  const uint4* w;  // LDS
  __device__ inline bf16x8_t w1(int t, int lane) const { return __builtin_bit_cast(bf16x8_t, w[t * 64 + lane]); }
  __device__ inline bf16x8_t w2(int t, int st, int lane) const {
    return __builtin_bit_cast(bf16x8_t, w[256 + (t * 2 + st) * 64 + lane]);
  }
};
constexpr int kNetOperands = 4 * 64 + 8 * 64;

// The same operands read from global memory (through the caches), for a kernel that runs the
// network only on some of its wavefronts.
struct MfmaNetGlobal {
  const uint4* w1a;
  const uint4* w2a;
  __device__ inline bf16x8_t w1(int t, int lane) const { return __builtin_bit_cast(bf16x8_t, w1a[t * 64 + lane]); }
  __device__ inline bf16x8_t w2(int t, int st, int lane) const {
    return __builtin_bit_cast(bf16x8_t, w2a[(t * 2 + st) * 64 + lane]);
  }
};

__device__ inline bf16x8_t as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8_t, v); }

// Copies the operands into the workgroup's LDS (every thread of the workgroup calls it).
__device__ inline MfmaNet stage_net(const MlpDevice& d, uint4* lds) {
  const uint4* w1 = reinterpret_cast<const uint4*>(d.w1a);
  const uint4* w2 = reinterpret_cast<const uint4*>(d.w2a);
  for (int i = threadIdx.x; i < kNetOperands; i += blockDim.x) lds[i] = i < 256 ? w1[i] : w2[i - 256];
  __syncthreads();
  return MfmaNet{lds};
}

// R_hat of query (lane & 15) from its 8 packed bf16 inputs held by lane (the 4 lanes of a
// query return the same value).
template <typename Net>
__device__ inline float mlp_tile(const MlpDevice& d, const Net& net, int lane, uint4 x) {
  const int g = lane >> 4;
  floatx4_t a1[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float4 b = *reinterpret_cast<const float4*>(d.b1f + 16 * t + 4 * g);
    a1[t] = floatx4_t{b.x, b.y, b.z, b.w};
    a1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(net.w1(t, lane), as_bf16x8(x), a1[t], 0, 0, 0);
  }
  uint4 h[2];
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    h[st].x = pack_bf16(gelu_f(a1[2 * st][0]), gelu_f(a1[2 * st][1]));
    h[st].y = pack_bf16(gelu_f(a1[2 * st][2]), gelu_f(a1[2 * st][3]));
    h[st].z = pack_bf16(gelu_f(a1[2 * st + 1][0]), gelu_f(a1[2 * st + 1][1]));
    h[st].w = pack_bf16(gelu_f(a1[2 * st + 1][2]), gelu_f(a1[2 * st + 1][3]));
  }
  float part = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float4 b = *reinterpret_cast<const float4*>(d.b2f + 16 * t + 4 * g);
    floatx4_t a2 = floatx4_t{b.x, b.y, b.z, b.w};
#pragma unroll
    for (int st = 0; st < 2; ++st)
      a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(net.w2(t, st, lane), as_bf16x8(h[st]), a2, 0, 0, 0);
    const float4 w = *reinterpret_cast<const float4*>(d.w3f + 16 * t + 4 * g);
    part = __builtin_fmaf(bf16_round(gelu_f(a2[0])), w.x, part);
    part = __builtin_fmaf(bf16_round(gelu_f(a2[1])), w.y, part);
    part = __builtin_fmaf(bf16_round(gelu_f(a2[2])), w.z, part);
    part = __builtin_fmaf(bf16_round(gelu_f(a2[3])), w.w, part);
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part + d.master[kOffB3];
}

__device__ inline uint4 pack8(const float (&f)[8]) {
  return uint4{pack_bf16(f[0], f[1]), pack_bf16(f[2], f[3]), pack_bf16(f[4], f[5]), pack_bf16(f[6], f[7])};
}

// aidw_mlp_forward on the matrix cores: features [m][27] -> out [m].  Each wavefront takes
// tiles of 16 queries until the queries are exhausted.
__global__ __launch_bounds__(256) void k_mlp_forward_mfma(MlpDevice d, const float* __restrict__ feat, int m,
                                                          float* __restrict__ out) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  __shared__ uint4 lds[kNetOperands];
  const MfmaNet net = stage_net(d, lds);
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  for (int tile = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; tile * 16 < m; tile += nwaves) {
    __asm__ volatile("" ::: "memory");  // keeps the operand reads from LDS inside the loop (registers)
    const int q = tile * 16 + c;
    float f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j;
      f[j] = (q < m && k < kIn) ? feat[(size_t)q * kIn + k] : 0.0f;
    }
    const float y = mlp_tile(d, net, lane, pack8(f));
    if (g == 0 && q < m) out[q] = y;
  }
}

// Fused front of the learned run under the network's own rules (0 and 1, where the network
// runs on every query) for the queries at positions t of the order perm (may be null): the
// 27 features (as k_features), the network, and the fallback rule; flag[t] = 1 marks a query
// that takes the exact kNN.  (The rules that start from the certificate run k_cert_front.)  Lane 16 g + c works on the query at position
// 16 tile + c: it computes features 8 g .. 8 g + 7, takes a quarter of the query's own cell
// in the scan of the 3 x 3 block for the nearest distance, and one of its four neighbour
// segments.
// Four wavefronts per SIMD (at most 128 registers per lane) hide more of the loads' latency;
// there the registers of the loads in flight across the network spill 6 dwords to scratch,
// which still measured faster than issuing those loads after the network (no spill) or
// than three wavefronts per SIMD.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_learned_front(
    MlpDevice d, const GridScalars* __restrict__ gs, const int32_t* __restrict__ cell_start,
    const float* __restrict__ sx, const float* __restrict__ sy, const float* __restrict__ qx,
    const float* __restrict__ qy, const uint32_t* __restrict__ perm, int m, int64_t n, AlphaParams ap, int rule,
    double delta, double r_sat_lo, double r_sat_hi, uint32_t* __restrict__ flag, float* __restrict__ alpha_f,
    float* __restrict__ d1sq, float* __restrict__ r_hat_out, uint8_t* __restrict__ route) {
  if (gs->status != AIDW_OK) return;  // a failed grid build: nothing to decide
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const double inv_occ = (double)gs->ncells / (double)n;
  const double slack_cells = aidw::slack_cells(gs->ncol, gs->nrow);
  __shared__ uint4 lds[kNetOperands];
  const MfmaNet net = stage_net(d, lds);
  const float minx = gs->minx, miny = gs->miny, inv = gs->inv_cw;
  const int ncol = gs->ncol, nrow = gs->nrow;
  const double cwd = gs->cwd, minxd = minx, minyd = miny;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  // A feature cell's count is the difference of two cell offsets.  Column indices are
  // clamped to [0, ncol], which makes a cell beyond the left or right edge count 0, and
  // the end of a cell is the start of the next one in its row: lane g loads the starts
  // of its cells 8 g .. 8 g + 8 (a), plus the ends of the (at most two) cells among
  // them that close a row of the 5 x 5 block, at j1 and j1 + 5 (e0, e1).
  const int j1 = (4 + 2 * g) % 5;  // the first j with 8 g + j = 4 (mod 5)
  struct Ahead {
    int q;               // query (-1 for an empty slot)
    float fx, fy;
    int a[9], e0, e1;    // cell offsets of the feature counts (0 in rows outside the grid)
  };
  auto query_of = [&](int tl) -> int {
    const int tt = tl * 16 + c;
    return tt < m ? (perm ? (int)perm[tt] : tt) : -1;
  };
  // the neighbour segment of lane g: g = 0 / 1 the row r0 - 1 / r0 + 1 (columns c0 - 1 .. c0 + 1,
  // clipped), g = 2 / 3 the cell left / right of the query's
  auto segment = [&](int c0, int r0, int& srow, int& sa, int& sb) -> bool {
    srow = g < 2 ? r0 - 1 + 2 * g : r0;
    sa = g < 2 ? (c0 > 0 ? c0 - 1 : 0) : c0 + (g == 2 ? -1 : 1);
    sb = g < 2 ? (c0 + 1 < ncol ? c0 + 1 : ncol - 1) : sa;
    return g < 2 ? (srow >= 0 && srow < nrow) : (sa >= 0 && sa < ncol);
  };
  // offset of column cc (clamped to [0, ncol]) in row r0 + dr of the block, 0 outside the grid
  auto offset = [&](int r0, int c0, int dr, int dc) -> int {
    const int r = r0 + dr, cc = min(max(c0 + dc, 0), ncol);
    return r >= 0 && r < nrow ? cell_start[r * ncol + cc] : 0;
  };
  auto issue = [&](int qq, Ahead& A) {
    A.q = qq;
    A.fx = qq >= 0 ? qx[qq] : minx;
    A.fy = qq >= 0 ? qy[qq] : miny;
    const int c0 = clamp_cell((A.fx - minx) * inv, ncol), r0 = clamp_cell((A.fy - miny) * inv, nrow);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int kk = 8 * g + j;
      A.a[j] = kk < 25 ? offset(r0, c0, kk / 5 - 2, kk % 5 - 2) : 0;
    }
    const int k1 = 8 * g + j1, k2 = k1 + 5;
    A.e0 = k1 < 25 ? offset(r0, c0, k1 / 5 - 2, 3) : 0;
    A.e1 = k2 < 8 * g + 8 && k2 < 25 ? offset(r0, c0, k2 / 5 - 2, 3) : 0;
  };
  // Software pipeline over a wavefront's tiles (it works through them in sequence): a
  // tile's query index is loaded two tiles ahead, its coordinates and the offsets of its
  // feature cells one tile ahead, so that those loads are in flight while the previous
  // tile runs its network and scan; the scan's bounds are loaded before the network.
  int tile = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  Ahead nx;
  issue(query_of(tile), nx);
  int q_next = query_of(tile + nwaves);  // the query of the tile after the one in nx
  for (; tile * 16 < m; tile += nwaves) {
    __asm__ volatile("" ::: "memory");  // keeps the operand reads from LDS inside the loop (registers)
    const Ahead cur = nx;
    const int t = tile * 16 + c;
    const int q = cur.q;
    const bool valid = q >= 0;
    const float fx = cur.fx, fy = cur.fy;
    const float tx = (fx - minx) * inv, ty = (fy - miny) * inv;
    const int c0 = clamp_cell(tx, ncol), r0 = clamp_cell(ty, nrow);
    // the scan's bounds: the own cell and lane g's neighbour segment
    const int o0 = cell_start[r0 * ncol + c0];
    int o1 = cell_start[r0 * ncol + c0 + 1];
    int srow, sa, sb, p0 = 0, p1 = 0;
    const bool seg = segment(c0, r0, srow, sa, sb);
    if (seg) {
      p0 = cell_start[srow * ncol + sa];
      p1 = cell_start[srow * ncol + sb + 1];
    }
    {
      const int qn = q_next;
      q_next = query_of(tile + 2 * nwaves);
      issue(qn, nx);
    }
    // features 8 g .. 8 g + 7: counts of the 5 x 5 block (row-major), then the in-cell offset
    // and this lane's share of the data points in the blocks of 1, 3 x 3 and 5 x 5 cells
    float f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kk = 8 * g + j;
      const int end = j == j1 ? cur.e0 : (j == j1 + 5 ? cur.e1 : cur.a[j + 1]);
      const int cnt = kk < 25 ? end - cur.a[j] : 0;
      f[j] = kk < 25 ? (float)((double)cnt * inv_occ)
                     : (kk == 25 ? tx - (float)c0 : (kk == 26 ? ty - (float)r0 : 0.0f));
    }
    const double px = fx, py = fy;
    const float y = mlp_tile(d, net, lane, pack8(f));
    double alpha_net = 0.0;
    const bool net_fall = decide_one((double)y, 1.0f, ap, rule, delta, r_sat_lo, r_sat_hi, &alpha_net);
    // a query that takes the exact kNN needs no scan (that search gives its d1); a skipped one
    // needs its nearest distance (all inputs here are the same on a query's four lanes)
    const bool scan = valid && !net_fall;
    if (!scan) {
      o1 = o0;
      p1 = p0;
    }
    // Nearest point in the 3 x 3 block: the own cell split over the 4 lanes, then each lane's
    // neighbour segment unless all of it lies farther than the own cell's nearest, then the
    // minimum over the 4 lanes.  float32 suffices: the value only sets the power-of-two
    // scale of the pair weights; a coincident point (which lies in the own cell) is found
    // exactly, as a zero difference.
    float best = INFINITY;
    int hit = 0;
    for (int p = o0 + g; p < o1; p += 4) {
      const float dx = sx[p] - fx, dy = sy[p] - fy;
      const float dd = __builtin_fmaf(dx, dx, dy * dy);
      hit |= (dx == 0.0f) & (dy == 0.0f);
      best = fminf(best, dd);
    }
    best = fminf(best, __shfl_xor(best, 16, 64));
    best = fminf(best, __shfl_xor(best, 32, 64));
    if (seg && best < INFINITY) {
      // every point of lane g's segment lies beyond one side of the own cell, the segment's
      // near edge moved toward the query by the binning slack: below it (g = 0), above (1),
      // left (2) or right (3); e = the distance from the query to that edge
      const double e = g == 0   ? py - (minyd + ((double)r0 + slack_cells) * cwd)
                       : g == 1 ? (minyd + ((double)r0 + 1.0 - slack_cells) * cwd) - py
                       : g == 2 ? px - (minxd + ((double)c0 + slack_cells) * cwd)
                                : (minxd + ((double)c0 + 1.0 - slack_cells) * cwd) - px;
      if (e > 0.0 && e * e > (double)best) p1 = p0;
    }
    if (seg) {
      for (int p = p0; p < p1; ++p) {
        const float dx = sx[p] - fx, dy = sy[p] - fy;
        best = fminf(best, __builtin_fmaf(dx, dx, dy * dy));
      }
    }
    best = fminf(best, __shfl_xor(best, 16, 64));
    best = fminf(best, __shfl_xor(best, 32, 64));
    hit |= __shfl_xor(hit, 16, 64);
    hit |= __shfl_xor(hit, 32, 64);
    if (g != 0 || !valid) continue;
    double dout = INFINITY;
    if (c0 - 1 > 0) dout = fmin(dout, px - (minxd + (double)(c0 - 1) * cwd));
    if (c0 + 1 < ncol - 1) dout = fmin(dout, (minxd + (double)(c0 + 2) * cwd) - px);
    if (r0 - 1 > 0) dout = fmin(dout, py - (minyd + (double)(r0 - 1) * cwd));
    if (r0 + 1 < nrow - 1) dout = fmin(dout, (minyd + (double)(r0 + 2) * cwd) - py);
    dout -= slack_cells * cwd;
    double v;
    if (dout == INFINITY || (double)best < dout * dout)
      v = best;                        // the nearest distance
    else
      v = dout > 0 ? dout * dout : 0;  // lower bound
    const float d1 = hit ? 0.0f : fmaxf((float)v, FLT_MIN);
    // the decision: a coincident query (d1 = 0) takes the exact path, else the network's rule
    const bool fall = !scan || d1 == 0.0f;
    flag[t] = fall ? 1u : 0u;
    if (!fall) {
      alpha_f[q] = (float)alpha_net;
      d1sq[q] = d1;
    }
    if (r_hat_out) r_hat_out[q] = y;
    if (route) route[q] = fall ? 0 : 4;
  }
}


// The front of the rules that start from the certificate (2, 3 and 4), one lane per query: the
// queries of a wavefront are 64 consecutive positions of the binned order, so they share most
// of their blocks' cells.  c_0, c_1, c_2 are differences of row offsets (a row of a block is
// one run of the cell order), the certificate from the counts, then, for a query it certifies
// or may still certify (or, rule 3, that the network lets skip the kNN), one scan of the 3 x 3
// block (three runs) for the nearest distance and the statistics below D_1.
// The network runs only on the queries the counts do not certify: rule 4 those whose 3 x 3
// block the certificate may scan (the network decides which of them are scanned), rule 3 all
// of them (the network's alpha-exact rule where the certificate fails).  A wavefront gathers
// those queries (a ballot), stores their 27 features as bf16 in LDS in the order of their
// lanes, and runs the network on the matrix cores over tiles of 16 of them, so a wavefront
// without such a query does not evaluate it.  r_hat_out receives the prediction for those
// queries and NaN for the others.
template <int kRule>
__global__ __launch_bounds__(256) void k_cert_front(MlpDevice d, const GridScalars* __restrict__ gs,
                                                    const int32_t* __restrict__ cell_start,
                                                    const float* __restrict__ sx, const float* __restrict__ sy,
                                                    const float* __restrict__ qx, const float* __restrict__ qy,
                                                    const uint32_t* __restrict__ perm, int m, int64_t n,
                                                    AlphaParams ap, int k, double cert_factor, double delta,
                                                    double r_sat_lo, double r_sat_hi, uint32_t* __restrict__ flag,
                                                    uint32_t* __restrict__ list, uint32_t* __restrict__ count,
                                                    float* __restrict__ alpha_f,
                                                    float* __restrict__ d1sq, float* __restrict__ r_hat_out,
                                                    uint8_t* __restrict__ route) {
  static_assert(kRule >= 2 && kRule <= 4, "rules 2, 3, 4");
  constexpr bool kNet = kRule != 2;
  constexpr int kWaves = 256 / 64;
  __shared__ __align__(16) uint16_t s_feat[kNet ? kWaves : 1][64][32];  // bf16 bits, 27 used
  __shared__ float s_y[kNet ? kWaves : 1][64];
  if (gs->status != AIDW_OK) return;  // a failed grid build: nothing to decide (the whole grid)
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // with the network every lane stays to the barriers; without it the tail leaves at once
  const bool valid = t < m;
  if (!kNet && !valid) return;
  const int q = valid ? (perm ? (int)perm[t] : t) : 0;
  const float minx = gs->minx, miny = gs->miny, inv = gs->inv_cw;
  const int ncol = gs->ncol, nrow = gs->nrow;
  const double cwd = gs->cwd, minxd = minx, minyd = miny;
  const double slack_cells = aidw::slack_cells(ncol, nrow);
  const float fx = valid ? qx[q] : minx, fy = valid ? qy[q] : miny;
  const float tx = (fx - minx) * inv, ty = (fy - miny) * inv;
  const int c0 = clamp_cell(tx, ncol), r0 = clamp_cell(ty, nrow);
  // row runs of the blocks: columns [c0 - L, c0 + L] clamped, so a run's end is the start of
  // the cell after it (the next row's first cell at the right edge)
  const int a2 = max(c0 - 2, 0), e2 = min(c0 + 3, ncol), a1 = max(c0 - 1, 0), e1 = min(c0 + 2, ncol);
  int s1[3], t1[3];
  int n2 = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int r = r0 - 2 + i;
    const bool in = r >= 0 && r < nrow;
    const int base = in ? r * ncol : 0;
    const int u = in ? cell_start[base + a2] : 0, v = in ? cell_start[base + e2] : 0;
    n2 += v - u;
    if (i >= 1 && i <= 3) {
      s1[i - 1] = in ? cell_start[base + a1] : 0;
      t1[i - 1] = in ? cell_start[base + e1] : 0;
    }
  }
  const int n1 = (t1[0] - s1[0]) + (t1[1] - s1[1]) + (t1[2] - s1[2]);
  const int n0 = cell_start[r0 * ncol + c0 + 1] - cell_start[r0 * ncol + c0];
  const double px = fx, py = fy;
  const double cert_sum_min = cert_factor * gs->r_exp;
  bool cert = valid && certified_saturated(px, py, c0, r0, ncol, nrow, minxd, minyd, cwd, slack_cells, n0, n1, n2,
                                           k, cert_sum_min);
  const bool cert_counts = cert;
  // the queries the counts leave open whose 3 x 3 block the certificate may scan (a block over
  // 8 k + 16 points is left to the exact path: such a query's R lies far below saturation)
  const bool open = valid && !cert && n1 <= 8 * k + 16;
  bool scan = open;
  float y = __builtin_nanf("");
  bool net_fall = true;  // rule 3: the network's alpha-exact rule sends the query to the exact kNN
  double alpha_net = 0.0;
  if constexpr (kNet) {
    const bool net_q = kRule == 4 ? open : valid && !cert;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t net_mask = __ballot(net_q);
    const int nnet = __popcll(net_mask);
    const int slot = __popcll(net_mask & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
    if (net_q) {
      // the 27 features: counts of the 5 x 5 block (row-major) over the mean occupancy, then
      // the offset inside the cell (a count is the difference of two offsets; columns clamped
      // to [0, ncol] count 0 beyond the edges, rows outside the grid count 0)
      const double inv_occ = (double)gs->ncells / (double)n;
      uint16_t* f = s_feat[wave][slot];
#pragma unroll
      for (int br = 0; br < 5; ++br) {
        const int r = r0 + br - 2;
        const bool in = r >= 0 && r < nrow;
        int o[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) o[j] = in ? cell_start[r * ncol + min(max(c0 + j - 2, 0), ncol)] : 0;
#pragma unroll
        for (int bc = 0; bc < 5; ++bc)
          f[5 * br + bc] = (uint16_t)bf16_bits((float)((double)(o[bc + 1] - o[bc]) * inv_occ));
      }
      f[25] = (uint16_t)bf16_bits(tx - (float)c0);
      f[26] = (uint16_t)bf16_bits(ty - (float)r0);
#pragma unroll
      for (int j = 27; j < 32; ++j) f[j] = 0;
    }
    __syncthreads();
    const MfmaNetGlobal net{reinterpret_cast<const uint4*>(d.w1a), reinterpret_cast<const uint4*>(d.w2a)};
    for (int tile = 0; tile * 16 < nnet; ++tile) {  // uniform over the wavefront: every lane runs the MFMA
      __asm__ volatile("" ::: "memory");  // keeps the operand reads from LDS inside the loop (registers)
      const int c = lane & 15, g = lane >> 4, sl = tile * 16 + c;
      const uint4 x = sl < nnet ? *reinterpret_cast<const uint4*>(&s_feat[wave][sl][8 * g]) : uint4{0u, 0u, 0u, 0u};
      const float yy = mlp_tile(d, net, lane, x);
      if (g == 0 && sl < nnet) s_y[wave][sl] = yy;
    }
    __syncthreads();
    if (net_q) y = s_y[wave][slot];
    if constexpr (kRule == 4) {
      // the scan is tried only where the prediction reaches the saturation point less delta
      scan = open && (double)y >= r_sat_hi - delta;
    } else {
      if (net_q) net_fall = decide_one((double)y, 1.0f, ap, 1, delta, r_sat_lo, r_sat_hi, &alpha_net);
    }
    if (!valid) return;
  }
  // mode 0: the exact kNN in any case (no scan); 1: skipped (certified, or by the network's
  // rule), needs d1; 2: may be certified by the distances
  const int mode = cert ? 1 : (scan ? 2 : (!net_fall ? 1 : 0));
  float best = INFINITY;
  bool hit = false;
  double d_1 = 0.0, v_sum = 0.0;
  float d_1sq = 0.0f, v_max = 0.0f;
  int v_cnt = 0;
  if (mode == 2) {
    d_1 = block_side_distance(px, py, c0, r0, 1, ncol, nrow, minxd, minyd, cwd, slack_cells);
    d_1sq = (float)(d_1 * d_1);
  }
  if (mode != 0) {
    // four points per step, their loads issued together
    constexpr int kStep = 4;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      for (int p = s1[i]; p < t1[i]; p += kStep) {
        float px4[kStep], py4[kStep];
#pragma unroll
        for (int j = 0; j < kStep; ++j) {
          const bool in = p + j < t1[i];
          px4[j] = in ? sx[p + j] : INFINITY;
          py4[j] = in ? sy[p + j] : INFINITY;
        }
#pragma unroll
        for (int j = 0; j < kStep; ++j) {
          if (p + j >= t1[i]) break;
          const float dx = px4[j] - fx, dy = py4[j] - fy;
          const float dd = __builtin_fmaf(dx, dx, dy * dy);
          hit |= (dx == 0.0f) & (dy == 0.0f);
          best = fminf(best, dd);
          if (dd < d_1sq) {
            const float dist = __builtin_sqrtf(dd);
            v_sum += (double)dist;
            v_max = fmaxf(v_max, dist);
            ++v_cnt;
          }
        }
      }
    }
  }
  // d1: the block's nearest when it lies within the block's open sides (less the slack),
  // else that distance as a lower bound
  double dout = INFINITY;
  if (c0 - 1 > 0) dout = fmin(dout, px - (minxd + (double)(c0 - 1) * cwd));
  if (c0 + 1 < ncol - 1) dout = fmin(dout, (minxd + (double)(c0 + 2) * cwd) - px);
  if (r0 - 1 > 0) dout = fmin(dout, py - (minyd + (double)(r0 - 1) * cwd));
  if (r0 + 1 < nrow - 1) dout = fmin(dout, (minyd + (double)(r0 + 2) * cwd) - py);
  dout -= slack_cells * cwd;
  const double v = (dout == INFINITY || (double)best < dout * dout) ? (double)best : (dout > 0 ? dout * dout : 0.0);
  const float d1 = hit ? 0.0f : fmaxf((float)v, FLT_MIN);
  // a coincident query (d1 = 0) and a query not scanned take the exact path; then the
  // certificate (counts, else the 3 x 3 distances), then (rule 3) the network's rule
  bool fall = true;
  double alpha = 0.0;
  if (mode != 0 && d1 != 0.0f) {
    if (mode == 2)
      cert = certified_by_distances(
          v_sum, v_cnt, v_max, n2, k, d_1,
          block_side_distance(px, py, c0, r0, 2, ncol, nrow, minxd, minyd, cwd, slack_cells), cert_sum_min);
    if (cert) {
      fall = false;
      alpha = ap.levels[4];
    } else if (!net_fall) {
      fall = false;
      alpha = alpha_net;
    }
  }
  if (list) {
    // the wavefront's exact-kNN queries go to the list together, in binned order (one atomic)
    const uint64_t fb = __ballot(fall);
    if (fb) {
      const int lane = threadIdx.x & 63, lead = __ffsll((long long)fb) - 1;
      uint32_t base = 0;
      if (lane == lead) base = atomicAdd(count, (uint32_t)__popcll(fb));
      base = __shfl(base, lead, 64);
      if (fall) list[base + __popcll(fb & (lane == 0 ? 0ull : (~0ull >> (64 - lane))))] = (uint32_t)q;
    }
  } else {
    flag[t] = fall ? 1u : 0u;
  }
  if (!fall) {
    alpha_f[q] = (float)alpha;
    d1sq[q] = d1;
  }
  if (r_hat_out) r_hat_out[q] = y;
  if (route) route[q] = fall ? (mode == 2 ? 1 : 0) : (cert ? (cert_counts ? 2 : 3) : 4);
}

}  // namespace

hipError_t launch_features(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                           const float* qx, const float* qy, const uint32_t* perm, int m, int64_t n, float* feat,
                           float* d1sq, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((m + 255) / 256), dim3(256), 0, s, gs, cell_start, sx, sy, qx, qy, perm, m, n,
                     feat, d1sq);
  return hipGetLastError();
}

static MlpWeights weights(const MlpDevice& d) {
  return MlpWeights{d.w1p, d.w2p, d.w3p, d.w2r, d.w3r, d.master};
}

hipError_t launch_mlp_repack(const MlpDevice& d, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_repack, dim3((kH * kH + 255) / 256), dim3(256), 0, s, d.master, d.w1p, d.w2p, d.w3p, d.w2r,
                     d.w3r);
  hipLaunchKernelGGL(k_mlp_repack_mfma, dim3(8), dim3(256), 0, s, d.master, d.w1a, d.w2a, d.b1f, d.b2f, d.w3f);
  return hipGetLastError();
}

namespace {
// Workgroups of a tile loop over m queries: as many as the chip holds at once for
// this kernel (a second, partial round would leave most of the chip idle), at most
// one tile per wavefront.
int tile_blocks(const void* kernel, int m) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || cus <= 0 ||
      per_cu <= 0) {
    cus = 256;
    per_cu = 2;
  }
  const int tiles = (m + 15) / 16;
  const int blocks = (tiles + 3) / 4;
  const int cap = cus * per_cu;
  return blocks < cap ? (blocks > 0 ? blocks : 1) : cap;
}
}  // namespace

hipError_t launch_learned_front(const MlpDevice& d, const GridScalars* gs, const int32_t* cell_start, const float* sx,
                                const float* sy, const float* qx, const float* qy, const uint32_t* perm, int m,
                                int64_t n, const AlphaParams& ap, int rule, double delta, double r_sat_lo,
                                double r_sat_hi, int k, double cert_factor, uint32_t* flag, uint32_t* list,
                                uint32_t* count, float* alpha_f, float* d1sq, float* r_hat_out, uint8_t* route,
                                hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if ((list != nullptr) != (count != nullptr) || (list && rule != 2 && rule != 3 && rule != 4))
    return hipErrorInvalidValue;
#define CERT_FRONT(R)                                                                                        \
  hipLaunchKernelGGL(k_cert_front<R>, dim3((m + 255) / 256), dim3(256), 0, s, d, gs, cell_start, sx, sy, qx, qy, \
                     perm, m, n, ap, k, cert_factor, delta, r_sat_lo, r_sat_hi, flag, list, count, alpha_f, d1sq,  \
                     r_hat_out, route)
  if (rule == 2)
    CERT_FRONT(2);
  else if (rule == 3)
    CERT_FRONT(3);
  else if (rule == 4)
    CERT_FRONT(4);
  else
    hipLaunchKernelGGL(k_learned_front, dim3(tile_blocks((const void*)k_learned_front, m)), dim3(256), 0, s, d, gs,
                       cell_start, sx, sy, qx, qy, perm, m, n, ap, rule, delta, r_sat_lo, r_sat_hi, flag, alpha_f,
                       d1sq, r_hat_out, route);
#undef CERT_FRONT
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDevice& d, const float* feat, int m, float* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward_mfma, dim3(tile_blocks((const void*)k_mlp_forward_mfma, m)), dim3(256), 0, s, d,
                     feat, m, out);
  return hipGetLastError();
}

size_t mlp_batch_scratch_floats(int B) { return (size_t)B * (28 + 4 * kH + 2) + (size_t)kGradChunks * (kParams + 1); }

hipError_t launch_mlp_gradients(const MlpDevice& d, const float* feat, const float* target, const uint32_t* sel, int B,
                                float* scratch, float* grad, hipStream_t s) {
  float* s_x = scratch;
  float* s_h1 = s_x + (size_t)B * 28;
  float* s_h2 = s_h1 + (size_t)B * kH;
  float* s_da1 = s_h2 + (size_t)B * kH;
  float* s_da2 = s_da1 + (size_t)B * kH;
  float* s_dy = s_da2 + (size_t)B * kH;
  float* s_err2 = s_dy + B;
  float* part = s_err2 + B;
  hipLaunchKernelGGL(k_mlp_train_sample, dim3((B + 63) / 64), dim3(64), 0, s, weights(d), feat, target, sel, B,
                     2.0f / (float)B, s_x, s_h1, s_h2, s_da1, s_da2, s_dy, s_err2);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((kParams + 1 + 255) / 256, kGradChunks), dim3(256), 0, s, B, s_x, s_h1, s_h2,
                     s_da1, s_da2, s_dy, s_err2, part);
  hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, B, part, grad);
  return hipGetLastError();
}

hipError_t launch_adam(const MlpDevice& d, const float* grad, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, d.master, grad, d.mom, d.vel, lr, b1, b2,
                     eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_accumulate_loss(const float* grad, float* epoch_loss, int epoch, float scale, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate_loss, dim3(1), dim3(64), 0, s, grad, epoch_loss, epoch, scale);
  return hipGetLastError();
}

}  // namespace aidw
