// Issue-rate microbenchmark of the vector ALU of one gfx950 GPU: how many float32
// FMA lanes and how many transcendental lanes (v_exp_f32, v_log_f32, v_rsq_f32) a
// compute unit issues per clock, and whether transcendentals overlap with FMAs when
// the two are mixed in the proportions of the interpolation kernel's pair loop.
// The figures set the peak of that kernel's roofline (pairs per second from its
// per-pair instruction counts).
//
// Each lane runs `iters` rounds over 8 independent dependency chains, so a wavefront
// always has independent work and enough wavefronts per SIMD (8) hide the latency:
// the launch is bound by issue throughput.  Chains step as
//   0 fma3   a = fma(a, m, c)                        (v_fma_f32, 64-bit encoding)
//   1 fmac   a = fma(m, v, a)                        (v_fmac_f32, 32-bit encoding)
//   2 exp    a = 2^-a                                (1 v_exp_f32; fixed point near 0.64)
//   3 log    a = log2(|a|)                           (1 v_log_f32; fixed point near -0.64)
//   4 rsq    a = rsq(a)                              (1 v_rsq_f32; fixed point 1)
//   5 mix5   r = rsq(a); 9 fmac on r                 (the integer-alpha pair's mix: 9 VALU + 1)
//   6 mixg   log2, exp2; 7 fmac                      (the general pair's mix: 7 VALU + 2)
//   8 mul    a = a * v                               (v_mul_f32)
//   9 add    a = a + v                               (v_add_f32)
//  10 pairv  the nine VALU operations of the integer-alpha pair without its rsq: 2 fma for
//            the offsets, mul + fma for d^2, 3 mul for the power, fma + add for the sums
//            (4 fma-type + 5 mul / add), chained through a
// and kind 7 runs the interpolation kernel's own pair loop (alpha = 5, one query per lane,
// data points streamed through the scalar cache) over a 512-point array that stays in
// that cache: the kernel's instruction stream without its memory traffic.
// Negation and absolute value are free source modifiers.  Thread 0 of block 0 reads the shader clock
// (s_memtime) and the constant 100 MHz clock (s_memrealtime) at its start and end,
// which gives the clock the chip held.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../csrc/pair_core.h"

namespace {

constexpr int kChains = 8;

template <int KIND>
__device__ __forceinline__ float step(float a, float m, float c) {
  if constexpr (KIND == 0) {
    return __builtin_fmaf(a, m, c);
  } else if constexpr (KIND == 1) {
    return __builtin_fmaf(m, c, a);
  } else if constexpr (KIND == 2) {
    return __builtin_amdgcn_exp2f(-a);
  } else if constexpr (KIND == 3) {
    return __builtin_amdgcn_logf(__builtin_fabsf(a));
  } else if constexpr (KIND == 4) {
    return __builtin_amdgcn_rsqf(a);
  } else if constexpr (KIND == 5) {
    float r = __builtin_amdgcn_rsqf(a);
#pragma unroll
    for (int i = 0; i < 9; ++i) r = __builtin_fmaf(m, c, r);
    return r;
  } else if constexpr (KIND == 6) {
    float r = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(a));
#pragma unroll
    for (int i = 0; i < 7; ++i) r = __builtin_fmaf(m, c, r);
    return r;
  } else if constexpr (KIND == 8) {
    return a * c;
  } else if constexpr (KIND == 9) {
    return a + c;
  } else {
    const float dx = __builtin_fmaf(m, c, a);
    const float dy = __builtin_fmaf(a, m, c);
    const float t = __builtin_fmaf(dx, dx, dy * dy);
    const float t2 = t * t, t4 = t2 * t2, w = t4 * t;
    return __builtin_fmaf(w, m, a) + w;
  }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_issue(int iters, float m, float c0, float* __restrict__ out,
                                               uint64_t* __restrict__ clocks) {
  const float c = c0 * (float)(1 + (threadIdx.x & 3));  // a per-lane value (a VGPR operand)
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = 0.6f + 0.01f * (float)((threadIdx.x + j) & 7);
  uint64_t t0 = 0, r0 = 0;
  const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
  if (timer) {
    t0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int j = 0; j < kChains; ++j) a[j] = step<KIND>(a[j], m, c);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += a[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (timer) {
    const uint64_t t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    clocks[0] = t1 - t0;
    clocks[1] = r1 - r0;
  }
}

// The interpolation kernel's pair loop (alpha = 5) over the 512 points of xyz (x, y, z arrays
// of kPairPoints each, zero-padded by one chunk), `iters` times.
constexpr int kPairPoints = 512;
__global__ __launch_bounds__(256) void k_pair_loop(int iters, const float* __restrict__ xs, const float* __restrict__ ys,
                                                   const float* __restrict__ zs, float* __restrict__ out,
                                                   uint64_t* __restrict__ clocks) {
  aidw::pair::Lane<1, 5> L;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  L.set(0, 0.25f + 1e-6f * (float)(t & 1023), 0.5f, 5.0f, 1e-6f);
  uint64_t t0 = 0, r0 = 0;
  const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
  if (timer) {
    t0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  for (int it = 0; it < iters; ++it) aidw::pair::pair_range<1, 5>(L, xs, ys, zs, 0, kPairPoints);
  out[t] = (float)(L.num(0) / L.den(0));
  if (timer) {
    const uint64_t t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    clocks[0] = t1 - t0;
    clocks[1] = r1 - r0;
  }
}

__global__ void k_fill_points(float* __restrict__ p, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * len) {
    const int a = i / len, j = i % len;
    const bool pad = j >= kPairPoints;
    p[i] = pad ? 0.0f : (a == 2 ? 0.001f * (float)j : 0.0009765625f * (float)((j * 37 + 11 * a) & 1023));
  }
}

template <int KIND>
hipError_t run(int iters, int blocks, float* out, uint64_t* clocks, hipStream_t s) {
  hipLaunchKernelGGL(k_issue<KIND>, dim3(blocks), dim3(256), 0, s, iters, 0.999f, 0.001f, out, clocks);
  return hipGetLastError();
}

}  // namespace

extern "C" {

// Instructions one lane executes per round of `kind` (VALU, transcendentals); for kind 7 the
// pair count per round (kPairPoints) with the per-pair minimum of the alpha = 5 form
// (9 VALU + 1 transcendental).
int aidw_ubench_counts(int kind, int* valu, int* trans) {
  static const int v[11] = {1, 1, 0, 0, 0, 9, 7, 0, 1, 1, 9}, t[11] = {0, 0, 1, 1, 1, 1, 2, 0, 0, 0, 0};
  if (kind < 0 || kind > 10 || !valu || !trans) return -1;
  if (kind == 7) {
    *valu = 9 * kPairPoints;
    *trans = kPairPoints;
    return 0;
  }
  *valu = v[kind] * kChains * 4;
  *trans = t[kind] * kChains * 4;
  return 0;
}

// Runs kind (see above) over `blocks` workgroups of 256
// lanes for `iters` rounds, once to warm up and then timed with HIP events.  *ms = the timed
// launch; shader_ticks / real_ticks = the two clocks over block 0's loop.  Returns 0 or the
// HIP error code.
int aidw_ubench_issue_rate(int kind, int iters, int blocks, float* ms, uint64_t* shader_ticks, uint64_t* real_ticks) {
  if (kind < 0 || kind > 10 || iters < 1 || blocks < 1 || !ms) return -1;
  float* out = nullptr;
  uint64_t* clk = nullptr;
  float* pts = nullptr;
  const int plen = aidw::pair::padded_len(kPairPoints);
  hipError_t e = hipMalloc(&out, sizeof(float) * (size_t)blocks * 256);
  if (e != hipSuccess) return (int)e;
  if ((e = hipMalloc(&clk, 2 * sizeof(uint64_t))) != hipSuccess || (e = hipMalloc(&pts, sizeof(float) * 3 * plen)) !=
                                                                        hipSuccess) {
    (void)hipFree(out);
    if (clk) (void)hipFree(clk);
    return (int)e;
  }
  hipLaunchKernelGGL(k_fill_points, dim3((3 * plen + 255) / 256), dim3(256), 0, nullptr, pts, plen);
  hipEvent_t ev[2];
  (void)hipEventCreate(&ev[0]);
  (void)hipEventCreate(&ev[1]);
  auto launch = [&](int it) -> hipError_t {
    switch (kind) {
      case 0: return run<0>(it, blocks, out, clk, nullptr);
      case 1: return run<1>(it, blocks, out, clk, nullptr);
      case 2: return run<2>(it, blocks, out, clk, nullptr);
      case 3: return run<3>(it, blocks, out, clk, nullptr);
      case 4: return run<4>(it, blocks, out, clk, nullptr);
      case 5: return run<5>(it, blocks, out, clk, nullptr);
      case 6: return run<6>(it, blocks, out, clk, nullptr);
      case 8: return run<8>(it, blocks, out, clk, nullptr);
      case 9: return run<9>(it, blocks, out, clk, nullptr);
      case 10: return run<10>(it, blocks, out, clk, nullptr);
      default:
        hipLaunchKernelGGL(k_pair_loop, dim3(blocks), dim3(256), 0, nullptr, it, pts, pts + plen, pts + 2 * plen, out,
                           clk);
        return hipGetLastError();
    }
  };
  e = launch(iters);
  if (e == hipSuccess) e = hipEventRecord(ev[0], nullptr);
  if (e == hipSuccess) e = launch(iters);
  if (e == hipSuccess) e = hipEventRecord(ev[1], nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  uint64_t h[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(h, clk, sizeof h, hipMemcpyDeviceToHost);
  if (shader_ticks) *shader_ticks = h[0];
  if (real_ticks) *real_ticks = h[1];
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  (void)hipFree(out);
  (void)hipFree(clk);
  (void)hipFree(pts);
  return (int)e;
}

}  // extern "C"
