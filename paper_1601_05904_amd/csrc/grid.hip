// Stage 1, grid build (Section 3.2.1-3.2.3 and 4.1.1-4.1.3 of the paper):
//   bounds over data and queries -> grid scalars (Eq. 2) -> cell key per data
//   point -> stable LSD radix sort of (cell, index) -> CSR cell offsets and the
//   data coordinates gathered into cell order.
// The paper sorts with a library sort_by_key and recovers per-cell size and head
// with segmented reduce / unique; here one stable counting sort per 8- or 10-bit digit
// produces the same cell-ordered segments, and the CSR offsets (head of cell c =
// cell_start[c], size = cell_start[c+1] - cell_start[c]) come from a binary
// search over the sorted keys, which also covers empty cells.
#include "aidw_internal.h"
#include "grid_core.h"

namespace aidw {

namespace {

using gridc::wave_max;
using gridc::wave_min;
using gridc::wave_or;

// Per-block min / max of x and y over the data points followed by the queries
// (Section 4.1.1: the grid encloses both sets), plus a non-finite flag.
__global__ __launch_bounds__(kBoundsThreads) void k_bounds(const float* __restrict__ x, const float* __restrict__ y,
                                                           int n, const float* __restrict__ qx,
                                                           const float* __restrict__ qy, int m,
                                                           BoundsPartial* __restrict__ partial) {
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  int bad = 0;
  auto take = [&](float a, float b) {
    bad |= !(isfinite(a) && isfinite(b));
    mnx = fminf(mnx, a);
    mxx = fmaxf(mxx, a);
    mny = fminf(mny, b);
    mxy = fmaxf(mxy, b);
  };
  // the data points, then the queries; four strides per step keep eight loads in flight
  auto sweep = [&](const float* __restrict__ a, const float* __restrict__ b, int64_t len) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < len; i += 4 * stride) {
      float av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = a[i + u * stride];
        bv[u] = b[i + u * stride];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) take(av[u], bv[u]);
    }
    for (; i < len; i += stride) take(a[i], b[i]);
  };
  sweep(x, y, n);
  if (m > 0) sweep(qx, qy, m);
  mnx = wave_min(mnx);
  mny = wave_min(mny);
  mxx = wave_max(mxx);
  mxy = wave_max(mxy);
  bad = wave_or(bad);
  __shared__ BoundsPartial s[kBoundsThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s[wave] = BoundsPartial{mnx, mny, mxx, mxy, bad, {0, 0, 0}};
  __syncthreads();
  if (threadIdx.x == 0) {
    BoundsPartial r = s[0];
    for (int w = 1; w < kBoundsThreads / 64; ++w) {
      r.minx = fminf(r.minx, s[w].minx);
      r.miny = fminf(r.miny, s[w].miny);
      r.maxx = fmaxf(r.maxx, s[w].maxx);
      r.maxy = fmaxf(r.maxy, s[w].maxy);
      r.nonfinite |= s[w].nonfinite;
    }
    partial[blockIdx.x] = r;
  }
}

// Reduces the partials and derives the grid scalars (Eq. 2, Section 4.1.1).
__global__ __launch_bounds__(256) void k_finalize(const BoundsPartial* __restrict__ partial, int nparts, int64_t n,
                                                  double area_in, double cw_in, double occ,
                                                  GridScalars* __restrict__ out) {
  const BoundsPartial r = gridc::block_reduce_bounds(partial, 0, nparts);
  if (threadIdx.x != 0) return;
  *out = gridc::grid_scalars(r.minx, r.miny, r.maxx, r.maxy, r.nonfinite != 0, n, area_in, cw_in, occ, 0);
}

// Section 4.1.2: cell of each data point, (x - minX) * inv_cw in float32 truncated,
// clamped into the grid; key = row * nCol + col, value = original index.
// Cell of a point (Section 4.1.2): column and row from float32 offsets scaled by 1 / cell width,
// truncated and clamped to the grid.
__device__ inline uint32_t cell_key(float x, float y, float minx, float miny, float inv, int ncol, int nrow) {
  const float tx = (x - minx) * inv;
  const float ty = (y - miny) * inv;
  int col = (int)tx, row = (int)ty;
  col = col > ncol - 1 ? ncol - 1 : (col < 0 ? 0 : col);
  row = row > nrow - 1 ? nrow - 1 : (row < 0 ? 0 : row);
  return (uint32_t)(row * ncol + col);
}
// ---- query binning -------------------------------------------------------------
// The kNN kernels and the learned front take the queries in cell order, so that a
// wavefront's queries scan neighbouring cells.  Each query's results depend on that
// query alone, so the order within a cell is free: a counting sort whose slot within
// a cell is the value a global atomic hands out (cell counts, their exclusive scan,
// placement) replaces a stable sort.

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t len, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = v;
}

__global__ __launch_bounds__(256) void k_query_slots(const float* __restrict__ qx, const float* __restrict__ qy, int m,
                                                     const GridScalars* __restrict__ gs, uint32_t* __restrict__ cnt,
                                                     uint32_t* __restrict__ key, uint32_t* __restrict__ slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float minx = gs->minx, miny = gs->miny, inv = gs->inv_cw;
  const int ncol = gs->ncol, nrow = gs->nrow;
  int col = (int)((qx[i] - minx) * inv), row = (int)((qy[i] - miny) * inv);
  col = col > ncol - 1 ? ncol - 1 : (col < 0 ? 0 : col);
  row = row > nrow - 1 ? nrow - 1 : (row < 0 ? 0 : row);
  const uint32_t c = (uint32_t)(row * ncol + col);
  key[i] = c;
  slot[i] = atomicAdd(&cnt[c], 1u);
}

__global__ __launch_bounds__(256) void k_query_place(const uint32_t* __restrict__ key, const uint32_t* __restrict__ slot,
                                                     int m, const uint32_t* __restrict__ start,
                                                     uint32_t* __restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) order[start[key[i]] + slot[i]] = (uint32_t)i;
}

// ---- stable LSD radix sort ------------------------------------------------------

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                             uint32_t* __restrict__ hist, int nblocks) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t h[R];
  for (int i = threadIdx.x; i < R; i += kSortThreads) h[i] = 0;
  // all of a thread's keys are loaded before the first count, so the block waits for memory once
  const int base = blockIdx.x * kSortTile;
  uint32_t key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    key[r] = i < n ? keys[i] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r)
    if (base + r * kSortThreads + (int)threadIdx.x < n) atomicAdd(&h[(key[r] >> shift) & (R - 1)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kSortThreads) hist[(size_t)d * nblocks + blockIdx.x] = h[d];
}
// The first pass's histogram (digit 0) fused with the cell keys: each point's key is computed
// (cell_key) and stored with its index, then counted.
template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist_cells(const float* __restrict__ x,
                                                                   const float* __restrict__ y, int n,
                                                                   const GridScalars* __restrict__ gs,
                                                                   uint32_t* __restrict__ keys,
                                                                   uint32_t* __restrict__ vals,
                                                                   uint32_t* __restrict__ hist, int nblocks) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t h[R];
  for (int i = threadIdx.x; i < R; i += kSortThreads) h[i] = 0;
  const float minx = gs->minx, miny = gs->miny, inv = gs->inv_cw;
  const int ncol = gs->ncol, nrow = gs->nrow;
  const int base = blockIdx.x * kSortTile;
  uint32_t key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = base + r * kSortThreads + threadIdx.x;
    key[r] = 0u;
    if (i < n) {
      key[r] = cell_key(x[i], y[i], minx, miny, inv, ncol, nrow);
      keys[i] = key[r];
      vals[i] = (uint32_t)i;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r)
    if (base + r * kSortThreads + (int)threadIdx.x < n) atomicAdd(&h[key[r] & (R - 1)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kSortThreads) hist[(size_t)d * nblocks + blockIdx.x] = h[d];
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;

// Exclusive block scan of one value per thread; returns the block total in *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t wpre = 0, tot = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) wpre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return wpre + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, size_t len,
                                                              uint32_t* __restrict__ sums) {
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < len) s += in[base + i];
  uint32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// The exclusive prefix of block b: the sum of the totals sums[0 .. b) of the blocks before it
// (the same value in every thread).
__device__ inline uint32_t block_prefix(const uint32_t* __restrict__ sums, int b) {
  uint32_t s = 0;
  for (int i = threadIdx.x; i < b; i += kScanThreads) s += sums[i];
  uint32_t tot;
  block_exclusive_scan(s, &tot);
  return tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ in, size_t len,
                                                            const uint32_t* __restrict__ sums,
                                                            uint32_t* __restrict__ out) {
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < len ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  const uint32_t pre = block_prefix(sums, blockIdx.x);
  uint32_t run = pre + block_exclusive_scan(s, &tot);
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < len) out[base + i] = run;
    run += v[i];
  }
}

// The last pass of an exclusive scan of 0 / 1 flags fused with the compaction it serves:
// list[number of flagged positions before i] = vals[i] for each flagged i, in order, and
// *total = the number of flagged positions.
__global__ __launch_bounds__(kScanThreads) void k_scan_compact(const uint32_t* __restrict__ flag, size_t len,
                                                               const uint32_t* __restrict__ sums,
                                                               const uint32_t* __restrict__ vals,
                                                               uint32_t* __restrict__ list,
                                                               uint32_t* __restrict__ total) {
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < len ? flag[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  const uint32_t pre = block_prefix(sums, blockIdx.x);
  uint32_t run = pre + block_exclusive_scan(s, &tot);
  for (int i = 0; i < kScanItems; ++i) {
    if (v[i]) list[run] = vals[base + i];
    run += v[i];
  }
  if (base < len && len <= base + kScanItems) *total = run;  // the thread holding the last flag
}

// Stable scatter of one digit: within a block, elements are taken in index order,
// one per thread per round; a wavefront ranks equal digits with ballots, waves
// are ordered by an LDS prefix, rounds by a running per-digit base.  A thread's
// elements are all loaded before the first round.  wcnt[w][d] holds wave w's
// count of digit d in the current round and is zero otherwise: the lane that
// wrote it (the digit's first lane in the wave) clears it once the round's
// positions are taken and adds the count to base[d].  Two barriers per round:
// after the counts are written, and after they are read; a wave's clear and its
// next write of the same entry are ordered by the wave's own program order.
template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint32_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, int n, int shift,
                                                                const uint32_t* __restrict__ offs, int nblocks) {
  constexpr int W = kSortThreads / 64;
  constexpr int R = 1 << BITS;
  __shared__ uint32_t base[R];
  __shared__ uint32_t wcnt[W][R];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = blockIdx.x * kSortTile;
  uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int i = tile + r * kSortThreads + tid;
    key[r] = i < n ? kin[i] : 0u;
    val[r] = i < n ? vin[i] : 0u;
  }
  for (int d = tid; d < R; d += kSortThreads) base[d] = offs[(size_t)d * nblocks + blockIdx.x];
  for (int d = tid; d < W * R; d += kSortThreads) (&wcnt[0][0])[d] = 0;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = tile + r * kSortThreads + tid < n;
    const uint32_t d = (key[r] >> shift) & (R - 1);
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      match &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(match & lt_mask);
    const uint32_t cnt = __popcll(match);
    const bool leader = valid && rank == 0;
    if (leader) wcnt[wave][d] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
      const uint32_t pos = base[d] + pre + rank;
      kout[pos] = key[r];
      vout[pos] = val[r];
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&base[d], cnt);
      wcnt[wave][d] = 0;
    }
  }
}

// CSR offsets: cell_start[c] = first sorted position whose key >= c (c = 0 .. ncells).
__global__ __launch_bounds__(256) void k_cell_start(const uint32_t* __restrict__ keys, int n, int64_t ncells,
                                                    int32_t* __restrict__ start) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncells) return;
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[c] = lo;
}

__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ vals, int n, const float* __restrict__ x,
                                                const float* __restrict__ y, float* __restrict__ sx,
                                                float* __restrict__ sy, int32_t* __restrict__ sidx) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t v = vals[p];
  sx[p] = x[v];
  sy[p] = y[v];
  sidx[p] = (int32_t)v;
}

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// 32-bit finaliser of MurmurHash3 (Appleby): a bijective avalanche mix.
__device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__global__ __launch_bounds__(256) void k_shuffle_keys(uint32_t seed_lo, uint32_t seed_hi, int epoch, int count,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  keys[i] = fmix32(fmix32((uint32_t)i ^ seed_lo) + fmix32((uint32_t)epoch ^ seed_hi));
  vals[i] = (uint32_t)i;
}

}  // namespace

hipError_t launch_shuffle_keys(uint64_t seed, int epoch, int count, uint32_t* keys, uint32_t* vals, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shuffle_keys, dim3(div_up(count, 256)), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), epoch, count, keys, vals);
  return hipGetLastError();
}

hipError_t launch_bounds(const float* x, const float* y, int n, const float* qx, const float* qy, int m,
                         BoundsPartial* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_bounds, dim3(kBoundsBlocks), dim3(kBoundsThreads), 0, s, x, y, n, qx, qy, m, partial);
  return hipGetLastError();
}

hipError_t launch_finalize(const BoundsPartial* partial, int nparts, int64_t n, double area_in, double cw_in,
                           double occ, GridScalars* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partial, nparts, n, area_in, cw_in, occ, out);
  return hipGetLastError();
}

hipError_t bin_queries(const GridScalars* gs, const float* qx, const float* qy, int m, int64_t ncells, uint32_t* cnt,
                       uint32_t* key, uint32_t* slot, uint32_t* scan_tmp, uint32_t* order, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t len = ncells + 1;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)div_up(len, 256)), dim3(256), 0, s, cnt, len, 0u);
  hipLaunchKernelGGL(k_query_slots, dim3(div_up(m, 256)), dim3(256), 0, s, qx, qy, m, gs, cnt, key, slot);
  hipError_t e = exclusive_scan_u32(cnt, cnt, (size_t)len, scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_query_place, dim3(div_up(m, 256)), dim3(256), 0, s, key, slot, m, cnt, order);
  return hipGetLastError();
}

size_t radix_hist_words(int n) { return (size_t)kRadixMax * (size_t)div_up(n > 0 ? n : 1, kSortTile); }

size_t radix_scan_tmp_words(int n) { return (size_t)div_up((int64_t)radix_hist_words(n), kScanChunk) + 1; }

namespace {
template <int BITS>
void radix_pass(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, int n, int shift, uint32_t* hist,
                uint32_t* scan_tmp, hipStream_t s) {
  const int nblocks = div_up(n, kSortTile);
  const size_t hlen = ((size_t)1 << BITS) * nblocks;
  const int nsb = div_up((int64_t)hlen, kScanChunk);
  hipLaunchKernelGGL(k_radix_hist<BITS>, dim3(nblocks), dim3(kSortThreads), 0, s, ki, n, shift, hist, nblocks);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kScanThreads), 0, s, hist, hlen, scan_tmp);
  hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kScanThreads), 0, s, hist, hlen, scan_tmp, hist);
  hipLaunchKernelGGL(k_radix_scatter<BITS>, dim3(nblocks), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n, shift, hist,
                     nblocks);
}

template <int BITS>
hipError_t radix_sort_passes(uint32_t*& ki, uint32_t*& vi, uint32_t*& ko, uint32_t*& vo, int n, int shift0, int bits,
                             uint32_t* hist, uint32_t* scan_tmp, hipStream_t s) {
  for (int shift = shift0; shift < bits; shift += BITS) {
    radix_pass<BITS>(ki, vi, ko, vo, n, shift, hist, scan_tmp, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* t = ki;
    ki = ko;
    ko = t;
    t = vi;
    vi = vo;
    vo = t;
  }
  return hipSuccess;
}
}  // namespace

hipError_t cell_keys_first_pass(const float* x, const float* y, int n, const GridScalars* gs, uint32_t* keys,
                                uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, uint32_t* hist,
                                uint32_t* scan_tmp, hipStream_t s) {
  constexpr int BITS = kRadixBitsWide;
  const int nblocks = div_up(n, kSortTile);
  const size_t hlen = ((size_t)1 << BITS) * nblocks;
  const int nsb = div_up((int64_t)hlen, kScanChunk);
  hipLaunchKernelGGL(k_radix_hist_cells<BITS>, dim3(nblocks), dim3(kSortThreads), 0, s, x, y, n, gs, keys, vals, hist,
                     nblocks);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kScanThreads), 0, s, hist, hlen, scan_tmp);
  hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kScanThreads), 0, s, hist, hlen, scan_tmp, hist);
  hipLaunchKernelGGL(k_radix_scatter<BITS>, dim3(nblocks), dim3(kSortThreads), 0, s, keys, vals, tmp_keys, tmp_vals, n,
                     0, hist, nblocks);
  return hipGetLastError();
}
hipError_t radix_sort_wide_from(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, int n,
                                int shift0, int bits, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s,
                                uint32_t** out_keys, uint32_t** out_vals) {
  *out_keys = keys;
  *out_vals = vals;
  if (n <= 1) return hipSuccess;
  uint32_t *ki = keys, *vi = vals, *ko = tmp_keys, *vo = tmp_vals;
  hipError_t e = radix_sort_passes<kRadixBitsWide>(ki, vi, ko, vo, n, shift0, bits, hist, scan_tmp, s);
  *out_keys = ki;
  *out_vals = vi;
  return e;
}

hipError_t radix_sort_pairs_to(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, int n, int bits,
                               uint32_t* hist, uint32_t* scan_tmp, hipStream_t s, uint32_t** out_keys,
                               uint32_t** out_vals) {
  *out_keys = keys;
  *out_vals = vals;
  if (n <= 1 || bits <= 0) return hipSuccess;
  uint32_t *ki = keys, *vi = vals, *ko = tmp_keys, *vo = tmp_vals;
  // 10-bit digits where they save a pass (each pass is five launches), 8-bit ones otherwise
  const bool wide = (bits + kRadixBitsWide - 1) / kRadixBitsWide < (bits + kRadixBits - 1) / kRadixBits;
  hipError_t e = wide ? radix_sort_passes<kRadixBitsWide>(ki, vi, ko, vo, n, 0, bits, hist, scan_tmp, s)
                      : radix_sort_passes<kRadixBits>(ki, vi, ko, vo, n, 0, bits, hist, scan_tmp, s);
  *out_keys = ki;
  *out_vals = vi;
  return e;
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, int n, int bits,
                            uint32_t* hist, uint32_t* scan_tmp, hipStream_t s) {
  uint32_t *rk, *rv;
  hipError_t e = radix_sort_pairs_to(keys, vals, tmp_keys, tmp_vals, n, bits, hist, scan_tmp, s, &rk, &rv);
  if (e != hipSuccess || rk == keys) return e;
  // an odd number of passes: the result is in the temporaries; copy it back
  e = hipMemcpyAsync(keys, rk, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(vals, rv, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
}

namespace {
__global__ void k_scan_total(const uint32_t* __restrict__ in, const uint32_t* __restrict__ ex, size_t len,
                             uint32_t* __restrict__ total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = len ? ex[len - 1] + in[len - 1] : 0u;
}
}  // namespace

size_t scan_tmp_words(size_t len) { return (len + kScanChunk - 1) / kScanChunk + 1; }

hipError_t compact_flags(const uint32_t* flag, const uint32_t* vals, size_t len, uint32_t* tmp, uint32_t* list,
                         uint32_t* total, hipStream_t s) {
  if (len == 0) return hipSuccess;
  const int nsb = (int)((len + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kScanThreads), 0, s, flag, len, tmp);
  hipLaunchKernelGGL(k_scan_compact, dim3(nsb), dim3(kScanThreads), 0, s, flag, len, tmp, vals, list, total);
  return hipGetLastError();
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t len, uint32_t* tmp, uint32_t* total,
                              hipStream_t s) {
  if (len == 0) return hipSuccess;
  const int nsb = (int)((len + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kScanThreads), 0, s, in, len, tmp);
  hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kScanThreads), 0, s, in, len, tmp, out);
  if (total) hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, in, out, len, total);
  return hipGetLastError();
}

hipError_t launch_cell_start_gather(const uint32_t* keys, const uint32_t* vals, int n, int64_t ncells, const float* x,
                                    const float* y, int32_t* cell_start, float* sx, float* sy, int32_t* sidx,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_cell_start, dim3(div_up(ncells + 1, 256)), dim3(256), 0, s, keys, n, ncells, cell_start);
  if (sx) hipLaunchKernelGGL(k_gather, dim3(div_up(n, 256)), dim3(256), 0, s, vals, n, x, y, sx, sy, sidx);
  return hipGetLastError();
}

}  // namespace aidw
