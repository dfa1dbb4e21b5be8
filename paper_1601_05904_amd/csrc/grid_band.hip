// Stage 1, grid build (Section 3.2.1-3.2.3 and 4.1.1-4.1.3 of the paper) together with
// the binning of the queries (Section 3.2.4), in five launches and without waiting for
// the host:
//
//   k_bounds          min / max of x and y over data and queries, per block.
//   k_band_hist       every block reduces the bounds partials and derives the grid
//                     scalars itself (Eq. 2; block 0 stores them), then counts its tile
//                     of points per digit: the digit of a data point is its band (the
//                     cell index >> band_shift), a query's is nbands + its band.
//   k_band_prefix     per digit, the exclusive scan of its counts over the blocks, and the
//                     digit's total (16 digits per block).
//   k_band_scatter    a stable counting sort of each tile by digit: ranks from wavefront
//                     ballots, the tile sorted in LDS, then written out in runs, so each
//                     block writes contiguous pieces of every digit's segment.
//   k_band_local      one block per digit: a stable counting sort of the digit's segment
//                     by cell inside the band; data blocks write the CSR offsets of their
//                     band's cells (head of cell c = cell_start[c], size = cell_start[c + 1]
//                     - cell_start[c], Section 3.2.3) and the points in cell order; query
//                     blocks write the queries in cell order.
//
// Every sort step is stable, so each cell's segment lists its points in index order, as
// the single stable sort of the paper's sort_by_key would.  The grid's cell count is not
// known on the host: arrays are sized for a cell budget and the finalize step widens the
// cell side if the bounds would need more cells (the kNN result does not depend on the
// side).  A failed status (non-finite coordinate, degenerate area) comes with one-cell
// scalars, so every kernel stays in bounds.
#include "aidw_internal.h"
#include "grid_core.h"

namespace aidw {

namespace {

constexpr int kThreads = 512;             // k_band_hist, k_band_scatter
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // points per block of k_band_hist / k_band_scatter
constexpr int kWaves = kThreads / 64;
constexpr int kDigits = 2 * kMaxBands;    // data bands, then query bands
constexpr int kDigitBits = 11;            // kDigits = 2^kDigitBits
static_assert(kDigits == 1 << kDigitBits, "digit count");
constexpr int kLocalThreads = 512;        // k_band_local
constexpr int kLocalItems = 8;
constexpr int kLocalTile = kLocalThreads * kLocalItems;  // points staged in LDS per band
constexpr int kLocalWaves = kLocalThreads / 64;

// Cell coordinate of a float32 offset t = (v - min) * inv_cw: truncated and clamped into
// [0, nc); NaN or negative -> 0 (the same cell formula as the oracle's for finite inputs).
__device__ inline int clamp_cell(float t, int nc) {
  if (!(t >= 0.0f)) return 0;
  if (t >= 2147483520.0f) return nc - 1;
  const int c = (int)t;
  return c > nc - 1 ? nc - 1 : c;
}

// Section 4.1.2: row * nCol + col from float32 offsets scaled by 1 / cell width.
__device__ inline uint32_t cell_of(float x, float y, const GridScalars& g) {
  const float tx = (x - g.minx) * g.inv_cw;
  const float ty = (y - g.miny) * g.inv_cw;
  return (uint32_t)clamp_cell(ty, g.nrow) * (uint32_t)g.ncol + (uint32_t)clamp_cell(tx, g.ncol);
}

// Smallest b with 2^b >= v.
__host__ __device__ inline int ceil_log2(int64_t v) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < v) ++b;
  return b;
}

// Bands of a grid: at most kMaxBands of 2^shift cells each.
__host__ __device__ inline int shift_for_cells(int64_t ncells) {
  const int bits = ceil_log2(ncells);
  return bits > 10 ? bits - 10 : 0;
}
__device__ inline void set_bands(GridScalars& g) {
  const int shift = shift_for_cells(g.ncells);
  g.band_shift = shift;
  g.nbands = (int32_t)((g.ncells + ((int64_t)1 << shift) - 1) >> shift);
  if (shift > kMaxBandShift && g.status == AIDW_OK) {
    // the host never sizes a banded build beyond kBandMaxCells; keep every kernel in bounds
    g.status = AIDW_ECAPACITY;
    g.ncol = g.nrow = 1;
    g.ncells = 1;
    g.inv_cw = 0.0f;
    g.band_shift = 0;
    g.nbands = 1;
  }
}

// Exclusive scan of one value per thread over a block of NT threads; *total = the block's sum.
template <int NT>
__device__ inline uint32_t block_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[NT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wave) pre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return pre + incl - v;
}

// In-place exclusive scan of a[0, len) in LDS by NT threads (len a multiple of NT, at most 8 NT);
// returns the total.
template <int NT>
__device__ inline uint32_t lds_exclusive_scan(uint32_t* a, int len) {
  const int per = len / NT;
  uint32_t v[8];
  uint32_t s = 0;
  for (int i = 0; i < per; ++i) {
    v[i] = a[threadIdx.x * per + i];
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = block_scan<NT>(s, &tot);
  for (int i = 0; i < per; ++i) {
    a[threadIdx.x * per + i] = run;
    run += v[i];
  }
  __syncthreads();
  return tot;
}

// Lanes of the wavefront holding the same key as this lane (bits of the key below `bits`),
// among the lanes in `live`.
__device__ inline uint64_t match_key(uint32_t key, int bits, uint64_t live) {
  uint64_t match = live;
  for (int b = 0; b < bits; ++b) {
    const bool bit = (key >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    match &= bit ? bb : ~bb;
  }
  return match;
}

// Number of the 16-bit values a[lo, hi) below `me`; a is 16-byte aligned, read 8 values per load.
__device__ inline uint32_t count_below(const uint16_t* a, uint32_t lo, uint32_t hi, uint16_t me) {
  uint32_t r = 0, j = lo;
  for (; j < hi && (j & 7u); ++j) r += a[j] < me ? 1u : 0u;
  const uint4* v = reinterpret_cast<const uint4*>(a);
  const uint32_t m = me;
  auto below2 = [m](uint32_t w) { return ((w & 0xffffu) < m ? 1u : 0u) + ((w >> 16) < m ? 1u : 0u); };
  for (; j + 8 <= hi; j += 8) {
    const uint4 q = v[j >> 3];
    r += below2(q.x) + below2(q.y) + below2(q.z) + below2(q.w);
  }
  for (; j < hi; ++j) r += a[j] < me ? 1u : 0u;
  return r;
}

// Element e of the joint index space (data points [0, n), then queries).
struct Elem {
  uint32_t idx;  // index within its set
  float x, y;
  bool query;
};
__device__ inline Elem load_elem(int64_t e, int64_t n, const float* __restrict__ x, const float* __restrict__ y,
                                 const float* __restrict__ qx, const float* __restrict__ qy) {
  Elem r;
  r.query = e >= n;
  if (!r.query) {
    r.idx = (uint32_t)e;
    r.x = x[e];
    r.y = y[e];
  } else {
    r.idx = (uint32_t)(e - n);
    r.x = qx[e - n];
    r.y = qy[e - n];
  }
  return r;
}

// Grid scalars reduced from the bounds partials by every block (block 0 stores them), then
// the tile's per-digit counts, block-major: hist[block][digit].
__global__ __launch_bounds__(kThreads) void k_band_hist(const BoundsPartial* __restrict__ partial, int nparts,
                                                        int64_t n, int64_t total, double area_in, double cw_in,
                                                        double occ, int64_t cap, const float* __restrict__ x,
                                                        const float* __restrict__ y, const float* __restrict__ qx,
                                                        const float* __restrict__ qy, GridScalars* __restrict__ gs_out,
                                                        uint32_t* __restrict__ hist) {
  __shared__ GridScalars sg;
  __shared__ uint32_t h[kDigits];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  // the tile's loads are issued before the bounds reduction, which they do not depend on
  Elem el[kItems];
  bool ok[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t e = base + it * kThreads + threadIdx.x;
    ok[it] = e < total;
    el[it] = ok[it] ? load_elem(e, n, x, y, qx, qy) : Elem{0u, 0.0f, 0.0f, false};
  }
  const BoundsPartial r = gridc::block_reduce_bounds(partial, 0, nparts);
  if (threadIdx.x == 0) {
    GridScalars g = gridc::grid_scalars(r.minx, r.miny, r.maxx, r.maxy, r.nonfinite != 0, n, area_in, cw_in, occ,
                                        cap);
    set_bands(g);
    sg = g;
    if (blockIdx.x == 0) *gs_out = g;
  }
  for (int i = threadIdx.x; i < kDigits; i += kThreads) h[i] = 0;
  __syncthreads();
  const GridScalars g = sg;
#pragma unroll
  for (int it = 0; it < kItems; ++it)
    if (ok[it])
      atomicAdd(&h[(cell_of(el[it].x, el[it].y, g) >> g.band_shift) + (el[it].query ? (uint32_t)g.nbands : 0u)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kDigits; d += kThreads) hist[(size_t)blockIdx.x * kDigits + d] = h[d];
}

// For 16 digits per block: each digit's counts over the blocks -> their exclusive prefix (in
// place), and the digit's total.  Thread (slice, j) walks a slice of the blocks for digit j, so
// a wavefront reads 16 consecutive words of four blocks' rows; 64 slices keep each thread's
// chain of dependent loads short (at 2^21 points, 8 rows per slice).
constexpr int kPrefixDigits = 16;
constexpr int kPrefixSlices = 64;
__global__ __launch_bounds__(kPrefixDigits * kPrefixSlices) void k_band_prefix(uint32_t* __restrict__ hist, int nblk,
                                                                               uint32_t* __restrict__ totals) {
  __shared__ uint32_t part[kPrefixSlices][kPrefixDigits];
  const int j = threadIdx.x % kPrefixDigits, slice = threadIdx.x / kPrefixDigits;
  const int d = blockIdx.x * kPrefixDigits + j;
  const int per = (nblk + kPrefixSlices - 1) / kPrefixSlices;
  const int b0 = slice * per, b1 = min(nblk, b0 + per);
  uint32_t sum = 0;
  int b = b0;
  for (; b + 4 <= b1; b += 4) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = hist[(size_t)(b + u) * kDigits + d];
    sum += v[0] + v[1] + v[2] + v[3];
  }
  for (; b < b1; ++b) sum += hist[(size_t)b * kDigits + d];
  part[slice][j] = sum;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (int s = 0; s < kPrefixSlices; ++s) {
    if (s < slice) run += part[s][j];
    tot += part[s][j];
  }
  for (b = b0; b + 4 <= b1; b += 4) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = hist[(size_t)(b + u) * kDigits + d];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      hist[(size_t)(b + u) * kDigits + d] = run;
      run += v[u];
    }
  }
  for (; b < b1; ++b) {
    const size_t i = (size_t)b * kDigits + d;
    const uint32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
  if (slice == 0) totals[d] = tot;
}

// Stable counting sort of one tile by digit, then each digit's run written to its segment at
// this block's prefix.  The tile's counts per digit (LDS atomics) and their exclusive scan give
// each digit's run in the tile.  Two ways to order a run by index:
//   rank path    (no digit holds more than kScatterRankMaxRun of the tile's elements): each
//                element takes a slot of its run by an LDS atomic, then its place in the run
//                is the number of the run's elements at a smaller tile position (tile position
//                order is index order);
//   ballot path  (otherwise): round it (0 .. kItems) takes element base + it * kThreads +
//                thread; a wavefront ranks equal digits by ballots, earlier wavefronts of the
//                round are counted through wcnt (written by each digit's leader lane, cleared
//                by it after the round), earlier rounds through the running cursor cur.
// The tile keeps tile positions (16 bits; the element is base + position) and coordinates.
constexpr int kScatterRankMaxRun = 64;
__global__ __launch_bounds__(kThreads) void k_band_scatter(const GridScalars* __restrict__ gs, int64_t n, int64_t total,
                                                           const float* __restrict__ x, const float* __restrict__ y,
                                                           const float* __restrict__ qx, const float* __restrict__ qy,
                                                           const uint32_t* __restrict__ prefix,
                                                           const uint32_t* __restrict__ totals,
                                                           uint32_t* __restrict__ dstart, uint32_t* __restrict__ oidx,
                                                           float* __restrict__ ox, float* __restrict__ oy) {
  static_assert(kTile <= 65536, "tile positions are 16-bit");
  __shared__ uint16_t t_pos[kTile];
  __shared__ float t_x[kTile], t_y[kTile];
  __shared__ __align__(16) union {
    uint16_t r_pos[kTile];            // rank path: tile positions in slot order
    uint8_t wcnt[kWaves][kDigits];    // ballot path
  } u;
  __shared__ uint32_t loff[kDigits];  // the tile's counts, then each digit's run start in the tile
  __shared__ uint32_t cur[kDigits];   // run cursors, then each digit's output start for this block
  __shared__ uint32_t s_maxrun;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // tiles in XCD-aware order: consecutive tiles write adjacent runs of each digit's segment
  // (partial cache lines), so on one XCD they meet in its L2 before going to HBM
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t base = (int64_t)tile * kTile;
  Elem el[kItems];
  bool ok[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t e = base + it * kThreads + tid;
    ok[it] = e < total;
    el[it] = ok[it] ? load_elem(e, n, x, y, qx, qy) : Elem{0u, 0.0f, 0.0f, false};
  }
  const GridScalars g = *gs;
  const uint32_t nb = (uint32_t)g.nbands;
  uint32_t dig[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it)
    dig[it] = ok[it] ? (cell_of(el[it].x, el[it].y, g) >> g.band_shift) + (el[it].query ? nb : 0u) : 0u;
  for (int d = tid; d < kDigits; d += kThreads) loff[d] = 0u;
  if (tid == 0) s_maxrun = 0u;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it)
    if (ok[it]) atomicAdd(&loff[dig[it]], 1u);
  __syncthreads();
  {
    uint32_t mx = 0u;
    for (int d = tid; d < kDigits; d += kThreads) mx = max(mx, loff[d]);
    if (mx > 0u) atomicMax(&s_maxrun, mx);
  }
  lds_exclusive_scan<kThreads>(loff, kDigits);
  for (int d = tid; d < kDigits; d += kThreads) cur[d] = loff[d];
  __syncthreads();
  if (s_maxrun <= (uint32_t)kScatterRankMaxRun) {
#pragma unroll
    for (int it = 0; it < kItems; ++it)
      if (ok[it]) u.r_pos[atomicAdd(&cur[dig[it]], 1u)] = (uint16_t)(it * kThreads + tid);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it)
      if (ok[it]) {
        const uint32_t d = dig[it], lo = loff[d], hi = cur[d];
        const uint16_t me = (uint16_t)(it * kThreads + tid);
        const uint32_t pos = lo + count_below(u.r_pos, lo, hi, me);
        t_pos[pos] = me;
        t_x[pos] = el[it].x;
        t_y[pos] = el[it].y;
      }
  } else {
    for (int i = tid; i < kWaves * kDigits; i += kThreads) (&u.wcnt[0][0])[i] = 0;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const uint32_t d = dig[it];
      const uint64_t match = match_key(d, kDigitBits, __ballot(ok[it]));
      const uint32_t rank = __popcll(match & lt_mask);
      const uint32_t cnt = __popcll(match);
      const bool leader = ok[it] && rank == 0;
      if (leader) u.wcnt[wave][d] = (uint8_t)cnt;
      __syncthreads();
      if (ok[it]) {
        uint32_t pre = 0;
        for (int w = 0; w < wave; ++w) pre += u.wcnt[w][d];
        const uint32_t pos = cur[d] + pre + rank;
        t_pos[pos] = (uint16_t)(it * kThreads + tid);
        t_x[pos] = el[it].x;
        t_y[pos] = el[it].y;
      }
      __syncthreads();
      if (leader) {
        atomicAdd(&cur[d], cnt);
        u.wcnt[wave][d] = 0;
      }
    }
  }
  __syncthreads();
  // each digit's output start for this block: the digit's start (exclusive scan of the totals,
  // stored by block 0) plus this block's prefix within the digit
  for (int d = tid; d < kDigits; d += kThreads) cur[d] = totals[d];
  __syncthreads();
  const uint32_t all = lds_exclusive_scan<kThreads>(cur, kDigits);
  const uint32_t* row = prefix + (size_t)tile * kDigits;
  for (int d = tid; d < kDigits; d += kThreads) {
    if (tile == 0) dstart[d] = cur[d];
    cur[d] += row[d];
  }
  if (tile == 0 && tid == 0) dstart[kDigits] = all;
  __syncthreads();
  const int64_t left = total - base;
  const int cnt_blk = left < kTile ? (int)left : kTile;
  for (int i = tid; i < cnt_blk; i += kThreads) {
    const int64_t e = base + t_pos[i];
    const bool query = e >= n;
    const float px = t_x[i], py = t_y[i];
    const uint32_t d = (cell_of(px, py, g) >> g.band_shift) + (query ? nb : 0u);
    const uint32_t gp = cur[d] + ((uint32_t)i - loff[d]);
    oidx[gp] = (uint32_t)(query ? e - n : e);
    ox[gp] = px;
    oy[gp] = py;
  }
}

// One block per digit: the stable counting sort of the digit's segment by cell inside its
// band.  The segment arrives in index order (the scatter is stable).  The cells' counts (LDS
// atomics) and their exclusive scan give the CSR offsets, which data blocks write (head of
// cell c = cell_start[c], size = cell_start[c + 1] - cell_start[c], Section 3.2.3).  Two ways
// to order the points inside each cell by index:
//   rank path    (no cell of the band holds more than kRankMaxCell points): the segment is
//                taken in chunks of kLocalTile points in order; in a chunk every point takes a
//                slot of its cell by an LDS atomic, its place among the chunk's points of the
//                cell is the number of them at a smaller segment position, and the chunks
//                before it add their counts of the cell;
//   ballot path  (otherwise): the segment is ranked in rounds of kLocalThreads points by
//                wavefront ballots on the local cell key, earlier rounds counted by a running
//                cursor per cell.
// A segment of one chunk is held in registers from the start (its counts come from them) and
// its sorted points are staged in LDS and written out in one coalesced pass; otherwise each
// point is written straight to its place in the segment.  Query blocks write the queries in
// cell order (and their coordinates).  Dynamic LDS: cnt [CB] (counts, then the cells' offsets
// in the segment), then one region used by one path:
//   rank path, one chunk   r_pos (16-bit chunk positions in slot order) [kLocalTile], then the
//                          sorted index, x, y [kLocalTile] each;
//   rank path, chunks      r_pos [kLocalTile], then done, coff, ccur [CB] each (the cell's points
//                          in earlier chunks; the chunk's run start and cursor per cell);
//   ballot path            wcnt [kLocalWaves][CB] bytes;
// CB = the largest band the host sized for.
constexpr int kRankMaxCell = 256;
__global__ __launch_bounds__(kLocalThreads) void k_band_local(const GridScalars* __restrict__ gs, int64_t n,
                                                              int cb_max, const uint32_t* __restrict__ dstart,
                                                              const uint32_t* __restrict__ bidx,
                                                              const float* __restrict__ bx,
                                                              const float* __restrict__ by,
                                                              int32_t* __restrict__ cell_start,
                                                              float* __restrict__ sx, float* __restrict__ sy,
                                                              int32_t* __restrict__ sidx,
                                                              uint32_t* __restrict__ qorder, float* __restrict__ qsx,
                                                              float* __restrict__ qsy) {
  static_assert(kLocalTile <= 65536, "chunk positions are 16-bit");
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t s_max;  // the largest cell count of the band
  const GridScalars g = *gs;
  const int nb = g.nbands;
  const int d = blockIdx.x;
  if (d >= 2 * nb) return;
  const bool query = d >= nb;
  const int band = query ? d - nb : d;
  const int shift = g.band_shift;
  const int cb = 1 << shift;
  const uint32_t cell0 = (uint32_t)band << shift;
  const int ncb = (int)(g.ncells - (int64_t)cell0 < cb ? g.ncells - (int64_t)cell0 : cb);
  uint32_t* cnt = lds;
  uint32_t* region = lds + ((cb_max + 3) & ~3);            // 16-byte aligned
  uint16_t* r_pos = reinterpret_cast<uint16_t*>(region);  // rank paths
  uint32_t* o_idx = region + kLocalTile / 2;               // one chunk
  float* o_x = reinterpret_cast<float*>(o_idx + kLocalTile);
  float* o_y = o_x + kLocalTile;
  uint32_t* done = region + kLocalTile / 2;                // chunks
  uint32_t* coff = done + cb_max;
  uint32_t* ccur = coff + cb_max;
  uint8_t* wcnt = reinterpret_cast<uint8_t*>(region);     // ballot path: [kLocalWaves][cb]
  const uint32_t s = dstart[d], e = dstart[d + 1];
  const bool one_chunk = e - s <= (uint32_t)kLocalTile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // in-place exclusive scan of a[0, cb); with `offsets`, the cells' CSR offsets are stored.
  // Other threads' entries are only complete after the caller's next barrier.
  auto scan_cells = [&](uint32_t* a, bool offsets) {
    uint32_t carry = 0;
    for (int c0 = 0; c0 < cb; c0 += kLocalThreads * 4) {
      uint32_t v[4];
      uint32_t sum = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = c0 + tid * 4 + i;
        v[i] = j < cb ? a[j] : 0u;
        sum += v[i];
      }
      uint32_t tot;
      uint32_t run = carry + block_scan<kLocalThreads>(sum, &tot);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = c0 + tid * 4 + i;
        if (j < cb) {
          a[j] = run;
          if (offsets && j < ncb) cell_start[cell0 + j] = (int32_t)(s + run);
        }
        run += v[i];
      }
      carry += tot;
    }
  };
  // the point at segment position p < end: local cell, index, x, y (lk = ~0u past the end)
  auto load_point = [&](uint32_t p, uint32_t end, uint32_t& lk, uint32_t& id, float& px, float& py) {
    lk = 0xffffffffu;
    id = 0u;
    px = py = 0.0f;
    if (p < end) {
      px = bx[p];
      py = by[p];
      id = bidx[p];
      lk = cell_of(px, py, g) - cell0;
    }
  };
  // writes the sorted point at segment position i
  auto emit = [&](uint32_t i, uint32_t pid, float fx, float fy) {
    if (!query) {
      sidx[s + i] = (int32_t)pid;
      sx[s + i] = fx;
      sy[s + i] = fy;
    } else {
      const uint32_t qp = s + i - (uint32_t)n;
      qorder[qp] = pid;
      if (qsx) {
        qsx[qp] = fx;
        qsy[qp] = fy;
      }
    }
  };

  for (int i = tid; i < cb; i += kLocalThreads) cnt[i] = 0u;
  if (tid == 0) s_max = 0u;
  uint32_t lk[kLocalItems], id[kLocalItems];
  float px[kLocalItems], py[kLocalItems];
  if (one_chunk) {
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it) load_point(s + it * kLocalThreads + tid, e, lk[it], id[it], px[it], py[it]);
  }
  __syncthreads();
  if (one_chunk) {
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      if (lk[it] != 0xffffffffu) atomicAdd(&cnt[lk[it]], 1u);
  } else {
    // eight loads in flight per thread
    uint32_t p = s + tid;
    for (; p + 7 * kLocalThreads < e; p += 8 * kLocalThreads) {
      float ax[8], ay[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        ax[u] = bx[p + u * kLocalThreads];
        ay[u] = by[p + u * kLocalThreads];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) atomicAdd(&cnt[cell_of(ax[u], ay[u], g) - cell0], 1u);
    }
    for (; p < e; p += kLocalThreads) atomicAdd(&cnt[cell_of(bx[p], by[p], g) - cell0], 1u);
  }
  __syncthreads();
  {
    uint32_t mx = 0u;
    for (int i = tid; i < cb; i += kLocalThreads) mx = max(mx, cnt[i]);
    if (mx > 0u) atomicMax(&s_max, mx);
  }
  scan_cells(cnt, !query);
  if (!query && band == nb - 1 && tid == 0) cell_start[g.ncells] = (int32_t)e;
  __syncthreads();
  if (s_max <= (uint32_t)kRankMaxCell && one_chunk) {
    // a slot of the point's cell, then its place among the cell's points
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      if (lk[it] != 0xffffffffu) r_pos[atomicAdd(&cnt[lk[it]], 1u)] = (uint16_t)(it * kLocalThreads + tid);
    __syncthreads();
    // cnt[c] is now the end of cell c, which is the start of cell c + 1
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      if (lk[it] != 0xffffffffu) {
        const uint32_t c = lk[it];
        const uint32_t c_end = cnt[c], c_begin = c == 0 ? 0u : cnt[c - 1];
        const uint16_t me = (uint16_t)(it * kLocalThreads + tid);
        const uint32_t pos = c_begin + count_below(r_pos, c_begin, c_end, me);
        o_idx[pos] = id[it];
        o_x[pos] = px[it];
        o_y[pos] = py[it];
      }
    __syncthreads();
    for (uint32_t i = tid; i < e - s; i += kLocalThreads) emit(i, o_idx[i], o_x[i], o_y[i]);
    return;
  }
  if (s_max <= (uint32_t)kRankMaxCell) {
    for (int i = tid; i < cb; i += kLocalThreads) done[i] = 0u;
    for (uint32_t c0 = s; c0 < e; c0 += kLocalTile) {
      const uint32_t c1 = e - c0 < (uint32_t)kLocalTile ? e : c0 + kLocalTile;
      uint32_t ck[kLocalItems], cid[kLocalItems];
      float cx[kLocalItems], cy[kLocalItems];
#pragma unroll
      for (int it = 0; it < kLocalItems; ++it) load_point(c0 + it * kLocalThreads + tid, c1, ck[it], cid[it], cx[it], cy[it]);
      for (int i = tid; i < cb; i += kLocalThreads) coff[i] = 0u;
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kLocalItems; ++it)
        if (ck[it] != 0xffffffffu) atomicAdd(&coff[ck[it]], 1u);
      __syncthreads();
      scan_cells(coff, false);
      __syncthreads();
      for (int i = tid; i < cb; i += kLocalThreads) ccur[i] = coff[i];
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kLocalItems; ++it)
        if (ck[it] != 0xffffffffu) r_pos[atomicAdd(&ccur[ck[it]], 1u)] = (uint16_t)(it * kLocalThreads + tid);
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kLocalItems; ++it)
        if (ck[it] != 0xffffffffu) {
          const uint32_t c = ck[it];
          const uint32_t lo = coff[c], hi = ccur[c];
          const uint16_t me = (uint16_t)(it * kLocalThreads + tid);
          const uint32_t pos = cnt[c] + done[c] + count_below(r_pos, lo, hi, me);
          emit(pos, cid[it], cx[it], cy[it]);
        }
      __syncthreads();
      for (int i = tid; i < cb; i += kLocalThreads) done[i] += ccur[i] - coff[i];
      __syncthreads();
    }
    return;
  }
  // ballot path: rounds of kLocalThreads points in segment order; the point of this thread goes
  // to cnt[key] + (earlier waves' and lanes' points of the same key in the round)
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int i = tid; i < kLocalWaves * cb / 4; i += kLocalThreads) reinterpret_cast<uint32_t*>(wcnt)[i] = 0u;
  __syncthreads();
  for (uint32_t r0 = s; r0 < e; r0 += kLocalThreads) {
    uint32_t key, pid;
    float fx, fy;
    load_point(r0 + tid, e, key, pid, fx, fy);
    const bool valid = key != 0xffffffffu;
    if (!valid) key = 0u;
    const uint64_t match = match_key(key, shift, __ballot(valid));
    const uint32_t rank = __popcll(match & lt_mask);
    const uint32_t c = __popcll(match);
    const bool leader = valid && rank == 0;
    if (leader) wcnt[wave * cb + key] = (uint8_t)c;
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int w = 0; w < wave; ++w) pre += wcnt[w * cb + key];
      emit(cnt[key] + pre + rank, pid, fx, fy);
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&cnt[key], c);
      wcnt[wave * cb + key] = 0;
    }
  }
}

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Dynamic LDS of k_band_local for bands of at most cb cells.
size_t local_lds_bytes(int cb) {
  const size_t w = sizeof(uint32_t);
  const size_t one_chunk = w * (kLocalTile / 2) + 3 * w * kLocalTile;
  const size_t chunks = w * (kLocalTile / 2) + 3 * w * (size_t)cb;
  const size_t ballot = (size_t)kLocalWaves * cb;
  size_t region = one_chunk > chunks ? one_chunk : chunks;
  region = region > ballot ? region : ballot;
  return w * (size_t)((cb + 3) & ~3) + region;
}

}  // namespace

size_t band_hist_words(int64_t total) { return (size_t)kDigits * (size_t)(total > 0 ? div_up(total, kTile) : 1); }

int band_shift_for(int64_t cap) { return shift_for_cells(cap); }

hipError_t build_grid_banded(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                             bool bin_q, double area_in, double cw_in, double occ, int64_t cap, GridScalars* gs,
                             int32_t* cell_start, float* sx, float* sy, int32_t* sidx, uint32_t* qorder, float* qsx,
                             float* qsy, const BandScratch& b, hipStream_t s) {
  if (cap < 1 || cap > kBandMaxCells) return hipErrorInvalidValue;
  hipError_t e = launch_bounds(x, y, (int)n, qx, qy, (int)m, b.partial, s);
  if (e != hipSuccess) return e;
  const int64_t total = n + (bin_q ? m : 0);
  const int nblk = div_up(total, kTile);
  hipLaunchKernelGGL(k_band_hist, dim3(nblk), dim3(kThreads), 0, s, b.partial, kBoundsBlocks, n, total, area_in, cw_in,
                     occ, cap, x, y, qx, qy, gs, b.hist);
  hipLaunchKernelGGL(k_band_prefix, dim3(kDigits / kPrefixDigits), dim3(kPrefixDigits * kPrefixSlices), 0, s, b.hist,
                     nblk, b.totals);
  hipLaunchKernelGGL(k_band_scatter, dim3(nblk), dim3(kThreads), 0, s, gs, n, total, x, y, qx, qy, b.hist, b.totals,
                     b.dstart, b.bidx, b.bx, b.by);
  const int cb = 1 << band_shift_for(cap);
  hipLaunchKernelGGL(k_band_local, dim3(kDigits), dim3(kLocalThreads), local_lds_bytes(cb), s, gs, n, cb, b.dstart,
                     b.bidx, b.bx, b.by, cell_start, sx, sy, sidx, qorder, qsx, qsy);
  return hipGetLastError();
}

}  // namespace aidw
