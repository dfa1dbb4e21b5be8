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
//                     digit's total (8 digits per block).
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
constexpr int kLocalThreads = 256;        // k_band_local
constexpr int kLocalItems = 16;
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

// For 8 digits per block: each digit's counts over the blocks -> their exclusive prefix (in
// place), and the digit's total.  Thread (slice, j) walks a slice of the blocks for digit j.
constexpr int kPrefixDigits = 8;
constexpr int kPrefixSlices = 32;
__global__ __launch_bounds__(kPrefixDigits * kPrefixSlices) void k_band_prefix(uint32_t* __restrict__ hist, int nblk,
                                                                               uint32_t* __restrict__ totals) {
  __shared__ uint32_t part[kPrefixSlices][kPrefixDigits];
  const int j = threadIdx.x % kPrefixDigits, slice = threadIdx.x / kPrefixDigits;
  const int d = blockIdx.x * kPrefixDigits + j;
  const int per = (nblk + kPrefixSlices - 1) / kPrefixSlices;
  const int b0 = slice * per, b1 = min(nblk, b0 + per);
  uint32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += hist[(size_t)b * kDigits + d];
  part[slice][j] = sum;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (int s = 0; s < kPrefixSlices; ++s) {
    if (s < slice) run += part[s][j];
    tot += part[s][j];
  }
  for (int b = b0; b < b1; ++b) {
    const size_t i = (size_t)b * kDigits + d;
    const uint32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
  if (slice == 0) totals[d] = tot;
}

// Stable counting sort of one tile by digit.  Round it (0 .. kItems) takes element
// base + it * kThreads + thread: a wavefront ranks equal digits by ballots, earlier
// wavefronts of the round are counted through wcnt (written by each digit's leader lane,
// cleared by it after the round), earlier rounds through the running cursor cur.  Each
// element's place in the tile's digit order goes to LDS; the sorted tile is then written
// to each digit's segment at this block's prefix, one contiguous run per digit.
__global__ __launch_bounds__(kThreads) void k_band_scatter(const GridScalars* __restrict__ gs, int64_t n, int64_t total,
                                                           const float* __restrict__ x, const float* __restrict__ y,
                                                           const float* __restrict__ qx, const float* __restrict__ qy,
                                                           const uint32_t* __restrict__ prefix,
                                                           const uint32_t* __restrict__ totals,
                                                           uint32_t* __restrict__ dstart, uint32_t* __restrict__ oidx,
                                                           float* __restrict__ ox, float* __restrict__ oy) {
  __shared__ uint32_t t_idx[kTile];
  __shared__ float t_x[kTile], t_y[kTile];
  __shared__ uint8_t wcnt[kWaves][kDigits];
  __shared__ uint32_t cur[kDigits];
  __shared__ uint32_t loff[kDigits];
  __shared__ uint32_t gstart[kDigits];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile;
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
  for (int d = tid; d < kDigits; d += kThreads) {
    cur[d] = 0u;
    gstart[d] = totals[d];
  }
  for (int i = tid; i < kWaves * kDigits; i += kThreads) (&wcnt[0][0])[i] = 0;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it)
    if (ok[it]) atomicAdd(&cur[dig[it]], 1u);
  __syncthreads();
  for (int d = tid; d < kDigits; d += kThreads) loff[d] = cur[d];
  __syncthreads();
  lds_exclusive_scan<kThreads>(loff, kDigits);
  const uint32_t all = lds_exclusive_scan<kThreads>(gstart, kDigits);
  const uint32_t* row = prefix + (size_t)blockIdx.x * kDigits;
  for (int d = tid; d < kDigits; d += kThreads) {
    if (blockIdx.x == 0) dstart[d] = gstart[d];
    cur[d] = loff[d];
    gstart[d] += row[d];
  }
  if (blockIdx.x == 0 && tid == 0) dstart[kDigits] = all;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint32_t d = dig[it];
    const uint64_t match = match_key(d, kDigitBits, __ballot(ok[it]));
    const uint32_t rank = __popcll(match & lt_mask);
    const uint32_t cnt = __popcll(match);
    const bool leader = ok[it] && rank == 0;
    if (leader) wcnt[wave][d] = (uint8_t)cnt;
    __syncthreads();
    if (ok[it]) {
      uint32_t pre = 0;
      for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
      const uint32_t pos = cur[d] + pre + rank;
      t_idx[pos] = el[it].idx;
      t_x[pos] = el[it].x;
      t_y[pos] = el[it].y;
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&cur[d], cnt);
      wcnt[wave][d] = 0;
    }
  }
  __syncthreads();
  const int64_t left = total - base;
  const int cnt_blk = left < kTile ? (int)left : kTile;
  const int64_t dleft = n - base;
  const int nd = dleft <= 0 ? 0 : (dleft < cnt_blk ? (int)dleft : cnt_blk);  // data points of this tile
  for (int i = tid; i < cnt_blk; i += kThreads) {
    const float px = t_x[i], py = t_y[i];
    const uint32_t d = (cell_of(px, py, g) >> g.band_shift) + (i >= nd ? nb : 0u);
    const uint32_t gp = gstart[d] + ((uint32_t)i - loff[d]);
    oidx[gp] = t_idx[i];
    ox[gp] = px;
    oy[gp] = py;
  }
}

// One block per digit: the stable counting sort of the digit's segment by cell inside its
// band.  The cells' counts (LDS atomics) and their exclusive scan give the CSR offsets, which
// data blocks write (head of cell c = cell_start[c], size = cell_start[c + 1] - cell_start[c],
// Section 3.2.3).  Two ways to order the points inside each cell by index:
//   rank path    (the segment fits the LDS tile and no cell of the band holds more than
//                kRankMaxCell points): every point takes a slot of its cell by an LDS atomic,
//                then its place in the cell is the number of the cell's points with a smaller
//                index; the sorted tile is written out in one coalesced pass.
//   ballot path  (otherwise): the segment, which the stable scatter left in index order, is
//                ranked in rounds of kLocalThreads points by wavefront ballots on the local
//                cell key, earlier rounds counted by a running cursor per cell; a segment that
//                fits the tile is sorted in LDS and written out, a longer one (a dense band) is
//                written directly.
// Query blocks write the queries in cell order (and their coordinates).  Dynamic LDS: cnt [CB]
// (counts, then offsets / cursors), then a region used either by the rank path (slot indices,
// sorted index, x, y [kLocalTile] each) or by the ballot path (wcnt [kLocalWaves][CB] bytes,
// then the staged index, x, y [kLocalTile] each); CB = the largest band the host sized for.
constexpr int kRankMaxCell = 64;
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
  extern __shared__ uint32_t lds[];
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
  uint32_t* region = lds + cb_max;
  // rank path
  uint32_t* r_slot = region;
  uint32_t* r_idx = region + kLocalTile;
  float* r_x = reinterpret_cast<float*>(region + 2 * kLocalTile);
  float* r_y = reinterpret_cast<float*>(region + 3 * kLocalTile);
  // ballot path
  uint8_t* wcnt = reinterpret_cast<uint8_t*>(region);  // [kLocalWaves][cb]
  uint32_t* t_idx = region + kLocalWaves * cb_max / 4;
  float* t_x = reinterpret_cast<float*>(t_idx + kLocalTile);
  float* t_y = t_x + kLocalTile;
  const uint32_t s = dstart[d], e = dstart[d + 1];
  const uint32_t size = e - s;
  const bool staged = size <= (uint32_t)kLocalTile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));

  for (int i = tid; i < cb; i += kLocalThreads) cnt[i] = 0u;
  if (tid == 0) s_max = 0u;
  // a staged segment stays in registers: (local cell, index, x, y) per item
  uint32_t lk[kLocalItems], id[kLocalItems];
  float px[kLocalItems], py[kLocalItems];
  if (staged) {
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it) {
      const uint32_t p = s + it * kLocalThreads + tid;
      lk[it] = 0xffffffffu;
      id[it] = 0u;
      px[it] = py[it] = 0.0f;
      if (p < e) {
        px[it] = bx[p];
        py[it] = by[p];
        id[it] = bidx[p];
        lk[it] = cell_of(px[it], py[it], g) - cell0;
      }
    }
  }
  __syncthreads();
  if (staged) {
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      if (lk[it] != 0xffffffffu) atomicAdd(&cnt[lk[it]], 1u);
  } else {
    for (uint32_t p = s + tid; p < e; p += kLocalThreads) atomicAdd(&cnt[cell_of(bx[p], by[p], g) - cell0], 1u);
  }
  __syncthreads();
  if (staged) {
    uint32_t mx = 0u;
    for (int i = tid; i < cb; i += kLocalThreads) mx = max(mx, cnt[i]);
    if (mx > 0u) atomicMax(&s_max, mx);
  }
  // exclusive scan of the band's counts; a data band writes its cells' offsets
  uint32_t carry = 0;
  for (int c0 = 0; c0 < cb; c0 += kLocalThreads * 4) {
    uint32_t v[4];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = c0 + tid * 4 + i;
      v[i] = j < cb ? cnt[j] : 0u;
      sum += v[i];
    }
    uint32_t tot;
    uint32_t run = carry + block_scan<kLocalThreads>(sum, &tot);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = c0 + tid * 4 + i;
      if (j < cb) {
        cnt[j] = run;
        if (!query && j < ncb) cell_start[cell0 + j] = (int32_t)(s + run);
      }
      run += v[i];
    }
    carry += tot;
  }
  if (!query && band == nb - 1 && tid == 0) cell_start[g.ncells] = (int32_t)e;
  __syncthreads();
  // writes the sorted point at segment position i (staged in LDS, or direct)
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
  if (staged && s_max <= (uint32_t)kRankMaxCell) {
    // rank path: a slot of the point's cell, then its place among the cell's points by index
    uint32_t slot[kLocalItems];
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      if (lk[it] != 0xffffffffu) {
        slot[it] = atomicAdd(&cnt[lk[it]], 1u);
        r_slot[slot[it]] = id[it];
      }
    __syncthreads();
    // cnt[c] is now the end of cell c, which is the start of cell c + 1
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      if (lk[it] != 0xffffffffu) {
        const uint32_t c = lk[it];
        const uint32_t c_end = cnt[c], c_begin = c == 0 ? 0u : cnt[c - 1];
        uint32_t pos = c_begin;
        for (uint32_t j = c_begin; j < c_end; ++j) pos += r_slot[j] < id[it] ? 1u : 0u;
        r_idx[pos] = id[it];
        r_x[pos] = px[it];
        r_y[pos] = py[it];
      }
    __syncthreads();
    for (uint32_t i = tid; i < size; i += kLocalThreads) emit(i, r_idx[i], r_x[i], r_y[i]);
    return;
  }
  // ballot path
  for (int i = tid; i < kLocalWaves * cb / 4; i += kLocalThreads) reinterpret_cast<uint32_t*>(wcnt)[i] = 0u;
  __syncthreads();
  // one ranking round: the point of this thread (valid, local cell key, index, x, y) goes to
  // position cur[key] + (earlier waves' and lanes' points of the same key) of the segment
  auto round = [&](bool valid, uint32_t key, uint32_t pid, float fx, float fy) {
    const uint64_t match = match_key(key, shift, __ballot(valid));
    const uint32_t rank = __popcll(match & lt_mask);
    const uint32_t c = __popcll(match);
    const bool leader = valid && rank == 0;
    if (leader) wcnt[wave * cb + key] = (uint8_t)c;
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int w = 0; w < wave; ++w) pre += wcnt[w * cb + key];
      const uint32_t pos = cnt[key] + pre + rank;
      if (staged) {
        t_idx[pos] = pid;
        t_x[pos] = fx;
        t_y[pos] = fy;
      } else {
        emit(pos, pid, fx, fy);
      }
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&cnt[key], c);
      wcnt[wave * cb + key] = 0;
    }
  };
  if (staged) {
#pragma unroll
    for (int it = 0; it < kLocalItems; ++it)
      round(lk[it] != 0xffffffffu, lk[it] == 0xffffffffu ? 0u : lk[it], id[it], px[it], py[it]);
    __syncthreads();
    for (uint32_t i = tid; i < size; i += kLocalThreads) emit(i, t_idx[i], t_x[i], t_y[i]);
  } else {
    for (uint32_t r0 = s; r0 < e; r0 += kLocalThreads) {
      const uint32_t p = r0 + tid;
      const bool valid = p < e;
      float fx = 0.0f, fy = 0.0f;
      uint32_t pid = 0, key = 0;
      if (valid) {
        fx = bx[p];
        fy = by[p];
        pid = bidx[p];
        key = cell_of(fx, fy, g) - cell0;
      }
      round(valid, key, pid, fx, fy);
    }
  }
}

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Dynamic LDS of k_band_local for bands of at most cb cells.
size_t local_lds_bytes(int cb) {
  const size_t rank = 4 * sizeof(uint32_t) * (size_t)kLocalTile;
  const size_t ballot = (size_t)kLocalWaves * cb + (sizeof(uint32_t) + 2 * sizeof(float)) * kLocalTile;
  return sizeof(uint32_t) * (size_t)cb + (rank > ballot ? rank : ballot);
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
