// Batched form: many independent AIDW problems ("jobs") of uneven size run as
// one pipeline on one stream.
//
// Every stage of the method is one launch over all jobs.  The jobs' inputs are
// first gathered into concatenated arrays (data padded per job for the pair
// loop's prefetch), so later kernels index one flat range and find their job
// by a binary search over the jobs' offsets:
//   gather -> bounds per job (Section 4.1.1) -> grid scalars per job (Eq. 2)
//   -> cell key per data point -> one stable radix sort of all jobs' points by
//   global cell (job j owns the cells [cbase_j, cbase_j + ccap_j)) -> one CSR
//   array for all grids -> query keys -> sort -> kNN and Eq. 3 (Section 3.2.4)
//   -> Eq. 4-6 and the pair-kernel class -> sort by (job, class)
//   -> ONE persistent pair launch (Eq. 1) -> fixed-order combine + fix-up.
// Sizes are fixed when the plan is made (host-known n, m per job), so running a
// plan allocates nothing and never waits for the device: a job's grid lives in
// a cell budget fixed from n, and the finalize kernel widens the cell side when
// the bounds would need more cells (the kNN result does not depend on the side).
//
// The persistent pair kernel.  The host lists work items (job, block of 256 * Q
// queries, range of data points) and orders them by decreasing cost (pairs),
// the longest-processing-time-first rule; the workgroups of one launch take
// items from that list through an atomic counter until it is exhausted, so
// jobs of very different size keep every compute unit busy to the end.  Each
// item writes its own float64 (num, den) partials; the finish kernel adds a
// query's partials in data-range order, so results do not depend on which
// workgroup ran which item.  Per item, the block of queries takes the integer
// power loop when all its queries share an integer alpha (as in the single-job
// path), else the general loop.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "aidw_internal.h"
#include "grid_core.h"
#include "knn_core.h"
#include "pair_core.h"

namespace aidw {
namespace {

struct BatchJob {
  const float* x;
  const float* y;
  const float* z;
  const float* qx;
  const float* qy;
  float* qz;
  float* alpha_out;
  float* r_obs_out;
  int32_t n, m, k;
  int32_t doff;    // first slot in the padded, concatenated data arrays
  int32_t noff;    // first slot in the unpadded data order (the grid sort's input)
  int32_t qoff;    // first query slot
  int32_t cbase;   // first global cell
  int32_t ccap;    // cell budget
  int32_t splits;  // data ranges per query block
  int32_t chunk;   // points per data range (a multiple of the pair loop's fetch)
  int64_t poff;    // first partial slot; the job has splits * m of them
  uint32_t intmask;  // bit p: the job has the integer level p, whose blocks may take the w = rsq(t)^p loop
  double area_in, cw_in, occ;
  double r_min, r_max, levels[5];
};

struct WorkItem {
  int32_t job, qblock, split, pad;
};

constexpr int kBoundsPerBlock = 4096;  // elements of one job per bounds workgroup

// Largest j in [0, nseg) with off[j] <= e (off ascending; empty segments repeat
// an offset, and the last of equal offsets is the segment that holds e).
__device__ inline int find_seg(const int32_t* __restrict__ off, int nseg, int e) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Data into zero-padded concatenated arrays, queries into concatenated arrays.
__global__ __launch_bounds__(256) void k_b_gather(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ doff,
                                                  const int32_t* __restrict__ qoff, int njobs, int sum_npad,
                                                  int sum_m, float* __restrict__ xp, float* __restrict__ yp,
                                                  float* __restrict__ zp, float* __restrict__ cqx,
                                                  float* __restrict__ cqy) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < sum_npad) {
    const int j = find_seg(doff, njobs, e);
    const BatchJob& J = jobs[j];
    const int i = e - J.doff;
    const bool in = i < J.n;
    xp[e] = in ? J.x[i] : 0.0f;
    yp[e] = in ? J.y[i] : 0.0f;
    zp[e] = in ? J.z[i] : 0.0f;
  } else if (e - sum_npad < sum_m) {
    const int q = e - sum_npad;
    const int j = find_seg(qoff, njobs, q);
    const BatchJob& J = jobs[j];
    cqx[q] = J.qx[q - J.qoff];
    cqy[q] = J.qy[q - J.qoff];
  }
}

// Bounds partial of one workgroup: elements [lb * kBoundsPerBlock, ...) of its
// job's data points followed by its queries (Section 4.1.1: the grid encloses both).
__global__ __launch_bounds__(256) void k_b_bounds(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ bstart,
                                                  int njobs, const float* __restrict__ xp,
                                                  const float* __restrict__ yp, const float* __restrict__ cqx,
                                                  const float* __restrict__ cqy, BoundsPartial* __restrict__ partial) {
  const int b = blockIdx.x;
  const int j = find_seg(bstart, njobs, b);
  const BatchJob& J = jobs[j];
  const int total = J.n + J.m;
  const int e0 = (b - bstart[j]) * kBoundsPerBlock;
  const int e1 = min(total, e0 + kBoundsPerBlock);
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  int bad = 0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
    float a, c;
    if (e < J.n) {
      a = xp[J.doff + e];
      c = yp[J.doff + e];
    } else {
      a = cqx[J.qoff + e - J.n];
      c = cqy[J.qoff + e - J.n];
    }
    bad |= !(isfinite(a) && isfinite(c));
    mnx = fminf(mnx, a);
    mxx = fmaxf(mxx, a);
    mny = fminf(mny, c);
    mxy = fmaxf(mxy, c);
  }
  mnx = gridc::wave_min(mnx);
  mny = gridc::wave_min(mny);
  mxx = gridc::wave_max(mxx);
  mxy = gridc::wave_max(mxy);
  bad = gridc::wave_or(bad);
  __shared__ BoundsPartial s[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s[wave] = BoundsPartial{mnx, mny, mxx, mxy, bad, {0, 0, 0}};
  __syncthreads();
  if (threadIdx.x == 0) {
    BoundsPartial r = s[0];
    for (int w = 1; w < 4; ++w) {
      r.minx = fminf(r.minx, s[w].minx);
      r.miny = fminf(r.miny, s[w].miny);
      r.maxx = fmaxf(r.maxx, s[w].maxx);
      r.maxy = fmaxf(r.maxy, s[w].maxy);
      r.nonfinite |= s[w].nonfinite;
    }
    partial[b] = r;
  }
}

// Grid scalars of job blockIdx.x within its cell budget.
__global__ __launch_bounds__(256) void k_b_finalize(const BatchJob* __restrict__ jobs,
                                                    const int32_t* __restrict__ bstart,
                                                    const BoundsPartial* __restrict__ partial,
                                                    GridScalars* __restrict__ gs) {
  const int j = blockIdx.x;
  const BoundsPartial r = gridc::block_reduce_bounds(partial, bstart[j], bstart[j + 1]);
  if (threadIdx.x != 0) return;
  const BatchJob& J = jobs[j];
  gs[j] = gridc::grid_scalars(r.minx, r.miny, r.maxx, r.maxy, r.nonfinite != 0, J.n, J.area_in, J.cw_in, J.occ,
                              J.ccap);
}

__device__ inline uint32_t global_cell(const GridScalars& g, int cbase, float x, float y) {
  const int col = knn::clamp_cell((x - g.minx) * g.inv_cw, g.ncol);
  const int row = knn::clamp_cell((y - g.miny) * g.inv_cw, g.nrow);
  return (uint32_t)(cbase + row * g.ncol + col);
}

// Section 4.1.2 for every job's points: key = the job's first cell + row * nCol + col,
// value = the point's padded slot (which orders a job's points by index).
__global__ __launch_bounds__(256) void k_b_cell_keys(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ noff,
                                                     int njobs, int sum_n, const GridScalars* __restrict__ gs,
                                                     const float* __restrict__ xp, const float* __restrict__ yp,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= sum_n) return;
  const int j = find_seg(noff, njobs, e);
  const BatchJob& J = jobs[j];
  const int p = J.doff + (e - J.noff);
  keys[e] = global_cell(gs[j], J.cbase, xp[p], yp[p]);
  vals[e] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_b_query_keys(const BatchJob* __restrict__ jobs,
                                                      const int32_t* __restrict__ qoff, int njobs, int sum_m,
                                                      const GridScalars* __restrict__ gs,
                                                      const float* __restrict__ cqx, const float* __restrict__ cqy,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= sum_m) return;
  const int j = find_seg(qoff, njobs, q);
  keys[q] = global_cell(gs[j], jobs[j].cbase, cqx[q], cqy[q]);
  vals[q] = (uint32_t)q;
}

// kNN + Eq. 3 for the queries at binned positions [t_begin, t_end); each lane searches its
// own job's grid.  The jobs are ordered by the length of their register k-list, so each
// length class is one range of positions and one launch.
template <int KMAX>
__global__ __launch_bounds__(256) void k_b_knn(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ qoff,
                                               int njobs, int t_begin, int t_end, const GridScalars* __restrict__ gs,
                                               const int32_t* __restrict__ cell_start, const float* __restrict__ sx,
                                               const float* __restrict__ sy, const int32_t* __restrict__ sidx,
                                               const float* __restrict__ cqx, const float* __restrict__ cqy,
                                               const uint32_t* __restrict__ qperm, float* __restrict__ r_obs,
                                               float* __restrict__ d1sq) {
  const int t = t_begin + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= t_end) return;
  const int q = (int)qperm[t];
  const int j = find_seg(qoff, njobs, q);
  const GridScalars& G = gs[j];
  if (G.status != AIDW_OK) {
    r_obs[q] = NAN;
    d1sq[q] = 1.0f;
    return;
  }
  const BatchJob& J = jobs[j];
  const knn::View g{G.minx, G.miny, G.inv_cw, G.ncol, G.nrow, G.cwd};
  double bk[KMAX];
  int32_t bi[KMAX];
  knn::search<KMAX>(g, cell_start + J.cbase, sx, sy, sidx, cqx[q], cqy[q], J.k, slack_cells(G.ncol, G.nrow), bk,
                    bi);
  float ro, d1;
  knn::summarise<KMAX>(bk, J.k, ro, d1);
  r_obs[q] = ro;
  d1sq[q] = d1;
}

// Eq. 4-6 per query with its job's parameters; key = job * 16 + pair-kernel class.
__global__ __launch_bounds__(256) void k_b_alpha(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ qoff,
                                                 int njobs, int sum_m, const GridScalars* __restrict__ gs,
                                                 const float* __restrict__ r_obs, int integer_powers,
                                                 float* __restrict__ alpha_f, uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= sum_m) return;
  const int j = find_seg(qoff, njobs, q);
  const GridScalars& G = gs[j];
  uint32_t cls = 0;
  if (G.status != AIDW_OK) {
    alpha_f[q] = NAN;
  } else {
    const BatchJob& J = jobs[j];
    const double R = (double)r_obs[q] / G.r_exp;                                                // Eq. 4
    const double alpha = pair::level_alpha(pair::fuzzy_mu(R, J.r_min, J.r_max), J.levels);  // Eq. 5, 6
    alpha_f[q] = (float)alpha;
    if (integer_powers) cls = pair::alpha_class(alpha);
  }
  if (keys) {
    keys[q] = ((uint32_t)j << 4) | cls;
    vals[q] = (uint32_t)q;
  }
}

__global__ void k_b_reset(uint32_t* __restrict__ counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// One work item for a block of queries: positions [pos0, posend) of the pair order.
template <int Q, int POW>
__device__ __forceinline__ void b_item(int pos0, int posend, const uint32_t* __restrict__ perm,
                                       const float* __restrict__ cqx, const float* __restrict__ cqy,
                                       const float* __restrict__ alpha_f, const float* __restrict__ d1sq,
                                       const float* __restrict__ xb, const float* __restrict__ yb,
                                       const float* __restrict__ zb, int lo, int hi, double2* __restrict__ partial,
                                       int64_t pbase) {
  pair::Lane<Q, POW> L;
  int qid[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int pos = pos0 + j * pair::kThreads + (int)threadIdx.x;
    qid[j] = -1;
    if (pos < posend) {
      const int q = perm ? (int)perm[pos] : pos;
      qid[j] = q;
      L.set(j, cqx[q], cqy[q], alpha_f[q], d1sq[q]);
    } else {
      L.clear(j);
    }
  }
  pair::pair_range<Q, POW>(L, xb, yb, zb, lo, hi);
#pragma unroll
  for (int j = 0; j < Q; ++j)
    if (qid[j] >= 0) partial[pbase + qid[j]] = make_double2(L.num(j), L.den(j));
}

// Persistent pair kernel (Eq. 1): workgroups take work items in list order
// (decreasing cost) until the list is exhausted; every workgroup reaches the
// exit test on every round.
template <int Q>
__global__ __launch_bounds__(pair::kThreads) void k_b_interp(
    const BatchJob* __restrict__ jobs, const WorkItem* __restrict__ items, int nitems,
    uint32_t* __restrict__ counter, const GridScalars* __restrict__ gs, const float* __restrict__ xp,
    const float* __restrict__ yp, const float* __restrict__ zp, const float* __restrict__ cqx,
    const float* __restrict__ cqy, const float* __restrict__ alpha_f, const float* __restrict__ d1sq,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ skeys, uint32_t fast_mask,
    double2* __restrict__ partial) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // every thread has read s_item before it is overwritten
    if (it >= nitems) break;
    const WorkItem w = items[it];
    const int j = w.job;
    if (gs[j].status != AIDW_OK) continue;
    const BatchJob& J = jobs[j];
    const int pos0 = J.qoff + w.qblock * pair::kThreads * Q;
    const int posend = min(J.qoff + J.m, pos0 + pair::kThreads * Q);
    const int lo = w.split * J.chunk;
    const int hi = min(J.n, lo + J.chunk);
    uint32_t cls = 0;
    if (fast_mask) {
      const uint32_t k0 = skeys[pos0] & 15u, kl = skeys[posend - 1] & 15u;
      if (k0 == kl && ((J.intmask >> k0) & 1u)) cls = k0;
    }
    const float* xb = xp + J.doff;
    const float* yb = yp + J.doff;
    const float* zb = zp + J.doff;
    const int64_t pbase = J.poff + (int64_t)w.split * J.m - J.qoff;
    switch (cls) {
#define AIDW_B_CASE(P) \
  case P: b_item<Q, P>(pos0, posend, perm, cqx, cqy, alpha_f, d1sq, xb, yb, zb, lo, hi, partial, pbase); break;
      AIDW_B_CASE(1)
      AIDW_B_CASE(2)
      AIDW_B_CASE(3)
      AIDW_B_CASE(4)
      AIDW_B_CASE(5)
      AIDW_B_CASE(6)
      AIDW_B_CASE(7)
      AIDW_B_CASE(8)
#undef AIDW_B_CASE
      default:
        b_item<Q, 0>(pos0, posend, perm, cqx, cqy, alpha_f, d1sq, xb, yb, zb, lo, hi, partial, pbase);
    }
  }
}

// Per query: the job's partials added in data-range order, num / den in float64,
// the coincident-query fix-up, and the outputs written to the caller's arrays.
// A job whose grid failed (non-finite or degenerate input) gets NaN everywhere.
__global__ __launch_bounds__(256) void k_b_finish(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ qoff,
                                                  int njobs, int sum_m, const GridScalars* __restrict__ gs,
                                                  const double2* __restrict__ partial,
                                                  const int32_t* __restrict__ cell_start,
                                                  const float* __restrict__ sx, const float* __restrict__ sy,
                                                  const int32_t* __restrict__ sidx, const float* __restrict__ zp,
                                                  const float* __restrict__ cqx, const float* __restrict__ cqy,
                                                  const float* __restrict__ r_obs, const float* __restrict__ alpha_f,
                                                  const float* __restrict__ d1sq) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= sum_m) return;
  const int j = find_seg(qoff, njobs, q);
  const BatchJob& J = jobs[j];
  const GridScalars& G = gs[j];
  const int i = q - J.qoff;
  float v = NAN, a = NAN, ro = NAN;
  if (G.status == AIDW_OK) {
    double num = 0.0, den = 0.0;
    for (int s = 0; s < J.splits; ++s) {
      const double2 p = partial[J.poff + (int64_t)s * J.m + i];
      num += p.x;
      den += p.y;
    }
    v = (float)(num / den);
    if (d1sq[q] == 0.0f) {
      const knn::View g{G.minx, G.miny, G.inv_cw, G.ncol, G.nrow, G.cwd};
      float c;
      if (knn::coincident_mean(g, cell_start + J.cbase, sx, sy, sidx, zp, cqx[q], cqy[q], c)) v = c;
    }
    a = alpha_f[q];
    ro = r_obs[q];
  }
  J.qz[i] = v;
  if (J.alpha_out) J.alpha_out[i] = a;
  if (J.r_obs_out) J.r_obs_out[i] = ro;
}

int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace
}  // namespace aidw

using namespace aidw;

struct aidw_batch {
  int njobs = 0;
  std::vector<int32_t> caller;  // internal job -> the caller's job index
  struct KnnRange {
    int kmax, t_begin, t_end;
  };
  std::vector<KnnRange> knn_ranges;
  aidw_batch_config cfg{};
  int kmax = 16;
  uint32_t fast_mask = 0;
  int sum_n = 0, sum_npad = 0, sum_m = 0, sum_cap = 0, nbblocks = 0, nitems = 0, workers = 0;
  int64_t sum_partial = 0;
  double sum_pairs = 0.0;
  int cell_bits = 0, class_bits = 0;
  void* mem = nullptr;
  size_t mem_bytes = 0;
  // device arrays carved from mem
  BatchJob* jobs = nullptr;
  int32_t *doff = nullptr, *noff = nullptr, *qoff = nullptr, *bstart = nullptr;
  WorkItem* items = nullptr;
  GridScalars* gs = nullptr;
  BoundsPartial* bpart = nullptr;
  float *xp = nullptr, *yp = nullptr, *zp = nullptr, *cqx = nullptr, *cqy = nullptr;
  uint32_t *keys = nullptr, *vals = nullptr, *tkeys = nullptr, *tvals = nullptr, *hist = nullptr, *scan_tmp = nullptr;
  int32_t* cell_start = nullptr;
  float *sx = nullptr, *sy = nullptr;
  int32_t* sidx = nullptr;
  uint32_t *qkeys = nullptr, *qperm = nullptr, *ckeys = nullptr, *cperm = nullptr;
  float *r_obs = nullptr, *d1sq = nullptr, *alpha_f = nullptr;
  double2* partial = nullptr;
  uint32_t* counter = nullptr;
  // graph replay
  hipGraphExec_t exec = nullptr;
  // timing
  bool timing = false, timed = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

aidw_status check_config(const aidw_batch_config* c) {
  if (c->q != 1 && c->q != 2) return fail(AIDW_EINVAL, "config.q must be 1 or 2 (got %d)", c->q);
  if (c->split_points < 0) return fail(AIDW_EINVAL, "config.split_points must be >= 0");
  if (c->workers_per_cu < 1 || c->workers_per_cu > 32)
    return fail(AIDW_EINVAL, "config.workers_per_cu must be in [1, 32] (got %d)", c->workers_per_cu);
  if (c->integer_powers != 0 && c->integer_powers != 1) return fail(AIDW_EINVAL, "config.integer_powers must be 0 or 1");
  if (c->use_graph != 0 && c->use_graph != 1) return fail(AIDW_EINVAL, "config.use_graph must be 0 or 1");
  return AIDW_OK;
}

// Cell budget of a job: twice the cells the default side would give on a square
// box, plus the rim of a box of any aspect ratio up to about 4:1.
int64_t cell_budget(int64_t n, const aidw_params& p) {
  const double occ = (p.cell_width > 0 || !(p.occupancy > 0)) ? 2.0 : p.occupancy;
  const double base = (double)n / occ;
  return (int64_t)(2.0 * ceil(base) + 4.0 * ceil(sqrt(base)) + 16.0);
}

// Next 256-byte aligned piece of count elements at byte offset off of base
// (base == nullptr: only advances off, to size the workspace).
template <typename T>
T* carve(char* base, size_t& off, size_t count) {
  T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
  off += (count * sizeof(T) + 255) / 256 * 256;
  return p;
}

void destroy_plan(aidw_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
}

aidw_status create_plan(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* cfg_in, aidw_batch** out) {
  if (!out) return fail(AIDW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!jobs || njobs < 1) return fail(AIDW_EINVAL, "need at least one job");
  if (njobs > (1 << 27)) return fail(AIDW_ECAPACITY, "too many jobs (%d)", njobs);
  aidw_batch_config cfg;
  if (cfg_in)
    cfg = *cfg_in;
  else
    aidw_batch_config_default(&cfg);
  aidw_status st = check_config(&cfg);
  if (st != AIDW_OK) return st;

  // ---- host checks and the job table ----
  std::vector<BatchJob> hj(njobs);
  std::vector<int32_t> doff(njobs + 1), noff(njobs + 1), qoff(njobs + 1), bstart(njobs + 1);
  int64_t sn = 0, snp = 0, sm = 0, scap = 0, sb = 0, spart = 0;
  int kmax = 1;
  uint32_t mask = 0;  // union of the jobs' integer levels
  double pairs = 0.0;
  const int qb = pair::kThreads * cfg.q;
  auto kclass = [](int k) { return knn_slots(k); };
  for (int j = 0; j < njobs; ++j) {
    const aidw_job& a = jobs[j];
    if (a.n < 1) return fail(AIDW_EINVAL, "job %d: n must be >= 1", j);
    if (a.m < 0) return fail(AIDW_EINVAL, "job %d: m must be >= 0", j);
    if (a.n > INT32_MAX / 2 || a.m > INT32_MAX / 2) return fail(AIDW_ECAPACITY, "job %d: size exceeds int32", j);
    if (!a.x || !a.y || !a.z) return fail(AIDW_EINVAL, "job %d: x, y, z must be non-NULL", j);
    if (a.m > 0 && (!a.qx || !a.qy || !a.qz)) return fail(AIDW_EINVAL, "job %d: qx, qy, qz must be non-NULL", j);
    if ((st = check_params(&a.params)) != AIDW_OK) return fail(st, "job %d: %s", j, aidw_last_error_detail());
    const int k = a.params.k;
    if (k < 1 || k > AIDW_KMAX || k > a.n)
      return fail(AIDW_EINVAL, "job %d: k = %d must be in [1, min(n, %d)]", j, k, AIDW_KMAX);
  }
  // internal order: by k-list class (stable), so that each class is one range of queries
  std::vector<int32_t> order(njobs);
  for (int j = 0; j < njobs; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return kclass(jobs[a].params.k) < kclass(jobs[b].params.k); });
  for (int jj = 0; jj < njobs; ++jj) {
    const int j = jj;  // internal index
    const aidw_job& a = jobs[order[jj]];
    const int k = a.params.k;
    kmax = std::max(kmax, k);
    uint32_t jm = 0;
    for (int l = 0; l < 5; ++l) {
      const double v = a.params.alpha[l];
      if (v >= 1.0 && v <= (double)pair::kMaxIntPow && v == floor(v)) jm |= 1u << (int)v;
    }
    if (!cfg.integer_powers) jm = 0;
    mask |= jm;
    BatchJob& J = hj[j];
    J.intmask = jm;
    J.x = a.x;
    J.y = a.y;
    J.z = a.z;
    J.qx = a.qx;
    J.qy = a.qy;
    J.qz = a.qz;
    J.alpha_out = a.alpha_out;
    J.r_obs_out = a.r_obs_out;
    J.n = (int32_t)a.n;
    J.m = (int32_t)a.m;
    J.k = k;
    J.doff = (int32_t)snp;
    J.noff = (int32_t)sn;
    J.qoff = (int32_t)sm;
    J.cbase = (int32_t)scap;
    const int64_t cap = cell_budget(a.n, a.params);
    J.ccap = (int32_t)std::min<int64_t>(cap, AIDW_MAX_CELLS);
    int64_t chunk = cfg.split_points > 0 ? std::min<int64_t>(cfg.split_points, a.n) : a.n;
    chunk = (chunk + pair::kChunk - 1) / pair::kChunk * pair::kChunk;
    J.chunk = (int32_t)chunk;
    J.splits = (int32_t)((a.n + chunk - 1) / chunk);
    J.poff = spart;
    J.area_in = a.params.area;
    J.cw_in = a.params.cell_width;
    J.occ = a.params.occupancy;
    J.r_min = a.params.r_min;
    J.r_max = a.params.r_max;
    for (int l = 0; l < 5; ++l) J.levels[l] = a.params.alpha[l];
    doff[j] = (int32_t)snp;
    noff[j] = (int32_t)sn;
    qoff[j] = (int32_t)sm;
    bstart[j] = (int32_t)sb;
    sn += a.n;
    snp += pair::padded_len((int)a.n);
    sm += a.m;
    scap += J.ccap;
    sb += (a.n + a.m + kBoundsPerBlock - 1) / kBoundsPerBlock;
    spart += (int64_t)J.splits * a.m;
    pairs += (double)a.n * (double)a.m;
    if (snp >= INT32_MAX / 2 || sm >= INT32_MAX / 2 || scap >= INT32_MAX / 2 || sb >= INT32_MAX / 2)
      return fail(AIDW_ECAPACITY, "batch totals exceed int32 (at job %d)", order[jj]);
  }
  doff[njobs] = (int32_t)snp;
  noff[njobs] = (int32_t)sn;
  qoff[njobs] = (int32_t)sm;
  bstart[njobs] = (int32_t)sb;

  // ---- work items, longest first ----
  std::vector<WorkItem> items;
  std::vector<int64_t> cost;
  for (int j = 0; j < njobs; ++j) {
    const BatchJob& J = hj[j];
    const int nqb = (J.m + qb - 1) / qb;
    for (int b = 0; b < nqb; ++b) {
      const int64_t nq = std::min(qb, J.m - b * qb);
      for (int s = 0; s < J.splits; ++s) {
        const int64_t np = std::min(J.chunk, J.n - s * J.chunk);
        items.push_back(WorkItem{j, b, s, 0});
        cost.push_back(nq * np);
      }
    }
  }
  if (items.size() >= (size_t)INT32_MAX) return fail(AIDW_ECAPACITY, "too many work items");
  std::vector<int32_t> by_cost(items.size());
  for (size_t i = 0; i < by_cost.size(); ++i) by_cost[i] = (int32_t)i;
  std::stable_sort(by_cost.begin(), by_cost.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  std::vector<WorkItem> sorted(items.size());
  for (size_t i = 0; i < by_cost.size(); ++i) sorted[i] = items[by_cost[i]];

  aidw_batch* b = new aidw_batch();
  b->njobs = njobs;
  b->cfg = cfg;
  b->kmax = kclass(kmax);
  b->caller = order;
  for (int jj = 0; jj < njobs;) {  // one kNN launch per k-list class: a contiguous range of jobs
    int je = jj;
    while (je < njobs && hj[je].k <= b->kmax && kclass(hj[je].k) == kclass(hj[jj].k)) ++je;
    if (qoff[je] > qoff[jj]) b->knn_ranges.push_back({kclass(hj[jj].k), qoff[jj], qoff[je]});
    jj = je;
  }
  b->fast_mask = mask;
  b->sum_n = (int)sn;
  b->sum_npad = (int)snp;
  b->sum_m = (int)sm;
  b->sum_cap = (int)scap;
  b->nbblocks = (int)sb;
  b->nitems = (int)sorted.size();
  b->sum_partial = spart;
  b->sum_pairs = pairs;
  b->cell_bits = bits_for(scap);
  b->class_bits = bits_for(njobs) + 4;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    destroy_plan(b);
    return hip_fail(e, "querying the device");
  }
  b->workers = (int)std::min<int64_t>((int64_t)cfg.workers_per_cu * std::max(cus, 1), std::max(b->nitems, 1));

  // ---- one device allocation for everything ----
  const size_t nmax = (size_t)std::max<int64_t>(std::max<int64_t>(sn, sm), 1);
  const size_t hist_words = radix_hist_words((int)nmax), scan_words = radix_scan_tmp_words((int)nmax);
  auto layout = [&](char* base) {
    size_t off = 0;
    b->jobs = carve<BatchJob>(base, off, njobs);
    b->doff = carve<int32_t>(base, off, njobs + 1);
    b->noff = carve<int32_t>(base, off, njobs + 1);
    b->qoff = carve<int32_t>(base, off, njobs + 1);
    b->bstart = carve<int32_t>(base, off, njobs + 1);
    b->items = carve<WorkItem>(base, off, std::max<size_t>(sorted.size(), 1));
    b->gs = carve<GridScalars>(base, off, njobs);
    b->bpart = carve<BoundsPartial>(base, off, std::max<int64_t>(sb, 1));
    b->xp = carve<float>(base, off, snp);
    b->yp = carve<float>(base, off, snp);
    b->zp = carve<float>(base, off, snp);
    b->cqx = carve<float>(base, off, std::max<int64_t>(sm, 1));
    b->cqy = carve<float>(base, off, std::max<int64_t>(sm, 1));
    b->keys = carve<uint32_t>(base, off, std::max<int64_t>(sn, 1));
    b->vals = carve<uint32_t>(base, off, std::max<int64_t>(sn, 1));
    b->tkeys = carve<uint32_t>(base, off, nmax);
    b->tvals = carve<uint32_t>(base, off, nmax);
    b->hist = carve<uint32_t>(base, off, hist_words);
    b->scan_tmp = carve<uint32_t>(base, off, scan_words);
    b->cell_start = carve<int32_t>(base, off, scap + 1);
    b->sx = carve<float>(base, off, sn);
    b->sy = carve<float>(base, off, sn);
    b->sidx = carve<int32_t>(base, off, sn);
    b->qkeys = carve<uint32_t>(base, off, std::max<int64_t>(sm, 1));
    b->qperm = carve<uint32_t>(base, off, std::max<int64_t>(sm, 1));
    b->ckeys = carve<uint32_t>(base, off, std::max<int64_t>(sm, 1));
    b->cperm = carve<uint32_t>(base, off, std::max<int64_t>(sm, 1));
    b->r_obs = carve<float>(base, off, std::max<int64_t>(sm, 1));
    b->d1sq = carve<float>(base, off, std::max<int64_t>(sm, 1));
    b->alpha_f = carve<float>(base, off, std::max<int64_t>(sm, 1));
    b->partial = carve<double2>(base, off, std::max<int64_t>(spart, 1));
    b->counter = carve<uint32_t>(base, off, 1);
    return off;
  };
  b->mem_bytes = layout(nullptr);
  if ((e = dmalloc(&b->mem, b->mem_bytes)) != hipSuccess) {
    destroy_plan(b);
    return hip_fail(e, "allocating the batch workspace");
  }
  layout(static_cast<char*>(b->mem));
  struct Up {
    void* dst;
    const void* src;
    size_t bytes;
  } ups[] = {{b->jobs, hj.data(), sizeof(BatchJob) * njobs},
             {b->doff, doff.data(), sizeof(int32_t) * (njobs + 1)},
             {b->noff, noff.data(), sizeof(int32_t) * (njobs + 1)},
             {b->qoff, qoff.data(), sizeof(int32_t) * (njobs + 1)},
             {b->bstart, bstart.data(), sizeof(int32_t) * (njobs + 1)},
             {b->items, sorted.data(), sizeof(WorkItem) * sorted.size()}};
  for (const Up& u : ups) {
    if (u.bytes == 0) continue;
    if ((e = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice)) != hipSuccess) {
      destroy_plan(b);
      return hip_fail(e, "uploading the job table");
    }
  }
  *out = b;
  return AIDW_OK;
}

#define STEP(expr, what)                                  \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ == hipSuccess) e_ = hipGetLastError();         \
    if (e_ != hipSuccess) return hip_fail(e_, what);      \
  } while (0)

template <int KMAX>
void launch_b_knn(const aidw_batch* b, int t_begin, int t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_b_knn<KMAX>, dim3(div_up(t_end - t_begin, 256)), dim3(256), 0, s, b->jobs, b->qoff, b->njobs,
                     t_begin, t_end, b->gs, b->cell_start, b->sx, b->sy, b->sidx, b->cqx, b->cqy, b->qperm, b->r_obs,
                     b->d1sq);
}

template <int Q>
void launch_b_interp(const aidw_batch* b, hipStream_t s) {
  const uint32_t* perm = b->fast_mask ? b->cperm : nullptr;
  hipLaunchKernelGGL(k_b_interp<Q>, dim3(b->workers), dim3(pair::kThreads), 0, s, b->jobs, b->items, b->nitems,
                     b->counter, b->gs, b->xp, b->yp, b->zp, b->cqx, b->cqy, b->alpha_f, b->d1sq, perm, b->ckeys,
                     b->fast_mask, b->partial);
}

// Queues the whole pipeline on s: no allocation, no host synchronisation.
aidw_status enqueue(aidw_batch* b, hipStream_t s, bool timed) {
  const int nj = b->njobs;
  if (timed) STEP(hipEventRecord(b->ev[0], s), "recording an event");
  // stage 1: gather, bounds, grid scalars, counting sort, CSR
  hipLaunchKernelGGL(k_b_gather, dim3(div_up((int64_t)b->sum_npad + b->sum_m, 256)), dim3(256), 0, s, b->jobs,
                     b->doff, b->qoff, nj, b->sum_npad, b->sum_m, b->xp, b->yp, b->zp, b->cqx, b->cqy);
  STEP(hipSuccess, "gathering the jobs");
  hipLaunchKernelGGL(k_b_bounds, dim3(b->nbblocks), dim3(256), 0, s, b->jobs, b->bstart, nj, b->xp, b->yp, b->cqx,
                     b->cqy, b->bpart);
  hipLaunchKernelGGL(k_b_finalize, dim3(nj), dim3(256), 0, s, b->jobs, b->bstart, b->bpart, b->gs);
  STEP(hipSuccess, "grid scalars");
  hipLaunchKernelGGL(k_b_cell_keys, dim3(div_up(b->sum_n, 256)), dim3(256), 0, s, b->jobs, b->noff, nj, b->sum_n,
                     b->gs, b->xp, b->yp, b->keys, b->vals);
  STEP(radix_sort_pairs(b->keys, b->vals, b->tkeys, b->tvals, b->sum_n, b->cell_bits, b->hist, b->scan_tmp, s),
       "sorting the data by cell");
  STEP(launch_cell_start_gather(b->keys, b->vals, b->sum_n, b->sum_cap, b->xp, b->yp, b->cell_start, b->sx, b->sy,
                                b->sidx, s),
       "cell offsets");
  if (timed) STEP(hipEventRecord(b->ev[1], s), "recording an event");
  if (b->sum_m > 0) {
    // stage 1: query binning, kNN + Eq. 3; stage 2 prologue: Eq. 4-6 and the class order
    const int gm = div_up(b->sum_m, 256);
    hipLaunchKernelGGL(k_b_query_keys, dim3(gm), dim3(256), 0, s, b->jobs, b->qoff, nj, b->sum_m, b->gs, b->cqx,
                       b->cqy, b->qkeys, b->qperm);
    STEP(radix_sort_pairs(b->qkeys, b->qperm, b->tkeys, b->tvals, b->sum_m, b->cell_bits, b->hist, b->scan_tmp, s),
         "binning the queries");
    for (const auto& r : b->knn_ranges) {
#define AIDW_B_KNN(K) launch_b_knn<K>(b, r.t_begin, r.t_end, s)
      AIDW_FOR_KNN_SLOTS(r.kmax, AIDW_B_KNN)
#undef AIDW_B_KNN
    }
    STEP(hipSuccess, "kNN search");
    const bool classes = b->fast_mask != 0;
    hipLaunchKernelGGL(k_b_alpha, dim3(gm), dim3(256), 0, s, b->jobs, b->qoff, nj, b->sum_m, b->gs, b->r_obs,
                       (int)classes, b->alpha_f, classes ? b->ckeys : nullptr, classes ? b->cperm : nullptr);
    STEP(hipSuccess, "adaptive power");
    if (classes)
      STEP(radix_sort_pairs(b->ckeys, b->cperm, b->tkeys, b->tvals, b->sum_m, b->class_bits, b->hist, b->scan_tmp,
                            s),
           "ordering the queries by class");
    if (timed) STEP(hipEventRecord(b->ev[2], s), "recording an event");
    // stage 2: the persistent pair kernel
    hipLaunchKernelGGL(k_b_reset, dim3(1), dim3(64), 0, s, b->counter);
    if (b->cfg.q == 1)
      launch_b_interp<1>(b, s);
    else
      launch_b_interp<2>(b, s);
    STEP(hipSuccess, "pair kernel");
    if (timed) STEP(hipEventRecord(b->ev[3], s), "recording an event");
    hipLaunchKernelGGL(k_b_finish, dim3(gm), dim3(256), 0, s, b->jobs, b->qoff, nj, b->sum_m, b->gs, b->partial,
                       b->cell_start, b->sx, b->sy, b->sidx, b->zp, b->cqx, b->cqy, b->r_obs, b->alpha_f, b->d1sq);
    STEP(hipSuccess, "combine");
  } else if (timed) {
    STEP(hipEventRecord(b->ev[2], s), "recording an event");
    STEP(hipEventRecord(b->ev[3], s), "recording an event");
  }
  if (timed) STEP(hipEventRecord(b->ev[4], s), "recording an event");
  return AIDW_OK;
}

aidw_status run_plan(aidw_batch* b, hipStream_t s) {
  if (b->timing) {
    for (auto& ev : b->ev)
      if (!ev) HIP_TRY(hipEventCreate(&ev), "creating events");
    aidw_status st = enqueue(b, s, true);
    b->timed = st == AIDW_OK;
    return st;
  }
  b->timed = false;
  if (!b->cfg.use_graph) return enqueue(b, s, false);
  if (!b->exec) {
    if (s == nullptr) return fail(AIDW_EINVAL, "graph mode needs a created stream (the null stream cannot be captured)");
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "beginning the graph capture");
    aidw_status st = enqueue(b, s, false);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != AIDW_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "ending the graph capture");
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return hip_fail(e, "instantiating the graph");
    }
  }
  HIP_TRY(hipGraphLaunch(b->exec, s), "launching the graph");
  return AIDW_OK;
}

aidw_status job_status(aidw_batch* b, int32_t* status, hipStream_t s) {
  std::vector<GridScalars> h(b->njobs);
  HIP_TRY(hipMemcpyAsync(h.data(), b->gs, sizeof(GridScalars) * b->njobs, hipMemcpyDeviceToHost, s),
          "reading job status");
  HIP_TRY(hipStreamSynchronize(s), "synchronising");
  std::vector<int32_t> by_caller(b->njobs);
  for (int jj = 0; jj < b->njobs; ++jj) by_caller[b->caller[jj]] = h[jj].status;
  aidw_status first = AIDW_OK;
  int first_job = -1;
  for (int j = 0; j < b->njobs; ++j) {
    if (status) status[j] = by_caller[j];
    if (by_caller[j] != AIDW_OK && first == AIDW_OK) {
      first = (aidw_status)by_caller[j];
      first_job = j;
    }
  }
  if (first != AIDW_OK) return fail(first, "job %d: %s", first_job, aidw_status_string(first));
  return AIDW_OK;
}

}  // namespace

extern "C" {

void aidw_batch_config_default(aidw_batch_config* c) {
  if (!c) return;
  c->q = 1;
  c->split_points = 0;
  c->workers_per_cu = 8;
  c->integer_powers = 1;
  c->use_graph = 0;
}

aidw_status aidw_batch_create(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* cfg, aidw_batch** out) {
  return create_plan(jobs, njobs, cfg, out);
}

aidw_status aidw_batch_run(aidw_batch* b, hipStream_t stream) {
  if (!b) return fail(AIDW_EINVAL, "plan is NULL");
  return run_plan(b, stream);
}

aidw_status aidw_batch_job_status(aidw_batch* b, int32_t* status, hipStream_t stream) {
  if (!b) return fail(AIDW_EINVAL, "plan is NULL");
  return job_status(b, status, stream);
}

aidw_status aidw_batch_describe(const aidw_batch* b, aidw_batch_desc* out) {
  if (!b || !out) return fail(AIDW_EINVAL, "plan and out must be non-NULL");
  out->njobs = b->njobs;
  out->total_data = b->sum_n;
  out->total_queries = b->sum_m;
  out->total_pairs = b->sum_pairs;
  out->total_cells = b->sum_cap;
  out->work_items = b->nitems;
  out->workers = b->workers;
  out->kmax = b->kmax;
  out->workspace_bytes = (int64_t)b->mem_bytes;
  out->config = b->cfg;
  return AIDW_OK;
}

aidw_status aidw_batch_set_timing(aidw_batch* b, int32_t enable) {
  if (!b) return fail(AIDW_EINVAL, "plan is NULL");
  b->timing = enable != 0;
  return AIDW_OK;
}

aidw_status aidw_batch_last_timing(aidw_batch* b, aidw_batch_timing* out) {
  if (!b || !out) return fail(AIDW_EINVAL, "plan and out must be non-NULL");
  if (!b->timed) return fail(AIDW_EINVAL, "no timed run of this plan");
  HIP_TRY(hipEventSynchronize(b->ev[4]), "waiting for the timed run");
  float t[4];
  for (int i = 0; i < 4; ++i) HIP_TRY(hipEventElapsedTime(&t[i], b->ev[i], b->ev[i + 1]), "reading events");
  out->grid_ms = t[0];
  out->knn_ms = t[1];
  out->interp_ms = t[2];
  out->finish_ms = t[3];
  return AIDW_OK;
}

void aidw_batch_destroy(aidw_batch* b) { destroy_plan(b); }

aidw_status aidw_run_batch(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* cfg, int32_t* status,
                           hipStream_t stream) {
  aidw_batch_config c;
  if (cfg)
    c = *cfg;
  else
    aidw_batch_config_default(&c);
  c.use_graph = 0;
  aidw_batch* b = nullptr;
  aidw_status st = create_plan(jobs, njobs, &c, &b);
  if (st != AIDW_OK) return st;
  st = run_plan(b, stream);
  if (st == AIDW_OK) st = job_status(b, status, stream);
  destroy_plan(b);
  return st;
}

aidw_status aidw_batch_tune(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* candidates,
                            int32_t ncandidates, int32_t reps, float* ms_out, hipStream_t stream) {
  if (!candidates || ncandidates < 1 || !ms_out || reps < 1)
    return fail(AIDW_EINVAL, "need candidates, ncandidates >= 1, reps >= 1 and ms_out");
  for (int c = 0; c < ncandidates; ++c) {
    aidw_status st = check_config(&candidates[c]);
    if (st != AIDW_OK) return fail(st, "candidate %d: %s", c, aidw_last_error_detail());
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "creating events");
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "creating events");
  }
  aidw_status st = AIDW_OK;
  for (int c = 0; c < ncandidates && st == AIDW_OK; ++c) {
    aidw_batch* b = nullptr;
    st = create_plan(jobs, njobs, &candidates[c], &b);
    if (st != AIDW_OK) break;
    st = run_plan(b, stream);  // warm-up (and graph capture)
    for (int r = 0; r < reps && st == AIDW_OK; ++r) {
      if (r == 0 && (he = hipEventRecord(e0, stream)) != hipSuccess) st = hip_fail(he, "recording an event");
      if (st == AIDW_OK) st = run_plan(b, stream);
    }
    if (st == AIDW_OK && (he = hipEventRecord(e1, stream)) != hipSuccess) st = hip_fail(he, "recording an event");
    if (st == AIDW_OK && (he = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(he, "waiting for the runs");
    float ms = 0.0f;
    if (st == AIDW_OK && (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) st = hip_fail(he, "reading events");
    if (st == AIDW_OK) ms_out[c] = ms / (float)reps;
    destroy_plan(b);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // extern "C"
