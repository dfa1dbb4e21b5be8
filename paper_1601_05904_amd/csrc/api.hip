// Host side of the C ABI declared in include/aidw.h: argument checks, device
// memory, stream ordering and the composition of the two stages.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "aidw_internal.h"

using namespace aidw;


namespace {

thread_local std::string g_detail;
thread_local int g_timing = 0;
thread_local int g_cfg_q = 0, g_cfg_split = 0, g_cfg_intpow = 1;
thread_local int g_split_cap = 0;  // > 0: at most this many data-axis splits (aidw_run_noalloc)
thread_local int g_knn_window = 0;  // 1: the one-lane kNN stages each workgroup's cells in LDS

// A fixed device region that a call carves its temporaries from instead of allocating
// (aidw_run_noalloc): 256-byte aligned pieces in request order, nothing is freed.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};
thread_local Arena* g_arena = nullptr;

hipError_t arena_take(void** p, size_t bytes) {
  const size_t b = (bytes + 255) / 256 * 256;
  if (b > g_arena->cap - g_arena->used) return hipErrorOutOfMemory;
  *p = g_arena->base + g_arena->used;
  g_arena->used += b;
  return hipSuccess;
}
bool in_arena(const void* p) {
  return g_arena && (const char*)p >= g_arena->base && (const char*)p < g_arena->base + g_arena->cap;
}

struct Timing {
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool valid = false;
  int q = 0, split = 0;
  ~Timing() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};
thread_local Timing g_tm;

}  // namespace

namespace aidw {

aidw_status fail(aidw_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_detail = buf;
  return st;
}

void clear_error_detail() { g_detail.clear(); }

aidw_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(AIDW_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(AIDW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Test hook: AIDW_FAULT=alloc makes every device allocation fail (host-forced ENOMEM).
bool fault_alloc() {
  const char* f = getenv("AIDW_FAULT");
  return f && strcmp(f, "alloc") == 0;
}

hipError_t dmalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (g_arena) return arena_take(p, bytes);
  if (fault_alloc()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes ? bytes : 1);
}

// Temporaries of a call come from a cache of device blocks that outlives the call:
// stream-ordered allocation from the default pool maps fresh memory on most calls
// (measured: ~60 us per allocation, ~0.9 ms per aidw_run), which would dominate the
// small stages.  A released block carries an event recorded on the releasing
// stream; a later request on the same stream reuses it without waiting (stream
// order), one on another stream waits for that event on the device (no host sync).
// Blocks are only freed by aidw_release_cached_memory.
struct CachedBlock {
  void* p = nullptr;
  size_t bytes = 0;
  int device = 0;
  hipStream_t stream = nullptr;  // stream of the last use
  hipEvent_t done = nullptr;     // recorded on that stream when the block was released
  bool busy = false;
};
std::mutex g_cache_mu;
std::vector<CachedBlock>& block_cache() {
  static std::vector<CachedBlock>* cache = new std::vector<CachedBlock>();  // lives until the process ends
  return *cache;
}

size_t block_size_class(size_t bytes) {
  if (bytes <= (1u << 20)) {  // powers of two up to 1 MiB
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    return c;
  }
  const size_t g = 1u << 20;  // 1 MiB steps beyond
  return (bytes + g - 1) / g * g;
}

hipError_t dmalloc_async(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (g_arena) return arena_take(p, bytes);
  if (fault_alloc()) return hipErrorOutOfMemory;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t want = block_size_class(bytes ? bytes : 1);
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto& cache = block_cache();
    int best = -1;
    for (int i = 0; i < (int)cache.size(); ++i) {
      const CachedBlock& b = cache[i];
      if (b.busy || b.device != dev || b.bytes < want || b.bytes > 2 * want) continue;
      if (best < 0 || b.bytes < cache[best].bytes || (b.bytes == cache[best].bytes && b.stream == s))
        best = i;
    }
    if (best >= 0) {
      CachedBlock& b = cache[best];
      if (b.stream != s && (e = hipStreamWaitEvent(s, b.done, 0)) != hipSuccess) return e;
      b.busy = true;
      b.stream = s;
      *p = b.p;
      return hipSuccess;
    }
  }
  CachedBlock nb;
  nb.bytes = want;
  nb.device = dev;
  nb.stream = s;
  nb.busy = true;
  if ((e = hipMalloc(&nb.p, want)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&nb.done, hipEventDisableTiming)) != hipSuccess) {
    (void)hipFree(nb.p);
    return e;
  }
  std::lock_guard<std::mutex> lock(g_cache_mu);
  block_cache().push_back(nb);
  *p = nb.p;
  return hipSuccess;
}

void dfree_async(void* p, hipStream_t s) {
  if (!p || in_arena(p)) return;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  for (CachedBlock& b : block_cache()) {
    if (b.p != p) continue;
    (void)hipEventRecord(b.done, s);
    b.stream = s;
    b.busy = false;
    return;
  }
}

// Scoped stream-ordered temporaries.
struct Temps {
  hipStream_t s;
  void* ptrs[32];
  int count = 0;
  explicit Temps(hipStream_t st) : s(st) {}
  ~Temps() {
    for (int i = 0; i < count; ++i) dfree_async(ptrs[i], s);
  }
  template <typename T>
  hipError_t get(T** out, size_t elems) {
    void* p = nullptr;
    if (count >= 32) return hipErrorInvalidValue;
    hipError_t e = dmalloc_async(&p, elems * sizeof(T), s);
    if (e != hipSuccess) return e;
    ptrs[count++] = p;
    *out = static_cast<T*>(p);
    return hipSuccess;
  }
};

bool finite_pos(double v) { return isfinite(v) && v > 0; }

aidw_status check_params(const aidw_params* p) {
  if (!p) return fail(AIDW_EINVAL, "params is NULL");
  for (int i = 0; i < 5; ++i)
    if (!finite_pos(p->alpha[i])) return fail(AIDW_EINVAL, "alpha[%d] = %g must be finite and > 0", i, p->alpha[i]);
  if (!isfinite(p->r_min) || !isfinite(p->r_max) || p->r_min < 0 || !(p->r_max > p->r_min))
    return fail(AIDW_EINVAL, "need 0 <= r_min < r_max (got %g, %g)", p->r_min, p->r_max);
  if (!isfinite(p->area)) return fail(AIDW_EINVAL, "area must be finite");
  if (!isfinite(p->cell_width)) return fail(AIDW_EINVAL, "cell_width must be finite");
  if (!(p->cell_width > 0) && !finite_pos(p->occupancy))
    return fail(AIDW_EINVAL, "occupancy must be finite and > 0 when cell_width <= 0");
  return AIDW_OK;
}

int bits_for(int64_t ncells) {
  int b = 0;
  while (b < 31 && (1LL << b) < ncells) ++b;
  return b;
}

}  // namespace aidw

namespace {

// Per host thread and device: a pinned landing slot for the grid scalars and an event.
// Calls on one thread run one at a time, so the slot is free when a call starts.
hipError_t scalar_staging(GridScalars** slot, hipEvent_t* ev) {
  constexpr int kMaxDevices = 64;
  thread_local GridScalars* pinned[kMaxDevices] = {};
  thread_local hipEvent_t events[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!pinned[dev] && (e = hipHostMalloc((void**)&pinned[dev], sizeof(GridScalars), hipHostMallocDefault)) != hipSuccess)
    return e;
  if (!events[dev] && (e = hipEventCreateWithFlags(&events[dev], hipEventDisableTiming)) != hipSuccess) return e;
  *slot = pinned[dev];
  *ev = events[dev];
  return hipSuccess;
}

// Cell budget of a grid in occupancy mode: twice the cells the default side gives on a square
// box plus the rim of a box of any aspect ratio up to about 4:1 (the batched form uses the same
// budget).  Grids within it are built without a host round trip (banded build).
int64_t occupancy_budget(int64_t n, double occ) {
  const double base = (double)n / occ;
  return (int64_t)(2.0 * ceil(base) + 4.0 * ceil(sqrt(base)) + 16.0);
}

// Queries binned by the grid build (the banded build bins the queries it bounds).
struct QueryBins {
  uint32_t* order = nullptr;  // [m] query indices in cell order
  float* qx = nullptr;        // [m] their coordinates in that order
  float* qy = nullptr;
  bool valid = false;
};

aidw_status status_error(const GridScalars& h) {
  if (h.status == AIDW_ENONFINITE) return fail(AIDW_ENONFINITE, "a coordinate is NaN or infinite");
  if (h.status == AIDW_EDEGENERATE)
    return fail(AIDW_EDEGENERATE, "the study area resolves to %g (collinear or coincident points); pass params.area",
                h.area);
  if (h.status == AIDW_ECAPACITY)
    return fail(AIDW_ECAPACITY, "grid would exceed %lld cells; increase cell_width or occupancy",
                (long long)AIDW_MAX_CELLS);
  if (h.status != AIDW_OK) return fail(AIDW_EDEVICE, "grid finalize status %d", h.status);
  return AIDW_OK;
}

// Waits for the grid build queued on s and fills g->host from the device scalars; returns the
// build's status.
aidw_status sync_grid_host(aidw_grid* g, hipStream_t s) {
  GridScalars* pinned = nullptr;
  hipEvent_t ready = nullptr;
  hipError_t e;
  if (g_arena) {  // no pinned landing slot (it would be allocated on first use): a pageable read
    GridScalars h{};
    if ((e = hipMemcpyAsync(&h, g->dev, sizeof(GridScalars), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "reading grid scalars");
    g->host = h;
    g->host_valid = true;
    return status_error(g->host);
  }
  if ((e = scalar_staging(&pinned, &ready)) != hipSuccess) return hip_fail(e, "scalar staging");
  if ((e = hipMemcpyAsync(pinned, g->dev, sizeof(GridScalars), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipEventRecord(ready, s)) != hipSuccess || (e = hipEventSynchronize(ready)) != hipSuccess)
    return hip_fail(e, "reading grid scalars");
  g->host = *pinned;
  g->host_valid = true;
  return status_error(g->host);
}

// The grid of the data points.  In occupancy mode with a cell budget within the banded build's
// limit, the whole build (and, with bins, the binning of the queries) is queued without waiting
// for the host: g->host is filled only with wait_host (the status is then checked too),
// otherwise the caller reads the status later (sync_grid_host).  With an explicit cell side
// (or a budget beyond the banded limit) the host waits once for the scalars, then sizes the
// grid exactly and sorts by a stable LSD radix sort; bins are then left invalid.
// outer (may be null): the caller's temporaries, released when the caller's call ends, so the
// release's event records are issued after the rest of the caller's work, not between the grid
// build and the next stage.
aidw_status build_grid_impl(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                            const aidw_params* p, hipStream_t s, bool async, aidw_grid** out, Temps* outer = nullptr,
                            QueryBins* bins = nullptr, bool wait_host = true, aidw_grid* storage = nullptr) {
  aidw_grid* g = storage ? storage : new aidw_grid();
  if (storage) {
    *g = aidw_grid();
    g->heap = false;
  }
  g->n = n;
  g->async = async;
  g->async_stream = s;
  auto cleanup = [&](aidw_status st) {
    aidw_grid_destroy(g);
    return st;
  };
  hipError_t e = async ? dmalloc_async((void**)&g->dev, sizeof(GridScalars), s)
                       : dmalloc((void**)&g->dev, sizeof(GridScalars));
  if (e != hipSuccess) return cleanup(hip_fail(e, "allocating grid scalars"));
  Temps local(s);
  Temps& t = outer ? *outer : local;
  auto alloc = [&](void** ptr, size_t bytes) { return async ? dmalloc_async(ptr, bytes, s) : dmalloc(ptr, bytes); };
  const bool occ_mode = !(p->cell_width > 0);
  const int64_t budget = occ_mode ? occupancy_budget(n, p->occupancy) : 0;
  if (occ_mode && budget <= kBandMaxCells) {
    const bool bin_q = bins != nullptr && m > 0;
    const int64_t total = n + (bin_q ? m : 0);
    BandScratch b{};
    if ((e = t.get(&b.partial, kBoundsBlocks)) != hipSuccess || (e = t.get(&b.hist, band_hist_words(total))) != hipSuccess ||
        (e = t.get(&b.totals, 2 * kMaxBands)) != hipSuccess || (e = t.get(&b.dstart, 2 * kMaxBands + 1)) != hipSuccess ||
        (e = t.get(&b.bidx, total)) != hipSuccess || (e = t.get(&b.bx, total)) != hipSuccess ||
        (e = t.get(&b.by, total)) != hipSuccess)
      return cleanup(hip_fail(e, "allocating grid-build buffers"));
    if (bin_q && ((e = t.get(&bins->order, m)) != hipSuccess || (e = t.get(&bins->qx, m)) != hipSuccess ||
                  (e = t.get(&bins->qy, m)) != hipSuccess))
      return cleanup(hip_fail(e, "allocating query-binning buffers"));
    g->cells_alloc = budget;
    if ((e = alloc((void**)&g->cell_start, sizeof(int32_t) * (budget + 1))) != hipSuccess ||
        (e = alloc((void**)&g->sx, sizeof(float) * n)) != hipSuccess ||
        (e = alloc((void**)&g->sy, sizeof(float) * n)) != hipSuccess ||
        (e = alloc((void**)&g->sidx, sizeof(int32_t) * n)) != hipSuccess)
      return cleanup(hip_fail(e, "allocating grid arrays"));
    if ((e = build_grid_banded(x, y, n, qx, qy, m, bin_q, p->area, p->cell_width, p->occupancy, budget, g->dev,
                               g->cell_start, g->sx, g->sy, g->sidx, bin_q ? bins->order : nullptr,
                               bin_q ? bins->qx : nullptr, bin_q ? bins->qy : nullptr, b, s)) != hipSuccess)
      return cleanup(hip_fail(e, "grid build"));
    if (bins) bins->valid = bin_q;
    g->host_valid = false;
    if (wait_host) {
      aidw_status st = sync_grid_host(g, s);
      if (st != AIDW_OK) return cleanup(st);
    }
    *out = g;
    return AIDW_OK;
  }
  // The host needs the cell count (to size the CSR array and the sort's passes) and the
  // status.  The scalars are copied into pinned memory behind an event; the cell keys and
  // the sort's first 10-bit pass, which do not depend on them, are queued before the host
  // waits for that event, so the device keeps working while the host reads them.
  GridScalars* pinned = nullptr;
  hipEvent_t ready = nullptr;
  if ((e = scalar_staging(&pinned, &ready)) != hipSuccess) return cleanup(hip_fail(e, "scalar staging"));
  BoundsPartial* part = nullptr;
  uint32_t *keys, *vals, *tk, *tv, *hist, *scan;
  if ((e = t.get(&part, kBoundsBlocks)) != hipSuccess || (e = t.get(&keys, n)) != hipSuccess ||
      (e = t.get(&vals, n)) != hipSuccess || (e = t.get(&tk, n)) != hipSuccess || (e = t.get(&tv, n)) != hipSuccess ||
      (e = t.get(&hist, radix_hist_words((int)n))) != hipSuccess ||
      (e = t.get(&scan, radix_scan_tmp_words((int)n))) != hipSuccess)
    return cleanup(hip_fail(e, "allocating grid-build buffers"));
  if ((e = launch_bounds(x, y, (int)n, qx, qy, (int)m, part, s)) != hipSuccess)
    return cleanup(hip_fail(e, "bounds kernel"));
  if ((e = launch_finalize(part, kBoundsBlocks, n, p->area, p->cell_width, p->occupancy, g->dev, s)) != hipSuccess)
    return cleanup(hip_fail(e, "finalize kernel"));
  if ((e = hipMemcpyAsync(pinned, g->dev, sizeof(GridScalars), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipEventRecord(ready, s)) != hipSuccess)
    return cleanup(hip_fail(e, "reading grid scalars"));
  if ((e = cell_keys_first_pass(x, y, (int)n, g->dev, keys, vals, tk, tv, hist, scan, s)) != hipSuccess)
    return cleanup(hip_fail(e, "cell keys / first sort pass"));
  uint32_t *sk = tk, *sv = tv;  // the pairs sorted so far (in keys / vals or in the temporaries)
  if ((e = hipEventSynchronize(ready)) != hipSuccess) return cleanup(hip_fail(e, "synchronising grid scalars"));
  g->host = *pinned;
  g->host_valid = true;
  aidw_status st = status_error(g->host);
  if (st != AIDW_OK) return cleanup(st);

  const int64_t ncells = g->host.ncells;
  g->cells_alloc = ncells;
  if ((e = alloc((void**)&g->cell_start, sizeof(int32_t) * (ncells + 1))) != hipSuccess ||
      (e = alloc((void**)&g->sx, sizeof(float) * n)) != hipSuccess ||
      (e = alloc((void**)&g->sy, sizeof(float) * n)) != hipSuccess ||
      (e = alloc((void**)&g->sidx, sizeof(int32_t) * n)) != hipSuccess)
    return cleanup(hip_fail(e, "allocating grid arrays"));
  // the remaining passes, on the buffers the first one left the pairs in
  uint32_t* ok = sk == keys ? tk : keys;
  uint32_t* ov = sv == vals ? tv : vals;
  if ((e = radix_sort_wide_from(sk, sv, ok, ov, (int)n, kRadixBitsWide, bits_for(ncells), hist, scan, s, &sk, &sv)) !=
      hipSuccess)
    return cleanup(hip_fail(e, "radix sort"));
  if ((e = launch_cell_start_gather(sk, sv, (int)n, ncells, x, y, g->cell_start, g->sx, g->sy, g->sidx, s)) !=
      hipSuccess)
    return cleanup(hip_fail(e, "cell offsets / gather"));
  if (bins) bins->valid = false;
  *out = g;
  return AIDW_OK;
}

aidw_status check_data(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m) {
  if (!x || !y) return fail(AIDW_EINVAL, "x / y is NULL");
  if (n < 1) return fail(AIDW_EINVAL, "n = %lld: need at least one data point", (long long)n);
  if (n > INT32_MAX) return fail(AIDW_ECAPACITY, "n = %lld exceeds INT32_MAX", (long long)n);
  if (m < 0) return fail(AIDW_EINVAL, "m = %lld < 0", (long long)m);
  if (m > INT32_MAX) return fail(AIDW_ECAPACITY, "m = %lld exceeds INT32_MAX", (long long)m);
  if (m > 0 && (!qx || !qy)) return fail(AIDW_EINVAL, "qx / qy is NULL");
  return AIDW_OK;
}

// The queries in cell order: those the grid build binned (bins), else a counting sort here,
// which needs the grid's host description.
aidw_status query_order(const aidw_grid* g, const float* qx, const float* qy, int64_t m, const QueryBins* bins,
                        Temps& t, hipStream_t s, const uint32_t** order_out) {
  if (bins && bins->valid) {
    *order_out = bins->order;
    return AIDW_OK;
  }
  if (!g->host_valid) return fail(AIDW_EDEVICE, "query binning needs the grid's description");
  const int64_t ncells = g->host.ncells;
  uint32_t *cnt, *key, *slot, *scan, *order;
  hipError_t e;
  if ((e = t.get(&cnt, ncells + 1)) != hipSuccess || (e = t.get(&key, m)) != hipSuccess ||
      (e = t.get(&slot, m)) != hipSuccess || (e = t.get(&scan, scan_tmp_words(ncells + 1))) != hipSuccess ||
      (e = t.get(&order, m)) != hipSuccess)
    return hip_fail(e, "allocating query-binning buffers");
  // bin the queries with the data's cell formula: order lists them in cell order
  HIP_TRY(bin_queries(g->dev, qx, qy, (int)m, ncells, cnt, key, slot, scan, order, s), "query binning");
  *order_out = order;
  return AIDW_OK;
}

aidw_status knn_impl(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, float* r_obs,
                     float* d1sq, int32_t* nn_idx, hipStream_t s, bool paper_rule = false,
                     const QueryBins* bins = nullptr) {
  Temps t(s);
  const uint32_t* order = nullptr;
  aidw_status st = query_order(g, qx, qy, m, bins, t, s, &order);
  if (st != AIDW_OK) return st;
  if (paper_rule) {
    HIP_TRY(launch_knn_paper(g->dev, g->cell_start, g->sx, g->sy, g->sidx, qx, qy, order, (int)m, k, r_obs, d1sq,
                             nn_idx, s),
            "kNN kernel (paper rule)");
    return AIDW_OK;
  }
  // below 2^17 queries one lane per query leaves the chip idle: four lanes share each query
  if (m >= (1 << 17) && g_knn_window) {
    HIP_TRY(launch_knn_window(g->dev, g->cell_start, g->sx, g->sy, g->sidx, qx, qy, order, (int)m, k, r_obs, d1sq,
                              nn_idx, s),
            "kNN kernel (LDS window)");
    return AIDW_OK;
  }
  auto knn = m < (1 << 17) ? launch_knn4 : launch_knn;
  HIP_TRY(knn(g->dev, g->cell_start, g->sx, g->sy, g->sidx, qx, qy, order, nullptr, (int)m, k, r_obs, d1sq, nn_idx, s),
          "kNN kernel");
  return AIDW_OK;
}

void choose_interp_config(int64_t n, int64_t m, int* q, int* split) {
  // One query per lane (the most wavefronts per SIMD: the pair loop is latency-bound on the
  // transcendental unit, and occupancy hides it better than in-lane ILP).  The data axis is
  // split as finely as the float64 partials allow: the largest power of two with at least
  // 2048 points per split, at most 256 splits and 16 split m bytes of partials <= 1 GiB.
  // Fine splits keep the chip full when the queries are few (measured at 2^18 clustered
  // with one launch per class: 8 splits 64 % of the roofline, 128 splits 82 %; at 2^20
  // uniform 32 -> 64 splits 86.0 -> 86.2 %).
  const int qq = g_cfg_q ? g_cfg_q : 1;
  int sp = 1;
  if (g_cfg_split) {
    sp = g_cfg_split;
  } else {
    const int64_t max_by_mem = ((int64_t)1 << 26) / (m > 0 ? m : 1);
    while (sp < 256 && (int64_t)sp * 2 <= max_by_mem && n / ((int64_t)sp * 2) >= 2048) sp *= 2;
  }
  if (g_split_cap > 0)
    while (sp > g_split_cap) sp >>= 1;
  if (sp > n) sp = (int)n;
  *q = qq;
  *split = sp < 1 ? 1 : sp;
}

aidw_status interp_impl(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy,
                        int64_t m, const float* r_obs, const float* d1sq, const aidw_params* p, const aidw_grid* g,
                        float* qz, float* alpha_out, hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end,
                        int* used_q, int* used_split, const float* alpha_in = nullptr, bool naive = false) {
  AlphaParams ap;
  if (p->area > 0) {
    ap.r_exp = 1.0 / (2.0 * sqrt((double)n / p->area));
  } else if (!g) {
    return fail(AIDW_EINVAL, "aidw_interpolate needs params.area > 0 or a grid");
  } else if (g->host_valid) {
    if (!(g->host.area > 0)) return fail(AIDW_EINVAL, "the grid's area is not positive");
    ap.r_exp = g->n == n ? g->host.r_exp : 1.0 / (2.0 * sqrt((double)n / g->host.area));
  } else {
    // a grid still being built on this stream (a run): its r_exp is read on the device
    ap.r_exp = 0.0;
    ap.r_exp_dev = &g->dev->r_exp;
  }
  ap.r_min = p->r_min;
  ap.r_max = p->r_max;
  for (int i = 0; i < 5; ++i) ap.levels[i] = p->alpha[i];
  int q, split;
  choose_interp_config(n, m, &q, &split);
  if (used_q) *used_q = q;
  if (used_split) *used_split = split;
  // integer levels get their own pair kernel (alpha == p: w = rsq(t)^p)
  uint32_t fast_mask = 0;
  if (g_cfg_intpow)
    for (int i = 0; i < 5; ++i) {
      const double a = p->alpha[i];
      if (a >= 1.0 && a <= 8.0 && a == floor(a)) fast_mask |= 1u << (int)a;
    }
  Temps t(s);
  double2* partial = nullptr;
  uint32_t *count, *list, *keys, *perm, *tk, *tv, *hist, *scan;
  float *alpha_f, *xp, *yp, *zp;
  const int npad = interp_padded_len((int)n);
  hipError_t e;
  if (split > 1 && (e = t.get(&partial, (size_t)split * m)) != hipSuccess) return hip_fail(e, "allocating partials");
  if ((e = t.get(&count, 1)) != hipSuccess || (e = t.get(&list, m)) != hipSuccess ||
      (e = t.get(&alpha_f, m)) != hipSuccess || (e = t.get(&keys, m)) != hipSuccess ||
      (e = t.get(&perm, m)) != hipSuccess || (e = t.get(&tk, m)) != hipSuccess || (e = t.get(&tv, m)) != hipSuccess ||
      (e = t.get(&hist, radix_hist_words((int)m))) != hipSuccess ||
      (e = t.get(&scan, radix_scan_tmp_words((int)m))) != hipSuccess || (e = t.get(&xp, npad)) != hipSuccess ||
      (e = t.get(&yp, npad)) != hipSuccess || (e = t.get(&zp, npad)) != hipSuccess)
    return hip_fail(e, "allocating interpolation buffers");
  // the coincident-query count is cleared by the padding copy (or on its own for the untiled
  // kernel) and the list filled by the class-key kernel
  if (!naive)
    HIP_TRY(launch_pad_copy(x, y, z, (int)n, xp, yp, zp, count, s), "padding copy");
  else
    HIP_TRY(hipMemsetAsync(count, 0, sizeof(uint32_t), s), "clearing coincidence count");
  const float* alpha_use = alpha_f;
  if (alpha_in) {  // alpha given per query: only the class keys are needed
    alpha_use = alpha_in;
    if (alpha_out)
      HIP_TRY(hipMemcpyAsync(alpha_out, alpha_in, sizeof(float) * m, hipMemcpyDeviceToDevice, s), "copying alpha");
    HIP_TRY(launch_class_keys(alpha_in, (int)m, keys, perm, d1sq, count, list, s), "class key kernel");
  } else {
    HIP_TRY(launch_alpha_class(r_obs, (int)m, ap, alpha_f, alpha_out, keys, perm, d1sq, count, list, s),
            "alpha kernel");
  }
  uint32_t *ckeys = keys, *cperm = perm;  // the class order (in keys / perm or in the temporaries)
  if (fast_mask && !naive)
    HIP_TRY(radix_sort_pairs_to(keys, perm, tk, tv, (int)m, 4, hist, scan, s, &ckeys, &cperm), "class sort");
  if (ev_begin) HIP_TRY(hipEventRecord(ev_begin, s), "event");
  if (naive) {
    HIP_TRY(launch_interp_naive(x, y, z, (int)n, qx, qy, alpha_use, d1sq, (int)m, qz, s),
            "interpolation kernel (untiled)");
  } else {
    HIP_TRY(launch_interp(xp, yp, zp, (int)n, qx, qy, alpha_use, d1sq, cperm, ckeys, (int)m, fast_mask, q, split, qz,
                          partial, g ? g->dev : nullptr, s),
            "interpolation kernel");
  }
  if (ev_end) HIP_TRY(hipEventRecord(ev_end, s), "event");
  if (split > 1 && !naive) HIP_TRY(launch_combine(partial, (int)m, split, qz, s), "combine kernel");
  if (g && g->n == n)
    HIP_TRY(launch_fixup_grid(count, list, qx, qy, g->dev, g->cell_start, g->sx, g->sy, g->sidx, z, qz, s),
            "coincidence fix-up kernel");
  else
    HIP_TRY(launch_fixup_scan(count, list, qx, qy, x, y, z, (int)n, qz, s), "coincidence fix-up kernel");
  return AIDW_OK;
}

}  // namespace

struct aidw_mlp {
  MlpDevice d{};
  void* block = nullptr;
  double occupancy = 2.0;
  uint64_t step = 0;
};

namespace {

constexpr int kP = AIDW_MLP_PARAMS;

// Float offsets of the network's arrays inside its single device allocation.
struct MlpLayout {
  static constexpr size_t master = 0, mom = kP, vel = 2 * kP, w1p = 3 * kP, w2p = w1p + 64 * 14, w3p = w2p + 64 * 32,
                          w2r = w3p + 32, w3r = w2r + 64 * 64,
                          w1a = (w3r + 64 + 63) / 64 * 64, w2a = w1a + 4 * 64 * 4, b1f = w2a + 8 * 64 * 4,
                          b2f = b1f + 64, w3f = b2f + 64, total = w3f + 64;
};

aidw_status mlp_alloc(aidw_mlp** out) {
  aidw_mlp* h = new aidw_mlp();
  hipError_t e = dmalloc(&h->block, sizeof(float) * MlpLayout::total);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "allocating the network");
  }
  float* b = static_cast<float*>(h->block);
  h->d.master = b + MlpLayout::master;
  h->d.mom = b + MlpLayout::mom;
  h->d.vel = b + MlpLayout::vel;
  h->d.w1p = reinterpret_cast<uint32_t*>(b + MlpLayout::w1p);
  h->d.w2p = reinterpret_cast<uint32_t*>(b + MlpLayout::w2p);
  h->d.w3p = reinterpret_cast<uint32_t*>(b + MlpLayout::w3p);
  h->d.w2r = b + MlpLayout::w2r;
  h->d.w3r = b + MlpLayout::w3r;
  h->d.w1a = reinterpret_cast<uint32_t*>(b + MlpLayout::w1a);
  h->d.w2a = reinterpret_cast<uint32_t*>(b + MlpLayout::w2a);
  h->d.b1f = b + MlpLayout::b1f;
  h->d.b2f = b + MlpLayout::b2f;
  h->d.w3f = b + MlpLayout::w3f;
  *out = h;
  return AIDW_OK;
}

// Uploads masters (and optionally the optimiser state), then rebuilds the bf16 copies.
aidw_status mlp_upload(aidw_mlp* h, const float* master, const float* mom, const float* vel) {
  HIP_TRY(hipMemcpy(h->d.master, master, sizeof(float) * kP, hipMemcpyHostToDevice), "uploading parameters");
  if (mom && vel) {
    HIP_TRY(hipMemcpy(h->d.mom, mom, sizeof(float) * kP, hipMemcpyHostToDevice), "uploading optimiser state");
    HIP_TRY(hipMemcpy(h->d.vel, vel, sizeof(float) * kP, hipMemcpyHostToDevice), "uploading optimiser state");
  } else {
    HIP_TRY(hipMemset(h->d.mom, 0, sizeof(float) * 2 * kP), "clearing optimiser state");
  }
  HIP_TRY(launch_mlp_repack(h->d, nullptr), "repacking weights");
  HIP_TRY(hipDeviceSynchronize(), "repacking weights");
  return AIDW_OK;
}

// SplitMix64 (Steele, Lea & Flood): the initial weights' generator.
uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr char kMlpMagic[8] = {'A', 'I', 'D', 'W', 'M', 'L', 'P', 1};

}  // namespace

extern "C" {

void aidw_params_default(aidw_params* p) {
  if (!p) return;
  p->k = 10;
  for (int i = 0; i < 5; ++i) p->alpha[i] = i + 1.0;
  p->r_min = 0.0;
  p->r_max = 2.0;
  p->area = 0.0;
  p->cell_width = 0.0;
  p->occupancy = 2.0;
}

aidw_status aidw_build_grid(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                            const aidw_params* p, hipStream_t stream, aidw_grid** out) {
  g_detail.clear();
  if (!out) return fail(AIDW_EINVAL, "out is NULL");
  *out = nullptr;
  aidw_status st = check_data(x, y, n, qx, qy, m);
  if (st != AIDW_OK) return st;
  if ((st = check_params(p)) != AIDW_OK) return st;
  return build_grid_impl(x, y, n, qx, qy, m, p, stream, false, out);
}

aidw_status aidw_grid_describe(const aidw_grid* g, aidw_grid_desc* out) {
  if (!g || !out) return fail(AIDW_EINVAL, "grid / out is NULL");
  out->n = g->n;
  out->min_x = g->host.minx;
  out->min_y = g->host.miny;
  out->max_x = g->host.maxx;
  out->max_y = g->host.maxy;
  out->area = g->host.area;
  out->r_exp = g->host.r_exp;
  out->cell_width = g->host.cw;
  out->inv_cell_width = g->host.inv_cw;
  out->ncol = g->host.ncol;
  out->nrow = g->host.nrow;
  return AIDW_OK;
}

aidw_status aidw_grid_info(const aidw_grid* g, double* area, double* r_exp, double* cell_width, int32_t* ncol,
                           int32_t* nrow) {
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  if (area) *area = g->host.area;
  if (r_exp) *r_exp = g->host.r_exp;
  if (cell_width) *cell_width = g->host.cw;
  if (ncol) *ncol = g->host.ncol;
  if (nrow) *nrow = g->host.nrow;
  return AIDW_OK;
}

aidw_status aidw_grid_arrays(const aidw_grid* g, const int32_t** cell_start, const float** sx, const float** sy,
                             const int32_t** sidx) {
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  if (cell_start) *cell_start = g->cell_start;
  if (sx) *sx = g->sx;
  if (sy) *sy = g->sy;
  if (sidx) *sidx = g->sidx;
  return AIDW_OK;
}

aidw_status aidw_grid_copy_arrays(const aidw_grid* g, int32_t* cell_start, float* sx, float* sy, int32_t* sidx,
                                  hipStream_t stream) {
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  const size_t n = (size_t)g->n;
  if (cell_start)
    HIP_TRY(hipMemcpyAsync(cell_start, g->cell_start, sizeof(int32_t) * (size_t)(g->host.ncells + 1),
                           hipMemcpyDeviceToDevice, stream),
            "copying cell_start");
  if (sx) HIP_TRY(hipMemcpyAsync(sx, g->sx, sizeof(float) * n, hipMemcpyDeviceToDevice, stream), "copying sx");
  if (sy) HIP_TRY(hipMemcpyAsync(sy, g->sy, sizeof(float) * n, hipMemcpyDeviceToDevice, stream), "copying sy");
  if (sidx) HIP_TRY(hipMemcpyAsync(sidx, g->sidx, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, stream), "copying sidx");
  return AIDW_OK;
}

void aidw_grid_destroy(aidw_grid* g) {
  if (!g) return;
  void* ptrs[5] = {g->dev, g->cell_start, g->sx, g->sy, g->sidx};
  for (void* p : ptrs) {
    if (!p) continue;
    if (g->async)
      dfree_async(p, g->async_stream);
    else
      (void)hipFree(p);
  }
  if (g->heap) delete g;
}

aidw_status aidw_knn(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, float* r_obs,
                     float* d1sq, int32_t* nn_idx, hipStream_t stream) {
  g_detail.clear();
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  if (m < 0) return fail(AIDW_EINVAL, "m = %lld < 0", (long long)m);
  if (m > INT32_MAX) return fail(AIDW_ECAPACITY, "m exceeds INT32_MAX");
  if (k < 1 || k > AIDW_KMAX || k > g->n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", k, (long long)g->n, AIDW_KMAX);
  if (m == 0) return AIDW_OK;
  if (!qx || !qy || !r_obs) return fail(AIDW_EINVAL, "qx / qy / r_obs is NULL");
  if ((int64_t)m * k > INT32_MAX && nn_idx) return fail(AIDW_ECAPACITY, "m * k exceeds INT32_MAX");
  return knn_impl(g, qx, qy, m, k, r_obs, d1sq, nn_idx, stream);
}

aidw_status aidw_knn_paper(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, float* r_obs,
                           float* d1sq, int32_t* nn_idx, hipStream_t stream) {
  g_detail.clear();
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  if (m < 0) return fail(AIDW_EINVAL, "m = %lld < 0", (long long)m);
  if (m > INT32_MAX) return fail(AIDW_ECAPACITY, "m exceeds INT32_MAX");
  if (k < 1 || k > AIDW_KMAX || k > g->n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", k, (long long)g->n, AIDW_KMAX);
  if (m == 0) return AIDW_OK;
  if (!qx || !qy || !r_obs) return fail(AIDW_EINVAL, "qx / qy / r_obs is NULL");
  if ((int64_t)m * k > INT32_MAX && nn_idx) return fail(AIDW_ECAPACITY, "m * k exceeds INT32_MAX");
  return knn_impl(g, qx, qy, m, k, r_obs, d1sq, nn_idx, stream, true);
}

aidw_status aidw_nn_statistic(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, double clip,
                              float* R, hipStream_t stream) {
  g_detail.clear();
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  if (m < 0) return fail(AIDW_EINVAL, "m = %lld < 0", (long long)m);
  if (m > INT32_MAX) return fail(AIDW_ECAPACITY, "m exceeds INT32_MAX");
  if (k < 1 || k > AIDW_KMAX || k > g->n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", k, (long long)g->n, AIDW_KMAX);
  if (isnan(clip)) return fail(AIDW_EINVAL, "clip is NaN");
  if (m == 0) return AIDW_OK;
  if (!qx || !qy || !R) return fail(AIDW_EINVAL, "qx / qy / R is NULL");
  Temps t(stream);
  float* r_obs = nullptr;
  HIP_TRY(t.get(&r_obs, m), "allocating r_obs");
  aidw_status st = knn_impl(g, qx, qy, m, k, r_obs, nullptr, nullptr, stream);
  if (st != AIDW_OK) return st;
  const double cap = isinf(clip) ? 0.0 : clip;
  HIP_TRY(launch_nn_statistic(r_obs, (int)m, g->host.r_exp, cap, R, stream), "statistic kernel");
  return AIDW_OK;
}

aidw_status aidw_interpolate(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                             const float* qy, int64_t m, const float* r_obs, const float* d1sq, const aidw_params* p,
                             const aidw_grid* g, float* qz, float* alpha_out, hipStream_t stream) {
  g_detail.clear();
  aidw_status st = check_data(x, y, n, qx, qy, m);
  if (st != AIDW_OK) return st;
  if (!z) return fail(AIDW_EINVAL, "z is NULL");
  if ((st = check_params(p)) != AIDW_OK) return st;
  if (m == 0) return AIDW_OK;
  if (!r_obs || !d1sq || !qz) return fail(AIDW_EINVAL, "r_obs / d1sq / qz is NULL");
  return interp_impl(x, y, z, n, qx, qy, m, r_obs, d1sq, p, g, qz, alpha_out, stream, nullptr, nullptr, nullptr,
                     nullptr);
}

aidw_status aidw_interpolate_naive(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                                   const float* qy, int64_t m, const float* r_obs, const float* d1sq,
                                   const aidw_params* p, const aidw_grid* g, float* qz, float* alpha_out,
                                   hipStream_t stream) {
  g_detail.clear();
  aidw_status st = check_data(x, y, n, qx, qy, m);
  if (st != AIDW_OK) return st;
  if (!z) return fail(AIDW_EINVAL, "z is NULL");
  if ((st = check_params(p)) != AIDW_OK) return st;
  if (m == 0) return AIDW_OK;
  if (!r_obs || !d1sq || !qz) return fail(AIDW_EINVAL, "r_obs / d1sq / qz is NULL");
  return interp_impl(x, y, z, n, qx, qy, m, r_obs, d1sq, p, g, qz, alpha_out, stream, nullptr, nullptr, nullptr,
                     nullptr, nullptr, true);
}

aidw_status aidw_knn_bruteforce(const float* x, const float* y, int64_t n, const float* qx, const float* qy,
                                int64_t m, int32_t k, float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t stream) {
  g_detail.clear();
  if (!x || !y) return fail(AIDW_EINVAL, "x / y is NULL");
  if (n < 1 || m < 0) return fail(AIDW_EINVAL, "need n >= 1 and m >= 0 (n = %lld, m = %lld)", (long long)n,
                                  (long long)m);
  if (n > INT32_MAX || m > INT32_MAX) return fail(AIDW_ECAPACITY, "sizes exceed INT32_MAX");
  if (k < 1 || k > AIDW_KMAX || k > n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", k, (long long)n, AIDW_KMAX);
  if (m == 0) return AIDW_OK;
  if (!qx || !qy || !r_obs) return fail(AIDW_EINVAL, "qx / qy / r_obs is NULL");
  if ((int64_t)m * k > INT32_MAX && nn_idx) return fail(AIDW_ECAPACITY, "m * k exceeds INT32_MAX");
  HIP_TRY(launch_knn_brute(x, y, (int)n, qx, qy, (int)m, k, r_obs, d1sq, nn_idx, stream), "brute-force kNN kernel");
  return AIDW_OK;
}

namespace {

aidw_status check_run_args(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                           const float* qy, int64_t m, const aidw_params* p, float* qz) {
  aidw_status st = check_data(x, y, n, qx, qy, m);
  if (st != AIDW_OK) return st;
  if (!z) return fail(AIDW_EINVAL, "z is NULL");
  if ((st = check_params(p)) != AIDW_OK) return st;
  if (p->k < 1 || p->k > AIDW_KMAX || p->k > n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", p->k, (long long)n, AIDW_KMAX);
  if (m > 0 && !qz) return fail(AIDW_EINVAL, "qz is NULL");
  return AIDW_OK;
}

// The whole method (arguments checked, m > 0).  grid_storage: where the grid's handle lives
// (null: the library allocates it).
aidw_status run_impl(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy,
                     int64_t m, const aidw_params* p, float* qz, float* alpha_out, float* r_obs_out,
                     hipStream_t stream, aidw_grid* grid_storage) {
  aidw_status st = AIDW_OK;
  hipEvent_t* ev = nullptr;
  if (g_timing) {
    for (auto& e : g_tm.ev)
      if (!e) HIP_TRY(hipEventCreate(&e), "creating timing events");
    ev = g_tm.ev;
    g_tm.valid = false;
    HIP_TRY(hipEventRecord(ev[0], stream), "event");
  }
  aidw_grid* g = nullptr;
  Temps grid_temps(stream);
  QueryBins bins;
  if ((st = build_grid_impl(x, y, n, qx, qy, m, p, stream, true, &g, &grid_temps, &bins, false, grid_storage)) !=
      AIDW_OK)
    return st;
  if (ev) {
    hipError_t e = hipEventRecord(ev[1], stream);
    if (e != hipSuccess) {
      aidw_grid_destroy(g);
      return hip_fail(e, "event");
    }
  }
  {
    Temps t(stream);
    float *robs = r_obs_out, *d1sq = nullptr;
    hipError_t e = hipSuccess;
    if (!robs) e = t.get(&robs, m);
    if (e == hipSuccess) e = t.get(&d1sq, m);
    if (e != hipSuccess) st = hip_fail(e, "allocating r_obs / d1sq");
    if (st == AIDW_OK) st = knn_impl(g, qx, qy, m, p->k, robs, d1sq, nullptr, stream, false, &bins);
    int q = 0, split = 0;
    if (st == AIDW_OK)
      st = interp_impl(x, y, z, n, qx, qy, m, robs, d1sq, p, g, qz, alpha_out, stream, ev ? ev[2] : nullptr,
                       ev ? ev[3] : nullptr, &q, &split);
    if (st == AIDW_OK && ev) {
      if ((e = hipEventRecord(ev[4], stream)) != hipSuccess) st = hip_fail(e, "event");
      g_tm.valid = st == AIDW_OK;
      g_tm.q = q;
      g_tm.split = split;
    }
  }
  // the grid was built without a host round trip: its status (non-finite input, degenerate
  // area) is read once everything is queued
  if (st == AIDW_OK && !g->host_valid) st = sync_grid_host(g, stream);
  aidw_grid_destroy(g);
  return st;
}

// ---- aidw_run_noalloc: every temporary of a run from one fixed device array per GPU

constexpr size_t kScratchBytes = (size_t)AIDW_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// This device's copy of `scratch` (its address is only known through the runtime).
hipError_t scratch_region(char** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static char* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    addr[dev] = static_cast<char*>(ptr);
  }
  *out = addr[dev];
  return hipSuccess;
}

size_t piece(size_t bytes) { return (bytes + 255) / 256 * 256; }

// Scratch bytes of run_impl in occupancy mode, split data-axis splits (the pieces it takes
// from the arena, in any order).
size_t run_scratch_bytes(int64_t n, int64_t m, double occ, bool robs_given, int split) {
  const int64_t total = n + m;
  const int64_t budget = occupancy_budget(n, occ);
  size_t b = piece(sizeof(GridScalars));
  b += piece(sizeof(BoundsPartial) * kBoundsBlocks) + piece(4 * band_hist_words(total)) +
       piece(4 * 2 * kMaxBands) + piece(4 * (2 * kMaxBands + 1)) + 3 * piece(4 * (size_t)total);  // band sort
  b += 3 * piece(4 * (size_t)m);                                                                 // query bins
  b += piece(4 * (size_t)(budget + 1)) + 3 * piece(4 * (size_t)n);                                // the grid
  b += (robs_given ? 0 : piece(4 * (size_t)m)) + piece(4 * (size_t)m);                          // r_obs, d1^2
  if (split > 1) b += piece(16 * (size_t)split * m);                                             // partials
  b += piece(4) + 6 * piece(4 * (size_t)m) + piece(4 * radix_hist_words((int)m)) +
       piece(4 * radix_scan_tmp_words((int)m)) + 3 * piece(4 * (size_t)interp_padded_len((int)n));  // Eq. 1-6
  return b;
}

}  // namespace

aidw_status aidw_run(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy,
                     int64_t m, const aidw_params* p, float* qz, float* alpha_out, float* r_obs_out,
                     hipStream_t stream) {
  g_detail.clear();
  aidw_status st = check_run_args(x, y, z, n, qx, qy, m, p, qz);
  if (st != AIDW_OK || m == 0) return st;
  return run_impl(x, y, z, n, qx, qy, m, p, qz, alpha_out, r_obs_out, stream, nullptr);
}

aidw_status aidw_run_noalloc(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                             const float* qy, int64_t m, const aidw_params* p, float* qz, float* alpha_out,
                             float* r_obs_out, hipStream_t stream) {
  g_detail.clear();
  aidw_status st = check_run_args(x, y, z, n, qx, qy, m, p, qz);
  if (st != AIDW_OK || m == 0) return st;
  if (p->cell_width > 0)
    return fail(AIDW_EINVAL, "aidw_run_noalloc sizes the grid by occupancy: params.cell_width must be <= 0");
  if (occupancy_budget(n, p->occupancy) > kBandMaxCells)
    return fail(AIDW_ECAPACITY, "n / occupancy too large for aidw_run_noalloc's grid (at most %lld cells)",
                (long long)kBandMaxCells);
  const bool robs_given = r_obs_out != nullptr;
  const size_t base = run_scratch_bytes(n, m, p->occupancy, robs_given, 1);
  if (base > kScratchBytes)
    return fail(AIDW_ECAPACITY, "n = %lld, m = %lld need %zu bytes of scratch; aidw_run_noalloc has %zu",
                (long long)n, (long long)m, base, kScratchBytes);
  // the largest power-of-two data-axis split whose float64 partials fit beside the rest
  int cap = 1;
  while (cap < 256 && run_scratch_bytes(n, m, p->occupancy, robs_given, cap * 2) <= kScratchBytes) cap *= 2;
  char* region = nullptr;
  hipError_t e = scratch_region(&region);
  if (e != hipSuccess) return hip_fail(e, "locating the scratch array");
  Arena arena{region, kScratchBytes, 0};
  aidw_grid grid;
  g_arena = &arena;
  g_split_cap = cap;
  st = run_impl(x, y, z, n, qx, qy, m, p, qz, alpha_out, r_obs_out, stream, &grid);
  g_split_cap = 0;
  g_arena = nullptr;
  return st;
}

aidw_status aidw_mlp_create(uint64_t seed, double occupancy, aidw_mlp** out) {
  g_detail.clear();
  if (!out) return fail(AIDW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!finite_pos(occupancy)) return fail(AIDW_EINVAL, "occupancy must be finite and > 0");
  float host[kP];
  uint64_t st = seed;
  auto uniform = [&](double a) { return (float)(a * (2.0 * ((splitmix64(st) >> 11) * 0x1.0p-53) - 1.0)); };
  int o = 0;
  for (int i = 0; i < 64 * 27; ++i) host[o++] = uniform(sqrt(6.0 / 27.0));
  for (int i = 0; i < 64; ++i) host[o++] = 0.0f;
  for (int i = 0; i < 64 * 64; ++i) host[o++] = uniform(sqrt(6.0 / 64.0));
  for (int i = 0; i < 64; ++i) host[o++] = 0.0f;
  for (int i = 0; i < 64; ++i) host[o++] = uniform(sqrt(6.0 / 64.0));
  host[o++] = 0.0f;
  aidw_mlp* h = nullptr;
  aidw_status stt = mlp_alloc(&h);
  if (stt != AIDW_OK) return stt;
  h->occupancy = occupancy;
  if ((stt = mlp_upload(h, host, nullptr, nullptr)) != AIDW_OK) {
    aidw_mlp_destroy(h);
    return stt;
  }
  *out = h;
  return AIDW_OK;
}

void aidw_mlp_destroy(aidw_mlp* mlp) {
  if (!mlp) return;
  if (mlp->block) (void)hipFree(mlp->block);
  delete mlp;
}

double aidw_mlp_occupancy(const aidw_mlp* mlp) { return mlp ? mlp->occupancy : 0.0; }

aidw_status aidw_mlp_set_params(aidw_mlp* mlp, const float* host_params) {
  g_detail.clear();
  if (!mlp || !host_params) return fail(AIDW_EINVAL, "network / params is NULL");
  for (int i = 0; i < kP; ++i)
    if (!isfinite(host_params[i])) return fail(AIDW_EINVAL, "parameter %d is not finite", i);
  mlp->step = 0;
  return mlp_upload(mlp, host_params, nullptr, nullptr);
}

aidw_status aidw_mlp_get_params(const aidw_mlp* mlp, float* host_params) {
  g_detail.clear();
  if (!mlp || !host_params) return fail(AIDW_EINVAL, "network / params is NULL");
  HIP_TRY(hipDeviceSynchronize(), "synchronising");
  HIP_TRY(hipMemcpy(host_params, mlp->d.master, sizeof(float) * kP, hipMemcpyDeviceToHost), "reading parameters");
  return AIDW_OK;
}

aidw_status aidw_mlp_save(const aidw_mlp* mlp, const char* path) {
  g_detail.clear();
  if (!mlp || !path) return fail(AIDW_EINVAL, "network / path is NULL");
  std::string buf(sizeof(float) * 3 * kP, '\0');
  HIP_TRY(hipDeviceSynchronize(), "synchronising");
  HIP_TRY(hipMemcpy(&buf[0], mlp->d.master, buf.size(), hipMemcpyDeviceToHost), "reading the network");
  FILE* f = fopen(path, "wb");
  if (!f) return fail(AIDW_EINVAL, "cannot open %s for writing", path);
  const uint32_t hdr[4] = {1u, AIDW_MLP_INPUTS, 64u, (uint32_t)kP};
  bool ok = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(hdr, sizeof hdr, 1, f) == 1 &&
            fwrite(&mlp->occupancy, sizeof(double), 1, f) == 1 && fwrite(&mlp->step, sizeof(uint64_t), 1, f) == 1 &&
            fwrite(buf.data(), 1, buf.size(), f) == buf.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? AIDW_OK : fail(AIDW_EINVAL, "writing %s failed", path);
}

aidw_status aidw_mlp_load(const char* path, aidw_mlp** out) {
  g_detail.clear();
  if (!path || !out) return fail(AIDW_EINVAL, "path / out is NULL");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(AIDW_EINVAL, "cannot open %s", path);
  char magic[8];
  uint32_t hdr[4];
  double occ = 0;
  uint64_t step = 0;
  std::string buf(sizeof(float) * 3 * kP, '\0');
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMlpMagic, 8) == 0 && fread(hdr, sizeof hdr, 1, f) == 1 &&
            hdr[0] == 1u && hdr[1] == AIDW_MLP_INPUTS && hdr[2] == 64u && hdr[3] == (uint32_t)kP &&
            fread(&occ, sizeof occ, 1, f) == 1 && fread(&step, sizeof step, 1, f) == 1 &&
            fread(&buf[0], 1, buf.size(), f) == buf.size() && finite_pos(occ);
  fclose(f);
  if (!ok) return fail(AIDW_EINVAL, "%s is not a network checkpoint of this version", path);
  aidw_mlp* h = nullptr;
  aidw_status st = mlp_alloc(&h);
  if (st != AIDW_OK) return st;
  h->occupancy = occ;
  h->step = step;
  const float* fb = reinterpret_cast<const float*>(buf.data());
  if ((st = mlp_upload(h, fb, fb + kP, fb + 2 * kP)) != AIDW_OK) {
    aidw_mlp_destroy(h);
    return st;
  }
  *out = h;
  return AIDW_OK;
}

aidw_status aidw_features(const aidw_grid* g, const float* qx, const float* qy, int64_t m, float* feat, float* d1sq,
                          hipStream_t stream) {
  g_detail.clear();
  if (!g) return fail(AIDW_EINVAL, "grid is NULL");
  if (m < 0 || m > INT32_MAX) return fail(AIDW_EINVAL, "m = %lld out of range", (long long)m);
  if (m == 0) return AIDW_OK;
  if (!qx || !qy || !feat) return fail(AIDW_EINVAL, "qx / qy / feat is NULL");
  HIP_TRY(launch_features(g->dev, g->cell_start, g->sx, g->sy, qx, qy, nullptr, (int)m, g->n, feat, d1sq, stream),
          "feature kernel");
  return AIDW_OK;
}

aidw_status aidw_mlp_forward(const aidw_mlp* mlp, const float* feat, int64_t m, float* r_hat, hipStream_t stream) {
  g_detail.clear();
  if (!mlp) return fail(AIDW_EINVAL, "network is NULL");
  if (m < 0 || m > INT32_MAX) return fail(AIDW_EINVAL, "m = %lld out of range", (long long)m);
  if (m == 0) return AIDW_OK;
  if (!feat || !r_hat) return fail(AIDW_EINVAL, "feat / r_hat is NULL");
  HIP_TRY(launch_mlp_forward(mlp->d, feat, (int)m, r_hat, stream), "network forward kernel");
  return AIDW_OK;
}

aidw_status aidw_mlp_gradients(const aidw_mlp* mlp, const float* feat, const float* target, int64_t batch,
                               float* grad, hipStream_t stream) {
  g_detail.clear();
  if (!mlp || !feat || !target || !grad) return fail(AIDW_EINVAL, "network / feat / target / grad is NULL");
  if (batch < 1 || batch > (1 << 20)) return fail(AIDW_EINVAL, "batch = %lld out of [1, 2^20]", (long long)batch);
  Temps t(stream);
  float* scratch;
  hipError_t e = t.get(&scratch, mlp_batch_scratch_floats((int)batch));
  if (e != hipSuccess) return hip_fail(e, "allocating batch scratch");
  HIP_TRY(launch_mlp_gradients(mlp->d, feat, target, nullptr, (int)batch, scratch, grad, stream), "gradient kernels");
  return AIDW_OK;
}

aidw_status aidw_mlp_train(aidw_mlp* mlp, const float* feat, const float* target, int64_t count, int32_t epochs,
                           int32_t batch, float lr, uint64_t seed, float* epoch_loss, hipStream_t stream) {
  g_detail.clear();
  if (!mlp || !feat || !target) return fail(AIDW_EINVAL, "network / feat / target is NULL");
  if (count < 1 || count > INT32_MAX) return fail(AIDW_EINVAL, "count = %lld out of range", (long long)count);
  if (epochs < 1 || batch < 1 || batch > (1 << 20)) return fail(AIDW_EINVAL, "need epochs >= 1 and 1 <= batch <= 2^20");
  if (!(lr > 0) || !isfinite(lr)) return fail(AIDW_EINVAL, "lr must be finite and > 0");
  const int N = (int)count, B = batch < N ? batch : N;
  const int nb = (N + B - 1) / B;
  Temps t(stream);
  uint32_t *keys, *vals, *tk, *tv, *hist, *scan;
  float *scratch, *grad, *eloss;
  hipError_t e;
  if ((e = t.get(&keys, N)) != hipSuccess || (e = t.get(&vals, N)) != hipSuccess || (e = t.get(&tk, N)) != hipSuccess ||
      (e = t.get(&tv, N)) != hipSuccess || (e = t.get(&hist, radix_hist_words(N))) != hipSuccess ||
      (e = t.get(&scan, radix_scan_tmp_words(N))) != hipSuccess ||
      (e = t.get(&scratch, mlp_batch_scratch_floats(B))) != hipSuccess || (e = t.get(&grad, kP + 1)) != hipSuccess ||
      (e = t.get(&eloss, epochs)) != hipSuccess)
    return hip_fail(e, "allocating training buffers");
  HIP_TRY(hipMemsetAsync(eloss, 0, sizeof(float) * epochs, stream), "clearing losses");
  const double b1 = 0.9, b2 = 0.999;
  for (int ep = 0; ep < epochs; ++ep) {
    HIP_TRY(launch_shuffle_keys(seed, ep, N, keys, vals, stream), "shuffle keys");
    HIP_TRY(radix_sort_pairs(keys, vals, tk, tv, N, 32, hist, scan, stream), "shuffle sort");
    for (int bi = 0; bi < nb; ++bi) {
      const int start = bi * B, cnt = N - start < B ? N - start : B;
      HIP_TRY(launch_mlp_gradients(mlp->d, feat, target, vals + start, cnt, scratch, grad, stream), "gradient kernels");
      mlp->step += 1;
      const float bc1 = (float)(1.0 - pow(b1, (double)mlp->step)), bc2 = (float)(1.0 - pow(b2, (double)mlp->step));
      HIP_TRY(launch_adam(mlp->d, grad, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2, stream), "Adam kernel");
      HIP_TRY(launch_mlp_repack(mlp->d, stream), "repack kernel");
      HIP_TRY(launch_accumulate_loss(grad, eloss, ep, 1.0f / (float)nb, stream), "loss kernel");
    }
  }
  if (epoch_loss) {
    HIP_TRY(hipMemcpyAsync(epoch_loss, eloss, sizeof(float) * epochs, hipMemcpyDeviceToHost, stream), "reading losses");
    HIP_TRY(hipStreamSynchronize(stream), "synchronising");
  }
  return AIDW_OK;
}

aidw_status aidw_run_learned(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                             const float* qy, int64_t m, const aidw_params* p, const aidw_mlp* mlp, int32_t rule,
                             double delta, float* qz, float* alpha_out, float* r_hat_out, int64_t* fallback_count,
                             hipStream_t stream) {
  g_detail.clear();
  aidw_status st = check_data(x, y, n, qx, qy, m);
  if (st != AIDW_OK) return st;
  if (!z) return fail(AIDW_EINVAL, "z is NULL");
  if ((st = check_params(p)) != AIDW_OK) return st;
  if (!mlp) return fail(AIDW_EINVAL, "network is NULL");
  if (rule < AIDW_FALLBACK_LITERAL || rule > AIDW_FALLBACK_NETWORK_GATED_CERTIFICATE)
    return fail(AIDW_EINVAL, "unknown rule %d", rule);
  if (!(delta >= 0) || !isfinite(delta)) return fail(AIDW_EINVAL, "delta must be finite and >= 0");
  if (p->cell_width > 0 || p->occupancy != mlp->occupancy)
    return fail(AIDW_EINVAL, "the grid must use the network's occupancy (%g) and no explicit cell width",
                mlp->occupancy);
  if (p->k < 1 || p->k > AIDW_KMAX || p->k > n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", p->k, (long long)n, AIDW_KMAX);
  if (fallback_count) *fallback_count = 0;
  if (m == 0) return AIDW_OK;
  if (!qz) return fail(AIDW_EINVAL, "qz is NULL");
  hipEvent_t* ev = nullptr;
  if (g_timing) {
    for (auto& e : g_tm.ev)
      if (!e) HIP_TRY(hipEventCreate(&e), "creating timing events");
    ev = g_tm.ev;
    g_tm.valid = false;
    HIP_TRY(hipEventRecord(ev[0], stream), "event");
  }
  aidw_grid* g = nullptr;
  Temps grid_temps(stream);
  QueryBins bins;
  if ((st = build_grid_impl(x, y, n, qx, qy, m, p, stream, true, &g, &grid_temps, &bins, false)) != AIDW_OK)
    return st;
  uint32_t host_count = 0;
  {
    Temps t(stream);
    hipError_t e = hipSuccess;
    if (ev) e = hipEventRecord(ev[1], stream);
    // Queries are processed in cell order (as the kNN kernel takes them): one kernel computes
    // the features, the network (on the matrix cores) and the decision per position of that
    // order.  The fallback list keeps that order, so the kNN kernel sees the queries binned as
    // well (its locality depends on it): the front of rules 2-4 appends each wavefront's
    // fallback queries together (one atomic per wavefront); for rules 0 and 1 the list is the
    // flagged positions, compacted in order by a prefix sum.
    const bool append = rule == AIDW_FALLBACK_CERTIFIED || rule == AIDW_FALLBACK_CERTIFIED_THEN_ALPHA_EXACT ||
                        rule == AIDW_FALLBACK_NETWORK_GATED_CERTIFICATE;
    float *d1sq = nullptr, *alpha_f = nullptr, *r_obs = nullptr;
    uint32_t *flag = nullptr, *list = nullptr, *stmp = nullptr, *count = nullptr;
    const int mm = (int)m;
    if (e == hipSuccess) e = t.get(&d1sq, mm);
    if (e == hipSuccess) e = t.get(&alpha_f, mm);
    if (e == hipSuccess) e = t.get(&r_obs, mm);
    if (e == hipSuccess && !append) e = t.get(&flag, mm);
    if (e == hipSuccess) e = t.get(&list, mm);
    if (e == hipSuccess && !append) e = t.get(&stmp, scan_tmp_words(mm));
    if (e == hipSuccess) e = t.get(&count, 1);
    if (e != hipSuccess) st = hip_fail(e, "allocating learned-R buffers");
    const uint32_t* order = nullptr;
    if (st == AIDW_OK) st = query_order(g, qx, qy, m, &bins, t, stream, &order);
    AlphaParams ap;
    ap.r_exp = 0.0;
    ap.r_exp_dev = &g->dev->r_exp;
    ap.r_min = p->r_min;
    ap.r_max = p->r_max;
    for (int i = 0; i < 5; ++i) ap.levels[i] = p->alpha[i];
    // R where mu = 0.1 and 0.9 (Eq. 5 as applied): alpha is saturated below / above them (Eq. 6)
    const double r_sat_lo = p->r_min + p->r_max / M_PI * acos(0.8);
    const double r_sat_hi = p->r_min + p->r_max / M_PI * acos(-0.8);
    // the certificate's threshold on the sum of the k nearest distances, in units of r_exp:
    // alpha = alpha_5 for R > min(r_sat_hi, R_max) (Eq. 5 is 1 from R_max on); the margin covers
    // the float32 rounding of r_obs and the rounding of mu near 0.9
    const double cert_factor = (double)p->k * fmin(r_sat_hi, p->r_max) * (1.0 + 1e-6);
#define STEP(expr, what) \
  if (st == AIDW_OK && (e = (expr)) != hipSuccess) st = hip_fail(e, what)
    if (append) STEP(hipMemsetAsync(count, 0, sizeof(uint32_t), stream), "clearing the fallback count");
    STEP(launch_learned_front(mlp->d, g->dev, g->cell_start, g->sx, g->sy, qx, qy, order, mm, n, ap, rule, delta,
                              r_sat_lo, r_sat_hi, p->k, cert_factor, flag, append ? list : nullptr,
                              append ? count : nullptr, alpha_f, d1sq, r_hat_out, nullptr, stream),
         "features / network / decision kernel");
    if (!append) STEP(compact_flags(flag, order, mm, stmp, list, count, stream), "fallback compaction");
    // the fallback queries are few and hard (cluster edges): eight lanes per query measured best
    STEP(launch_knn_lanes(g->dev, g->cell_start, g->sx, g->sy, g->sidx, qx, qy, list, count, mm, p->k, r_obs, d1sq,
                          nullptr, 8, stream, &ap, alpha_f),
         "kNN kernel (with Eq. 4-6)");
#undef STEP
    int q = 0, split = 0;
    if (st == AIDW_OK)
      st = interp_impl(x, y, z, n, qx, qy, m, nullptr, d1sq, p, g, qz, alpha_out, stream, ev ? ev[2] : nullptr,
                       ev ? ev[3] : nullptr, &q, &split, alpha_f);
    if (st == AIDW_OK && fallback_count)
      if ((e = hipMemcpyAsync(&host_count, count, sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess)
        st = hip_fail(e, "reading the fallback count");
    if (st == AIDW_OK && ev) {
      if ((e = hipEventRecord(ev[4], stream)) != hipSuccess) st = hip_fail(e, "event");
      g_tm.valid = st == AIDW_OK;
      g_tm.q = q;
      g_tm.split = split;
    }
  }
  if (st == AIDW_OK && !g->host_valid) st = sync_grid_host(g, stream);
  aidw_grid_destroy(g);
  if (st == AIDW_OK && fallback_count) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "synchronising");
    *fallback_count = host_count;
  }
  return st;
}

aidw_status aidw_learned_routes(const float* x, const float* y, int64_t n, const float* qx, const float* qy,
                                int64_t m, const aidw_params* p, const aidw_mlp* mlp, int32_t rule, double delta,
                                uint8_t* route_out, float* r_hat_out, hipStream_t stream) {
  g_detail.clear();
  aidw_status st = check_data(x, y, n, qx, qy, m);
  if (st != AIDW_OK) return st;
  if ((st = check_params(p)) != AIDW_OK) return st;
  if (!mlp) return fail(AIDW_EINVAL, "network is NULL");
  if (rule < AIDW_FALLBACK_LITERAL || rule > AIDW_FALLBACK_NETWORK_GATED_CERTIFICATE)
    return fail(AIDW_EINVAL, "unknown rule %d", rule);
  if (!(delta >= 0) || !isfinite(delta)) return fail(AIDW_EINVAL, "delta must be finite and >= 0");
  if (p->cell_width > 0 || p->occupancy != mlp->occupancy)
    return fail(AIDW_EINVAL, "the grid must use the network's occupancy (%g) and no explicit cell width",
                mlp->occupancy);
  if (p->k < 1 || p->k > AIDW_KMAX || p->k > n)
    return fail(AIDW_EINVAL, "k = %d must be in [1, min(n = %lld, %d)]", p->k, (long long)n, AIDW_KMAX);
  if (m == 0) return AIDW_OK;
  if (!route_out) return fail(AIDW_EINVAL, "route_out is NULL");
  aidw_grid* g = nullptr;
  Temps grid_temps(stream);
  QueryBins bins;
  if ((st = build_grid_impl(x, y, n, qx, qy, m, p, stream, true, &g, &grid_temps, &bins, false)) != AIDW_OK)
    return st;
  {
    Temps t(stream);
    const int mm = (int)m;
    float *d1sq = nullptr, *alpha_f = nullptr;
    uint32_t* flag = nullptr;
    hipError_t e = t.get(&d1sq, mm);
    if (e == hipSuccess) e = t.get(&alpha_f, mm);
    if (e == hipSuccess) e = t.get(&flag, mm);
    if (e != hipSuccess) st = hip_fail(e, "allocating learned-R buffers");
    const uint32_t* order = nullptr;
    if (st == AIDW_OK) st = query_order(g, qx, qy, m, &bins, t, stream, &order);
    AlphaParams ap;
    ap.r_exp = 0.0;
    ap.r_exp_dev = &g->dev->r_exp;
    ap.r_min = p->r_min;
    ap.r_max = p->r_max;
    for (int i = 0; i < 5; ++i) ap.levels[i] = p->alpha[i];
    const double r_sat_lo = p->r_min + p->r_max / M_PI * acos(0.8);
    const double r_sat_hi = p->r_min + p->r_max / M_PI * acos(-0.8);
    const double cert_factor = (double)p->k * fmin(r_sat_hi, p->r_max) * (1.0 + 1e-6);
    if (st == AIDW_OK &&
        (e = launch_learned_front(mlp->d, g->dev, g->cell_start, g->sx, g->sy, qx, qy, order, mm, n, ap, rule, delta,
                                  r_sat_lo, r_sat_hi, p->k, cert_factor, flag, nullptr, nullptr, alpha_f, d1sq,
                                  r_hat_out, route_out, stream)) != hipSuccess)
      st = hip_fail(e, "features / network / decision kernel");
  }
  if (st == AIDW_OK && !g->host_valid) st = sync_grid_host(g, stream);
  aidw_grid_destroy(g);
  return st;
}

aidw_status aidw_set_timing(int enable) {
  g_timing = enable ? 1 : 0;
  if (!enable) g_tm.valid = false;
  return AIDW_OK;
}

aidw_status aidw_last_timing(aidw_timing* out) {
  if (!out) return fail(AIDW_EINVAL, "out is NULL");
  if (!g_timing || !g_tm.valid) return fail(AIDW_EINVAL, "no timed run (enable with aidw_set_timing(1))");
  HIP_TRY(hipEventSynchronize(g_tm.ev[4]), "waiting for timed run");
  float a = 0, b = 0, c = 0, d = 0;
  HIP_TRY(hipEventElapsedTime(&a, g_tm.ev[0], g_tm.ev[1]), "event time");
  HIP_TRY(hipEventElapsedTime(&b, g_tm.ev[1], g_tm.ev[2]), "event time");
  HIP_TRY(hipEventElapsedTime(&c, g_tm.ev[2], g_tm.ev[3]), "event time");
  HIP_TRY(hipEventElapsedTime(&d, g_tm.ev[3], g_tm.ev[4]), "event time");
  out->grid_ms = a;
  out->knn_ms = b;
  out->interp_ms = c;
  out->finish_ms = d;
  out->interp_q = g_tm.q;
  out->interp_split = g_tm.split;
  return AIDW_OK;
}

aidw_status aidw_set_knn_config(int32_t lds_window) {
  g_detail.clear();
  if (lds_window != 0 && lds_window != 1) return fail(AIDW_EINVAL, "lds_window must be 0 or 1");
  g_knn_window = lds_window;
  return AIDW_OK;
}

aidw_status aidw_set_interp_config(int32_t q, int32_t split, int32_t integer_powers) {
  if (!(q == 0 || q == 1 || q == 2 || q == 4 || q == 8)) return fail(AIDW_EINVAL, "q must be 0, 1, 2, 4 or 8");
  if (split < 0) return fail(AIDW_EINVAL, "split must be >= 0");
  if (integer_powers < -1 || integer_powers > 1) return fail(AIDW_EINVAL, "integer_powers must be -1, 0 or 1");
  g_cfg_q = q;
  g_cfg_split = split;
  g_cfg_intpow = integer_powers != 0;
  return AIDW_OK;
}

const char* aidw_status_string(aidw_status st) {
  switch (st) {
    case AIDW_OK: return "ok";
    case AIDW_EINVAL: return "invalid argument";
    case AIDW_EDEGENERATE: return "degenerate study area";
    case AIDW_ENOMEM: return "out of device memory";
    case AIDW_EDEVICE: return "HIP runtime error";
    case AIDW_ENONFINITE: return "non-finite coordinate";
    case AIDW_ECAPACITY: return "capacity exceeded";
  }
  return "unknown status";
}

const char* aidw_last_error_detail(void) { return g_detail.c_str(); }

aidw_status aidw_release_cached_memory(void) {
  g_detail.clear();
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "querying the device");
  HIP_TRY(hipDeviceSynchronize(), "synchronising");
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto& cache = block_cache();
  std::vector<CachedBlock> keep;
  for (CachedBlock& b : cache) {
    if (b.busy || b.device != dev) {
      keep.push_back(b);
      continue;
    }
    (void)hipEventDestroy(b.done);
    (void)hipFree(b.p);
  }
  cache.swap(keep);
  return AIDW_OK;
}

const char* aidw_version(void) { return "aidw-mi355x 0.1 (gfx950)"; }

}  // extern "C"
