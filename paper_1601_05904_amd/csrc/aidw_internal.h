// Internal declarations shared by the HIP sources of libaidw (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/aidw.h"

namespace aidw {

// Device-resident grid scalars, written by the finalize kernel (Section 4.1.1, Eq. 2).
struct GridScalars {
  float minx, miny, maxx, maxy;
  double area;    // A
  double r_exp;   // 1 / (2 sqrt(n / A))
  double cw;      // cell side
  double cwd;     // 1 / (double)inv_cw: the side implied by the float32 reciprocal
  float inv_cw;   // float32 reciprocal used for binning
  int32_t ncol, nrow;
  int32_t status; // 0 ok, else an aidw_status value
  int64_t ncells;
  int32_t band_shift;  // banded build: a band is 2^band_shift consecutive cells
  int32_t nbands;      // banded build: bands covering the ncells cells
};

// Per-block partial of the bounds reduction.
// Workgroups are dealt to the chip's 8 XCDs in turn (workgroup b to XCD b mod 8), and each XCD
// has its own L2.  This maps the hardware workgroup id to a logical one so that XCD x takes a
// contiguous range of logical workgroups: with binned queries, an XCD then reads one region
// of the grid through its L2 instead of every region.  A bijection of [0, nblk).
__device__ inline int xcd_block(int bid, int nblk) {
  constexpr int kXcds = 8;
  const int per = nblk / kXcds, rem = nblk % kXcds;
  const int x = bid % kXcds, s = bid / kXcds;
  return x * per + min(x, rem) + s;
}

struct BoundsPartial {
  float minx, miny, maxx, maxy;
  int32_t nonfinite;
  int32_t pad[3];
};

// Length of the register k-list of the kNN kernels for a given k: the insertion of a
// candidate runs one compare-and-swap step per slot, so the list is kept close to k.
__host__ __device__ inline int knn_slots(int k) {
  return k <= 8    ? 8
         : k <= 10 ? 10
         : k <= 12 ? 12
         : k <= 15 ? 15
         : k <= 16 ? 16
         : k <= 24 ? 24
         : k <= 32 ? 32
         : k <= 48 ? 48
                   : 64;
}
// M(KMAX) for the list length of k (a statement).
#define AIDW_FOR_KNN_SLOTS(k, M)   \
  switch (::aidw::knn_slots(k)) {  \
    case 8: M(8); break;           \
    case 10: M(10); break;         \
    case 12: M(12); break;         \
    case 15: M(15); break;         \
    case 16: M(16); break;         \
    case 24: M(24); break;         \
    case 32: M(32); break;         \
    case 48: M(48); break;         \
    default: M(64); break;         \
  }

// Slack, in cells, that covers the float32 binning error of a coordinate in a
// grid of ncol x nrow cells: |fl(fl(x - minX) * inv) - (x - minX) * inv| <= (c + 1) * 2^-23
// for column c, taken with a wide margin.
__host__ __device__ inline double slack_cells(int32_t ncol, int32_t nrow) {
  const double span = (double)(ncol > nrow ? ncol : nrow) + 1.0;
  return span * 4.76837158203125e-07 /* 2^-21 */ + 1e-9;
}
inline double slack_cells(const GridScalars& g) { return slack_cells(g.ncol, g.nrow); }

// ---- host helpers shared by the ABI sources (api.hip, batch.hip, noalloc.hip) ----

// Clears the message of aidw_last_error_detail on the calling thread.
void clear_error_detail();

// Records a message for aidw_last_error_detail on the calling thread and returns st.
aidw_status fail(aidw_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// AIDW_ENOMEM for allocation failures, else AIDW_EDEVICE, with the HIP message.
aidw_status hip_fail(hipError_t e, const char* what);
// hipMalloc of at least one byte; honours the AIDW_FAULT=alloc test hook.
hipError_t dmalloc(void** p, size_t bytes);
// Checks the method parameters other than k (alpha levels, r_min / r_max, area, cell side).
aidw_status check_params(const aidw_params* p);
// Smallest b with 2^b >= ncells (at most 31).
int bits_for(int64_t ncells);

#define HIP_TRY(expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, what);   \
  } while (0)

constexpr int kBoundsBlocks = 512;
constexpr int kBoundsThreads = 256;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                       // elements per thread per block
constexpr int kSortTile = kSortThreads * kSortItems; // elements per block
constexpr int kRadixBits = 8;                        // digit width of the sort passes
constexpr int kRadixBitsWide = 10;                   // used where it saves a pass
constexpr int kRadixMax = 1 << kRadixBitsWide;

// ---- banded grid build (grid_band.hip) ----
// The data points and the queries are sorted by cell in two steps: a stable counting sort by
// band (2^band_shift consecutive cells, at most kMaxBands bands per point set), then, per
// band, a stable counting sort by cell inside the band.  Limits: at most kMaxBands bands of at
// most 2^kMaxBandShift cells, i.e. kBandMaxCells cells.
constexpr int kMaxBands = 1024;
constexpr int kMaxBandShift = 12;
constexpr int64_t kBandMaxCells = (int64_t)kMaxBands << kMaxBandShift;
struct BandScratch {
  BoundsPartial* partial;  // [kBoundsBlocks]
  uint32_t* hist;          // [band_hist_words(total)]: per digit and block counts, then prefixes
  uint32_t* totals;        // [2 kMaxBands] per-digit totals
  uint32_t* dstart;        // [2 kMaxBands + 1]
  uint32_t* bidx;          // [total] band-sorted indices
  float* bx;               // [total] band-sorted coordinates
  float* by;
};
size_t band_hist_words(int64_t total);
// Largest band shift a grid of at most cap cells can need.
int band_shift_for(int64_t cap);
// Bounds over data and queries, the grid scalars (Eq. 2, Section 4.1.1; the cell side widened if
// the grid would exceed cap cells), and the stable sort of the data points into cell order:
// cell_start [cap + 1], sx, sy, sidx [n].  With bin_q, the queries too: qorder [m] lists them in
// cell order, qsx, qsy [m] (may be null) their coordinates in that order.  No host synchronisation.
hipError_t build_grid_banded(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                             bool bin_q, double area_in, double cw_in, double occ, int64_t cap, GridScalars* gs,
                             int32_t* cell_start, float* sx, float* sy, int32_t* sidx, uint32_t* qorder, float* qsx,
                             float* qsy, const BandScratch& b, hipStream_t s);

// Host-side launchers (all asynchronous on `s`; return the first HIP error).
hipError_t launch_bounds(const float* x, const float* y, int n, const float* qx, const float* qy, int m,
                         BoundsPartial* partial, hipStream_t s);
hipError_t launch_finalize(const BoundsPartial* partial, int nparts, int64_t n, double area_in, double cw_in,
                           double occ, GridScalars* out, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the keys.
// tmp_* are ping-pong buffers of n entries; hist needs radix_hist_words(n) words and
// scan_tmp radix_scan_tmp_words(n) words.  The result ends in (keys, vals).
size_t radix_hist_words(int n);
size_t radix_scan_tmp_words(int n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, int n, int bits,
                            uint32_t* hist, uint32_t* scan_tmp, hipStream_t s);
// The same without the copy-back: *out_keys / *out_vals receive the buffers (keys / vals or
// the temporaries) that hold the sorted result.
hipError_t radix_sort_pairs_to(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, int n, int bits,
                               uint32_t* hist, uint32_t* scan_tmp, hipStream_t s, uint32_t** out_keys,
                               uint32_t** out_vals);
// The 10-bit passes of the same sort for the digits at shift0, shift0 + 10, ... below `bits`
// (shift0 = 0 and bits = 10 is one pass; a later call with shift0 = 10 continues it on the
// buffers the first call returned).
// Cell keys of the data points (keys [n], vals [n] = index) and the first 10-bit pass of their
// stable radix sort into tmp_keys / tmp_vals, the key computation fused into the histogram.
hipError_t cell_keys_first_pass(const float* x, const float* y, int n, const GridScalars* gs, uint32_t* keys,
                                uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, uint32_t* hist,
                                uint32_t* scan_tmp, hipStream_t s);
hipError_t radix_sort_wide_from(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, int n,
                                int shift0, int bits, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s,
                                uint32_t** out_keys, uint32_t** out_vals);
// out[i] = in[0] + ... + in[i-1] (in and out may alias); *total (device, may be null) = the sum.
// tmp needs scan_tmp_words(len) words.
size_t scan_tmp_words(size_t len);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t len, uint32_t* tmp, uint32_t* total,
                              hipStream_t s);
// The queries in cell order (any order within a cell): order[m] lists them; cnt needs
// ncells + 1 words, key and slot m words each, scan_tmp scan_tmp_words(ncells + 1).
hipError_t bin_queries(const GridScalars* gs, const float* qx, const float* qy, int m, int64_t ncells, uint32_t* cnt,
                       uint32_t* key, uint32_t* slot, uint32_t* scan_tmp, uint32_t* order, hipStream_t s);
// Order-preserving compaction of 0 / 1 flags: list[j] = vals[i] for the j-th flagged i;
// *total (device) = the count.  tmp needs scan_tmp_words(len) words.
hipError_t compact_flags(const uint32_t* flag, const uint32_t* vals, size_t len, uint32_t* tmp, uint32_t* list,
                         uint32_t* total, hipStream_t s);
hipError_t launch_cell_start_gather(const uint32_t* keys, const uint32_t* vals, int n, int64_t ncells, const float* x,
                                    const float* y, int32_t* cell_start, float* sx, float* sy, int32_t* sidx,
                                    hipStream_t s);

// qperm (may be null) lists the queries in processing order; active (may be null) is a device
// count: only the first *active entries of qperm are processed.
// The kernels derive the binning slack (slack_cells) from the device scalars gs, and do no work
// when gs->status reports a failed grid build.
hipError_t launch_knn(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                      const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                      const uint32_t* active, int m, int k, float* r_obs, float* d1sq, int32_t* nn_idx,
                      hipStream_t s);
// The same search with each workgroup's neighbourhood of cells staged in LDS (k_knn_window).
hipError_t launch_knn_window(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                             const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm, int m, int k,
                             float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t s);
// Brute-force kNN over all n points per query (the method the grid search replaces); exact.
hipError_t launch_knn_brute(const float* x, const float* y, int n, const float* qx, const float* qy, int m, int k,
                            float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t s);
// The paper's stop rule (one more level after the block holds >= k points; not exact in general).
hipError_t launch_knn_paper(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                            const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm, int m, int k,
                            float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t s);
struct AlphaParams;
// The same with `lanes` (2, 4 or 8) lanes per query (for small or sparse query sets); identical results.
// With ap and alpha_f non-null, alpha_f[q] also receives Eq. 4-6 of each query's r_obs.
hipError_t launch_knn_lanes(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                            const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                            const uint32_t* active, int m, int k, float* r_obs, float* d1sq, int32_t* nn_idx,
                            int lanes, hipStream_t s, const AlphaParams* ap = nullptr, float* alpha_f = nullptr);
// Four lanes per query.
hipError_t launch_knn4(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                       const int32_t* sidx, const float* qx, const float* qy, const uint32_t* qperm,
                       const uint32_t* active, int m, int k, float* r_obs, float* d1sq, int32_t* nn_idx,
                       hipStream_t s);

struct AlphaParams {
  double r_exp;
  double r_min, r_max;
  double levels[5];
  const double* r_exp_dev = nullptr;  // non-null: r_exp is read here (a grid's device scalars)
};
__host__ __device__ inline double alpha_r_exp(const AlphaParams& ap) { return ap.r_exp_dev ? *ap.r_exp_dev : ap.r_exp; }

// Eq. 4-6 per query -> alpha_f [m] (and alpha_out if non-null); class keys [m] (p in 1..8 when
// alpha == p exactly, else 0) and the identity permutation vals [m], ready for a stable sort by key;
// the queries with d1sq = 0 appended to list, *count (cleared before) their number.
hipError_t launch_alpha_class(const float* r_obs, int m, const AlphaParams& ap, float* alpha_f, float* alpha_out,
                              uint32_t* keys, uint32_t* vals, const float* d1sq, uint32_t* count, uint32_t* list,
                              hipStream_t s);
// Eq. 4 per query: R[j] = min(r_obs[j] / r_exp, clip) in float64, stored as float32 (clip <= 0: none).
hipError_t launch_nn_statistic(const float* r_obs, int m, double r_exp, double clip, float* R, hipStream_t s);
// Pair kernels over the queries in class order (perm, sorted keys skeys); fast_mask bit p
// requests the integer-power kernel for class p (the general kernel covers every other block).
// x, y, z are the padded copies made by launch_pad_copy.
// gs (may be null): a grid whose failed status makes the launch do nothing.
hipError_t launch_interp(const float* x, const float* y, const float* z, int n, const float* qx, const float* qy,
                         const float* alpha_f, const float* d1sq, const uint32_t* perm, const uint32_t* skeys, int m,
                         uint32_t fast_mask, int q, int split, float* qz, double2* partial, const GridScalars* gs,
                         hipStream_t s);
// The untiled pair kernel (per-lane global loads, general alpha form, one data range).
hipError_t launch_interp_naive(const float* x, const float* y, const float* z, int n, const float* qx, const float* qy,
                               const float* alpha_f, const float* d1sq, int m, float* qz, hipStream_t s);
// Zero-padded copies of x, y, z for the pair kernels, which may prefetch one chunk past n.
int interp_padded_len(int n);
// zero_word (may be null) is cleared by the same launch.
hipError_t launch_pad_copy(const float* x, const float* y, const float* z, int n, float* xp, float* yp, float* zp,
                           uint32_t* zero_word, hipStream_t s);
hipError_t launch_combine(const double2* partial, int m, int split, float* qz, hipStream_t s);
hipError_t launch_fixup_grid(const uint32_t* count, const uint32_t* list, const float* qx, const float* qy,
                             const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                             const int32_t* sidx, const float* z, float* qz, hipStream_t s);
hipError_t launch_fixup_scan(const uint32_t* count, const uint32_t* list, const float* qx, const float* qy,
                             const float* x, const float* y, const float* z, int n, float* qz, hipStream_t s);

// ---- learned-R form ----

// Device buffers of the learned-R network (one allocation, see api.hip).
struct MlpDevice {
  float* master;   // [AIDW_MLP_PARAMS] float32 parameters
  float* mom;      // Adam first moment
  float* vel;      // Adam second moment
  uint32_t* w1p;   // [64][14] bf16 pairs
  uint32_t* w2p;   // [64][32]
  uint32_t* w3p;   // [32]
  float* w2r;      // [64][64] float32 of the bf16-rounded W2
  float* w3r;      // [64]
  // MFMA operands of the inference kernels (16-byte aligned): per lane of a wavefront
  // 8 bf16 of W1 per 16-row tile and of W2 per (tile, k-step); float32 b1, b2 and the
  // bf16-rounded W3 as float32.
  uint32_t* w1a;   // [4][64 lanes][4]
  uint32_t* w2a;   // [4][2][64 lanes][4]
  float* b1f;      // [64]
  float* b2f;      // [64]
  float* w3f;      // [64]
};

// perm (may be null): lane t handles query perm[t] and writes its outputs at position t.
// n = the grid's data points (the counts are scaled by nCells / n).
hipError_t launch_features(const GridScalars* gs, const int32_t* cell_start, const float* sx, const float* sy,
                           const float* qx, const float* qy, const uint32_t* perm, int m, int64_t n, float* feat,
                           float* d1sq, hipStream_t s);
hipError_t launch_mlp_repack(const MlpDevice& d, hipStream_t s);
hipError_t launch_mlp_forward(const MlpDevice& d, const float* feat, int m, float* out, hipStream_t s);
// Fused inference front of the learned run, per position t of the order perm (may be null):
// features, the network (MFMA) and the fallback decision in one kernel; flag[t] = 1 marks a
// query that takes the exact kNN.  Rules 2-4 may instead append those queries to list (with
// *count cleared before; both null: flag), a wavefront's queries together in binned order.
// route[q] (may be null) receives the query's route: 0 exact
// kNN, 1 exact kNN after a failed 3 x 3 certificate, 2 certified by the block counts, 3
// certified by the 3 x 3 distances, 4 alpha from the network.
// The certificate's threshold on the sum of the k nearest distances is cert_factor * r_exp (r_exp
// from gs).
hipError_t launch_learned_front(const MlpDevice& d, const GridScalars* gs, const int32_t* cell_start, const float* sx,
                                const float* sy, const float* qx, const float* qy, const uint32_t* perm, int m,
                                int64_t n, const AlphaParams& ap, int rule, double delta, double r_sat_lo,
                                double r_sat_hi, int k, double cert_factor, uint32_t* flag, uint32_t* list,
                                uint32_t* count, float* alpha_f, float* d1sq, float* r_hat_out, uint8_t* route,
                                hipStream_t s);
size_t mlp_batch_scratch_floats(int B);
// grad [AIDW_MLP_PARAMS + 1]: the batch gradient, then the batch's mean squared error.
hipError_t launch_mlp_gradients(const MlpDevice& d, const float* feat, const float* target, const uint32_t* sel, int B,
                                float* scratch, float* grad, hipStream_t s);
hipError_t launch_adam(const MlpDevice& d, const float* grad, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, hipStream_t s);
hipError_t launch_accumulate_loss(const float* grad, float* epoch_loss, int epoch, float scale, hipStream_t s);
// Pair-kernel class keys from a given alpha (alpha == p in 1..8 -> p, else 0) and the identity permutation;
// the coincident-query list as launch_alpha_class.
hipError_t launch_class_keys(const float* alpha_f, int m, uint32_t* keys, uint32_t* vals, const float* d1sq,
                             uint32_t* count, uint32_t* list, hipStream_t s);
// Shuffle keys for training: a 32-bit hash of (seed, epoch, i), and the identity values.
hipError_t launch_shuffle_keys(uint64_t seed, int epoch, int count, uint32_t* keys, uint32_t* vals, hipStream_t s);

}  // namespace aidw

// The grid handle of the C ABI (opaque to callers).
struct aidw_grid {
  int64_t n = 0;
  aidw::GridScalars host{};  // host copy of the device scalars (valid when host_valid)
  bool host_valid = false;
  int64_t cells_alloc = 0;         // cells cell_start is sized for (the budget of a banded build)
  aidw::GridScalars* dev = nullptr;  // device scalars
  int32_t* cell_start = nullptr;   // [ncells + 1]
  float* sx = nullptr;             // [n]
  float* sy = nullptr;             // [n]
  int32_t* sidx = nullptr;         // [n]
  hipStream_t async_stream = nullptr;  // non-null: arrays are stream-ordered allocations on this stream
  bool async = false;
  bool heap = true;  // the handle itself was allocated by the library (else it is the caller's storage)
};


