/*
 * aidw.h -- C ABI of the MI355X (gfx950) implementation of Adaptive IDW
 * interpolation with even-grid kNN search (Mei, Xu & Xu, arXiv 1601.05904).
 *
 * The method has two stages (Section 3.1, Fig. 1):
 *   stage 1  bin the data points into an even grid (Section 4.1.1-4.1.3) and
 *            find, for every interpolated ("query") point, its k nearest data
 *            points by searching rings of cells outward (Section 3.2.4, 4.1.4);
 *            r_obs = mean of the k distances (Eq. 3);
 *   stage 2  R = r_obs / r_exp (Eq. 2, 4), mu = fuzzy membership of R (Eq. 5),
 *            alpha = triangular membership of mu over five levels (Eq. 6), and
 *            z = sum_i z_i d_i^-alpha / sum_i d_i^-alpha over ALL n data points (Eq. 1).
 *
 * Conventions for every entry point
 *   - n = number of data points (x, y, z), m = number of query points (qx, qy).
 *   - Arrays are structure-of-arrays float32 (Section 4.2), DEVICE pointers owned
 *     by the caller, contiguous, naturally aligned.  They must stay valid until
 *     the work queued on the given stream has completed.
 *   - Work is queued on the given HIP stream (0 = the null stream).  Calls
 *     return when the work is queued, except where a call states that it
 *     synchronises the stream.
 *   - Errors are reported by return code only; nothing is thrown and nothing
 *     aborts.  Argument checks run on the host before any GPU work is queued,
 *     so a call that returns AIDW_EINVAL has touched neither the GPU nor the
 *     outputs.  After any other error the output contents are unspecified.
 *     aidw_last_error_detail() gives a message for the last error on the
 *     calling thread.
 *   - Results are deterministic: the same inputs give bitwise identical outputs
 *     (no floating-point atomics; every reduction has a fixed order).
 */
#ifndef AIDW_H
#define AIDW_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AIDW_OK = 0,
  AIDW_EINVAL = -1,       /* invalid argument (null pointer, size, k, parameters)            */
  AIDW_EDEGENERATE = -2,  /* the area A of Eq. 2 resolves to <= 0 (collinear / single point) */
  AIDW_ENOMEM = -3,       /* device allocation failed                                        */
  AIDW_EDEVICE = -4,      /* a HIP runtime call failed                                        */
  AIDW_ENONFINITE = -5,   /* a coordinate is NaN or infinite                                  */
  AIDW_ECAPACITY = -6     /* the grid would exceed AIDW_MAX_CELLS cells, or a size exceeds int32 */
} aidw_status;

#define AIDW_KMAX 64                 /* largest supported k */
#define AIDW_MAX_CELLS (1LL << 28)   /* largest grid (nCol * nRow) */

/*
 * Method parameters.
 *   k          neighbours used for r_obs (Eq. 3); 1 <= k <= min(n, AIDW_KMAX).
 *   alpha[5]   the five distance-decay levels alpha_1..alpha_5 of Eq. 6 (finite, > 0).
 *   r_min, r_max  the bounds of the fuzzy membership of Eq. 5; 0 <= r_min < r_max.
 *              Eq. 5 is applied as printed: the cosine argument is
 *              (pi / r_max) (R - r_min); this equals the symmetric ramp only
 *              when r_min = 0 (the paper's suggested 0 and 2).
 *   area       A of Eq. 2.  <= 0 selects the bounding-box area of data and
 *              queries (the region the grid covers, Section 4.1.1).
 *   cell_width > 0 fixes the grid's cell side; <= 0 selects
 *              sqrt(occupancy * A / n).  (The paper's own choice, the width of
 *              Eq. 2, is occupancy = 0.25.)  The kNN result does not depend on
 *              the cell width: the search stops only when no point outside the
 *              searched block can be nearer than the current k-th neighbour.
 *   occupancy  target mean data points per cell when cell_width <= 0 (> 0).
 */
typedef struct {
  int32_t k;
  double alpha[5];
  double r_min, r_max;
  double area;
  double cell_width;
  double occupancy;
} aidw_params;

/* Fills the defaults: k = 10, alpha = {1,2,3,4,5}, r_min = 0, r_max = 2 (Eq. 5's
 * suggested values), area = 0 (bounding box), cell_width = 0, occupancy = 2. */
void aidw_params_default(aidw_params* p);

/* Opaque even grid over the data points (device-resident, library-owned,
 * immutable after aidw_build_grid; safe for concurrent read-only use). */
typedef struct aidw_grid aidw_grid;

/* Host-side description of a grid (Section 4.1.1).  The grid covers
 * [min_x, min_x + ncol * cell_width) x [min_y, min_y + nrow * cell_width);
 * a point's cell is row * ncol + col with col = (int)((x - min_x) * inv_cell_width)
 * computed in float32 and clamped to [0, ncol - 1] (rows likewise). */
typedef struct {
  int64_t n;                 /* data points binned                                 */
  float min_x, min_y;        /* lower bounds over data and queries                 */
  float max_x, max_y;        /* upper bounds over data and queries                 */
  double area;               /* A used by Eq. 2                                    */
  double r_exp;              /* Eq. 2: 1 / (2 sqrt(n / A))                          */
  double cell_width;         /* cell side                                          */
  float inv_cell_width;      /* float32 reciprocal used for binning                */
  int32_t ncol, nrow;        /* (int)((max - min + cell_width) / cell_width)       */
} aidw_grid_desc;

/*
 * Stage 1, grid build (Section 3.2.1-3.2.3, 4.1.1-4.1.3).
 * Bounds over the n data points AND the m query points (qx, qy may be NULL
 * when m = 0); A, r_exp and the cell width from Eq. 2 and p; every data point
 * binned to its cell; the points sorted by cell with a stable counting sort,
 * so that each cell is one contiguous segment ordered by original index and
 * is described by two integers (Section 3.2.3: head and size, stored here as
 * CSR offsets cell_start[c] .. cell_start[c + 1]).
 * Waits once for the device-computed scalars (an event behind their copy to the
 * host): in occupancy mode (p->cell_width <= 0) after the whole build is queued,
 * to report its status; with an explicit cell width after the bounds (the
 * grid's size depends on them), with the cell keys and the sort's first pass
 * queued before that wait.  On success *out owns device memory until
 * aidw_grid_destroy.
 * Errors: AIDW_EINVAL (null pointers, n < 1, m < 0, sizes > INT32_MAX, invalid p),
 * AIDW_ENONFINITE (a NaN / inf coordinate), AIDW_EDEGENERATE (A <= 0),
 * AIDW_ECAPACITY (more than AIDW_MAX_CELLS cells), AIDW_ENOMEM, AIDW_EDEVICE.
 */
aidw_status aidw_build_grid(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                            const aidw_params* p, hipStream_t stream, aidw_grid** out);

/* Copies the grid's description to *out (host only, no GPU work). */
aidw_status aidw_grid_describe(const aidw_grid* g, aidw_grid_desc* out);

/* The scalars of Eq. 2 and the grid's shape (host only, no GPU work): A, r_exp,
 * the cell width (float64) and nCol, nRow.  Any output pointer may be NULL.
 * Errors: AIDW_EINVAL (g NULL). */
aidw_status aidw_grid_info(const aidw_grid* g, double* area, double* r_exp, double* cell_width, int32_t* ncol,
                           int32_t* nrow);

/* Device pointers of the grid's arrays (library-owned, read-only, valid until
 * aidw_grid_destroy): cell_start [ncol*nrow + 1] int32 CSR offsets;
 * sx, sy [n] float32 and sidx [n] int32 = the data points in cell order.
 * Any output pointer may be NULL. */
aidw_status aidw_grid_arrays(const aidw_grid* g, const int32_t** cell_start, const float** sx, const float** sy,
                             const int32_t** sidx);

/* Copies the grid's arrays (see aidw_grid_arrays) into caller-owned device
 * buffers on `stream`: cell_start [ncol*nrow + 1], sx, sy, sidx [n]; any may be
 * NULL.  Asynchronous. */
aidw_status aidw_grid_copy_arrays(const aidw_grid* g, int32_t* cell_start, float* sx, float* sy, int32_t* sidx,
                                  hipStream_t stream);

/* Frees the grid (waits for the device to finish using it).  NULL is a no-op. */
void aidw_grid_destroy(aidw_grid* g);

/*
 * Stage 1, kNN search (Section 3.2.4, 4.1.4) and Eq. 3.
 * For each query j: the k data points nearest to (qx[j], qy[j]) in the order
 * of (squared distance, data index) -- ties go to the smaller index, so the
 * neighbour set is unique.  Squared distances are formed in float64 from the
 * float32 inputs (exact for coordinates on a 2^-20 lattice in [0, 1)).
 * The search visits rings of cells around the query's cell and stops only when
 * the block searched so far provably contains the k nearest points (the
 * paper's "one more level" rule, the Remark in Section 3.2.4, is not always
 * sufficient and is not used).  The queries are binned to cells first so that
 * the lanes of a wavefront search neighbouring cells.
 * Outputs (device, caller-owned):
 *   r_obs [m]   float32, (1/k) * sum of the k distances, summed in float64 in
 *               ascending order (Eq. 3);
 *   d1sq  [m]   float32 squared distance to the nearest neighbour, or NULL;
 *               exactly 0 iff the query coincides with a data point;
 *   nn_idx [m*k] int32 neighbour indices, row-major, ascending order, or NULL.
 * Errors: AIDW_EINVAL (null grid / pointers, m < 0, k outside [1, min(n, AIDW_KMAX)]),
 * AIDW_ENOMEM, AIDW_EDEVICE.  m = 0 is AIDW_OK and does nothing.
 */
aidw_status aidw_knn(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, float* r_obs,
                     float* d1sq, int32_t* nn_idx, hipStream_t stream);

/*
 * The paper's own stop rule for the grid kNN search (Section 3.2.4 and its
 * Remark), for measuring it: the level grows until the block of
 * (2L + 1) x (2L + 1) cells around the query's cell holds at least k points,
 * one more level is searched, and the k nearest points found in that block are
 * returned in (squared distance, index) order.  This is NOT exact kNN in
 * general: the final block only guarantees the distance to its own edge, so a
 * nearer point just outside it can be missed (the case of the Remark's
 * figure).  The paper pairs the rule with the cell width of Eq. 2 (build the
 * grid with occupancy = 0.25).  Arguments, outputs and errors as aidw_knn.
 */
aidw_status aidw_knn_paper(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, float* r_obs,
                           float* d1sq, int32_t* nn_idx, hipStream_t stream);

/*
 * The nearest-neighbour statistic of Eq. 4 for m queries on grid g:
 *   R[j] = min(r_obs[j] / r_exp, clip),
 * with r_obs[j] the mean distance of query j to its k nearest data points (Eq. 3,
 * computed exactly as aidw_knn does, stored as float32) and r_exp = 1 / (2 sqrt(n / A))
 * the grid's expected distance (Eq. 2).  The quotient is formed in float64 and
 * rounded to float32.  clip > 0 caps R (the learned-R form trains on min(R, 3): alpha is
 * saturated well before that); clip <= 0 or +inf leaves R uncapped.
 * Arguments: qx, qy [m] and R [m] are device pointers (caller-owned).
 * Errors: AIDW_EINVAL (null grid / pointers, m < 0, k outside [1, min(n, AIDW_KMAX)],
 * clip NaN), AIDW_ECAPACITY (m > INT32_MAX), AIDW_ENOMEM, AIDW_EDEVICE.  m = 0 is AIDW_OK.
 */
aidw_status aidw_nn_statistic(const aidw_grid* g, const float* qx, const float* qy, int64_t m, int32_t k, double clip,
                              float* R, hipStream_t stream);

/*
 * Stage 2, adaptive power and weighted interpolation (Eq. 1, 2, 4, 5, 6;
 * Section 3.3, 4.2).
 * For each query j: R = r_obs[j] / r_exp with r_exp = 1 / (2 sqrt(n / A)),
 * mu(R) by Eq. 5 and alpha(mu) by Eq. 6 (float64), then
 *   qz[j] = sum_i z_i d_ij^-alpha / sum_i d_ij^-alpha  over all n data points.
 * Pairs are evaluated in float32 on t = s^2 d^2, with s the smallest power of
 * two such that s^2 d1sq[j] >= 1 (an exact scaling, so t is s^2 times the float32
 * d^2 and the common factor s^-alpha cancels; it keeps w <= ~1): w = rsq(t)^p
 * when alpha is an integer p in 1..8, else w = 2^(-(alpha/2) log2 t); the data are
 * streamed through the chip in tiles shared by every query of a wavefront, the
 * per-tile float32 partial sums are folded into compensated (two-sum) pairs,
 * and the final numerator / denominator are combined in float64.
 * A query with d1sq[j] == 0 coincides with data points and gets the mean z of
 * those points (the limit of Eq. 1).
 * Arguments: r_obs, d1sq as produced by aidw_knn (device, [m]); p->alpha,
 * p->r_min, p->r_max are used and p->area must be > 0 unless a grid g is
 * given, whose area is then used; g (may be NULL) also speeds up the
 * coincident-query fix-up.  alpha_out [m] (may be NULL) receives alpha.
 * Accuracy: |qz - z_exact| <= ~1e-5 * max(|z_exact|, sum_i w_i |z_i| / sum_i w_i).
 * Errors: AIDW_EINVAL, AIDW_ENOMEM, AIDW_EDEVICE.  m = 0 is AIDW_OK.
 */
aidw_status aidw_interpolate(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                             const float* qy, int64_t m, const float* r_obs, const float* d1sq,
                             const aidw_params* p, const aidw_grid* g, float* qz, float* alpha_out,
                             hipStream_t stream);

/*
 * Baselines the paper measures its method against, for comparison runs.
 *
 * aidw_knn_bruteforce: the per-query kNN of the earlier GPU AIDW (Section 3.1):
 * every query scans all n data points and keeps its k best; no grid.  Same
 * definition and outputs as aidw_knn (x, y [n] device arrays; r_obs, d1sq,
 * nn_idx as there), so the two agree bit for bit; the cost is O(n m).
 * Errors: AIDW_EINVAL (pointers, n < 1, m < 0, k outside [1, min(n, AIDW_KMAX)]),
 * AIDW_ECAPACITY (sizes beyond int32).
 *
 * aidw_interpolate_naive: the untiled interpolation kernel (Section 4.2): one
 * query per thread, every thread reads each data point from global memory
 * itself (no sharing of the loaded points across the threads of a wavefront),
 * general alpha form only, one pass over the data.  Arguments, outputs and
 * errors as aidw_interpolate; the sums are those of aidw_interpolate with one
 * data range and integer powers off (aidw_set_interp_config(1, 1, 0)), bit for bit.
 */
aidw_status aidw_knn_bruteforce(const float* x, const float* y, int64_t n, const float* qx, const float* qy,
                                int64_t m, int32_t k, float* r_obs, float* d1sq, int32_t* nn_idx, hipStream_t stream);
aidw_status aidw_interpolate_naive(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                                   const float* qy, int64_t m, const float* r_obs, const float* d1sq,
                                   const aidw_params* p, const aidw_grid* g, float* qz, float* alpha_out,
                                   hipStream_t stream);

/*
 * The whole method (Fig. 1): aidw_build_grid -> aidw_knn -> aidw_interpolate
 * on one stream, with library-owned temporaries.  qz [m] receives the
 * interpolated values; alpha_out [m] and r_obs_out [m] may be NULL.
 * Synchronises the stream once: in occupancy mode at the end (the grid
 * build's status), with an explicit cell width after the bounds (grid sizing).
 * Errors: those of the three stages.
 */
aidw_status aidw_run(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy,
                     int64_t m, const aidw_params* p, float* qz, float* alpha_out, float* r_obs_out,
                     hipStream_t stream);

/*
 * aidw_run for callers that cannot allocate device memory (serving loops or
 * harnesses that forbid hipMalloc): the same method,
 * arguments, outputs and errors as aidw_run, with every temporary (grid, band
 * sort, query bins, r_obs / d1^2, alpha and class keys, padded data, float64
 * partials) taken from one fixed device array of AIDW_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends.  The
 * call makes no hipMalloc / hipFree or other allocation; it reads the grid's
 * status once at the end with a pageable copy (the stream is synchronised), so
 * it cannot be recorded into a HIP graph as it stands.
 *   - The grid is sized by occupancy: params.cell_width must be <= 0
 *     (AIDW_EINVAL otherwise).
 *   - Sizes whose scratch exceeds the array are rejected before any work with
 *     AIDW_ECAPACITY (about 100 bytes per data point plus query: n = m = 2^20
 *     fits).  The data axis of the pair kernel is split only as far as its
 *     float64 partials fit beside the rest.
 *   - Every call on one GPU uses that GPU's single array: calls that overlap on
 *     one GPU (other streams, other host threads) race and give undefined
 *     results.  The array keeps the last call's contents; each call
 *     initialises what it reads.
 */
#define AIDW_NOALLOC_SCRATCH_BYTES (128ull << 20)
aidw_status aidw_run_noalloc(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                             const float* qy, int64_t m, const aidw_params* p, float* qz, float* alpha_out,
                             float* r_obs_out, hipStream_t stream);

/* Per-stage device times of the last aidw_run on the calling thread, recorded
 * with HIP events on the run's stream when timing is enabled. */
typedef struct {
  float grid_ms;        /* bounds, binning, counting sort                  */
  float knn_ms;         /* query binning and kNN search with Eq. 3         */
  float interp_ms;      /* the pair-evaluation kernel(s) of Eq. 1          */
  float finish_ms;      /* split combine and coincident-query fix-up       */
  int32_t interp_q;     /* queries per lane used by the pair kernel        */
  int32_t interp_split; /* data-axis splits used by the pair kernel        */
} aidw_timing;

/* Enables (1) or disables (0) per-stage timing for aidw_run on the calling
 * thread.  Timing adds events only; the kernels are unchanged. */
aidw_status aidw_set_timing(int enable);

/* Waits for the last timed aidw_run of the calling thread and reports its
 * stage times.  AIDW_EINVAL if timing was off or no run was timed. */
aidw_status aidw_last_timing(aidw_timing* out);

/* Overrides the pair kernel's launch shape for later calls on the calling
 * thread: q = queries per lane (1, 2, 4 or 8), split = data-axis splits
 * (>= 1); 0 for either restores the built-in choice.  integer_powers = 0
 * evaluates every query with the general w = 2^(-(alpha/2) log2 t); 1 or -1
 * (the default) lets queries whose alpha equals an integer level p in 1..8
 * use w = rsq(t)^p (one transcendental instead of two). */
aidw_status aidw_set_interp_config(int32_t q, int32_t split, int32_t integer_powers);

/*
 * kNN kernel choice for later aidw_knn / aidw_run calls on the calling thread
 * (Section 3.2.4 and 4.1.4: the ring search over the grid): lds_window = 0
 * (default) reads every candidate through the caches; 1 stages, per workgroup
 * of 256 binned queries, the cells within two of theirs (when they fit 2048
 * points) in LDS and reads the candidates of those cells from there.  Both give
 * the same index sets, r_obs and d1^2 bit for bit; the choice applies to query
 * sets of 2^17 or more (smaller ones take the four-lanes-per-query kernel).
 * Errors: AIDW_EINVAL for any other value.
 */
aidw_status aidw_set_knn_config(int32_t lds_window);

/* ---------------------------------------------------------------------------
 * Learned-R form.  A small network predicts the nearest-neighbour statistic R
 * of Eq. 4 from the grid's occupancy around each query (inputs: the counts of
 * the 5 x 5 cells around the query's cell relative to the mean occupancy, and
 * the query's offset inside its cell), so that most queries skip the kNN search
 * of Section 3.2.4.  Exact kNN stays the fallback wherever the prediction could
 * change alpha (Eq. 5, 6).  27 -> 64 -> 64 -> 1, GELU (tanh form), bf16 weights
 * and activations as operands, float32 accumulation, trained on the GPU by the
 * library's own forward / backward / Adam kernels.
 * Parameter vector (float32, AIDW_MLP_PARAMS entries): W1 [64 x 27 row-major],
 * b1 [64], W2 [64 x 64], b2 [64], W3 [64], b3 [1].
 * ------------------------------------------------------------------------- */
#define AIDW_MLP_INPUTS 27
#define AIDW_MLP_PARAMS 6017

typedef struct aidw_mlp aidw_mlp; /* opaque, device-resident, library-owned */

typedef enum {
  AIDW_FALLBACK_LITERAL = 0,     /* kNN when |R_hat - r_min| < delta or |R_hat - r_max| < delta; else alpha(R_hat) */
  AIDW_FALLBACK_ALPHA_EXACT = 1, /* skip kNN only when R_hat is delta beyond the points where alpha
                                    saturates (mu = 0.1 / 0.9 in Eq. 6); skipped queries get alpha_1 / alpha_5 */
  AIDW_FALLBACK_CERTIFIED = 2,   /* skip kNN only when a lower bound of Eq. 3's r_obs proves mu > 0.9
                                    (alpha = alpha_5 by Eq. 6); the bound comes from the point counts of the
                                    1, 3 x 3 and 5 x 5 cell blocks around the query and the exact distances of
                                    the 3 x 3 block's points.  Every query gets the alpha of the exact path; the
                                    network is not evaluated (r_hat_out receives NaN); delta is checked, unused */
  AIDW_FALLBACK_CERTIFIED_THEN_ALPHA_EXACT = 3, /* skip when certified as in 2, else apply rule 1; the network runs
                                                   only on the queries the block counts do not certify (r_hat_out:
                                                   NaN for the others) */
  AIDW_FALLBACK_NETWORK_GATED_CERTIFICATE = 4   /* skip only when certified as in 2 (every alpha is the exact
                                                   path's); the network decides which queries the 3 x 3 distance
                                                   certificate is tried on: those the block counts do not already
                                                   certify and whose r_hat >= (R where mu = 0.9) - delta; the others
                                                   go to the exact kNN without that scan.  The network runs only on
                                                   the queries the counts leave open whose 3 x 3 block holds at
                                                   most 8 k + 16 points (r_hat_out: NaN for the others) */
} aidw_fallback_rule;

/* New network with weights drawn from `seed` (uniform in +-sqrt(6 / fan_in),
 * biases 0) for grids of the given occupancy (> 0; points per cell).  Errors:
 * AIDW_EINVAL, AIDW_ENOMEM, AIDW_EDEVICE. */
aidw_status aidw_mlp_create(uint64_t seed, double occupancy, aidw_mlp** out);
void aidw_mlp_destroy(aidw_mlp* mlp);

/* Copies the float32 parameters from / to host memory (AIDW_MLP_PARAMS floats).
 * set_params also clears the optimiser state.  Both synchronise the device. */
aidw_status aidw_mlp_set_params(aidw_mlp* mlp, const float* host_params);
aidw_status aidw_mlp_get_params(const aidw_mlp* mlp, float* host_params);

/* Checkpoint: a versioned binary file holding the parameters, the optimiser
 * state, the step count and the occupancy.  Errors: AIDW_EINVAL (bad file). */
aidw_status aidw_mlp_save(const aidw_mlp* mlp, const char* path);
aidw_status aidw_mlp_load(const char* path, aidw_mlp** out);

/* Occupancy the network was created for (0 on a NULL handle). */
double aidw_mlp_occupancy(const aidw_mlp* mlp);

/* Network inputs of m queries on grid g: feat [m x 27] float32 (device,
 * row-major); d1sq [m] (device, may be NULL) receives the squared distance to
 * the nearest data point when it lies in the 3 x 3 cells around the query and
 * nearer than their outer edge, else a lower bound of it (exactly 0 iff the
 * query coincides with a data point). */
aidw_status aidw_features(const aidw_grid* g, const float* qx, const float* qy, int64_t m, float* feat, float* d1sq,
                          hipStream_t stream);

/* r_hat [m] = network output for feat [m x 27] (device pointers). */
aidw_status aidw_mlp_forward(const aidw_mlp* mlp, const float* feat, int64_t m, float* r_hat, hipStream_t stream);

/* Gradient of the mean squared error over a batch (feat [batch x 27], target
 * [batch], device) with respect to the parameter vector: grad [AIDW_MLP_PARAMS + 1]
 * (device), the last entry being the loss.  No update is made. */
aidw_status aidw_mlp_gradients(const aidw_mlp* mlp, const float* feat, const float* target, int64_t batch,
                               float* grad, hipStream_t stream);

/* Trains on `count` (feature, target) pairs (device): `epochs` passes of Adam
 * (beta 0.9 / 0.999, eps 1e-8, learning rate lr) over minibatches of `batch`
 * pairs, reshuffled each epoch from `seed`.  epoch_loss (host, [epochs], may be
 * NULL) receives the mean batch loss of each epoch (this synchronises). */
aidw_status aidw_mlp_train(aidw_mlp* mlp, const float* feat, const float* target, int64_t count, int32_t epochs,
                           int32_t batch, float lr, uint64_t seed, float* epoch_loss, hipStream_t stream);

/* The whole method with the learned R: grid build, features, network, exact
 * kNN on the fallback queries only (rule, delta >= 0), alpha, and the weighted
 * interpolation of aidw_interpolate for every query.  p->cell_width must be
 * <= 0 and p->occupancy must equal the network's.  r_hat_out [m] (may be NULL)
 * receives the predictions; *fallback_count (host, may be NULL) the number of
 * queries that took the exact kNN path.  Synchronises the stream once at the
 * end (the grid build's status, and the count).  Timing as aidw_run (the kNN
 * stage time covers features, network and the fallback search). */
aidw_status aidw_run_learned(const float* x, const float* y, const float* z, int64_t n, const float* qx,
                             const float* qy, int64_t m, const aidw_params* p, const aidw_mlp* mlp, int32_t rule,
                             double delta, float* qz, float* alpha_out, float* r_hat_out, int64_t* fallback_count,
                             hipStream_t stream);

/* The learned form's decision for every query, without the kNN search or the
 * interpolation (for inspecting a rule and a network): the grid build and the fused
 * front of aidw_run_learned.  route_out [m] (device, uint8) receives the query's route:
 *   0  exact kNN
 *   1  exact kNN after the 3 x 3 distance certificate was tried and failed
 *   2  skipped: alpha = alpha_5 certified by the block counts
 *   3  skipped: alpha = alpha_5 certified by the 3 x 3 distances
 *   4  skipped: alpha set from the network's prediction (rules 0, 1, 3)
 * r_hat_out [m] (may be NULL) as for aidw_run_learned.  Arguments and errors as
 * aidw_run_learned; synchronises the stream once at the end. */
aidw_status aidw_learned_routes(const float* x, const float* y, int64_t n, const float* qx, const float* qy,
                                int64_t m, const aidw_params* p, const aidw_mlp* mlp, int32_t rule, double delta,
                                uint8_t* route_out, float* r_hat_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched form.  Many independent interpolation problems ("jobs") of uneven
 * size run as one pipeline on one stream: each stage of the method (bounds and
 * grid scalars, counting sort, query binning, kNN with Eq. 3, Eq. 4-6) is one
 * launch over all jobs, and the pair evaluation of Eq. 1 is ONE persistent
 * launch whose workgroups take work items (job, block of queries, range of
 * data points) from a list ordered by decreasing cost until it is exhausted.
 * Every item writes its own float64 partial sums and a last pass adds a
 * query's partials in a fixed order, so results are bitwise reproducible.
 * Each job's outputs are those aidw_run gives for the job alone (bitwise when
 * aidw_run uses the same pair-kernel shape: q, and split = the job's number of
 * data ranges, see split_points).
 *
 * A plan fixes the jobs (pointers and sizes) and the launch shape once: it
 * checks everything on the host, allocates one device workspace and uploads
 * the job table.  Running a plan reads the current contents of the jobs'
 * input arrays, queues the whole pipeline and returns: it allocates nothing
 * and never waits for the device, so it can be captured in a HIP graph (the
 * plan does this itself with use_graph) and replayed.  In the batched form a
 * job's grid has a cell budget fixed by n (about 2 n / occupancy cells); when
 * the bounds would need more cells the cell side is widened, which changes
 * only the search cost, never a result.
 * ------------------------------------------------------------------------- */

/* One job.  Inputs as for aidw_run (device pointers, caller-owned, valid while
 * the plan is in use); params.k <= min(n, AIDW_KMAX); cell_width > 0 is a
 * lower bound here (see above).  qz [m] receives the interpolated values;
 * alpha_out [m] and r_obs_out [m] may be NULL.  m = 0 is allowed. */
typedef struct {
  const float* x;
  const float* y;
  const float* z;
  int64_t n;
  const float* qx;
  const float* qy;
  int64_t m;
  aidw_params params;
  float* qz;
  float* alpha_out;
  float* r_obs_out;
} aidw_job;

/* Launch shape of a plan (what the autotuner searches over).
 *   q               queries per lane in the pair kernel: 1 or 2.
 *   split_points    data points per work item, rounded up to a multiple of 8;
 *                   0 = a job's whole data set (one range per query block).
 *   workers_per_cu  persistent pair-kernel workgroups per compute unit, 1..32.
 *   integer_powers  1: a block of queries whose alpha is the same integer p in
 *                   1..8 uses w = rsq(t)^p; 0: every query the general form.
 *   use_graph       1: the first aidw_batch_run captures the pipeline into a
 *                   HIP graph (it needs a created stream, not the null stream)
 *                   and every run launches that graph. */
typedef struct {
  int32_t q;
  int32_t split_points;
  int32_t workers_per_cu;
  int32_t integer_powers;
  int32_t use_graph;
} aidw_batch_config;

/* Defaults: q = 1, split_points = 0, workers_per_cu = 8, integer_powers = 1, use_graph = 0. */
void aidw_batch_config_default(aidw_batch_config* c);

/* Opaque plan (library-owned). */
typedef struct aidw_batch aidw_batch;

/* Checks the jobs and the config on the host, allocates the device workspace
 * and uploads the job table (synchronous).  cfg may be NULL (defaults).
 * Errors: AIDW_EINVAL (njobs < 1, a job's pointers, sizes, k or params, the
 * config), AIDW_ECAPACITY (totals beyond int32 indexing), AIDW_ENOMEM,
 * AIDW_EDEVICE.  On success *out owns the workspace until aidw_batch_destroy. */
aidw_status aidw_batch_create(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* cfg, aidw_batch** out);

/* Queues the pipeline for all jobs on `stream` (or launches its graph).
 * Asynchronous; overlapping runs of one plan race on its workspace.  A job
 * whose input is non-finite or spans no area gets NaN outputs and its status
 * is reported by aidw_batch_job_status; the other jobs are unaffected.
 * Errors: AIDW_EINVAL (NULL plan; graph mode on the null stream), AIDW_EDEVICE. */
aidw_status aidw_batch_run(aidw_batch* b, hipStream_t stream);

/* Waits for `stream` and reports each job's status of the last run into
 * status [njobs] (host array, may be NULL): AIDW_OK, AIDW_ENONFINITE or
 * AIDW_EDEGENERATE.  Returns AIDW_OK if every job succeeded, else the status
 * of the first job that failed. */
aidw_status aidw_batch_job_status(aidw_batch* b, int32_t* status, hipStream_t stream);

/* Sizes of a plan (host only). */
typedef struct {
  int32_t njobs;
  int64_t total_data;       /* sum of n                              */
  int64_t total_queries;    /* sum of m                              */
  double total_pairs;       /* sum of n * m: pair evaluations of Eq. 1 */
  int64_t total_cells;      /* sum of the jobs' cell budgets         */
  int32_t work_items;       /* items of the persistent pair launch   */
  int32_t workers;          /* its workgroups                        */
  int32_t kmax;             /* register k-list length of the kNN kernel */
  int64_t workspace_bytes;  /* device workspace                      */
  aidw_batch_config config;
} aidw_batch_desc;

aidw_status aidw_batch_describe(const aidw_batch* b, aidw_batch_desc* out);

/* Per-stage device times of a plan's runs, recorded with HIP events when
 * enabled (a timed run is launched directly, not through the graph). */
typedef struct {
  float grid_ms;    /* gather, bounds, grid scalars, counting sort, CSR     */
  float knn_ms;     /* query binning, kNN + Eq. 3, Eq. 4-6, class ordering  */
  float interp_ms;  /* the persistent pair kernel of Eq. 1                  */
  float finish_ms;  /* combine, coincident-query fix-up, outputs            */
} aidw_batch_timing;

aidw_status aidw_batch_set_timing(aidw_batch* b, int32_t enable);
/* Waits for the last timed run of the plan and reports its stage times. */
aidw_status aidw_batch_last_timing(aidw_batch* b, aidw_batch_timing* out);

/* Frees the plan and its workspace (waits for the device).  NULL is a no-op. */
void aidw_batch_destroy(aidw_batch* b);

/* One-shot: create a plan (cfg may be NULL; use_graph is ignored), run it,
 * report per-job status into status [njobs] (may be NULL) and destroy it.
 * Synchronises the stream.  Returns as aidw_batch_job_status. */
aidw_status aidw_run_batch(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* cfg, int32_t* status,
                           hipStream_t stream);

/* Autotuner kernel: for each candidate config, builds a plan for the jobs, runs
 * it once (warm-up, graph capture) and then `reps` times, and stores the mean
 * device time per run in ms_out [ncandidates].  The jobs' outputs are written
 * by every run.  Synchronises the stream.  Errors: those of aidw_batch_create
 * and aidw_batch_run for the failing candidate. */
aidw_status aidw_batch_tune(const aidw_job* jobs, int32_t njobs, const aidw_batch_config* candidates,
                            int32_t ncandidates, int32_t reps, float* ms_out, hipStream_t stream);

/* Temporaries of the calls above come from a cache of device blocks that the
 * library keeps between calls (reused in stream order, or after an event wait
 * on another stream).  This waits for the current device and frees the cached
 * blocks not in use on it.  Errors: AIDW_EDEVICE. */
aidw_status aidw_release_cached_memory(void);

/* Static text for a status code. */
const char* aidw_status_string(aidw_status st);

/* Message for the last error on the calling thread ("" if none). */
const char* aidw_last_error_detail(void);

/* Library version string. */
const char* aidw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AIDW_H */
