/*
 * Plain FP64 CPU oracle for Adaptive IDW with kNN-based adaptive power
 * (Mei, Xu & Xu, "Improving GPU-accelerated Adaptive IDW Interpolation
 * Algorithm Using Fast kNN Search", arXiv 1601.05904).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP library is checked against.  It is called only by
 * the tests, by the smoke check and by the benchmark's CPU-baseline leg; the
 * library never links, loads or calls it, and the two share no source.
 *
 * Precision: every quantity the method defines is computed in double.  The
 * inputs are the FP32 coordinates / values the GPU sees, promoted exactly.
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp (no contraction,
 * so every product and sum below is one IEEE operation in the written order).
 *
 * Parity status of each function (see the tests for the pins):
 *   oracle_bounds, oracle_grid_params, oracle_cell_index  pinned (closed forms, boundary cases)
 *   oracle_knn, oracle_robs                               pinned (brute force by full sort, lattice closed form, Poisson statistic)
 *   oracle_alpha                                          pinned (knot values, closed form of Eq. 5-6 for alpha = 1..5)
 *   oracle_idw                                            pinned (coincidence, constant field, hull, symmetric closed forms, hand-derived worked examples)
 *   oracle_aidw                                           composition of the above
 *   oracle_features                                       pinned (counts of a constructed grid, window clipping, offsets)
 *   oracle_knn_paper                                      pinned (a constructed miss of the "+1 level" rule, single-cell
 *                                                         grid = brute force, block and distance invariants)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_EDEGENERATE (-2)
#define ORACLE_ECAPACITY (-6)
#define ORACLE_MAX_CELLS (1LL << 28)

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/*
 * Section 4.1.1 (creating the even grid): the grid covers the planar region
 * holding all data points AND all interpolated points, so the bounds are the
 * min / max of x and y over both sets.
 * out = {minX, minY, maxX, maxY}.
 */
void oracle_bounds(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                   double out[4]) {
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    if (x[i] < mnx) mnx = x[i];
    if (x[i] > mxx) mxx = x[i];
    if (y[i] < mny) mny = y[i];
    if (y[i] > mxy) mxy = y[i];
  }
  for (int64_t j = 0; j < m; ++j) {
    if (qx[j] < mnx) mnx = qx[j];
    if (qx[j] > mxx) mxx = qx[j];
    if (qy[j] < mny) mny = qy[j];
    if (qy[j] > mxy) mxy = qy[j];
  }
  out[0] = mnx;
  out[1] = mny;
  out[2] = mxx;
  out[3] = mxy;
}

/*
 * Grid scalars.
 *  - A, "the area of the study region" of Eq. 2: the bounding-box area of
 *    data and queries (the region the grid covers), unless the caller gives
 *    one (area_in > 0).
 *  - r_exp = 1 / (2 sqrt(n / A))  (Eq. 2, n = number of DATA points).
 *  - cell width: given (cw_in > 0), else sqrt(occ * A / n), i.e. a target
 *    of occ data points per cell (the paper ties the width to Eq. 2, which
 *    is the occ = 1/4 case).
 *  - inv_cw: the single-precision reciprocal used to bin points.
 *  - nCol = (int)((maxX - minX + cw) / cw), nRow likewise (Section 4.1.1).
 * out_d = {area, r_exp, cw}.  Returns ORACLE_EDEGENERATE when the area is
 * not positive, ORACLE_ECAPACITY when the grid would exceed 2^28 cells.
 */
int oracle_grid_params(const double bounds[4], int64_t n, double area_in, double cw_in, double occ, double out_d[3],
                       float* inv_cw, int32_t* ncol, int32_t* nrow) {
  if (n <= 0) return ORACLE_EINVAL;
  double W = bounds[2] - bounds[0];
  double H = bounds[3] - bounds[1];
  double area = area_in > 0 ? area_in : W * H;
  if (!(area > 0) || !isfinite(area)) return ORACLE_EDEGENERATE;
  double r_exp = 1.0 / (2.0 * sqrt((double)n / area));
  double cw = cw_in > 0 ? cw_in : sqrt(occ * area / (double)n);
  if (!(cw > 0) || !isfinite(cw)) return ORACLE_EINVAL;
  double fc = (W + cw) / cw;
  double fr = (H + cw) / cw;
  if (!(fc < (double)ORACLE_MAX_CELLS) || !(fr < (double)ORACLE_MAX_CELLS)) return ORACLE_ECAPACITY;
  int32_t c = (int32_t)fc, r = (int32_t)fr;
  if ((int64_t)c * (int64_t)r > ORACLE_MAX_CELLS) return ORACLE_ECAPACITY;
  out_d[0] = area;
  out_d[1] = r_exp;
  out_d[2] = cw;
  *inv_cw = (float)(1.0 / cw);
  *ncol = c;
  *nrow = r;
  return ORACLE_OK;
}

/*
 * Section 4.1.2 (distributing data points into cells): the column is the
 * offset from minX divided by the cell width (done in single precision as
 * (x - minX) * inv_cw, then truncated), likewise the row; the flat index is
 * row * nCol + col.  Indices are clamped to the last column / row so that a
 * point on the upper bound lands inside the grid.
 */
void oracle_cell_index(const float* x, const float* y, int64_t n, float minX, float minY, float inv_cw, int32_t ncol,
                       int32_t nrow, int32_t* cell) {
  for (int64_t i = 0; i < n; ++i) {
    float tx = (x[i] - minX) * inv_cw;
    float ty = (y[i] - minY) * inv_cw;
    int32_t col = (int32_t)tx;
    int32_t row = (int32_t)ty;
    if (col > ncol - 1) col = ncol - 1;
    if (row > nrow - 1) row = nrow - 1;
    if (col < 0) col = 0;
    if (row < 0) row = 0;
    cell[i] = row * ncol + col;
  }
}

/* squared Euclidean distance of data point i to query j, in double (Section 4.1.4: compare squared distances). */
static double dist2(float ax, float ay, float bx, float by) {
  double dx = (double)ax - (double)bx;
  double dy = (double)ay - (double)by;
  return dx * dx + dy * dy;
}

/* (d2, index) lexicographic order: ties in distance are broken by the smaller index. */
static int key_less(double da, int32_t ia, double db, int32_t ib) { return da < db || (da == db && ia < ib); }

/*
 * Brute-force kNN (Section 2.3): all n distances, ordered increasingly, the
 * first k kept.  The ordering is by (squared distance, index).  Selecting
 * the k smallest is done with a k-long list kept sorted by insertion (the
 * per-query procedure of Section 3.1 with the list initialised to +inf); the
 * result is exactly the first k entries of a full sort.
 * Outputs (row-major m x k): idx = data indices, d2 = squared distances, ascending.
 */
void oracle_knn(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m, int32_t k,
                int32_t* idx, double* d2) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < m; ++j) {
    double* bd = d2 + j * (int64_t)k;
    int32_t* bi = idx + j * (int64_t)k;
    for (int32_t s = 0; s < k; ++s) {
      bd[s] = INFINITY;
      bi[s] = INT32_MAX;
    }
    for (int64_t i = 0; i < n; ++i) {
      double d = dist2(x[i], y[i], qx[j], qy[j]);
      if (!key_less(d, (int32_t)i, bd[k - 1], bi[k - 1])) continue;
      int32_t s = k - 1;
      while (s > 0 && key_less(d, (int32_t)i, bd[s - 1], bi[s - 1])) {
        bd[s] = bd[s - 1];
        bi[s] = bi[s - 1];
        --s;
      }
      bd[s] = d;
      bi[s] = (int32_t)i;
    }
  }
}

/*
 * The paper's grid kNN search as printed (Section 3.2.4 and its Remark; Fig. 3, 4):
 * the "level" L block is the (2L + 1) x (2L + 1) cells centred on the query's cell
 * (clipped to the grid).  Starting at L = 0 the level grows until the block holds
 * at least k data points (the worked example expands at 14 < 15, read as count >= k
 * to stop); the search then takes one more level, and the k nearest data points
 * among those in that final block, ordered by (squared distance, index), are the
 * result.  Binning as oracle_cell_index.  This is NOT exact kNN in general: the
 * final block only guarantees the distance to its own edge (the failure class the
 * Remark's Fig. 4 illustrates); it is kept to measure that rule.
 * Outputs as oracle_knn (m x k, ascending); idx = INT32_MAX / d2 = +inf if fewer than k.
 */
void oracle_knn_paper(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                      int32_t k, float minX, float minY, float inv_cw, int32_t ncol, int32_t nrow, int32_t* idx,
                      double* d2) {
  int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* qcell = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!cell || !qcell) {
    free(cell);
    free(qcell);
    return;
  }
  oracle_cell_index(x, y, n, minX, minY, inv_cw, ncol, nrow, cell);
  oracle_cell_index(qx, qy, m, minX, minY, inv_cw, ncol, nrow, qcell);
  const int32_t maxlev = ncol > nrow ? ncol : nrow;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < m; ++j) {
    const int32_t c0 = qcell[j] % ncol, r0 = qcell[j] / ncol;
    int32_t L = 0;
    for (;; ++L) {  /* smallest level whose block holds >= k points (the whole grid always does) */
      int64_t count = 0;
      for (int64_t i = 0; i < n; ++i) {
        const int32_t c = cell[i] % ncol, r = cell[i] / ncol;
        if (abs(c - c0) <= L && abs(r - r0) <= L) ++count;
      }
      if (count >= k || L >= maxlev) break;
    }
    const int32_t Lf = L + 1; /* the Remark: one more level */
    double* bd = d2 + j * (int64_t)k;
    int32_t* bi = idx + j * (int64_t)k;
    for (int32_t s = 0; s < k; ++s) {
      bd[s] = INFINITY;
      bi[s] = INT32_MAX;
    }
    for (int64_t i = 0; i < n; ++i) {
      const int32_t c = cell[i] % ncol, r = cell[i] / ncol;
      if (abs(c - c0) > Lf || abs(r - r0) > Lf) continue;
      const double d = dist2(x[i], y[i], qx[j], qy[j]);
      if (!key_less(d, (int32_t)i, bd[k - 1], bi[k - 1])) continue;
      int32_t s = k - 1;
      while (s > 0 && key_less(d, (int32_t)i, bd[s - 1], bi[s - 1])) {
        bd[s] = bd[s - 1];
        bi[s] = bi[s - 1];
        --s;
      }
      bd[s] = d;
      bi[s] = (int32_t)i;
    }
  }
  free(cell);
  free(qcell);
}

/* Eq. 3: r_obs = (1/k) * sum of the k nearest-neighbour distances (summed in ascending order). */
void oracle_robs(const double* d2, int64_t m, int32_t k, double* r_obs) {
  for (int64_t j = 0; j < m; ++j) {
    double s = 0.0;
    for (int32_t t = 0; t < k; ++t) s += sqrt(d2[j * (int64_t)k + t]);
    r_obs[j] = s / (double)k;
  }
}

/* Eq. 5, literally: the cosine ramp uses pi / R_max (not pi / (R_max - R_min)). */
static double membership(double R, double rmin, double rmax) {
  if (R <= rmin) return 0.0;
  if (R >= rmax) return 1.0;
  return 0.5 - 0.5 * cos((M_PI / rmax) * (R - rmin));
}

/* Eq. 6: triangular membership over the five levels alpha_1..alpha_5 at mu = 0.1, 0.3, 0.5, 0.7, 0.9. */
static double alpha_of_mu(double mu, const double a[5]) {
  if (mu <= 0.1) return a[0];
  if (mu <= 0.3) return a[0] * (1.0 - 5.0 * (mu - 0.1)) + 5.0 * a[1] * (mu - 0.1);
  if (mu <= 0.5) return 5.0 * a[2] * (mu - 0.3) + a[1] * (1.0 - 5.0 * (mu - 0.3));
  if (mu <= 0.7) return a[2] * (1.0 - 5.0 * (mu - 0.5)) + 5.0 * a[3] * (mu - 0.5);
  if (mu <= 0.9) return 5.0 * a[4] * (mu - 0.7) + a[3] * (1.0 - 5.0 * (mu - 0.7));
  return a[4];
}

/* Eq. 4 -> 5 -> 6 for each query: R = r_obs / r_exp, mu(R), alpha(mu).  Any of R / mu may be NULL. */
void oracle_alpha(const double* r_obs, int64_t m, double r_exp, double rmin, double rmax, const double alpha5[5],
                  double* R_out, double* mu_out, double* alpha_out) {
  for (int64_t j = 0; j < m; ++j) {
    double R = r_obs[j] / r_exp;
    double mu = membership(R, rmin, rmax);
    if (R_out) R_out[j] = R;
    if (mu_out) mu_out[j] = mu;
    alpha_out[j] = alpha_of_mu(mu, alpha5);
  }
}

/*
 * Eq. 1 over ALL n data points with the per-query power alpha[j]:
 *   z = sum_i z_i d_i^-alpha / sum_i d_i^-alpha,   d_i^-alpha = (d_i^2)^(-alpha/2),
 * summed in index order.  A query that coincides with data points (d = 0)
 * takes the mean z of those points (the limit of Eq. 1 as the query
 * approaches them; exactly z_i for a single one).
 * s_norm[j] (may be NULL) = sum_i w_i |z_i| / sum_i w_i, the scale used by the
 * relative-error metric (|z| of the coincident mean for coincident queries).
 */
void oracle_idw(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy, int64_t m,
                const double* alpha, double* zq, double* s_norm) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j = 0; j < m; ++j) {
    int64_t ncoin = 0;
    double zc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      if (dist2(x[i], y[i], qx[j], qy[j]) == 0.0) {
        zc += (double)z[i];
        ++ncoin;
      }
    }
    if (ncoin > 0) {
      zq[j] = zc / (double)ncoin;
      if (s_norm) s_norm[j] = fabs(zq[j]);
      continue;
    }
    double e = -0.5 * alpha[j];
    double num = 0.0, den = 0.0, absnum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double w = pow(dist2(x[i], y[i], qx[j], qy[j]), e);
      num += w * (double)z[i];
      den += w;
      absnum += w * fabs((double)z[i]);
    }
    zq[j] = num / den;
    if (s_norm) s_norm[j] = absnum / den;
  }
}

/*
 * The whole method on a selection of the queries (Fig. 1's two stages):
 * bounds over data and ALL m queries -> grid scalars (A, r_exp) -> kNN of each
 * selected query -> r_obs -> R, mu, alpha -> weighted mean.  qsel (length
 * msel) lists the selected query indices; NULL selects all (msel = m).
 * Outputs have msel entries (knn_idx / knn_d2: msel x k; any output may be NULL
 * except zq).  scal_out = {area, r_exp, cw} (may be NULL).
 */
int oracle_aidw(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy, int64_t m,
                const int64_t* qsel, int64_t msel, int32_t k, const double alpha5[5], double rmin, double rmax,
                double area_in, double cw_in, double occ, double* zq, double* alpha_out, double* r_obs_out,
                double* R_out, double* s_norm, int32_t* knn_idx, double* knn_d2, double* scal_out) {
  if (n <= 0 || k <= 0 || k > n || msel < 0) return ORACLE_EINVAL;
  double b[4], sc[3];
  float inv;
  int32_t nc, nr;
  oracle_bounds(x, y, n, qx, qy, m, b);
  int st = oracle_grid_params(b, n, area_in, cw_in, occ, sc, &inv, &nc, &nr);
  if (st != ORACLE_OK) return st;
  if (scal_out) memcpy(scal_out, sc, sizeof(sc));
  float* sx = (float*)malloc(sizeof(float) * (size_t)(msel > 0 ? msel : 1));
  float* sy = (float*)malloc(sizeof(float) * (size_t)(msel > 0 ? msel : 1));
  int32_t* ki = (int32_t*)malloc(sizeof(int32_t) * (size_t)(msel > 0 ? msel : 1) * (size_t)k);
  double* kd = (double*)malloc(sizeof(double) * (size_t)(msel > 0 ? msel : 1) * (size_t)k);
  double* ro = (double*)malloc(sizeof(double) * (size_t)(msel > 0 ? msel : 1));
  double* al = (double*)malloc(sizeof(double) * (size_t)(msel > 0 ? msel : 1));
  if (!sx || !sy || !ki || !kd || !ro || !al) {
    free(sx); free(sy); free(ki); free(kd); free(ro); free(al);
    return ORACLE_EINVAL;
  }
  for (int64_t t = 0; t < msel; ++t) {
    int64_t j = qsel ? qsel[t] : t;
    sx[t] = qx[j];
    sy[t] = qy[j];
  }
  oracle_knn(x, y, n, sx, sy, msel, k, ki, kd);
  oracle_robs(kd, msel, k, ro);
  oracle_alpha(ro, msel, sc[1], rmin, rmax, alpha5, R_out, NULL, al);
  oracle_idw(x, y, z, n, sx, sy, msel, al, zq, s_norm);
  if (alpha_out) memcpy(alpha_out, al, sizeof(double) * (size_t)msel);
  if (r_obs_out) memcpy(r_obs_out, ro, sizeof(double) * (size_t)msel);
  if (knn_idx) memcpy(knn_idx, ki, sizeof(int32_t) * (size_t)msel * (size_t)k);
  if (knn_d2) memcpy(knn_d2, kd, sizeof(double) * (size_t)msel * (size_t)k);
  free(sx); free(sy); free(ki); free(kd); free(ro); free(al);
  return ORACLE_OK;
}

/*
 * Learned-R input features of each query (the surrogate that predicts R of Eq. 4
 * from the grid's occupancy instead of a kNN search):
 *   feat[0..24]  number of data points in each cell of the 5 x 5 block of cells
 *                centred on the query's cell (row offset -2..2 outer, column
 *                offset -2..2 inner; 0 for cells outside the grid), times
 *                inv_occ = nCells / n (i.e. relative to the mean occupancy);
 *   feat[25..26] the query's offset inside its cell along x and y, in [0, 1),
 *                from the same single-precision binning as the data points.
 * Counts come from a histogram of oracle_cell_index over the data.
 */
void oracle_features(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                     float minX, float minY, float inv_cw, int32_t ncol, int32_t nrow, float* feat) {
  int64_t ncells = (int64_t)ncol * nrow;
  int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t* count = (int64_t*)calloc((size_t)ncells, sizeof(int64_t));
  if (!cell || !count) {
    free(cell);
    free(count);
    return;
  }
  oracle_cell_index(x, y, n, minX, minY, inv_cw, ncol, nrow, cell);
  for (int64_t i = 0; i < n; ++i) count[cell[i]] += 1;
  double inv_occ = (double)ncells / (double)n;
  for (int64_t j = 0; j < m; ++j) {
    float tx = (qx[j] - minX) * inv_cw;
    float ty = (qy[j] - minY) * inv_cw;
    int32_t c0 = tx < 0.0f ? 0 : (int32_t)tx;
    int32_t r0 = ty < 0.0f ? 0 : (int32_t)ty;
    if (c0 > ncol - 1) c0 = ncol - 1;
    if (r0 > nrow - 1) r0 = nrow - 1;
    float* f = feat + j * 27;
    for (int dr = -2; dr <= 2; ++dr) {
      for (int dc = -2; dc <= 2; ++dc) {
        int32_t r = r0 + dr, c = c0 + dc;
        int64_t cnt = (r >= 0 && r < nrow && c >= 0 && c < ncol) ? count[(int64_t)r * ncol + c] : 0;
        f[(dr + 2) * 5 + (dc + 2)] = (float)((double)cnt * inv_occ);
      }
    }
    f[25] = tx - (float)c0;
    f[26] = ty - (float)r0;
  }
  free(cell);
  free(count);
}
