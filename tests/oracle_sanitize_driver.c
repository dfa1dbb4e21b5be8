/* Drives every entry point of the C oracle on small lattice inputs (duplicated points,
 * queries on data points, k = n, one data point) so that a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer checks its memory accesses and arithmetic.  Test
 * infrastructure: built and run by tests/test_oracle_sanitizers.py.  Exit status 0 when
 * every call returned its expected status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_bounds(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                   double out[4]);
int oracle_grid_params(const double bounds[4], int64_t n, double area_in, double cw_in, double occ, double out_d[3],
                       float* inv_cw, int32_t* ncol, int32_t* nrow);
void oracle_cell_index(const float* x, const float* y, int64_t n, float minX, float minY, float inv_cw, int32_t ncol,
                       int32_t nrow, int32_t* cell);
void oracle_knn(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m, int32_t k,
                int32_t* idx, double* d2);
void oracle_knn_paper(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                      int32_t k, float minX, float minY, float inv_cw, int32_t ncol, int32_t nrow, int32_t* idx,
                      double* d2);
void oracle_robs(const double* d2, int64_t m, int32_t k, double* r_obs);
void oracle_alpha(const double* r_obs, int64_t m, double r_exp, double rmin, double rmax, const double alpha5[5],
                  double* R_out, double* mu_out, double* alpha_out);
void oracle_idw(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy, int64_t m,
                const double* alpha, double* zq, double* s_norm);
int oracle_aidw(const float* x, const float* y, const float* z, int64_t n, const float* qx, const float* qy, int64_t m,
                const int64_t* qsel, int64_t msel, int32_t k, const double alpha5[5], double rmin, double rmax,
                double area_in, double cw_in, double occ, double* zq, double* alpha_out, double* r_obs_out,
                double* R_out, double* s_norm, int32_t* knn_idx, double* knn_d2, double* scal_out);
void oracle_features(const float* x, const float* y, int64_t n, const float* qx, const float* qy, int64_t m,
                     float minX, float minY, float inv_cw, int32_t ncol, int32_t nrow, float* feat);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static float lattice(void) { /* a point of the 2^-10 lattice in [0, 1) (coarse, so points repeat) */
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (float)((state >> 40) & 1023u) / 1024.0f;
}

static int run_case(int64_t n, int64_t m, int32_t k) {
  float* x = malloc(sizeof(float) * (size_t)n);
  float* y = malloc(sizeof(float) * (size_t)n);
  float* z = malloc(sizeof(float) * (size_t)n);
  float* qx = malloc(sizeof(float) * (size_t)m);
  float* qy = malloc(sizeof(float) * (size_t)m);
  for (int64_t i = 0; i < n; ++i) {
    x[i] = lattice();
    y[i] = lattice();
    z[i] = lattice() - 0.5f;
  }
  for (int64_t j = 0; j < m; ++j) {
    if (j % 5 == 0) { /* a query on a data point */
      qx[j] = x[j % n];
      qy[j] = y[j % n];
    } else {
      qx[j] = lattice();
      qy[j] = lattice();
    }
  }
  int bad = 0;
  double b[4], sc[3];
  float inv_cw;
  int32_t ncol, nrow;
  oracle_bounds(x, y, n, qx, qy, m, b);
  const double alpha5[5] = {1, 2, 3, 4, 5};
  if (b[2] > b[0] && b[3] > b[1]) {
    bad |= oracle_grid_params(b, n, 0.0, 0.0, 2.0, sc, &inv_cw, &ncol, &nrow) != 0;
    int32_t* cell = malloc(sizeof(int32_t) * (size_t)n);
    oracle_cell_index(x, y, n, (float)b[0], (float)b[1], inv_cw, ncol, nrow, cell);
    for (int64_t i = 0; i < n; ++i) bad |= cell[i] < 0 || cell[i] >= ncol * nrow;
    free(cell);
    int32_t* idx = malloc(sizeof(int32_t) * (size_t)(m * k));
    double* d2 = malloc(sizeof(double) * (size_t)(m * k));
    oracle_knn_paper(x, y, n, qx, qy, m, k, (float)b[0], (float)b[1], inv_cw, ncol, nrow, idx, d2);
    float* feat = malloc(sizeof(float) * (size_t)(m * 27));
    oracle_features(x, y, n, qx, qy, m, (float)b[0], (float)b[1], inv_cw, ncol, nrow, feat);
    free(feat);
    oracle_knn(x, y, n, qx, qy, m, k, idx, d2);
    double* ro = malloc(sizeof(double) * (size_t)m);
    double* al = malloc(sizeof(double) * (size_t)m);
    double* R = malloc(sizeof(double) * (size_t)m);
    double* zq = malloc(sizeof(double) * (size_t)m);
    double* s = malloc(sizeof(double) * (size_t)m);
    oracle_robs(d2, m, k, ro);
    oracle_alpha(ro, m, sc[1], 0.0, 2.0, alpha5, R, NULL, al);
    oracle_idw(x, y, z, n, qx, qy, m, al, zq, s);
    int64_t sel[3] = {0, m / 2, m - 1};
    bad |= oracle_aidw(x, y, z, n, qx, qy, m, NULL, m, k, alpha5, 0.0, 2.0, 0.0, 0.0, 2.0, zq, al, ro, R, s, idx, d2,
                       sc) != 0;
    bad |= oracle_aidw(x, y, z, n, qx, qy, m, sel, 3, k, alpha5, 0.0, 2.0, 0.0, 0.0, 2.0, zq, al, ro, R, s, idx, d2,
                       NULL) != 0;
    free(idx);
    free(d2);
    free(ro);
    free(al);
    free(R);
    free(zq);
    free(s);
  } else {
    /* degenerate bounds: the grid is refused, the run too unless an area is given */
    bad |= oracle_grid_params(b, n, 0.0, 0.0, 2.0, sc, &inv_cw, &ncol, &nrow) == 0;
  }
  free(x);
  free(y);
  free(z);
  free(qx);
  free(qy);
  return bad;
}

int main(void) {
  int bad = 0;
  bad |= run_case(300, 64, 10);  /* duplicates on the coarse lattice, coincident queries */
  bad |= run_case(40, 17, 40);   /* k = n */
  bad |= run_case(1, 3, 1);      /* one data point: a degenerate box */
  bad |= run_case(2000, 5, 15);
  if (bad) fprintf(stderr, "an oracle call returned an unexpected status\n");
  return bad;
}
