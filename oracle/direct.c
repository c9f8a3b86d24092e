/* Direct FP64 sums for the oracle (test infrastructure only).
 *
 * real_space: (M^(t) mu)_m = sum over n != m with |r_mn| <= r_c (minimum
 *   image) of G^(r)(r_mn) mu_n, where (eq. 3.15)
 *   G^(r)(r) = 1/(4 pi eta) [ E1(xi^2 r^2)/2 I + (r r^T/r^2 - I) exp(-xi^2 r^2) ].
 *   Plain double loop over all sources for each requested target.
 * real_space_cells: the same sum with the sources binned into n_c x n_c cells
 *   of side L / n_c >= r_c, so only the 3 x 3 cells around a target are
 *   visited (the CPU fast path; n_c >= 3 keeps the nine cells distinct).
 * spread / interp: the Gaussian gridding of the spectral-Ewald wave part
 *   (Section 3.2): H_c(x_g) += c e^{-a |x_g - x_n|^2} mu_{n,c} over the P x P
 *   nearest grid points (periodic), and v_{n,c} = sum_g c e^{-a |x_n - x_g|^2}
 *   U_c(x_g) (the h^2 factor is left to the caller).
 * wave_space: (M^(w) mu)_m = sum_k B(k) Re[ e^{-i k.x_m} S(k) ],
 *   S(k) = sum_n mu_n e^{i k.x_n}  (eqs. 3.14, 3.18), B(k) given per k.
 * E1 follows Abramowitz & Stegun 5.1.11 (series, z <= 1) and 5.1.22
 * (continued fraction, z > 1), as in the Python oracle.
 */
#include <math.h>
#include <stdlib.h>

static const double EULER_GAMMA = 0.57721566490153286060651209008240243;

static double e1(double z) {
  if (z <= 1.0) {
    double acc = 0.0, p = 1.0;
    for (int k = 1; k < 40; ++k) {
      p *= -z / k;
      acc += p / k;
    }
    return -EULER_GAMMA - log(z) - acc;
  }
  const int depth = 120;
  double t = z + 2.0 * depth + 1.0;
  for (int k = depth; k >= 1; --k) t = z + 2.0 * k - 1.0 - (double)k * k / t;
  return exp(-z) / t;
}

double oracle_e1(double z) { return e1(z); }

/* adds 4 pi eta G^(r)(x_m - x_n) mu_n to (vx, vy) when n != m is within r_c */
static inline void pair(const double *X, const double *mu, int m, int n, double L, double xi, double rc,
                        double *vx, double *vy) {
  if (n == m) return;
  double dx = X[2 * m] - X[2 * n], dy = X[2 * m + 1] - X[2 * n + 1];
  dx -= L * nearbyint(dx / L);
  dy -= L * nearbyint(dy / L);
  double r2 = dx * dx + dy * dy;
  if (r2 > rc * rc) return;
  double z = xi * xi * r2;
  double a = 0.5 * e1(z), ez = exp(-z);
  double gxx = a + (dx * dx / r2 - 1.0) * ez;
  double gyy = a + (dy * dy / r2 - 1.0) * ez;
  double gxy = dx * dy / r2 * ez;
  *vx += gxx * mu[2 * n] + gxy * mu[2 * n + 1];
  *vy += gxy * mu[2 * n] + gyy * mu[2 * n + 1];
}

void oracle_real_space(int n_src, const double *X, const double *mu, double L, double xi,
                       double eta, double rc, int n_tgt, const int *tgt, double *out) {
  const double c = 1.0 / (4.0 * M_PI * eta);
#pragma omp parallel for schedule(dynamic, 16)
  for (int t = 0; t < n_tgt; ++t) {
    int m = tgt[t];
    double vx = 0.0, vy = 0.0;
    for (int n = 0; n < n_src; ++n) pair(X, mu, m, n, L, xi, rc, &vx, &vy);
    out[2 * t] = c * vx;
    out[2 * t + 1] = c * vy;
  }
}

static int cell_of(double x, double L, int nc) {
  double w = x - L * floor(x / L); /* wrapped into [0, L) */
  int i = (int)(w / L * nc);
  return i < 0 ? 0 : (i >= nc ? nc - 1 : i);
}

/* returns 0, or -1 when n_c < 3 (then the direct sum is the one to use) */
int oracle_real_space_cells(int N, const double *X, const double *mu, double L, double xi, double eta,
                            double rc, double *out) {
  const int nc = (int)floor(L / rc);
  if (nc < 3) return -1;
  const double c = 1.0 / (4.0 * M_PI * eta);
  int *cell = (int *)malloc(sizeof(int) * (size_t)N);
  int *start = (int *)calloc((size_t)nc * nc + 1, sizeof(int));
  int *fill = (int *)malloc(sizeof(int) * ((size_t)nc * nc + 1));
  int *order = (int *)malloc(sizeof(int) * (size_t)N);
  for (int n = 0; n < N; ++n) {
    cell[n] = cell_of(X[2 * n + 1], L, nc) * nc + cell_of(X[2 * n], L, nc);
    start[cell[n] + 1]++;
  }
  for (int k = 0; k < nc * nc; ++k) start[k + 1] += start[k];
  for (int k = 0; k <= nc * nc; ++k) fill[k] = start[k];
  for (int n = 0; n < N; ++n) order[fill[cell[n]]++] = n;
#pragma omp parallel for schedule(dynamic, 64)
  for (int m = 0; m < N; ++m) {
    const int cx = cell[m] % nc, cy = cell[m] / nc;
    double vx = 0.0, vy = 0.0;
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        const int k = ((cy + oy + nc) % nc) * nc + (cx + ox + nc) % nc;
        for (int s = start[k]; s < start[k + 1]; ++s) pair(X, mu, m, order[s], L, xi, rc, &vx, &vy);
      }
    out[2 * m] = c * vx;
    out[2 * m + 1] = c * vy;
  }
  free(cell);
  free(start);
  free(fill);
  free(order);
  return 0;
}

/* grid indices i_p and offsets d_p = x - i_p h of the P nearest points, i_p wrapped */
static void stencil(double x, double L, double h, int M, int P, int *idx, double *d) {
  double w = x - L * floor(x / L);
  long near = (long)floor(w / h + 0.5);
  for (int p = 0; p < P; ++p) {
    long i = near + p - (P - 1) / 2;
    d[p] = w - (double)i * h;
    idx[p] = (int)(((i % M) + M) % M);
  }
}

#define ORACLE_PMAX 32

void oracle_spread(int N, const double *X, const double *mu, double L, double h, int M, int P, double c, double a,
                   double *H) {
  const size_t MM = (size_t)M * M;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    int ix[ORACLE_PMAX], iy[ORACLE_PMAX];
    double dx[ORACLE_PMAX], dy[ORACLE_PMAX], gy[ORACLE_PMAX];
    stencil(X[2 * n], L, h, M, P, ix, dx);
    stencil(X[2 * n + 1], L, h, M, P, iy, dy);
    for (int q = 0; q < P; ++q) gy[q] = exp(-a * dy[q] * dy[q]);
    for (int p = 0; p < P; ++p) {
      const double gx = c * exp(-a * dx[p] * dx[p]);
      for (int q = 0; q < P; ++q) {
        const double g = gx * gy[q];
        const size_t at = (size_t)iy[q] * M + ix[p];
#pragma omp atomic
        H[at] += g * mu[2 * n];
#pragma omp atomic
        H[MM + at] += g * mu[2 * n + 1];
      }
    }
  }
}

void oracle_interp(int N, const double *X, const double *U, double L, double h, int M, int P, double c, double a,
                   double *out) {
  const size_t MM = (size_t)M * M;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    int ix[ORACLE_PMAX], iy[ORACLE_PMAX];
    double dx[ORACLE_PMAX], dy[ORACLE_PMAX], gy[ORACLE_PMAX];
    stencil(X[2 * n], L, h, M, P, ix, dx);
    stencil(X[2 * n + 1], L, h, M, P, iy, dy);
    for (int q = 0; q < P; ++q) gy[q] = exp(-a * dy[q] * dy[q]);
    double vx = 0.0, vy = 0.0;
    for (int p = 0; p < P; ++p) {
      const double gx = c * exp(-a * dx[p] * dx[p]);
      for (int q = 0; q < P; ++q) {
        const double g = gx * gy[q];
        const size_t at = (size_t)iy[q] * M + ix[p];
        vx += g * U[at];
        vy += g * U[MM + at];
      }
    }
    out[2 * n] = vx;
    out[2 * n + 1] = vy;
  }
}

void oracle_wave_space(int n_src, const double *X, const double *mu, int K, const double *kv,
                       const double *B, int n_tgt, const int *tgt, double *out) {
  double *S = (double *)malloc(sizeof(double) * 4 * (size_t)K); /* Re/Im of S_x, S_y */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < K; ++k) {
    double srx = 0, six = 0, sry = 0, siy = 0;
    for (int n = 0; n < n_src; ++n) {
      double ph = kv[2 * k] * X[2 * n] + kv[2 * k + 1] * X[2 * n + 1];
      double cs = cos(ph), sn = sin(ph);
      srx += mu[2 * n] * cs;
      six += mu[2 * n] * sn;
      sry += mu[2 * n + 1] * cs;
      siy += mu[2 * n + 1] * sn;
    }
    S[4 * k] = srx;
    S[4 * k + 1] = six;
    S[4 * k + 2] = sry;
    S[4 * k + 3] = siy;
  }
#pragma omp parallel for schedule(static)
  for (int t = 0; t < n_tgt; ++t) {
    int m = tgt[t];
    double vx = 0, vy = 0;
    for (int k = 0; k < K; ++k) {
      double ph = kv[2 * k] * X[2 * m] + kv[2 * k + 1] * X[2 * m + 1];
      double cs = cos(ph), sn = sin(ph);
      /* Re[(cs - i sn)(sr + i si)] = cs sr + sn si */
      double fx = cs * S[4 * k] + sn * S[4 * k + 1];
      double fy = cs * S[4 * k + 2] + sn * S[4 * k + 3];
      vx += B[3 * k] * fx + B[3 * k + 1] * fy;
      vy += B[3 * k + 1] * fx + B[3 * k + 2] * fy;
    }
    out[2 * t] = vx;
    out[2 * t + 1] = vy;
  }
  free(S);
}
