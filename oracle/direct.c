/* Direct FP64 sums for the oracle (test infrastructure only).
 *
 * real_space: (M^(t) mu)_m = sum over n != m with |r_mn| <= r_c (minimum
 *   image) of G^(r)(r_mn) mu_n, where (eq. 3.15)
 *   G^(r)(r) = 1/(4 pi eta) [ E1(xi^2 r^2)/2 I + (r r^T/r^2 - I) exp(-xi^2 r^2) ].
 *   Plain double loop over all sources for each requested target.
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

void oracle_real_space(int n_src, const double *X, const double *mu, double L, double xi,
                       double eta, double rc, int n_tgt, const int *tgt, double *out) {
  const double c = 1.0 / (4.0 * M_PI * eta);
#pragma omp parallel for schedule(dynamic, 16)
  for (int t = 0; t < n_tgt; ++t) {
    int m = tgt[t];
    double vx = 0.0, vy = 0.0;
    for (int n = 0; n < n_src; ++n) {
      if (n == m) continue;
      double dx = X[2 * m] - X[2 * n], dy = X[2 * m + 1] - X[2 * n + 1];
      dx -= L * nearbyint(dx / L);
      dy -= L * nearbyint(dy / L);
      double r2 = dx * dx + dy * dy;
      if (r2 > rc * rc) continue;
      double z = xi * xi * r2;
      double a = 0.5 * e1(z), ez = exp(-z);
      double gxx = a + (dx * dx / r2 - 1.0) * ez;
      double gyy = a + (dy * dy / r2 - 1.0) * ez;
      double gxy = dx * dy / r2 * ez;
      vx += gxx * mu[2 * n] + gxy * mu[2 * n + 1];
      vy += gxy * mu[2 * n] + gyy * mu[2 * n + 1];
    }
    out[2 * t] = c * vx;
    out[2 * t + 1] = c * vy;
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
