// Host-side numerics: parameter rule, special functions, Alpert rules,
// reference matrices of a body shape.  FP64 / long double, CPU only.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace fbim {

// ---------------------------------------------------------------- parameters
std::string derive(const fbim_params &p, Derived &d) {
  if (!(p.L > 0) || !(p.tol_ewald > 0 && p.tol_ewald < 1)) return "L > 0 and 0 < tol_ewald < 1 required";
  if (p.grid_M < 0 || p.n_box < 0 || p.P < 0 || p.xi < 0) return "negative parameter";
  const double L = p.L, eps = p.tol_ewald;
  const double lr = std::sqrt(std::log(kCr / eps));
  const double lw = std::sqrt(std::log(kCw / eps));
  double xi = p.xi;
  int n_box = p.n_box;
  if (xi == 0.0) {
    if (n_box == 0) {
      if (p.grid_M == 0) return "one of n_box, grid_M, xi must be given";
      const double xi_max = (kPi * p.grid_M / L) / (2.0 * lw);
      n_box = (int)std::floor(L * xi_max / lr);
    }
    xi = lr * n_box / L;
  }
  if (n_box == 0) n_box = (int)std::floor(L * xi / lr);
  if (n_box < 3) return "n_box must be >= 3 (cutoff r_c = L/n_box at most L/3)";
  int M = p.grid_M;
  if (M == 0) {
    M = (int)std::ceil(2.0 * xi * lw * L / kPi);
    M += M % 2;
  }
  if (M % 2) return "grid_M must be even";
  int P = p.P;
  if (P == 0) {
    P = (int)std::ceil(2.0 * std::log(1.0 / eps) / kPi);
    P += 1 - P % 2;
  }
  if (P % 2 == 0 || P < 3) return "P must be odd and >= 3";
  const double h = L / M;
  const double m = std::sqrt(kPi * P);
  const double w = P * h / 2.0;
  int tile = p.tile;
  const int half = (P - 1) / 2;
  if (tile == 0) {
    for (int t = 32; t >= 4; --t)
      if (M % t == 0 && M / t >= 3 && t >= half) { tile = t; break; }
    if (tile == 0) return "no spreading tile fits the grid (need T | M, M/T >= 3, T >= (P-1)/2)";
  } else if (tile > 32 || M % tile || M / tile < 3 || tile < half) {
    return "invalid tile";
  }
  d.L = L;
  d.xi = xi;
  d.n_box = n_box;
  d.r_c = L / n_box;
  if (xi * d.r_c > 8.0) return "xi r_c must not exceed 8 (the real-space E1 series covers xi^2 r^2 <= 64)";
  d.M = M;
  d.P = P;
  d.h = h;
  d.eta_s = (2.0 * w * xi / m) * (2.0 * w * xi / m);
  d.tile = tile;
  return "";
}

// ---------------------------------------------------------------- E1
long double e1l(long double z) {
  const long double g = 0.577215664901532860606512090082402431L;
  if (z <= 2.0L) {
    long double acc = 0, p = 1;
    for (int k = 1; k < 80; ++k) {
      p *= -z / k;
      acc += p / k;
    }
    return -g - logl(z) - acc;
  }
  // continued fraction E1(z) = e^-z / (z+1 - 1/(z+3 - 4/(z+5 - ...))), evaluated
  // forward by the modified Lentz method until a step changes it by < 1e-19
  const long double tiny = 1e-300L;
  long double f = z + 1.0L, C = f, D = 0.0L;
  for (int k = 1; k < 2000; ++k) {
    const long double a = -(long double)k * k, b = z + 2.0L * k + 1.0L;
    D = b + a * D;
    if (D == 0.0L) D = tiny;
    D = 1.0L / D;
    C = b + a / C;
    if (C == 0.0L) C = tiny;
    const long double delta = C * D;
    f *= delta;
    if (fabsl(delta - 1.0L) < 1e-19L) break;
  }
  return expl(-z) / f;
}

// interval ends of the far rows: every binade [2^e, 2^(e+1)] from 2 to 64 split at
// 1.5 * 2^e, so that a far row is the float's exponent and leading mantissa bit
static const double kFarEnds[kE1Intervals] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};

static void interval(int k, double &lo, double &hi) {
  if (k == 0) { lo = 0.0; hi = 2.0; return; }
  lo = kFarEnds[k - 1];
  hi = kFarEnds[k];
}

int e1_row(double z) {
  if (z <= 2.0) return 0;
  int k = 1;
  while (k < kE1Intervals - 1 && z >= kFarEnds[k]) ++k;
  return k;
}

static long double e1_target(int k, long double z) {
  if (k == 0) {
    if (z == 0.0L) return -0.577215664901532860606512090082402431L;  // limit of E1 + ln z
    return e1l(z) + logl(z);
  }
  return expl(z) * e1l(z);
}

std::vector<double> e1_table(int deg) {
  const int n = deg + 1, stride = deg + 3;
  std::vector<double> tab(kE1Intervals * stride);
  for (int k = 0; k < kE1Intervals; ++k) {
    double lo, hi;
    interval(k, lo, hi);
    const long double c = 0.5L * ((long double)lo + hi), hw = 0.5L * ((long double)hi - lo);
    std::vector<long double> f(n);
    for (int j = 0; j < n; ++j) {
      long double x = cosl(3.14159265358979323846264338327950288L * (j + 0.5L) / n);
      f[j] = e1_target(k, c + hw * x);
    }
    std::vector<long double> cc(n);
    for (int m = 0; m < n; ++m) {
      long double s = 0;
      for (int j = 0; j < n; ++j)
        s += f[j] * cosl(3.14159265358979323846264338327950288L * m * (j + 0.5L) / n);
      s *= 2.0L / n;
      if (m == 0) s *= 0.5L;
      cc[m] = s;
    }
    // Chebyshev series -> power series in x (T_{m+1} = 2x T_m - T_{m-1}); the
    // power coefficients decay like the Taylor coefficients of the target about
    // the interval centre, so Horner's rule loses nothing
    std::vector<long double> a(n, 0.0L), tp(n, 0.0L), tc(n, 0.0L), tn(n);
    tp[0] = 1.0L;   // T_0
    if (n > 1) tc[1] = 1.0L;  // T_1
    a[0] += cc[0];
    if (n > 1) a[1] += cc[1];
    for (int m = 2; m < n; ++m) {
      for (int q = 0; q < n; ++q) tn[q] = (q > 0 ? 2.0L * tc[q - 1] : 0.0L) - tp[q];
      for (int q = 0; q < n; ++q) a[q] += cc[m] * tn[q];
      tp = tc;
      tc = tn;
    }
    double *row = &tab[k * stride];
    row[0] = (double)(1.0L / hw);  // x = z row[0] + row[1]
    row[1] = (double)(-c / hw);
    for (int m = 0; m < n; ++m) row[2 + m] = (double)a[m];
  }
  return tab;
}

double e1_table_eval(const std::vector<double> &tab, int deg, double z) {
  const int stride = deg + 3;
  const int k = e1_row(z);
  const double *row = &tab[k * stride];
  const double x = std::fma(z, row[0], row[1]);
  double f = row[2 + deg];
  for (int m = deg - 1; m >= 0; --m) f = std::fma(f, x, row[2 + m]);
  return k == 0 ? f - std::log(z) : std::exp(-z) * f;
}

// ---------------------------------------------------------------- zeta values
// Bernoulli numbers B_0..B_n (B_1 = -1/2) by the standard recurrence.
static std::vector<long double> bernoulli(int n) {
  std::vector<long double> B(n + 1, 0.0L);
  B[0] = 1.0L;
  for (int m = 1; m <= n; ++m) {
    long double s = 0, binom = 1;  // binom = C(m+1, k)
    for (int k = 0; k < m; ++k) {
      s += binom * B[k];
      binom = binom * (m + 1 - k) / (k + 1);
    }
    B[m] = -s / (m + 1);
  }
  return B;
}

// zeta(s) and zeta'(s) for real s >= 2 by Euler-Maclaurin with N terms summed.
static void zeta_em(long double s, long double &z, long double &dz) {
  const int N = 30, K = 12;
  auto B = bernoulli(2 * K);
  z = 0;
  dz = 0;
  for (int n = 1; n < N; ++n) {
    long double t = powl((long double)n, -s);
    z += t;
    dz -= logl((long double)n) * t;
  }
  const long double lN = logl((long double)N);
  const long double N1s = powl((long double)N, 1.0L - s), Ns = powl((long double)N, -s);
  z += N1s / (s - 1) + 0.5L * Ns;
  dz += -lN * N1s / (s - 1) - N1s / ((s - 1) * (s - 1)) - 0.5L * lN * Ns;
  long double fact = 1;  // (2k)!
  for (int k = 1; k <= K; ++k) {
    fact *= (2.0L * k - 1) * (2.0L * k);
    // rising factorial (s)_{2k-1} and its derivative
    long double P = 1, dP = 0;
    for (int i = 0; i <= 2 * k - 2; ++i) {
      dP = dP * (s + i) + P;
      P *= (s + i);
    }
    const long double Nk = powl((long double)N, -s - 2 * k + 1);
    z += B[2 * k] / fact * P * Nk;
    dz += B[2 * k] / fact * (dP - P * lN) * Nk;
  }
}

// zeta(-p) and zeta'(-p) for integer p >= 0 (reflection formula for the derivative).
static void zeta_negative(int p, long double &z, long double &dz) {
  const long double pi = 3.14159265358979323846264338327950288L;
  const long double ln2pi = logl(2.0L * pi);
  auto B = bernoulli(p + 2);
  if (p == 0) {
    z = -0.5L;
    dz = -0.5L * ln2pi;
    return;
  }
  z = -B[p + 1] / (p + 1);
  long double fac = 1;
  for (int i = 2; i <= p; ++i) fac *= i;  // p!
  if (p % 2 == 0) {
    const int m = p / 2;
    long double zs, dzs;
    zeta_em((long double)(p + 1), zs, dzs);
    const long double sign = (m % 2) ? -1.0L : 1.0L;
    dz = sign * fac * zs / (2.0L * powl(2.0L * pi, (long double)p));
  } else {
    const int m = (p + 1) / 2;
    long double zs, dzs;
    zeta_em((long double)(2 * m), zs, dzs);
    long double psi = -0.577215664901532860606512090082402431L;
    for (int k = 1; k <= 2 * m - 1; ++k) psi += 1.0L / k;
    dz = z * (ln2pi - psi - dzs / zs);
  }
}

// ---------------------------------------------------------------- Alpert rule
static bool solve_dense(int n, std::vector<long double> A, std::vector<long double> &b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(A[r * n + c]) > fabsl(A[piv * n + c])) piv = r;
    if (fabsl(A[piv * n + c]) < 1e-300L) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      long double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    long double s = b[c];
    for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
    b[c] = s / A[c * n + c];
  }
  return true;
}

bool alpert_rule(int order, int &j, int &a, double *chi, double *w, std::string &err) {
  if (order == 4) { j = 3; a = 2; }
  else if (order == 8) { j = 7; a = 5; }
  else { err = "alpert_order must be 4 or 8"; return false; }
  const int n = 2 * j;
  // right-hand sides: moments of x^p and x^p ln x lost by dropping 0 < i < a
  std::vector<long double> r1(j), r2(j);
  for (int p = 0; p < j; ++p) {
    long double z, dz;
    zeta_negative(p, z, dz);
    long double s1 = 0, s2 = 0;
    for (int i = 1; i < a; ++i) {
      s1 += powl((long double)i, p);
      s2 += powl((long double)i, p) * logl((long double)i);
    }
    r1[p] = -z + s1;
    r2[p] = dz + s2;
  }
  auto residual = [&](const std::vector<long double> &v, std::vector<long double> &f) {
    long double nrm = 0;
    for (int p = 0; p < j; ++p) {
      long double s1 = 0, s2 = 0;
      for (int k = 0; k < j; ++k) {
        long double e = expl(p * v[k]);
        s1 += v[j + k] * e;
        s2 += v[j + k] * e * v[k];
      }
      f[p] = s1 - r1[p];
      f[j + p] = s2 - r2[p];
      nrm += f[p] * f[p] + f[j + p] * f[j + p];
    }
    return sqrtl(nrm);
  };
  uint64_t lcg = 0x9E3779B97F4A7C15ull;
  auto urand = [&]() {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
  };
  for (int attempt = 0; attempt < 500; ++attempt) {
    // start: the j-a+1 innermost nodes spread geometrically in (0, 1), the rest
    // next to the dropped integers 1..a-1; weights ~ node spacing
    std::vector<long double> v(n);
    const int inner = j - a + 1;
    for (int k = 0; k < j; ++k) {
      double x = (k < inner) ? 0.6 * std::pow(0.25, inner - 1 - k) : (double)(k - inner + 1);
      if (attempt > 0) x *= std::exp(0.5 * (urand() - 0.5));
      v[k] = logl((long double)x);
      v[j + k] = (k < inner) ? x : 1.0;
      if (attempt > 0) v[j + k] *= 0.5 + urand();
    }
    std::vector<long double> f(n), J(n * n);
    long double res = residual(v, f);
    bool ok = false;
    for (int it = 0; it < 200; ++it) {
      for (int p = 0; p < j; ++p)
        for (int k = 0; k < j; ++k) {
          long double e = expl(p * v[k]);
          J[p * n + k] = v[j + k] * p * e;
          J[p * n + j + k] = e;
          J[(j + p) * n + k] = v[j + k] * e * (p * v[k] + 1.0L);
          J[(j + p) * n + j + k] = e * v[k];
        }
      std::vector<long double> step = f;
      if (!solve_dense(n, J, step)) break;
      long double lam = 1;
      std::vector<long double> trial(n), ft(n);
      long double rt = 0;
      for (int ls = 0; ls < 40; ++ls) {
        for (int i = 0; i < n; ++i) trial[i] = v[i] - lam * step[i];
        rt = residual(trial, ft);
        if (rt < res) break;
        lam *= 0.5L;
      }
      if (!(rt < res)) break;
      v = trial;
      f = ft;
      res = rt;
      if (res < 1e-17L) { ok = true; break; }
    }
    if (!ok) continue;
    bool admissible = true;
    for (int k = 0; k < j; ++k) {
      long double x = expl(v[k]);
      if (!(x > 0 && x < a && v[j + k] > 0)) admissible = false;
    }
    if (!admissible) continue;
    std::vector<std::pair<double, double>> cw(j);
    for (int k = 0; k < j; ++k) cw[k] = {(double)expl(v[k]), (double)v[j + k]};
    std::sort(cw.begin(), cw.end());
    bool distinct = true;
    for (int k = 1; k < j; ++k)
      if (cw[k].first - cw[k - 1].first < 1e-6) distinct = false;
    if (!distinct) continue;
    for (int k = 0; k < j; ++k) {
      chi[k] = cw[k].first;
      w[k] = cw[k].second;
    }
    return true;
  }
  err = "Alpert moment system did not converge";
  return false;
}

// ---------------------------------------------------------------- kernels on the host
void G_real(double dx, double dy, double xi, double eta, double g[3]) {
  const double r2 = dx * dx + dy * dy;
  const double z = xi * xi * r2;
  const double a = 0.5 * (double)e1l(z), ez = std::exp(-z);
  const double c = 1.0 / (4.0 * kPi * eta);
  g[0] = c * (a + (dx * dx / r2 - 1.0) * ez);
  g[1] = c * (dx * dy / r2 * ez);
  g[2] = c * (a + (dy * dy / r2 - 1.0) * ez);
}

void G_wave(double dx, double dy, double xi, double L, double eta, double g[3]) {
  const double xip = 3.0 / L;  // small splitting parameter: few k terms and images
  const double c = 1.0 / (4.0 * kPi * eta);
  g[0] = g[1] = g[2] = 0.0;
  // k-sum at xi' (terms with k^2/4xi'^2 <= 40)
  const double kmax = 2.0 * xip * std::sqrt(40.0);
  const int kap = (int)std::ceil(kmax * L / (2.0 * kPi));
  for (int i = -kap; i <= kap; ++i)
    for (int jj = -kap; jj <= kap; ++jj) {
      if (i == 0 && jj == 0) continue;
      const double kx = 2.0 * kPi * i / L, ky = 2.0 * kPi * jj / L;
      const double k2 = kx * kx + ky * ky;
      if (k2 > kmax * kmax) continue;
      const double u = k2 / (4.0 * xip * xip);
      const double s = (1.0 + u) * std::exp(-u) / k2 / (eta * L * L) * std::cos(kx * dx + ky * dy);
      g[0] += s * (1.0 - kx * kx / k2);
      g[1] += s * (-kx * ky / k2);
      g[2] += s * (1.0 - ky * ky / k2);
    }
  // image sums of the real-space difference
  const int pm = (int)std::ceil(std::sqrt(40.0) / xip / L) + 1;
  for (int px = -pm; px <= pm; ++px)
    for (int py = -pm; py <= pm; ++py) {
      const double rx = dx + px * L, ry = dy + py * L;
      const double r2 = rx * rx + ry * ry;
      if (r2 == 0.0) {
        // limit of [E1(xi'^2 r^2) - E1(xi^2 r^2)] / 2 as r -> 0
        const double a = 0.5 * std::log((xi * xi) / (xip * xip));
        g[0] += c * a;
        g[2] += c * a;
        continue;
      }
      // a term whose Gaussian exponent exceeds 60 is below e^-60 of the kernel's scale
      double g1[3] = {0.0, 0.0, 0.0}, g2[3] = {0.0, 0.0, 0.0};
      if (xip * xip * r2 <= 60.0) G_real(rx, ry, xip, eta, g1);
      if (xi * xi * r2 <= 60.0) G_real(rx, ry, xi, eta, g2);
      for (int k = 0; k < 3; ++k) g[k] += g1[k] - g2[k];
    }
}

// ---------------------------------------------------------------- symmetric eigensolver
// A = V diag(lam) V^T for a symmetric row-major n x n A: Householder reduction to
// tridiagonal form (reflectors accumulated into V), then implicit symmetric QR
// steps with the Wilkinson shift on the tridiagonal matrix, rotations
// accumulated into V (Golub and Van Loan, Matrix Computations, Sections 8.3.1-8.3.3).
void eigh_sym(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  lam.assign(n, 0.0);
  if (n == 0) return;
  std::vector<double> d(n), e(n, 0.0), v(n), p(n), w(n);
  auto at = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
  // Householder: zero A[k+2.., k] with H = I - beta v v^T acting on rows / columns k+1..
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += at(i, k) * at(i, k);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double alpha = at(k + 1, k) > 0 ? -xn : xn;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = at(i, k) - (i == k + 1 ? alpha : 0.0);
      vn += v[i] * v[i];
    }
    if (vn == 0.0) continue;
    const double beta = 2.0 / vn;
    double pv = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += at(i, j) * v[j];
      p[i] = beta * acc;
      pv += p[i] * v[i];
    }
    const double K = 0.5 * beta * pv;
    for (int i = k + 1; i < n; ++i) w[i] = p[i] - K * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) at(i, j) -= v[i] * w[j] + w[i] * v[j];
    at(k + 1, k) = at(k, k + 1) = alpha;
    for (int i = k + 2; i < n; ++i) at(i, k) = at(k, i) = 0.0;
    for (int r = 0; r < n; ++r) {  // V <- V H
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += V[(size_t)r * n + j] * v[j];
      acc *= beta;
      for (int j = k + 1; j < n; ++j) V[(size_t)r * n + j] -= acc * v[j];
    }
  }
  for (int i = 0; i < n; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);
  // the rotations act on column pairs of V: work on its transpose, whose rows are contiguous
  std::vector<double> &Vt = A;
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) Vt[(size_t)j * n + r] = V[(size_t)r * n + j];
  // implicit QR steps on the unreduced block [lo, hi]
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, guard = 0;
  while (hi > 0 && guard < 64 * n) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    ++guard;
    const double dl = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double mu = d[hi] - eh * eh / (dl + (dl >= 0 ? 1.0 : -1.0) * std::hypot(dl, eh));
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r > 0 ? x / r : 1.0, s = r > 0 ? -z / r : 0.0;
      if (k > lo) e[k - 1] = r;  // the bulge is chased down
      const double a = d[k], b = e[k], dd = d[k + 1];
      d[k] = c * c * a - 2.0 * c * s * b + s * s * dd;
      d[k + 1] = s * s * a + 2.0 * c * s * b + c * c * dd;
      e[k] = c * s * (a - dd) + (c * c - s * s) * b;
      if (k + 1 < hi) {
        x = e[k];
        z = -s * e[k + 1];
        e[k + 1] *= c;
      }
      double *vk = &Vt[(size_t)k * n], *vk1 = vk + n;
      for (int rr = 0; rr < n; ++rr) {
        const double a0 = vk[rr], a1 = vk1[rr];
        vk[rr] = c * a0 - s * a1;
        vk1[rr] = s * a0 + c * a1;
      }
    }
  }
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) V[(size_t)r * n + j] = Vt[(size_t)j * n + r];
  lam = d;
}

// ---------------------------------------------------------------- shape data
namespace {

struct TrigInterp {
  int n;
  std::vector<double> re[2], im[2];  // coefficients k = 0..n/2
  TrigInterp(int n_, const double *xy) : n(n_) {
    for (int c = 0; c < 2; ++c) {
      re[c].assign(n / 2 + 1, 0.0);
      im[c].assign(n / 2 + 1, 0.0);
      for (int k = 0; k <= n / 2; ++k) {
        long double sr = 0, si = 0;
        for (int j = 0; j < n; ++j) {
          long double ang = 2.0L * 3.14159265358979323846264338327950288L * k * j / n;
          sr += xy[2 * j + c] * cosl(ang);
          si -= xy[2 * j + c] * sinl(ang);
        }
        re[c][k] = (double)(sr / n);
        im[c][k] = (double)(si / n);
      }
    }
  }
  // real trigonometric interpolant; the Nyquist term is taken as a cosine
  void eval(double s, double out[2]) const {
    for (int c = 0; c < 2; ++c) {
      double v = re[c][0];
      for (int k = 1; k < n / 2; ++k) v += 2.0 * (re[c][k] * std::cos(k * s) - im[c][k] * std::sin(k * s));
      v += re[c][n / 2] * std::cos(0.5 * n * s);
      out[c] = v;
    }
  }
};

void lagrange(double x, int ell, int *offs, double *wts) {
  const int i0 = (int)std::floor(x) - ell / 2 + 1;
  for (int m = 0; m < ell; ++m) offs[m] = i0 + m;
  for (int m = 0; m < ell; ++m) {
    double v = 1.0;
    for (int q = 0; q < ell; ++q)
      if (q != m) v *= (x - (i0 + q)) / (double)(m - q);
    wts[m] = v;
  }
}

inline double wrapd(double d, double L) { return d - L * std::nearbyint(d / L); }

void sym_functions(int n, const std::vector<double> &A, double tau, std::vector<double> &finv_half,
                   std::vector<double> &fhalf, std::vector<double> &finv) {
  std::vector<double> lam, V;
  eigh_sym(n, A, lam, V);
  double lmax = 0;
  for (double l : lam) lmax = std::max(lmax, l);
  std::vector<double> d1(n), d2(n), d3(n);
  for (int i = 0; i < n; ++i) {
    // square roots: positive eigenvalues above the spurious threshold only;
    // inverse: every eigenvalue of magnitude above the threshold, with its sign,
    // so that the block preconditioner stays nonsingular (the near-null normal
    // mode of a body carries a small eigenvalue of either sign)
    const bool keep = lam[i] > tau * lmax;
    d1[i] = keep ? 1.0 / std::sqrt(lam[i]) : 0.0;
    d2[i] = keep ? std::sqrt(lam[i]) : 0.0;
    d3[i] = std::fabs(lam[i]) > tau * lmax ? 1.0 / lam[i] : 0.0;
  }
  auto build = [&](const std::vector<double> &d, std::vector<double> &out) {
    out.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        double s = 0;
        for (int k = 0; k < n; ++k) s += V[(size_t)r * n + k] * d[k] * V[(size_t)c * n + k];
        out[(size_t)c * n + r] = s;  // column-major (symmetric anyway)
      }
  };
  build(d1, finv_half);
  build(d2, fhalf);
  build(d3, finv);
}

}  // namespace

std::string build_shape(int n_p, const double *ref_xy, const Derived &d, double eta, int order,
                        double tau, ShapeHost &S) {
  if (n_p < 16 || n_p > 512 || n_p % 2) return "n_p must be even, 16 <= n_p <= 512";
  int j, a;
  double chi[8], w[8];
  std::string err;
  if (!alpert_rule(order, j, a, chi, w, err)) return err;
  S.n_p = n_p;
  S.ref_xy.assign(ref_xy, ref_xy + 2 * n_p);
  const TrigInterp gam(n_p, ref_xy);
  const double ds = 2.0 * kPi / n_p;
  const int ell = order;
  const double rc2 = d.r_c * d.r_c;
  // band half-width from the Lagrange stencils and the dropped points
  int band = a - 1;
  for (int k = 0; k < j; ++k) {
    int offs[16];
    double wts[16];
    lagrange(chi[k], ell, offs, wts);
    for (int m = 0; m < ell; ++m) band = std::max(band, std::abs(offs[m]));
    lagrange(-chi[k], ell, offs, wts);
    for (int m = 0; m < ell; ++m) band = std::max(band, std::abs(offs[m]));
  }
  if (2 * band + 1 > n_p) return "n_p too small for the Alpert stencil";
  S.band = band;
  const int nb = 2 * band + 1;
  // unsymmetrised Alpert correction, dense per block (t, l) in a (n_p x n_p) 2x2 array
  std::vector<double> A((size_t)n_p * n_p * 4, 0.0);
  auto add = [&](int t, int l, const double g[3], double f) {
    double *blk = &A[((size_t)t * n_p + l) * 4];
    blk[0] += f * g[0];
    blk[1] += f * g[1];
    blk[2] += f * g[1];
    blk[3] += f * g[2];
  };
  for (int t = 0; t < n_p; ++t) {
    const double xt = ref_xy[2 * t], yt = ref_xy[2 * t + 1];
    for (int k = 0; k < j; ++k)
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        double y[2];
        gam.eval(t * ds + sgn * chi[k] * ds, y);
        double g[3];
        G_real(xt - y[0], yt - y[1], d.xi, eta, g);
        int offs[16];
        double wts[16];
        lagrange(sgn * chi[k], ell, offs, wts);
        for (int m = 0; m < ell; ++m) add(t, ((t + offs[m]) % n_p + n_p) % n_p, g, w[k] * wts[m]);
      }
    for (int i = 1; i < a; ++i)
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int l = ((t + sgn * i) % n_p + n_p) % n_p;
        const double dx = wrapd(xt - ref_xy[2 * l], d.L), dy = wrapd(yt - ref_xy[2 * l + 1], d.L);
        if (dx * dx + dy * dy > rc2) continue;
        double g[3];
        G_real(dx, dy, d.xi, eta, g);
        add(t, l, g, -1.0);
      }
  }
  // symmetrise: As = (A + A^T)/2 over the full 2n_p x 2n_p matrix
  S.alpert.assign((size_t)n_p * nb * 4, 0.0);
  double r_alpert = 0.0;
  for (int t = 0; t < n_p; ++t)
    for (int o = -band; o <= band; ++o) {
      const int l = ((t + o) % n_p + n_p) % n_p;
      const double *b1 = &A[((size_t)t * n_p + l) * 4];
      const double *b2 = &A[((size_t)l * n_p + t) * 4];
      double *dst = &S.alpert[((size_t)t * nb + (o + band)) * 4];
      dst[0] = 0.5 * (b1[0] + b2[0]);
      dst[1] = 0.5 * (b1[1] + b2[2]);
      dst[2] = 0.5 * (b1[2] + b2[1]);
      dst[3] = 0.5 * (b1[3] + b2[3]);
      if (dst[0] != 0.0 || dst[1] != 0.0 || dst[3] != 0.0) {
        const double dx = ref_xy[2 * t] - ref_xy[2 * l], dy = ref_xy[2 * t + 1] - ref_xy[2 * l + 1];
        r_alpert = std::max(r_alpert, std::sqrt(dx * dx + dy * dy));
      }
    }
  S.r_alpert = r_alpert;
  // dense reference blocks: M^(r)_ref = M^(t)_ref + M^(a)_ref,sym and M_ref = M^(r)_ref + M^(w)_ref
  const int n2 = 2 * n_p;
  std::vector<double> Mr((size_t)n2 * n2, 0.0), Mf((size_t)n2 * n2, 0.0);
  for (int m = 0; m < n_p; ++m)
    for (int n = 0; n < n_p; ++n) {
      double dx = wrapd(ref_xy[2 * m] - ref_xy[2 * n], d.L);
      double dy = wrapd(ref_xy[2 * m + 1] - ref_xy[2 * n + 1], d.L);
      double gt[3] = {0, 0, 0}, gw[3];
      if (m != n && dx * dx + dy * dy <= rc2) G_real(dx, dy, d.xi, eta, gt);
      G_wave(ref_xy[2 * m] - ref_xy[2 * n], ref_xy[2 * m + 1] - ref_xy[2 * n + 1], d.xi, d.L, eta, gw);
      const double vt[4] = {gt[0], gt[1], gt[1], gt[2]};
      const double vw[4] = {gw[0], gw[1], gw[1], gw[2]};
      for (int c1 = 0; c1 < 2; ++c1)
        for (int c2 = 0; c2 < 2; ++c2) {
          Mr[(size_t)(2 * m + c1) * n2 + 2 * n + c2] += vt[c1 * 2 + c2];
          Mf[(size_t)(2 * m + c1) * n2 + 2 * n + c2] += vt[c1 * 2 + c2] + vw[c1 * 2 + c2];
        }
    }
  for (int t = 0; t < n_p; ++t)
    for (int o = -band; o <= band; ++o) {
      const int l = ((t + o) % n_p + n_p) % n_p;
      const double *blk = &S.alpert[((size_t)t * nb + (o + band)) * 4];
      for (int c1 = 0; c1 < 2; ++c1)
        for (int c2 = 0; c2 < 2; ++c2) {
          Mr[(size_t)(2 * t + c1) * n2 + 2 * l + c2] += blk[c1 * 2 + c2];
          Mf[(size_t)(2 * t + c1) * n2 + 2 * l + c2] += blk[c1 * 2 + c2];
        }
    }
  // symmetrise numerically (entries are symmetric up to rounding)
  for (int r = 0; r < n2; ++r)
    for (int c = r + 1; c < n2; ++c) {
      double s = 0.5 * (Mr[(size_t)r * n2 + c] + Mr[(size_t)c * n2 + r]);
      Mr[(size_t)r * n2 + c] = Mr[(size_t)c * n2 + r] = s;
      s = 0.5 * (Mf[(size_t)r * n2 + c] + Mf[(size_t)c * n2 + r]);
      Mf[(size_t)r * n2 + c] = Mf[(size_t)c * n2 + r] = s;
    }
  std::vector<double> tmp1, tmp2;
  sym_functions(n2, Mr, tau, S.Gref, S.Gpref, tmp1);
  sym_functions(n2, Mf, tau, tmp1, tmp2, S.Mpinv);
  // preconditioner: P_ref = M^+ K_ref (2n_p x 3), N_ref = (K^T M^+ K)^-1
  S.Pref.assign((size_t)n2 * 3, 0.0);
  for (int r = 0; r < n2; ++r) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int n = 0; n < n_p; ++n) {
      const double mx = S.Mpinv[(size_t)(2 * n) * n2 + r], my = S.Mpinv[(size_t)(2 * n + 1) * n2 + r];
      s0 += mx;
      s1 += my;
      s2 += -ref_xy[2 * n + 1] * mx + ref_xy[2 * n] * my;
    }
    S.Pref[r] = s0;
    S.Pref[n2 + r] = s1;
    S.Pref[2 * n2 + r] = s2;
  }
  double KMK[9] = {0};
  for (int n = 0; n < n_p; ++n) {
    const double kx[3] = {1.0, 0.0, -ref_xy[2 * n + 1]};
    const double ky[3] = {0.0, 1.0, ref_xy[2 * n]};
    for (int c1 = 0; c1 < 3; ++c1)
      for (int c2 = 0; c2 < 3; ++c2)
        KMK[c1 * 3 + c2] += kx[c1] * S.Pref[c2 * n2 + 2 * n] + ky[c1] * S.Pref[c2 * n2 + 2 * n + 1];
  }
  for (int c1 = 0; c1 < 3; ++c1)
    for (int c2 = c1 + 1; c2 < 3; ++c2) KMK[c1 * 3 + c2] = KMK[c2 * 3 + c1] = 0.5 * (KMK[c1 * 3 + c2] + KMK[c2 * 3 + c1]);
  const double det = KMK[0] * (KMK[4] * KMK[8] - KMK[5] * KMK[7]) - KMK[1] * (KMK[3] * KMK[8] - KMK[5] * KMK[6]) +
                     KMK[2] * (KMK[3] * KMK[7] - KMK[4] * KMK[6]);
  if (!(std::fabs(det) > 0)) return "singular reference body mobility";
  S.Nt.assign(9, 0.0);
  S.Nt[0] = (KMK[4] * KMK[8] - KMK[5] * KMK[7]) / det;
  S.Nt[1] = (KMK[2] * KMK[7] - KMK[1] * KMK[8]) / det;
  S.Nt[2] = (KMK[1] * KMK[5] - KMK[2] * KMK[4]) / det;
  S.Nt[3] = (KMK[5] * KMK[6] - KMK[3] * KMK[8]) / det;
  S.Nt[4] = (KMK[0] * KMK[8] - KMK[2] * KMK[6]) / det;
  S.Nt[5] = (KMK[2] * KMK[3] - KMK[0] * KMK[5]) / det;
  S.Nt[6] = (KMK[3] * KMK[7] - KMK[4] * KMK[6]) / det;
  S.Nt[7] = (KMK[1] * KMK[6] - KMK[0] * KMK[7]) / det;
  S.Nt[8] = (KMK[0] * KMK[4] - KMK[1] * KMK[3]) / det;
  return "";
}

// ---------------------------------------------------------------- curve data (second kind)
std::string curve_data(int n_p, const double *ref_xy, std::vector<double> &node6, double &length, double &W) {
  if (n_p < 8 || n_p % 2) return "curve data needs an even n_p >= 8";
  const int n = n_p;
  // first and second derivatives in s of each coordinate: DFT, multiply by (i k),
  // (i k)^2 with k in (-n/2, n/2) (the Nyquist mode dropped from the first
  // derivative, kept in the second), inverse DFT; O(n^2), long double
  std::vector<double> d1(2 * n), d2(2 * n);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int c = 0; c < 2; ++c) {
    std::vector<long double> re(n), im(n);
    for (int k = 0; k < n; ++k) {
      long double a = 0, b = 0;
      for (int j = 0; j < n; ++j) {
        const long double ang = -2.0L * pi * (long double)((long long)j * k % n) / n;
        a += ref_xy[2 * j + c] * cosl(ang);
        b += ref_xy[2 * j + c] * sinl(ang);
      }
      re[k] = a;
      im[k] = b;
    }
    for (int j = 0; j < n; ++j) {
      long double s1 = 0, s2 = 0;
      for (int k = 0; k < n; ++k) {
        const int kk = k < n / 2 ? k : k - n;
        const long double ang = 2.0L * pi * (long double)((long long)j * k % n) / n;
        const long double cr = re[k] * cosl(ang) - im[k] * sinl(ang);  // Re(c_k e^{i ang})
        const long double ci = re[k] * sinl(ang) + im[k] * cosl(ang);  // Im(c_k e^{i ang})
        if (k != n / 2) s1 += -(long double)kk * ci;                   // Re(i kk c_k e^{i ang})
        const long double kq = k == n / 2 ? (long double)(n / 2) : (long double)kk;
        s2 += -kq * kq * cr;
      }
      d1[2 * j + c] = (double)(s1 / n);
      d2[2 * j + c] = (double)(s2 / n);
    }
  }
  // orientation from the signed area (1/2) int (x y' - y x') ds
  double area = 0;
  for (int j = 0; j < n; ++j) area += ref_xy[2 * j] * d1[2 * j + 1] - ref_xy[2 * j + 1] * d1[2 * j];
  if (!(std::fabs(area) > 0)) return "degenerate curve";
  const double sgn = area > 0 ? 1.0 : -1.0;
  node6.assign(6 * (size_t)n, 0.0);
  length = 0;
  W = 0;
  for (int j = 0; j < n; ++j) {
    const double xp = d1[2 * j], yp = d1[2 * j + 1], xpp = d2[2 * j], ypp = d2[2 * j + 1];
    const double sp = std::hypot(xp, yp);
    if (!(sp > 0)) return "curve with a stationary point";
    const double tx = xp / sp, ty = yp / sp;
    double *o = &node6[6 * (size_t)j];
    o[0] = sgn * ty;  // outward: the tangent turned clockwise for a counterclockwise curve
    o[1] = -sgn * tx;
    o[2] = tx;
    o[3] = ty;
    o[4] = sgn * (xp * ypp - yp * xpp) / (sp * sp * sp);
    o[5] = sp * 2.0 * (double)pi / n;
    length += o[5];
    W += (ref_xy[2 * j] * ref_xy[2 * j] + ref_xy[2 * j + 1] * ref_xy[2 * j + 1]) * o[5];
  }
  return "";
}

}  // namespace fbim
