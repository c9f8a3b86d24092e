// Host-side numerics of the FBIM library (FP64 / long double, no device code).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fbim.h"

namespace fbim {

constexpr double kCr = 100.0;  // real-space truncation constant (Section 3.2)
constexpr double kCw = 1.0;    // wave-space truncation constant (Section 3.2)
constexpr double kPi = 3.14159265358979323846264338327950288;

struct Derived {
  double L, xi, r_c, h, eta_s;
  int n_box, M, P, tile;
};

// Parameter rule of eq. 3.26; returns an error message or "".
std::string derive(const fbim_params &p, Derived &d);

// E1 in long double (series for z <= 2, continued fraction by modified Lentz beyond).
long double e1l(long double z);

// Piecewise polynomial tables for the device E1 evaluation: per interval with
// centre c and half-width h, deg + 1 power-series coefficients in x = (z - c) / h
// of the interval's Chebyshev interpolant.
//   interval 0:  [0, 2],          f = E1(z) + ln z
//   interval k:  [b_(k-1), b_k],  f = e^z E1(z), ends b = 2, 3, 4, 6, 8, ..., 48, 64
//                (each binade split at 1.5 times its start)
// Layout per interval: {1/h, -c/h, a_0, a_1, ..., a_deg}: x = z row[0] + row[1],
// f = sum a_m x^m.
constexpr int kE1Intervals = 11;
constexpr int kE1Deg64 = 16;
constexpr int kE1Deg32 = 9;
std::vector<double> e1_table(int deg);
double e1_table_eval(const std::vector<double> &tab, int deg, double z);  // host check
int e1_row(double z);  // table row of argument z

// Alpert log-singular end correction: j nodes chi, weights w, a dropped points.
bool alpert_rule(int order, int &j, int &a, double *chi, double *w, std::string &err);

// Real-space Ewald Stokeslet G^(r) (eq. 3.15) at displacement (dx, dy); g = {xx, xy, yy}.
void G_real(double dx, double dy, double xi, double eta, double g[3]);
// Wave-space Stokeslet G^(w)(r) of eq. 3.14 evaluated through the xi-independence
// of the split: G^(w)_xi = G^(w)_xi' + sum_p [G^(r)_xi'(r+pL) - G^(r)_xi(r+pL)].
void G_wave(double dx, double dy, double xi, double L, double eta, double g[3]);

// Symmetric eigen-decomposition (Householder tridiagonalisation, then implicit
// QR with the Wilkinson shift): A (n x n, row-major) ->
// eigenvalues lam[n], eigenvectors as columns of V (row-major).
void eigh_sym(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &V);

struct ShapeHost {
  int n_p = 0;
  int band = 0;                    // half-width of the Alpert band (in nodes)
  double r_alpert = 0.0;
  std::vector<double> ref_xy;      // 2 n_p
  std::vector<double> alpert;      // [t][o=-band..band][xx, xy, yx, yy], symmetrised
  std::vector<double> Mpinv;       // (2n_p)^2, column-major
  std::vector<double> Pref;        // 2n_p x 3, column-major: M_ref^+ K_ref
  std::vector<double> Nt;          // 3x3 row-major: (K^T M^+ K)^{-1}
  std::vector<double> Gref, Gpref; // (2n_p)^2 column-major (symmetric)
};

// Second-kind data of a closed curve sampled at n_p equispaced parameter values
// s_j = 2 pi j / n_p (either orientation): derivatives by trigonometric
// interpolation; per node [n_x, n_y, t_x, t_y, kappa, ds] with n the outward unit
// normal, t the unit tangent, kappa the curvature (positive where the curve is
// convex), ds = |gamma'(s_j)| 2 pi / n_p; length = sum ds, W = sum |x|^2 ds
// (about the reference origin, the tracking point).  Returns "" on success.
std::string curve_data(int n_p, const double *ref_xy, std::vector<double> &node6, double &length, double &W);

// Build all per-shape reference data; returns "" on success.
std::string build_shape(int n_p, const double *ref_xy, const Derived &d, double eta, int order,
                        double tau, ShapeHost &out);

}  // namespace fbim
