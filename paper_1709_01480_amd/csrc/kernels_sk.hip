// Completed second-kind formulation (Appendix B): per-node curve data, the
// wave-space parts of the periodic stresslet and of the completion flow
// (Stokeslet and rotlet at the tracking points) by the spectral-Ewald steps,
// and the rigid-body and closure terms of the second-kind operator.  The real-
// space kernels are in kernels_real.hip (they share the neighbour lists and the
// E1 tables there).
#include "kernels.h"

namespace fbim {

namespace {

// per node: w = n ds (outward normal times arc weight), the trapezoid diagonal
// 2 kappa ds t t^T (xx, xy, yy), ds, and r = x - q, all rotated by the body's angle;
// wc[k] = w of the k-th cell-sorted node
__global__ void k_sk_geom(int N, const int *__restrict__ body, const int *__restrict__ off,
                          const int *__restrict__ shape, const double *__restrict__ theta,
                          const double *const *ref, const double *const *sk6, double2 *__restrict__ w,
                          double *__restrict__ diag, double *__restrict__ ds, double2 *__restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = body[i], t = i - off[b];
  const double *c6 = sk6[shape[b]] + 6 * t;
  const double *rf = ref[shape[b]];
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  const double nx = cs * c6[0] - sn * c6[1], ny = sn * c6[0] + cs * c6[1];
  const double tx = cs * c6[2] - sn * c6[3], ty = sn * c6[2] + cs * c6[3];
  const double d = c6[5], k2 = 2.0 * c6[4] * d;
  w[i] = make_double2(nx * d, ny * d);
  diag[3 * i] = k2 * tx * tx;
  diag[3 * i + 1] = k2 * tx * ty;
  diag[3 * i + 2] = k2 * ty * ty;
  ds[i] = d;
  r[i] = make_double2(cs * rf[2 * t] - sn * rf[2 * t + 1], sn * rf[2 * t] + cs * rf[2 * t + 1]);
}

__global__ void k_gather_d2(int N, const int *__restrict__ perm, const double2 *__restrict__ a,
                            double2 *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) out[k] = a[perm[k]];
}

// spreading inputs in tile order: A = (phi_x w_x, phi_x w_y), B = (phi_y w_x, phi_y w_y),
// the components S_lm = phi_l w_m with l the density component
__global__ void k_sk_prep(int N, const int *__restrict__ tperm, const double2 *__restrict__ phi,
                          const double2 *__restrict__ w, double2 *__restrict__ A, double2 *__restrict__ B) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int i = tperm[k];
  const double2 p = phi[i], v = w[i];
  A[k] = make_double2(p.x * v.x, p.x * v.y);
  B[k] = make_double2(p.y * v.x, p.y * v.y);
}

// point sources at the tracking points spread to the grid with the Gaussian of the
// spreading kernel: planes 0, 1 take (f_x, f_y), plane 2 the torque.  One block per
// body, one thread per stencil point (P <= 15), FP64 atomics on the grid.
__global__ void k_point_spread(int n, const double *__restrict__ q, const double *__restrict__ F, int M, int P,
                               double h, double L, double ag, double cg, double *__restrict__ grid) {
  const int c = blockIdx.x, s = threadIdx.x;
  if (c >= n || s >= P * P) return;
  double x = q[2 * c] - L * floor(q[2 * c] / L), y = q[2 * c + 1] - L * floor(q[2 * c + 1] / L);
  const long ix0 = (long)floor(x / h + 0.5) - (P - 1) / 2, iy0 = (long)floor(y / h + 0.5) - (P - 1) / 2;
  const long ix = ix0 + s % P, iy = iy0 + s / P;
  const double dx = x - ix * h, dy = y - iy * h;
  const double g = cg * exp(-ag * (dx * dx + dy * dy));
  const long gx = ((ix % M) + M) % M, gy = ((iy % M) + M) % M;
  const size_t at = (size_t)gy * M + gx, MM = (size_t)M * M;
  atomicAdd(&grid[at], g * F[3 * c]);
  atomicAdd(&grid[MM + at], g * F[3 * c + 1]);
  atomicAdd(&grid[2 * MM + at], g * F[3 * c + 2]);
}

// Fourier multipliers on the half spectra [planes][M][M/2+1] (row = ky, col = kx).
// mode 0 (stresslet): planes S_xx, S_xy, S_yx, S_yy -> U_x, U_y in planes 0, 1:
//   U_j = i sc e^{-(1-eta_s) u} / k^4 sum_lm [(1 + u) t1_jlm + t2_jlm] S_lm,
//   t1 = k^2 (k_j d_lm + k_l d_mj) - 2 k_j k_l k_m, t2 = k^2 k_m d_jl
// (the wave term of the periodic stresslet with the sine written as -i e^{i k x},
// the Gaussian of spreading and interpolation divided out);
// mode 1 (completion): planes f_x, f_y, tau -> U_x, U_y:
//   U = sc (1 + u) e^{-(1-eta_s) u} [(I - k k^T / k^2) f / k^2 - i k^perp tau / (2 k^2)].
// sc = h^2 / (eta L^2).  Zero at k = 0 and on the Nyquist row and column (the odd
// terms there have no real-to-complex counterpart; they are below the Ewald
// tolerance).
__global__ void k_sk_mult(int M, double twopi_L, double inv4xi2, double one_m_eta, double sc, int mode,
                          double2 *__restrict__ spec) {
  const int nh = M / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * nh) return;
  const int row = idx / nh, col = idx - row * nh;
  const size_t pl = (size_t)M * nh;
  const double kx = twopi_L * col, ky = twopi_L * (row < M / 2 ? row : row - M);
  const double k2 = kx * kx + ky * ky;
  if (k2 == 0.0 || row == M / 2 || col == M / 2) {
    spec[idx] = make_double2(0, 0);
    spec[pl + idx] = make_double2(0, 0);
    return;
  }
  const double u = k2 * inv4xi2, e = exp(-one_m_eta * u);
  if (mode == 0) {
    const double2 sxx = spec[idx], sxy = spec[pl + idx], syx = spec[2 * pl + idx], syy = spec[3 * pl + idx];
    const double k[2] = {kx, ky};
    double2 out[2];
    for (int j = 0; j < 2; ++j) {
      // sum_lm t1_jlm S_lm and t2_jlm S_lm, real and imaginary parts
      const double2 tr = make_double2(sxx.x + syy.x, sxx.y + syy.y);
      const double2 klj = j == 0 ? make_double2(kx * sxx.x + ky * syx.x, kx * sxx.y + ky * syx.y)
                                 : make_double2(kx * sxy.x + ky * syy.x, kx * sxy.y + ky * syy.y);  // k_l S_lj
      const double2 kks = make_double2(kx * kx * sxx.x + kx * ky * (sxy.x + syx.x) + ky * ky * syy.x,
                                       kx * kx * sxx.y + kx * ky * (sxy.y + syx.y) + ky * ky * syy.y);
      const double2 kjm = j == 0 ? make_double2(kx * sxx.x + ky * sxy.x, kx * sxx.y + ky * sxy.y)
                                 : make_double2(kx * syx.x + ky * syy.x, kx * syx.y + ky * syy.y);  // k_m S_jm
      const double t1r = k2 * (k[j] * tr.x + klj.x) - 2.0 * k[j] * kks.x;
      const double t1i = k2 * (k[j] * tr.y + klj.y) - 2.0 * k[j] * kks.y;
      const double vr = (1.0 + u) * t1r + k2 * kjm.x, vi = (1.0 + u) * t1i + k2 * kjm.y;
      const double f = sc * e / (k2 * k2);
      out[j] = make_double2(-f * vi, f * vr);  // times i
    }
    spec[idx] = out[0];
    spec[pl + idx] = out[1];
  } else {
    const double2 fx = spec[idx], fy = spec[pl + idx], tq = spec[2 * pl + idx];
    const double s0 = sc * (1.0 + u) * e / k2;
    const double pxx = 1.0 - kx * kx / k2, pxy = -kx * ky / k2, pyy = 1.0 - ky * ky / k2;
    // -i k^perp tau / 2 with k^perp = (-ky, kx)
    const double2 rx = make_double2(-0.5 * ky * tq.y, 0.5 * ky * tq.x) /* -i (-ky) tau / 2 = i ky tau / 2 */;
    const double2 ry = make_double2(0.5 * kx * tq.y, -0.5 * kx * tq.x); /* -i kx tau / 2 */
    spec[idx] = make_double2(s0 * (pxx * fx.x + pxy * fy.x + rx.x), s0 * (pxx * fx.y + pxy * fy.y + rx.y));
    spec[pl + idx] = make_double2(s0 * (pxy * fx.x + pyy * fy.x + ry.x), s0 * (pxy * fx.y + pyy * fy.y + ry.y));
  }
}

// one 64-lane work group per body: the closure rows y_U = U - Z phi,
//   Z phi = ((1/|Gamma|) sum phi ds, (1/W) sum phi . r^perp ds), r^perp = (-r_y, r_x),
// and the body's share of the stresslet mean term, sum (q + r)_j (phi . w)
__global__ __launch_bounds__(64) void k_sk_body(const int *__restrict__ off, const int *__restrict__ shape,
                                                const double *__restrict__ q, const double *__restrict__ lw,
                                                const double2 *__restrict__ phi, const double2 *__restrict__ w,
                                                const double *__restrict__ ds, const double2 *__restrict__ r,
                                                const double *__restrict__ U, double *__restrict__ yU,
                                                double *__restrict__ part) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const int a = off[b], e = off[b + 1];
  double sx = 0, sy = 0, st = 0, fl = 0, mx = 0, my = 0;
  for (int i = a + lane; i < e; i += 64) {
    const double2 p = phi[i], rr = r[i], ww = w[i];
    const double d = ds[i];
    sx += p.x * d;
    sy += p.y * d;
    st += (-rr.y * p.x + rr.x * p.y) * d;
    const double pw = p.x * ww.x + p.y * ww.y;
    fl += pw;
    mx += rr.x * pw;
    my += rr.y * pw;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_down(sx, o);
    sy += __shfl_down(sy, o);
    st += __shfl_down(st, o);
    fl += __shfl_down(fl, o);
    mx += __shfl_down(mx, o);
    my += __shfl_down(my, o);
  }
  if (lane == 0) {
    const double len = lw[2 * shape[b]], W = lw[2 * shape[b] + 1];
    yU[3 * b] = U[3 * b] - sx / len;
    yU[3 * b + 1] = U[3 * b + 1] - sy / len;
    yU[3 * b + 2] = U[3 * b + 2] - st / W;
    part[2 * b] = q[2 * b] * fl + mx;
    part[2 * b + 1] = q[2 * b + 1] * fl + my;
  }
}

// the mean term's constant velocity: cm * sum over bodies of part (one block)
__global__ __launch_bounds__(256) void k_sk_mean(int n, const double *__restrict__ part, double cm,
                                                 double *__restrict__ mean) {
  __shared__ double sx[256], sy[256];
  double ax = 0, ay = 0;
  for (int b = threadIdx.x; b < n; b += 256) {
    ax += part[2 * b];
    ay += part[2 * b + 1];
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[0] = cm * sx[0];
    mean[1] = cm * sy[0];
  }
}

// y_phi = -phi/2 + D_out phi + U_b + omega_b r^perp, with
// D_out phi = real + wave + mean + cG diag phi (outward-normal double layer; the
// formulation's D is its negative, so -phi/2 - D phi = -phi/2 + D_out phi)
__global__ void k_sk_combine(int N, const int *__restrict__ body, const double2 *__restrict__ phi,
                             const double2 *__restrict__ real, const double2 *__restrict__ wave,
                             const double *__restrict__ mean, const double *__restrict__ diag, double cG,
                             const double2 *__restrict__ r, const double *__restrict__ U, double2 *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = body[i];
  const double2 p = phi[i], a = real[i], v = wave[i], rr = r[i];
  const double dx = diag[3 * i] * p.x + diag[3 * i + 1] * p.y, dy = diag[3 * i + 1] * p.x + diag[3 * i + 2] * p.y;
  const double ux = U[3 * b], uy = U[3 * b + 1], om = U[3 * b + 2];
  y[i] = make_double2(-0.5 * p.x + a.x + v.x + mean[0] + cG * dx + ux - om * rr.y,
                      -0.5 * p.y + a.y + v.y + mean[1] + cG * dy + uy + om * rr.x);
}

}  // namespace

hipError_t launch_sk_geom(const GeomDev &g, const double *const *sk6, const int *cperm, double *w, double *wc,
                          double *diag, double *ds, double *r, hipStream_t s) {
  if (g.N == 0) return hipSuccess;
  const dim3 grid((g.N + 255) / 256);
  hipLaunchKernelGGL(k_sk_geom, grid, dim3(256), 0, s, g.N, g.body, g.off, g.shape, g.theta, g.ref, sk6,
                     (double2 *)w, diag, ds, (double2 *)r);
  hipLaunchKernelGGL(k_gather_d2, grid, dim3(256), 0, s, g.N, cperm, (const double2 *)w, (double2 *)wc);
  return hipGetLastError();
}

hipError_t launch_sk_prep(int N, const int *tperm, const double *phi, const double *w, double *A, double *B,
                          hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sk_prep, dim3((N + 255) / 256), dim3(256), 0, s, N, tperm, (const double2 *)phi,
                     (const double2 *)w, (double2 *)A, (double2 *)B);
  return hipGetLastError();
}

hipError_t launch_point_spread(int n, const double *q, const double *F, const WaveArgs &w, double *grid,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (w.P * w.P > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_point_spread, dim3(n), dim3(256), 0, s, n, q, F, w.M, w.P, w.h, w.L, w.ag, w.cg, grid);
  return hipGetLastError();
}

hipError_t launch_sk_mult(int M, double L, double xi, double eta_s, double sc, int mode, double *spec,
                          hipStream_t s) {
  const int n = M * (M / 2 + 1);
  hipLaunchKernelGGL(k_sk_mult, dim3((n + 255) / 256), dim3(256), 0, s, M, 2.0 * M_PI / L, 1.0 / (4.0 * xi * xi),
                     1.0 - eta_s, sc, mode, (double2 *)spec);
  return hipGetLastError();
}

hipError_t launch_sk_body(const GeomDev &g, const double *lw, const double *phi, const double *w, const double *ds,
                          const double *r, const double *U, double *yU, double *part, double cm, double *mean,
                          hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sk_body, dim3(g.n), dim3(64), 0, s, g.off, g.shape, g.q, lw, (const double2 *)phi,
                     (const double2 *)w, ds, (const double2 *)r, U, yU, part);
  hipLaunchKernelGGL(k_sk_mean, dim3(1), dim3(256), 0, s, g.n, part, cm, mean);
  return hipGetLastError();
}

hipError_t launch_sk_combine(const GeomDev &g, const double *phi, const double *real, const double *wave,
                             const double *mean, const double *diag, double cG, const double *r, const double *U,
                             double *y, hipStream_t s) {
  if (g.N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sk_combine, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, g.body, (const double2 *)phi,
                     (const double2 *)real, (const double2 *)wave, mean, diag, cG, (const double2 *)r, U,
                     (double2 *)y);
  return hipGetLastError();
}

}  // namespace fbim
