// Learned correction of the block-diagonal preconditioner: per-body features,
// a 32 -> 128 -> 128 -> 6 tanh MLP whose matrix products run on the MFMA units
// in BF16 with FP32 accumulation, its backward pass, the regression loss and
// Adam.
//
// The network maps each body's neighbourhood (body frame) to a symmetric
// correction dN of the isolated-body mobility N_ref used by the preconditioner
// (eqs. 3.31-3.37).  It is trained on solves of the method itself: for random
// forces F with independent unit components, the mobility solve gives U = N F,
// and E[U_b F_b^T] = N_bb, the body's own mobility block in the suspension, so
// least squares of (N_ref + dN_b) F_b against U_b targets N_bb - N_ref.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace fbim {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even (finite inputs)
__device__ inline short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

}  // namespace

// ------------------------------------------------------------------ features
// Neighbours: bodies whose centre lies within R_nb = 3 r_max (minimum image),
// nearest first (ties by index), at most kMlpNeighbours.  Bodies are binned
// into cells of side >= R_nb (k_body_keys, then the generic scan and scatter),
// and one thread per body visits the 3 x 3 cells around its own (all bodies
// when there are fewer than three cells per side).  The order of the visit
// does not matter: the neighbour ranking is a total order.
__global__ void k_body_keys(int n, const double *__restrict__ q, double L, int nbc, int *__restrict__ key,
                            int *__restrict__ count) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double x = q[2 * b] - L * floor(q[2 * b] / L), y = q[2 * b + 1] - L * floor(q[2 * b + 1] / L);
  const int cx = min(max((int)(x * nbc / L), 0), nbc - 1), cy = min(max((int)(y * nbc / L), 0), nbc - 1);
  key[b] = cy * nbc + cx;
  atomicAdd(&count[cy * nbc + cx], 1);
}

__global__ __launch_bounds__(256) void k_mlp_features(int n, const double *__restrict__ q,
                                                      const double *__restrict__ theta, double L, double r_max,
                                                      int sym, int nbc, const int *__restrict__ key,
                                                      const int *__restrict__ start, const int *__restrict__ perm,
                                                      float *__restrict__ X) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double R = 3.0 * r_max;
  const double qx = q[2 * b], qy = q[2 * b + 1];
  double bd[kMlpNeighbours];
  int bi[kMlpNeighbours];
#pragma unroll
  for (int k = 0; k < kMlpNeighbours; ++k) {
    bd[k] = 1e300;
    bi[k] = -1;
  }
  int count = 0;
  const int kb = key[b], bx = kb % nbc, by = kb / nbc;
  const int span = nbc >= 3 ? 1 : 0;  // fewer than three cells: one cell holds everything
  for (int oy = -span; oy <= span; ++oy)
    for (int ox = -span; ox <= span; ++ox) {
      const int cell = ((by + oy + nbc) % nbc) * nbc + (bx + ox + nbc) % nbc;
      for (int e = start[cell]; e < start[cell + 1]; ++e) {
        const int c = perm[e];
        if (c == b) continue;
        double dx = q[2 * c] - qx, dy = q[2 * c + 1] - qy;
        dx -= L * rint(dx / L);
        dy -= L * rint(dy / L);
        const double d = sqrt(dx * dx + dy * dy);
        if (d >= R) continue;
        ++count;
        // insert (d, c) into the sorted list
        double cd = d;
        int ci = c;
#pragma unroll
        for (int k = 0; k < kMlpNeighbours; ++k) {
          const bool less = cd < bd[k] || (cd == bd[k] && ci < bi[k]);
          if (less) {
            const double td = bd[k];
            const int ti = bi[k];
            bd[k] = cd;
            bi[k] = ci;
            cd = td;
            ci = ti;
          }
        }
      }
    }
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  float *f = X + (size_t)b * kMlpIn;
#pragma unroll
  for (int k = 0; k < kMlpNeighbours; ++k) {
    float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (bi[k] >= 0) {
      const int c = bi[k];
      double dx = q[2 * c] - qx, dy = q[2 * c + 1] - qy;
      dx -= L * rint(dx / L);
      dy -= L * rint(dy / L);
      const double ux = cs * dx + sn * dy, uy = -sn * dx + cs * dy;
      double s2, c2;
      sincos(sym * (theta[c] - theta[b]), &s2, &c2);
      v[0] = (float)(ux / R);
      v[1] = (float)(uy / R);
      v[2] = (float)(r_max / bd[k]);
      v[3] = (float)c2;
      v[4] = (float)s2;
    }
#pragma unroll
    for (int e = 0; e < 5; ++e) f[5 * k + e] = v[e];
  }
  f[30] = (float)count / (float)kMlpNeighbours;
  const double dmin = bi[0] >= 0 ? bd[0] : R;
  f[31] = (float)fmin(2.0, fmax(-2.0, (dmin - 2.0 * r_max) / r_max));
}

int mlp_body_cells(double L, double r_max) {
  const int nbc = (int)std::floor(L / (3.0 * r_max));
  return nbc >= 3 ? std::min(nbc, 256) : 1;  // cells of side >= R_nb; the scan is one work group
}

hipError_t launch_mlp_features(int n, const double *q, const double *theta, double L, double r_max, int sym,
                               const MlpCells &cells, float *X, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nbc = cells.nbc, nc = nbc * nbc;
  hipError_t e = launch_fill_int((size_t)nc, 0, cells.count, s);
  if (e != hipSuccess) return e;
  e = launch_fill_int((size_t)nc, 0, cells.cursor, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_body_keys, dim3((n + 255) / 256), dim3(256), 0, s, n, q, L, nbc, cells.key, cells.count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_scan(nc, cells.count, cells.start, cells.maxcount, s)) != hipSuccess) return e;
  if ((e = launch_scatter(n, cells.key, cells.start, cells.cursor, cells.perm, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_features, dim3((n + 255) / 256), dim3(256), 0, s, n, q, theta, L, r_max, sym, nbc,
                     cells.key, cells.start, cells.perm, X);
  return hipGetLastError();
}

// ------------------------------------------------------------------ BF16 MFMA GEMM
// C[M x N] = op(A)[M x K] op(B)[K x N], A(i, k) = A[i * sam + k * sak], B(k, j) = B[k * sbk + j * sbn]
// (strides express the transposes).  64 x 64 tile per 256-thread work group,
// each wave a 32 x 32 quarter as 2 x 2 v_mfma_f32_16x16x16_bf16 blocks; K in
// steps of 16 staged through LDS as BF16.  blockIdx.z splits K (epilogue
// kGemmAtomic adds into C).
// MFMA operand layout (16 x 16 x 16): lane l holds A(l % 16, 4 (l / 16) + r) and
// B(4 (l / 16) + r, l % 16) for r < 4, and receives D(4 (l / 16) + r, l % 16).
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ short As[64][16 + 4];  // [i][k], rows padded
  __shared__ short Bs[64][16 + 4];  // [j][k]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kc = (g.K + (int)gridDim.z - 1) / (int)gridDim.z;
  const int kb = blockIdx.z * ((kc + 15) / 16) * 16;
  const int ke = min(g.K, kb + ((kc + 15) / 16) * 16);
  const int wm = wv >> 1, wn = wv & 1;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    // stage: 64 x 16 elements of each operand, 4 per thread
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e;
      const int r = idx >> 4, k = idx & 15;
      const int gi = m0 + r, gk = k0 + k;
      const float av = (gi < g.M && gk < ke) ? g.A[(size_t)gi * g.sam + (size_t)gk * g.sak] : 0.f;
      As[r][k] = to_bf16(av);
      const int gj = n0 + r;
      const float bv = (gj < g.N && gk < ke) ? g.B[(size_t)gk * g.sbk + (size_t)gj * g.sbn] : 0.f;
      Bs[r][k] = to_bf16(bv);
    }
    __syncthreads();
    bf16x4 av[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int row = 32 * wm + 16 * t + (lane & 15);
      const int col = 32 * wn + 16 * t + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        av[t][r] = As[row][4 * (lane >> 4) + r];
        bv[t][r] = Bs[col][4 * (lane >> 4) + r];
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + 32 * wm + 16 * a + 4 * (lane >> 4) + r;
        const int j = n0 + 32 * wn + 16 * b + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        float v = acc[a][b][r];
        float *c = g.C + (size_t)i * g.ldc + j;
        switch (g.epi) {
          case kGemmStore: *c = v; break;
          case kGemmBiasTanh: *c = tanhf(v + g.bias[j]); break;
          case kGemmBias: *c = v + g.bias[j]; break;
          case kGemmAtomic: atomicAdd(c, v); break;
          case kGemmTanhGrad: {
            const float h = g.aux[(size_t)i * g.ldc + j];
            *c = v * (1.f - h * h);
            break;
          }
        }
      }
}

hipError_t launch_gemm_bf16(const GemmArgs &g, int ksplit, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (ksplit < 1 || (ksplit > 1 && g.epi != kGemmAtomic)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm_bf16, dim3((g.N + 63) / 64, (g.M + 63) / 64, ksplit), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ loss
// Per body b and sample s, body frame (R_b^T on the translational part):
//   r = (N_ref + dN(Y_b)) F~ - U~,   loss = mean over (s, b) of sum_i (r_i / N_ref,ii)^2
// dN(Y) = [[y0 sx, y3 sxy, y4 sxt], [y3 sxy, y1 sy, y5 syt], [y4 sxt, y5 syt, y2 st]]
// with s. = diagonal of N_ref and sxy = sqrt(sx sy) etc.  dY = d loss / d Y.
__global__ __launch_bounds__(256) void k_mlp_loss(int n, int ns, const int *__restrict__ shape,
                                                  const double *__restrict__ theta, const double *const *Nt,
                                                  const float *__restrict__ Y, const double *__restrict__ F,
                                                  const double *__restrict__ U, float *__restrict__ dY,
                                                  float *__restrict__ loss) {
  __shared__ float red[4];
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  float lsum = 0.f;
  if (b < n) {
    const double *Nm = Nt[shape[b]];
    const double sx = Nm[0], sy = Nm[4], st = Nm[8];
    const double sxy = sqrt(sx * sy), sxt = sqrt(sx * st), syt = sqrt(sy * st);
    const float *y = Y + 6 * (size_t)b;
    double Nb[3][3];
    Nb[0][0] = Nm[0] + y[0] * sx;
    Nb[1][1] = Nm[4] + y[1] * sy;
    Nb[2][2] = Nm[8] + y[2] * st;
    Nb[0][1] = Nm[1] + y[3] * sxy;
    Nb[1][0] = Nm[3] + y[3] * sxy;
    Nb[0][2] = Nm[2] + y[4] * sxt;
    Nb[2][0] = Nm[6] + y[4] * sxt;
    Nb[1][2] = Nm[5] + y[5] * syt;
    Nb[2][1] = Nm[7] + y[5] * syt;
    const double w[3] = {1.0 / (sx * sx), 1.0 / (sy * sy), 1.0 / (st * st)};
    double sn, cs;
    sincos(theta[b], &sn, &cs);
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double l = 0.0;
    const double norm = 1.0 / ((double)ns * n);
    for (int s = 0; s < ns; ++s) {
      const double *f = F + (size_t)s * 3 * n + 3 * (size_t)b;
      const double *u = U + (size_t)s * 3 * n + 3 * (size_t)b;
      const double ft[3] = {cs * f[0] + sn * f[1], -sn * f[0] + cs * f[1], f[2]};
      const double ut[3] = {cs * u[0] + sn * u[1], -sn * u[0] + cs * u[1], u[2]};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double r = Nb[i][0] * ft[0] + Nb[i][1] * ft[1] + Nb[i][2] * ft[2] - ut[i];
        l += w[i] * r * r;
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] += 2.0 * w[i] * r * ft[j];
      }
    }
    lsum = (float)(l * norm);
    float *d = dY + 6 * (size_t)b;
    d[0] = (float)(G[0][0] * sx * norm);
    d[1] = (float)(G[1][1] * sy * norm);
    d[2] = (float)(G[2][2] * st * norm);
    d[3] = (float)((G[0][1] + G[1][0]) * sxy * norm);
    d[4] = (float)((G[0][2] + G[2][0]) * sxt * norm);
    d[5] = (float)((G[1][2] + G[2][1]) * syt * norm);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_down(lsum, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1]) + (red[2] + red[3]));
}

hipError_t launch_mlp_loss(int n, int ns, const int *shape, const double *theta, const double *const *Nt,
                           const float *Y, const double *F, const double *U, float *dY, float *loss, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_loss, dim3((n + 255) / 256), dim3(256), 0, s, n, ns, shape, theta, Nt, Y, F, U, dY, loss);
  return hipGetLastError();
}

// dN[b] (FP64, [n][6]) from the network output: xx, yy, tt, xy, xt, yt
__global__ void k_mlp_correction(int n, const int *__restrict__ shape, const double *const *Nt,
                                 const float *__restrict__ Y, double *__restrict__ dN) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double *Nm = Nt[shape[b]];
  const double sx = Nm[0], sy = Nm[4], st = Nm[8];
  const float *y = Y + 6 * (size_t)b;
  double *d = dN + 6 * (size_t)b;
  d[0] = y[0] * sx;
  d[1] = y[1] * sy;
  d[2] = y[2] * st;
  d[3] = y[3] * sqrt(sx * sy);
  d[4] = y[4] * sqrt(sx * st);
  d[5] = y[5] * sqrt(sy * st);
}

hipError_t launch_mlp_correction(int n, const int *shape, const double *const *Nt, const float *Y, double *dN,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_correction, dim3((n + 255) / 256), dim3(256), 0, s, n, shape, Nt, Y, dN);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Adam (Kingma & Ba), bias-corrected
__global__ void k_adam(int n, float lr, float b1, float b2, float eps, float c1, float c2, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(int n, float lr, float b1, float b2, float eps, int t, const float *g, float *m, float *v,
                       float *w, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, n, lr, b1, b2, eps, c1, c2, g, m, v, w);
  return hipGetLastError();
}

__global__ void k_fill_f32(size_t n, float v, float *__restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = v;
}

hipError_t launch_fill_f32(size_t n, float v, float *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_f32, dim3(nb), dim3(256), 0, s, n, v, y);
  return hipGetLastError();
}

}  // namespace fbim
