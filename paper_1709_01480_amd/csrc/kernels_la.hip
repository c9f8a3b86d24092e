// Rigid-body maps K, K^T (Section 3.1), the block-diagonal preconditioner and
// the per-body G / G^+ applies (Section 3.4), and FP64 Krylov vector kernels.
#include <algorithm>

#include "kernels.h"

namespace fbim {

// y_mu[i] -= u_b + omega_b (-r_y, r_x),  r = R(theta_b) ref_t
__global__ void k_sub_KU(int N, const int *__restrict__ body, const int *__restrict__ off,
                         const int *__restrict__ shape, const double *__restrict__ theta,
                         const double *const *ref, const double *__restrict__ U, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = body[i];
  const int t = i - off[b];
  const double *r = ref[shape[b]];
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  const double rx = cs * r[2 * t] - sn * r[2 * t + 1];
  const double ry = sn * r[2 * t] + cs * r[2 * t + 1];
  const double w = U[3 * b + 2];
  y[2 * i] -= U[3 * b] - w * ry;
  y[2 * i + 1] -= U[3 * b + 1] + w * rx;
}

hipError_t launch_sub_KU(const GeomDev &g, const double *U, double *y, hipStream_t s) {
  if (g.N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub_KU, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, g.body, g.off, g.shape, g.theta,
                     g.ref, U, y);
  return hipGetLastError();
}

// out[b] = sgn * (sum mu, sum r x mu), one 64-lane work group per body
__global__ __launch_bounds__(64) void k_KT(const int *__restrict__ off, const int *__restrict__ shape,
                                           const double *__restrict__ theta, const double *const *ref,
                                           const double *__restrict__ mu, double sgn, double *__restrict__ out) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int a = off[b], e = off[b + 1];
  const double *r = ref[shape[b]];
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  double fx = 0, fy = 0, tq = 0;
  for (int i = a + lane; i < e; i += 64) {
    const int t = i - a;
    const double rx = cs * r[2 * t] - sn * r[2 * t + 1];
    const double ry = sn * r[2 * t] + cs * r[2 * t + 1];
    const double mx = mu[2 * i], my = mu[2 * i + 1];
    fx += mx;
    fy += my;
    tq += rx * my - ry * mx;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    fx += __shfl_down(fx, o);
    fy += __shfl_down(fy, o);
    tq += __shfl_down(tq, o);
  }
  if (lane == 0) {
    out[3 * b] = sgn * fx;
    out[3 * b + 1] = sgn * fy;
    out[3 * b + 2] = sgn * tq;
  }
}

hipError_t launch_KT(const GeomDev &g, const double *mu, double sgn, double *out, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_KT, dim3(g.n), dim3(64), 0, s, g.off, g.shape, g.theta, g.ref, mu, sgn, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ per-body dense operators
// Block-diagonal preconditioner (eqs. 3.31-3.37) with all bodies of a shape
// sharing M_ref^+: in the body frame a~ = R^T a,
//   c = M_ref^+ a~,  U_ref = -N_ref (R'^T b + K_ref^T c),  mu_ref = c + (M_ref^+ K_ref) U_ref,
// then mu = R mu_ref, U = R' U_ref.
__global__ __launch_bounds__(1024) void k_precond(const int *__restrict__ off, const int *__restrict__ shape,
                                                  const double *__restrict__ theta, const double *const *ref,
                                                  const int *__restrict__ np, const double *const *Mp,
                                                  const double *const *Pref, const double *const *Nt, int N,
                                                  const double *__restrict__ z, double *__restrict__ y) {
  __shared__ double at[1024];
  __shared__ double red[3][32];
  __shared__ double Ur[3];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int sh = shape[b];
  const int n2 = 2 * np[sh];
  const int base = off[b];
  const double *r = ref[sh];
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  if (tid < n2 / 2) {
    const double ax = z[2 * (base + tid)], ay = z[2 * (base + tid) + 1];
    at[2 * tid] = cs * ax + sn * ay;
    at[2 * tid + 1] = -sn * ax + cs * ay;
  }
  __syncthreads();
  double c = 0.0;
  if (tid < n2) {
    const double *A = Mp[sh];
    for (int k = 0; k < n2; ++k) c += A[(size_t)k * n2 + tid] * at[k];
  }
  // f = K_ref^T c
  double f0 = 0, f1 = 0, f2 = 0;
  if (tid < n2) {
    const int t = tid >> 1;
    if (tid & 1) {
      f1 = c;
      f2 = r[2 * t] * c;
    } else {
      f0 = c;
      f2 = -r[2 * t + 1] * c;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    f0 += __shfl_down(f0, o);
    f1 += __shfl_down(f1, o);
    f2 += __shfl_down(f2, o);
  }
  const int wv = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    red[0][wv] = f0;
    red[1][wv] = f1;
    red[2][wv] = f2;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0, s1 = 0, s2 = 0;
    const int nw = (blockDim.x + 63) / 64;
    for (int k = 0; k < nw; ++k) {
      s0 += red[0][k];
      s1 += red[1][k];
      s2 += red[2][k];
    }
    const double *bb = z + 2 * (size_t)N + 3 * (size_t)b;
    const double g0 = cs * bb[0] + sn * bb[1] + s0;  // R'^T b + K^T c
    const double g1 = -sn * bb[0] + cs * bb[1] + s1;
    const double g2 = bb[2] + s2;
    const double *Nm = Nt[sh];
    Ur[0] = -(Nm[0] * g0 + Nm[1] * g1 + Nm[2] * g2);
    Ur[1] = -(Nm[3] * g0 + Nm[4] * g1 + Nm[5] * g2);
    Ur[2] = -(Nm[6] * g0 + Nm[7] * g1 + Nm[8] * g2);
    double *yU = y + 2 * (size_t)N + 3 * (size_t)b;
    yU[0] = cs * Ur[0] - sn * Ur[1];
    yU[1] = sn * Ur[0] + cs * Ur[1];
    yU[2] = Ur[2];
  }
  __syncthreads();
  if (tid < n2) {
    const double *Pm = Pref[sh];
    at[tid] = c + Pm[tid] * Ur[0] + Pm[n2 + tid] * Ur[1] + Pm[2 * n2 + tid] * Ur[2];
  }
  __syncthreads();
  if (tid < n2 / 2) {
    const double mx = at[2 * tid], my = at[2 * tid + 1];
    y[2 * (base + tid)] = cs * mx - sn * my;
    y[2 * (base + tid) + 1] = sn * mx + cs * my;
  }
}

hipError_t launch_precond(const GeomDev &g, const BodyMats &m, const double *z, double *y, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const int threads = ((2 * m.max_np + 63) / 64) * 64;
  hipLaunchKernelGGL(k_precond, dim3(g.n), dim3(threads), 0, s, g.off, g.shape, g.theta, g.ref, g.np, m.Mp,
                     m.Pref, m.Nt, g.N, z, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_body_apply(const int *__restrict__ off, const int *__restrict__ shape,
                                                     const double *__restrict__ theta, const int *__restrict__ np,
                                                     const double *const *X, const double *__restrict__ x,
                                                     double *__restrict__ y) {
  __shared__ double at[1024];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int sh = shape[b];
  const int n2 = 2 * np[sh];
  const int base = off[b];
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  if (tid < n2 / 2) {
    const double ax = x[2 * (base + tid)], ay = x[2 * (base + tid) + 1];
    at[2 * tid] = cs * ax + sn * ay;
    at[2 * tid + 1] = -sn * ax + cs * ay;
  }
  __syncthreads();
  double c = 0.0;
  if (tid < n2) {
    const double *A = X[sh];
    for (int k = 0; k < n2; ++k) c += A[(size_t)k * n2 + tid] * at[k];
  }
  __syncthreads();
  if (tid < n2) at[tid] = c;
  __syncthreads();
  if (tid < n2 / 2) {
    const double mx = at[2 * tid], my = at[2 * tid + 1];
    y[2 * (base + tid)] = cs * mx - sn * my;
    y[2 * (base + tid) + 1] = sn * mx + cs * my;
  }
}

hipError_t launch_body_apply(const GeomDev &g, const BodyMats &m, int which, const double *x, double *y,
                             hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const int threads = ((2 * m.max_np + 63) / 64) * 64;
  hipLaunchKernelGGL(k_body_apply, dim3(g.n), dim3(threads), 0, s, g.off, g.shape, g.theta, g.np,
                     which ? m.Gp : m.G, x, y);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Krylov vector kernels
constexpr int kDotCols = 8;

// Column sums of a block-partial array partial[j * nblk + b] by the last block to
// finish (fixed summation order, so the result is deterministic).
__device__ void last_block_reduce(double *__restrict__ partial, int nblk, int k, unsigned *__restrict__ counter,
                                  double *__restrict__ out) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = wv; j < k; j += nw) {
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64)
      s += __hip_atomic_load(&partial[(size_t)j * nblk + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if (lane == 0) out[j] = s;
  }
  if (threadIdx.x == 0) *counter = 0u;  // ready for the next launch on this stream
}

// out[j] = V[:, j]^T w for j < k, and out[k] = w^T w if with_norm
__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ V, size_t ld, int k,
                                              const double *__restrict__ w, size_t n, int with_norm,
                                              const double *__restrict__ cond, double *__restrict__ partial,
                                              unsigned *__restrict__ counter, double *__restrict__ out) {
  __shared__ double red[kDotCols][4];
  if (cond && cond[0] == 0.0) return;  // conditional pass not requested
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kk = k + (with_norm ? 1 : 0);
  for (int j0 = 0; j0 < kk; j0 += kDotCols) {
    double acc[kDotCols];
#pragma unroll
    for (int c = 0; c < kDotCols; ++c) acc[c] = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + tid; i < n; i += (size_t)gridDim.x * 256) {
      const double wi = w[i];
#pragma unroll
      for (int c = 0; c < kDotCols; ++c) {
        const int j = j0 + c;
        if (j < k)
          acc[c] += V[(size_t)j * ld + i] * wi;
        else if (j == k && with_norm)
          acc[c] += wi * wi;
      }
    }
#pragma unroll
    for (int c = 0; c < kDotCols; ++c) {
      double v = acc[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
      if (lane == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (tid < kDotCols && j0 + tid < kk)
      partial[(size_t)(j0 + tid) * gridDim.x + blockIdx.x] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
    __syncthreads();
  }
  last_block_reduce(partial, gridDim.x, kk, counter, out);
}

hipError_t launch_dots(const double *V, size_t ld, int k, const double *w, size_t n, int with_norm,
                       const double *cond, double *partial, int nblk, unsigned *counter, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(nblk), dim3(256), 0, s, V, ld, k, w, n, with_norm, cond, partial, counter, out);
  return hipGetLastError();
}

// w[i] -= sum_j V[j*ld + i] h[j]; nrm[0] = ||w||^2 afterwards and, if before is
// given, nrm[1] = 1 when nrm[0] < before[0] / 2 (a second pass is needed), else 0
__global__ __launch_bounds__(256) void k_sub_Vh(const double *__restrict__ V, size_t ld, int k,
                                                const double *__restrict__ h, double *__restrict__ w, size_t n,
                                                const double *__restrict__ cond, const double *__restrict__ before,
                                                double *__restrict__ partial, unsigned *__restrict__ counter,
                                                double *__restrict__ nrm) {
  __shared__ double red[4];
  __shared__ double hs[512];
  const int tid = threadIdx.x;
  if (cond && cond[0] == 0.0) return;
  for (int j = tid; j < k && j < 512; j += 256) hs[j] = h[j];
  __syncthreads();
  double acc2 = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + tid; i < n; i += (size_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += V[(size_t)j * ld + i] * hs[j];
    const double v = w[i] - acc;
    w[i] = v;
    acc2 += v * v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc2 += __shfl_down(acc2, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc2;
  __syncthreads();
  if (tid == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  last_block_reduce(partial, gridDim.x, 1, counter, nrm);
}

// flag[0] = nrm[0] < before[0] / 2 ? 1 : 0
__global__ void k_need_second_pass(const double *__restrict__ nrm, const double *__restrict__ before,
                                   double *__restrict__ flag) {
  flag[0] = nrm[0] < 0.5 * before[0] ? 1.0 : 0.0;
}

hipError_t launch_sub_Vh(const double *V, size_t ld, int k, const double *h, double *w, size_t n,
                         const double *cond, double *partial, int nblk, unsigned *counter, double *nrm,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sub_Vh, dim3(nblk), dim3(256), 0, s, V, ld, k, h, w, n, cond, (const double *)nullptr,
                     partial, counter, nrm);
  return hipGetLastError();
}

hipError_t launch_need_second_pass(const double *nrm, const double *before, double *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_need_second_pass, dim3(1), dim3(1), 0, s, nrm, before, flag);
  return hipGetLastError();
}

__global__ void k_Vc(const double *__restrict__ V, size_t ld, int k, const double *__restrict__ c,
                     double *__restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += V[(size_t)j * ld + i] * c[j];
    y[i] = acc;
  }
}

hipError_t launch_Vc(const double *V, size_t ld, int k, const double *c, double *y, size_t n, hipStream_t s) {
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_Vc, dim3(nb), dim3(256), 0, s, V, ld, k, c, y, n);
  return hipGetLastError();
}

__global__ void k_axpby(size_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

hipError_t launch_axpby(size_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(256), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

__global__ void k_scale_copy(size_t n, const double *__restrict__ x, const double *__restrict__ alpha, int invert,
                             double *__restrict__ y) {
  const double a = invert ? 1.0 / sqrt(alpha[0]) : alpha[0];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// invert != 0: y = x / sqrt(alpha[0]) (normalise by a squared norm kept on the device)
hipError_t launch_scale_copy(size_t n, const double *x, const double *alpha_dev, int invert, double *y,
                             hipStream_t s) {
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scale_copy, dim3(nb), dim3(256), 0, s, n, x, alpha_dev, invert, y);
  return hipGetLastError();
}

__global__ void k_vec_add(int k, const double *__restrict__ a, double *__restrict__ b) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) b[j] += a[j];
}

hipError_t launch_vec_add(int k, const double *a, double *b, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_add, dim3((k + 63) / 64), dim3(64), 0, s, k, a, b);
  return hipGetLastError();
}

__global__ void k_fill(size_t n, double v, double *__restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = v;
}

hipError_t launch_fill(size_t n, double v, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, n, v, y);
  return hipGetLastError();
}

__global__ void k_fill_int(size_t n, int v, int *__restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = v;
}

hipError_t launch_fill_int(size_t n, int v, int *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill_int, dim3(nb), dim3(256), 0, s, n, v, y);
  return hipGetLastError();
}

__global__ void k_cast_f32(size_t n, const double *__restrict__ x, float *__restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

hipError_t launch_cast_f32(size_t n, const double *x, float *y, hipStream_t s) {
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_cast_f32, dim3(nb), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

}  // namespace fbim
