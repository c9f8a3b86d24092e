// Rigid-body maps K, K^T (Section 3.1), the block-diagonal preconditioner and
// the per-body G / G^+ applies (Section 3.4), and FP64 Krylov vector kernels.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <type_traits>

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

// batched saddle rigid-body terms: y_mu -= K x_U over the nodes, then
// y_U = -K^T x_mu with one wave per body (4 bodies per 256-thread block)
__device__ __forceinline__ void sub_KU_batch_body(const RigidJob *__restrict__ jobs, const BatchGrid &bg, int blk) {
  const int s = batch_system(bg.begin, bg.S, blk);
  const RigidJob &j = jobs[s];
  const GeomDev &g = j.g;
  const int i = (blk - bg.begin[s]) * 256 + threadIdx.x;
  if (i >= g.N) return;
  const int b = g.body[i];
  const int t = i - g.off[b];
  const double *r = g.ref[g.shape[b]];
  double sn, cs;
  sincos(g.theta[b], &sn, &cs);
  const double rx = cs * r[2 * t] - sn * r[2 * t + 1];
  const double ry = sn * r[2 * t] + cs * r[2 * t + 1];
  const double *U = j.x + 2 * (size_t)g.N;
  const double w = U[3 * b + 2];
  j.y[2 * i] -= U[3 * b] - w * ry;
  j.y[2 * i + 1] -= U[3 * b + 1] + w * rx;
}

__device__ __forceinline__ void KT_batch_body(const RigidJob *__restrict__ jobs, const BatchGrid &bg, int blk) {
  const int s = batch_system(bg.begin, bg.S, blk);
  const RigidJob &j = jobs[s];
  const GeomDev &g = j.g;
  const int b = (blk - bg.begin[s]) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= g.n) return;  // whole wave
  const int a = g.off[b], e = g.off[b + 1];
  const double *r = g.ref[g.shape[b]];
  double sn, cs;
  sincos(g.theta[b], &sn, &cs);
  double fx = 0, fy = 0, tq = 0;
  for (int i = a + lane; i < e; i += 64) {
    const int t = i - a;
    const double rx = cs * r[2 * t] - sn * r[2 * t + 1];
    const double ry = sn * r[2 * t] + cs * r[2 * t + 1];
    const double mx = j.x[2 * i], my = j.x[2 * i + 1];
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
    double *out = j.y + 2 * (size_t)g.N + 3 * (size_t)b;
    out[0] = -fx;
    out[1] = -fy;
    out[2] = -tq;
  }
}

// the two rigid-body maps of the saddle operator touch disjoint rows of y and read
// only x: one launch, the node blocks first, then the body blocks
__global__ __launch_bounds__(256) void k_rigid_batch(const RigidJob *__restrict__ jobs, BatchGrid bg_nodes,
                                                     BatchGrid bg_bodies) {
  if ((int)blockIdx.x < bg_nodes.nblocks)
    sub_KU_batch_body(jobs, bg_nodes, blockIdx.x);
  else
    KT_batch_body(jobs, bg_bodies, blockIdx.x - bg_nodes.nblocks);
}

hipError_t launch_rigid_batch(const RigidJob *jobs, BatchGrid bg_nodes, BatchGrid bg_bodies, hipStream_t s) {
  const int nb = bg_nodes.nblocks + bg_bodies.nblocks;
  if (nb > 0) hipLaunchKernelGGL(k_rigid_batch, dim3(nb), dim3(256), 0, s, jobs, bg_nodes, bg_bodies);
  return hipGetLastError();
}

// ------------------------------------------------------------------ per-body dense operators
// All bodies of a shape share their reference matrices, so in the body frame the
// per-body products are one matrix times a batch of vectors: C = X A with X the
// shared (2 n_p) x (2 n_p) matrix and A the body-frame inputs of a tile of up to
// body_tile_cap(2 n_p) bodies of one shape, one column per body.  A work group
// rotates its bodies' inputs into A (LDS, k-major), streams X through LDS in
// chunks of body_tile_kc rows (the two chunks after the current one are in flight
// in registers while it is used), and each thread accumulates a 4 x 4 block of C
// (four rows, four bodies) in registers; then it finishes each body.
//
// MODE 0: y_b = R_b X_ref R_b^T x_b, X = G_ref or G_ref^+ (eqs. 3.40-3.42).
// MODE 1: block-diagonal preconditioner (eqs. 3.31-3.37): in the body frame
//   c = M_ref^+ a~,  U_ref = -N_ref (R'^T b + K_ref^T c),  mu_ref = c + (M_ref^+ K_ref) U_ref,
//   mu = R mu_ref, U = R' U_ref.  With a learned symmetric correction C = dN_b
//   (body frame) it applies the exact inverse of the body block whose M_bb is
//   replaced by M_bb + K C K^T: by the Woodbury identity that body's mobility
//   becomes N_ref + C, mu is unchanged and U_ref gains -C R'^T b.
template <int MODE>
__device__ __forceinline__ void body_tile(const BodyTiles &bt, int tile, const int *__restrict__ off,
                                          const double *__restrict__ theta, const double *const *ref,
                                          const int *__restrict__ np, const double *const *X,
                                          const double *const *Pref, const double *const *Nt,
                                          const double *__restrict__ dN, int N, const double *__restrict__ z,
                                          double *__restrict__ y) {
  extern __shared__ double sm[];  // A (n2 x NB, k-major), later C ([NB][n2]); then the X chunk (KC x n2)
  __shared__ double cs_[kBodyTileMax], sn_[kBodyTileMax];
  __shared__ int base_[kBodyTileMax], body_[kBodyTileMax];
  // MODE 1: rigid-body data per body, the shape's reference nodes and N_ref
  __shared__ double Ur[MODE == 1 ? kBodyTileMax : 1][3], bb_[MODE == 1 ? kBodyTileMax : 1][3];
  __shared__ double dn_[MODE == 1 ? kBodyTileMax : 1][6], f_[MODE == 1 ? kBodyTileMax : 1][3];
  __shared__ double rf_[MODE == 1 ? 1024 : 1], Nm_[9];
  const int4 tl = bt.tile[tile];
  const int sh = tl.x, nb = tl.z;
  const int npt = np[sh], n2 = 2 * npt;
  const int NB = body_tile_cap(n2), KC = body_tile_kc(n2);
  double *__restrict__ Xs = sm + (size_t)n2 * NB;
  const int tid = threadIdx.x;
  // the first matrix chunk is requested before anything else (KC * n2 <= 2048:
  // at most 1024 double2, four per thread)
  const double2 *__restrict__ A2 = reinterpret_cast<const double2 *>(X[sh]);
  // two chunks in flight: p0..p3 hold the chunk stored next, p4..p7 the one after
  double2 p0 = make_double2(0.0, 0.0), p1 = p0, p2 = p0, p3 = p0, p4 = p0, p5 = p0, p6 = p0, p7 = p0;
  int lim = min(KC, n2) * n2 / 2;
  int lim1 = max(0, min(KC, n2 - KC)) * n2 / 2;
  if (tid < lim) p0 = A2[tid];
  if (tid + 256 < lim) p1 = A2[tid + 256];
  if (tid + 512 < lim) p2 = A2[tid + 512];
  if (tid + 768 < lim) p3 = A2[tid + 768];
  {
    const double2 *__restrict__ src = A2 + (size_t)KC * n2 / 2;
    if (tid < lim1) p4 = src[tid];
    if (tid + 256 < lim1) p5 = src[tid + 256];
    if (tid + 512 < lim1) p6 = src[tid + 512];
    if (tid + 768 < lim1) p7 = src[tid + 768];
  }
  if (tid < nb) {
    const int b = bt.list[tl.y + tid];
    double sn, cs;
    sincos(theta[b], &sn, &cs);
    cs_[tid] = cs;
    sn_[tid] = sn;
    base_[tid] = off[b];
    body_[tid] = b;
    if (MODE == 1) {  // the body's rigid-body right-hand side and its correction (zero without one)
      const double *bb = z + 2 * (size_t)N + 3 * (size_t)b;
      bb_[tid][0] = bb[0];
      bb_[tid][1] = bb[1];
      bb_[tid][2] = bb[2];
#pragma unroll
      for (int q = 0; q < 6; ++q) dn_[tid][q] = dN ? dN[6 * (size_t)b + q] : 0.0;
    }
  }
  if (MODE == 1) {
    if (tid < 9) Nm_[tid] = Nt[sh][tid];
    for (int i = tid; i < n2; i += 256) rf_[i] = ref[sh][i];
  }
  __syncthreads();
  // body-frame inputs into A, four elements per thread in flight
  for (int i0 = 0; i0 < NB * npt; i0 += 1024) {
    double zx[4], zy[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = i0 + q * 256 + tid;
      const int j = idx / npt, t = idx - j * npt;
      zx[q] = zy[q] = 0.0;
      if (idx < NB * npt && j < nb) {
        const size_t gi = 2 * (size_t)(base_[j] + t);
        zx[q] = z[gi];
        zy[q] = z[gi + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = i0 + q * 256 + tid;
      const int j = idx / npt, t = idx - j * npt;
      if (idx < NB * npt) {
        const double c = j < nb ? cs_[j] : 0.0, sn = j < nb ? sn_[j] : 0.0;
        sm[(2 * t) * NB + j] = c * zx[q] + sn * zy[q];
        sm[(2 * t + 1) * NB + j] = -sn * zx[q] + c * zy[q];
      }
    }
  }
  // C = X A: thread (rq, jq) owns rows rq + m n2 / 4 (m < 4) and bodies 4 jq .. 4 jq + 3
  // (X is stored k-major: X[k * n2 + r] multiplies input k of output r)
  const int RQ = n2 / 4, JQ = NB / 4;
  const int rq = tid % RQ, jq = tid / RQ;
  const bool active = jq < JQ;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[r][b] = 0.0;
  double2 *__restrict__ X2 = reinterpret_cast<double2 *>(Xs);
  for (int kc = 0; kc < n2; kc += KC) {
    __syncthreads();  // the previous chunk has been used (and A is complete)
    if (tid < lim) X2[tid] = p0;
    if (tid + 256 < lim) X2[tid + 256] = p1;
    if (tid + 512 < lim) X2[tid + 512] = p2;
    if (tid + 768 < lim) X2[tid + 768] = p3;
    __syncthreads();
    p0 = p4;
    p1 = p5;
    p2 = p6;
    p3 = p7;
    lim = lim1;
    if (kc + 2 * KC < n2) {  // fetch the chunk after next while this one is used
      const double2 *__restrict__ src = A2 + (size_t)(kc + 2 * KC) * n2 / 2;
      lim1 = min(KC, n2 - kc - 2 * KC) * n2 / 2;
      if (tid < lim1) p4 = src[tid];
      if (tid + 256 < lim1) p5 = src[tid + 256];
      if (tid + 512 < lim1) p6 = src[tid + 512];
      if (tid + 768 < lim1) p7 = src[tid + 768];
    } else {
      lim1 = 0;
    }
    if (active) {
      const int kn = min(KC, n2 - kc);
      for (int kk = 0; kk < kn; ++kk) {
        // rows rq + m RQ: consecutive lanes read consecutive doubles (no bank conflicts)
        const double *xr = &Xs[kk * n2 + rq];
        const double2 a01 = *reinterpret_cast<const double2 *>(&sm[(kc + kk) * NB + 4 * jq]);
        const double2 a23 = *reinterpret_cast<const double2 *>(&sm[(kc + kk) * NB + 4 * jq + 2]);
        const double xv[4] = {xr[0], xr[RQ], xr[2 * RQ], xr[3 * RQ]}, av[4] = {a01.x, a01.y, a23.x, a23.y};
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[r][b] = fma(xv[r], av[b], acc[r][b]);
      }
    }
  }
  __syncthreads();  // every thread is done reading A
  if (active) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double *row = &sm[(size_t)(4 * jq + b) * n2 + rq];
#pragma unroll
      for (int r = 0; r < 4; ++r) row[r * RQ] = acc[r][b];
    }
  }
  __syncthreads();
  if (MODE == 1) {
    // per body: f = K_ref^T c (one wave per body), then U_ref = -N_ref (R'^T b + f)
    // (one thread per body)
    const int lane = tid & 63, wv = tid >> 6;
    for (int j = wv; j < nb; j += 4) {
      double f0 = 0, f1 = 0, f2 = 0;
      for (int t = lane; t < npt; t += 64) {
        const double c0 = sm[j * n2 + 2 * t], c1 = sm[j * n2 + 2 * t + 1];
        f0 += c0;
        f1 += c1;
        f2 += rf_[2 * t] * c1 - rf_[2 * t + 1] * c0;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        f0 += __shfl_down(f0, o);
        f1 += __shfl_down(f1, o);
        f2 += __shfl_down(f2, o);
      }
      if (lane == 0) {
        f_[j][0] = f0;
        f_[j][1] = f1;
        f_[j][2] = f2;
      }
    }
    __syncthreads();
    if (tid < nb) {
      const int j = tid, b = body_[j];
      const double cs = cs_[j], sn = sn_[j];
      const double b0 = cs * bb_[j][0] + sn * bb_[j][1], b1 = -sn * bb_[j][0] + cs * bb_[j][1], b2 = bb_[j][2];
      const double g0 = b0 + f_[j][0], g1 = b1 + f_[j][1], g2 = b2 + f_[j][2];
      const double u0 = -(Nm_[0] * g0 + Nm_[1] * g1 + Nm_[2] * g2);
      const double u1 = -(Nm_[3] * g0 + Nm_[4] * g1 + Nm_[5] * g2);
      const double u2 = -(Nm_[6] * g0 + Nm_[7] * g1 + Nm_[8] * g2);
      Ur[j][0] = u0;
      Ur[j][1] = u1;
      Ur[j][2] = u2;
      // learned correction C = dN_b (xx, yy, tt, xy, xt, yt): the exact inverse of
      // the body block with M_bb replaced by M_bb + K C K^T keeps mu and adds
      // -C R'^T b to U
      const double *d = dn_[j];
      const double v0 = u0 - (d[0] * b0 + d[3] * b1 + d[4] * b2);
      const double v1 = u1 - (d[3] * b0 + d[1] * b1 + d[5] * b2);
      const double v2 = u2 - (d[4] * b0 + d[5] * b1 + d[2] * b2);
      double *yU = y + 2 * (size_t)N + 3 * (size_t)b;
      yU[0] = cs * v0 - sn * v1;
      yU[1] = sn * v0 + cs * v1;
      yU[2] = v2;
    }
    // mu_ref = c + (M_ref^+ K_ref) U_ref: each thread keeps its rows of P
    const double *Pm = Pref[sh];
    double q0[4], q1[4], q2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = tid + 256 * m;
      q0[m] = q1[m] = q2[m] = 0.0;
      if (r < n2) {
        q0[m] = Pm[r];
        q1[m] = Pm[n2 + r];
        q2[m] = Pm[2 * n2 + r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = tid + 256 * m;
      if (r < n2)
        for (int j = 0; j < nb; ++j) sm[j * n2 + r] += q0[m] * Ur[j][0] + q1[m] * Ur[j][1] + q2[m] * Ur[j][2];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * npt; idx += 256) {
    const int j = idx / npt, t = idx - j * npt;
    const double mx = sm[j * n2 + 2 * t], my = sm[j * n2 + 2 * t + 1];
    const size_t gi = 2 * (size_t)(base_[j] + t);
    y[gi] = cs_[j] * mx - sn_[j] * my;
    y[gi + 1] = sn_[j] * mx + cs_[j] * my;
  }
}

// The same operators on the FP64 matrix cores, 16 bodies per 256-thread work
// group (columns of one 16 x 16 x 4 MFMA block).  MODE 1 forms the rigid-body
// part before the product: with M_ref^+ symmetric, f = K_ref^T M_ref^+ a~ =
// P_ref^T a~ (P_ref = M_ref^+ K_ref), so U_ref = -N_ref (R'^T b + P_ref^T a~) is
// known first and mu_ref = M_ref^+ (a~ + K_ref U_ref) is a single product.
// v_mfma_f64_16x16x4f64 operands (checked on the device): lane l holds A(l % 16,
// l / 16) and B(l / 16, l % 16) and item r of its accumulator is D(4 r + l / 16,
// l % 16).  Wave w computes the 16-row blocks w, w + 4, ... of the n2 x 16 product;
// the shared matrix comes from global memory (L2-resident, 128-byte rows per
// step), the tile's vectors from LDS.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int MODE, int RB>
__device__ __forceinline__ void body_mfma(const BodyTiles &bt, int tile, const int *__restrict__ off,
                                          const double *__restrict__ theta, const double *const *ref,
                                          const int *__restrict__ np, const double *const *X,
                                          const double *const *Pref, const double *const *Nt,
                                          const double *__restrict__ dN, int N, const double *__restrict__ z,
                                          double *__restrict__ y) {
  constexpr int NB = kBodyMfmaCols;
  constexpr int kLd = NB * 256 / 2 / 256;  // node pairs per thread at 2 n_p = 256 (loads in flight)
  extern __shared__ double sm[];           // T[k][NB]: body-frame inputs, then the product
  __shared__ double cs_[NB], sn_[NB], Ur[NB][3], fpart[4][NB][3];
  __shared__ double Ps[MODE == 1 ? 3 * 256 : 1], rfs[MODE == 1 ? 256 : 1];  // P_ref, reference nodes
  __shared__ int base_[NB];
  const int4 tl = bt.tile[tile];
  const int sh = tl.x, nb = tl.z;
  const int npt = np[sh], n2 = 2 * npt;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (MODE == 1) {  // P_ref and the reference nodes into LDS
    const double *Pm = Pref[sh], *rf = ref[sh];
    for (int i = tid; i < 3 * n2; i += 256) Ps[i] = Pm[i];
    for (int i = tid; i < n2; i += 256) rfs[i] = rf[i];
  }
  // MODE 1: each body's rigid-body inputs, requested now (used after the first products)
  double bq[3] = {0.0, 0.0, 0.0}, dq[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, nm[9];
  if (tid < NB) {
    double sn = 0.0, cs = 0.0;
    int bs = 0;
    if (tid < nb) {
      const int b = bt.list[tl.y + tid];
      if (MODE == 1) {
        const double *bb = z + 2 * (size_t)N + 3 * (size_t)b;
        bq[0] = bb[0];
        bq[1] = bb[1];
        bq[2] = bb[2];
        if (dN)
#pragma unroll
          for (int q = 0; q < 6; ++q) dq[q] = dN[6 * (size_t)b + q];
        const double *Nm = Nt[sh];
#pragma unroll
        for (int q = 0; q < 9; ++q) nm[q] = Nm[q];
      }
      sincos(theta[b], &sn, &cs);
      bs = off[b];
    }
    cs_[tid] = cs;
    sn_[tid] = sn;
    base_[tid] = bs;
  }
  __syncthreads();
  // body-frame inputs: T[2t + c][j] = (R_j^T a_j)_{t, c}; columns of absent bodies are zero.
  // Every load of a thread is issued before the first is used.
  {
    double2 av[kLd];
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int idx = tid + 256 * u, j = idx / npt, t = idx - j * npt;
      av[u] = make_double2(0.0, 0.0);
      if (idx < NB * npt && j < nb) av[u] = reinterpret_cast<const double2 *>(z)[base_[j] + t];
    }
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int idx = tid + 256 * u, j = idx / npt, t = idx - j * npt;
      if (idx < NB * npt) {
        sm[(2 * t) * NB + j] = cs_[j] * av[u].x + sn_[j] * av[u].y;
        sm[(2 * t + 1) * NB + j] = -sn_[j] * av[u].x + cs_[j] * av[u].y;
      }
    }
  }
  __syncthreads();
  if constexpr (MODE == 1) {
    // f_j = P_ref^T a~_j: thread (j = tid % 16, part p = tid / 16) sums rows p, p + 16, ...
    const int j = tid % NB, p = tid / NB;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int k = p; k < n2; k += 256 / NB) {
      const double a = sm[k * NB + j];
      f0 = fma(Ps[k], a, f0);
      f1 = fma(Ps[n2 + k], a, f1);
      f2 = fma(Ps[2 * n2 + k], a, f2);
    }
    // the four parts of a wave that share j (lanes j, j + 16, j + 32, j + 48)
    f0 += __shfl_xor(f0, 16);
    f1 += __shfl_xor(f1, 16);
    f2 += __shfl_xor(f2, 16);
    f0 += __shfl_xor(f0, 32);
    f1 += __shfl_xor(f1, 32);
    f2 += __shfl_xor(f2, 32);
    if (lane < NB) {
      fpart[wv][lane][0] = f0;
      fpart[wv][lane][1] = f1;
      fpart[wv][lane][2] = f2;
    }
    __syncthreads();
    if (tid < nb) {
      const int jj = tid, b = bt.list[tl.y + jj];
      const double cs = cs_[jj], sn = sn_[jj];
      const double *d = dq;
      const double bx = bq[0], by = bq[1], b2 = bq[2];
      const double b0 = cs * bx + sn * by, b1 = -sn * bx + cs * by;
      double g[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) g[q] = ((fpart[0][jj][q] + fpart[1][jj][q]) + (fpart[2][jj][q] + fpart[3][jj][q]));
      g[0] += b0;
      g[1] += b1;
      g[2] += b2;
      const double u0 = -(nm[0] * g[0] + nm[1] * g[1] + nm[2] * g[2]);
      const double u1 = -(nm[3] * g[0] + nm[4] * g[1] + nm[5] * g[2]);
      const double u2 = -(nm[6] * g[0] + nm[7] * g[1] + nm[8] * g[2]);
      Ur[jj][0] = u0;
      Ur[jj][1] = u1;
      Ur[jj][2] = u2;
      // learned correction C = dN_b (xx, yy, tt, xy, xt, yt): mu unchanged, U gains -C R'^T b
      const double v0 = u0 - (d[0] * b0 + d[3] * b1 + d[4] * b2);
      const double v1 = u1 - (d[3] * b0 + d[1] * b1 + d[5] * b2);
      const double v2 = u2 - (d[4] * b0 + d[5] * b1 + d[2] * b2);
      double *yU = y + 2 * (size_t)N + 3 * (size_t)b;
      yU[0] = cs * v0 - sn * v1;
      yU[1] = sn * v0 + cs * v1;
      yU[2] = v2;
    } else if (tid < NB) {
      Ur[tid][0] = Ur[tid][1] = Ur[tid][2] = 0.0;
    }
    __syncthreads();
    // a~ + K_ref U_ref: (u_x - omega r_y, u_y + omega r_x) at each reference node
    for (int idx = tid; idx < NB * npt; idx += 256) {
      const int j = idx % NB, t = idx / NB;
      sm[(2 * t) * NB + j] += Ur[j][0] - Ur[j][2] * rfs[2 * t + 1];
      sm[(2 * t + 1) * NB + j] += Ur[j][1] + Ur[j][2] * rfs[2 * t];
    }
    __syncthreads();
  }
  // product X T on the matrix cores (X[k n2 + r] multiplies input k of output r), the
  // operands of kStep k-steps loaded before their products
  constexpr int kStep = 16;
  const double *__restrict__ Xm = X[sh];
  const int nrb = n2 / 16, nk = n2 / 4, li = lane & 15, lk = lane >> 4;
  constexpr int kMaxRb = RB;          // row blocks per wave at the largest n2 of the launch
  const int nq = (nrb - wv + 3) / 4;  // this wave's row blocks wv, wv + 4, ...
  f64x4 acc[kMaxRb];
#pragma unroll
  for (int q = 0; q < kMaxRb; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  const double *xa = Xm + (size_t)lk * n2 + 16 * wv + li;
  const double *tb = sm + lk * NB + li;
  for (int s0 = 0; s0 < nk; s0 += kStep) {
    // one batch: the X operands of every row block of the wave, then the products
    double xv[kMaxRb][kStep], tv[kStep];
#pragma unroll
    for (int u = 0; u < kStep; ++u) {
      const bool ok = s0 + u < nk;
      tv[u] = ok ? tb[4 * (s0 + u) * NB] : 0.0;
#pragma unroll
      for (int q = 0; q < kMaxRb; ++q)
        xv[q][u] = (ok && q < nq) ? xa[(size_t)(4 * (s0 + u)) * n2 + 64 * q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kMaxRb; ++q)
      if (q < nq)
#pragma unroll
        for (int u = 0; u < kStep; ++u)
          if (s0 + u < nk) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[q][u], tv[u], acc[q], 0, 0, 0);
  }
  __syncthreads();  // every wave is done reading T
#pragma unroll
  for (int q = 0; q < kMaxRb; ++q) {
    const int rb = wv + 4 * q;
    if (rb < nrb)
#pragma unroll
      for (int r = 0; r < 4; ++r) sm[(16 * rb + 4 * r + lk) * NB + li] = acc[q][r];
  }
  __syncthreads();
  // back to the lab frame, each body's nodes written contiguously
  for (int idx = tid; idx < nb * npt; idx += 256) {
    const int j = idx / npt, t = idx - j * npt;
    const double mx = sm[(2 * t) * NB + j], my = sm[(2 * t + 1) * NB + j];
    reinterpret_cast<double2 *>(y)[base_[j] + t] = make_double2(cs_[j] * mx - sn_[j] * my, sn_[j] * mx + cs_[j] * my);
  }
}

template <int MODE, int RB>
__global__ __launch_bounds__(256) void k_body_mfma(BodyTiles bt, const int *__restrict__ off,
                                                   const double *__restrict__ theta, const double *const *ref,
                                                   const int *__restrict__ np, const double *const *X,
                                                   const double *const *Pref, const double *const *Nt,
                                                   const double *__restrict__ dN, int N,
                                                   const double *__restrict__ z, double *__restrict__ y) {
  body_mfma<MODE, RB>(bt, blockIdx.x, off, theta, ref, np, X, Pref, Nt, dN, N, z, y);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_body_tile(BodyTiles bt, const int *__restrict__ off,
                                                   const double *__restrict__ theta, const double *const *ref,
                                                   const int *__restrict__ np, const double *const *X,
                                                   const double *const *Pref, const double *const *Nt,
                                                   const double *__restrict__ dN, int N,
                                                   const double *__restrict__ z, double *__restrict__ y) {
  body_tile<MODE>(bt, blockIdx.x, off, theta, ref, np, X, Pref, Nt, dN, N, z, y);
}

__global__ __launch_bounds__(256) void k_precond_batch(const PrecondJob *__restrict__ jobs, BatchGrid bg) {
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  const PrecondJob &j = jobs[s];
  if (j.bt.mfma)  // a list mixing both forms: the instance for every n2
    body_mfma<1, 4>(j.bt, blockIdx.x - bg.begin[s], j.g.off, j.g.theta, j.g.ref, j.g.np, j.m.Mp, j.m.Pref, j.m.Nt, j.dN,
                 j.g.N, j.z, j.y);
  else
    body_tile<1>(j.bt, blockIdx.x - bg.begin[s], j.g.off, j.g.theta, j.g.ref, j.g.np, j.m.Mp, j.m.Pref, j.m.Nt, j.dN,
                 j.g.N, j.z, j.y);
}

template <int RB>
__global__ __launch_bounds__(256) void k_precond_mfma_batch(const PrecondJob *__restrict__ jobs, BatchGrid bg) {
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  const PrecondJob &j = jobs[s];
  body_mfma<1, RB>(j.bt, blockIdx.x - bg.begin[s], j.g.off, j.g.theta, j.g.ref, j.g.np, j.m.Mp, j.m.Pref, j.m.Nt, j.dN,
               j.g.N, j.z, j.y);
}

// the matrix-core instance for `rb` row blocks per wave
template <typename F>
static hipError_t body_mfma_dispatch(int rb, F &&launch) {
  switch (rb) {
    case 1: return launch(std::integral_constant<int, 1>{});
    case 2: return launch(std::integral_constant<int, 2>{});
    case 4: return launch(std::integral_constant<int, 4>{});
  }
  return hipErrorInvalidValue;
}

hipError_t launch_precond_batch(const PrecondJob *jobs, BatchGrid bg, size_t lds_bytes, int all_mfma,
                                hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (all_mfma)
    return body_mfma_dispatch(all_mfma, [&](auto rb) {
      hipLaunchKernelGGL((k_precond_mfma_batch<decltype(rb)::value>), dim3(bg.nblocks), dim3(256), lds_bytes, s,
                         jobs, bg);
      return hipGetLastError();
    });
  hipLaunchKernelGGL(k_precond_batch, dim3(bg.nblocks), dim3(256), lds_bytes, s, jobs, bg);
  return hipGetLastError();
}

hipError_t launch_precond(const GeomDev &g, const BodyMats &m, const BodyTiles &bt, const double *dN,
                          const double *z, double *y, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if (bt.mfma)
    return body_mfma_dispatch(bt.mfma, [&](auto rb) {
      hipLaunchKernelGGL((k_body_mfma<1, decltype(rb)::value>), dim3(bt.ntile), dim3(256), bt.lds_bytes, s, bt, g.off,
                         g.theta, g.ref, g.np, m.Mp, m.Pref, m.Nt, dN, g.N, z, y);
      return hipGetLastError();
    });
  hipLaunchKernelGGL(k_body_tile<1>, dim3(bt.ntile), dim3(256), bt.lds_bytes, s, bt, g.off, g.theta, g.ref, g.np,
                       m.Mp, m.Pref, m.Nt, dN, g.N, z, y);
  return hipGetLastError();
}

hipError_t launch_body_apply(const GeomDev &g, const BodyMats &m, const BodyTiles &bt, int which, const double *x,
                             double *y, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if (bt.mfma)
    return body_mfma_dispatch(bt.mfma, [&](auto rb) {
      hipLaunchKernelGGL((k_body_mfma<0, decltype(rb)::value>), dim3(bt.ntile), dim3(256), bt.lds_bytes, s, bt, g.off,
                         g.theta, g.ref, g.np, which ? m.Gp : m.G, m.Pref, m.Nt, (const double *)nullptr, g.N, x, y);
      return hipGetLastError();
    });
  hipLaunchKernelGGL(k_body_tile<0>, dim3(bt.ntile), dim3(256), bt.lds_bytes, s, bt, g.off, g.theta, g.ref, g.np,
                       which ? m.Gp : m.G, m.Pref, m.Nt, (const double *)nullptr, g.N, x, y);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Krylov vector kernels
// A batch vector is cut into chunks of at most kChunk elements, each inside one
// system; the chunks of a system are contiguous in the chunk table.  One work
// group reduces one chunk into partial[chunk][j]; a second launch with one work
// group per (column, system) sums the system's chunk rows in a fixed order, so
// every result is deterministic.  (A last-block-done reduction inside the first
// launch would need an agent-scope release fence per work group, which writes
// back the XCD's L2 each time; the second launch is far cheaper.)

__global__ __launch_bounds__(256) void k_orth_finish(Segs seg, int kk, const double *__restrict__ cond,
                                                     const double *__restrict__ partial, double *__restrict__ out,
                                                     int ostride) {
  __shared__ double red[4];
  const int j = blockIdx.x, sys = blockIdx.y;
  if (cond && cond[sys] == 0.0) return;
  const int c0 = seg.sys_chunk[sys], c1 = seg.sys_chunk[sys + 1];
  double s = 0.0;
  for (int c = c0 + (int)threadIdx.x; c < c1; c += 256) s += partial[(size_t)c * kk + j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[(size_t)sys * ostride + j] = (red[0] + red[1]) + (red[2] + red[3]);
}

constexpr int pow2_ceil(int n) { return n <= 1 ? 1 : 2 * pow2_ceil((n + 1) / 2); }
constexpr int log2_exact(int n) { return n <= 1 ? 0 : 1 + log2_exact(n / 2); }

// Column sums of a 256-thread block: dst[c] = sum over threads of acc[c], c < nv.
// Few columns: one shuffle reduction per column.  More: a halving exchange across
// the wave (at offset o the lanes with bit o set keep the upper half of their
// padded columns, the others the lower half, each adding the partner's copy), so
// that after log2(P) rounds lane l holds column l >> (6 - log2 P) summed over the
// lanes that differ in the high bits; the low bits are reduced by plain shuffles.
// P - 1 + 6 - log2 P shuffles per wave instead of 6 NV; the order is fixed.
template <int NV>
__device__ inline void block_sum_store(const double (&acc)[NV], int nv, double *__restrict__ dst) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if constexpr (NV <= 4) {
    __shared__ double red[4][NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double v = acc[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
      if (lane == 0) red[wv][c] = v;
    }
    __syncthreads();
    for (int c = tid; c < nv; c += 256) dst[c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    __syncthreads();
  } else {
    constexpr int P = pow2_ceil(NV), LP = log2_exact(P);
    static_assert(P <= 64, "at most 64 columns");
    __shared__ double red[4][P];
    double v[P];
#pragma unroll
    for (int c = 0; c < P; ++c) v[c] = c < NV ? acc[c] : 0.0;
#pragma unroll
    for (int r = 0; r < LP; ++r) {
      const int o = 32 >> r, h = P >> (r + 1);
      const bool upper = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const double send = upper ? v[i] : v[i + h];
        const double recv = __shfl_xor(send, o);
        v[i] = (upper ? v[i + h] : v[i]) + recv;
      }
    }
#pragma unroll
    for (int o = 32 >> LP; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o);
    if ((lane & ((64 >> LP) - 1)) == 0) red[wv][lane >> (6 - LP)] = v[0];
    __syncthreads();
    for (int c = tid; c < nv; c += 256) dst[c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    __syncthreads();
  }
}

// Exact column count K (0..kOrthFused), fully unrolled:
//   MODE 0: out[j] = V_j . w (j < K), out[K] = w . w
//   MODE 1: w -= V h; out[j] = V_j . w (j < K), out[K] = w . w
//   MODE 2: w -= V h; out[0] = w . w
// E elements per thread and iteration keep E (K + 1) loads in flight.
// At most two waves per SIMD: the passes launch one work group per chunk (~2.5 per
// CU at 640k nodes), so occupancy buys nothing, and the register room lets every
// thread keep all of its column loads in flight (at the default target the dot
// pass issued them one after another, waiting on each).
template <int MODE, int K, typename VT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_orth(OrthArgs a) {
  constexpr int E = K <= 4 ? 4 : (K <= 12 ? 2 : 1);
  constexpr int NV = MODE == 2 ? 1 : K + 1;
  const int cidx = blockIdx.x;
  const int sys = a.seg.chunk_sys[cidx];
  if (a.cond && a.cond[sys] == 0.0) return;  // conditional pass not requested for this system
  const int2 rg = a.seg.chunk[cidx];
  const int tid = threadIdx.x;
  double hr[K > 0 ? K : 1];
  if (MODE != 0) {
    const double *h = a.h + (size_t)sys * a.hstride;
#pragma unroll
    for (int j = 0; j < K; ++j) hr[j] = h[j];
  }
  const VT *__restrict__ V = reinterpret_cast<const VT *>(a.Vs ? a.Vs[sys] : a.V);
  double *__restrict__ w = a.ws ? a.ws[sys] : a.w;
  const size_t ld = a.lds ? a.lds[sys] : a.ld;
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = 0.0;
  for (int i0 = rg.x + tid; i0 < rg.y; i0 += 256 * E) {
    double vv[E][K > 0 ? K : 1], wv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = min(i0 + 256 * e, rg.y - 1);  // clamped: out-of-chunk lanes reload a valid element
      wv[e] = w[i];
#pragma unroll
      for (int j = 0; j < K; ++j) vv[e][j] = (double)V[(size_t)j * ld + i];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool ok = i0 + 256 * e < rg.y;
      double x = wv[e];
      if (MODE != 0) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          if (j & 1)
            s1 += vv[e][j] * hr[j];
          else
            s0 += vv[e][j] * hr[j];
        }
        x -= s0 + s1;
        if (ok) w[i0 + 256 * e] = x;
      }
      if (!ok) x = 0.0;
      if (MODE != 2) {
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] += vv[e][j] * x;
      }
      acc[NV - 1] += x * x;
    }
  }
  block_sum_store<NV>(acc, NV, a.partial + (size_t)cidx * NV);
}

// Runtime column count k (any k < kOrthMaxCols): MODE 0 in passes of 32 columns,
// MODE 2 with a runtime loop.  Used beyond the unrolled range.
template <int MODE, typename VT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_orth_any(OrthArgs a) {
  constexpr int KR = 32;
  const int cidx = blockIdx.x;
  const int sys = a.seg.chunk_sys[cidx];
  if (a.cond && a.cond[sys] == 0.0) return;
  const int2 rg = a.seg.chunk[cidx];
  const int tid = threadIdx.x;
  const int k = a.k;
  const VT *__restrict__ V = reinterpret_cast<const VT *>(a.Vs ? a.Vs[sys] : a.V);
  double *__restrict__ w = a.ws ? a.ws[sys] : a.w;
  const size_t ld = a.lds ? a.lds[sys] : a.ld;
  if (MODE == 2) {
    __shared__ double hs[kOrthMaxCols];
    const double *h = a.h + (size_t)sys * a.hstride;
    for (int j = tid; j < k; j += 256) hs[j] = h[j];
    __syncthreads();
    double acc[1] = {0.0};
    for (int i = rg.x + tid; i < rg.y; i += 256) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int j = 0;
      for (; j + 3 < k; j += 4) {
        s0 += (double)V[(size_t)j * ld + i] * hs[j];
        s1 += (double)V[(size_t)(j + 1) * ld + i] * hs[j + 1];
        s2 += (double)V[(size_t)(j + 2) * ld + i] * hs[j + 2];
        s3 += (double)V[(size_t)(j + 3) * ld + i] * hs[j + 3];
      }
      for (; j < k; ++j) s0 += (double)V[(size_t)j * ld + i] * hs[j];
      const double v = w[i] - ((s0 + s1) + (s2 + s3));
      w[i] = v;
      acc[0] += v * v;
    }
    block_sum_store<1>(acc, 1, a.partial + cidx);
    return;
  }
  const int kk = k + 1;
  double *part = a.partial + (size_t)cidx * kk;
  for (int j0 = 0; j0 == 0 || j0 < k; j0 += KR) {
    double acc[KR + 1];
#pragma unroll
    for (int c = 0; c <= KR; ++c) acc[c] = 0.0;
    const int nc = min(KR, k - j0);
    for (int i = rg.x + tid; i < rg.y; i += 256) {
      const double wi = w[i];
#pragma unroll
      for (int c = 0; c < KR; ++c)
        if (c < nc) acc[c] += (double)V[(size_t)(j0 + c) * ld + i] * wi;
      if (j0 == 0) acc[KR] += wi * wi;
    }
    __shared__ double red[4][KR + 1];
    const int lane = tid & 63, wvi = tid >> 6;
#pragma unroll
    for (int c = 0; c <= KR; ++c) {
      double v = acc[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
      if (lane == 0) red[wvi][c] = v;
    }
    __syncthreads();
    if (tid < nc) part[j0 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    if (j0 == 0 && tid == 0) part[k] = (red[0][KR] + red[1][KR]) + (red[2][KR] + red[3][KR]);
    __syncthreads();
  }
}

hipError_t finish(int kk, const OrthArgs &a, hipStream_t s) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_orth_finish, dim3(kk, a.seg.S), dim3(256), 0, s, a.seg, kk, a.cond, a.partial, a.out,
                     a.ostride);
  return hipGetLastError();
}

template <int MODE, int K, typename VT>
hipError_t launch_orth_k(const OrthArgs &a, hipStream_t s) {
  if constexpr (K > kOrthFused) {
    return hipErrorInvalidValue;
  } else {
    if (a.k == K) {
      hipLaunchKernelGGL((k_orth<MODE, K, VT>), dim3(a.seg.nchunk), dim3(256), 0, s, a);
      return finish(MODE == 2 ? 1 : K + 1, a, s);
    }
    return launch_orth_k<MODE, K + 1, VT>(a, s);
  }
}

template <typename VT>
hipError_t launch_orth_t(int mode, const OrthArgs &a, hipStream_t s) {
  if (a.k <= kOrthFused) {
    if (mode == 0) return launch_orth_k<0, 0, VT>(a, s);
    if (mode == 1) return launch_orth_k<1, 0, VT>(a, s);
    return launch_orth_k<2, 0, VT>(a, s);
  }
  if (mode == 0) {
    hipLaunchKernelGGL((k_orth_any<0, VT>), dim3(a.seg.nchunk), dim3(256), 0, s, a);
    return finish(a.k + 1, a, s);
  }
  hipLaunchKernelGGL((k_orth_any<2, VT>), dim3(a.seg.nchunk), dim3(256), 0, s, a);
  return finish(1, a, s);
}

hipError_t launch_orth(int mode, const OrthArgs &a, hipStream_t s) {
  if (a.seg.nchunk == 0) return hipSuccess;
  if (a.k < 0 || a.k + 1 > kOrthMaxCols || (mode == 1 && a.k > kOrthFused)) return hipErrorInvalidValue;
  return a.v32 ? launch_orth_t<float>(mode, a, s) : launch_orth_t<double>(mode, a, s);
}

// Lagged pass of delayed classical Gram-Schmidt with reorthogonalisation (DCGS2:
// Swirydowicz, Langou, Ananthan, Yang and Thomas 2020; Bielich, Langou, Thomas et al.
// 2022).  The reorthogonalisation of the newest basis vector u, due one Arnoldi step
// earlier, is applied in the same read of the basis that projects w, so a step reads
// the basis twice (this pass and the dot-product pass before it) instead of three
// times.  The coefficients are computed from h and lag in every work group (K + 1
// values).  E elements per thread as in k_orth.
template <int K, typename VT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_orth_lag(OrthArgs a) {
  constexpr int E = K <= 4 ? 4 : (K <= 12 ? 2 : 1);
  constexpr int NV = K + 2;
  const int cidx = blockIdx.x;
  const int sys = a.seg.chunk_sys[cidx];
  const int2 rg = a.seg.chunk[cidx];
  const int tid = threadIdx.x;
  const double *h = a.h + (size_t)sys * a.hstride;
  double sc[K > 0 ? K : 1], tc[K > 0 ? K : 1];
  double ss = 0.0, st = 0.0, inu = 1.0;
  if constexpr (K > 0) {
    const double *lag = a.lag + (size_t)sys * a.lagstride;
    const double nu = sqrt(fmax(lag[K], 0.0));
    inu = nu > 0.0 ? 1.0 / nu : 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      sc[j] = lag[j] * inu;
      tc[j] = h[j] * inu;
      ss += sc[j] * sc[j];
      st += sc[j] * tc[j];
    }
  }
  const double rho = sqrt(fmax(1.0 - ss, 0.0));
  const double irho = rho > 0.0 ? 1.0 / rho : 0.0;
  const double ecoef = (h[K] * inu * inu - st) * irho;
  double *__restrict__ xs = a.next ? a.xs[sys] : nullptr;
  VT *__restrict__ V = reinterpret_cast<VT *>(const_cast<double *>(a.Vs ? a.Vs[sys] : a.V));
  double *__restrict__ w = a.ws ? a.ws[sys] : a.w;
  const size_t ld = a.lds ? a.lds[sys] : a.ld;
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = 0.0;
  for (int i0 = rg.x + tid; i0 < rg.y; i0 += 256 * E) {
    double vv[E][K > 0 ? K : 1], uv[E], wv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = min(i0 + 256 * e, rg.y - 1);  // clamped: out-of-chunk lanes reload a valid element
      wv[e] = w[i];
      uv[e] = (double)V[(size_t)K * ld + i];
#pragma unroll
      for (int j = 0; j < K; ++j) vv[e][j] = (double)V[(size_t)j * ld + i];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool ok = i0 + 256 * e < rg.y;
      double v = uv[e] * inu;
      double p0 = 0.0, p1 = 0.0;
      if constexpr (K > 0) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          if (j & 1) {
            s1 += vv[e][j] * sc[j];
            p1 += vv[e][j] * tc[j];
          } else {
            s0 += vv[e][j] * sc[j];
            p0 += vv[e][j] * tc[j];
          }
        }
        v = (v - (s0 + s1)) * irho;
        if (ok) V[(size_t)K * ld + i0 + 256 * e] = (VT)v;
      }
      double x = (wv[e] * inu - (p0 + p1) - v * ecoef) * irho;
      if (ok) {
        const int i = i0 + 256 * e;
        if (xs) {
          V[(size_t)(K + 1) * ld + i] = (VT)x;
          xs[i] = x;
        } else {
          w[i] = x;
        }
      }
      if (!ok) x = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) acc[j] += vv[e][j] * x;
      acc[K] += v * x;
      acc[K + 1] += x * x;
    }
  }
  block_sum_store<NV>(acc, NV, a.partial + (size_t)cidx * NV);
}

template <int K, typename VT>
hipError_t launch_orth_lag_k(const OrthArgs &a, hipStream_t s) {
  if constexpr (K >= kOrthFused) {
    return hipErrorInvalidValue;
  } else {
    if (a.k == K) {
      hipLaunchKernelGGL((k_orth_lag<K, VT>), dim3(a.seg.nchunk), dim3(256), 0, s, a);
      return finish(K + 2, a, s);
    }
    return launch_orth_lag_k<K + 1, VT>(a, s);
  }
}

hipError_t launch_orth_lag(const OrthArgs &a, hipStream_t s) {
  if (a.seg.nchunk == 0) return hipSuccess;
  if (a.k < 0 || a.k >= kOrthFused || (a.k > 0 && !a.lag) || a.cond || (a.next && !a.xs)) return hipErrorInvalidValue;
  return a.v32 ? launch_orth_lag_k<0, float>(a, s) : launch_orth_lag_k<0, double>(a, s);
}

// ------------------------------------------------------------------ segmented vector kernels (batches)
template <typename T>
__device__ inline T *vec_ptr(const VecRef &v, int s) {
  return reinterpret_cast<T *>(const_cast<double *>(v.base[s])) + (size_t)v.col * (v.ld ? v.ld[s] : 0);
}

// y_s = a[s] x_s + b[s] y_s (x_s not read when a[s] == 0, y_s not when b[s] == 0); one work group per chunk;
// FP64 arithmetic, FP32 vectors widened on load and rounded on store
template <typename XT, typename YT>
__global__ __launch_bounds__(256) void k_seg_axpby(Segs seg, VecRef x, VecRef y, const double *__restrict__ a,
                                                   const double *__restrict__ b) {
  const int c = blockIdx.x;
  const int s = seg.chunk_sys[c];
  const int2 rg = seg.chunk[c];
  const XT *xp = vec_ptr<XT>(x, s);
  YT *yp = vec_ptr<YT>(y, s);
  const double as = a[s], bs = b[s];
  // a zero coefficient reads nothing, so uninitialised vectors can be cleared
  for (int i = rg.x + threadIdx.x; i < rg.y; i += 256)
    yp[i] = (YT)((as == 0.0 ? 0.0 : as * (double)xp[i]) + (bs == 0.0 ? 0.0 : bs * (double)yp[i]));
}

hipError_t launch_seg_axpby(const Segs &seg, const VecRef &x, const VecRef &y, const double *a, const double *b,
                            hipStream_t s) {
  if (seg.nchunk == 0) return hipSuccess;
  const dim3 g(seg.nchunk), t(256);
  if (!x.f32 && !y.f32)
    hipLaunchKernelGGL((k_seg_axpby<double, double>), g, t, 0, s, seg, x, y, a, b);
  else if (x.f32 && !y.f32)
    hipLaunchKernelGGL((k_seg_axpby<float, double>), g, t, 0, s, seg, x, y, a, b);
  else if (!x.f32 && y.f32)
    hipLaunchKernelGGL((k_seg_axpby<double, float>), g, t, 0, s, seg, x, y, a, b);
  else
    hipLaunchKernelGGL((k_seg_axpby<float, float>), g, t, 0, s, seg, x, y, a, b);
  return hipGetLastError();
}

template <typename YT>
__global__ __launch_bounds__(256) void k_seg_scale2(Segs seg, VecRef x, VecRef y, VecRef z,
                                                    const double *__restrict__ a) {
  const int c = blockIdx.x;
  const int s = seg.chunk_sys[c];
  const int2 rg = seg.chunk[c];
  const double *xp = vec_ptr<double>(x, s);
  YT *yp = vec_ptr<YT>(y, s);
  double *zp = vec_ptr<double>(z, s);
  const double as = a[s];
  for (int i = rg.x + threadIdx.x; i < rg.y; i += 256) {
    const YT v = (YT)(as == 0.0 ? 0.0 : as * xp[i]);
    yp[i] = v;
    zp[i] = (double)v;
  }
}

hipError_t launch_seg_scale2(const Segs &seg, const VecRef &x, const VecRef &y, const VecRef &z, const double *a,
                             hipStream_t s) {
  if (seg.nchunk == 0) return hipSuccess;
  if (x.f32 || z.f32) return hipErrorInvalidValue;
  if (y.f32)
    hipLaunchKernelGGL((k_seg_scale2<float>), dim3(seg.nchunk), dim3(256), 0, s, seg, x, y, z, a);
  else
    hipLaunchKernelGGL((k_seg_scale2<double>), dim3(seg.nchunk), dim3(256), 0, s, seg, x, y, z, a);
  return hipGetLastError();
}

// y_s = sum_{j < k} V_s[:, j] c[s * cstride + j]
template <typename VT>
__global__ __launch_bounds__(256) void k_seg_Vc(Segs seg, VecRef V, int k, const double *__restrict__ c, int cstride,
                                                VecRef y) {
  const int ci = blockIdx.x;
  const int s = seg.chunk_sys[ci];
  const int2 rg = seg.chunk[ci];
  const VT *Vp = reinterpret_cast<const VT *>(V.base[s]);
  const size_t ld = V.ld[s];
  const double *cs = c + (size_t)s * cstride;
  double *yp = vec_ptr<double>(y, s);
  // zero coefficients are skipped: a system that stopped earlier pads its
  // coefficients with zeros, and its basis columns beyond that are not written
  for (int i = rg.x + threadIdx.x; i < rg.y; i += 256) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j)
      if (cs[j] != 0.0) acc += (double)Vp[(size_t)j * ld + i] * cs[j];
    yp[i] = acc;
  }
}

hipError_t launch_seg_Vc(const Segs &seg, const VecRef &V, int k, const double *c, int cstride, const VecRef &y,
                         hipStream_t s) {
  if (seg.nchunk == 0) return hipSuccess;
  if (y.f32) return hipErrorInvalidValue;
  if (V.f32)
    hipLaunchKernelGGL((k_seg_Vc<float>), dim3(seg.nchunk), dim3(256), 0, s, seg, V, k, c, cstride, y);
  else
    hipLaunchKernelGGL((k_seg_Vc<double>), dim3(seg.nchunk), dim3(256), 0, s, seg, V, k, c, cstride, y);
  return hipGetLastError();
}

// flag[s] = nrm[s * ns] < before[s * nb] / 2 ? 1 : 0
__global__ void k_need_second_pass(int S, const double *__restrict__ nrm, int ns, const double *__restrict__ before,
                                   int nb, double *__restrict__ flag) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) flag[s] = nrm[(size_t)s * ns] < 0.5 * before[(size_t)s * nb] ? 1.0 : 0.0;
}

hipError_t launch_need_second_pass(int S, const double *nrm, int ns, const double *before, int nb, double *flag,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_need_second_pass, dim3((S + 63) / 64), dim3(64), 0, s, S, nrm, ns, before, nb, flag);
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

__global__ void k_scale(size_t n, double a, double *__restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] *= a;
}

hipError_t launch_scale(size_t n, double a, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scale, dim3(nb), dim3(256), 0, s, n, a, y);
  return hipGetLastError();
}

hipError_t pub_alloc(HostPub &p, size_t n) {
  if (p.tag && n <= p.cap) return hipSuccess;
  pub_free(p);
  void *h = nullptr, *d = nullptr;
  hipError_t e = hipHostMalloc(&h, (n + 1) * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return e;
  e = hipHostGetDevicePointer(&d, h, 0);
  if (e != hipSuccess) {
    (void)hipHostFree(h);
    return e;
  }
  p.tag = static_cast<unsigned long long *>(h);
  p.tag_dev = static_cast<unsigned long long *>(d);
  p.v = static_cast<double *>(h) + 1;
  p.v_dev = static_cast<double *>(d) + 1;
  *p.tag = 0;  // the sequence keeps counting, so no tag it waits for is 0
  p.cap = n;
  return hipSuccess;
}

void pub_free(HostPub &p) {
  if (p.tag) (void)hipHostFree(p.tag);  // teardown: nothing to report to
  p.tag = p.tag_dev = nullptr;
  p.v = p.v_dev = nullptr;
  p.cap = 0;
}

hipError_t pub_wait(const HostPub &p, unsigned long long tag, hipStream_t s) {
  const volatile unsigned long long *t = p.tag;
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned spins = 1; *t != tag; ++spins) {
    // long queues (or a failed launch) end in the stream synchronisation
    if ((spins & 1023u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
      const hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      if (*t != tag) return hipErrorUnknown;
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return hipSuccess;
}

// one work group: the values, a system-scope fence, then the tag
__global__ __launch_bounds__(256) void k_orth_publish(OrthPublish o, double *__restrict__ v, unsigned long long *tag_out,
                                                      unsigned long long tag) {
  const int k1 = o.k + 1, total = o.S * k1;
  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    const int sys = i / k1, j = i - sys * k1;
    const bool second = !o.selective || o.flag[(size_t)sys * o.fs] != 0.0;
    const size_t hb = (size_t)sys * o.hs;
    double x;
    if (j < o.k) {
      x = o.h[hb + j] + (second ? o.h2[hb + j] : 0.0);
    } else {
      const double after = second ? o.nrm_b[(size_t)sys * o.ns] : (o.fused ? o.h2[hb + o.k] : o.nrm_a[(size_t)sys * o.ns]);
      x = sqrt(fmax(after, 0.0));
      o.a[(size_t)sys * o.as] = x > 0.0 ? 1.0 / x : 0.0;
    }
    v[i] = x;
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) *reinterpret_cast<volatile unsigned long long *>(tag_out) = tag;
}

hipError_t launch_orth_publish(const OrthPublish &o, HostPub &p, unsigned long long tag, hipStream_t s) {
  if (o.S <= 0 || o.k < 0 || (size_t)o.S * (o.k + 1) > p.cap || !p.tag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_orth_publish, dim3(1), dim3(256), 0, s, o, p.v_dev, p.tag_dev, tag);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_publish(int n, const double *__restrict__ src, int stride,
                                                 double *__restrict__ v, unsigned long long *tag_out,
                                                 unsigned long long tag) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = src[(size_t)i * stride];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) *reinterpret_cast<volatile unsigned long long *>(tag_out) = tag;
}

__global__ __launch_bounds__(256) void k_publish2(int S, int n0, const double *__restrict__ src0, int stride0, int n1,
                                                  const double *__restrict__ src1, int stride1,
                                                  double *__restrict__ v, unsigned long long *tag_out,
                                                  unsigned long long tag) {
  const int n = n0 + n1;
  for (int i = threadIdx.x; i < S * n; i += blockDim.x) {
    const int sys = i / n, j = i - sys * n;
    v[i] = j < n0 ? src0[(size_t)sys * stride0 + j] : src1[(size_t)sys * stride1 + j - n0];
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) *reinterpret_cast<volatile unsigned long long *>(tag_out) = tag;
}

hipError_t launch_publish2(int S, int n0, const double *src0, int stride0, int n1, const double *src1, int stride1,
                           HostPub &p, unsigned long long tag, hipStream_t s) {
  if (S < 0 || n0 < 0 || n1 < 0 || (size_t)S * (n0 + n1) > p.cap || !p.tag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_publish2, dim3(1), dim3(256), 0, s, S, n0, src0, stride0, n1, src1, stride1, p.v_dev,
                     p.tag_dev, tag);
  return hipGetLastError();
}

hipError_t launch_publish(int n, const double *src, int stride, HostPub &p, unsigned long long tag, hipStream_t s) {
  if (n < 0 || (size_t)n > p.cap || !p.tag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, s, n, src, stride, p.v_dev, p.tag_dev, tag);
  return hipGetLastError();
}

__global__ void k_scale_dev(size_t n, const double *__restrict__ a, double *__restrict__ y) {
  const double f = a[0];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] *= f;
}

hipError_t launch_scale_dev(size_t n, const double *a, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scale_dev, dim3(nb), dim3(256), 0, s, n, a, y);
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
