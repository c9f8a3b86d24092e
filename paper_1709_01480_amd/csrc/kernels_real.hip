// Real-space part of the single-layer matvec (Section 3.2):
//   M^(t): trapezoid pairs within the cutoff r_c through the cell list, with the
//          Hasimoto real-space Stokeslet G^(r) of eq. 3.15;
//   M^(a): banded Alpert correction applied as R_b A_ref R_b^T per body.
#include "kernels.h"

namespace fbim {

namespace {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

constexpr int kPairChunk = 256;   // sources staged in LDS per pass
constexpr int kE1Int = 9;         // intervals of the E1 table

// blockIdx -> work item such that consecutive items land on the same XCD
// (work groups are dealt round-robin over the 8 XCDs)
__device__ inline int xcd_remap(int b, int n) {
  const int q = n / 8, r = n % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

__device__ inline double dev_exp(double x) { return exp(x); }
__device__ inline float dev_exp(float x) { return __expf(x); }
__device__ inline double dev_log(double x) { return log(x); }
__device__ inline float dev_log(float x) { return __logf(x); }
__device__ inline double dev_rint(double x) { return rint(x); }
__device__ inline float dev_rint(float x) { return rintf(x); }

// E1(z) from the piecewise Chebyshev table: interval 0 holds E1 + ln z on [0, 2],
// interval k >= 1 holds e^z E1(z) on [2*1.5^(k-1), 2*1.5^k].
template <typename T, int DEG>
__device__ inline T e1_eval(T z, T lz, T ez, const T *tab) {
  int k = 0;
  if (z > T(2)) k = min(kE1Int - 1, 1 + (int)((lz - T(0.69314718055994530942)) * T(2.46630346237643166674)));
  const T *row = tab + k * (DEG + 3);
  const T x = (z - row[0]) * row[1];
  T b1 = 0, b2 = 0;
#pragma unroll
  for (int m = DEG; m >= 1; --m) {
    const T b0 = row[2 + m] + T(2) * x * b1 - b2;
    b2 = b1;
    b1 = b0;
  }
  const T f = row[2] + x * b1 - b2;
  return k == 0 ? f - lz : ez * f;
}

template <typename T, int DEG>
__global__ __launch_bounds__(64) void k_pair(const int *__restrict__ cell_start, const int *__restrict__ perm,
                                             int nb, int nbatch, T L, T rc2, T xi2, T cG,
                                             const T *__restrict__ e1tab,
                                             const typename Vec2<T>::type *__restrict__ xs,
                                             const typename Vec2<T>::type *__restrict__ mus,
                                             double *__restrict__ out) {
  __shared__ T sx[kPairChunk], sy[kPairChunk], smx[kPairChunk], smy[kPairChunk];
  __shared__ int sid[kPairChunk];
  __shared__ T tx[64], ty[64], ax[64], ay[64], cx[64], cy[64];
  __shared__ int qbuf[128];
  __shared__ T tab[kE1Int * (DEG + 3)];

  const int lane = threadIdx.x;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int c = w / nbatch, bt = w % nbatch;
  const int cs = cell_start[c], ce = cell_start[c + 1];
  const int t0 = cs + bt * 64;
  if (t0 >= ce) return;  // uniform over the work group
  const int nt = min(64, ce - t0);
  for (int i = lane; i < kE1Int * (DEG + 3); i += 64) tab[i] = e1tab[i];
  if (lane < nt) {
    const auto p = xs[t0 + lane];
    tx[lane] = p.x;
    ty[lane] = p.y;
  }
  ax[lane] = ay[lane] = cx[lane] = cy[lane] = T(0);

  // the 3x3 neighbourhood (n_box >= 3, so the nine cells are distinct)
  const int ccx = c % nb, ccy = c / nb;
  int nstart[9], pre[10];
  pre[0] = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int dx = k % 3 - 1, dy = k / 3 - 1;
    const int cc = ((ccy + dy + nb) % nb) * nb + (ccx + dx + nb) % nb;
    nstart[k] = cell_start[cc];
    pre[k + 1] = pre[k] + cell_start[cc + 1] - cell_start[cc];
  }
  const int ns = pre[9];
  const T invL = T(1) / L;
  int qn = 0;
  __syncthreads();

  // evaluate queued (target, source) pairs and reduce them per target
  auto process = [&](int cnt) {
    __syncthreads();
    const int e = lane < cnt ? qbuf[lane] : -1;
    const int t = e >= 0 ? (e >> 16) : -1;
    T vx = 0, vy = 0;
    if (e >= 0) {
      const int s = e & 0xffff;
      T dx = tx[t] - sx[s], dy = ty[t] - sy[s];
      dx -= L * dev_rint(dx * invL);
      dy -= L * dev_rint(dy * invL);
      const T r2 = dx * dx + dy * dy;
      const T z = xi2 * r2;
      const T lz = dev_log(z);
      const T ez = dev_exp(-z);
      const T e1 = e1_eval<T, DEG>(z, lz, ez, tab);
      const T a = T(0.5) * e1 - ez;
      const T mx = smx[s], my = smy[s];
      const T sdot = ez * (dx * mx + dy * my) / r2;
      vx = a * mx + sdot * dx;
      vy = a * my + sdot * dy;
    }
    // segmented suffix sums over lanes; the queue is ordered by target
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const T ox = __shfl_down(vx, off), oy = __shfl_down(vy, off);
      const int ot = __shfl_down(t, off);
      if (lane + off < 64 && ot == t) {
        vx += ox;
        vy += oy;
      }
    }
    const int tp = __shfl_up(t, 1);
    if (t >= 0 && (lane == 0 || tp != t)) {
      // compensated accumulation (exact ordering: one head per target per batch)
      T y = vx - cx[t];
      T s2 = ax[t] + y;
      cx[t] = (s2 - ax[t]) - y;
      ax[t] = s2;
      y = vy - cy[t];
      s2 = ay[t] + y;
      cy[t] = (s2 - ay[t]) - y;
      ay[t] = s2;
    }
    __syncthreads();
  };

  for (int v0 = 0; v0 < ns; v0 += kPairChunk) {
    const int len = min(kPairChunk, ns - v0);
    for (int i = lane; i < len; i += 64) {
      const int v = v0 + i;
      int k = 0;
      while (k < 8 && v >= pre[k + 1]) ++k;
      const int g = nstart[k] + (v - pre[k]);
      const auto p = xs[g];
      const auto m = mus[g];
      sx[i] = p.x;
      sy[i] = p.y;
      smx[i] = m.x;
      smy[i] = m.y;
      sid[i] = g;
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const T px = tx[t], py = ty[t];
      const int gt = t0 + t;
      for (int s0 = 0; s0 < len; s0 += 64) {
        const int s = s0 + lane;
        bool ok = false;
        if (s < len) {
          T dx = px - sx[s], dy = py - sy[s];
          dx -= L * dev_rint(dx * invL);
          dy -= L * dev_rint(dy * invL);
          ok = (dx * dx + dy * dy <= rc2) && (sid[s] != gt);
        }
        const unsigned long long m = __ballot(ok);
        if (ok) qbuf[qn + __popcll(m & ((1ull << lane) - 1ull))] = (t << 16) | s;
        qn += __popcll(m);
        if (qn >= 64) {
          process(64);
          const int rest = qn - 64;
          const int keep = lane < rest ? qbuf[64 + lane] : 0;
          __syncthreads();
          if (lane < rest) qbuf[lane] = keep;
          qn = rest;
          __syncthreads();
        }
      }
    }
    if (qn > 0) {
      process(qn);
      qn = 0;
    }
    __syncthreads();
  }
  if (lane < nt) {
    const int node = perm[t0 + lane];
    out[2 * node] = (double)(cG * ax[lane]);
    out[2 * node + 1] = (double)(cG * ay[lane]);
  }
}

template <typename T, int DEG>
hipError_t pair_launch(const PairArgs &a, const T *xs, const T *mus, const T *tab, double *out, hipStream_t s) {
  const int ncell = a.nb * a.nb;
  const int nwg = ncell * a.nbatch;
  if (nwg == 0) return hipSuccess;
  using V = typename Vec2<T>::type;
  hipLaunchKernelGGL((k_pair<T, DEG>), dim3(nwg), dim3(64), 0, s, a.cell_start, a.perm, a.nb, a.nbatch, (T)a.L,
                     (T)a.rc2, (T)a.xi2, (T)a.cG, tab, (const V *)xs, (const V *)mus, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pair_f64(const PairArgs &a, const double *xs, const double *mus, double *out, hipStream_t s) {
  return pair_launch<double, 16>(a, xs, mus, a.e1tab, out, s);
}

hipError_t launch_pair_f32(const PairArgs &a, const float *xs, const float *mus, double *out, hipStream_t s) {
  return pair_launch<float, 9>(a, xs, mus, a.e1tab32, out, s);
}

// ------------------------------------------------------------------ Alpert band
__global__ void k_alpert(int N, const int *__restrict__ body, const int *__restrict__ off,
                         const int *__restrict__ shape, const double *__restrict__ theta,
                         const double *const *band_tab, const int *__restrict__ band, const int *__restrict__ np,
                         const double2 *__restrict__ mu, double2 *__restrict__ out, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = body[i];
  const int base = off[b];
  const int t = i - base;
  const int sh = shape[b];
  const int B = band[sh], n_p = np[sh];
  const double *A = band_tab[sh] + (size_t)t * (2 * B + 1) * 4;
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  double ax = 0.0, ay = 0.0;
  for (int o = -B; o <= B; ++o) {
    int l = t + o;
    l += (l < 0) ? n_p : 0;
    l -= (l >= n_p) ? n_p : 0;
    const double2 m = mu[base + l];
    const double rx = cs * m.x + sn * m.y, ry = -sn * m.x + cs * m.y;  // R^T mu
    const double *blk = A + (o + B) * 4;
    ax += blk[0] * rx + blk[1] * ry;
    ay += blk[2] * rx + blk[3] * ry;
  }
  const double2 r = make_double2(cs * ax - sn * ay, sn * ax + cs * ay);
  if (accumulate) {
    const double2 o = out[i];
    out[i] = make_double2(o.x + r.x, o.y + r.y);
  } else {
    out[i] = r;
  }
}

hipError_t launch_alpert(const GeomDev &g, const double *const *band_tab, const int *band, const double *mu,
                         double *out, int accumulate, hipStream_t s) {
  if (g.N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpert, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, g.body, g.off, g.shape, g.theta,
                     band_tab, band, g.np, (const double2 *)mu, (double2 *)out, accumulate);
  return hipGetLastError();
}

}  // namespace fbim
