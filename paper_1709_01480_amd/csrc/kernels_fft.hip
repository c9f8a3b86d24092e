// Fused wave-space convolution on power-of-two grids (Section 3.2, eqs. 3.21-3.25,
// and the random Fourier field of Section 3.3): the two real grid planes are
// transformed, multiplied and transformed back by three kernels that hold whole
// 1D transforms in LDS:
//   rows forward : per grid row y, one complex FFT of g_x + i g_y along x, split
//                  into the two half spectra H_c(kx, y), kx <= M/2, and written
//                  transposed: S[kx][y] = (H_x, H_y);
//   columns      : per kx, the two length-M columns of S are transformed along
//                  y, multiplied by the 2 x 2 Fourier multiplier, transformed back;
//   rows inverse : per row, the Hermitian extension of both half spectra packed
//                  as U_x + i U_y, one inverse complex FFT whose real and imaginary
//                  parts are the two grid planes.
// Up to rounding this is the real-to-complex 2D transform, the multiplier and the
// complex-to-real 2D transform (the imaginary parts of the kx = 0 and kx = M/2
// terms are dropped, as a complex-to-real transform does).  Each 1D transform is
// a Stockham autosort FFT (radix-8 stages, then one radix-2 or radix-4 stage)
// over a block's sequences in LDS, with twiddles from a table W[k] = exp(-2 pi i k / M);
// LDS indices are padded by one element per 16 (FP64) or 32 (FP32) so that the
// strided stores of the early stages spread over the banks.
#include "kernels.h"

namespace fbim {

namespace {

template <typename T> struct Cx;
template <> struct Cx<double> { using type = double2; };
template <> struct Cx<float> { using type = float2; };

// threads and complex elements per work group (8 per thread) and LDS padding.  At
// 4096 elements (34 KB of LDS in FP32) four work groups share a CU: the FP32 column
// kernel at 2048^2 ran 34.5 us with 8192 elements (two per CU) and 28 us with 4096.
constexpr int kThreads = 512;
template <typename T> constexpr int kElems = 4096;
// elements of a row-kernel work group: whole rows, at most the grid
template <typename T, int M> constexpr int kRowElems = kElems<T> < M * M ? kElems<T> : M * M;
template <typename T> constexpr int kPadShift = sizeof(T) == 8 ? 4 : 5;

// blockIdx -> work item such that consecutive items run on the same XCD (work
// groups are dealt round-robin over the 8 XCDs): the row kernels of neighbouring
// row groups then share the L2 lines of the kx-major spectrum (each group reads or
// writes part of a line)
__device__ inline int xcd_remap(int b, int n) {
  const int q = n / 8, r = n % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}
template <typename T> __device__ __forceinline__ int pad(int i) { return i + (i >> kPadShift<T>); }

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}
template <typename V> __device__ __forceinline__ V csub(V a, V b) {
  a.x -= b.x;
  a.y -= b.y;
  return a;
}
// a * (-i) for the forward transform, a * (+i) for the inverse
template <typename V, bool INV> __device__ __forceinline__ V rot(V a) {
  V r;
  if (INV) {
    r.x = -a.y;
    r.y = a.x;
  } else {
    r.x = a.y;
    r.y = -a.x;
  }
  return r;
}

// in-register DFT of length R (natural order in and out), sign - (forward) or + (inverse)
template <typename V, bool INV> __device__ __forceinline__ void dft2(V &a, V &b) {
  const V t = a;
  a = cadd(t, b);
  b = csub(t, b);
}
template <typename V, bool INV> __device__ __forceinline__ void dft4(V &v0, V &v1, V &v2, V &v3) {
  const V t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = rot<V, INV>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}
template <typename V, int R, bool INV> __device__ __forceinline__ void dft(V (&v)[R]) {
  if constexpr (R == 2) {
    dft2<V, INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<V, INV>(v[0], v[1], v[2], v[3]);
  } else {
    static_assert(R == 8, "radix 2, 4 or 8");
    // even / odd halves, then X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k]
    V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<V, INV>(e0, e1, e2, e3);
    dft4<V, INV>(o0, o1, o2, o3);
    using T = decltype(o0.x);
    const T c = T(0.70710678118654752440);
    V w1, w3;  // W8 o1 and W8^3 o3; W8 = (1 -+ i) / sqrt(2)
    if (INV) {
      w1.x = c * (o1.x - o1.y);
      w1.y = c * (o1.x + o1.y);
      w3.x = -c * (o3.x + o3.y);
      w3.y = c * (o3.x - o3.y);
    } else {
      w1.x = c * (o1.x + o1.y);
      w1.y = c * (o1.y - o1.x);
      w3.x = c * (o3.y - o3.x);
      w3.y = -c * (o3.x + o3.y);
    }
    const V w2 = rot<V, INV>(o2);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
  }
}

// Twiddles W_N^m = exp(-2 pi i m / N) from a two-level table in LDS: lo[i] = W_N^i
// (i < 64) and hi[i] = W_N^(64 i) (i < N / 64), W_N^m = hi[m >> 6] lo[m & 63].
template <typename V> struct TwLds {
  V lo[64], hi[32];
};
template <typename V, int N> __device__ __forceinline__ void tw_fill(TwLds<V> &t, const V *__restrict__ tw) {
  const int tid = threadIdx.x;
  if (tid < (N < 64 ? N : 64)) t.lo[tid] = tw[tid];
  if (tid < (N >= 64 ? N / 64 : 0)) t.hi[tid] = tw[64 * tid];
}
template <typename V, int N> __device__ __forceinline__ V tw_get(const TwLds<V> &t, int m) {
  if constexpr (N <= 64) return t.lo[m];
  else return cmul(t.hi[m >> 6], t.lo[m & 63]);
}

// One Stockham stage of radix R over NSEQ sequences of length N in LDS; Ns is the
// length of the sub-transforms already combined.  Butterfly j of a sequence reads
// elements j + r N/R, applies the twiddles W_N^{(j mod Ns) r N/(Ns R)}, takes the
// length-R DFT and writes element (j / Ns) Ns R + (j mod Ns) + r Ns.  All reads of
// the stage complete (barrier) before its writes.
template <typename T, int N, int R, int NSEQ, bool INV>
__device__ __forceinline__ void fft_stage(typename Cx<T>::type *buf, int Ns, const TwLds<typename Cx<T>::type> &tw) {
  using V = typename Cx<T>::type;
  constexpr int NB = NSEQ * N / R, PER = NB / kThreads;
  static_assert(NB % kThreads == 0, "whole butterflies per thread");
  const int tid = threadIdx.x;
  V v[PER][R];
  int dst[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + kThreads * q;
    const int seq = b / (N / R), j = b % (N / R);
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = buf[pad<T>(seq * N + j + r * (N / R))];
    const int k = j & (Ns - 1);
    if (Ns > 1) {
      const int step = N / (Ns * R);
      if constexpr (sizeof(T) == 8) {
        // FP64: one table twiddle per butterfly, its powers by products (at most
        // R - 1 more roundings, ~1e-15); the per-r table reads of FP64 entries
        // were the kernels' main LDS bank conflicts
        V w1 = tw_get<V, N>(tw, k * step);
        if (INV) w1.y = -w1.y;
        V w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[q][r] = cmul(v[q][r], w);
          if (r + 1 < R) w = cmul(w, w1);
        }
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw_get<V, N>(tw, k * r * step);
          if (INV) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
    }
    dft<V, R, INV>(v[q]);
    dst[q] = seq * N + (j / Ns) * Ns * R + k;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pad<T>(dst[q] + r * Ns)] = v[q][r];
  __syncthreads();
}

// unnormalised FFT (INV: exponent sign +) of NSEQ sequences of length 2^LOG2N in LDS
template <typename T, int LOG2N, int NSEQ, bool INV>
__device__ __forceinline__ void fft_lds(typename Cx<T>::type *buf, const TwLds<typename Cx<T>::type> &tw) {
  constexpr int N = 1 << LOG2N;
  int Ns = 1;
#pragma unroll
  for (int s = 0; s < LOG2N / 3; ++s) {
    fft_stage<T, N, 8, NSEQ, INV>(buf, Ns, tw);
    Ns *= 8;
  }
  if constexpr (LOG2N % 3 == 1) fft_stage<T, N, 2, NSEQ, INV>(buf, Ns, tw);
  if constexpr (LOG2N % 3 == 2) fft_stage<T, N, 4, NSEQ, INV>(buf, Ns, tw);
}

// rows forward: grid planes [2][M][M] -> S[kx][y] = (H_x, H_y), kx <= M/2
template <typename T, int LOG2M>
__global__ __launch_bounds__(kThreads) void k_rows_fwd(const T *__restrict__ grid, typename Cx<T>::type *__restrict__ S,
                                                  const typename Cx<T>::type *__restrict__ tw) {
  using V = typename Cx<T>::type;
  constexpr int M = 1 << LOG2M, E = kRowElems<T, M>, B = E / M;
  __shared__ V buf[E + (E >> kPadShift<T>)];
  __shared__ TwLds<V> twl;
  const int tid = threadIdx.x;
  const int y0 = xcd_remap(blockIdx.x, gridDim.x) * B;
  const size_t plane = (size_t)M * M;
  constexpr int NL = E / kThreads;  // every load of the thread in flight before the first store
  static_assert(E % kThreads == 0, "whole rows per work group");
  V z[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const size_t g = (size_t)y0 * M + tid + q * kThreads;  // rows y0 .. y0 + B - 1 are contiguous
    z[q].x = grid[g];
    z[q].y = grid[plane + g];
  }
  tw_fill<V, M>(twl, tw);
#pragma unroll
  for (int q = 0; q < NL; ++q) buf[pad<T>(tid + q * kThreads)] = z[q];
  __syncthreads();
  fft_lds<T, LOG2M, B, false>(buf, twl);
  // H_x = (Z[k] + conj Z[M-k]) / 2, H_y = (Z[k] - conj Z[M-k]) / 2i; row index fastest
  for (int e = tid; e < (M / 2 + 1) * B; e += kThreads) {
    const int r = e % B, kx = e / B;
    const V Z = buf[pad<T>(r * M + kx)], Zm = buf[pad<T>(r * M + ((M - kx) & (M - 1)))];
    V h0, h1;
    h0.x = T(0.5) * (Z.x + Zm.x);
    h0.y = T(0.5) * (Z.y - Zm.y);
    h1.x = T(0.5) * (Z.y + Zm.y);
    h1.y = T(-0.5) * (Z.x - Zm.x);
    V *dst = S + 2 * ((size_t)kx * M + y0 + r);
    dst[0] = h0;
    dst[1] = h1;
  }
}

// columns: per kx, FFT along y of both components, multiplier, inverse FFT.
// The M/2 + 1 columns kx = 0 .. M/2 occupy M/2 column slots: H_c(0, y) and
// H_c(M/2, y) are real (sums of real data along x), so slot 0 carries them as
// one complex column H_c(0, y) + i H_c(M/2, y), whose spectrum splits by
// Hermitian symmetry into the two columns' spectra (as the row transform splits
// g_x + i g_y).  Without that, the one column past M/2 slots would run as an
// extra round of work groups after all the others.
template <typename T, int LOG2M, int MODE>
__global__ __launch_bounds__(kThreads) void k_cols(typename Cx<T>::type *__restrict__ S,
                                              const typename Cx<T>::type *__restrict__ tw,
                                              const T *__restrict__ ey, T twopi_L, T inv4xi2, T one_m_eta, T scale) {
  using V = typename Cx<T>::type;
  constexpr int M = 1 << LOG2M, E = kElems<T>, CB = E / (2 * M), NSLOT = M / 2;
  __shared__ V buf[E + (E >> kPadShift<T>)];
  __shared__ TwLds<V> twl;
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * CB;
  constexpr int NL = CB * M / kThreads;
  static_assert((CB * M) % kThreads == 0, "whole columns per work group");
  V a[NL], b[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + q * kThreads, c = e >> LOG2M, y = e & (M - 1), kxi = c0 + c;
    a[q].x = a[q].y = b[q].x = b[q].y = T(0);
    if (kxi == 0) {  // packed slot: real parts of the kx = 0 and kx = M/2 columns
      const V *s0 = S + 2 * (size_t)y, *sn = S + 2 * ((size_t)(M / 2) * M + y);
      a[q].x = s0[0].x;
      a[q].y = sn[0].x;
      b[q].x = s0[1].x;
      b[q].y = sn[1].x;
    } else if (kxi < NSLOT) {
      const V *src = S + 2 * ((size_t)kxi * M + y);
      a[q] = src[0];
      b[q] = src[1];
    }
  }
  tw_fill<V, M>(twl, tw);
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + q * kThreads, c = e >> LOG2M, y = e & (M - 1);
    buf[pad<T>(2 * c * M + y)] = a[q];
    buf[pad<T>((2 * c + 1) * M + y)] = b[q];
  }
  __syncthreads();
  fft_lds<T, LOG2M, 2 * CB, false>(buf, twl);
  // (g0, g1) = multiplier(kxi, ky) (f0, f1)
  auto mult = [&](int kxi, int ky, const V &f0, const V &f1, V &g0, V &g1) {
    T sc, pxx, pxy, pyy;
    bool nz;
    if (MODE == 0) {
      // M^(w): the Gaussian factor exp(-(1-eta_s) k^2 / 4 xi^2) is the product of
      // its kx and ky factors, both read from the table ey (indexed by frequency index)
      const T kx = twopi_L * kxi, kyv = twopi_L * (ky < M / 2 ? ky : ky - M);
      const T k2 = kx * kx + kyv * kyv;
      nz = k2 != T(0);
      if (nz) {
        const T ik2 = T(1) / k2;
        sc = (T(1) + k2 * inv4xi2) * ey[kxi] * ey[ky] * ik2 * scale;
        pxx = T(1) - kx * kx * ik2;
        pyy = T(1) - kyv * kyv * ik2;
        pxy = (kxi == M / 2 || ky == M / 2) ? T(0) : -kx * kyv * ik2;
      }
    } else {
      nz = wave_multiplier<T>(M, ky, kxi, twopi_L, inv4xi2, one_m_eta, scale, MODE, sc, pxx, pxy, pyy);
    }
    if (nz) {
      g0.x = sc * (pxx * f0.x + pxy * f1.x);
      g0.y = sc * (pxx * f0.y + pxy * f1.y);
      g1.x = sc * (pxy * f0.x + pyy * f1.x);
      g1.y = sc * (pxy * f0.y + pyy * f1.y);
    } else {
      g0.x = g0.y = g1.x = g1.y = T(0);
    }
  };
  for (int e = tid; e < CB * M; e += kThreads) {
    const int c = e >> LOG2M, ky = e & (M - 1), kxi = c0 + c;
    if (kxi >= NSLOT) continue;
    V &f0 = buf[pad<T>(2 * c * M + ky)];
    V &f1 = buf[pad<T>((2 * c + 1) * M + ky)];
    if (kxi != 0) {
      V g0, g1;
      mult(kxi, ky, f0, f1, g0, g1);
      f0 = g0;
      f1 = g1;
      continue;
    }
    // packed slot, by pairs (ky, M - ky): the spectra A (kx = 0) and B (kx = M/2)
    // of each component are A = (Z(ky) + conj Z(-ky)) / 2, B = (Z(ky) - conj Z(-ky)) / 2i;
    // both stay Hermitian under their multipliers, so Z' = A' + i B' at ky and
    // conj A' + i conj B' at -ky
    if (ky > M / 2) continue;
    const int km = (M - ky) & (M - 1);
    V &m0 = buf[pad<T>(2 * c * M + km)];
    V &m1 = buf[pad<T>((2 * c + 1) * M + km)];
    V A0, B0, A1, B1;
    A0.x = T(0.5) * (f0.x + m0.x);
    A0.y = T(0.5) * (f0.y - m0.y);
    B0.x = T(0.5) * (f0.y + m0.y);
    B0.y = T(-0.5) * (f0.x - m0.x);
    A1.x = T(0.5) * (f1.x + m1.x);
    A1.y = T(0.5) * (f1.y - m1.y);
    B1.x = T(0.5) * (f1.y + m1.y);
    B1.y = T(-0.5) * (f1.x - m1.x);
    V a0, a1, b0, b1;
    mult(0, ky, A0, A1, a0, a1);
    mult(M / 2, ky, B0, B1, b0, b1);
    V z0, z1, w0, w1;
    z0.x = a0.x - b0.y;
    z0.y = a0.y + b0.x;
    z1.x = a1.x - b1.y;
    z1.y = a1.y + b1.x;
    w0.x = a0.x + b0.y;
    w0.y = b0.x - a0.y;
    w1.x = a1.x + b1.y;
    w1.y = b1.x - a1.y;
    m0 = w0;  // ky = 0 and M/2 are their own partners; there z and w agree
    m1 = w1;
    f0 = z0;
    f1 = z1;
  }
  __syncthreads();
  fft_lds<T, LOG2M, 2 * CB, true>(buf, twl);
  for (int e = tid; e < CB * M; e += kThreads) {
    const int c = e >> LOG2M, y = e & (M - 1), kxi = c0 + c;
    if (kxi >= NSLOT) continue;
    const V u0 = buf[pad<T>(2 * c * M + y)], u1 = buf[pad<T>((2 * c + 1) * M + y)];
    if (kxi == 0) {  // real parts: kx = 0; imaginary parts: kx = M/2
      V *d0 = S + 2 * (size_t)y, *dn = S + 2 * ((size_t)(M / 2) * M + y);
      V r;
      r.y = T(0);
      r.x = u0.x;
      d0[0] = r;
      r.x = u1.x;
      d0[1] = r;
      r.x = u0.y;
      dn[0] = r;
      r.x = u1.y;
      dn[1] = r;
    } else {
      V *dst = S + 2 * ((size_t)kxi * M + y);
      dst[0] = u0;
      dst[1] = u1;
    }
  }
}

// rows inverse: S -> grid planes; Z[k] = U_x[k] + i U_y[k] over the Hermitian extension
template <typename T, int LOG2M>
__global__ __launch_bounds__(kThreads) void k_rows_inv(const typename Cx<T>::type *__restrict__ S, T *__restrict__ grid,
                                                  const typename Cx<T>::type *__restrict__ tw) {
  using V = typename Cx<T>::type;
  constexpr int M = 1 << LOG2M, E = kRowElems<T, M>, B = E / M;
  __shared__ V buf[E + (E >> kPadShift<T>)];
  __shared__ TwLds<V> twl;
  const int tid = threadIdx.x;
  const int y0 = xcd_remap(blockIdx.x, gridDim.x) * B;
  constexpr int NI = (M / 2 + 1) * B, NL = (NI + kThreads - 1) / kThreads;
  V a[NL], b[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + q * kThreads, r = e % B, k = e / B;
    if (e < NI) {
      const V *src = S + 2 * ((size_t)k * M + y0 + r);
      a[q] = src[0];
      b[q] = src[1];
    }
  }
  tw_fill<V, M>(twl, tw);
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + q * kThreads, r = e % B, k = e / B;
    if (e >= NI) continue;
    V g0 = a[q], g1 = b[q];
    if (k == 0 || k == M / 2) g0.y = g1.y = T(0);
    V z;
    z.x = g0.x - g1.y;
    z.y = g0.y + g1.x;
    buf[pad<T>(r * M + k)] = z;
    if (k > 0 && k < M / 2) {  // conj(U_x[k]) + i conj(U_y[k]) at M - k
      V zc;
      zc.x = g0.x + g1.y;
      zc.y = g1.x - g0.y;
      buf[pad<T>(r * M + M - k)] = zc;
    }
  }
  __syncthreads();
  fft_lds<T, LOG2M, B, true>(buf, twl);
  const size_t plane = (size_t)M * M;
  for (int e = tid; e < E; e += kThreads) {
    const V z = buf[pad<T>(e)];
    const size_t g = (size_t)y0 * M + e;
    grid[g] = z.x;
    grid[plane + g] = z.y;
  }
}

template <typename T, int LOG2M>
hipError_t conv_launch(const WaveConvArgs &a, T *grid, typename Cx<T>::type *spec,
                       const typename Cx<T>::type *tw, const T *ey, hipStream_t s) {
  constexpr int M = 1 << LOG2M, E = kElems<T>, ER = kRowElems<T, M>;
  constexpr int rows_blocks = M / (ER / M), col_blocks = (M / 2 + E / (2 * M) - 1) / (E / (2 * M));
  hipLaunchKernelGGL((k_rows_fwd<T, LOG2M>), dim3(rows_blocks), dim3(kThreads), 0, s, grid, spec, tw);
  const T twopi_L = (T)(2.0 * M_PI / a.L), inv4xi2 = (T)(1.0 / (4.0 * a.xi * a.xi)), ome = (T)(1.0 - a.eta_s);
  if (a.mode == 0)
    hipLaunchKernelGGL((k_cols<T, LOG2M, 0>), dim3(col_blocks), dim3(kThreads), 0, s, spec, tw, ey, twopi_L, inv4xi2,
                       ome, (T)a.scale);
  else
    hipLaunchKernelGGL((k_cols<T, LOG2M, 1>), dim3(col_blocks), dim3(kThreads), 0, s, spec, tw, ey, twopi_L, inv4xi2,
                       ome, (T)a.scale);
  hipLaunchKernelGGL((k_rows_inv<T, LOG2M>), dim3(rows_blocks), dim3(kThreads), 0, s, spec, grid, tw);
  return hipGetLastError();
}

template <typename T>
hipError_t conv_dispatch(const WaveConvArgs &a, T *grid, T *spec, const T *tw, const T *ey, hipStream_t s) {
  using V = typename Cx<T>::type;
  V *sp = reinterpret_cast<V *>(spec);
  const V *t = reinterpret_cast<const V *>(tw);
  switch (a.M) {
    case 64: return conv_launch<T, 6>(a, grid, sp, t, ey, s);
    case 128: return conv_launch<T, 7>(a, grid, sp, t, ey, s);
    case 256: return conv_launch<T, 8>(a, grid, sp, t, ey, s);
    case 512: return conv_launch<T, 9>(a, grid, sp, t, ey, s);
    case 1024: return conv_launch<T, 10>(a, grid, sp, t, ey, s);
    case 2048: return conv_launch<T, 11>(a, grid, sp, t, ey, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool wave_conv_supported(int M) { return M >= 64 && M <= 2048 && (M & (M - 1)) == 0; }

hipError_t launch_wave_conv_f64(const WaveConvArgs &a, double *grid, double *spec, const double *tw, const double *ey,
                                hipStream_t s) {
  return conv_dispatch<double>(a, grid, spec, tw, ey, s);
}

hipError_t launch_wave_conv_f32(const WaveConvArgs &a, float *grid, float *spec, const float *tw, const float *ey,
                                hipStream_t s) {
  return conv_dispatch<float>(a, grid, spec, tw, ey, s);
}

}  // namespace fbim
