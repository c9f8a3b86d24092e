// Wave-space part of the single-layer matvec (Section 3.2, eqs. 3.21-3.25) and
// the random Fourier field (Section 3.3, eqs. 3.28-3.30):
//   spread  S : H_c(x_g) = sum_n mu_{n,c} g(x_g - x_n), g = cg exp(-ag r^2), P x P
//               nearest grid points; each work group owns a T x T grid tile and
//               accumulates it in LDS (no global atomics);
//   multiply B: on the half spectrum, with the Gaussian deconvolution folded in;
//   interp  S*: v_n = h^2 sum_g g(x_n - x_g) U(x_g), grid window staged in LDS.
// The FFTs in between are rocFFT plans owned by the context.
#include <type_traits>

#include "kernels.h"

namespace fbim {

namespace {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

__device__ inline double dev_exp(double x) { return exp(x); }
__device__ inline float dev_exp(float x) { return __expf(x); }

constexpr int kTmax = 32;
constexpr int kPmax = 15;

__device__ inline int wrapi(int i, int M) {
  i %= M;
  return i < 0 ? i + M : i;
}

__device__ inline int xcd_remap(int b, int n) {
  const int q = n / 8, r = n % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// One 256-thread work group per T x T grid tile, accumulated in LDS (no global
// atomics).  The nodes whose stencil touches the tile come from the tile's
// spreading list (built once per configuration); they are taken in chunks of
// kSpreadChunk: per chunk the P x- and P y-weights of every node are computed
// once (x and y weights by two threads), then the (node, stencil row) items are
// spread over the threads and added with LDS atomics.  The node data of the first
// kSpreadPre chunks is requested before any of them is used.
constexpr int kSpreadChunk = 128;
constexpr int kSpreadPre = 4;
// dynamic LDS of the spreading kernels: x and y weights of a chunk, P per entry
inline size_t spread_lds_bytes(int P, size_t elem) { return 2 * (size_t)kSpreadChunk * P * elem; }

__device__ inline int wrap_near(int i, int M) {  // valid for -M <= i < 2M
  return i < 0 ? i + M : (i >= M ? i - M : i);
}

// stencil origin (first column or row) of a node relative to the tile origin g0, in [0, M)
__device__ inline int stencil_origin(int a, int half, int g0, int M) {
  return wrap_near((a - half) - g0 + (a - half < 0 ? M : 0), M);
}

__global__ __launch_bounds__(256) void k_spread_lists(int M, int TT, int P, int nts, const int *__restrict__ tile_start,
                                                      const int2 *__restrict__ anchor, int *__restrict__ count,
                                                      const int *__restrict__ start, int *__restrict__ list,
                                                      int mode) {
  __shared__ int wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int tile = blockIdx.x;
  const int tyi = tile / nts, txi = tile % nts;
  const int gx0 = txi * TT, gy0 = tyi * TT;
  const int half = (P - 1) / 2;
  int nstart[9], pre[10];
  pre[0] = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int dx = k % 3 - 1, dy = k / 3 - 1;
    const int tt = wrap_near(tyi + dy, nts) * nts + wrap_near(txi + dx, nts);
    nstart[k] = tile_start[tt];
    pre[k + 1] = pre[k] + tile_start[tt + 1] - tile_start[tt];
  }
  const int ncand = pre[9];
  const int base = mode ? start[tile] : 0;
  int running = 0;
  for (int v0 = 0; v0 < ncand; v0 += 256) {
    const int v = v0 + tid;
    bool ok = false;
    int g = 0;
    if (v < ncand) {
      int k = 0;
      while (k < 8 && v >= pre[k + 1]) ++k;
      g = nstart[k] + (v - pre[k]);
      const int2 an = anchor[g];
      const int ux = stencil_origin(an.x, half, gx0, M), uy = stencil_origin(an.y, half, gy0, M);
      ok = (ux < TT || ux + P - 1 >= M) && (uy < TT || uy + P - 1 >= M);
    }
    const unsigned long long m = __ballot(ok);
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      off += q < wv ? wsum[q] : 0;
      tot += wsum[q];
    }
    if (mode && ok) list[base + running + off + __popcll(m & ((1ull << lane) - 1ull))] = g;
    running += tot;
    __syncthreads();
  }
  if (mode == 0 && tid == 0) count[tile] = running;
}

// Gaussian weights w_k = scale exp(-ag d_k^2) on the stencil, d_k = x + (half - k) h.
// FP64 uses the product recurrence of fast Gaussian gridding: with d0 = x + half h,
// w_{k+1} = w_k exp(2 ag d0 h) exp(-ag h^2 (2k + 1)), the last factors being the
// per-kernel constants ck[k] = gauss_step(k): two exponentials per node and
// direction instead of P, at most P more roundings (~1e-15).  FP32 evaluates each
// weight directly (the hardware exponential is cheap and the recurrence's
// roundings would be ~1e-6).
template <typename T>
__device__ inline T gauss_step(T ag, T h, int k) {
  return dev_exp(-ag * h * h * T(2 * k + 1));
}
template <typename T>
__device__ inline void gauss_row(T x, T scale, T ag, T h, int half, int P, const T *ck, T *w) {
  if constexpr (sizeof(T) == 8) {
    const T d0 = x + T(half) * h;
    const T e1 = dev_exp(T(2) * ag * d0 * h);
    T v = scale * dev_exp(-ag * d0 * d0);
    for (int k = 0; k < P; ++k) {
      w[k] = v;
      v = v * e1 * ck[k];
    }
  } else {
    for (int k = 0; k < P; ++k) {
      const T d = x + T(half - k) * h;
      w[k] = scale * dev_exp(-ag * d * d);
    }
  }
}

__device__ __forceinline__ unsigned long long to_fixed(float v) { return (unsigned long long)__float2ll_rn(v); }
__device__ __forceinline__ unsigned long long to_fixed(double v) { return (unsigned long long)__double2ll_rn(v); }

// T: weights and positions; A: LDS accumulator.  FP64: double (FP64 LDS atomic
// adds).  FP32: 64-bit fixed point (unsigned long long, two's complement) with a
// per-tile power-of-two scale S: a grid point of the tile receives at most one
// term per list entry, each at most cg max|mu| in magnitude (weights <= cg in y,
// <= 1 in x), so with B = 2 n cg max|mu| (n entries, factor 2 for FP32 rounding)
// and S B <= 2^62 no sum can overflow, and the resolution B / 2^62 is far below
// the FP32 rounding of the terms: the sums are exact.  64-bit integer LDS atomics
// ran at 83 us against 95 us for FP64 ones (FP32 LDS atomics: 550 us; 32-bit
// fixed point, 65 us, was too coarse at B / 2^30 and cost GMRES iterations), and
// integer sums do not depend on their order.
template <typename T, typename A>
__device__ __forceinline__ void spread_body(int M, int TT, int P, int nts, T h, T ag, T cg, const int *__restrict__ slist_start,
                            const int *__restrict__ slist, const typename Vec2<T>::type *__restrict__ xt,
                            const int2 *__restrict__ anchor, const typename Vec2<T>::type *__restrict__ mut,
                            T *__restrict__ grid, int tile) {
  using V2 = typename Vec2<T>::type;
  __shared__ A acc[2][kTmax * (kTmax + 1)];  // rows padded by one: a node's P rows fall in distinct banks
  // the P x- and y-weights of each chunk entry, rows of P: dynamic LDS sized for
  // the launch's P (spread_lds_bytes), so small stencils leave room for more
  // work groups per CU
  extern __shared__ double spread_wbuf[];
  T *wgx = reinterpret_cast<T *>(spread_wbuf), *wgy = wgx + kSpreadChunk * P;
  __shared__ T nmx[kSpreadChunk], nmy[kSpreadChunk], ck[kPmax];
  __shared__ int nbx[kSpreadChunk], nby[kSpreadChunk], ncol[kSpreadChunk];
  const int tid = threadIdx.x;
  const int tyi = tile / nts, txi = tile % nts;
  const int gx0 = txi * TT, gy0 = tyi * TT;
  const int half = (P - 1) / 2;
  const int ST = TT + 1;
  const int ls = slist_start[tile], n = slist_start[tile + 1] - ls;
  // thread t serves entry (chunk base + t % 128): its x weights (t < 128) or y weights
  const int e0 = tid & (kSpreadChunk - 1);
  const bool ycomp = tid >= kSpreadChunk;
  V2 pr[kSpreadPre], mr[kSpreadPre];
  int2 ar[kSpreadPre];
#pragma unroll
  for (int r = 0; r < kSpreadPre; ++r) {
    const int e = e0 + kSpreadChunk * r;
    if (e < n) {
      const int g = slist[ls + e];
      pr[r] = xt[g];
      mr[r] = mut[g];
      ar[r] = anchor[g];
    }
  }
  for (int i = tid; i < TT * ST; i += 256) acc[0][i] = acc[1][i] = A(0);
  if (tid < P) ck[tid] = gauss_step<T>(ag, h, tid);
  constexpr bool kFixed = std::is_same<A, unsigned long long>::value;
  T S = T(1);       // fixed-point scale (kFixed)
  bool finite = true;  // a non-finite density makes the tile's grid NaN (as floating-point sums would)
  if constexpr (kFixed) {
    __shared__ T red[4];
    // max |mu| over the list; any NaN or infinity (which fmax would skip) is flagged
    T m = T(0);
    int bad = 0;
    auto take = [&](V2 mu) {
      const T a = fmax(fabs(mu.x), fabs(mu.y));
      bad |= !(fabs(mu.x) <= T(3.0e38) && fabs(mu.y) <= T(3.0e38));
      m = fmax(m, a);
    };
#pragma unroll
    for (int r = 0; r < kSpreadPre; ++r)
      if (e0 + kSpreadChunk * r < n) take(mr[r]);
    for (int e = kSpreadChunk * kSpreadPre + tid; e < n; e += 256) take(mut[slist[ls + e]]);  // rare: crowded tiles
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((tid & 63) == 0) red[tid >> 6] = m;
    finite = __syncthreads_or(bad) == 0;  // also the barrier for red
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double B = 2.0 * (double)n * (double)cg * (double)m;  // no overflow for finite FP32 inputs
    if (finite && B > 0.0) {
      int k;
      frexp(B, &k);  // B < 2^k
      constexpr int kMaxE = sizeof(T) == 4 ? 126 : 1000;
      S = ldexp(T(1), max(min(62 - k, kMaxE), -kMaxE));
    }
  }
  __syncthreads();  // ck (and the zeroed accumulator) before any use

  // per entry: the stencil's first row / column relative to the tile (negative when
  // it starts in the neighbouring tile across a periodic edge), the columns
  // [pc0, pc1) that fall in the tile, and the P weights per direction
  auto weights = [&](V2 p, V2 mu, int2 an) {
    if (!ycomp) {
      const int ox = stencil_origin(an.x, half, gx0, M);
      const int xs = ox < TT ? ox : ox - M;
      nbx[e0] = xs;
      ncol[e0] = max(0, -xs) | (min(P, TT - xs) << 8);
      nmx[e0] = mu.x;
      nmy[e0] = mu.y;
      gauss_row<T>(p.x, T(1), ag, h, half, P, ck, wgx + e0 * P);
    } else {
      const int oy = stencil_origin(an.y, half, gy0, M);
      nby[e0] = oy < TT ? oy : oy - M;
      gauss_row<T>(p.y, cg, ag, h, half, P, ck, wgy + e0 * P);
    }
  };
  const float invP = 1.0f / (float)P;
  auto items = [&](int cnt) {
    for (int it = tid; it < cnt * P; it += 256) {
      const int j = (int)(((float)it + 0.5f) * invP), q = it - j * P;  // it / P, exact for it < 2^20
      const int ry = nby[j] + q;
      if (ry < 0 || ry >= TT) continue;
      const T wy = wgy[j * P + q];
      const T ux = wy * nmx[j], uy = wy * nmy[j];
      const int cr = ncol[j], xs = nbx[j];
      A *a0 = &acc[0][ry * ST + xs], *a1 = &acc[1][ry * ST + xs];
      if constexpr (kFixed) {
        const T sx = ux * S, sy = uy * S;  // exact: S is a power of two
        for (int pc = cr & 255; pc < (cr >> 8); ++pc) {
          const T wx = wgx[j * P + pc];
          atomicAdd(a0 + pc, to_fixed(sx * wx));
          atomicAdd(a1 + pc, to_fixed(sy * wx));
        }
      } else {
        for (int pc = cr & 255; pc < (cr >> 8); ++pc) {
          const T wx = wgx[j * P + pc];
          atomicAdd(a0 + pc, (A)(ux * wx));
          atomicAdd(a1 + pc, (A)(uy * wx));
        }
      }
    }
  };
#pragma unroll
  for (int r = 0; r < kSpreadPre; ++r) {
    const int c = kSpreadChunk * r;
    if (c >= n) break;  // n is uniform over the work group
    const int cnt = min(kSpreadChunk, n - c);
    if (e0 < cnt) weights(pr[r], mr[r], ar[r]);
    __syncthreads();
    items(cnt);
    __syncthreads();
  }
  for (int c = kSpreadChunk * kSpreadPre; c < n; c += kSpreadChunk) {  // rare: crowded tiles
    const int cnt = min(kSpreadChunk, n - c);
    if (e0 < cnt) {
      const int g = slist[ls + c + e0];
      weights(xt[g], mut[g], anchor[g]);
    }
    __syncthreads();
    items(cnt);
    __syncthreads();
  }
  for (int i = tid; i < TT * TT; i += 256) {
    const int ry = i / TT, rx = i - ry * TT;
    const size_t gidx = (size_t)(gy0 + ry) * M + gx0 + rx;
    if constexpr (kFixed) {
      const T inv = finite ? T(1) / S : T(NAN);  // exact power of two
      grid[gidx] = (T)(long long)acc[0][ry * ST + rx] * inv;
      grid[(size_t)M * M + gidx] = (T)(long long)acc[1][ry * ST + rx] * inv;
    } else {
      grid[gidx] = (T)acc[0][ry * ST + rx];
      grid[(size_t)M * M + gidx] = (T)acc[1][ry * ST + rx];
    }
  }
}

template <typename T>
__device__ __forceinline__ void interp_body(int M, int TT, int P, int nts, T h, T ag, T scale, const int *__restrict__ tile_start,
                            const typename Vec2<T>::type *__restrict__ xt, const int2 *__restrict__ anchor,
                            const int *__restrict__ tperm, const T *__restrict__ grid, double *__restrict__ out,
                            int tile) {
  constexpr int W = kTmax + kPmax - 1;
  __shared__ T win[2][W * W];
  __shared__ T ck[kPmax];
  const int tid = threadIdx.x;
  const int tyi = tile / nts, txi = tile % nts;
  const int gx0 = txi * TT, gy0 = tyi * TT;
  const int half = (P - 1) / 2;
  const int w = TT + P - 1;
  for (int i = tid; i < w * w; i += 256) {
    const int ry = i / w, rx = i - ry * w;
    const size_t gidx = (size_t)wrapi(gy0 - half + ry, M) * M + wrapi(gx0 - half + rx, M);
    win[0][i] = grid[gidx];
    win[1][i] = grid[(size_t)M * M + gidx];
  }
  if (tid < P) ck[tid] = gauss_step<T>(ag, h, tid);
  __syncthreads();
  const int a = tile_start[tile], b = tile_start[tile + 1];
  for (int k = a + tid; k < b; k += 256) {
    const auto p = xt[k];
    const int2 an = anchor[k];
    const int ixn = an.x, iyn = an.y;
    const int bx = wrapi(ixn - half - (gx0 - half), M);  // window column of the first stencil point
    const int by = wrapi(iyn - half - (gy0 - half), M);
    // weights of the stencil's columns and rows (offsets p + (half - k) h from the
    // nearest grid point) by the product recurrence
    T wx[kPmax], wyr[kPmax];
    gauss_row<T>(p.x, T(1), ag, h, half, P, ck, wx);
    gauss_row<T>(p.y, T(1), ag, h, half, P, ck, wyr);
    T sx = 0, sy = 0;
    for (int qr = 0; qr < P; ++qr) {
      const T wy = wyr[qr];
      const T *r0 = &win[0][(by + qr) * w + bx];
      const T *r1 = &win[1][(by + qr) * w + bx];
      T rx0 = 0, rx1 = 0;
      for (int pc = 0; pc < P; ++pc) {
        rx0 += wx[pc] * r0[pc];
        rx1 += wx[pc] * r1[pc];
      }
      sx += wy * rx0;
      sy += wy * rx1;
    }
    const int node = tperm[k];
    out[2 * node] += (double)(scale * sx);
    out[2 * node + 1] += (double)(scale * sy);
  }
}

// multiplier on the rocFFT half spectrum (plane c at [c][row][col], col <= M/2),
// coefficients from wave_multiplier
template <typename T>
__device__ __forceinline__ void multiplier_body(int M, T twopi_L, T inv4xi2, T one_m_eta, T scale, int mode,
                                typename Vec2<T>::type *__restrict__ spec, int idx) {
  const int nh = M / 2 + 1;
  if (idx >= M * nh) return;
  const int row = idx / nh, col = idx - row * nh;
  auto &Fx = spec[idx];
  auto &Fy = spec[(size_t)M * nh + idx];
  T sc, pxx, pxy, pyy;
  if (!wave_multiplier<T>(M, row, col, twopi_L, inv4xi2, one_m_eta, scale, mode, sc, pxx, pxy, pyy)) {
    Fx.x = Fx.y = Fy.x = Fy.y = T(0);
    return;
  }
  const auto fx = Fx, fy = Fy;
  Fx.x = sc * (pxx * fx.x + pxy * fy.x);
  Fx.y = sc * (pxx * fx.y + pxy * fy.y);
  Fy.x = sc * (pxy * fx.x + pyy * fy.x);
  Fy.y = sc * (pxy * fx.y + pyy * fy.y);
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_spread(int M, int TT, int P, int nts, T h, T ag, T cg,
                                                const int *__restrict__ slist_start, const int *__restrict__ slist,
                                                const typename Vec2<T>::type *__restrict__ xt,
                                                const int2 *__restrict__ anchor,
                                                const typename Vec2<T>::type *__restrict__ mut,
                                                T *__restrict__ grid) {
  spread_body<T, A>(M, TT, P, nts, h, ag, cg, slist_start, slist, xt, anchor, mut, grid,
                    xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T>
__global__ __launch_bounds__(256) void k_interp(int M, int TT, int P, int nts, T h, T ag, T scale,
                                                const int *__restrict__ tile_start,
                                                const typename Vec2<T>::type *__restrict__ xt,
                                                const int2 *__restrict__ anchor,
                                                const int *__restrict__ tperm, const T *__restrict__ grid,
                                                double *__restrict__ out) {
  interp_body<T>(M, TT, P, nts, h, ag, scale, tile_start, xt, anchor, tperm, grid, out,
                 xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T>
__global__ void k_multiplier(int M, T twopi_L, T inv4xi2, T one_m_eta, T scale, int mode,
                             typename Vec2<T>::type *__restrict__ spec) {
  multiplier_body<T>(M, twopi_L, inv4xi2, one_m_eta, scale, mode, spec, blockIdx.x * blockDim.x + threadIdx.x);
}

// batched forms: the XCD-aware order is taken over the whole grid, then the
// block's system and its tile within that system are found
template <typename T, typename A>
__global__ __launch_bounds__(256) void k_spread_batch(const SpreadJob *__restrict__ jobs, BatchGrid bg) {
  using V2 = typename Vec2<T>::type;
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = batch_system(bg.begin, bg.S, gb);
  const SpreadJob &j = jobs[s];
  spread_body<T, A>(j.w.M, j.w.T, j.w.P, j.w.nts, (T)j.w.h, (T)j.w.ag, (T)j.w.cg, j.w.slist_start, j.w.slist,
                    reinterpret_cast<const V2 *>(j.xt), reinterpret_cast<const int2 *>(j.w.anchor),
                    reinterpret_cast<const V2 *>(j.mut), reinterpret_cast<T *>(j.grid), gb - bg.begin[s]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_interp_batch(const InterpJob *__restrict__ jobs, BatchGrid bg) {
  using V2 = typename Vec2<T>::type;
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = batch_system(bg.begin, bg.S, gb);
  const InterpJob &j = jobs[s];
  interp_body<T>(j.w.M, j.w.T, j.w.P, j.w.nts, (T)j.w.h, (T)j.w.ag, (T)(j.w.h * j.w.h * j.w.cg), j.w.tile_start,
                 reinterpret_cast<const V2 *>(j.xt), reinterpret_cast<const int2 *>(j.w.anchor), j.tperm,
                 reinterpret_cast<const T *>(j.grid), j.out, gb - bg.begin[s]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_multiplier_batch(const MultJob *__restrict__ jobs, BatchGrid bg, int mode) {
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  const MultJob &j = jobs[s];
  multiplier_body<T>(j.M, (T)(2.0 * M_PI / j.L), (T)(1.0 / (4.0 * j.xi * j.xi)), (T)(1.0 - j.eta_s), (T)j.scale,
                     mode, reinterpret_cast<typename Vec2<T>::type *>(j.spec),
                     (blockIdx.x - bg.begin[s]) * 256 + threadIdx.x);
}

}  // namespace

hipError_t launch_spread_batch(const SpreadJob *jobs, BatchGrid bg, int f32, int pmax, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (pmax < 1 || pmax > kPmax) return hipErrorInvalidValue;
  if (f32)
    hipLaunchKernelGGL((k_spread_batch<float, unsigned long long>), dim3(bg.nblocks), dim3(256), spread_lds_bytes(pmax, 4), s,
                       jobs, bg);
  else
    hipLaunchKernelGGL((k_spread_batch<double, unsigned long long>), dim3(bg.nblocks), dim3(256), spread_lds_bytes(pmax, 8), s,
                       jobs, bg);
  return hipGetLastError();
}

hipError_t launch_interp_batch(const InterpJob *jobs, BatchGrid bg, int f32, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL((k_interp_batch<float>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg);
  else
    hipLaunchKernelGGL((k_interp_batch<double>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg);
  return hipGetLastError();
}

hipError_t launch_multiplier_batch(const MultJob *jobs, BatchGrid bg, int f32, int mode, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL((k_multiplier_batch<float>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg, mode);
  else
    hipLaunchKernelGGL((k_multiplier_batch<double>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg, mode);
  return hipGetLastError();
}

hipError_t launch_spread_lists(const WaveArgs &w, int *count, const int *start, int *list, int mode, hipStream_t s) {
  const int nt = w.nts * w.nts;
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spread_lists, dim3(nt), dim3(256), 0, s, w.M, w.T, w.P, w.nts, w.tile_start,
                     (const int2 *)w.anchor, count, start, list, mode);
  return hipGetLastError();
}

hipError_t launch_spread_f64(const WaveArgs &w, const double *xt, const double *mut, double *grid, hipStream_t s) {
  const int nt = w.nts * w.nts;
  hipLaunchKernelGGL((k_spread<double, unsigned long long>), dim3(nt), dim3(256), spread_lds_bytes(w.P, 8), s, w.M, w.T, w.P, w.nts, w.h, w.ag, w.cg,
                     w.slist_start, w.slist, (const double2 *)xt, (const int2 *)w.anchor, (const double2 *)mut, grid);
  return hipGetLastError();
}

hipError_t launch_spread_f32(const WaveArgs &w, const float *xt, const float *mut, float *grid, hipStream_t s) {
  const int nt = w.nts * w.nts;
  hipLaunchKernelGGL((k_spread<float, unsigned long long>), dim3(nt), dim3(256), spread_lds_bytes(w.P, 4), s, w.M, w.T, w.P, w.nts, (float)w.h, (float)w.ag,
                     (float)w.cg, w.slist_start, w.slist, (const float2 *)xt, (const int2 *)w.anchor, (const float2 *)mut,
                     grid);
  return hipGetLastError();
}

hipError_t launch_interp_f64(const WaveArgs &w, const double *xt, const int *tperm, const double *grid,
                             double *out, hipStream_t s) {
  const int nt = w.nts * w.nts;
  hipLaunchKernelGGL(k_interp<double>, dim3(nt), dim3(256), 0, s, w.M, w.T, w.P, w.nts, w.h, w.ag,
                     w.h * w.h * w.cg, w.tile_start, (const double2 *)xt, (const int2 *)w.anchor, tperm, grid, out);
  return hipGetLastError();
}

hipError_t launch_interp_f32(const WaveArgs &w, const float *xt, const int *tperm, const float *grid, double *out,
                             hipStream_t s) {
  const int nt = w.nts * w.nts;
  hipLaunchKernelGGL(k_interp<float>, dim3(nt), dim3(256), 0, s, w.M, w.T, w.P, w.nts, (float)w.h, (float)w.ag,
                     (float)(w.h * w.h * w.cg), w.tile_start, (const float2 *)xt, (const int2 *)w.anchor, tperm,
                     grid, out);
  return hipGetLastError();
}

hipError_t launch_multiplier_f64(int M, double L, double xi, double eta_s, double scale, int mode, double *spec,
                                 hipStream_t s) {
  const int n = M * (M / 2 + 1);
  hipLaunchKernelGGL(k_multiplier<double>, dim3((n + 255) / 256), dim3(256), 0, s, M, 2.0 * M_PI / L,
                     1.0 / (4.0 * xi * xi), 1.0 - eta_s, scale, mode, (double2 *)spec);
  return hipGetLastError();
}

hipError_t launch_multiplier_f32(int M, double L, double xi, double eta_s, double scale, int mode, float *spec,
                                 hipStream_t s) {
  const int n = M * (M / 2 + 1);
  hipLaunchKernelGGL(k_multiplier<float>, dim3((n + 255) / 256), dim3(256), 0, s, M, (float)(2.0 * M_PI / L),
                     (float)(1.0 / (4.0 * xi * xi)), (float)(1.0 - eta_s), (float)scale, mode, (float2 *)spec);
  return hipGetLastError();
}

}  // namespace fbim
