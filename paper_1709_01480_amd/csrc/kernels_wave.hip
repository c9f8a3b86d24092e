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
// the same over a compile-time bound PP >= P (registers, unrolled; entries past P
// are computed and must be discarded by the caller)
template <typename T, int PP>
__device__ __forceinline__ void gauss_row_pp(T x, T ag, T h, int half, const T *ck, T (&w)[PP]) {
  if constexpr (sizeof(T) == 8) {
    const T d0 = x + T(half) * h;
    const T e1 = dev_exp(T(2) * ag * d0 * h);
    T v = dev_exp(-ag * d0 * d0);
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      w[k] = v;
      v = v * e1 * ck[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      const T d = x + T(half - k) * h;
      w[k] = dev_exp(-ag * d * d);
    }
  }
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

// Spreading: one 256-thread work group per T x T grid tile, accumulated in LDS
// (no global atomics) over the tile's spreading list (the nodes whose stencil
// touches the tile, built once per configuration).  Per chunk of list entries
// each entry's P x- and P y-weights are computed once into LDS; then every
// (entry, stencil row) item loads its P x-weights into registers and adds its P
// values to one accumulator row with back-to-back LDS atomics (no wait between
// them: a load inside the column loop would wait for the atomics before it).
// Accumulator rows are padded by PP - 1 columns on each side, so a stencil that
// reaches past the tile needs no masks (those columns are discarded), and the
// row stride is odd so that the P rows of one item fall in distinct banks.
//
// Accumulation is in fixed point with a power-of-two scale S per tile, in
// 64-bit integer LDS atomics (the fast LDS atomic here: FP32 LDS atomic adds ran
// about 8x slower), so the sums, and the spread grid, do not depend on the order
// of the atomics.  S comes from a bound on every partial sum of the tile: per
// 8 x 8 block of the tile, cg times the sum of max(|mu_x|, |mu_y|) over the
// entries whose stencil meets the block (the weights are at most cg).
//   FP32: both components in one 64-bit word as two 32-bit signed halves, with
//     S B <= 2^30.  A half's sum stays within 31 bits, so the borrows of the low
//     half into the high half are undone exactly when the word is read back:
//     one atomic per grid point and entry, and a resolution of B / 2^30, below
//     the FP32 rounding of the terms.
//   FP64: one 64-bit word per component, S B <= 2^62.
// Terms are converted to integers by rounding (FP32) or by a floor computed in
// two 32-bit halves (FP64, within one unit of the scaled term).  A NaN or
// infinite density makes its tile's grid NaN, as floating-point sums would.
constexpr int kSpreadBlock = 8;  // side of the bound blocks
constexpr int kSpreadMaxBlocks = (kTmax + kSpreadBlock - 1) / kSpreadBlock;

// list entries per chunk (weights in LDS) and accumulator words per grid point;
// FP64 with the widest stencils takes smaller chunks to stay within 64 KB of LDS.
// FP32 takes 128: ~26 instead of ~35 KB per work group, six groups per CU instead
// of four, which hides more of each group's serial list gathers and barriers
// (58 vs 60 us at 640k nodes) at the cost of a second chunk in most 32 x 32 tiles.
template <typename T, int PP>
__host__ __device__ constexpr int spread_chunk() {
  return sizeof(T) == 4 ? 128 : (PP >= 15 ? 64 : 128);
}
template <typename T>
__host__ __device__ constexpr int spread_nacc() {
  return sizeof(T) == 4 ? 1 : 2;
}

// padded accumulator row stride for tile edge TT and stencil bound PP (odd)
__host__ __device__ inline int spread_stride(int TT, int PP) { return (TT + 2 * (PP - 1)) | 1; }
template <typename T, int PP>
inline size_t spread_lds_bytes() {
  return (size_t)spread_nacc<T>() * kTmax * spread_stride(kTmax, PP) * sizeof(unsigned long long) +
         2 * (size_t)spread_chunk<T, PP>() * PP * sizeof(T);
}

__device__ __forceinline__ unsigned long long fix64(double v) {  // floor-like integer of v, |v| < 2^62
  const double hf = floor(v * 0x1p-32);
  const double lf = fmin(fma(hf, -0x1p32, v), 4294967295.0);  // in [0, 2^32): rounding may reach 2^32
  return ((unsigned long long)(unsigned)(int)hf << 32) + (unsigned long long)(unsigned)lf;
}
__device__ __forceinline__ unsigned long long pack32(float x, float y) {  // (round(y) << 32) + round(x)
  const int tx = __float2int_rn(x), ty = __float2int_rn(y);
  return ((unsigned long long)((unsigned)ty + (unsigned)(tx >> 31)) << 32) | (unsigned)tx;
}

template <typename T, int PP>
__device__ __forceinline__ void spread_body(int M, int TT, int P, int nts, T h, T ag, T cg,
                                            const int *__restrict__ slist_start, const int *__restrict__ slist,
                                            const typename Vec2<T>::type *__restrict__ xt,
                                            const int2 *__restrict__ anchor,
                                            const typename Vec2<T>::type *__restrict__ mut, T *__restrict__ grid,
                                            int tile) {
  using V2 = typename Vec2<T>::type;
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int CH = spread_chunk<T, PP>(), NACC = spread_nacc<T>(), PADC = PP - 1;
  extern __shared__ unsigned long long spread_lds[];
  const int ST = spread_stride(TT, PP);
  unsigned long long *acc0 = spread_lds, *acc1 = spread_lds + (size_t)TT * ST;  // acc1: FP64 only
  T *wgx = reinterpret_cast<T *>(spread_lds + (size_t)NACC * TT * ST), *wgy = wgx + CH * PP;
  __shared__ T nmx[CH], nmy[CH], ck[kPmax];
  __shared__ int nbx[CH], nby[CH];
  __shared__ unsigned s_max, s_bad, s_blk[kSpreadMaxBlocks * kSpreadMaxBlocks];
  const int tid = threadIdx.x, lane = tid & 63;
  const int tyi = tile / nts, txi = tile % nts;
  const int gx0 = txi * TT, gy0 = tyi * TT;
  const int half = (P - 1) / 2;
  const int ls = slist_start[tile], n = slist_start[tile + 1] - ls;
  const int nbk = (TT + kSpreadBlock - 1) / kSpreadBlock;
  // list entry tid (most tiles have at most 256), gathered once before the LDS is
  // cleared and kept in registers for the two bound passes and the first chunk
  V2 fp, fmu;
  fp.x = fp.y = fmu.x = fmu.y = T(0);
  int2 fan = make_int2(0, 0);
  if (tid < n) {
    const int g = slist[ls + tid];
    fp = xt[g];
    fmu = mut[g];
    fan = anchor[g];
  }
  for (int i = tid; i < NACC * TT * ST; i += 256) spread_lds[i] = 0ull;
  if (tid < nbk * nbk) s_blk[tid] = 0u;
  if (tid == 0) s_max = s_bad = 0u;
  if (tid < P) ck[tid] = gauss_step<T>(ag, h, tid);
  __syncthreads();
  // bound of the partial sums: max |mu| of the tile, then per block the sum of
  // the quantised max(|mu_x|, |mu_y|) (rounded up) of the entries meeting it
  auto origin = [&](int a, int g0) {
    const int o = stencil_origin(a, half, g0, M);
    return o < TT ? o : o - M;
  };
  {
    float mloc = 0.f;
    bool bad = false;
    for (int e = tid; e < n; e += 256) {
      const V2 mu = e < 256 ? fmu : mut[slist[ls + e]];
      const T a = fmax(fabs(mu.x), fabs(mu.y));
      bad |= !isfinite(mu.x) || !isfinite(mu.y);
      mloc = fmaxf(mloc, (float)a);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mloc = fmaxf(mloc, __shfl_xor(mloc, o));
    const unsigned long long anybad = __ballot(bad);
    if (lane == 0) {
      atomicMax(&s_max, __float_as_uint(isfinite(mloc) ? mloc : 0.f));
      if (anybad) atomicOr(&s_bad, 1u);
    }
  }
  __syncthreads();
  const float mmax = __uint_as_float(s_max);
  const bool finite = s_bad == 0u;
  int E = 0;  // quantisation exponent of the block sums: n (mmax 2^E + 1) < 2^32
  if (mmax > 0.f) {
    int k;
    frexpf(mmax * (float)max(n, 1) * 1.0001f, &k);  // n mmax < 2^k
    E = 31 - k;
  }
  for (int e = tid; e < n; e += 256) {
    V2 mu = fmu;
    int2 an = fan;
    if (e >= 256) {
      const int g = slist[ls + e];
      mu = mut[g];
      an = anchor[g];
    }
    const int ox = origin(an.x, gx0), oy = origin(an.y, gy0);
    const int bx0 = max(ox, 0) / kSpreadBlock, bx1 = min(ox + P - 1, TT - 1) / kSpreadBlock;
    const int by0 = max(oy, 0) / kSpreadBlock, by1 = min(oy + P - 1, TT - 1) / kSpreadBlock;
    const float m = finite ? (float)fmax(fabs(mu.x), fabs(mu.y)) : 0.f;
    const unsigned qv = (unsigned)ceilf(ldexpf(m, E));
    for (int by = by0; by <= by1; ++by)
      for (int bx = bx0; bx <= bx1; ++bx) atomicAdd(&s_blk[by * nbk + bx], qv);
  }
  __syncthreads();
  T S = T(1);
  if (finite && mmax > 0.f) {
    unsigned bq = 0u;
    for (int b = 0; b < nbk * nbk; ++b) bq = max(bq, s_blk[b]);
    const double B = (double)cg * ldexp((double)bq, -E) * (1.0 + 0x1p-20);
    int k;
    frexp(B, &k);  // B < 2^k
    constexpr int kTop = F32 ? 30 : 62, kMaxE = F32 ? 126 : 1000;
    S = ldexp(T(1), max(min(kTop - k, kMaxE), -kMaxE));
  }
  static_assert(256 % CH == 0, "a chunk lies inside or past the first 256 entries");
  for (int c = 0; c < n; c += CH) {
    const int cnt = min(CH, n - c);
    // entry c + sl at slot sl: inside the first 256 entries the thread that holds it
    // stages it, past them thread sl gathers it
    const bool held = c < 256;
    const int sl = held ? tid - c : tid;
    if (sl >= 0 && sl < cnt) {
      V2 p = fp, mu = fmu;
      int2 an = fan;
      if (!held) {
        const int g = slist[ls + c + sl];
        p = xt[g];
        mu = mut[g];
        an = anchor[g];
      }
      nbx[sl] = origin(an.x, gx0) + PADC;
      nby[sl] = origin(an.y, gy0);
      nmx[sl] = mu.x * S;  // exact: S is a power of two
      nmy[sl] = mu.y * S;
      T wr[kPmax];
      gauss_row<T>(p.x, T(1), ag, h, half, P, ck, wr);
#pragma unroll
      for (int k = 0; k < PP; ++k) wgx[sl * PP + k] = k < P ? wr[k] : T(0);
      gauss_row<T>(p.y, cg, ag, h, half, P, ck, wr);
#pragma unroll
      for (int k = 0; k < PP; ++k) wgy[sl * PP + k] = k < P ? wr[k] : T(0);
    }
    __syncthreads();
    const float invP = 1.0f / (float)P;
    for (int it = tid; it < cnt * P; it += 256) {
      const int j = (int)(((float)it + 0.5f) * invP), q = it - j * P;  // it / P, exact for it < 2^20
      const int ry = nby[j] + q;
      if ((unsigned)ry >= (unsigned)TT) continue;
      T w[PP];
#pragma unroll
      for (int k = 0; k < PP; ++k) w[k] = wgx[j * PP + k];
      const T wy = wgy[j * PP + q];
      const T sx = wy * nmx[j], sy = wy * nmy[j];
      const int base = ry * ST + nbx[j];
#pragma unroll
      for (int k = 0; k < PP; ++k) {
        if constexpr (F32) {
          atomicAdd(acc0 + base + k, pack32(sx * w[k], sy * w[k]));
        } else {
          atomicAdd(acc0 + base + k, fix64(sx * w[k]));
          atomicAdd(acc1 + base + k, fix64(sy * w[k]));
        }
      }
    }
    __syncthreads();
  }
  const T inv = finite ? T(1) / S : T(NAN);  // exact power of two
  for (int i = tid; i < TT * TT; i += 256) {
    const int ry = i / TT, rx = i - ry * TT;
    const size_t gidx = (size_t)(gy0 + ry) * M + gx0 + rx;
    const int a = ry * ST + rx + PADC;
    if constexpr (F32) {
      const unsigned long long v = acc0[a];
      const int lo = (int)(unsigned)v;
      const int hi = (int)((v - (unsigned long long)(long long)lo) >> 32);
      grid[gidx] = (T)lo * inv;
      grid[(size_t)M * M + gidx] = (T)hi * inv;
    } else {
      grid[gidx] = (T)(long long)acc0[a] * inv;
      grid[(size_t)M * M + gidx] = (T)(long long)acc1[a] * inv;
    }
  }
}

// Interpolation: one work group per grid tile, the tile's window of grid points
// (both components interleaved) in LDS, one thread per node of the tile.  The
// stencil bound PP (odd, >= P) is a template parameter, so the P x P loop is
// unrolled with one 64-bit (FP32) or 128-bit (FP64) LDS read per point; for P < PP
// the extra weights are zero and the window's extra columns and rows hold zeros.
template <typename T, int PP>
__device__ __forceinline__ void interp_body(int M, int TT, int P, int nts, T h, T ag, T scale,
                                            const int *__restrict__ tile_start,
                                            const typename Vec2<T>::type *__restrict__ xt,
                                            const int2 *__restrict__ anchor, const int *__restrict__ tperm,
                                            const T *__restrict__ grid, double *__restrict__ out, int tile) {
  using V2 = typename Vec2<T>::type;
  constexpr int W = kTmax + PP - 1;
  __shared__ V2 win[W * W];
  __shared__ T ck[PP];
  const int tid = threadIdx.x;
  const int tyi = tile / nts, txi = tile % nts;
  const int gx0 = txi * TT, gy0 = tyi * TT;
  const int half = (P - 1) / 2;
  const int w = TT + P - 1, wa = TT + PP - 1;  // window edge, and as allocated for PP
  for (int i = tid; i < wa * wa; i += 256) {
    const int ry = i / wa, rx = i - ry * wa;
    V2 g;
    g.x = g.y = T(0);
    if (ry < w && rx < w) {
      const size_t gidx = (size_t)wrapi(gy0 - half + ry, M) * M + wrapi(gx0 - half + rx, M);
      g.x = grid[gidx];
      g.y = grid[(size_t)M * M + gidx];
    }
    win[i] = g;
  }
  if (tid < PP) ck[tid] = tid < P ? gauss_step<T>(ag, h, tid) : T(0);
  __syncthreads();
  const int a = tile_start[tile], b = tile_start[tile + 1];
  for (int k = a + tid; k < b; k += 256) {
    const auto p = xt[k];
    const int2 an = anchor[k];
    const int bx = wrapi(an.x - half - (gx0 - half), M);  // window column of the first stencil point
    const int by = wrapi(an.y - half - (gy0 - half), M);
    // weights of the stencil's columns and rows (offsets p + (half - k) h from the
    // nearest grid point) by the product recurrence; zero past P
    T wx[PP], wyr[PP];
    gauss_row_pp<T, PP>(p.x, ag, h, half, ck, wx);
    gauss_row_pp<T, PP>(p.y, ag, h, half, ck, wyr);
#pragma unroll
    for (int q = 0; q < PP; ++q)
      if (q >= P) wx[q] = wyr[q] = T(0);
    T sx = 0, sy = 0;
    const V2 *r = win + by * wa + bx;
#pragma unroll
    for (int qr = 0; qr < PP; ++qr) {
      T rx0 = 0, rx1 = 0;
#pragma unroll
      for (int pc = 0; pc < PP; ++pc) {
        const V2 g = r[qr * wa + pc];
        rx0 += wx[pc] * g.x;
        rx1 += wx[pc] * g.y;
      }
      sx += wyr[qr] * rx0;
      sy += wyr[qr] * rx1;
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

template <typename T, int PP>
__global__ __launch_bounds__(256) void k_spread(int M, int TT, int P, int nts, T h, T ag, T cg,
                                                const int *__restrict__ slist_start, const int *__restrict__ slist,
                                                const typename Vec2<T>::type *__restrict__ xt,
                                                const int2 *__restrict__ anchor,
                                                const typename Vec2<T>::type *__restrict__ mut,
                                                T *__restrict__ grid) {
  spread_body<T, PP>(M, TT, P, nts, h, ag, cg, slist_start, slist, xt, anchor, mut, grid,
                     xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int PP>
__global__ __launch_bounds__(256) void k_interp(int M, int TT, int P, int nts, T h, T ag, T scale,
                                                const int *__restrict__ tile_start,
                                                const typename Vec2<T>::type *__restrict__ xt,
                                                const int2 *__restrict__ anchor,
                                                const int *__restrict__ tperm, const T *__restrict__ grid,
                                                double *__restrict__ out) {
  interp_body<T, PP>(M, TT, P, nts, h, ag, scale, tile_start, xt, anchor, tperm, grid, out,
                 xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T>
__global__ void k_multiplier(int M, T twopi_L, T inv4xi2, T one_m_eta, T scale, int mode,
                             typename Vec2<T>::type *__restrict__ spec) {
  multiplier_body<T>(M, twopi_L, inv4xi2, one_m_eta, scale, mode, spec, blockIdx.x * blockDim.x + threadIdx.x);
}

// batched forms: the XCD-aware order is taken over the whole grid, then the
// block's system and its tile within that system are found
template <typename T, int PP>
__global__ __launch_bounds__(256) void k_spread_batch(const SpreadJob *__restrict__ jobs, BatchGrid bg) {
  using V2 = typename Vec2<T>::type;
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = batch_system(bg.begin, bg.S, gb);
  const SpreadJob &j = jobs[s];
  spread_body<T, PP>(j.w.M, j.w.T, j.w.P, j.w.nts, (T)j.w.h, (T)j.w.ag, (T)j.w.cg, j.w.slist_start, j.w.slist,
                     reinterpret_cast<const V2 *>(j.xt), reinterpret_cast<const int2 *>(j.w.anchor),
                     reinterpret_cast<const V2 *>(j.mut), reinterpret_cast<T *>(j.grid), gb - bg.begin[s]);
}

template <typename T, int PP>
__global__ __launch_bounds__(256) void k_interp_batch(const InterpJob *__restrict__ jobs, BatchGrid bg) {
  using V2 = typename Vec2<T>::type;
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = batch_system(bg.begin, bg.S, gb);
  const InterpJob &j = jobs[s];
  interp_body<T, PP>(j.w.M, j.w.T, j.w.P, j.w.nts, (T)j.w.h, (T)j.w.ag, (T)(j.w.h * j.w.h * j.w.cg), j.w.tile_start,
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

// the stencil bound PP (odd, >= P) of a launch selects the kernel instance
template <typename T, typename F>
static hipError_t spread_dispatch(int pp, F &&launch) {
  switch (pp) {
    case 1: case 3: return launch(std::integral_constant<int, 3>{});
    case 5: return launch(std::integral_constant<int, 5>{});
    case 7: return launch(std::integral_constant<int, 7>{});
    case 9: return launch(std::integral_constant<int, 9>{});
    case 11: return launch(std::integral_constant<int, 11>{});
    case 13: return launch(std::integral_constant<int, 13>{});
    case 15: return launch(std::integral_constant<int, 15>{});
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t spread_batch_t(const SpreadJob *jobs, BatchGrid bg, int pmax, hipStream_t s) {
  return spread_dispatch<T>(pmax, [&](auto pp) {
    constexpr int PP = decltype(pp)::value;
    const size_t lds = spread_lds_bytes<T, PP>();
    hipLaunchKernelGGL((k_spread_batch<T, PP>), dim3(bg.nblocks), dim3(256), lds, s, jobs, bg);
    return hipGetLastError();
  });
}

hipError_t launch_spread_batch(const SpreadJob *jobs, BatchGrid bg, int f32, int pmax, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (pmax < 1 || pmax > kPmax) return hipErrorInvalidValue;
  return f32 ? spread_batch_t<float>(jobs, bg, pmax, s) : spread_batch_t<double>(jobs, bg, pmax, s);
}

hipError_t launch_interp_batch(const InterpJob *jobs, BatchGrid bg, int f32, int pmax, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (pmax < 1 || pmax > kPmax) return hipErrorInvalidValue;
  return spread_dispatch<float>(pmax, [&](auto pp) {
    constexpr int PP = decltype(pp)::value;
    if (f32)
      hipLaunchKernelGGL((k_interp_batch<float, PP>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg);
    else
      hipLaunchKernelGGL((k_interp_batch<double, PP>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg);
    return hipGetLastError();
  });
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

template <typename T>
static hipError_t spread_one(const WaveArgs &w, const T *xt, const T *mut, T *grid, hipStream_t s) {
  using V2 = typename Vec2<T>::type;
  const int nt = w.nts * w.nts;
  if (w.P < 1 || w.P > kPmax || w.T > kTmax) return hipErrorInvalidValue;
  return spread_dispatch<T>(w.P, [&](auto pp) {
    constexpr int PP = decltype(pp)::value;
    const size_t lds = spread_lds_bytes<T, PP>();
    hipLaunchKernelGGL((k_spread<T, PP>), dim3(nt), dim3(256), lds, s, w.M, w.T, w.P, w.nts,
                       (T)w.h, (T)w.ag, (T)w.cg, w.slist_start, w.slist, (const V2 *)xt, (const int2 *)w.anchor,
                       (const V2 *)mut, grid);
    return hipGetLastError();
  });
}

hipError_t launch_spread_f64(const WaveArgs &w, const double *xt, const double *mut, double *grid, hipStream_t s) {
  return spread_one<double>(w, xt, mut, grid, s);
}

hipError_t launch_spread_f32(const WaveArgs &w, const float *xt, const float *mut, float *grid, hipStream_t s) {
  return spread_one<float>(w, xt, mut, grid, s);
}

hipError_t launch_interp_f64(const WaveArgs &w, const double *xt, const int *tperm, const double *grid,
                             double *out, hipStream_t s) {
  const int nt = w.nts * w.nts;
  if (w.P < 1 || w.P > kPmax || w.T > kTmax) return hipErrorInvalidValue;
  return spread_dispatch<double>(w.P, [&](auto pp) {
    constexpr int PP = decltype(pp)::value;
    hipLaunchKernelGGL((k_interp<double, PP>), dim3(nt), dim3(256), 0, s, w.M, w.T, w.P, w.nts, w.h, w.ag,
                       w.h * w.h * w.cg, w.tile_start, (const double2 *)xt, (const int2 *)w.anchor, tperm, grid,
                       out);
    return hipGetLastError();
  });
}

hipError_t launch_interp_f32(const WaveArgs &w, const float *xt, const int *tperm, const float *grid, double *out,
                             hipStream_t s) {
  const int nt = w.nts * w.nts;
  if (w.P < 1 || w.P > kPmax || w.T > kTmax) return hipErrorInvalidValue;
  return spread_dispatch<float>(w.P, [&](auto pp) {
    constexpr int PP = decltype(pp)::value;
    hipLaunchKernelGGL((k_interp<float, PP>), dim3(nt), dim3(256), 0, s, w.M, w.T, w.P, w.nts, (float)w.h,
                       (float)w.ag, (float)(w.h * w.h * w.cg), w.tile_start, (const float2 *)xt,
                       (const int2 *)w.anchor, tperm, grid, out);
    return hipGetLastError();
  });
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
