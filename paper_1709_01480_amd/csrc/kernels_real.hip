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

constexpr int kE1Int = 11;        // intervals of the E1 table

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
// arguments here are normal numbers, so the hardware log2 needs no rescaling
__device__ inline float dev_log(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }

// E1(z) from the piecewise polynomial table: interval 0 holds E1 + ln z on [0, 2],
// interval k >= 1 holds e^z E1(z) on [b_(k-1), b_k] with ends b = 2, 3, 4, 6, 8,
// 12, ..., 48, 64 (each binade of z split at 1.5 times its start); a row is
// {1 / half-width, -centre / half-width, a_0 .. a_DEG} of the power series in
// x = (z - centre) / half-width, evaluated by Horner's rule.
template <typename T, int DEG>
__device__ inline T poly(const T *row, T z) {
  const T x = fma(z, row[0], row[1]);
  T f = row[2 + DEG];
#pragma unroll
  for (int m = DEG - 1; m >= 0; --m) f = fma(f, x, row[2 + m]);
  return f;
}

// ---------------------------------------------------------------- neighbour lists
// Per configuration the in-range (target, source) pairs are stored in an ELL
// layout grouped by 64 consecutive cell-sorted targets (one wavefront): group g
// owns slots [goff[g], goff[g] + 64 (nn_g + nf_g)); slot i of target lane l is
// goff[g] + 64 i + l.  The first nn_g rows hold near pairs (xi^2 r^2 <= 2), the
// next nf_g rows far pairs.  A 16-bit entry holds the source's neighbour cell k
// (bits 12-15; k = 9 an empty slot) and its index within that cell (bits 0-11).
constexpr int kEllK = 10;  // neighbour cells 0..8 and the empty slot
constexpr int kOffMask = kEllMaxCell - 1;

// One thread per cell-sorted target: it scans the nodes of the 3 x 3 neighbouring
// cells (cell by cell, node order -- the order of its list rows), counts its near
// and far pairs (mode 0) or writes them into its ELL slots (mode 1).  With `flag`
// (mode 0) it also flags nodes of distinct bodies closer than sqrt(thresh2).
// Mode 1 with maxrows > 0 stages each group's rows in LDS (a lane writes only its
// own column, empty slots N) and stores them as whole contiguous rows; with
// maxrows = 0 it writes the slots directly (ell pre-set to N).
constexpr int kListBlock = 128;  // two groups of 64 targets

__global__ __launch_bounds__(kListBlock) void k_pair_lists(int N, int ngroups, const int *__restrict__ cell_start,
                                                           const int *__restrict__ ckey,
                                                           const int *__restrict__ perm, int nb, double cell,
                                                           double rc2, double r2near, const double2 *__restrict__ xs,
                                                           int *__restrict__ cnt_near, int *__restrict__ cnt_far,
                                                           const int *__restrict__ goff, const int *__restrict__ gnn,
                                                           const int *__restrict__ gnf, uint16_t *__restrict__ ell,
                                                           int mode, int maxrows, const int *__restrict__ body,
                                                           double thresh2, int *__restrict__ flag) {
  extern __shared__ uint16_t stile[];  // mode 1 staged: [kListBlock / 64][maxrows][64]
  const int gt = xcd_remap(blockIdx.x, gridDim.x) * kListBlock + threadIdx.x;
  const int grp = gt >> 6, gl = gt & 63;
  const bool staged = mode && maxrows > 0;
  int nn = 0, rows = 0;
  if (mode && grp < ngroups) {
    nn = gnn[grp];
    rows = nn + gnf[grp];
  }
  uint16_t *col = stile + (threadIdx.x >> 6) * maxrows * 64 + gl;
  if (staged)
    for (int r = 0; r < rows; ++r) col[r * 64] = kEllEmpty;
  if (gt < N) {
    const int c = ckey[perm[gt]];
    const int ccx = c % nb, ccy = c / nb;
    const double2 p = xs[gt];
    const int base = (mode && !staged) ? goff[grp] : 0;
    int cn = 0, cf = 0;
    for (int k = 0; k < 9; ++k) {
      const int dx = k % 3 - 1, dy = k / 3 - 1;
      const int cc = ((ccy + dy + nb) % nb) * nb + (ccx + dx + nb) % nb;
      const double ox = p.x - dx * cell, oy = p.y - dy * cell;  // target relative to cell cc's corner frame
      const int g0 = cell_start[cc], g1 = cell_start[cc + 1];
#pragma unroll 4
      for (int g = g0; g < g1; ++g) {
        const double2 q = xs[g];
        const double ex = ox - q.x, ey = oy - q.y;
        const double r2 = ex * ex + ey * ey;
        if (r2 > rc2 || g == gt) continue;
        if (flag && r2 < thresh2 && body[perm[gt]] != body[perm[g]]) atomicOr(flag, 1);
        const bool near = r2 <= r2near;
        const int row = near ? cn : nn + cf;
        const uint16_t e = (uint16_t)((k << 12) | (g - g0));
        if (staged)
          col[row * 64] = e;
        else if (mode)
          ell[base + (size_t)row * 64 + gl] = e;
        cn += near;
        cf += !near;
      }
    }
    if (mode == 0) {
      cnt_near[gt] = cn;
      cnt_far[gt] = cf;
    }
  }
  if (staged) {
    __syncthreads();
    if (grp < ngroups) {  // the group's rows, contiguous
      const uint16_t *tile = stile + (threadIdx.x >> 6) * maxrows * 64;
      uint16_t *dst = ell + goff[grp];
      for (int i = gl; i < rows * 64; i += 64) dst[i] = tile[i];
    }
  }
}

// per group of 64 targets: row counts (max over lanes) and the slot total
__global__ void k_group_rows(int N, int ngroups, const int *__restrict__ cnt_near, const int *__restrict__ cnt_far,
                             int *__restrict__ gnn, int *__restrict__ gnf, int *__restrict__ gsize) {
  const int g = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= ngroups) return;
  const int t = g * 64 + lane;
  int a = t < N ? cnt_near[t] : 0, b = t < N ? cnt_far[t] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a = max(a, __shfl_down(a, o));
    b = max(b, __shfl_down(b, o));
  }
  if (lane == 0) {
    gnn[g] = a;
    gnf[g] = b;
    gsize[g] = 64 * (a + b);
  }
}

// real-space pair sum over the neighbour lists: one thread per cell-sorted
// target; `blk` is the block's index within its system (256 threads = 4 groups)
// Packed source records: (x, y, mu_x, mu_y) in one 16-byte (FP32) or 32-byte
// (FP64) record per cell-sorted node, so a pair gathers one record.
template <typename T> struct Rec;
// Record indices are below 2^26 (at most kMaxNodes + 1 records), so a record's
// byte offset fits 32 bits: one unsigned (base + index) << shift, no 64-bit
// address math.
template <> struct Rec<float> {
  __device__ static inline float4 load(const void *p, unsigned i) {
    __builtin_assume(i < (1u << 26));
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(p) + (i << 4));
  }
};
template <> struct Rec<double> {
  __device__ static inline double4 load(const void *p, unsigned i) {
    __builtin_assume(i < (1u << 26));
    const double2 *q = reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(p) + (i << 5));
    const double2 a = q[0], b = q[1];
    return make_double4(a.x, a.y, b.x, b.y);
  }
};

__device__ inline float dev_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double dev_rcp(double x) {
  // hardware reciprocal estimate refined by two Newton steps to FP64 accuracy
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  return fma(fma(-x, y, 1.0), y, y);
}

// row of a far argument z > 2 of the E1 table, read off the FP32 bits of z: bits
// 22-30 are twice the biased exponent plus the leading mantissa bit, 256 on
// [2, 3), 257 on [3, 4), 258 on [4, 6), ...; less 255 and clamped to
// [1, kE1Int - 1].  Taken in FP32 for either precision (an argument within
// rounding of an interval end may take the neighbouring interval, whose series is
// accurate there too).
template <typename T>
__device__ inline int far_interval(T z) {
  const int key = ((int)__float_as_uint((float)z) - (255 << 22)) >> 22;
  return min(max(key, 1), kE1Int - 1);
}

// One 256-thread work group per group of 64 targets: wave w takes rows w, w + 4,
// w + 8, ... of the group's ELL block (near rows come first, so every wave gets a
// share of both kinds) and the four partial sums meet in LDS.  Four short waves
// per group instead of one long one: at 640k nodes the 10^4 groups fill the
// chip's wave slots about five times over instead of 1.2 times (a second round
// of 0.2 of the machine).
// An entry is resolved through the group's neighbour-cell table in LDS: row k of
// lane l holds the first source of target l's neighbour cell k and the cell's
// offsets (row 9: the zero record, offsets 0).
// Row indices are wave-uniform (scalar loop control and near / far branch).  The
// FP32 loop takes two rows per trip (rows i and i + 4 of the wave) with the next
// trip's list entries and the second row's source record in flight while the
// first row is evaluated; a trip's two terms are added in FP32 and the ~8 trip
// sums of a lane per wave in FP64, so the sum rounds about once per term (as a
// compensated FP32 sum would) without the compensation's instructions.
constexpr int kPairWaves = 4;

template <typename T, int DEG>
__device__ __forceinline__ void pair_ell_body(const PairJob &j, const T *__restrict__ tab, int g) {
  __shared__ double part[kPairWaves - 1][64][2];
  __shared__ int4 nbr[kEllK][64];  // (first source, dcx, dcy as float bits, 0)
  const T cell = (T)j.cell, xi2 = (T)j.xi2;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int t = g * 64 + lane;
  {
    const int tc = t < j.N ? j.tcell[t] : 0, nb = j.nb;
    const int cx = tc % nb, cy = tc / nb;
    for (int k = wv; k < kEllK; k += kPairWaves) {
      int4 e = make_int4(j.N, 0, 0, 0);
      if (k < 9) {
        const int dx = k % 3 - 1, dy = k / 3 - 1;
        int ux = cx + dx, uy = cy + dy;  // periodic wrap of a neighbour one cell away
        ux += ux < 0 ? nb : (ux >= nb ? -nb : 0);
        uy += uy < 0 ? nb : (uy >= nb ? -nb : 0);
        e = make_int4(j.cell_start[uy * nb + ux], __float_as_int((float)dx), __float_as_int((float)dy), 0);
      }
      nbr[k][lane] = e;
    }
  }
  // positions are relative to their cell's corner: a source in neighbour cell
  // (dcx, dcy) sits at r + (dcx, dcy) cell, so d = (tx - r.x) - dcx cell (exact
  // difference of nearby coordinates, then one rounding)
  T tx = 0, ty = 0;
  if (t < j.N) {
    const auto p = Rec<T>::load(j.src, t);
    tx = p.x;
    ty = p.y;
  }
  const int base = j.goff[g], nn = j.gnn[g], rows = nn + j.gnf[g];
  const uint16_t *__restrict__ col = j.ell + base + lane;
  double vx = 0, vy = 0;
  __syncthreads();
  // rows past the group's last are read without a test (the next group's entries,
  // or the kEllSlack slots after the last group) and never resolved
  auto entry = [&](int i) { return (unsigned)col[(size_t)i * 64]; };
  // source record and cell offsets of entry e
  auto resolve = [&](unsigned e, float &ox, float &oy) {
    const int4 c = nbr[e >> 12][lane];
    ox = __int_as_float(c.y);
    oy = __int_as_float(c.z);
    return Rec<T>::load(j.src, (unsigned)c.x + (e & kOffMask));
  };
  // one slot's term (cx, cy); an empty slot reads the zero record: a source at
  // 1.5 to 2.5 cells (finite z, every series finite) with density 0, term 0
  auto eval = [&](const auto &r, float ox, float oy, bool near, T &cx, T &cy) {
    const T dx = fma(-(T)ox, cell, tx - r.x), dy = fma(-(T)oy, cell, ty - r.y);
    const T r2 = fma(dx, dx, dy * dy);
    const T z = xi2 * r2;
    const T ez = dev_exp(-z);
    // near rows: E1 + ln z on [0, 2]; far rows: e^z E1 on the table interval of z
    // (FP64: one series evaluation on the selected row, fewer registers for the
    // degree-16 coefficients) or a rational form (FP32).
    T e1, ir2;  // E1(z) and 1 / r^2
    if constexpr (sizeof(T) == 8) {
      const T p = poly<T, DEG>(tab + (near ? 0 : far_interval(z) * (DEG + 3)), z);
      e1 = near ? p - dev_log(z) : ez * p;
      ir2 = dev_rcp(r2);
    } else if (near) {
      e1 = poly<T, DEG>(tab, z) - dev_log(z);
      ir2 = dev_rcp(r2);
    } else {
      // FP32 far rows: z e^z E1(z) = P(z) / Q(z) with the quartics of Abramowitz
      // and Stegun 5.1.56 (absolute error below 2e-8 for z >= 1), no table reads;
      // one reciprocal of r^2 z Q gives both 1 / (z Q) and 1 / r^2
      const T P = fma(fma(fma(z + T(8.5733287401), z, T(18.0590169730)), z, T(8.6347608925)), z,
                      T(0.2677737343));
      const T Q = fma(fma(fma(z + T(9.5733223454), z, T(25.6329561486)), z, T(21.0996530827)), z,
                      T(3.9584969228));
      const T zq = z * Q;
      const T inv = dev_rcp(r2 * zq);
      ir2 = zq * inv;
      e1 = ez * (P * (r2 * inv));
    }
    const T a = fma(T(0.5), e1, -ez);
    const T sdot = ez * fma(dx, r.z, dy * r.w) * ir2;
    cx = fma(a, r.z, sdot * dx);
    cy = fma(a, r.w, sdot * dy);
  };
  int i = wv;
  unsigned eb = entry(wv + kPairWaves);
  float oxa = 0, oya = 0;
  decltype(Rec<T>::load(nullptr, 0)) ra{};
  if (i < rows) ra = resolve(entry(wv), oxa, oya);
  // FP32: two trips per loop turn, so that the loads in flight alternate between
  // two register sets instead of being copied at the back edge (FP64 keeps one:
  // its records are twice as wide)
  constexpr int kTrips = sizeof(T) == 4 ? 2 : 1;
#pragma unroll kTrips
  for (; i + kPairWaves < rows; i += 2 * kPairWaves) {
    float oxb, oyb;
    const auto rb = resolve(eb, oxb, oyb);
    const unsigned na = entry(i + 2 * kPairWaves);
    eb = entry(i + 3 * kPairWaves);
    T ax, ay, bx, by;
    eval(ra, oxa, oya, i < nn, ax, ay);
    if constexpr (sizeof(T) == 8) {
      vx += ax;
      vy += ay;
    }
    if (i + 2 * kPairWaves < rows) ra = resolve(na, oxa, oya);
    eval(rb, oxb, oyb, i + kPairWaves < nn, bx, by);
    if constexpr (sizeof(T) == 8) {
      vx += bx;
      vy += by;
    } else {  // the trip's two terms meet in FP32 (one rounding), then the FP64 sums
      vx += (double)(ax + bx);
      vy += (double)(ay + by);
    }
  }
  if (i < rows) {  // the wave's last row when its count is odd
    T ax, ay;
    eval(ra, oxa, oya, i < nn, ax, ay);
    vx += (double)ax;
    vy += (double)ay;
  }
  if (wv > 0) {
    part[wv - 1][lane][0] = vx;
    part[wv - 1][lane][1] = vy;
  }
  __syncthreads();
  if (wv == 0 && t < j.N) {
    double sx = vx, sy = vy;
#pragma unroll
    for (int w = 0; w < kPairWaves - 1; ++w) {
      sx += part[w][lane][0];
      sy += part[w][lane][1];
    }
    const int node = j.perm[t];
    j.out[2 * node] = j.cG * sx;
    j.out[2 * node + 1] = j.cG * sy;
  }
}

template <typename T, int DEG>
__device__ inline void load_table(T *tab, const T *__restrict__ e1tab) {
  for (int i = threadIdx.x; i < kE1Int * (DEG + 3); i += 256) tab[i] = e1tab[i];
  __syncthreads();
}

template <typename T, int DEG>
__global__ __launch_bounds__(256) void k_pair_ell(PairJob j, const T *__restrict__ e1tab) {
  __shared__ T tab[kE1Int * (DEG + 3)];
  load_table<T, DEG>(tab, e1tab);
  pair_ell_body<T, DEG>(j, tab, blockIdx.x);
}

template <typename T, int DEG>
__global__ __launch_bounds__(256) void k_pair_ell_batch(const PairJob *__restrict__ jobs, BatchGrid bg,
                                                        const T *__restrict__ e1tab) {
  __shared__ T tab[kE1Int * (DEG + 3)];
  load_table<T, DEG>(tab, e1tab);
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  pair_ell_body<T, DEG>(jobs[s], tab, blockIdx.x - bg.begin[s]);
}

template <typename T, int DEG>
hipError_t pair_ell_launch(const PairLists &pl, const PairArgs &a, const T *src, const T *tab, double *out,
                           hipStream_t s) {
  if (pl.N == 0) return hipSuccess;
  PairJob j;
  j.N = pl.N;
  j.ngroups = pl.ngroups;
  j.perm = a.perm;
  j.goff = pl.goff;
  j.gnn = pl.gnn;
  j.gnf = pl.gnf;
  j.ell = pl.ell;
  j.tcell = a.tcell;
  j.cell_start = a.cell_start;
  j.nb = a.nb;
  j.cell = a.cell;
  j.xi2 = a.xi2;
  j.cG = a.cG;
  j.src = src;
  j.out = out;
  hipLaunchKernelGGL((k_pair_ell<T, DEG>), dim3(pl.ngroups), dim3(256), 0, s, j, tab);  // one group each
  return hipGetLastError();
}

}  // namespace

int pair_lists_stage_rows(int maxrows) {
  return (size_t)(kListBlock / 64) * maxrows * 64 * sizeof(uint16_t) <= kListStageBytes ? maxrows : 0;
}

hipError_t launch_pair_lists(const PairArgs &a, PairLists &pl, const double *xs, int mode, hipStream_t s,
                             const int *body, double thresh2, int *flag, int maxrows) {
  if (pl.N == 0) return hipSuccess;
  const size_t lds = (mode && maxrows > 0) ? (size_t)(kListBlock / 64) * maxrows * 64 * sizeof(uint16_t) : 0;
  hipLaunchKernelGGL(k_pair_lists, dim3((pl.N + kListBlock - 1) / kListBlock), dim3(kListBlock), lds, s, pl.N,
                     pl.ngroups, a.cell_start, a.ckey, a.perm, a.nb, a.cell, a.rc2, 2.0 / a.xi2, (const double2 *)xs,
                     pl.cnt_near, pl.cnt_far, pl.goff, pl.gnn, pl.gnf, pl.ell, mode, mode ? maxrows : 0, body,
                     thresh2, mode == 0 ? flag : nullptr);
  return hipGetLastError();
}

hipError_t launch_group_rows(PairLists &pl, int *gsize, hipStream_t s) {
  if (pl.ngroups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_rows, dim3((pl.ngroups + 3) / 4), dim3(256), 0, s, pl.N, pl.ngroups, pl.cnt_near,
                     pl.cnt_far, pl.gnn, pl.gnf, gsize);
  return hipGetLastError();
}

hipError_t launch_pair_f64(const PairLists &pl, const PairArgs &a, const double *src, double *out, hipStream_t s) {
  return pair_ell_launch<double, 16>(pl, a, src, a.e1tab, out, s);
}

hipError_t launch_pair_f32(const PairLists &pl, const PairArgs &a, const float *src, double *out, hipStream_t s) {
  return pair_ell_launch<float, 9>(pl, a, src, a.e1tab32, out, s);
}

// ------------------------------------------------------------------ Alpert band
__device__ __forceinline__ void alpert_body(const GeomDev &g, const double *const *band_tab, const int *__restrict__ band,
                            const double2 *__restrict__ mu, double2 *__restrict__ out, int accumulate, int i) {
  if (i >= g.N) return;
  const int b = g.body[i];
  const int base = g.off[b];
  const int t = i - base;
  const int sh = g.shape[b];
  const int B = band[sh], n_p = g.np[sh];
  const double *A = band_tab[sh] + (size_t)t * 4;  // o-major: block (o, t) at ((o + B) n_p + t) 4
  double sn, cs;
  sincos(g.theta[b], &sn, &cs);
  double ax = 0.0, ay = 0.0;
  for (int o = -B; o <= B; ++o) {
    int l = t + o;
    l += (l < 0) ? n_p : 0;
    l -= (l >= n_p) ? n_p : 0;
    const double2 m = mu[base + l];
    const double rx = cs * m.x + sn * m.y, ry = -sn * m.x + cs * m.y;  // R^T mu
    const double *blk = A + (size_t)(o + B) * n_p * 4;
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

__global__ __launch_bounds__(256) void k_alpert(GeomDev g, const double *const *band_tab, const int *__restrict__ band,
                                                const double2 *__restrict__ mu, double2 *__restrict__ out,
                                                int accumulate) {
  alpert_body(g, band_tab, band, mu, out, accumulate, blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_alpert_batch(const AlpertJob *__restrict__ jobs, BatchGrid bg) {
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  const AlpertJob &j = jobs[s];
  alpert_body(j.g, j.band_tab, j.band, reinterpret_cast<const double2 *>(j.mu), reinterpret_cast<double2 *>(j.out),
              1, (blockIdx.x - bg.begin[s]) * 256 + threadIdx.x);
}

hipError_t launch_alpert(const GeomDev &g, const double *const *band_tab, const int *band, const double *mu,
                         double *out, int accumulate, hipStream_t s) {
  if (g.N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpert, dim3((g.N + 255) / 256), dim3(256), 0, s, g, band_tab, band, (const double2 *)mu,
                     (double2 *)out, accumulate);
  return hipGetLastError();
}

hipError_t launch_alpert_batch(const AlpertJob *jobs, BatchGrid bg, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpert_batch, dim3(bg.nblocks), dim3(256), 0, s, jobs, bg);
  return hipGetLastError();
}

hipError_t launch_pair_batch(const PairJob *jobs, BatchGrid bg, int f32, const double *tab64, const float *tab32,
                             hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL((k_pair_ell_batch<float, 9>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg, tab32);
  else
    hipLaunchKernelGGL((k_pair_ell_batch<double, 16>), dim3(bg.nblocks), dim3(256), 0, s, jobs, bg, tab64);
  return hipGetLastError();
}

// ------------------------------------------------------------------ second kind (Appendix B)
namespace {

// Real-space periodic stresslet over the neighbour lists: for each cell-sorted
// target, sum over its in-range sources of T^(r)_jlm(d) phi_l w_m with
// d = x_t - x_s, w = n ds (outward normal times arc weight):
//   T^(r)_jlm phi_l w_m = e [-4 (1 + z) / r^4 (d.phi)(d.w) d_j + 2 xi^2 ((phi.w) d_j + (d.phi) w_j)],
// z = xi^2 r^2, e = exp(-z).  One thread per target; output (times cG) in node order.
__global__ __launch_bounds__(256) void k_dl_ell(PairJob j, const double2 *__restrict__ wc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= j.N) return;
  const int g = t >> 6, lane = t & 63;
  const double4 me = Rec<double>::load(j.src, t);
  const double cell = j.cell, xi2 = j.xi2;
  const int base = j.goff[g], rows = j.gnn[g] + j.gnf[g];
  const int nb = j.nb, cx = j.tcell[t] % nb, cy = j.tcell[t] / nb;
  double vx = 0, vy = 0;
  for (int i = 0; i < rows; ++i) {
    const unsigned ent = j.ell[base + (size_t)i * 64 + lane];
    const int k = (int)(ent >> 12);
    if (k >= 9) continue;  // empty slot
    const int dcx = k % 3 - 1, dcy = k / 3 - 1;
    const int cc = ((cy + dcy + nb) % nb) * nb + (cx + dcx + nb) % nb;
    const int sidx = j.cell_start[cc] + (int)(ent & kOffMask);
    const double4 r = Rec<double>::load(j.src, sidx);
    const double2 w = wc[sidx];
    const double ox = (double)dcx, oy = (double)dcy;
    const double dx = me.x - (r.x + ox * cell), dy = me.y - (r.y + oy * cell);
    const double r2 = dx * dx + dy * dy;
    const double z = xi2 * r2;
    const double e = exp(-z);
    const double dp = dx * r.z + dy * r.w, dw = dx * w.x + dy * w.y, pw = r.z * w.x + r.w * w.y;
    const double a = -4.0 * (1.0 + z) / (r2 * r2) * dp * dw + 2.0 * xi2 * pw;
    const double b = 2.0 * xi2 * dp;
    vx += e * (a * dx + b * w.x);
    vy += e * (a * dy + b * w.y);
  }
  const int node = j.perm[t];
  j.out[2 * node] = j.cG * vx;
  j.out[2 * node + 1] = j.cG * vy;
}

// Real-space part of the completion flow: at every node, the Hasimoto-split
// Stokeslet G^(r) (eq. 3.15) and rotlet R^(r) = r^perp / r^2 (1 - z) e^-z of every
// body's tracking point within r_c (minimum image), with force f_c and torque
// tau_c (F = [f_x, f_y, tau] per body), times cG = 1 / (4 pi eta).  One thread per
// node, a loop over the bodies: O(N n), evaluated once per solve.
__global__ __launch_bounds__(256) void k_sk_complete_real(int N, int n, const double *__restrict__ x,
                                                         const double *__restrict__ q, const double *__restrict__ F,
                                                         double L, double rc2, double xi2, double cG,
                                                         const double *__restrict__ tab, double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double xx = x[2 * i], xy = x[2 * i + 1];
  double vx = 0, vy = 0;
  for (int c = 0; c < n; ++c) {
    double dx = xx - q[2 * c], dy = xy - q[2 * c + 1];
    dx -= L * rint(dx / L);
    dy -= L * rint(dy / L);
    const double r2 = dx * dx + dy * dy;
    if (r2 > rc2 || r2 == 0.0) continue;
    const double z = xi2 * r2;
    const double ez = exp(-z);
    const double e1 = z <= 2.0 ? poly<double, 16>(tab, z) - log(z) : ez * poly<double, 16>(tab + far_interval(z) * 19, z);
    const double fx = F[3 * c], fy = F[3 * c + 1], tq = F[3 * c + 2];
    const double a = 0.5 * e1 - ez;
    const double sdot = ez * (dx * fx + dy * fy) / r2;
    const double rot = (1.0 - z) * ez / r2 * tq;
    vx += a * fx + sdot * dx - rot * dy;
    vy += a * fy + sdot * dy + rot * dx;
  }
  out[2 * i] = cG * vx;
  out[2 * i + 1] = cG * vy;
}

}  // namespace

hipError_t launch_dl_real(const PairLists &pl, const PairArgs &a, const double *src, const double *wc, double *out,
                          hipStream_t s) {
  if (pl.N == 0) return hipSuccess;
  PairJob j;
  j.N = pl.N;
  j.ngroups = pl.ngroups;
  j.perm = a.perm;
  j.goff = pl.goff;
  j.gnn = pl.gnn;
  j.gnf = pl.gnf;
  j.ell = pl.ell;
  j.tcell = a.tcell;
  j.cell_start = a.cell_start;
  j.nb = a.nb;
  j.cell = a.cell;
  j.xi2 = a.xi2;
  j.cG = a.cG;
  j.src = src;
  j.out = out;
  hipLaunchKernelGGL(k_dl_ell, dim3((pl.N + 255) / 256), dim3(256), 0, s, j, (const double2 *)wc);
  return hipGetLastError();
}

hipError_t launch_sk_complete_real(int N, int n, const double *x, const double *q, const double *F, double L,
                                   const PairArgs &a, double *out, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sk_complete_real, dim3((N + 255) / 256), dim3(256), 0, s, N, n, x, q, F, L, a.rc2, a.xi2,
                     a.cG, a.e1tab, out);
  return hipGetLastError();
}

}  // namespace fbim
