// Launch wrappers of the FBIM device kernels (gfx950).  All pointers are device
// pointers; every wrapper enqueues on `s` and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fbim {

struct GeomDev {
  int n, N;
  const int *shape;      // [n]
  const int *off;        // [n+1] first node of each body
  const int *body;       // [N] body of each node
  const double *q;       // [2n]
  const double *theta;   // [n]
  const double *const *ref;  // per shape: ref_xy [2 n_p]   (device array of device pointers)
  const int *np;         // per shape: n_p
};

// nodes (wrapped into [0, L)) -> x[2N]
hipError_t launch_nodes(const GeomDev &g, double L, double *x, hipStream_t s);
// bodies moved on the device: q = q_src + a dQ_xy, theta = th_src + a dQ_theta (dQ [3n] or null)
hipError_t launch_move_bodies(int n, const double *q_src, const double *th_src, const double *dQ, double a,
                              double *q, double *theta, hipStream_t s);

// binning: key per node, counts (atomic), exclusive scan, scatter, in-bin sort
hipError_t launch_cell_keys(int N, const double *x, double L, int nb, int *key, int *count, hipStream_t s);
hipError_t launch_tile_keys(int N, const double *x, double h, int M, int T, int *key, int *count, hipStream_t s);
hipError_t launch_scan(int n, const int *count, int *start, int *maxcount, hipStream_t s);
hipError_t launch_scatter(int N, const int *key, const int *start, int *cursor, int *perm, hipStream_t s);
hipError_t launch_sort_bins(int nbins, const int *start, int *perm, hipStream_t s);
hipError_t launch_gather2(int N, const int *perm, const double *src, double *dst, hipStream_t s);
hipError_t launch_gather2f(int N, const int *perm, const double *src, float *dst, hipStream_t s);
// tile order: nearest grid indices a = floor(x / h + 1/2) and offsets x - a h (FP64, and FP32 if off32)
hipError_t launch_anchors(int N, const int *tperm, const double *x, double h, int *anchor, double *off64,
                          float *off32, hipStream_t s);
// cell order: each node's cell (tcell) and coordinates relative to the cell's corner (loc64 FP64 pairs; and the
// (x, y) halves of the packed source records src64 and, if given, src32, which hold
// N + 1 records: the last is the zero record of empty neighbour-list slots)
hipError_t launch_cell_local(int N, const int *cperm, const int *key, const double *x, int nb, double cell,
                             double *loc64, double *src64, float *src32, int *tcell, hipStream_t s);
// packed pair-kernel sources: (x, y) from launch_cell_local, densities here:
// src[i].zw = mu[perm[i]] (src64: double4 records, src32: float4 records)
hipError_t launch_gather_src(int N, const int *perm, const double *mu, double *src64, float *src32, hipStream_t s);

// closest approach of nodes of distinct bodies (cell list, absolute positions xa); flag set if < thresh
hipError_t launch_overlap(int N, const int *cell_start, const int *perm, const double *xa, const int *body,
                          int nb, double L, double thresh, int *flag, hipStream_t s);

// real-space pair sum (eq. 3.15, trapezoid pairs within r_c): out[perm[i]] = sum;
// xs are cell-local coordinates (launch_cell_local)
struct PairArgs {
  const int *cell_start;
  const int *perm;
  const int *ckey;      // cell of each original node
  const int *tcell;     // cell of each cell-sorted node
  int nb;
  double cell, rc2, xi2, cG;  // cell side L / n_box
  const double *e1tab;  // FP64 table
  const float *e1tab32; // FP32 table
};
// Neighbour lists in ELL layout (groups of 64 cell-sorted targets; near rows first)
struct PairLists {
  int N, ngroups;
  int *cnt_near, *cnt_far;  // [N]
  int *gnn, *gnf, *goff;    // [ngroups], goff [ngroups + 1]
  uint16_t *ell;            // [goff[ngroups] + kEllSlack]
};
// An ELL entry (16 bits) names a source by the neighbour cell of its target's cell
// it lies in and its place there: bits 12-15 hold k = (dcx + 1) + 3 (dcy + 1)
// (0..8), bits 0-11 the source's index within that cell (cells hold at most
// kEllMaxCell nodes).  k = 9 (kEllEmpty) marks an empty slot, which the pair
// kernel maps to the zero record after the N sources of the packed record arrays
// (position (-1.5, -1.5) cells from its cell corner, density 0): it is evaluated
// like any source and adds exactly 0.  kEllSlack slots after the last group, kept
// empty: the pair kernel reads up to 12 rows past a group's end (list entries in
// flight for rows it then skips).
constexpr int kEllMaxCell = 4096;
// nodes per context: the N + 1 packed records are indexed below 2^26
constexpr int kMaxNodes = (1 << 26) - 2;
constexpr uint16_t kEllEmpty = 9 << 12;
constexpr int kEllSlack = 16 * 64;
// mode 0: per-target near / far counts; mode 1: fill pl.ell.  With `flag`
// (mode 0), *flag is set when nodes of distinct bodies (body[] per original node
// index) are closer than sqrt(thresh2) (which must not exceed r_c).  Mode 1 with
// maxrows (the longest group, from pair_lists_stage_rows) > 0 writes every slot
// (empty ones kEllEmpty) through LDS; with maxrows = 0 pl.ell must be pre-set to
// kEllEmpty.
constexpr size_t kListStageBytes = 64 * 1024;
int pair_lists_stage_rows(int maxrows);  // maxrows if its staging fits kListStageBytes, else 0
hipError_t launch_pair_lists(const PairArgs &a, PairLists &pl, const double *xs, int mode, hipStream_t s,
                             const int *body = nullptr, double thresh2 = 0.0, int *flag = nullptr,
                             int maxrows = 0);
// gnn, gnf and gsize[g] = 64 (gnn + gnf) from the counts
hipError_t launch_group_rows(PairLists &pl, int *gsize, hipStream_t s);
// src: packed (x, y, mu_x, mu_y) records in cell order (launch_cell_local + launch_gather_src)
hipError_t launch_pair_f64(const PairLists &pl, const PairArgs &a, const double *src, double *out, hipStream_t s);
hipError_t launch_pair_f32(const PairLists &pl, const PairArgs &a, const float *src, double *out, hipStream_t s);
hipError_t launch_fill_int(size_t n, int v, int *y, hipStream_t s);

// Alpert band: out[i] += R_b A_ref R_b^T mu (per node); accumulate=1 adds.  band_tab[shape]
// holds the 2 x 2 blocks o-major: block (o, t) at ((o + band) n_p + t) 4
hipError_t launch_alpert(const GeomDev &g, const double *const *band_tab, const int *band, const double *mu,
                         double *out, int accumulate, hipStream_t s);

// spectral Ewald
struct WaveArgs {
  int M, T, P, nts;
  double h, L, ag, cg;  // Gaussian exp(-ag r^2) * cg
  const int *tile_start;
  const int *anchor;    // per tile-sorted node: nearest grid indices (ix, iy), unwrapped, from FP64 positions
  const int *slist_start, *slist;  // spreading lists (launch_spread_lists)
};
// Spreading lists: per grid tile, the tile-sorted indices of the nodes whose
// P x P stencil touches the tile (all in the 3 x 3 neighbouring tiles), in a
// fixed order (neighbour tile, then node order).  mode 0: count[tile] = their
// number; mode 1: list[start[tile] + rank] = node.
hipError_t launch_spread_lists(const WaveArgs &w, int *count, const int *start, int *list, int mode, hipStream_t s);
// xt are the tile-ordered offsets from the nearest grid point (launch_anchors)
hipError_t launch_spread_f64(const WaveArgs &w, const double *xt, const double *mut, double *grid, hipStream_t s);
hipError_t launch_spread_f32(const WaveArgs &w, const float *xt, const float *mut, float *grid, hipStream_t s);
hipError_t launch_interp_f64(const WaveArgs &w, const double *xt, const int *tperm, const double *grid,
                             double *out, hipStream_t s);
hipError_t launch_interp_f32(const WaveArgs &w, const float *xt, const int *tperm, const float *grid,
                             double *out, hipStream_t s);
// multiplier on the half spectrum [2][M][M/2+1]: mode 0 = M^(w) (eq. 3.23-3.25),
// mode 1 = random field B^(1/2) (eq. 3.28-3.30)
// Fourier multiplier of the wave-space operator at grid frequency (row, col),
// row = ky index in [0, M), col = kx index in [0, M/2]:
//   mode 0: (1+u) exp(-(1-eta_s) u) / k^2 (I - k k^T/k^2)          (M^(w), eq. 3.23)
//   mode 1: sqrt(1+u) exp(-(1-eta_s) u/2) / k (I - k k^T/k^2)       (B^(1/2), eq. 3.29)
// with u = k^2 / 4 xi^2, times `scale`, as s * [[pxx, pxy], [pxy, pyy]]; false
// (multiplier zero) at k = 0.  On the Nyquist row and column the off-diagonal
// term is dropped, which makes the complex-to-real inverse transform equal to
// the real part of the full inverse transform.
template <typename T>
__device__ inline bool wave_multiplier(int M, int row, int col, T twopi_L, T inv4xi2, T one_m_eta, T scale, int mode,
                                       T &s, T &pxx, T &pxy, T &pyy) {
  const T kx = twopi_L * col;
  const T ky = twopi_L * (row < M / 2 ? row : row - M);
  const T k2 = kx * kx + ky * ky;
  if (k2 == T(0)) return false;
  const T u = k2 * inv4xi2;
  if (mode == 0)
    s = (T(1) + u) * exp(-one_m_eta * u) / k2 * scale;
  else
    s = sqrt(T(1) + u) * exp(T(-0.5) * one_m_eta * u) / sqrt(k2) * scale;
  pxx = T(1) - kx * kx / k2;
  pyy = T(1) - ky * ky / k2;
  pxy = (col == M / 2 || row == M / 2) ? T(0) : -kx * ky / k2;
  return true;
}

hipError_t launch_multiplier_f64(int M, double L, double xi, double eta_s, double scale, int mode, double *spec,
                                 hipStream_t s);
// Fused wave-space convolution (kernels_fft.hip) for power-of-two 64 <= M <= 2048:
// grid planes [2][M][M] -> same planes after transform, multiplier (mode, scale as
// launch_multiplier) and inverse transform; spec is scratch of 4 M (M/2+1) reals
// (the half spectra, kx-major); tw holds exp(-2 pi i k / M), k < M (interleaved);
// ey[i] = exp(-(1 - eta_s) k_i^2 / 4 xi^2) with k_i = 2 pi / L (i < M/2 ? i : i - M).
struct WaveConvArgs {
  int M, mode;
  double L, xi, eta_s, scale;
};
bool wave_conv_supported(int M);
hipError_t launch_wave_conv_f64(const WaveConvArgs &a, double *grid, double *spec, const double *tw, const double *ey,
                                hipStream_t s);
hipError_t launch_wave_conv_f32(const WaveConvArgs &a, float *grid, float *spec, const float *tw, const float *ey,
                                hipStream_t s);
hipError_t launch_multiplier_f32(int M, double L, double xi, double eta_s, double scale, int mode, float *spec,
                                 hipStream_t s);

// second-kind formulation (Appendix B; kernels_real.hip, kernels_sk.hip)
// real-space periodic stresslet over the neighbour lists: out[node] = cG sum_s
// T^(r)_jlm phi_l w_m with src the pair records (x, y, phi) and wc[k] = n ds of the
// k-th cell-sorted node (outward normal)
hipError_t launch_dl_real(const PairLists &pl, const PairArgs &a, const double *src, const double *wc, double *out,
                          hipStream_t s);
// real-space completion flow at every node from the bodies' (f_x, f_y, tau) F[3n]
// at q[2n] (x: wrapped node positions), O(N n)
hipError_t launch_sk_complete_real(int N, int n, const double *x, const double *q, const double *F, double L,
                                   const PairArgs &a, double *out, hipStream_t s);
// per node: w = n ds, diag = 2 kappa ds t t^T (xx, xy, yy), ds, r = x - q (rotated
// reference data sk6[shape][n_p][nx, ny, tx, ty, kappa, ds]); wc = w in cell order
hipError_t launch_sk_geom(const GeomDev &g, const double *const *sk6, const int *cperm, double *w, double *wc,
                          double *diag, double *ds, double *r, hipStream_t s);
// tile-ordered spreading inputs A = phi_x w, B = phi_y w
hipError_t launch_sk_prep(int N, const int *tperm, const double *phi, const double *w, double *A, double *B,
                          hipStream_t s);
// the bodies' (f_x, f_y, tau) spread with the Gaussian of w into grid planes 0..2
// (added; FP64 atomics, P <= 15)
hipError_t launch_point_spread(int n, const double *q, const double *F, const WaveArgs &w, double *grid,
                               hipStream_t s);
// multiplier on [4][M][M/2+1] half spectra: mode 0 stresslet (S_xx, S_xy, S_yx, S_yy
// -> U_x, U_y), mode 1 completion (f_x, f_y, tau -> U_x, U_y); sc = h^2 / (eta L^2)
hipError_t launch_sk_mult(int M, double L, double xi, double eta_s, double sc, int mode, double *spec,
                          hipStream_t s);
// closure rows yU = U - Z phi per body and the stresslet mean term mean[2] =
// cm sum_s (q + r)_s (phi . w)_s (lw: per shape length, W; part: n x 2 scratch)
hipError_t launch_sk_body(const GeomDev &g, const double *lw, const double *phi, const double *w, const double *ds,
                          const double *r, const double *U, double *yU, double *part, double cm, double *mean,
                          hipStream_t s);
// y_phi = -phi/2 + real + wave + mean + cG diag phi + U_b + omega_b r^perp
hipError_t launch_sk_combine(const GeomDev &g, const double *phi, const double *real, const double *wave,
                             const double *mean, const double *diag, double cG, const double *r, const double *U,
                             double *y, hipStream_t s);

// rigid-body maps (Section 3.1)
// y_mu[i] = y_mu[i] - (K U)_i ; y_U[b] = sgn * (K^T mu)_b
hipError_t launch_sub_KU(const GeomDev &g, const double *U, double *y, hipStream_t s);
hipError_t launch_KT(const GeomDev &g, const double *mu, double sgn, double *out, hipStream_t s);

// per-body dense operators (Sections 3.3-3.4), single shape per launch group
struct BodyMats {
  const double *const *Mp;    // per shape (2n_p)^2 column-major
  const double *const *Pref;  // per shape 2n_p x 3 column-major
  const double *const *Nt;    // per shape 3x3
  const double *const *G;     // per shape
  const double *const *Gp;    // per shape
  int max_np;
};
// Tiles of bodies of one shape (host-built): tile = (shape, first index into
// list, count, 0); list holds body indices grouped by shape.  A tile of a shape
// with n2 = 2 n_p unknowns (n2 a multiple of 4, 32 <= n2 <= 1024) holds up to
// body_tile_cap(n2) bodies, so that (n2 / 4) x (cap / 4) <= 256 threads each own
// a 4 x 4 output block; the matrix streams through LDS body_tile_kc(n2) rows at
// a time, and body_tile_lds(n2) bytes of dynamic LDS hold both.
constexpr int kBodyTileMax = 64;
__host__ __device__ inline int body_tile_cap(int n2) {
  const int c = 4 * (1024 / n2);
  return c < 4 ? 4 : (c > kBodyTileMax ? kBodyTileMax : c);
}
__host__ __device__ inline int body_tile_kc(int n2) {  // KC * n2 <= 2048 (16 KB of LDS)
  const int c = 2048 / n2;
  return c < 2 ? 2 : (c > 16 ? 16 : c);
}
__host__ __device__ inline size_t body_tile_lds(int n2) {
  return ((size_t)n2 * body_tile_cap(n2) + (size_t)body_tile_kc(n2) * n2) * sizeof(double);
}
struct BodyTiles {
  const int4 *tile;
  const int *list;
  int ntile;
  size_t lds_bytes;
  int mfma = 0;  // matrix-core form: row blocks per wave (body_mfma_rb), 0: the other form
};
// The FP64 matrix-core form of the per-body operators: tiles of 16 bodies, the
// shared matrix times the tile's body-frame vectors as 16 x 16 x 4 FP64 MFMA
// blocks.  It serves shapes with 16 | 2 n_p and 2 n_p <= 256.
constexpr int kBodyMfmaCols = 16;
__host__ __device__ inline bool body_mfma_ok(int n2) { return n2 % 16 == 0 && n2 >= 32 && n2 <= 256; }
__host__ __device__ inline size_t body_mfma_lds(int n2) { return (size_t)n2 * kBodyMfmaCols * sizeof(double); }
// 16-row blocks of the product per wave (four waves) for the largest 2 n_p of the tiles
__host__ __device__ inline int body_mfma_rb(int n2max) { return n2max <= 64 ? 1 : (n2max <= 128 ? 2 : 4); }
// block-diagonal saddle preconditioner: z = [a (2N) | b (3n)] -> y = [mu | U];
// dN (optional, [n][6] = xx, yy, tt, xy, xt, yt) corrects N_ref per body in the body frame
hipError_t launch_precond(const GeomDev &g, const BodyMats &m, const BodyTiles &bt, const double *dN,
                          const double *z, double *y, hipStream_t s);
// y_b = R_b X_ref R_b^T x_b with X = G (which = 0) or G^+ (which = 1)
hipError_t launch_body_apply(const GeomDev &g, const BodyMats &m, const BodyTiles &bt, int which, const double *x,
                             double *y, hipStream_t s);

// Krylov helpers (FP64)
// A batch vector is cut into chunks of at most kChunk elements, each inside one
// system; the chunks of a system are contiguous (sys_chunk[s] .. sys_chunk[s+1]).
constexpr int kChunk = 2048;
constexpr int kOrthMaxCols = 512;  // largest column count k + 1 of one orthogonalisation
constexpr int kOrthFused = 32;     // largest k of the fused subtract-and-project pass
constexpr int kLagSlot = kOrthFused + 8;  // per-system room of a lagged-pass output (K + 2 <= 33 values)
struct Segs {
  const int2 *chunk;     // [nchunk] element ranges [x, y)
  const int *chunk_sys;  // [nchunk]
  const int *sys_chunk;  // [S + 1]
  int nchunk, S;
};
// Gram-Schmidt passes over the k columns of V (leading dimension ld) and w:
//   mode 0: out[s][j] = V_j . w (j < k), out[s][k] = w . w
//   mode 1: w -= V h[s]; then out[s][j] = V_j . w (j < k), out[s][k] = w . w   (k <= kOrthFused)
//   mode 2: w -= V h[s]; out[s][0] = w . w
// h[s][j] = h[s * hstride + j] on the device; out[s][j] = out[s * ostride + j].
// If cond is given, systems with cond[s] == 0 are skipped (conditional second pass).
// partial holds nchunk * (k + 1) doubles (reduced by a second launch).
struct OrthArgs {
  Segs seg;
  const double *V;
  size_t ld;
  int k;
  double *w;
  // batches: per-system basis, vector and leading dimension (used when Vs is set)
  const double *const *Vs = nullptr;
  double *const *ws = nullptr;
  const size_t *lds = nullptr;
  const double *h;
  int hstride;
  const double *cond;
  double *partial;
  double *out;
  int ostride;
  int v32 = 0;  // V / Vs address FP32 columns (widened to FP64 for the arithmetic)
  // lagged pass only: the previous lagged pass's output per system (lag[s * lagstride + j]);
  // with next set, the new vector goes to basis slot K + 1 and to xs[s] (FP64) instead of w
  const double *lag = nullptr;
  int lagstride = 0;
  int next = 0;
  double *const *xs = nullptr;
};
hipError_t launch_orth(int mode, const OrthArgs &a, hipStream_t s);
// Lagged pass of delayed reorthogonalisation (one Arnoldi step reads the basis
// twice instead of three times) over the k = K final columns V_0..V_{K-1}, the
// column in slot K and w, K < kOrthFused.  Slot K holds nu u, u of unit norm and
// orthogonal to V_{<K} but for s = lag[0..K) / nu, where nu = sqrt(lag[K]) (lag: the
// previous lagged pass's output; nu = 1 and no lag for K = 0), and w = nu A u.
// h[0..K] = V_{<=K}^T w from a mode-0 pass over slots 0..K.  With rho = sqrt(1 - s.s),
// t = h[0..K) / nu and e = (h[K] / nu^2 - s.t) / rho:
//   V_K = (u - V_{<K} s) / rho             (over slot K; not written for K = 0)
//   x   = (w / nu - V_{<K} t - V_K e) / rho  into w, or with `next` into slot K + 1
//                                           and xs (FP64)
//   out[j] = V_j . x (j <= K), out[K + 1] = x . x
hipError_t launch_orth_lag(const OrthArgs &a, hipStream_t s);
// vector of system s in a batch: base[s] + col * ld[s] (ld may be null: col ignored)
struct VecRef {
  const double *const *base;
  const size_t *ld;
  int col;
  int f32 = 0;  // the vectors are FP32 (base pointers address floats; ld counts floats)
};
// y_s = a[s] x_s + b[s] y_s over the chunks of each system (a, b: device, [S])
hipError_t launch_seg_axpby(const Segs &seg, const VecRef &x, const VecRef &y, const double *a, const double *b,
                            hipStream_t s);
// y_s = a[s] x_s (rounded to y's precision) and z_s = the same values in FP64
// (z FP64; x_s not read when a[s] == 0): a basis column and its FP64 copy in one pass
hipError_t launch_seg_scale2(const Segs &seg, const VecRef &x, const VecRef &y, const VecRef &z, const double *a,
                             hipStream_t s);
// y_s = V_s[:, 0..k) c_s with c_s = c + s * cstride (device)
hipError_t launch_seg_Vc(const Segs &seg, const VecRef &V, int k, const double *c, int cstride, const VecRef &y,
                         hipStream_t s);
// flag[s] = 1 if nrm[s * ns] < before[s * nb] / 2 (the pass lost more than half of ||w||^2)
hipError_t launch_need_second_pass(int S, const double *nrm, int ns, const double *before, int nb, double *flag,
                                   hipStream_t s);
// Host-visible results (pinned, fine-grained host memory read by the host
// without a copy): `v` holds the values, `tag` is written after them, so the
// host that sees the tag it waits for may read the values.
struct HostPub {
  unsigned long long *tag = nullptr, *tag_dev = nullptr;
  double *v = nullptr, *v_dev = nullptr;
  size_t cap = 0;
  unsigned long long seq = 0;
};
hipError_t pub_alloc(HostPub &p, size_t n);  // room for n values
void pub_free(HostPub &p);
// Blocks the host until the launches that publish `tag` on stream s have written
// it (a spin on host memory, then a stream synchronisation as the fallback).
hipError_t pub_wait(const HostPub &p, unsigned long long tag, hipStream_t s);
// Orthogonalisation results of S systems (CGS2 / selective second pass):
// second = !selective || flag[s fs] != 0; for j < k
// v[s (k+1) + j] = h[s hs + j] + (second ? h2[s hs + j] : 0);
// after = second ? nrm_b[s ns] : (fused ? h2[s hs + k] : nrm_a[s ns]);
// v[s (k+1) + k] = sqrt(max(after, 0)) = hn_s and a[s as] = hn_s > 0 ? 1 / hn_s : 0
// (device), the scale that normalises w_s; then the tag.
struct OrthPublish {
  int S = 1, k = 0, hs = 0, ns = 0, fs = 0, as = 0;
  bool fused = true, selective = false;
  const double *h = nullptr, *h2 = nullptr, *nrm_a = nullptr, *nrm_b = nullptr, *flag = nullptr;
  double *a = nullptr;
};
hipError_t launch_orth_publish(const OrthPublish &o, HostPub &p, unsigned long long tag, hipStream_t s);
// v[i] = src[i stride] for i < n, then the tag
hipError_t launch_publish(int n, const double *src, int stride, HostPub &p, unsigned long long tag, hipStream_t s);
// per system s < S: v[s (n0 + n1) + j] = src0[s stride0 + j] (j < n0), then
// src1[s stride1 + j - n0] (j < n0 + n1); then the tag
hipError_t launch_publish2(int S, int n0, const double *src0, int stride0, int n1, const double *src1, int stride1,
                           HostPub &p, unsigned long long tag, hipStream_t s);
// y *= a[0] with a on the device
hipError_t launch_scale_dev(size_t n, const double *a, double *y, hipStream_t s);
// y[i] = sum_j V[j*ld + i] * c[j]
hipError_t launch_Vc(const double *V, size_t ld, int k, const double *c, double *y, size_t n, hipStream_t s);
hipError_t launch_axpby(size_t n, double a, const double *x, double b, double *y, hipStream_t s);  // y = a x + b y
hipError_t launch_scale(size_t n, double a, double *y, hipStream_t s);  // y *= a
hipError_t launch_vec_add(int k, const double *a, double *b, hipStream_t s);  // b += a
hipError_t launch_cast_f32(size_t n, const double *x, float *y, hipStream_t s);
hipError_t launch_fill(size_t n, double v, double *y, hipStream_t s);

// counter-based standard normals (kernels_rng.hip): out[i] for i < n of stream
// `stream` at draw `counter` (Philox4x32-10 keyed by seed, Box-Muller)
hipError_t launch_normals(uint64_t seed, uint32_t stream, uint64_t counter, size_t n, double *out, hipStream_t s);
// the raw Philox output words behind them: out[4 j .. 4 j + 3] of pair j < npairs
hipError_t launch_philox_words(uint64_t seed, uint32_t stream, uint64_t counter, size_t npairs, uint32_t *out,
                               hipStream_t s);

// ---------------------------------------------------------------- batched launches
// Several independent systems (suspensions) go through one launch per stage:
// system s owns blocks [begin[s], begin[s+1]) of the grid, and each block reads
// its system's job description (pointers and parameters) from a device table.
struct BatchGrid {
  const int *begin;  // [S + 1] block offsets
  int S, nblocks;
};
// last s < S with begin[s] <= blk (empty systems own no block)
__device__ inline int batch_system(const int *begin, int S, int blk) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
struct GatherJob {  // dst[i] = src[perm[i]] for N (x, y) pairs; dst FP64 or FP32 per launch
  int N;
  const int *perm;
  const double *src;
  void *dst;
  int packed;  // 1: dst holds 4-vector records and receives their (z, w) halves
};
struct PairJob {  // one system's real-space pair sum (launch_pair_f64 / _f32 arguments)
  int N, ngroups;
  const int *perm, *goff, *gnn, *gnf;
  const uint16_t *ell;
  const int *tcell, *cell_start;  // cell of each cell-sorted node; cell offsets
  int nb;
  double cell, xi2, cG;
  const void *src;  // packed (x, y, mu_x, mu_y) records in cell order (double4 or float4)
  double *out;
};
struct AlpertJob {
  GeomDev g;
  const double *const *band_tab;
  const int *band;
  const double *mu;
  double *out;
};
struct SpreadJob {
  WaveArgs w;
  const void *xt, *mut;
  void *grid;
};
struct InterpJob {
  WaveArgs w;
  const void *xt;
  const int *tperm;
  const void *grid;
  double *out;
};
struct MultJob {  // multiplier on one system's half spectrum
  int M;
  double L, xi, eta_s, scale;
  void *spec;
};
struct RigidJob {  // saddle rigid-body terms: y_mu -= K x_U, y_U = -K^T x_mu
  GeomDev g;
  const double *x;
  double *y;
};
struct PrecondJob {
  GeomDev g;
  BodyMats m;
  BodyTiles bt;
  const double *dN;
  const double *z;
  double *y;
};
// grids: blocks of 256 threads per system as listed with each launcher
hipError_t launch_gather2_batch(const GatherJob *jobs, BatchGrid bg, int f32, hipStream_t s);
// both job tables (same node counts per system) in one launch
hipError_t launch_gather2x2_batch(const GatherJob *ja, const GatherJob *jb, BatchGrid bg, int f32, hipStream_t s);   // ceil(N/256)
hipError_t launch_pair_batch(const PairJob *jobs, BatchGrid bg, int f32, const double *tab64, const float *tab32,
                             hipStream_t s);                                                     // ceil(64 ngroups/256)
hipError_t launch_alpert_batch(const AlpertJob *jobs, BatchGrid bg, hipStream_t s);              // ceil(N/256)
// pmax: the largest stencil width P of the batch (sizes the dynamic LDS)
hipError_t launch_spread_batch(const SpreadJob *jobs, BatchGrid bg, int f32, int pmax, hipStream_t s);  // nts^2
hipError_t launch_interp_batch(const InterpJob *jobs, BatchGrid bg, int f32, int pmax, hipStream_t s);  // nts^2
hipError_t launch_multiplier_batch(const MultJob *jobs, BatchGrid bg, int f32, int mode,
                                   hipStream_t s);                                                // ceil(M(M/2+1)/256)
hipError_t launch_rigid_batch(const RigidJob *jobs, BatchGrid bg_nodes, BatchGrid bg_bodies, hipStream_t s);
                                                                        // ceil(N/256); bodies: ceil(n/4) (64 per body)
// bt.ntile blocks per system; lds_bytes = the largest bt.lds_bytes of the systems
// all_mfma: row blocks per wave when every system's tiles take the matrix-core form (a kernel
// without the other form), else 0
hipError_t launch_precond_batch(const PrecondJob *jobs, BatchGrid bg, size_t lds_bytes, int all_mfma,
                                hipStream_t s);

// learned preconditioner correction (MLP 32 -> 128 -> 128 -> 6, tanh)
constexpr int kMlpNeighbours = 6, kMlpIn = 32, kMlpHid = 128, kMlpOut = 6;
// features [n][32] of each body's neighbourhood in its body frame, found on a
// cell list of the bodies (cells of side >= 3 r_max; device scratch below)
struct MlpCells {
  int nbc;  // cells per side (mlp_body_cells)
  int *key, *count, *cursor, *start, *perm, *maxcount;  // [n], [nbc^2] x 2, [nbc^2 + 1], [n], [1]
};
int mlp_body_cells(double L, double r_max);
hipError_t launch_mlp_features(int n, const double *q, const double *theta, double L, double r_max, int sym,
                               const MlpCells &cells, float *X, hipStream_t s);
enum { kGemmStore = 0, kGemmBiasTanh = 1, kGemmBias = 2, kGemmAtomic = 3, kGemmTanhGrad = 4 };
// C = op(A) op(B) in BF16 MFMA with FP32 accumulation; epilogues: store, tanh(. + bias[j]),
// . + bias[j], atomic add (split K), . * (1 - aux[i][j]^2) (aux has leading dimension ldc)
struct GemmArgs {
  int M, N, K;
  const float *A;
  size_t sam, sak;
  const float *B;
  size_t sbk, sbn;
  float *C;
  size_t ldc;
  const float *bias, *aux;
  int epi;
};
hipError_t launch_gemm_bf16(const GemmArgs &g, int ksplit, hipStream_t s);
hipError_t launch_mlp_loss(int n, int ns, const int *shape, const double *theta, const double *const *Nt,
                           const float *Y, const double *F, const double *U, float *dY, float *loss, hipStream_t s);
hipError_t launch_mlp_correction(int n, const int *shape, const double *const *Nt, const float *Y, double *dN,
                                 hipStream_t s);
hipError_t launch_adam(int n, float lr, float b1, float b2, float eps, int t, const float *g, float *m, float *v,
                       float *w, hipStream_t s);
hipError_t launch_fill_f32(size_t n, float v, float *y, hipStream_t s);

}  // namespace fbim
