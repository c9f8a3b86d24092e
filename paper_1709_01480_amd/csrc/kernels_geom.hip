// Geometry kernels: node positions (Section 3.1), cell and tile binning for the
// real-space cell list (Section 3.2) and the spreading tiles.
#include "kernels.h"

namespace fbim {

__global__ void k_nodes(int N, const int *__restrict__ body, const int *__restrict__ off,
                        const int *__restrict__ shape, const double *__restrict__ q,
                        const double *__restrict__ theta, const double *const *ref, double L,
                        double *__restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = body[i];
  const int t = i - off[b];
  const double *r = ref[shape[b]];
  double sn, cs;
  sincos(theta[b], &sn, &cs);
  const double rx = r[2 * t], ry = r[2 * t + 1];
  double px = q[2 * b] + cs * rx - sn * ry;
  double py = q[2 * b + 1] + sn * rx + cs * ry;
  px -= L * floor(px / L);
  py -= L * floor(py / L);
  if (px >= L) px -= L;  // guard against rounding up to L
  if (py >= L) py -= L;
  x[2 * i] = px;
  x[2 * i + 1] = py;
}

// q[b] = q_src[b] + a dQ[3b, 3b+1], theta[b] = theta_src[b] + a dQ[3b+2] (dQ null: a copy);
// in place when q_src == q
__global__ void k_move_bodies(int n, const double *q_src, const double *th_src, const double *__restrict__ dQ,
                              double a, double *q, double *theta) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double qx = q_src[2 * b], qy = q_src[2 * b + 1], th = th_src[b];
  if (dQ) {
    qx += a * dQ[3 * b];
    qy += a * dQ[3 * b + 1];
    th += a * dQ[3 * b + 2];
  }
  q[2 * b] = qx;
  q[2 * b + 1] = qy;
  theta[b] = th;
}

hipError_t launch_move_bodies(int n, const double *q_src, const double *th_src, const double *dQ, double a,
                              double *q, double *theta, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_move_bodies, dim3((n + 255) / 256), dim3(256), 0, s, n, q_src, th_src, dQ, a, q, theta);
  return hipGetLastError();
}

hipError_t launch_nodes(const GeomDev &g, double L, double *x, hipStream_t s) {
  if (g.N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nodes, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, g.body, g.off, g.shape, g.q,
                     g.theta, g.ref, L, x);
  return hipGetLastError();
}

// counter[k] += 1 for every active lane of the wave, with one atomic per distinct
// key k among the wave's lanes (nodes of one body share few bins); returns what a
// per-lane atomicAdd(&counter[k], 1) would, the lanes of one key taking
// consecutive values in lane order.  Every lane of the wave must call it.
__device__ inline int wave_atomic_inc(int *counter, int k, bool active) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(active);
  int result = 0;
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int kl = __shfl(k, leader);
    const unsigned long long peers = __ballot(active && k == kl) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counter[kl], (int)__popcll(peers));
    base = __shfl(base, leader);
    if ((peers >> lane) & 1ull) result = base + (int)__popcll(peers & ((1ull << lane) - 1ull));
    todo &= ~peers;
  }
  return result;
}

__global__ void k_cell_keys(int N, const double *__restrict__ x, double inv_cell, int nb, int *__restrict__ key,
                            int *__restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < N;
  int c = 0;
  if (on) {
    int cx = (int)floor(x[2 * i] * inv_cell), cy = (int)floor(x[2 * i + 1] * inv_cell);
    cx = min(max(cx, 0), nb - 1);
    cy = min(max(cy, 0), nb - 1);
    c = cy * nb + cx;
    key[i] = c;
  }
  wave_atomic_inc(count, c, on);
}

hipError_t launch_cell_keys(int N, const double *x, double L, int nb, int *key, int *count, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_keys, dim3((N + 255) / 256), dim3(256), 0, s, N, x, nb / L, nb, key, count);
  return hipGetLastError();
}

// tile of the grid point nearest to the node (the centre of its spreading stencil)
__global__ void k_tile_keys(int N, const double *__restrict__ x, double inv_h, int M, int T,
                            int *__restrict__ key, int *__restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < N;
  int c = 0;
  if (on) {
    int ix = (int)floor(x[2 * i] * inv_h + 0.5), iy = (int)floor(x[2 * i + 1] * inv_h + 0.5);
    ix = ((ix % M) + M) % M;
    iy = ((iy % M) + M) % M;
    const int nts = M / T;
    c = (iy / T) * nts + ix / T;
    key[i] = c;
  }
  wave_atomic_inc(count, c, on);
}

hipError_t launch_tile_keys(int N, const double *x, double h, int M, int T, int *key, int *count, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_keys, dim3((N + 255) / 256), dim3(256), 0, s, N, x, 1.0 / h, M, T, key, count);
  return hipGetLastError();
}

// single-workgroup exclusive scan (n up to a few 10^5), also the maximum count.
// Tiles of 4096 counts: each thread sums four consecutive counts, the 64 lanes of a
// wave scan their sums by shuffles, the 16 wave totals meet in LDS, and each thread
// writes its four starts; two barriers per tile.
__global__ __launch_bounds__(1024) void k_scan(int n, const int *__restrict__ count, int *__restrict__ start,
                                               int *__restrict__ maxcount) {
  __shared__ int wsum[16], wmax[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int carry = 0, lmax = 0;
  for (int base = 0; base < n; base += 4096) {
    int v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + 4 * tid + q;
      v[q] = i < n ? count[i] : 0;
      lmax = max(lmax, v[q]);
    }
    const int tsum = (v[0] + v[1]) + (v[2] + v[3]);
    int x = tsum;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int woff = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const int t = wsum[w];
      woff += w < wv ? t : 0;
      total += t;
    }
    int run = carry + woff + x - tsum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + 4 * tid + q;
      if (i < n) start[i] = run;
      run += v[q];
    }
    carry += total;
    __syncthreads();  // every thread has read wsum before the next tile writes it
  }
  if (tid == 0) start[n] = carry;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lmax = max(lmax, __shfl_xor(lmax, o));
  if (lane == 0) wmax[wv] = lmax;
  __syncthreads();
  if (tid == 0) {
    int m = wmax[0];
    for (int w = 1; w < 16; ++w) m = max(m, wmax[w]);
    *maxcount = m;
  }
}

hipError_t launch_scan(int n, const int *count, int *start, int *maxcount, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, n, count, start, maxcount);
  return hipGetLastError();
}

__global__ void k_scatter(int N, const int *__restrict__ key, const int *__restrict__ start, int *__restrict__ cursor,
                          int *__restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = i < N;
  const int c = on ? key[i] : 0;
  const int slot = wave_atomic_inc(cursor, c, on);
  if (on) perm[start[c] + slot] = i;
}

hipError_t launch_scatter(int N, const int *key, const int *start, int *cursor, int *perm, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((N + 255) / 256), dim3(256), 0, s, N, key, start, cursor, perm);
  return hipGetLastError();
}

// Order the nodes inside each bin by node index (makes the permutation
// deterministic).  One work group per bin: the bin is staged in LDS and every
// entry is written to the position given by its rank (all entries distinct).
constexpr int kSortCap = 2048;

__global__ __launch_bounds__(256) void k_sort_bins(const int *__restrict__ start, int *__restrict__ perm) {
  __shared__ int buf[kSortCap];
  const int a = start[blockIdx.x], n = start[blockIdx.x + 1] - a;
  if (n <= 1) return;
  if (n > kSortCap) {  // rare oversized bin: serial insertion sort
    if (threadIdx.x == 0)
      for (int i = a + 1; i < a + n; ++i) {
        const int v = perm[i];
        int j = i - 1;
        while (j >= a && perm[j] > v) {
          perm[j + 1] = perm[j];
          --j;
        }
        perm[j + 1] = v;
      }
    return;
  }
  for (int i = threadIdx.x; i < n; i += 256) buf[i] = perm[a + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    const int v = buf[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += buf[j] < v;
    perm[a + rank] = v;
  }
}

hipError_t launch_sort_bins(int nbins, const int *start, int *perm, hipStream_t s) {
  if (nbins == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_bins, dim3(nbins), dim3(256), 0, s, start, perm);
  return hipGetLastError();
}

__global__ void k_gather2(int N, const int *__restrict__ perm, const double2 *__restrict__ src,
                          double2 *__restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[i] = src[perm[i]];
}

__global__ void k_gather2f(int N, const int *__restrict__ perm, const double2 *__restrict__ src,
                           float2 *__restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    const double2 v = src[perm[i]];
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

hipError_t launch_gather2(int N, const int *perm, const double *src, double *dst, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather2, dim3((N + 255) / 256), dim3(256), 0, s, N, perm, (const double2 *)src,
                     (double2 *)dst);
  return hipGetLastError();
}

hipError_t launch_gather2f(int N, const int *perm, const double *src, float *dst, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather2f, dim3((N + 255) / 256), dim3(256), 0, s, N, perm, (const double2 *)src,
                     (float2 *)dst);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather2_batch(const GatherJob *__restrict__ jobs, BatchGrid bg, int f32) {
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  const GatherJob j = jobs[s];
  const int i = (blockIdx.x - bg.begin[s]) * 256 + threadIdx.x;
  if (i >= j.N) return;
  const double2 v = reinterpret_cast<const double2 *>(j.src)[j.perm[i]];
  const int k = j.packed ? 2 * i + 1 : i;  // packed records: the (z, w) half of record i
  if (f32)
    reinterpret_cast<float2 *>(j.dst)[k] = make_float2((float)v.x, (float)v.y);
  else
    reinterpret_cast<double2 *>(j.dst)[k] = v;
}

hipError_t launch_gather2_batch(const GatherJob *jobs, BatchGrid bg, int f32, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather2_batch, dim3(bg.nblocks), dim3(256), 0, s, jobs, bg, f32);
  return hipGetLastError();
}

// the same for two job tables over the same node counts (one launch)
__global__ __launch_bounds__(256) void k_gather2x2_batch(const GatherJob *__restrict__ ja,
                                                         const GatherJob *__restrict__ jb, BatchGrid bg, int f32) {
  const int s = batch_system(bg.begin, bg.S, blockIdx.x);
  const int i = (blockIdx.x - bg.begin[s]) * 256 + threadIdx.x;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const GatherJob j = t == 0 ? ja[s] : jb[s];
    if (i >= j.N) continue;
    const double2 v = reinterpret_cast<const double2 *>(j.src)[j.perm[i]];
    const int k = j.packed ? 2 * i + 1 : i;
    if (f32)
      reinterpret_cast<float2 *>(j.dst)[k] = make_float2((float)v.x, (float)v.y);
    else
      reinterpret_cast<double2 *>(j.dst)[k] = v;
  }
}

hipError_t launch_gather2x2_batch(const GatherJob *ja, const GatherJob *jb, BatchGrid bg, int f32, hipStream_t s) {
  if (bg.nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather2x2_batch, dim3(bg.nblocks), dim3(256), 0, s, ja, jb, bg, f32);
  return hipGetLastError();
}

// Tile-ordered stencil data: nearest grid indices a = floor(x/h + 1/2) (unwrapped)
// and the FP64 offsets x - a h, |offset| <= h/2 (also stored in FP32).
__global__ void k_anchors(int N, const int *__restrict__ tperm, const double *__restrict__ x, double h,
                          int2 *__restrict__ anchor, double2 *__restrict__ off64, float2 *__restrict__ off32) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int i = tperm[k];
  const double px = x[2 * i], py = x[2 * i + 1];
  const int ax = (int)floor(px / h + 0.5), ay = (int)floor(py / h + 0.5);
  anchor[k] = make_int2(ax, ay);
  const double ox = px - ax * h, oy = py - ay * h;
  off64[k] = make_double2(ox, oy);
  if (off32) off32[k] = make_float2((float)ox, (float)oy);
}

hipError_t launch_anchors(int N, const int *tperm, const double *x, double h, int *anchor, double *off64,
                          float *off32, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_anchors, dim3((N + 255) / 256), dim3(256), 0, s, N, tperm, x, h, (int2 *)anchor,
                     (double2 *)off64, (float2 *)off32);
  return hipGetLastError();
}

// Cell-ordered coordinates relative to the lower-left corner of the node's cell;
// thread N writes the zero record after the sources of the packed record arrays
// (the source of every empty neighbour-list slot): position (-1.5, -1.5) cells,
// 1.5 to 2.5 cells from any target of the cell frame, density 0.
__global__ void k_cell_local(int N, const int *__restrict__ cperm, const int *__restrict__ key,
                             const double *__restrict__ x, int nb, double cell, double2 *__restrict__ loc64,
                             double2 *__restrict__ src64, float4 *__restrict__ src32, int *__restrict__ tcell) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == N) {
    src64[2 * N] = make_double2(-1.5 * cell, -1.5 * cell);
    src64[2 * N + 1] = make_double2(0.0, 0.0);
    if (src32) src32[N] = make_float4((float)(-1.5 * cell), (float)(-1.5 * cell), 0.0f, 0.0f);
  }
  if (k >= N) return;
  const int i = cperm[k];
  const int c = key[i];
  const double lx = x[2 * i] - (c % nb) * cell, ly = x[2 * i + 1] - (c / nb) * cell;
  tcell[k] = c;
  loc64[k] = make_double2(lx, ly);
  src64[2 * k] = make_double2(lx, ly);
  if (src32) {
    float4 r = src32[k];
    r.x = (float)lx;
    r.y = (float)ly;
    src32[k] = r;
  }
}

hipError_t launch_cell_local(int N, const int *cperm, const int *key, const double *x, int nb, double cell,
                             double *loc64, double *src64, float *src32, int *tcell, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_local, dim3((N + 256) / 256), dim3(256), 0, s, N, cperm, key, x, nb, cell,
                     (double2 *)loc64, (double2 *)src64, (float4 *)src32, tcell);
  return hipGetLastError();
}

__global__ void k_gather_src(int N, const int *__restrict__ perm, const double2 *__restrict__ mu,
                             double2 *__restrict__ src64, float2 *__restrict__ src32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double2 v = mu[perm[i]];
  if (src32)
    src32[2 * i + 1] = make_float2((float)v.x, (float)v.y);
  else
    src64[2 * i + 1] = v;
}

hipError_t launch_gather_src(int N, const int *perm, const double *mu, double *src64, float *src32, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_src, dim3((N + 255) / 256), dim3(256), 0, s, N, perm, (const double2 *)mu,
                     (double2 *)src64, (float2 *)src32);
  return hipGetLastError();
}

// one thread per node: scan the 3x3 neighbouring cells for nodes of other bodies
__global__ void k_overlap(int N, const int *__restrict__ cell_start, const int *__restrict__ perm,
                          const double *__restrict__ xa, const int *__restrict__ body, int nb, double L,
                          double thresh2, int *__restrict__ flag) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double x = xa[2 * perm[p]], y = xa[2 * perm[p] + 1];
  const int bi = body[perm[p]];
  const double inv = nb / L;
  const int cx = min(max((int)floor(x * inv), 0), nb - 1), cy = min(max((int)floor(y * inv), 0), nb - 1);
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int c = ((cy + dy + nb) % nb) * nb + (cx + dx + nb) % nb;
      for (int k = cell_start[c]; k < cell_start[c + 1]; ++k) {
        if (body[perm[k]] == bi) continue;
        double ex = x - xa[2 * perm[k]], ey = y - xa[2 * perm[k] + 1];
        ex -= L * rint(ex / L);
        ey -= L * rint(ey / L);
        if (ex * ex + ey * ey < thresh2) atomicOr(flag, 1);
      }
    }
}

hipError_t launch_overlap(int N, const int *cell_start, const int *perm, const double *xa, const int *body, int nb,
                          double L, double thresh, int *flag, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_overlap, dim3((N + 255) / 256), dim3(256), 0, s, N, cell_start, perm, xa, body, nb, L,
                     thresh * thresh, flag);
  return hipGetLastError();
}

}  // namespace fbim
