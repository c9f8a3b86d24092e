// C ABI of the FBIM library: context, geometry, the single-layer matvec
// pipeline, GMRES (mobility), Lanczos ((M^(r))^(1/2)), Brownian velocity and
// the EM-RFD step.  Host code driving the gfx950 kernels and rocFFT.
#include <mutex>

#include "ctx.h"

namespace fbim {

void resolve_timing(fbim_ctx *c) {
  if (c->pending.empty()) return;
  hipStreamSynchronize(c->stream);
  for (auto &kv : c->pending) {
    auto &a = c->acc[kv.first];
    for (auto &t : kv.second) {
      float ms = 0;
      hipEventElapsedTime(&ms, t.a, t.b);
      a.first += ms;
      a.second += 1;
      hipEventDestroy(t.a);
      hipEventDestroy(t.b);
    }
  }
  c->pending.clear();
}

fbim_status rebuild_shape_arrays(fbim_ctx *c) {
  std::vector<double *> ref, band, Mp, Pref, Nt, G, Gp;
  std::vector<int> bw, np;
  for (auto &s : c->shapes) {
    ref.push_back(s.ref);
    band.push_back(s.band);
    Mp.push_back(s.Mp);
    Pref.push_back(s.Pref);
    Nt.push_back(s.Nt);
    G.push_back(s.G);
    Gp.push_back(s.Gp);
    bw.push_back(s.h.band);
    np.push_back(s.h.n_p);
  }
  STCHK(upload(c, c->d_ref_arr, ref));
  STCHK(upload(c, c->d_band_arr, band));
  STCHK(upload(c, c->d_Mp_arr, Mp));
  STCHK(upload(c, c->d_Pref_arr, Pref));
  STCHK(upload(c, c->d_Nt_arr, Nt));
  STCHK(upload(c, c->d_G_arr, G));
  STCHK(upload(c, c->d_Gp_arr, Gp));
  STCHK(upload(c, c->d_band, bw));
  STCHK(upload(c, c->d_np, np));
  return FBIM_OK;
}

fbim_status setup_fft(fbim_ctx *c) {
  const size_t M = c->d.M;
  HIPCHK(c, dalloc(c->d_grid, 2 * M * M));
  HIPCHK(c, dalloc(c->d_spec, 2 * 2 * M * (M / 2 + 1)));
  if (c->mixed) {
    HIPCHK(c, dalloc(c->d_grid32, 2 * M * M));
    HIPCHK(c, dalloc(c->d_spec32, 2 * 2 * M * (M / 2 + 1)));
  }
  c->conv = wave_conv_supported(c->d.M) && !(c->p.flags & FBIM_FLAG_LIBRARY_FFT);
  if (c->conv) {
    // twiddles exp(-2 pi i k / M), evaluated in long double
    std::vector<double> tw(2 * M);
    for (size_t k = 0; k < M; ++k) {
      const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)M;
      tw[2 * k] = (double)cosl(a);
      tw[2 * k + 1] = (double)-sinl(a);
    }
    std::vector<float> tw32(tw.begin(), tw.end());
    STCHK(upload(c, c->d_tw, tw));
    STCHK(upload(c, c->d_tw32, tw32));
    std::vector<double> ey(M);
    for (size_t i = 0; i < M; ++i) {
      const double k = 2.0 * kPi / c->d.L * (i < M / 2 ? (double)i : (double)i - (double)M);
      ey[i] = std::exp(-(1.0 - c->d.eta_s) * k * k / (4.0 * c->d.xi * c->d.xi));
    }
    std::vector<float> ey32(ey.begin(), ey.end());
    STCHK(upload(c, c->d_ey, ey));
    STCHK(upload(c, c->d_ey32, ey32));
    return FBIM_OK;
  }
  if (!g_rocfft_ready) {
    FFTCHK(c, rocfft_setup());
    g_rocfft_ready = true;
  }
  const size_t len[2] = {(size_t)c->d.M, (size_t)c->d.M};
  FFTCHK(c, rocfft_plan_create(&c->fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                               rocfft_precision_double, 2, len, 2, nullptr));
  FFTCHK(c, rocfft_plan_create(&c->inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                               rocfft_precision_double, 2, len, 2, nullptr));
  size_t w1 = 0, w2 = 0, w3 = 0, w4 = 0;
  FFTCHK(c, rocfft_plan_get_work_buffer_size(c->fwd, &w1));
  FFTCHK(c, rocfft_plan_get_work_buffer_size(c->inv, &w2));
  if (c->mixed) {
    FFTCHK(c, rocfft_plan_create(&c->fwd32, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                                 rocfft_precision_single, 2, len, 2, nullptr));
    FFTCHK(c, rocfft_plan_create(&c->inv32, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                                 rocfft_precision_single, 2, len, 2, nullptr));
    FFTCHK(c, rocfft_plan_get_work_buffer_size(c->fwd32, &w3));
    FFTCHK(c, rocfft_plan_get_work_buffer_size(c->inv32, &w4));
  }
  c->fft_work_bytes = std::max(std::max(w1, w2), std::max(w3, w4));
  if (c->fft_work_bytes) HIPCHK(c, hipMalloc(&c->fft_work, c->fft_work_bytes));
  FFTCHK(c, rocfft_execution_info_create(&c->einfo));
  if (c->fft_work_bytes) FFTCHK(c, rocfft_execution_info_set_work_buffer(c->einfo, c->fft_work, c->fft_work_bytes));
  FFTCHK(c, rocfft_execution_info_set_stream(c->einfo, c->stream));
  return FBIM_OK;
}

fbim_status ensure_krylov(fbim_ctx *c) {
  const size_t ntot = 2 * (size_t)c->N + 3 * (size_t)c->n;
  const size_t cols = (size_t)std::max(c->restart, c->lanczos_max) + 1;
  if (ntot == c->ntot && c->capV == cols && c->kn == c->n) return FBIM_OK;
  c->kn = c->n;
  c->ntot = ntot;
  c->capV = cols;
  HIPCHK(c, dalloc(c->d_V, cols * ntot));
  HIPCHK(c, dalloc(c->d_w, ntot));
  HIPCHK(c, dalloc(c->d_t1, ntot));
  HIPCHK(c, dalloc(c->d_t2, ntot));
  HIPCHK(c, dalloc(c->d_b, ntot));
  HIPCHK(c, dalloc(c->d_x2, ntot));
  HIPCHK(c, dalloc(c->d_r, ntot));
  if (c->mixed) {
    HIPCHK(c, dalloc(c->d_irx, ntot));
    HIPCHK(c, dalloc(c->d_irr, ntot));
    HIPCHK(c, dalloc(c->d_ird, ntot));
  }
  // chunk tables (one system): saddle chunks first, then node chunks
  std::vector<int2> ch;
  auto cut = [&](size_t n) {
    for (size_t x = 0; x < n; x += kChunk) ch.push_back(make_int2((int)x, (int)std::min(n, x + kChunk)));
  };
  cut(ntot);
  const int nsad = (int)ch.size();
  cut(2 * (size_t)c->N);
  const int nnod = (int)ch.size() - nsad;
  STCHK(upload(c, c->d_chunks, ch));
  STCHK(upload(c, c->d_chunk_sys, std::vector<int>(ch.size(), 0)));
  STCHK(upload(c, c->d_sys_chunk, std::vector<int>{0, nsad, 0, nnod}));
  c->seg_sad = Segs{c->d_chunks, c->d_chunk_sys, c->d_sys_chunk, nsad, 1};
  c->seg_nod = Segs{c->d_chunks + nsad, c->d_chunk_sys + nsad, c->d_sys_chunk + 2, nnod, 1};
  HIPCHK(c, dalloc(c->d_partial, (size_t)std::max(nsad, 1) * (cols + 1)));
  HIPCHK(c, dalloc(c->d_h, cols));
  HIPCHK(c, dalloc(c->d_h2, cols));
  HIPCHK(c, dalloc(c->d_nrm, 4));
  HIPCHK(c, dalloc(c->d_lag, 3 * (size_t)kLagSlot));
  HIPCHK(c, pub_alloc(c->pub, std::max(cols + 1, (size_t)2 * kLagSlot)));
  HIPCHK(c, dalloc(c->d_c, cols));
  HIPCHK(c, dalloc(c->d_vec_a, 2 * (size_t)c->N));
  HIPCHK(c, dalloc(c->d_vec_b, 2 * (size_t)c->N));
  HIPCHK(c, dalloc(c->d_U3, 3 * (size_t)c->n));
  HIPCHK(c, dalloc(c->d_U4, 3 * (size_t)c->n));
  HIPCHK(c, dalloc(c->d_U5, 3 * (size_t)c->n));
  HIPCHK(c, dalloc(c->d_U6, 3 * (size_t)c->n));
  return FBIM_OK;
}

// tiles of same-shape bodies: kBodyMfmaCols per tile when every shape takes the
// matrix-core form, else up to body_tile_cap(2 n_p)
fbim_status build_body_tiles(fbim_ctx *c) {
  std::vector<int> list;
  std::vector<int4> tiles;
  size_t lds = 0;
  bool mfma = true;
  int n2max = 0;
  for (auto &sh : c->shapes) {
    mfma = mfma && body_mfma_ok(2 * sh.h.n_p);
    n2max = std::max(n2max, 2 * sh.h.n_p);
  }
  for (int sh = 0; sh < (int)c->shapes.size(); ++sh) {
    const int n2 = 2 * c->shapes[sh].h.n_p;
    const int per = mfma ? kBodyMfmaCols : body_tile_cap(n2);
    const int first = (int)list.size();
    for (int b = 0; b < c->n; ++b)
      if (c->h_shape[b] == sh) list.push_back(b);
    const int cnt = (int)list.size() - first;
    for (int t = 0; t < cnt; t += per) tiles.push_back(make_int4(sh, first + t, std::min(per, cnt - t), 0));
    if (cnt > 0) lds = std::max(lds, mfma ? body_mfma_lds(n2) : body_tile_lds(n2));
  }
  STCHK(upload(c, c->d_blist, list));
  STCHK(upload(c, c->d_btile, tiles));
  c->bt = BodyTiles{c->d_btile, c->d_blist, (int)tiles.size(), lds, mfma ? body_mfma_rb(n2max) : 0};
  return FBIM_OK;
}

// ------------------------------------------------------------------ learned preconditioner correction
constexpr int kNParam = FBIM_MLP_NPARAM;
constexpr int kOffW1 = 0, kOffB1 = kMlpIn * kMlpHid, kOffW2 = kOffB1 + kMlpHid, kOffB2 = kOffW2 + kMlpHid * kMlpHid,
              kOffW3 = kOffB2 + kMlpHid, kOffB3 = kOffW3 + kMlpHid * kMlpOut;
static_assert(kOffB3 + kMlpOut == kNParam, "weight layout");

double shapes_r_max(const fbim_ctx *c) {
  double r = 0.0;
  for (auto &sh : c->shapes)
    for (int j = 0; j < sh.h.n_p; ++j) r = std::max(r, std::hypot(sh.h.ref_xy[2 * j], sh.h.ref_xy[2 * j + 1]));
  return r;
}

fbim_status ensure_mlp(fbim_ctx *c, int n) {
  if (!c->d_mw) {
    HIPCHK(c, dalloc(c->d_mw, kNParam));
    HIPCHK(c, dalloc(c->d_am, kNParam));
    HIPCHK(c, dalloc(c->d_av, kNParam));
    HIPCHK(c, dalloc(c->d_g, kNParam));
    HIPCHK(c, dalloc(c->d_loss, 1));
  }
  if (n > c->mlp_cap) {
    HIPCHK(c, dalloc(c->d_X, (size_t)n * kMlpIn));
    HIPCHK(c, dalloc(c->d_H1, (size_t)n * kMlpHid));
    HIPCHK(c, dalloc(c->d_H2, (size_t)n * kMlpHid));
    HIPCHK(c, dalloc(c->d_Z1, (size_t)n * kMlpHid));
    HIPCHK(c, dalloc(c->d_Z2, (size_t)n * kMlpHid));
    HIPCHK(c, dalloc(c->d_Y, (size_t)n * kMlpOut));
    HIPCHK(c, dalloc(c->d_dY, (size_t)n * kMlpOut));
    HIPCHK(c, dalloc(c->d_dN, (size_t)n * kMlpOut));
    HIPCHK(c, dalloc(c->d_ones, (size_t)n));
    HIPCHK(c, launch_fill_f32((size_t)n, 1.0f, c->d_ones, c->stream));
    c->mlp_cap = n;
  }
  return FBIM_OK;
}

GemmArgs gemm(int M, int N, int K, const float *A, size_t sam, size_t sak, const float *B, size_t sbk, size_t sbn,
              float *C, size_t ldc, int epi, const float *bias = nullptr, const float *aux = nullptr) {
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = B;
  g.sbk = sbk;
  g.sbn = sbn;
  g.C = C;
  g.ldc = ldc;
  g.bias = bias;
  g.aux = aux;
  g.epi = epi;
  return g;
}

// Y = MLP(X) with the hidden activations in H1, H2 ([n][kMlpHid] each)
fbim_status mlp_forward_into(fbim_ctx *c, const float *X, int n, float *Y, float *H1, float *H2) {
  hipStream_t s = c->stream;
  const float *w = c->d_mw;
  HIPCHK(c, launch_gemm_bf16(gemm(n, kMlpHid, kMlpIn, X, kMlpIn, 1, w + kOffW1, kMlpHid, 1, H1, kMlpHid,
                                  kGemmBiasTanh, w + kOffB1), 1, s));
  HIPCHK(c, launch_gemm_bf16(gemm(n, kMlpHid, kMlpHid, H1, kMlpHid, 1, w + kOffW2, kMlpHid, 1, H2, kMlpHid,
                                  kGemmBiasTanh, w + kOffB2), 1, s));
  HIPCHK(c, launch_gemm_bf16(gemm(n, kMlpOut, kMlpHid, H2, kMlpHid, 1, w + kOffW3, kMlpOut, 1, Y, kMlpOut,
                                  kGemmBias, w + kOffB3), 1, s));
  return FBIM_OK;
}

// Y = MLP(X); hidden activations kept in d_H1, d_H2 (the backward pass reads them)
fbim_status mlp_forward(fbim_ctx *c, const float *X, int n, float *Y) {
  Timer t(c, "mlp");
  return mlp_forward_into(c, X, n, Y, c->d_H1, c->d_H2);
}

// ------------------------------------------------------------------ no-allocation scratch
// Device scratch of fbim_mlp_forward_noalloc: the two hidden activation
// arrays of up to FBIM_NOALLOC_MAX_BODIES bodies, one copy per GPU for the
// life of the process.  Host code never uses the array's name as an address:
// its device address is looked up once per device (hipGetSymbolAddress, at
// fbim_create on that device) and kept in g_noalloc_ptr.
constexpr size_t kNoAllocFloats = 2 * (size_t)kMlpHid * FBIM_NOALLOC_MAX_BODIES;
__device__ __align__(256) float noalloc_scratch[kNoAllocFloats];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
float *g_noalloc_ptr[kMaxDevices] = {};

fbim_status resolve_noalloc_scratch(fbim_ctx *c) {
  if (c->device < 0 || c->device >= kMaxDevices) return fail(c, FBIM_ENOTSUP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  if (!g_noalloc_ptr[c->device]) {
    void *ptr = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)));
    g_noalloc_ptr[c->device] = static_cast<float *>(ptr);
  }
  c->noalloc_scratch = g_noalloc_ptr[c->device];
  return FBIM_OK;
}

// grad = d(sum dY . Y)/dw at X (recomputes the forward activations)
fbim_status mlp_backward(fbim_ctx *c, const float *X, const float *dY, int n, float *grad) {
  STCHK(mlp_forward(c, X, n, c->d_Y));
  Timer t(c, "mlp");
  hipStream_t s = c->stream;
  const float *w = c->d_mw;
  const int ks = std::max(1, std::min(64, n / 256));  // split of the sums over bodies
  HIPCHK(c, launch_fill_f32(kNParam, 0.0f, grad, s));
  // layer 3
  HIPCHK(c, launch_gemm_bf16(gemm(kMlpHid, kMlpOut, n, c->d_H2, 1, kMlpHid, dY, kMlpOut, 1, grad + kOffW3, kMlpOut,
                                  kGemmAtomic), ks, s));
  HIPCHK(c, launch_gemm_bf16(gemm(1, kMlpOut, n, c->d_ones, 0, 1, dY, kMlpOut, 1, grad + kOffB3, kMlpOut,
                                  kGemmAtomic), ks, s));
  HIPCHK(c, launch_gemm_bf16(gemm(n, kMlpHid, kMlpOut, dY, kMlpOut, 1, w + kOffW3, 1, kMlpOut, c->d_Z2, kMlpHid,
                                  kGemmTanhGrad, nullptr, c->d_H2), 1, s));
  // layer 2
  HIPCHK(c, launch_gemm_bf16(gemm(kMlpHid, kMlpHid, n, c->d_H1, 1, kMlpHid, c->d_Z2, kMlpHid, 1, grad + kOffW2,
                                  kMlpHid, kGemmAtomic), ks, s));
  HIPCHK(c, launch_gemm_bf16(gemm(1, kMlpHid, n, c->d_ones, 0, 1, c->d_Z2, kMlpHid, 1, grad + kOffB2, kMlpHid,
                                  kGemmAtomic), ks, s));
  HIPCHK(c, launch_gemm_bf16(gemm(n, kMlpHid, kMlpHid, c->d_Z2, kMlpHid, 1, w + kOffW2, 1, kMlpHid, c->d_Z1, kMlpHid,
                                  kGemmTanhGrad, nullptr, c->d_H1), 1, s));
  // layer 1
  HIPCHK(c, launch_gemm_bf16(gemm(kMlpIn, kMlpHid, n, X, 1, kMlpIn, c->d_Z1, kMlpHid, 1, grad + kOffW1, kMlpHid,
                                  kGemmAtomic), ks, s));
  HIPCHK(c, launch_gemm_bf16(gemm(1, kMlpHid, n, c->d_ones, 0, 1, c->d_Z1, kMlpHid, 1, grad + kOffB1, kMlpHid,
                                  kGemmAtomic), ks, s));
  return FBIM_OK;
}

fbim_status mlp_features(fbim_ctx *c, float *X) {
  const double r_max = shapes_r_max(c);
  MlpCells cells;
  cells.nbc = mlp_body_cells(c->d.L, r_max);
  const size_t nc = (size_t)cells.nbc * cells.nbc;
  if (c->n > c->bc_cap_n) {
    HIPCHK(c, dalloc(c->d_bc_key, (size_t)c->n));
    HIPCHK(c, dalloc(c->d_bc_perm, (size_t)c->n));
    c->bc_cap_n = c->n;
  }
  if (nc + 1 > c->bc_cap_c) {
    HIPCHK(c, dalloc(c->d_bc_count, nc + 1));
    HIPCHK(c, dalloc(c->d_bc_cursor, nc + 1));
    HIPCHK(c, dalloc(c->d_bc_start, nc + 2));
    c->bc_cap_c = nc + 1;
  }
  cells.key = c->d_bc_key;
  cells.perm = c->d_bc_perm;
  cells.count = c->d_bc_count;
  cells.cursor = c->d_bc_cursor;
  cells.start = c->d_bc_start;
  cells.maxcount = c->d_bc_start + nc + 1;
  Timer t(c, "mlp");
  HIPCHK(c, launch_mlp_features(c->n, c->d_q, c->d_theta, c->d.L, r_max, c->mlp_sym, cells, X, c->stream));
  return FBIM_OK;
}

// d_dN for the current bodies (called whenever the bodies change while in use)
fbim_status mlp_refresh(fbim_ctx *c) {
  STCHK(ensure_mlp(c, c->n));
  STCHK(mlp_features(c, c->d_X));
  STCHK(mlp_forward(c, c->d_X, c->n, c->d_Y));
  HIPCHK(c, launch_mlp_correction(c->n, c->d_shape, c->d_Nt_arr, c->d_Y, c->d_dN, c->stream));
  return FBIM_OK;
}

// ------------------------------------------------------------------ geometry
// geometry of the configuration in d_q, d_theta
fbim_status build_geometry_dev(fbim_ctx *c) {
  const int N = c->N;
  hipStream_t s = c->stream;
  HIPCHK(c, launch_nodes(c->geom(), c->d.L, c->d_x, s));
  // cell list
  HIPCHK(c, hipMemsetAsync(c->d_ccount, 0, c->ncell * sizeof(int), s));
  HIPCHK(c, hipMemsetAsync(c->d_ccursor, 0, c->ncell * sizeof(int), s));
  HIPCHK(c, launch_cell_keys(N, c->d_x, c->d.L, c->d.n_box, c->d_ckey, c->d_ccount, s));
  HIPCHK(c, launch_scan(c->ncell, c->d_ccount, c->d_cstart, c->d_scal_int, s));
  HIPCHK(c, launch_scatter(N, c->d_ckey, c->d_cstart, c->d_ccursor, c->d_cperm, s));
  HIPCHK(c, launch_sort_bins(c->ncell, c->d_cstart, c->d_cperm, s));
  HIPCHK(c, launch_cell_local(N, c->d_cperm, c->d_ckey, c->d_x, c->d.n_box, c->d.L / c->d.n_box, c->d_xs,
                              c->d_src64, c->mixed ? c->d_src32 : nullptr, c->d_tcell, s));
  // tiles
  HIPCHK(c, hipMemsetAsync(c->d_tcount, 0, c->ntile * sizeof(int), s));
  HIPCHK(c, hipMemsetAsync(c->d_tcursor, 0, c->ntile * sizeof(int), s));
  HIPCHK(c, launch_tile_keys(N, c->d_x, c->d.h, c->d.M, c->d.tile, c->d_tkey, c->d_tcount, s));
  HIPCHK(c, launch_scan(c->ntile, c->d_tcount, c->d_tstart, c->d_scal_int + 2, s));
  HIPCHK(c, launch_scatter(N, c->d_tkey, c->d_tstart, c->d_tcursor, c->d_tperm, s));
  HIPCHK(c, launch_sort_bins(c->ntile, c->d_tstart, c->d_tperm, s));
  HIPCHK(c, launch_anchors(N, c->d_tperm, c->d_x, c->d.h, c->d_anchor, c->d_xt, c->mixed ? c->d_xt32 : nullptr, s));
  // overlap check: nodes of distinct bodies closer than 5% of the smallest node spacing
  double spacing = 1e300;
  for (auto &sh : c->shapes) {
    for (int j = 0; j < sh.h.n_p; ++j) {
      const int k = (j + 1) % sh.h.n_p;
      const double dx = sh.h.ref_xy[2 * j] - sh.h.ref_xy[2 * k], dy = sh.h.ref_xy[2 * j + 1] - sh.h.ref_xy[2 * k + 1];
      spacing = std::min(spacing, std::sqrt(dx * dx + dy * dy));
    }
  }
  // the count pass of the neighbour lists sees every pair within r_c, so it takes
  // the check when the threshold is below r_c; otherwise a pass of its own does
  const double thresh = 0.05 * spacing;
  const bool fused = thresh < c->d.r_c;
  HIPCHK(c, hipMemsetAsync(c->d_scal_int + 1, 0, sizeof(int), s));
  if (!fused)
    HIPCHK(c, launch_overlap(N, c->d_cstart, c->d_cperm, c->d_x, c->d_body, c->d.n_box, c->d.L, thresh,
                             c->d_scal_int + 1, s));
  int *hv = c->h_pin;  // pinned: no staging copy
  HIPCHK(c, hipMemcpyAsync(hv, c->d_scal_int, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->max_cell = hv[0];
  c->max_tile = hv[2];
  const char *overlap_msg = "nodes of distinct bodies closer than 5% of the node spacing";
  if (hv[1]) return fail(c, FBIM_EOVERLAP, overlap_msg);
  if (c->max_cell > kEllMaxCell)
    return fail(c, FBIM_EINVAL, "more than 4096 nodes in one cutoff cell (raise n_box)");
  // neighbour lists of the real-space sum (count, group rows, offsets, fill) and
  // spreading lists of the tiles (count, offsets, fill); one read of both totals
  PairArgs pa = c->pair_args();
  PairLists pl = c->lists();
  HIPCHK(c, launch_pair_lists(pa, pl, c->d_xs, 0, s, c->d_body, thresh * thresh, fused ? c->d_scal_int + 1 : nullptr));
  HIPCHK(c, launch_group_rows(pl, c->d_gsize, s));
  HIPCHK(c, launch_scan(c->ngroups, c->d_gsize, c->d_goff, c->d_scal_int + 3, s));
  HIPCHK(c, launch_spread_lists(c->wave(), c->d_scount, nullptr, nullptr, 0, s));
  HIPCHK(c, launch_scan(c->ntile, c->d_scount, c->d_sstart, c->d_scal_int + 4, s));
  int *pin = c->h_pin + 4;  // pinned: [0] pair slots, [1] spreading entries, [2] overlap flag, [3] longest group
  HIPCHK(c, hipMemcpyAsync(pin + 0, c->d_goff + c->ngroups, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(pin + 3, c->d_scal_int + 3, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(pin + 1, c->d_sstart + c->ntile, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(pin + 2, c->d_scal_int + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const int total[2] = {pin[0], pin[1]}, olap = pin[2], maxslots = pin[3];
  if (olap) return fail(c, FBIM_EOVERLAP, overlap_msg);
  if ((size_t)total[0] + kEllSlack > c->ell_cap) {
    const size_t cap = (size_t)total[0] + total[0] / 4 + kEllSlack;
    HIPCHK(c, dalloc(c->d_ell, cap));
    c->ell_cap = cap;
    pl.ell = c->d_ell;
  }
  const int stage = pair_lists_stage_rows(maxslots / 64);
  // empty slots (16-bit, two per fill word; total is a multiple of 64)
  const int empty2 = (int)((unsigned)kEllEmpty | ((unsigned)kEllEmpty << 16));
  HIPCHK(c, launch_fill_int((stage ? (size_t)kEllSlack : (size_t)total[0] + kEllSlack) / 2, empty2,
                            reinterpret_cast<int *>(c->d_ell + (stage ? total[0] : 0)), s));
  HIPCHK(c, launch_pair_lists(pa, pl, c->d_xs, 1, s, nullptr, 0.0, nullptr, stage));
  if ((size_t)total[1] > c->slist_cap) {
    const size_t cap = (size_t)total[1] + total[1] / 4 + 64;
    HIPCHK(c, dalloc(c->d_slist, cap));
    c->slist_cap = cap;
  }
  HIPCHK(c, launch_spread_lists(c->wave(), nullptr, c->d_sstart, c->d_slist, 1, s));
  ++c->geom_serial;
  if (c->mlp_on) STCHK(mlp_refresh(c));
  return FBIM_OK;
}

// geometry of the caller's configuration h_q, h_theta (uploaded through pinned staging)
fbim_status build_geometry(fbim_ctx *c) {
  const size_t n = c->n;
  hipStream_t s = c->stream;
  HIPCHK(c, hipStreamSynchronize(s));  // the staging buffer may still feed an earlier upload
  std::memcpy(c->h_qpin, c->h_q.data(), 2 * n * sizeof(double));
  std::memcpy(c->h_qpin + 2 * n, c->h_theta.data(), n * sizeof(double));
  HIPCHK(c, hipMemcpyAsync(c->d_q, c->h_qpin, 2 * n * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_theta, c->h_qpin + 2 * n, n * sizeof(double), hipMemcpyHostToDevice, s));
  return build_geometry_dev(c);
}

fbim_status move_bodies(fbim_ctx *c, const double *q_src, const double *th_src, const double *dQ, double a) {
  const size_t n = c->n;
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(c->d_qprev, c->d_q, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_thprev, c->d_theta, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, launch_move_bodies((int)n, q_src, th_src, dQ, a, c->d_q, c->d_theta, s));
  const fbim_status st = build_geometry_dev(c);
  if (st != FBIM_OK) {
    const std::string msg = c->err;
    fbim_status st2 = FBIM_OK;
    if (hipMemcpyAsync(c->d_q, c->d_qprev, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->d_theta, c->d_thprev, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      st2 = FBIM_EDEVICE;
    if (st2 != FBIM_OK || build_geometry_dev(c) != FBIM_OK) c->have_bodies = false;
    c->err = msg;
  }
  return st;
}

// ------------------------------------------------------------------ matvec
fbim_status apply_M(fbim_ctx *c, const double *mu, double *out, unsigned parts) {
  hipStream_t s = c->stream;
  const int N = c->N;
  if (!c->have_bodies) return fail(c, FBIM_EINVAL, "no bodies set");
  const bool f32 = c->mixed && c->cur32;
  if (parts & FBIM_PART_REAL) {
    const PairArgs a = c->pair_args();
    const PairLists pl = c->lists();
    if (f32) {
      HIPCHK(c, launch_gather_src(N, c->d_cperm, mu, nullptr, c->d_src32, s));
      Timer t(c, "pair32");
      HIPCHK(c, launch_pair_f32(pl, a, c->d_src32, out, s));
    } else {
      HIPCHK(c, launch_gather_src(N, c->d_cperm, mu, c->d_src64, nullptr, s));
      Timer t(c, "pair");
      HIPCHK(c, launch_pair_f64(pl, a, c->d_src64, out, s));
    }
  } else {
    HIPCHK(c, launch_fill(2 * (size_t)N, 0.0, out, s));
  }
  if (parts & FBIM_PART_ALPERT) {
    Timer t(c, "alpert");
    HIPCHK(c, launch_alpert(c->geom(), c->d_band_arr, c->d_band, mu, out, 1, s));
  }
  if (parts & FBIM_PART_WAVE) {
    const WaveArgs w = c->wave();
    const double scale = c->d.h * c->d.h / (c->p.eta * c->d.L * c->d.L);
    if (f32) {
      HIPCHK(c, launch_gather2f(N, c->d_tperm, mu, c->d_mut32, s));
      {
        Timer t(c, "spread32");
        HIPCHK(c, launch_spread_f32(w, c->d_xt32, c->d_mut32, c->d_grid32, s));
      }
      if (c->conv) {
        Timer t(c, "fft32");
        HIPCHK(c, launch_wave_conv_f32(WaveConvArgs{c->d.M, 0, c->d.L, c->d.xi, c->d.eta_s, scale}, c->d_grid32,
                                       c->d_spec32, c->d_tw32, c->d_ey32, s));
      } else {
        {
          Timer t(c, "fft32");
          void *in[1] = {c->d_grid32}, *o[1] = {c->d_spec32};
          FFTCHK(c, rocfft_execute(c->fwd32, in, o, c->einfo));
        }
        {
          Timer t(c, "multiplier32");
          HIPCHK(c, launch_multiplier_f32(c->d.M, c->d.L, c->d.xi, c->d.eta_s, scale, 0, c->d_spec32, s));
        }
        Timer t(c, "fft32");
        void *in[1] = {c->d_spec32}, *o[1] = {c->d_grid32};
        FFTCHK(c, rocfft_execute(c->inv32, in, o, c->einfo));
      }
      Timer t(c, "interp32");
      HIPCHK(c, launch_interp_f32(w, c->d_xt32, c->d_tperm, c->d_grid32, out, s));
    } else {
      HIPCHK(c, launch_gather2(N, c->d_tperm, mu, c->d_mut, s));
      {
        Timer t(c, "spread");
        HIPCHK(c, launch_spread_f64(w, c->d_xt, c->d_mut, c->d_grid, s));
      }
      if (c->conv) {
        Timer t(c, "fft");
        HIPCHK(c, launch_wave_conv_f64(WaveConvArgs{c->d.M, 0, c->d.L, c->d.xi, c->d.eta_s, scale}, c->d_grid,
                                       c->d_spec, c->d_tw, c->d_ey, s));
      } else {
        {
          Timer t(c, "fft");
          void *in[1] = {c->d_grid}, *o[1] = {c->d_spec};
          FFTCHK(c, rocfft_execute(c->fwd, in, o, c->einfo));
        }
        {
          Timer t(c, "multiplier");
          HIPCHK(c, launch_multiplier_f64(c->d.M, c->d.L, c->d.xi, c->d.eta_s, scale, 0, c->d_spec, s));
        }
        Timer t(c, "fft");
        void *in[1] = {c->d_spec}, *o[1] = {c->d_grid};
        FFTCHK(c, rocfft_execute(c->inv, in, o, c->einfo));
      }
      Timer t(c, "interp");
      HIPCHK(c, launch_interp_f64(w, c->d_xt, c->d_tperm, c->d_grid, out, s));
    }
  }
  return FBIM_OK;
}

fbim_status random_field(fbim_ctx *c, const double *W_grid, double *out) {
  hipStream_t s = c->stream;
  const size_t M = c->d.M;
  const WaveArgs w = c->wave();
  const double scale = 1.0 / ((double)M * std::sqrt(c->p.eta * c->d.L * c->d.L));
  HIPCHK(c, launch_fill(2 * (size_t)c->N, 0.0, out, s));
  HIPCHK(c, hipMemcpyAsync(c->d_grid, W_grid, 2 * M * M * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (c->conv) {
    Timer t(c, "fft");
    HIPCHK(c, launch_wave_conv_f64(WaveConvArgs{c->d.M, 1, c->d.L, c->d.xi, c->d.eta_s, scale}, c->d_grid, c->d_spec,
                                   c->d_tw, c->d_ey, s));
  } else {
    {
      Timer t(c, "fft");
      void *in[1] = {c->d_grid}, *o[1] = {c->d_spec};
      FFTCHK(c, rocfft_execute(c->fwd, in, o, c->einfo));
    }
    {
      Timer t(c, "multiplier");
      HIPCHK(c, launch_multiplier_f64(c->d.M, c->d.L, c->d.xi, c->d.eta_s, scale, 1, c->d_spec, s));
    }
    Timer t(c, "fft");
    void *in[1] = {c->d_spec}, *o[1] = {c->d_grid};
    FFTCHK(c, rocfft_execute(c->inv, in, o, c->einfo));
  }
  Timer t(c, "interp");
  HIPCHK(c, launch_interp_f64(w, c->d_xt, c->d_tperm, c->d_grid, out, s));
  return FBIM_OK;
}

// saddle operator of eq. 3.8: y = [M mu - K U; -K^T mu]
fbim_status apply_saddle(fbim_ctx *c, const double *x, double *y) {
  if (c->op == 1) return apply_second_kind(c, x, y);
  const size_t twoN = 2 * (size_t)c->N;
  STCHK(apply_M(c, x, y, FBIM_PART_ALL));
  HIPCHK(c, launch_sub_KU(c->geom(), x + twoN, y, c->stream));
  HIPCHK(c, launch_KT(c->geom(), x, -1.0, y + twoN, c->stream));
  return FBIM_OK;
}

fbim_status apply_precond(fbim_ctx *c, const double *z, double *y) {
  if (c->op == 1) {  // the second-kind system runs unpreconditioned
    HIPCHK(c, hipMemcpyAsync(y, z, c->ntot * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return FBIM_OK;
  }
  Timer t(c, "precond");
  HIPCHK(c, launch_precond(c->geom(), c->mats(), c->bt, c->mlp_on ? c->d_dN : nullptr, z, y, c->stream));
  return FBIM_OK;
}

const Segs &segs_for(const fbim_ctx *c, size_t n) { return n == c->ntot ? c->seg_sad : c->seg_nod; }

// one Gram-Schmidt pass (launch_orth) over vectors of length n
fbim_status orth_pass(fbim_ctx *c, int mode, size_t n, const double *V, int k, double *w, const double *h,
                      const double *cond, double *out) {
  Timer t(c, "blas");
  OrthArgs a;
  a.seg = segs_for(c, n);
  a.V = V;
  a.ld = c->ntot;
  a.k = k;
  a.w = w;
  a.h = h;
  a.hstride = (int)c->capV + 1;
  a.cond = cond;
  a.partial = c->d_partial;
  a.out = out;
  a.ostride = (int)c->capV + 1;
  HIPCHK(c, launch_orth(mode, a, c->stream));
  return FBIM_OK;
}

// Classical Gram-Schmidt of w against the k columns of V, twice (CGS2), or with
// the second pass only when the first one cancels more than half of ||w||^2
// (Daniel-Gragg-Kaufman-Stewart criterion, FBIM_FLAG_SELECTIVE_REORTH).  For
// k <= kOrthFused the first subtraction and the second projection share one
// read of V.  The decision is taken on the device, which also writes the
// combined coefficients and ||w|| to host memory, so the host waits once per
// call and copies nothing.  On return h[0..k) holds the projection
// coefficients and hn = ||w|| after orthogonalisation; with `normalise`, w has
// been scaled by 1 / hn (by 0 when hn = 0).
fbim_status orthogonalise(fbim_ctx *c, const double *V, int k, double *w, size_t n, double *h, double &hn,
                          bool normalise = false) {
  hipStream_t s = c->stream;
  double *flag = c->d_nrm + 1, *nrm2 = c->d_nrm + 2;
  const bool selective = (c->p.flags & FBIM_FLAG_SELECTIVE_REORTH) != 0;
  const bool fused = k <= kOrthFused;
  STCHK(orth_pass(c, 0, n, V, k, w, nullptr, nullptr, c->d_h));  // h, h[k] = ||w||^2
  if (fused) {
    STCHK(orth_pass(c, 1, n, V, k, w, c->d_h, nullptr, c->d_h2));  // w1 = w - V h; h2 = V^T w1, h2[k] = ||w1||^2
    if (selective) HIPCHK(c, launch_need_second_pass(1, c->d_h2 + k, 0, c->d_h + k, 0, flag, s));
    STCHK(orth_pass(c, 2, n, V, k, w, c->d_h2, selective ? flag : nullptr, nrm2));  // w2 = w1 - V h2
  } else {
    STCHK(orth_pass(c, 2, n, V, k, w, c->d_h, nullptr, c->d_nrm));  // w1, ||w1||^2
    if (selective) HIPCHK(c, launch_need_second_pass(1, c->d_nrm, 0, c->d_h + k, 0, flag, s));
    STCHK(orth_pass(c, 0, n, V, k, w, nullptr, selective ? flag : nullptr, c->d_h2));
    STCHK(orth_pass(c, 2, n, V, k, w, c->d_h2, selective ? flag : nullptr, nrm2));
  }
  OrthPublish o;
  o.k = k;
  o.fused = fused;
  o.selective = selective;
  o.h = c->d_h;
  o.h2 = c->d_h2;
  o.nrm_a = c->d_nrm;
  o.nrm_b = nrm2;
  o.flag = flag;
  o.a = c->d_nrm + 3;  // 1 / ||w||
  const unsigned long long tag = ++c->pub.seq;
  HIPCHK(c, launch_orth_publish(o, c->pub, tag, s));
  if (normalise) {
    Timer t(c, "blas");
    HIPCHK(c, launch_scale_dev(n, c->d_nrm + 3, w, s));
  }
  HIPCHK(c, pub_wait(c->pub, tag, s));
  std::memcpy(h, c->pub.v, k * sizeof(double));
  hn = c->pub.v[k];
  return FBIM_OK;
}

// Host half of a lagged Arnoldi step (the relations are given with arnoldi_lagged):
// dots = V_{<=j}^T w (and w . w) and out = (V_{<=j}^T w', w' . w') as published, where
// slot j holds nu u_j and w = nu A u_j; s is the lag of u_j.  Writes the unrotated
// column j into col[0..j+1] and replaces s and nu by the lag and norm of w' = |w'|
// u_{j+1} (left unnormalised in slot j + 1); false if a value is not finite.  s, rho,
// t and e are computed as the lagged pass computes them on the device.
bool lagged_column(int j, const double *dots, const double *out, const std::vector<double> &Hu, int m,
                   std::vector<double> &s, double &nu, double *col) {
  const double inu = nu > 0.0 ? 1.0 / nu : 0.0;
  std::vector<double> t(j);
  double ss = 0.0, stt = 0.0;
  for (int i = 0; i < j; ++i) {
    t[i] = dots[i] * inu;
    ss += s[i] * s[i];
    stt += s[i] * t[i];
  }
  const double rho = std::sqrt(std::max(1.0 - ss, 0.0)), irho = rho > 0.0 ? 1.0 / rho : 0.0;
  const double e_j = (dots[j] * inu * inu - stt) * irho;
  const double nw = std::sqrt(std::max(out[j + 1], 0.0)), inw = nw > 0.0 ? 1.0 / nw : 0.0;
  std::vector<double> sn(j + 1);
  double sn2 = 0.0;
  for (int i = 0; i <= j; ++i) {
    sn[i] = out[i] * inw;
    sn2 += sn[i] * sn[i];
  }
  for (int i = 0; i <= j; ++i) {
    double hs = 0.0;  // (H_{<j} s)_i
    for (int l = 0; l < j; ++l) hs += Hu[(size_t)i * m + l] * s[l];
    col[i] = ((i < j ? t[i] : e_j) - hs) * irho + nw * sn[i];
  }
  col[j + 1] = nw * std::sqrt(std::max(1.0 - sn2, 0.0));
  s = std::move(sn);
  nu = nw;
  for (int i = 0; i <= j + 1; ++i)
    if (!std::isfinite(col[i])) return false;
  return std::isfinite(dots[j + 1]);
}

// One Arnoldi step with delayed reorthogonalisation (FBIM_FLAG_LAGGED_REORTH).
// On entry slot j of V holds nu u_j, u_j of unit norm and orthogonal to V_0..V_{j-1}
// but for s = V_{<j}^T u_j (host, from the previous step; empty, and nu = 1, for
// j = 0), and w = nu A u_j (the operator was applied to the slot as it stands).  A
// dot-product pass gives V_{<=j}^T w and ||w||^2; the lagged pass turns the slot into
// the final V_j = (u_j - V_{<j} s) / rho (rho = sqrt(1 - s.s)), projects w out of
// V_{<=j} and returns its dot products with V_{<=j} and its norm; w is left
// unnormalised (its norm is the next step's nu).  With t = V_{<j}^T A u_j and
// e = (t, (u_j . A u_j - s.t) / rho) = V_{<=j}^T A u_j, the step's Arnoldi column
// follows without touching the vectors again (w below is A u_j):
//   A V_j = (w - A V_{<j} s) / rho,   A V_{<j} = V H_{<j}   (columns 0..j-1 final)
//   h = (e - H s) / rho,  w' = (w - V_{<=j} e) / rho = |w'| u_{j+1}
//   u_{j+1} = rho' V_{j+1} + V_{<=j} s'  =>  col[0..j] = h + |w'| s',  col[j+1] = |w'| rho'
// Hu holds the unrotated Arnoldi columns (row i of column l at Hu[i * m + l]);
// col[0..j+1] is column j on return, s is replaced by s' and nu by |w'|.
fbim_status arnoldi_lagged(fbim_ctx *c, int j, double *w, size_t n, const std::vector<double> &Hu, int m,
                           std::vector<double> &s, double &nu, double *col) {
  hipStream_t st = c->stream;
  double *dots = c->d_lag, *cur = c->d_lag + kLagSlot * (1 + (j & 1)), *prev = c->d_lag + kLagSlot * (1 + (~j & 1));
  STCHK(orth_pass(c, 0, n, c->d_V, j + 1, w, nullptr, nullptr, dots));  // t, u_j . w, ||w||^2
  {
    Timer t(c, "blas");
    OrthArgs a{};
    a.seg = segs_for(c, n);
    a.cond = nullptr;
    a.V = c->d_V;
    a.ld = c->ntot;
    a.k = j;
    a.w = w;
    a.h = dots;
    a.hstride = 0;
    a.partial = c->d_partial;
    a.out = cur;
    a.ostride = 0;
    a.lag = j > 0 ? prev : nullptr;
    a.lagstride = 0;
    HIPCHK(c, launch_orth_lag(a, st));
  }
  const unsigned long long tag = ++c->pub.seq;
  HIPCHK(c, launch_publish2(1, j + 2, dots, 0, j + 2, cur, 0, c->pub, tag, st));
  HIPCHK(c, pub_wait(c->pub, tag, st));
  if (!lagged_column(j, c->pub.v, c->pub.v + j + 2, Hu, m, s, nu, col))
    return fail(c, FBIM_EDEVICE, "non-finite Krylov vector");
  return FBIM_OK;
}

fbim_status norm2(fbim_ctx *c, const double *x, size_t n, double &out) {
  STCHK(orth_pass(c, 0, n, x, 0, const_cast<double *>(x), nullptr, nullptr, c->d_nrm));
  const unsigned long long tag = ++c->pub.seq;
  HIPCHK(c, launch_publish(1, c->d_nrm, 1, c->pub, tag, c->stream));
  HIPCHK(c, pub_wait(c->pub, tag, c->stream));
  out = std::sqrt(std::max(c->pub.v[0], 0.0));
  return FBIM_OK;
}

constexpr double kRelax = 1e-1;  // relaxed-matvec threshold of mixed contexts

// right-preconditioned restarted GMRES for the saddle system; b, x device (ntot)
// warm: start from the x given (else x0 = 0)
// relax > 0 (mixed contexts): inexact Krylov with a relaxed matvec -- an
// iteration uses the FP32 operator once the residual estimate is below
// relax ||b|| (the matvec error may grow as the residual falls, Bouras and
// Fraysse; Simoncini and Szyld), the FP64 operator before; restart residuals,
// and with them the stopping test, are always FP64.
fbim_status gmres(fbim_ctx *c, const double *b, double *x, double tol, int &iters, double &relres, int maxit,
                  bool warm = false, double relax = 0.0) {
  const size_t nt = c->ntot;
  hipStream_t s = c->stream;
  const bool lagged = (c->p.flags & FBIM_FLAG_LAGGED_REORTH) != 0;
  const int m = lagged ? std::min(c->restart, kOrthFused) : c->restart;
  iters = 0;
  relres = 0;
  double nb;
  STCHK(norm2(c, b, nt, nb));
  if (!std::isfinite(nb)) return fail(c, FBIM_EINVAL, "non-finite right-hand side");
  if (!warm || nb == 0.0) HIPCHK(c, launch_fill(nt, 0.0, x, s));
  if (nb == 0.0) return FBIM_OK;
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), hcol(m + 3), y(m);
  std::vector<double> Hu(lagged ? (size_t)(m + 1) * m : 0), slag;  // unrotated columns, lag of the newest vector
  double nlag = 1.0;                                                 // and its norm as it stands in V
  bool first = !warm;
  const bool saved32 = c->cur32;
  struct Restore {
    fbim_ctx *c;
    bool v;
    ~Restore() { c->cur32 = v; }
  } restore{c, saved32};
  for (;;) {
    // r = b - A x
    if (first) {
      HIPCHK(c, hipMemcpyAsync(c->d_r, b, nt * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      if (relax > 0) c->cur32 = false;
      STCHK(apply_saddle(c, x, c->d_r));
      HIPCHK(c, launch_axpby(nt, 1.0, b, -1.0, c->d_r, s));
    }
    double beta;
    STCHK(norm2(c, c->d_r, nt, beta));
    if (!std::isfinite(beta)) return fail(c, FBIM_EDEVICE, "non-finite GMRES residual");
    relres = beta / nb;
    if (relres <= tol) return FBIM_OK;
    if (iters >= maxit) return fail(c, FBIM_ENOCONV, "GMRES iteration limit reached");
    first = false;
    {
      Timer t(c, "blas");
      HIPCHK(c, launch_axpby(nt, 1.0 / beta, c->d_r, 0.0, c->d_V, s));
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    slag.clear();
    nlag = 1.0;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double *vj = c->d_V + (size_t)j * nt;
      double *w = c->d_V + (size_t)(j + 1) * nt;
      if (relax > 0) c->cur32 = std::fabs(g[j]) <= relax * nb;
      STCHK(apply_precond(c, vj, c->d_t1));
      STCHK(apply_saddle(c, c->d_t1, w));
      double hn = 0;
      if (lagged) {
        STCHK(arnoldi_lagged(c, j, w, nt, Hu, m, slag, nlag, hcol.data()));
        for (int i = 0; i <= j + 1; ++i) Hu[(size_t)i * m + j] = hcol[i];
        hn = hcol[j + 1];
      } else {
        STCHK(orthogonalise(c, c->d_V, j + 1, w, nt, hcol.data(), hn, true));
      }
      if (!std::isfinite(hn)) return fail(c, FBIM_EDEVICE, "non-finite Krylov vector");
      hcol[j + 1] = hn;
      for (int i = 0; i < j; ++i) {  // previous rotations
        const double t1 = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
        hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
        hcol[i] = t1;
      }
      const double den = std::hypot(hcol[j], hcol[j + 1]);
      cs[j] = den > 0 ? hcol[j] / den : 1.0;
      sn[j] = den > 0 ? hcol[j + 1] / den : 0.0;
      hcol[j] = den;
      hcol[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
      ++iters;
      jend = j + 1;
      if (std::fabs(g[j + 1]) <= tol * nb || iters >= maxit || hn == 0.0) break;
    }
    // y = H^-1 g, x += P^-1 V y
    for (int i = jend - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int k = i + 1; k < jend; ++k) sacc -= H[(size_t)i * m + k] * y[k];
      y[i] = sacc / H[(size_t)i * m + i];
    }
    HIPCHK(c, hipMemcpyAsync(c->d_c, y.data(), jend * sizeof(double), hipMemcpyHostToDevice, s));
    {
      Timer t(c, "blas");
      HIPCHK(c, launch_Vc(c->d_V, nt, jend, c->d_c, c->d_t2, nt, s));
    }
    STCHK(apply_precond(c, c->d_t2, c->d_t1));
    HIPCHK(c, launch_axpby(nt, 1.0, c->d_t1, 1.0, x, s));
  }
}

// Solve the saddle system to tol.  FP64 contexts: GMRES directly.  Mixed
// contexts, by default: relaxed-matvec GMRES (FP64 operator until the residual
// estimate falls below kRelax ||b||, then the FP32 operator; every restart and
// the stopping test use the FP64 residual).  With FBIM_FLAG_REFINEMENT: iterative
// refinement -- the residual b - A x is formed with the FP64 matvec, and each
// correction solves A d = r with GMRES on the FP32 matvec to a relative
// tolerance of 1e-3.
fbim_status solve_saddle(fbim_ctx *c, const double *b, double *x, double tol, int &iters, double &relres,
                         bool warm = false) {
  if (!c->mixed) return gmres(c, b, x, tol, iters, relres, c->gmres_max, warm);
  if (!(c->p.flags & FBIM_FLAG_REFINEMENT)) return gmres(c, b, x, tol, iters, relres, c->gmres_max, warm, kRelax);
  const size_t nt = c->ntot;
  hipStream_t s = c->stream;
  iters = 0;
  double nb;
  STCHK(norm2(c, b, nt, nb));
  relres = nb > 0 ? 1.0 : 0.0;
  if (warm && nb > 0.0) {
    // residual of the initial guess, FP64
    c->cur32 = false;
    fbim_status st0 = apply_saddle(c, x, c->d_irr);
    c->cur32 = true;
    STCHK(st0);
    HIPCHK(c, launch_axpby(nt, 1.0, b, -1.0, c->d_irr, s));
    double nr;
    STCHK(norm2(c, c->d_irr, nt, nr));
    relres = nr / nb;
    if (relres <= tol) return FBIM_OK;
  } else {
    HIPCHK(c, launch_fill(nt, 0.0, x, s));
    HIPCHK(c, hipMemcpyAsync(c->d_irr, b, nt * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  if (nb == 0.0) return FBIM_OK;
  for (int outer = 0; outer < 20; ++outer) {
    int it = 0;
    double rr = 0;
    c->cur32 = true;
    fbim_status st = gmres(c, c->d_irr, c->d_ird, 1e-3, it, rr, std::max(1, c->gmres_max - iters));
    iters += it;
    if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
    HIPCHK(c, launch_axpby(nt, 1.0, c->d_ird, 1.0, x, s));
    c->cur32 = false;  // FP64 residual of the refined solution
    fbim_status st2 = apply_saddle(c, x, c->d_irr);
    c->cur32 = true;
    STCHK(st2);
    HIPCHK(c, launch_axpby(nt, 1.0, b, -1.0, c->d_irr, s));
    double nr;
    STCHK(norm2(c, c->d_irr, nt, nr));
    relres = nr / nb;
    if (relres <= tol) return FBIM_OK;
    if (iters >= c->gmres_max) break;
  }
  return fail(c, FBIM_ENOCONV, "GMRES iterative refinement did not reach the tolerance");
}

// Lanczos for (G M^(r) G^T)^(1/2) b with full reorthogonalisation; y = ||b|| V f(T) e_1
fbim_status lanczos_sqrt(fbim_ctx *c, const double *b, double *out, int &iters, double &change) {
  const size_t n2 = 2 * (size_t)c->N;
  hipStream_t s = c->stream;
  iters = 0;
  change = 0;
  double beta0;
  STCHK(norm2(c, b, n2, beta0));
  if (!std::isfinite(beta0)) return fail(c, FBIM_EINVAL, "non-finite Lanczos start vector");
  if (beta0 == 0.0) {
    HIPCHK(c, launch_fill(n2, 0.0, out, s));
    return FBIM_OK;
  }
  const int kmax = std::min(c->lanczos_max, (int)c->capV - 1);
  HIPCHK(c, launch_axpby(n2, 1.0 / beta0, b, 0.0, c->d_V, s));
  std::vector<double> alpha, beta, cprev, cur, hbuf(kmax + 3);
  fbim_status st = FBIM_OK;
  int k = 0;
  for (;; ++k) {
    double *vk = c->d_V + (size_t)k * c->ntot;
    double *w = c->d_V + (size_t)(k + 1) * c->ntot;
    HIPCHK(c, launch_body_apply(c->geom(), c->mats(), c->bt, 0, vk, c->d_vec_a, s));
    STCHK(apply_M(c, c->d_vec_a, c->d_vec_b, FBIM_PART_REAL | FBIM_PART_ALPERT));
    HIPCHK(c, launch_body_apply(c->geom(), c->mats(), c->bt, 0, c->d_vec_b, w, s));
    double bk = 0;
    STCHK(orthogonalise(c, c->d_V, k + 1, w, n2, hbuf.data(), bk, true));  // w / bk: next basis vector
    if (!std::isfinite(bk) || !std::isfinite(hbuf[k])) return fail(c, FBIM_EDEVICE, "non-finite Lanczos vector");
    alpha.push_back(hbuf[k]);
    // coefficients c = beta0 Q sqrt(max(L, 0)) Q^T e1 of the (k+1) x (k+1) tridiagonal
    const int m = k + 1;
    std::vector<double> T((size_t)m * m, 0.0), lam, Q;
    for (int i = 0; i < m; ++i) {
      T[(size_t)i * m + i] = alpha[i];
      if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = beta[i];
    }
    eigh_sym(m, T, lam, Q);
    cur.assign(m, 0.0);
    for (int r = 0; r < m; ++r) {
      double sacc = 0;
      for (int q = 0; q < m; ++q) sacc += Q[(size_t)r * m + q] * std::sqrt(std::max(lam[q], 0.0)) * Q[q];
      cur[r] = beta0 * sacc;
    }
    double dn = 0, cn = 0;
    for (int r = 0; r < m; ++r) {
      const double pv = r < (int)cprev.size() ? cprev[r] : 0.0;
      dn += (cur[r] - pv) * (cur[r] - pv);
      cn += cur[r] * cur[r];
    }
    change = std::sqrt(dn / std::max(cn, 1e-300));
    cprev = cur;
    iters = m;
    const bool breakdown = bk <= 1e-14 * std::fabs(alpha[0]);
    if ((k > 0 && change <= c->p.tol_lanczos) || breakdown) break;
    if (m >= kmax) {
      st = FBIM_ENOCONV;
      c->err = "Lanczos iteration limit reached";
      break;
    }
    beta.push_back(bk);
  }
  HIPCHK(c, hipMemcpyAsync(c->d_c, cur.data(), cur.size() * sizeof(double), hipMemcpyHostToDevice, s));
  {
    Timer t(c, "blas");
    HIPCHK(c, launch_Vc(c->d_V, c->ntot, (int)cur.size(), c->d_c, c->d_vec_a, n2, s));
  }
  HIPCHK(c, launch_body_apply(c->geom(), c->mats(), c->bt, 1, c->d_vec_a, out, s));
  return st;
}

fbim_status fill_noise(fbim_ctx *c, const double *&W_r, const double *&W_grid, const double **W_tilde) {
  const bool need_t = W_tilde && !*W_tilde;
  if (W_r && W_grid && !need_t) return FBIM_OK;
  const uint64_t k = c->noise_next;
  hipStream_t s = c->stream;
  const uint64_t seed = c->p.seed;
  if (!W_r) {
    const size_t n = 2 * (size_t)c->N;
    if (n > c->nz_cap_r) {
      HIPCHK(c, dalloc(c->d_nz_r, n));
      c->nz_cap_r = n;
    }
    HIPCHK(c, launch_normals(seed, FBIM_NOISE_W_R, k, n, c->d_nz_r, s));
    W_r = c->d_nz_r;
  }
  if (!W_grid) {
    const size_t n = 2 * (size_t)c->d.M * c->d.M;
    if (n > c->nz_cap_g) {
      HIPCHK(c, dalloc(c->d_nz_g, n));
      c->nz_cap_g = n;
    }
    HIPCHK(c, launch_normals(seed, FBIM_NOISE_W_GRID, k, n, c->d_nz_g, s));
    W_grid = c->d_nz_g;
  }
  if (need_t) {
    const size_t n = 3 * (size_t)c->n;
    if (n > c->nz_cap_t) {
      HIPCHK(c, dalloc(c->d_nz_t, n));
      c->nz_cap_t = n;
    }
    HIPCHK(c, launch_normals(seed, FBIM_NOISE_W_TILDE, k, n, c->d_nz_t, s));
    *W_tilde = c->d_nz_t;
  }
  c->noise_next = k + 1;
  return FBIM_OK;
}

// warm: start GMRES from the solution of the previous solve of this context
fbim_status mobility(fbim_ctx *c, const double *F, const double *slip, double *U, double *mu_out, int &its,
                     double &res, bool warm = false, double tol = 0.0) {
  const size_t twoN = 2 * (size_t)c->N, nt = c->ntot;
  hipStream_t s = c->stream;
  // b = -[slip; F]
  if (slip)
    HIPCHK(c, launch_axpby(twoN, -1.0, slip, 0.0, c->d_b, s));
  else
    HIPCHK(c, launch_fill(twoN, 0.0, c->d_b, s));
  HIPCHK(c, launch_axpby(3 * (size_t)c->n, -1.0, F, 0.0, c->d_b + twoN, s));
  fbim_status st = solve_saddle(c, c->d_b, c->d_x2, tol > 0 ? tol : c->p.tol_gmres, its, res, warm);
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  HIPCHK(c, hipMemcpyAsync(U, c->d_x2 + twoN, 3 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (mu_out) HIPCHK(c, hipMemcpyAsync(mu_out, c->d_x2, twoN * sizeof(double), hipMemcpyDeviceToDevice, s));
  (void)nt;
  return st;
}

// slip_out[2N] = sqrt(2 kT / dt) (v^(r) + v^(w)) of eq. 3.27 (slip_out must not be d_r)
fbim_status brownian_slip(fbim_ctx *c, double dt, const double *W_r, const double *W_grid, double *slip_out,
                          fbim_info *info) {
  hipStream_t s = c->stream;
  const size_t twoN = 2 * (size_t)c->N;
  int li = 0;
  double lc = 0;
  double *acc = c->d_r;  // scratch outside GMRES
  fbim_status st = lanczos_sqrt(c, W_r, acc, li, lc);
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  STCHK(random_field(c, W_grid, c->d_vec_b));
  const double amp = std::sqrt(2.0 * c->p.kT / dt);
  HIPCHK(c, launch_axpby(twoN, 1.0, c->d_vec_b, 1.0, acc, s));
  HIPCHK(c, launch_axpby(twoN, amp, acc, 0.0, slip_out, s));
  if (info) {
    info->lanczos_iters += li;
    info->lanczos_change = lc;
  }
  return st;
}

fbim_status brownian(fbim_ctx *c, double dt, const double *F, const double *W_r, const double *W_grid, double *U,
                     fbim_info *info) {
  int gi = 0;
  double gr = 0;
  fbim_status st = brownian_slip(c, dt, W_r, W_grid, c->d_w, info);
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  fbim_status st2 = mobility(c, F, c->d_w, U, nullptr, gi, gr);
  if (info) {
    info->gmres_iters += gi;
    info->gmres_solves += 1;
    info->gmres_residual = std::max(info->gmres_residual, gr);
  }
  if (st2 != FBIM_OK) return st2;
  return st;
}

}  // namespace fbim

// ====================================================================== C ABI
extern "C" {

const char *fbim_status_string(fbim_status s) {
  switch (s) {
    case FBIM_OK: return "ok";
    case FBIM_EINVAL: return "invalid argument";
    case FBIM_ENOMEM: return "out of memory";
    case FBIM_EOVERLAP: return "bodies overlap";
    case FBIM_ENOCONV: return "solver did not converge";
    case FBIM_EDEVICE: return "device error";
    case FBIM_ENOTSUP: return "not supported";
    case FBIM_WACCURACY: return "accuracy warning";
  }
  return "unknown status";
}

const char *fbim_last_error(const fbim_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

fbim_status fbim_derive_params(const fbim_params *in, fbim_derived *out) {
  if (!in || !out) return FBIM_EINVAL;
  Derived d;
  if (!derive(*in, d).empty()) return FBIM_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->xi = d.xi;
  out->r_c = d.r_c;
  out->h = d.h;
  out->eta_s = d.eta_s;
  out->n_box = d.n_box;
  out->grid_M = d.M;
  out->P = d.P;
  out->tile = d.tile;
  return FBIM_OK;
}

fbim_status fbim_alpert_rule(int32_t order, int32_t *j, int32_t *a, double *chi, double *w) {
  if (!j || !a || !chi || !w) return FBIM_EINVAL;
  int jj, aa;
  std::string err;
  if (!fbim::alpert_rule(order, jj, aa, chi, w, err)) return FBIM_EINVAL;
  *j = jj;
  *a = aa;
  return FBIM_OK;
}

void fbim_starfish(double r_s, double b, int32_t n_arm, int32_t n_p, double *ref_xy) {
  for (int j = 0; j < n_p; ++j) {
    const double sj = 2.0 * kPi * j / n_p;
    const double r = r_s * (1.0 + b * std::cos(n_arm * sj));
    ref_xy[2 * j] = r * std::cos(sj);
    ref_xy[2 * j + 1] = r * std::sin(sj);
  }
}

fbim_status fbim_create(const fbim_params *params, fbim_ctx **out) {
  if (!params || !out) return FBIM_EINVAL;
  *out = nullptr;
  auto *c = new fbim_ctx();
  c->p = *params;
  if (hipGetDevice(&c->device) != hipSuccess || resolve_noalloc_scratch(c) != FBIM_OK ||
      hipHostMalloc((void **)&c->h_pin, 16 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    fbim_destroy(c);
    return FBIM_EDEVICE;
  }
  if (c->p.eta <= 0) c->p.eta = 1.0;
  if (c->p.tau_spurious <= 0) c->p.tau_spurious = 1e-8;
  if (c->p.tol_gmres <= 0) c->p.tol_gmres = 1e-6;
  if (c->p.tol_lanczos <= 0) c->p.tol_lanczos = 1e-6;
  if (!(c->p.tol_rfd >= 0 && c->p.tol_rfd < 1)) {  // NaN included
    fbim_destroy(c);
    return FBIM_EINVAL;
  }
  if (c->p.tol_rfd == 0) c->p.tol_rfd = c->p.tol_gmres;
  if (c->p.alpert_order == 0) c->p.alpert_order = 4;
  c->restart = c->p.gmres_restart > 0 ? c->p.gmres_restart : 100;
  c->gmres_max = c->p.gmres_maxiter > 0 ? c->p.gmres_maxiter : 1000;
  c->lanczos_max = c->p.lanczos_maxiter > 0 ? c->p.lanczos_maxiter : 200;
  c->mixed = c->p.precision == FBIM_PREC_MIXED;
  if (c->restart > 500 || c->lanczos_max > 500) {
    fbim_destroy(c);
    return FBIM_EINVAL;
  }
  if (c->p.precision != FBIM_PREC_FP64 && c->p.precision != FBIM_PREC_MIXED) {
    fbim_destroy(c);
    return FBIM_EINVAL;
  }
  std::string err = derive(c->p, c->d);
  if (!err.empty()) {
    fbim_destroy(c);
    return FBIM_EINVAL;
  }
  if (c->d.P > 15) {
    fbim_destroy(c);
    return FBIM_ENOTSUP;
  }
  c->order = c->p.alpert_order;
  if (!fbim::alpert_rule(c->order, c->aj, c->aa, c->chi, c->w, err)) {
    fbim_destroy(c);
    return FBIM_EINVAL;
  }
  c->ncell = c->d.n_box * c->d.n_box;
  c->nts = c->d.M / c->d.tile;
  c->ntile = c->nts * c->nts;
  fbim_status st = FBIM_OK;
  auto t64 = e1_table(kE1Deg64);
  auto t32d = e1_table(kE1Deg32);
  std::vector<float> t32(t32d.begin(), t32d.end());
  if ((st = upload(c, c->d_e1tab, t64)) != FBIM_OK || (st = upload(c, c->d_e1tab32, t32)) != FBIM_OK ||
      hipMalloc((void **)&c->d_scal_int, 8 * sizeof(int)) != hipSuccess ||
      dalloc(c->d_ccount, c->ncell) != hipSuccess || dalloc(c->d_ccursor, c->ncell) != hipSuccess ||
      dalloc(c->d_cstart, c->ncell + 1) != hipSuccess || dalloc(c->d_tcount, c->ntile) != hipSuccess ||
      dalloc(c->d_tcursor, c->ntile) != hipSuccess || dalloc(c->d_tstart, c->ntile + 1) != hipSuccess ||
      dalloc(c->d_scount, c->ntile) != hipSuccess || dalloc(c->d_sstart, c->ntile + 1) != hipSuccess) {
    fbim_destroy(c);
    return FBIM_EDEVICE;
  }
  if ((st = setup_fft(c)) != FBIM_OK) {
    fbim_destroy(c);
    return st;
  }
  *out = c;
  return FBIM_OK;
}

void fbim_destroy(fbim_ctx *c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  resolve_timing(c);
  sk_destroy(c);
  for (auto &s : c->shapes) {
    dfree(s.ref);
    dfree(s.band);
    dfree(s.Mp);
    dfree(s.Pref);
    dfree(s.Nt);
    dfree(s.G);
    dfree(s.Gp);
  }
  if (c->fwd) rocfft_plan_destroy(c->fwd);
  if (c->inv) rocfft_plan_destroy(c->inv);
  if (c->fwd32) rocfft_plan_destroy(c->fwd32);
  if (c->inv32) rocfft_plan_destroy(c->inv32);
  if (c->einfo) rocfft_execution_info_destroy(c->einfo);
  if (c->fft_work) hipFree(c->fft_work);
  void *ptrs[] = {c->d_ref_arr, c->d_band_arr, c->d_Mp_arr, c->d_Pref_arr, c->d_Nt_arr, c->d_G_arr, c->d_Gp_arr,
                  c->d_band, c->d_np, c->d_shape, c->d_off, c->d_body, c->d_q, c->d_theta, c->d_x,
                  c->d_ckey, c->d_ccount, c->d_cstart, c->d_cperm, c->d_ccursor, c->d_xs, c->d_tkey,
                  c->d_tcount, c->d_tstart, c->d_tperm, c->d_tcursor, c->d_xt, c->d_anchor, c->d_scal_int, c->d_src64,
                  c->d_mut, c->d_src32, c->d_xt32, c->d_mut32, c->d_grid, c->d_spec, c->d_grid32,
                  c->d_spec32, c->d_e1tab, c->d_e1tab32, c->d_V, c->d_w, c->d_t1, c->d_t2, c->d_b, c->d_x2,
                  c->d_r, c->d_partial, c->d_h, c->d_h2, c->d_nrm, c->d_lag, c->d_c, c->d_vec_a, c->d_vec_b, c->d_U3,
                  c->d_U4, c->d_U5, c->d_U6, c->d_irx, c->d_irr, c->d_ird, c->d_cnt_near, c->d_cnt_far, c->d_tcell, c->d_gnn, c->d_gnf, c->d_goff, c->d_gsize, c->d_ell, c->d_chunks, c->d_chunk_sys, c->d_sys_chunk, c->d_btile, c->d_blist, c->d_dN, c->d_mw, c->d_am, c->d_av, c->d_g, c->d_X, c->d_H1, c->d_H2, c->d_Y, c->d_dY, c->d_Z2, c->d_Z1, c->d_ones, c->d_loss, c->d_trF, c->d_trU, c->d_bx, c->d_by, c->d_tw, c->d_tw32, c->d_ey, c->d_ey32, c->d_scount, c->d_sstart, c->d_slist, c->d_nz_r, c->d_nz_g, c->d_nz_t, c->d_bc_key, c->d_bc_perm, c->d_bc_count, c->d_bc_cursor, c->d_bc_start, c->d_qprev, c->d_thprev, c->d_qstep, c->d_thstep};
  pub_free(c->pub);
  if (c->h_pin) hipHostFree(c->h_pin);
  if (c->h_qpin) hipHostFree(c->h_qpin);
  engine_delete(c->rfd_engine);
  for (fbim_ctx *r : c->rfd)
    if (r) fbim_destroy(r);
  for (void *p : ptrs)
    if (p) hipFree(p);
  delete c;
}

fbim_status fbim_set_stream(fbim_ctx *c, void *stream) {
  if (!c) return FBIM_EINVAL;
  c->stream = (hipStream_t)stream;
  if (c->einfo) FFTCHK(c, rocfft_execution_info_set_stream(c->einfo, c->stream));
  return FBIM_OK;
}

fbim_status fbim_add_shape(fbim_ctx *c, int32_t n_p, const double *ref_xy, int32_t *shape_id) {
  if (!c || !ref_xy || !shape_id) return fail(c, FBIM_EINVAL, "null argument");
  ShapeDev sd;
  std::string err = build_shape(n_p, ref_xy, c->d, c->p.eta, c->order, c->p.tau_spurious, sd.h);
  if (!err.empty()) return fail(c, FBIM_EINVAL, err);
  STCHK(upload(c, sd.ref, sd.h.ref_xy));
  {  // the band o-major on the device, [o = -band..band][t][2 x 2], so that the
     // nodes of a body (consecutive lanes) read consecutive blocks for each offset
    const int nb = 2 * sd.h.band + 1;
    std::vector<double> bt(sd.h.alpert.size());
    for (int t = 0; t < n_p; ++t)
      for (int o = 0; o < nb; ++o)
        for (int q = 0; q < 4; ++q) bt[((size_t)o * n_p + t) * 4 + q] = sd.h.alpert[((size_t)t * nb + o) * 4 + q];
    STCHK(upload(c, sd.band, bt));
  }
  STCHK(upload(c, sd.Mp, sd.h.Mpinv));
  STCHK(upload(c, sd.Pref, sd.h.Pref));
  STCHK(upload(c, sd.Nt, sd.h.Nt));
  STCHK(upload(c, sd.G, sd.h.Gref));
  STCHK(upload(c, sd.Gp, sd.h.Gpref));
  c->shapes.push_back(sd);
  c->max_np = std::max(c->max_np, n_p);
  STCHK(rebuild_shape_arrays(c));
  *shape_id = (int32_t)c->shapes.size() - 1;
  if (sd.h.r_alpert > 0.6 * c->d.r_c) {
    c->err = "r_Alpert / r_c exceeds 0.6";
    return FBIM_WACCURACY;
  }
  return FBIM_OK;
}

fbim_status fbim_set_bodies(fbim_ctx *c, int32_t n, const int32_t *shape_id, const double *q,
                            const double *theta) {
  if (!c || n <= 0 || !shape_id || !q || !theta) return fail(c, FBIM_EINVAL, "invalid bodies");
  std::vector<int> off(n + 1, 0);
  for (int b = 0; b < n; ++b) {
    if (shape_id[b] < 0 || shape_id[b] >= (int)c->shapes.size()) return fail(c, FBIM_EINVAL, "bad shape id");
    if (!std::isfinite(q[2 * b]) || !std::isfinite(q[2 * b + 1]) || !std::isfinite(theta[b]))
      return fail(c, FBIM_EINVAL, "non-finite body coordinate");
    off[b + 1] = off[b] + c->shapes[shape_id[b]].h.n_p;
  }
  const int N = off[n];
  if (N > kMaxNodes) return fail(c, FBIM_EINVAL, "too many nodes (at most 2^26 - 2 per context)");
  if (c->have_bodies && n == c->n && std::equal(shape_id, shape_id + n, c->h_shape.begin())) {
    // same bodies moved: only positions and angles change.  A rejected move
    // (overlap, device error) rebuilds the previous configuration, so the
    // context stays where it was.
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(c->d_qprev, c->d_q, 2 * (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_thprev, c->d_theta, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<double> q_old = c->h_q, th_old = c->h_theta;
    c->h_q.assign(q, q + 2 * n);
    c->h_theta.assign(theta, theta + n);
    const fbim_status st = build_geometry(c);
    if (st != FBIM_OK) {
      const std::string msg = c->err;
      c->h_q.swap(q_old);
      c->h_theta.swap(th_old);
      if (hipMemcpyAsync(c->d_q, c->d_qprev, 2 * (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s) !=
              hipSuccess ||
          hipMemcpyAsync(c->d_theta, c->d_thprev, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s) !=
              hipSuccess ||
          build_geometry_dev(c) != FBIM_OK)
        c->have_bodies = false;
      c->err = msg;
    }
    return st;
  }
  const bool realloc_n = n != c->capn, realloc_N = N != c->capN;
  c->h_shape.assign(shape_id, shape_id + n);
  c->h_off = off;
  c->h_q.assign(q, q + 2 * n);
  c->h_theta.assign(theta, theta + n);
  c->n = n;
  c->N = N;
  if (realloc_n) {
    HIPCHK(c, dalloc(c->d_shape, n));
    HIPCHK(c, dalloc(c->d_off, n + 1));
    HIPCHK(c, dalloc(c->d_q, 2 * n));
    HIPCHK(c, dalloc(c->d_theta, n));
    HIPCHK(c, dalloc(c->d_qprev, 2 * n));
    HIPCHK(c, dalloc(c->d_thprev, n));
    HIPCHK(c, dalloc(c->d_qstep, 2 * n));
    HIPCHK(c, dalloc(c->d_thstep, n));
    if (c->h_qpin) {
      HIPCHK(c, hipStreamSynchronize(c->stream));
      hipHostFree(c->h_qpin);
      c->h_qpin = nullptr;
    }
    HIPCHK(c, hipHostMalloc((void **)&c->h_qpin, 3 * (size_t)n * sizeof(double), hipHostMallocDefault));
    c->capn = n;
  }
  if (realloc_N) {
    HIPCHK(c, dalloc(c->d_body, N));
    HIPCHK(c, dalloc(c->d_x, 2 * N));
    HIPCHK(c, dalloc(c->d_ckey, N));
    HIPCHK(c, dalloc(c->d_cperm, N));
    HIPCHK(c, dalloc(c->d_xs, 2 * N));
    HIPCHK(c, dalloc(c->d_tkey, N));
    HIPCHK(c, dalloc(c->d_tperm, N));
    HIPCHK(c, dalloc(c->d_xt, 2 * N));
    HIPCHK(c, dalloc(c->d_anchor, 2 * N));
    HIPCHK(c, dalloc(c->d_src64, 4 * (N + 1)));  // + the zero record
    HIPCHK(c, dalloc(c->d_mut, 2 * N));
    c->ngroups = (N + 63) / 64;
    HIPCHK(c, dalloc(c->d_cnt_near, N));
    HIPCHK(c, dalloc(c->d_cnt_far, N));
    HIPCHK(c, dalloc(c->d_tcell, N));
    HIPCHK(c, dalloc(c->d_gnn, c->ngroups));
    HIPCHK(c, dalloc(c->d_gnf, c->ngroups));
    HIPCHK(c, dalloc(c->d_gsize, c->ngroups));
    HIPCHK(c, dalloc(c->d_goff, c->ngroups + 1));
    if (c->mixed) {
      HIPCHK(c, dalloc(c->d_src32, 4 * (N + 1)));
      HIPCHK(c, dalloc(c->d_xt32, 2 * N));
      HIPCHK(c, dalloc(c->d_mut32, 2 * N));
    }
    c->capN = N;
  }
  std::vector<int> body(N);
  for (int b = 0; b < n; ++b)
    for (int i = off[b]; i < off[b + 1]; ++i) body[i] = b;
  HIPCHK(c, hipMemcpy(c->d_shape, c->h_shape.data(), n * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_off, off.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_body, body.data(), N * sizeof(int), hipMemcpyHostToDevice));
  STCHK(build_body_tiles(c));
  c->have_bodies = true;
  STCHK(ensure_krylov(c));
  const fbim_status st = build_geometry(c);
  if (st != FBIM_OK) c->have_bodies = false;  // a new body set that failed leaves no bodies
  return st;
}

fbim_status fbim_get_derived(const fbim_ctx *c, fbim_derived *out) {
  if (!c || !out) return FBIM_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->xi = c->d.xi;
  out->r_c = c->d.r_c;
  out->h = c->d.h;
  out->eta_s = c->d.eta_s;
  out->n_box = c->d.n_box;
  out->grid_M = c->d.M;
  out->P = c->d.P;
  out->tile = c->d.tile;
  out->alpert_j = c->aj;
  out->alpert_a = c->aa;
  out->n_bodies = c->n;
  out->n_nodes = c->N;
  double ra = 0;
  for (auto &s : c->shapes) ra = std::max(ra, s.h.r_alpert);
  out->r_alpert = ra;
  return FBIM_OK;
}

fbim_status fbim_get_nodes(fbim_ctx *c, double *x) {
  if (!c || !x || !c->have_bodies) return fail(c, FBIM_EINVAL, "no bodies");
  HIPCHK(c, hipMemcpyAsync(x, c->d_x, 2 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return FBIM_OK;
}

fbim_status fbim_apply_M(fbim_ctx *c, const double *mu, double *out, uint32_t parts) {
  if (!c || !mu || !out || mu == out) return fail(c, FBIM_EINVAL, "invalid pointers");
  if (parts == 0 || parts > FBIM_PART_ALL) return fail(c, FBIM_EINVAL, "invalid parts");
  return apply_M(c, mu, out, parts);
}

fbim_status fbim_random_field(fbim_ctx *c, const double *W_grid, double *out) {
  if (!c || !W_grid || !out || !c->have_bodies) return fail(c, FBIM_EINVAL, "invalid arguments");
  return random_field(c, W_grid, out);
}

fbim_status fbim_sqrt_Mr(fbim_ctx *c, const double *W_r, double *out, fbim_info *info) {
  if (!c || !W_r || !out || !c->have_bodies) return fail(c, FBIM_EINVAL, "invalid arguments");
  info_reset(info);
  const double t0 = now_ms();
  int it = 0;
  double ch = 0;
  fbim_status st = lanczos_sqrt(c, W_r, out, it, ch);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->lanczos_iters = it;
    info->lanczos_change = ch;
    info->status = st;
    info->ms_total = now_ms() - t0;
  }
  return st;
}

fbim_status fbim_apply_precond(fbim_ctx *c, const double *z, double *y) {
  if (!c || !z || !y || z == y || !c->have_bodies) return fail(c, FBIM_EINVAL, "invalid arguments");
  return apply_precond(c, z, y);
}

fbim_status fbim_mobility(fbim_ctx *c, const double *F, const double *slip, double *U, double *mu_out,
                          fbim_info *info) {
  if (!c || !F || !U || !c->have_bodies) return fail(c, FBIM_EINVAL, "invalid arguments");
  info_reset(info);
  const double t0 = now_ms();
  int it = 0;
  double res = 0;
  fbim_status st = mobility(c, F, slip, U, mu_out, it, res);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->gmres_iters = it;
    info->gmres_solves = 1;
    info->gmres_residual = res;
    info->status = st;
    info->ms_total = now_ms() - t0;
  }
  return st;
}

fbim_status fbim_brownian_velocity(fbim_ctx *c, double dt, const double *F, const double *W_r,
                                   const double *W_grid, double *U, fbim_info *info) {
  if (!c || !F || !U || !(dt > 0) || !c->have_bodies) return fail(c, FBIM_EINVAL, "invalid arguments");
  info_reset(info);
  const double t0 = now_ms();
  STCHK(fill_noise(c, W_r, W_grid, nullptr));
  fbim_status st = brownian(c, dt, F, W_r, W_grid, U, info);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->status = st;
    info->ms_total = now_ms() - t0;
  }
  return st;
}

fbim_status fbim_step_em_rfd(fbim_ctx *c, double dt, double delta, const double *F, const double *W_r,
                             const double *W_grid, const double *W_tilde, double *dQ, int32_t apply,
                             fbim_info *info) {
  if (!c || !F || !dQ || !(dt > 0) || !(delta >= 0) || !c->have_bodies)
    return fail(c, FBIM_EINVAL, "invalid arguments");
  info_reset(info);
  const double t0 = now_ms();
  STCHK(fill_noise(c, W_r, W_grid, delta > 0 ? &W_tilde : nullptr));
  if (c->p.flags & FBIM_FLAG_BATCH_RFD) {
    // the three solves in one lockstep batch with two copies of the context
    if (!c->rfd_engine) c->rfd_engine = engine_new();
    engine_set_stream(c->rfd_engine, c->stream);
    engine_set_flags(c->rfd_engine, (c->p.flags & FBIM_FLAG_GRAPH) ? FBIM_BATCH_GRAPH : 0u);
    fbim_status st = em_rfd_batch(c->rfd_engine, {c}, dt, delta, &F, &W_r, &W_grid, &W_tilde, &dQ, apply, info);
    if (st != FBIM_OK) c->err = engine_error(c->rfd_engine);
    if (info) info->ms_total = now_ms() - t0;
    return st;
  }
  hipStream_t s = c->stream;
  const int n = c->n;
  const size_t n3 = 3 * (size_t)n;
  // Q^n on the device; every configuration of the step is moved from it there
  HIPCHK(c, hipMemcpyAsync(c->d_qstep, c->d_q, 2 * (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_thstep, c->d_theta, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // any error after the configuration has left Q puts the bodies back at Q
  struct BackToQ {
    fbim_ctx *c;
    bool moved = false, armed = true;
    ~BackToQ() {
      if (!armed || !moved || !c->have_bodies) return;
      const std::string msg = c->err;
      move_bodies(c, c->d_qstep, c->d_thstep, nullptr, 0.0);
      c->err = msg;
    }
  } guard{c};
  // U0 = N F + sqrt(2kT/dt) N^(1/2) W at Q
  fbim_status st = brownian(c, dt, F, W_r, W_grid, c->d_U3, info);
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  fbim_status worst = st;
  // RFD solves N(Q +- delta/2 Wt) Wt (none without the RFD term)
  for (int sgn = 1; delta > 0 && sgn >= -1; sgn -= 2) {
    guard.moved = true;
    STCHK(move_bodies(c, c->d_qstep, c->d_thstep, W_tilde, sgn * 0.5 * delta));
    int it = 0;
    double res = 0;
    // the second configuration starts from the first one's solution (same right-hand
    // side, configurations delta apart): the initial residual is O(delta)
    fbim_status s2 =
        mobility(c, W_tilde, nullptr, sgn > 0 ? c->d_U4 : c->d_U5, nullptr, it, res, sgn < 0, c->p.tol_rfd);
    if (s2 != FBIM_OK && s2 != FBIM_ENOCONV) return s2;
    if (s2 != FBIM_OK) worst = s2;
    if (info) {
      info->gmres_iters += it;
      info->gmres_solves += 1;
      info->gmres_residual = std::max(info->gmres_residual, res);
    }
  }
  // dQ = dt U0 + dt kT/delta (U+ - U-)
  HIPCHK(c, launch_axpby(n3, dt, c->d_U3, 0.0, dQ, s));
  if (delta > 0) {
    HIPCHK(c, launch_axpby(n3, dt * c->p.kT / delta, c->d_U4, 1.0, dQ, s));
    HIPCHK(c, launch_axpby(n3, -dt * c->p.kT / delta, c->d_U5, 1.0, dQ, s));
  }
  // Q^{n+1} = Q^n + dQ (apply), else back to Q^n
  STCHK(move_bodies(c, c->d_qstep, c->d_thstep, apply ? dQ : nullptr, 1.0));
  guard.armed = false;
  HIPCHK(c, hipStreamSynchronize(s));
  if (info) {
    info->status = worst;
    info->ms_total = now_ms() - t0;
  }
  return worst;
}

fbim_status fbim_step_ab2_rfd(fbim_ctx *c, double dt, double delta, const double *F, const double *W_r,
                              const double *W_grid, const double *W_tilde, double *NF_hist, int32_t have_hist,
                              double *dQ, int32_t apply, fbim_info *info) {
  if (!c || !F || !dQ || !NF_hist || !(dt > 0) || !(delta >= 0) || !c->have_bodies)
    return fail(c, FBIM_EINVAL, "invalid arguments");
  const double t0 = now_ms();
  // the EM-RFD displacement at Q (configuration left at Q)
  fbim_status st = fbim_step_em_rfd(c, dt, delta, F, W_r, W_grid, W_tilde, dQ, 0, info);
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  fbim_status worst = st;
  // N^n F^n: F alone, zero slip
  int it = 0;
  double res = 0;
  fbim_status s2 = mobility(c, F, nullptr, c->d_U6, nullptr, it, res);
  if (s2 != FBIM_OK && s2 != FBIM_ENOCONV) return s2;
  if (s2 != FBIM_OK) worst = s2;
  if (info) {
    info->gmres_iters += it;
    info->gmres_solves += 1;
    info->gmres_residual = std::max(info->gmres_residual, res);
  }
  hipStream_t s = c->stream;
  const size_t n3 = 3 * (size_t)c->n;
  // dQ += dt/2 (N^n F^n - N^(n-1) F^(n-1)); the history becomes N^n F^n
  if (have_hist) {
    HIPCHK(c, launch_axpby(n3, 0.5 * dt, c->d_U6, 1.0, dQ, s));
    HIPCHK(c, launch_axpby(n3, -0.5 * dt, NF_hist, 1.0, dQ, s));
  }
  HIPCHK(c, hipMemcpyAsync(NF_hist, c->d_U6, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (apply) {
    HIPCHK(c, hipMemcpyAsync(c->d_qstep, c->d_q, 2 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_thstep, c->d_theta, (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    STCHK(move_bodies(c, c->d_qstep, c->d_thstep, dQ, 1.0));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  if (info) {
    info->status = worst;
    info->ms_total = now_ms() - t0;
  }
  return worst;
}

fbim_status fbim_noise_normals(fbim_ctx *c, uint32_t stream, uint64_t counter, size_t n, double *out) {
  if (!c || (!out && n)) return fail(c, FBIM_EINVAL, "invalid arguments");
  if ((n + 1) / 2 > 0xFFFFFFFFull) return fail(c, FBIM_EINVAL, "too many normals in one draw");
  HIPCHK(c, launch_normals(c->p.seed, stream, counter, n, out, c->stream));
  return FBIM_OK;
}

fbim_status fbim_noise_words(fbim_ctx *c, uint32_t stream, uint64_t counter, size_t n_pairs, uint32_t *out) {
  if (!c || (!out && n_pairs)) return fail(c, FBIM_EINVAL, "invalid arguments");
  if (n_pairs > 0xFFFFFFFFull) return fail(c, FBIM_EINVAL, "too many pairs in one draw");
  HIPCHK(c, launch_philox_words(c->p.seed, stream, counter, n_pairs, out, c->stream));
  return FBIM_OK;
}

fbim_status fbim_noise_counter(const fbim_ctx *c, uint64_t *counter) {
  if (!c || !counter) return FBIM_EINVAL;
  *counter = c->noise_next;
  return FBIM_OK;
}

fbim_status fbim_set_noise_counter(fbim_ctx *c, uint64_t counter) {
  if (!c) return FBIM_EINVAL;
  c->noise_next = counter;
  return FBIM_OK;
}

fbim_status fbim_mlp_init(fbim_ctx *c, uint64_t seed, int32_t sym_order) {
  if (!c || sym_order < 1) return fail(c, FBIM_EINVAL, "invalid MLP initialisation");
  STCHK(ensure_mlp(c, std::max(c->n, 1)));
  std::vector<float> w(kNParam, 0.0f);
  std::mt19937_64 gen(seed);
  auto glorot = [&](int off, int fan_in, int fan_out, float scale) {
    const float a = scale * std::sqrt(6.0f / (float)(fan_in + fan_out));
    std::uniform_real_distribution<float> u(-a, a);
    for (int i = 0; i < fan_in * fan_out; ++i) w[off + i] = u(gen);
  };
  glorot(kOffW1, kMlpIn, kMlpHid, 1.0f);
  glorot(kOffW2, kMlpHid, kMlpHid, 1.0f);
  glorot(kOffW3, kMlpHid, kMlpOut, 1e-2f);
  HIPCHK(c, hipMemcpy(c->d_mw, w.data(), kNParam * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(c, launch_fill_f32(kNParam, 0.0f, c->d_am, c->stream));
  HIPCHK(c, launch_fill_f32(kNParam, 0.0f, c->d_av, c->stream));
  c->mlp_t = 0;
  c->mlp_sym = sym_order;
  c->mlp_init = true;
  if (c->mlp_on && c->have_bodies) STCHK(mlp_refresh(c));
  return FBIM_OK;
}

fbim_status fbim_mlp_set_weights(fbim_ctx *c, const float *w, size_t n) {
  if (!c || !w || n != (size_t)kNParam) return fail(c, FBIM_EINVAL, "weights must hold FBIM_MLP_NPARAM floats");
  if (!c->mlp_init) return fail(c, FBIM_EINVAL, "fbim_mlp_init first");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->d_mw, w, n * sizeof(float), hipMemcpyHostToDevice));
  if (c->mlp_on && c->have_bodies) STCHK(mlp_refresh(c));
  return FBIM_OK;
}

fbim_status fbim_mlp_get_weights(fbim_ctx *c, float *w, size_t n) {
  if (!c || !w || n != (size_t)kNParam) return fail(c, FBIM_EINVAL, "weights must hold FBIM_MLP_NPARAM floats");
  if (!c->mlp_init) return fail(c, FBIM_EINVAL, "fbim_mlp_init first");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(w, c->d_mw, n * sizeof(float), hipMemcpyDeviceToHost));
  return FBIM_OK;
}

fbim_status fbim_mlp_features(fbim_ctx *c, float *X) {
  if (!c || !X) return fail(c, FBIM_EINVAL, "null argument");
  if (!c->have_bodies) return fail(c, FBIM_EINVAL, "no bodies set");
  return mlp_features(c, X);
}

fbim_status fbim_mlp_forward(fbim_ctx *c, const float *X, int32_t n, float *Y) {
  if (!c || !X || !Y || n < 0) return fail(c, FBIM_EINVAL, "invalid argument");
  if (!c->mlp_init) return fail(c, FBIM_EINVAL, "fbim_mlp_init first");
  STCHK(ensure_mlp(c, n));
  return mlp_forward(c, X, n, Y);
}

fbim_status fbim_mlp_forward_noalloc(fbim_ctx *c, const float *X, int32_t n, float *Y) {
  if (!c || !X || !Y || n < 0) return fail(c, FBIM_EINVAL, "invalid argument");
  if (n > FBIM_NOALLOC_MAX_BODIES)
    return fail(c, FBIM_EINVAL, "fbim_mlp_forward_noalloc: n exceeds FBIM_NOALLOC_MAX_BODIES");
  if (!c->mlp_init) return fail(c, FBIM_EINVAL, "fbim_mlp_init first");
  if (!c->noalloc_scratch) return fail(c, FBIM_EDEVICE, "no-allocation scratch not resolved");
  float *H1 = c->noalloc_scratch, *H2 = c->noalloc_scratch + (size_t)kMlpHid * FBIM_NOALLOC_MAX_BODIES;
  return mlp_forward_into(c, X, n, Y, H1, H2);
}

fbim_status fbim_mlp_backward(fbim_ctx *c, const float *X, const float *dY, int32_t n, float *grad) {
  if (!c || !X || !dY || !grad || n < 0) return fail(c, FBIM_EINVAL, "invalid argument");
  if (!c->mlp_init) return fail(c, FBIM_EINVAL, "fbim_mlp_init first");
  STCHK(ensure_mlp(c, n));
  return mlp_backward(c, X, dY, n, grad);
}

fbim_status fbim_mlp_loss(fbim_ctx *c, const float *Y, int32_t ns, const double *F, const double *U, float *loss,
                          float *dY) {
  if (!c || !Y || !F || !U || !loss || !dY || ns < 1) return fail(c, FBIM_EINVAL, "invalid argument");
  if (!c->have_bodies) return fail(c, FBIM_EINVAL, "no bodies set");
  STCHK(ensure_mlp(c, c->n));
  HIPCHK(c, launch_fill_f32(1, 0.0f, c->d_loss, c->stream));
  HIPCHK(c, launch_mlp_loss(c->n, ns, c->d_shape, c->d_theta, c->d_Nt_arr, Y, F, U, dY, c->d_loss, c->stream));
  HIPCHK(c, hipMemcpyAsync(loss, c->d_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FBIM_OK;
}

fbim_status fbim_mlp_train(fbim_ctx *c, const fbim_train_cfg *cfg, fbim_train_info *info) {
  if (!c || !cfg || cfg->n_solves < 1 || cfg->epochs < 0 || !(cfg->lr > 0.0f))
    return fail(c, FBIM_EINVAL, "invalid training configuration");
  if (!c->mlp_init || !c->have_bodies) return fail(c, FBIM_EINVAL, "fbim_mlp_init and fbim_set_bodies first");
  const int n = c->n, ns = cfg->n_solves;
  const size_t n3 = 3 * (size_t)n;
  hipStream_t s = c->stream;
  STCHK(ensure_mlp(c, n));
  if ((size_t)ns * n3 > c->train_cap) {
    HIPCHK(c, dalloc(c->d_trF, (size_t)ns * n3));
    HIPCHK(c, dalloc(c->d_trU, (size_t)ns * n3));
    c->train_cap = (size_t)ns * n3;
  }
  fbim_train_info inf{};
  std::mt19937_64 gen(cfg->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> F(n3);
  fbim_status worst = FBIM_OK;
  for (int k = 0; k < ns; ++k) {
    for (auto &v : F) v = nd(gen);
    HIPCHK(c, hipMemcpyAsync(c->d_trF + k * n3, F.data(), n3 * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    int its = 0;
    double res = 0;
    fbim_status st = mobility(c, c->d_trF + k * n3, nullptr, c->d_trU + k * n3, nullptr, its, res);
    if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
    if (st != FBIM_OK) worst = st;
    inf.gmres_iters += its;
  }
  inf.samples = ns * n;
  STCHK(mlp_features(c, c->d_X));
  float l = 0.0f;
  for (int e = 0; e <= cfg->epochs; ++e) {
    STCHK(mlp_forward(c, c->d_X, n, c->d_Y));
    {
      Timer t(c, "mlp");
      HIPCHK(c, launch_fill_f32(1, 0.0f, c->d_loss, s));
      HIPCHK(c, launch_mlp_loss(n, ns, c->d_shape, c->d_theta, c->d_Nt_arr, c->d_Y, c->d_trF, c->d_trU, c->d_dY,
                                c->d_loss, s));
    }
    if (e == 0 || e == cfg->epochs) {
      HIPCHK(c, hipMemcpyAsync(&l, c->d_loss, sizeof(float), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (e == 0) inf.loss_first = l;
      inf.loss_last = l;
    }
    if (e == cfg->epochs) break;
    STCHK(mlp_backward(c, c->d_X, c->d_dY, n, c->d_g));
    Timer t(c, "mlp");
    HIPCHK(c, launch_adam(kNParam, cfg->lr, 0.9f, 0.999f, 1e-8f, ++c->mlp_t, c->d_g, c->d_am, c->d_av, c->d_mw, s));
  }
  if (c->mlp_on) STCHK(mlp_refresh(c));
  HIPCHK(c, hipStreamSynchronize(s));
  if (info) *info = inf;
  return worst;
}

fbim_status fbim_mlp_use(fbim_ctx *c, int32_t on) {
  if (!c) return FBIM_EINVAL;
  if (on && !c->mlp_init) return fail(c, FBIM_EINVAL, "fbim_mlp_init first");
  c->mlp_on = on != 0;
  if (c->mlp_on && c->have_bodies) STCHK(mlp_refresh(c));
  return FBIM_OK;
}

fbim_status fbim_set_timing(fbim_ctx *c, int32_t enable) {
  if (!c) return FBIM_EINVAL;
  resolve_timing(c);
  c->acc.clear();
  c->timing = enable != 0;
  return FBIM_OK;
}

fbim_status fbim_kernel_time(fbim_ctx *c, const char *name, double *ms, int64_t *count) {
  if (!c || !name || !ms || !count) return FBIM_EINVAL;
  resolve_timing(c);
  auto it = c->acc.find(name);
  *ms = it == c->acc.end() ? 0.0 : it->second.first;
  *count = it == c->acc.end() ? 0 : it->second.second;
  return FBIM_OK;
}

}  // extern "C"
