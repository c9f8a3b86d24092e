// Completed second-kind formulation of the mobility problem (Appendix B) and the
// mixed first/second-kind Brownian velocity (its closing remark): host side.
// The unknowns x = [phi (2N); U (3n)] use the saddle system's vector layout, so
// the context's GMRES runs on them unchanged with the operator
//   A [phi; U] = [-(1/2 + D) phi + K U;  U - Z phi]
// (Z: the closure of u and omega by phi) and no preconditioner (the second-kind
// system is well conditioned).  Right-hand side [C F + slip; 0], C F the
// completion flow of the bodies' forces and torques.
#include "ctx.h"

namespace fbim {

// declared here: defined with default arguments in fbim_api.hip
fbim_status gmres(fbim_ctx *c, const double *b, double *x, double tol, int &iters, double &relres, int maxit,
                  bool warm, double relax);

struct SecondKindState {
  uint64_t serial = ~0ull;   // geometry serial the per-node data belong to
  int capN = 0, capn = 0;
  size_t nshapes = 0;
  std::vector<double *> sk6;  // per shape [n_p][6] curve data (device)
  double **d_sk6_arr = nullptr;
  double *d_lw = nullptr;     // per shape (length, W)
  double *d_w = nullptr, *d_wc = nullptr, *d_diag = nullptr, *d_ds = nullptr, *d_r = nullptr;
  double *d_A = nullptr, *d_B = nullptr, *d_real = nullptr, *d_wave = nullptr, *d_part = nullptr,
         *d_mean = nullptr;
  double *d_grid = nullptr, *d_spec = nullptr;  // [4][M][M], [4][M][M/2+1] complex
  rocfft_plan fwd4 = nullptr, inv2 = nullptr;
  rocfft_execution_info info = nullptr;
  void *work = nullptr;
};

void sk_destroy(fbim_ctx *c) {
  SecondKindState *k = c->sk;
  if (!k) return;
  for (double *p : k->sk6) hipFree(p);
  void *ptrs[] = {k->d_sk6_arr, k->d_lw, k->d_w, k->d_wc, k->d_diag, k->d_ds, k->d_r, k->d_A, k->d_B,
                  k->d_real, k->d_wave, k->d_part, k->d_mean, k->d_grid, k->d_spec, k->work};
  for (void *p : ptrs)
    if (p) hipFree(p);
  if (k->fwd4) rocfft_plan_destroy(k->fwd4);
  if (k->inv2) rocfft_plan_destroy(k->inv2);
  if (k->info) rocfft_execution_info_destroy(k->info);
  delete k;
  c->sk = nullptr;
}

namespace {

fbim_status sk_fft_setup(fbim_ctx *c, SecondKindState *k) {
  const size_t M = c->d.M;
  HIPCHK(c, dalloc(k->d_grid, 4 * M * M));
  HIPCHK(c, dalloc(k->d_spec, 8 * M * (M / 2 + 1)));
  static bool setup_done = false;
  if (!setup_done) {
    FFTCHK(c, rocfft_setup());
    setup_done = true;
  }
  const size_t len[2] = {M, M};
  FFTCHK(c, rocfft_plan_create(&k->fwd4, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                               rocfft_precision_double, 2, len, 4, nullptr));
  FFTCHK(c, rocfft_plan_create(&k->inv2, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                               rocfft_precision_double, 2, len, 2, nullptr));
  size_t w1 = 0, w2 = 0;
  FFTCHK(c, rocfft_plan_get_work_buffer_size(k->fwd4, &w1));
  FFTCHK(c, rocfft_plan_get_work_buffer_size(k->inv2, &w2));
  FFTCHK(c, rocfft_execution_info_create(&k->info));
  const size_t wb = std::max(w1, w2);
  if (wb) {
    HIPCHK(c, hipMalloc(&k->work, wb));
    FFTCHK(c, rocfft_execution_info_set_work_buffer(k->info, k->work, wb));
  }
  return FBIM_OK;
}

// buffers, per-shape curve data and per-node data of the current configuration
fbim_status sk_prepare(fbim_ctx *c) {
  if (!c->have_bodies) return fail(c, FBIM_EINVAL, "no bodies set");
  if (!c->sk) {
    c->sk = new SecondKindState();
    fbim_status st = sk_fft_setup(c, c->sk);
    if (st != FBIM_OK) {
      sk_destroy(c);
      return st;
    }
  }
  SecondKindState *k = c->sk;
  if (k->nshapes != c->shapes.size()) {
    std::vector<double> lw;
    for (size_t s = k->nshapes; s < c->shapes.size(); ++s) {
      std::vector<double> d6;
      double len = 0, W = 0;
      const std::string e = curve_data(c->shapes[s].h.n_p, c->shapes[s].h.ref_xy.data(), d6, len, W);
      if (!e.empty()) return fail(c, FBIM_EINVAL, "second kind: " + e);
      double *p = nullptr;
      STCHK(upload(c, p, d6));
      k->sk6.push_back(p);
    }
    k->nshapes = c->shapes.size();
    for (size_t s = 0; s < c->shapes.size(); ++s) {
      std::vector<double> d6;
      double len = 0, W = 0;
      curve_data(c->shapes[s].h.n_p, c->shapes[s].h.ref_xy.data(), d6, len, W);
      lw.push_back(len);
      lw.push_back(W);
    }
    STCHK(upload(c, k->d_lw, lw));
    STCHK(upload(c, k->d_sk6_arr, k->sk6));
  }
  const int N = c->N, n = c->n;
  if (N > k->capN) {
    HIPCHK(c, dalloc(k->d_w, 2 * (size_t)N));
    HIPCHK(c, dalloc(k->d_wc, 2 * (size_t)N));
    HIPCHK(c, dalloc(k->d_diag, 3 * (size_t)N));
    HIPCHK(c, dalloc(k->d_ds, (size_t)N));
    HIPCHK(c, dalloc(k->d_r, 2 * (size_t)N));
    HIPCHK(c, dalloc(k->d_A, 2 * (size_t)N));
    HIPCHK(c, dalloc(k->d_B, 2 * (size_t)N));
    HIPCHK(c, dalloc(k->d_real, 2 * (size_t)N));
    HIPCHK(c, dalloc(k->d_wave, 2 * (size_t)N));
    k->capN = N;
  }
  if (n > k->capn) {
    HIPCHK(c, dalloc(k->d_part, 2 * (size_t)n));
    HIPCHK(c, dalloc(k->d_mean, 2));
    k->capn = n;
  }
  if (k->serial != c->geom_serial) {
    HIPCHK(c, launch_sk_geom(c->geom(), k->d_sk6_arr, c->d_cperm, k->d_w, k->d_wc, k->d_diag, k->d_ds, k->d_r,
                             c->stream));
    k->serial = c->geom_serial;
  }
  return FBIM_OK;
}

// grid planes [0..3] -> half spectra, multiplier `mode`, planes 0, 1 back, interp -> out
fbim_status sk_wave(fbim_ctx *c, int mode, double *out) {
  SecondKindState *k = c->sk;
  hipStream_t s = c->stream;
  FFTCHK(c, rocfft_execution_info_set_stream(k->info, s));
  {
    void *in[1] = {k->d_grid}, *o[1] = {k->d_spec};
    FFTCHK(c, rocfft_execute(k->fwd4, in, o, k->info));
  }
  const double sc = c->d.h * c->d.h / (c->p.eta * c->d.L * c->d.L);
  HIPCHK(c, launch_sk_mult(c->d.M, c->d.L, c->d.xi, c->d.eta_s, sc, mode, k->d_spec, s));
  {
    void *in[1] = {k->d_spec}, *o[1] = {k->d_grid};
    FFTCHK(c, rocfft_execute(k->inv2, in, o, k->info));
  }
  HIPCHK(c, launch_fill(2 * (size_t)c->N, 0.0, out, s));  // interpolation adds into out
  HIPCHK(c, launch_interp_f64(c->wave(), c->d_xt, c->d_tperm, k->d_grid, out, s));
  return FBIM_OK;
}

// b = [C F + slip; 0]
fbim_status sk_rhs(fbim_ctx *c, const double *F, const double *slip, double *b) {
  SecondKindState *k = c->sk;
  hipStream_t s = c->stream;
  const size_t twoN = 2 * (size_t)c->N, M = c->d.M;
  HIPCHK(c, launch_sk_complete_real(c->N, c->n, c->d_x, c->d_q, F, c->d.L, c->pair_args(), k->d_real, s));
  HIPCHK(c, launch_fill(4 * M * M, 0.0, k->d_grid, s));
  HIPCHK(c, launch_point_spread(c->n, c->d_q, F, c->wave(), k->d_grid, s));
  STCHK(sk_wave(c, 1, k->d_wave));
  HIPCHK(c, launch_axpby(twoN, 1.0, k->d_real, 0.0, b, s));
  HIPCHK(c, launch_axpby(twoN, 1.0, k->d_wave, 1.0, b, s));
  if (slip) HIPCHK(c, launch_axpby(twoN, 1.0, slip, 1.0, b, s));
  HIPCHK(c, launch_fill(3 * (size_t)c->n, 0.0, b + twoN, s));
  return FBIM_OK;
}

// selects the second-kind operator in apply_saddle / apply_precond for a scope
struct SecondKindOp {
  fbim_ctx *c;
  int saved;
  explicit SecondKindOp(fbim_ctx *cc) : c(cc), saved(cc->op) { c->op = 1; }
  ~SecondKindOp() { c->op = saved; }
};

}  // namespace

fbim_status apply_second_kind(fbim_ctx *c, const double *x, double *y) {
  SecondKindState *k = c->sk;
  hipStream_t s = c->stream;
  const int N = c->N;
  const size_t twoN = 2 * (size_t)N;
  const double cG = 1.0 / (4.0 * kPi * c->p.eta);
  // real space over the neighbour lists (sources gathered into the pair records)
  HIPCHK(c, launch_gather_src(N, c->d_cperm, x, c->d_src64, nullptr, s));
  HIPCHK(c, launch_dl_real(c->lists(), c->pair_args(), c->d_src64, k->d_wc, k->d_real, s));
  // wave space: the four components S_lm = phi_l w_m spread, transformed, multiplied
  const WaveArgs w = c->wave();
  const size_t MM = (size_t)c->d.M * c->d.M;
  HIPCHK(c, launch_sk_prep(N, c->d_tperm, x, k->d_w, k->d_A, k->d_B, s));
  HIPCHK(c, launch_spread_f64(w, c->d_xt, k->d_A, k->d_grid, s));
  HIPCHK(c, launch_spread_f64(w, c->d_xt, k->d_B, k->d_grid + 2 * MM, s));
  STCHK(sk_wave(c, 0, k->d_wave));
  // closure rows and the mean term, then the node rows
  const double cm = 1.0 / (c->p.eta * c->d.L * c->d.L);
  HIPCHK(c, launch_sk_body(c->geom(), k->d_lw, x, k->d_w, k->d_ds, k->d_r, x + twoN, y + twoN, k->d_part, cm,
                           k->d_mean, s));
  HIPCHK(c, launch_sk_combine(c->geom(), x, k->d_real, k->d_wave, k->d_mean, k->d_diag, cG, k->d_r, x + twoN, y,
                              s));
  return FBIM_OK;
}

}  // namespace fbim

using namespace fbim;

extern "C" {

fbim_status fbim_apply_double_layer(fbim_ctx *c, const double *phi, double *out) {
  if (!c || !phi || !out || phi == out) return fail(c, FBIM_EINVAL, "invalid arguments");
  STCHK(sk_prepare(c));
  hipStream_t s = c->stream;
  const size_t twoN = 2 * (size_t)c->N, nt = c->ntot;
  // [phi; 0] through the operator: y_phi = -(1/2 + D) phi, so D phi = -(y_phi + phi/2)
  HIPCHK(c, launch_fill(nt, 0.0, c->d_t1, s));
  HIPCHK(c, launch_axpby(twoN, 1.0, phi, 0.0, c->d_t1, s));
  STCHK(apply_second_kind(c, c->d_t1, c->d_t2));
  HIPCHK(c, launch_axpby(twoN, -1.0, c->d_t2, 0.0, out, s));
  HIPCHK(c, launch_axpby(twoN, -0.5, phi, 1.0, out, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return FBIM_OK;
}

fbim_status fbim_mobility_second_kind(fbim_ctx *c, const double *F, const double *slip, double *U,
                                      double *phi_out, fbim_info *info) {
  if (!c || !F || !U) return fail(c, FBIM_EINVAL, "invalid arguments");
  info_reset(info);
  const double t0 = now_ms();
  STCHK(sk_prepare(c));
  hipStream_t s = c->stream;
  const size_t twoN = 2 * (size_t)c->N, n3 = 3 * (size_t)c->n;
  STCHK(sk_rhs(c, F, slip, c->d_b));
  int its = 0;
  double res = 0;
  fbim_status st;
  {
    SecondKindOp op(c);
    st = gmres(c, c->d_b, c->d_x2, c->p.tol_gmres, its, res, c->gmres_max, false, 0.0);
  }
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  HIPCHK(c, hipMemcpyAsync(U, c->d_x2 + twoN, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (phi_out) HIPCHK(c, hipMemcpyAsync(phi_out, c->d_x2, twoN * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (info) {
    info->gmres_iters = its;
    info->gmres_solves = 1;
    info->gmres_residual = res;
    info->status = st;
    info->ms_total = now_ms() - t0;
  }
  return st;
}

fbim_status fbim_brownian_velocity_mixed(fbim_ctx *c, double dt, const double *F, const double *W_r,
                                         const double *W_grid, double *U, fbim_info *info) {
  if (!c || !F || !U || !(dt > 0) || !c->have_bodies) return fail(c, FBIM_EINVAL, "invalid arguments");
  info_reset(info);
  const double t0 = now_ms();
  STCHK(fill_noise(c, W_r, W_grid, nullptr));
  // the slip of the first-kind formulation (eq. 3.27), then the second-kind solve
  fbim_info si{};
  fbim_status st = brownian_slip(c, dt, W_r, W_grid, c->d_vec_a, &si);
  if (st != FBIM_OK && st != FBIM_ENOCONV) return st;
  fbim_info mi{};
  fbim_status st2 = fbim_mobility_second_kind(c, F, c->d_vec_a, U, nullptr, &mi);
  if (st2 != FBIM_OK && st2 != FBIM_ENOCONV) return st2;
  if (info) {
    *info = mi;
    info->lanczos_iters = si.lanczos_iters;
    info->lanczos_change = si.lanczos_change;
    info->status = st2 != FBIM_OK ? st2 : st;
    info->ms_total = now_ms() - t0;
  }
  return st2 != FBIM_OK ? st2 : st;
}

}  // extern "C"
