// Internal host-side state of a library context (fbim_ctx) and the helpers
// shared by the single-system entry points and the batched ones.
#pragma once
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "../../include/fbim.h"
#include "host_math.h"
#include "kernels.h"

namespace fbim {

struct BatchEngine;      // launch set of a batch of systems (batch_api.hip)
struct SecondKindState;  // second-kind solver state, allocated on first use (second_kind.hip)

struct ShapeDev {
  ShapeHost h;
  double *ref = nullptr, *band = nullptr, *Mp = nullptr, *Pref = nullptr, *Nt = nullptr, *G = nullptr,
         *Gp = nullptr;
};

template <class T>
hipError_t dalloc(T *&p, size_t n) {
  if (p) {
    hipFree(p);
    p = nullptr;
  }
  if (n == 0) return hipSuccess;
  return hipMalloc((void **)&p, n * sizeof(T));
}

template <class T>
void dfree(T *&p) {
  if (p) hipFree(p);
  p = nullptr;
}

struct TimedLaunch {
  hipEvent_t a, b;
};

inline bool g_rocfft_ready = false;  // rocfft_setup() done (once per process)


}  // namespace fbim

using namespace fbim;

struct fbim_ctx {
  fbim_params p{};
  Derived d{};
  int order = 4, aj = 0, aa = 0;
  double chi[8]{}, w[8]{};
  std::string err;
  hipStream_t stream = nullptr;
  int device = 0;  // HIP device current at fbim_create
  float *noalloc_scratch = nullptr;  // this device's copy of the no-allocation scratch array
  bool mixed = false;
  bool cur32 = true;  // in a mixed context: matvecs use the FP32 kernels
  int op = 0;         // operator of apply_saddle / apply_precond: 0 first kind, 1 second kind
  uint64_t geom_serial = 0;  // incremented by every geometry build
  SecondKindState *sk = nullptr;

  std::vector<ShapeDev> shapes;
  double **d_ref_arr = nullptr, **d_band_arr = nullptr, **d_Mp_arr = nullptr, **d_Pref_arr = nullptr,
         **d_Nt_arr = nullptr, **d_G_arr = nullptr, **d_Gp_arr = nullptr;
  int *d_band = nullptr, *d_np = nullptr;
  int max_np = 0;

  // geometry
  int n = 0, N = 0, capN = 0, capn = 0;
  std::vector<int> h_shape, h_off;
  std::vector<double> h_q, h_theta;
  int *d_shape = nullptr, *d_off = nullptr, *d_body = nullptr;
  // tiles of same-shape bodies for the per-body dense operators
  BodyTiles bt{};
  int4 *d_btile = nullptr;
  int *d_blist = nullptr;
  double *d_dN = nullptr;  // learned per-body correction of N_ref, [n][6]

  // learned preconditioner correction
  bool mlp_init = false, mlp_on = false;
  int mlp_sym = 1, mlp_cap = 0, mlp_t = 0;
  size_t train_cap = 0;
  float *d_mw = nullptr, *d_am = nullptr, *d_av = nullptr, *d_g = nullptr;
  float *d_X = nullptr, *d_H1 = nullptr, *d_H2 = nullptr, *d_Y = nullptr, *d_dY = nullptr, *d_Z2 = nullptr,
        *d_Z1 = nullptr, *d_ones = nullptr, *d_loss = nullptr;
  double *d_trF = nullptr, *d_trU = nullptr;
  // body cell list of the MLP features
  int *d_bc_key = nullptr, *d_bc_perm = nullptr, *d_bc_count = nullptr, *d_bc_cursor = nullptr,
      *d_bc_start = nullptr;
  size_t bc_cap_n = 0, bc_cap_c = 0;
  double *d_q = nullptr, *d_theta = nullptr, *d_x = nullptr;
  // device snapshots of (q, theta): the configuration before a move (restored when
  // the move is rejected) and the configuration at the start of a step.  d_q and
  // d_theta hold the current configuration; h_q / h_theta the one last given by
  // the caller (steps move the bodies on the device).
  double *d_qprev = nullptr, *d_thprev = nullptr, *d_qstep = nullptr, *d_thstep = nullptr;
  double *h_qpin = nullptr;  // pinned staging of caller configurations (3 capn doubles)
  int *h_pin = nullptr;      // pinned host words for small device -> host reads
  bool have_bodies = false;

  // cell list
  int ncell = 0, max_cell = 0;
  int *d_ckey = nullptr, *d_ccount = nullptr, *d_cstart = nullptr, *d_cperm = nullptr, *d_ccursor = nullptr;
  double *d_xs = nullptr;
  // tiles
  int nts = 0, ntile = 0, max_tile = 0;
  int *d_tkey = nullptr, *d_tcount = nullptr, *d_tstart = nullptr, *d_tperm = nullptr, *d_tcursor = nullptr;
  double *d_xt = nullptr;
  int *d_anchor = nullptr;
  int *d_scal_int = nullptr;  // [0] max count, [1] overlap flag
  // neighbour lists of the real-space sum
  int ngroups = 0;
  size_t ell_cap = 0;
  // spreading lists: per tile, the tile-sorted nodes whose stencil touches it
  int *d_scount = nullptr, *d_sstart = nullptr, *d_slist = nullptr;
  size_t slist_cap = 0;
  int *d_cnt_near = nullptr, *d_cnt_far = nullptr, *d_gnn = nullptr, *d_gnf = nullptr, *d_goff = nullptr,
      *d_gsize = nullptr, *d_tcell = nullptr;
  uint16_t *d_ell = nullptr;

  // matvec scratch
  double *d_mut = nullptr;
  double *d_src64 = nullptr;  // packed pair sources (x, y, mu_x, mu_y), cell order
  float *d_src32 = nullptr, *d_xt32 = nullptr, *d_mut32 = nullptr;
  double *d_grid = nullptr, *d_spec = nullptr;
  float *d_grid32 = nullptr, *d_spec32 = nullptr;
  rocfft_plan fwd = nullptr, inv = nullptr, fwd32 = nullptr, inv32 = nullptr;
  bool conv = false;  // fused transform kernels (else the rocFFT plans)
  double *d_tw = nullptr, *d_ey = nullptr;  // twiddles; Gaussian factors per frequency index
  float *d_tw32 = nullptr, *d_ey32 = nullptr;
  rocfft_execution_info einfo = nullptr;
  void *fft_work = nullptr;
  size_t fft_work_bytes = 0;
  double *d_e1tab = nullptr;
  float *d_e1tab32 = nullptr;

  // Krylov
  int restart = 100, gmres_max = 1000, lanczos_max = 200;
  size_t ntot = 0, capV = 0;
  int kn = -1;
  double *d_V = nullptr;      // (restart+1) * ntot  (also Lanczos basis)
  double *d_w = nullptr, *d_t1 = nullptr, *d_t2 = nullptr, *d_b = nullptr, *d_x2 = nullptr, *d_r = nullptr;
  double *d_partial = nullptr, *d_h = nullptr, *d_h2 = nullptr, *d_nrm = nullptr, *d_c = nullptr;
  double *d_lag = nullptr;  // lagged reorthogonalisation: dot products, then two lagged-pass outputs
  HostPub pub;  // orthogonalisation coefficients and norms read by the host
  // chunk tables of the Krylov vectors: saddle vectors (2N + 3n) and node vectors (2N)
  Segs seg_sad{}, seg_nod{};
  int2 *d_chunks = nullptr;
  int *d_chunk_sys = nullptr, *d_sys_chunk = nullptr;
  double *d_irx = nullptr, *d_irr = nullptr, *d_ird = nullptr;
  double *d_bx = nullptr, *d_by = nullptr;  // batched saddle operator: preconditioner input, operator output
  size_t cap_bxy = 0;
  fbim_ctx *rfd[2] = {nullptr, nullptr};     // copies at Q +- delta/2 Wt for batched EM-RFD solves
  fbim::BatchEngine *rfd_engine = nullptr;   // launch set of the batched EM-RFD solves
  double *d_vec_a = nullptr, *d_vec_b = nullptr, *d_U3 = nullptr, *d_U4 = nullptr, *d_U5 = nullptr,
         *d_U6 = nullptr;

  // noise drawn by the context (NULL noise arguments): draw counter and buffers
  uint64_t noise_next = 0;
  double *d_nz_r = nullptr, *d_nz_g = nullptr, *d_nz_t = nullptr;
  size_t nz_cap_r = 0, nz_cap_g = 0, nz_cap_t = 0;

  // timing
  bool timing = false;
  std::map<std::string, std::vector<TimedLaunch>> pending;
  std::map<std::string, std::pair<double, int64_t>> acc;

  WaveArgs wave() const {
    WaveArgs w;
    w.M = d.M;
    w.T = d.tile;
    w.P = d.P;
    w.nts = nts;
    w.h = d.h;
    w.L = d.L;
    w.ag = 2.0 * d.xi * d.xi / d.eta_s;
    w.cg = 2.0 * d.xi * d.xi / (kPi * d.eta_s);
    w.tile_start = d_tstart;
    w.anchor = d_anchor;
    w.slist_start = d_sstart;
    w.slist = d_slist;
    return w;
  }
  PairArgs pair_args() const {
    PairArgs a;
    a.cell_start = d_cstart;
    a.perm = d_cperm;
    a.ckey = d_ckey;
    a.tcell = d_tcell;
    a.nb = d.n_box;
    a.cell = d.L / d.n_box;
    a.rc2 = d.r_c * d.r_c;
    a.xi2 = d.xi * d.xi;
    a.cG = 1.0 / (4.0 * kPi * p.eta);
    a.e1tab = d_e1tab;
    a.e1tab32 = d_e1tab32;
    return a;
  }
  PairLists lists() const {
    PairLists pl;
    pl.N = N;
    pl.ngroups = ngroups;
    pl.cnt_near = d_cnt_near;
    pl.cnt_far = d_cnt_far;
    pl.gnn = d_gnn;
    pl.gnf = d_gnf;
    pl.goff = d_goff;
    pl.ell = d_ell;
    return pl;
  }
  GeomDev geom() const {
    GeomDev g;
    g.n = n;
    g.N = N;
    g.shape = d_shape;
    g.off = d_off;
    g.body = d_body;
    g.q = d_q;
    g.theta = d_theta;
    g.ref = d_ref_arr;
    g.np = d_np;
    return g;
  }
  BodyMats mats() const {
    BodyMats m;
    m.Mp = d_Mp_arr;
    m.Pref = d_Pref_arr;
    m.Nt = d_Nt_arr;
    m.G = d_G_arr;
    m.Gp = d_Gp_arr;
    m.max_np = max_np;
    return m;
  }
};

namespace fbim {

inline fbim_status fail(fbim_ctx *c, fbim_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, FBIM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define FFTCHK(ctx, expr)                                                                        \
  do {                                                                                           \
    rocfft_status e_ = (expr);                                                                   \
    if (e_ != rocfft_status_success)                                                             \
      return fail(ctx, FBIM_EDEVICE, std::string(#expr) + ": rocfft status " + std::to_string((int)e_)); \
  } while (0)

#define STCHK(expr)                    \
  do {                                 \
    fbim_status s_ = (expr);           \
    if (s_ != FBIM_OK) return s_;      \
  } while (0)

// RAII timing bracket of one launch class
struct Timer {
  fbim_ctx *c;
  const char *name;
  TimedLaunch t{};
  Timer(fbim_ctx *c_, const char *n_) : c(c_), name(n_) {
    if (c->timing) {
      hipEventCreate(&t.a);
      hipEventCreate(&t.b);
      hipEventRecord(t.a, c->stream);
    }
  }
  ~Timer() {
    if (c->timing) {
      hipEventRecord(t.b, c->stream);
      c->pending[name].push_back(t);
    }
  }
};

template <class T>
fbim_status upload(fbim_ctx *c, T *&dst, const std::vector<T> &src) {
  HIPCHK(c, dalloc(dst, src.size()));
  if (!src.empty()) HIPCHK(c, hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return FBIM_OK;
}

void resolve_timing(fbim_ctx *c);
inline void info_reset(fbim_info *info) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
}
inline double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// single-system operations used by the batched entry points
fbim_status random_field(fbim_ctx *c, const double *W_grid, double *out);
fbim_status lanczos_sqrt(fbim_ctx *c, const double *b, double *out, int &iters, double &change);
fbim_status norm2(fbim_ctx *c, const double *x, size_t n, double &out);
// host half of an Arnoldi step with delayed reorthogonalisation (fbim_api.hip)
bool lagged_column(int j, const double *dots, const double *out, const std::vector<double> &Hu, int m,
                   std::vector<double> &s, double &nu, double *col);
fbim_status brownian_slip(fbim_ctx *c, double dt, const double *W_r, const double *W_grid, double *slip_out,
                          fbim_info *info);
fbim_status setup_fft(fbim_ctx *c);
// move the bodies to (q_src, th_src) + a dQ (device arrays; dQ null: exactly
// there) and rebuild the geometry; a rejected move restores the previous
// configuration (device snapshot) and returns the error
fbim_status move_bodies(fbim_ctx *c, const double *q_src, const double *th_src, const double *dQ, double a);

// fills the noise arrays a call did not receive (NULL pointers; W_tilde may be
// null when the call takes none) from the context's generator at one draw
// counter, which is then advanced; the pointers are redirected to the draws
fbim_status fill_noise(fbim_ctx *c, const double *&W_r, const double *&W_grid, const double **W_tilde);
// weights and activations of the learned correction for n bodies (fbim_api.hip)
fbim_status ensure_mlp(fbim_ctx *c, int n);
// the second-kind operator [phi; U] -> [-(1/2 + D) phi + K U; U - Z phi] and the
// release of its state (second_kind.hip)
fbim_status apply_second_kind(fbim_ctx *c, const double *x, double *y);
void sk_destroy(fbim_ctx *c);

// batches (batch_api.hip)
BatchEngine *engine_new();
void engine_delete(BatchEngine *E);
const char *engine_error(const BatchEngine *E);
void engine_set_stream(BatchEngine *E, hipStream_t s);
void engine_set_flags(BatchEngine *E, uint32_t flags);
fbim_status em_rfd_batch(BatchEngine *E, const std::vector<fbim_ctx *> &mem, double dt, double delta,
                         const double *const *F, const double *const *W_r, const double *const *W_grid,
                         const double *const *W_tilde, double *const *dQ, int32_t apply, fbim_info *info);

}  // namespace fbim
