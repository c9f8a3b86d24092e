/* fbim.h -- C ABI of the MI355X (gfx950) fluctuating boundary integral library.
 *
 * The library implements the hot path of the fluctuating boundary integral
 * method (Bao, Rachh, Keaveny, Greengard, Donev, "A fluctuating boundary
 * integral method for Brownian suspensions", arXiv:1709.01480) for rigid
 * bodies in a two-dimensional periodic Stokes fluid:
 *
 *   - the single-layer matvec M mu = (M^(t) + M^(a) + M^(w)) mu of Section 3.2
 *     (Ewald split of the periodic Stokeslet, eqs. 3.13-3.20: real-space pair
 *     sum with cell lists, Alpert self-correction, and the spectral-Ewald
 *     spread / FFT / multiplier / inverse FFT / interpolate chain);
 *   - the first-kind mobility solve (saddle point system eq. 3.8) by GMRES
 *     with the block-diagonal preconditioner of Section 3.4;
 *   - the Brownian slip M^(1/2) W split as in eq. 3.27: preconditioned
 *     Lanczos for (M^(r))^(1/2) (eqs. 3.38-3.42) plus the random Fourier
 *     field (eq. 3.30);
 *   - the Euler-Maruyama random-finite-difference step (eq. 4.3).
 *
 * Conventions (all entry points):
 *   - Pointers documented as DEVICE point to memory on the GPU of the
 *     context; HOST pointers to ordinary host memory.  The caller owns every
 *     array it passes; the library keeps no pointer after a call returns.
 *   - Node vectors have 2N doubles: for body b = 0..n-1 (in the order given to
 *     fbim_set_bodies) and node j = 0..N_p-1 of that body, entries
 *     (x, y) of node j at parameter s_j = 2 pi j / N_p.
 *   - Body vectors have 3n doubles: (f_x, f_y, tau) or (u_x, u_y, omega) per
 *     body; omega x r = omega (-r_y, r_x), tau = r_x f_y - r_y f_x.
 *   - All work is enqueued on the context's stream (fbim_set_stream); calls
 *     that return solver information synchronise that stream.
 *   - Every call returns an fbim_status; on error nothing is written to the
 *     outputs unless stated, and fbim_last_error() describes the failure.
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef FBIM_H
#define FBIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FBIM_OK = 0,
  FBIM_EINVAL = 1,     /* invalid argument or parameter combination */
  FBIM_ENOMEM = 2,     /* device or host allocation failed */
  FBIM_EOVERLAP = 3,   /* bodies overlap or nodes of distinct bodies are unresolved */
  FBIM_ENOCONV = 4,    /* Krylov solver hit its iteration limit (outputs still written) */
  FBIM_EDEVICE = 5,    /* HIP / rocFFT runtime error */
  FBIM_ENOTSUP = 6,    /* unsupported option */
  FBIM_WACCURACY = 7   /* warning: r_Alpert / r_c > 0.6 (Section 4.1); context usable */
} fbim_status;

enum { FBIM_PREC_FP64 = 0, FBIM_PREC_MIXED = 1 };

/* bits of fbim_params.flags */
enum {
  /* Arnoldi / Lanczos: second Gram-Schmidt pass only when the first cancels more than
     half of ||w||^2 (default: always two passes) */
  FBIM_FLAG_SELECTIVE_REORTH = 1u,
  /* fbim_step_em_rfd: the three mobility solves in one lockstep batch (two
     internal copies of the context hold the configurations Q +- delta/2 Wt) */
  FBIM_FLAG_BATCH_RFD = 2u,
  /* with FBIM_FLAG_BATCH_RFD: replay the batch's preconditioner + saddle operator
     from a HIP graph (as FBIM_BATCH_GRAPH for batches) */
  FBIM_FLAG_GRAPH = 4u,
  /* mixed contexts: iterative refinement (FP64 residuals, FP32 GMRES corrections to
     1e-3) instead of the default relaxed-matvec GMRES (FP64 operator until the residual
     estimate falls below 1e-1 ||b||, then the FP32 operator; FP64 restart residuals) */
  FBIM_FLAG_REFINEMENT = 8u,
  /* wave-space transforms through rocFFT plans (real-to-complex, multiplier kernel,
     complex-to-real) even where the fused transform kernels apply; those serve
     power-of-two grids 64 <= M <= 2048 and every other M uses rocFFT anyway */
  FBIM_FLAG_LIBRARY_FFT = 16u,
  /* mixed contexts, batched solves (batches and FBIM_FLAG_BATCH_RFD): the GMRES
     basis is stored in FP32 (half the Gram-Schmidt traffic); projections, Hessenberg
     entries, residuals and solution updates stay FP64, and every restart residual is
     the FP64 one, so the stopping test is unchanged.  Ignored by FP64 contexts and
     by single-context solves.  Applies to a batch when all of its members set it. */
  FBIM_FLAG_BASIS32 = 32u,
  /* GMRES (single contexts; batches when all members set it): delayed
     reorthogonalisation, DCGS2 (Swirydowicz et al. 2020, Bielich et al. 2022).  The
     second Gram-Schmidt pass of each new basis vector is applied one Arnoldi step
     later, in the same read of the basis that projects the next vector, so a step
     reads the basis twice instead of three times; the Hessenberg entries are
     corrected on the host.  The Krylov dimension is then at most 32 before a restart.
     Takes precedence over FBIM_FLAG_SELECTIVE_REORTH in GMRES; Lanczos unchanged. */
  FBIM_FLAG_LAGGED_REORTH = 64u
};

/* bits of `parts` in fbim_apply_M */
enum { FBIM_PART_REAL = 1u, FBIM_PART_ALPERT = 2u, FBIM_PART_WAVE = 4u, FBIM_PART_ALL = 7u };

/* Numerical parameters (Section 3.2, eq. 3.26).  Fields set to 0 are derived:
 *   r_c = L / n_box;  C_r exp(-xi^2 r_c^2) <= tol_ewald  (C_r = 100);
 *   C_w exp(-k_max^2 / 4 xi^2) <= tol_ewald (C_w = 1, k_max = pi M / L);
 *   exp(-pi P / 2) <= tol_ewald (P odd); Gaussian shape m = sqrt(pi P),
 *   eta_s = (P h xi / m)^2 with h = L / M.
 * When the grid is given but neither n_box nor xi, n_box is the largest box
 * count whose xi still satisfies the wave-space estimate. */
typedef struct {
  double L;              /* periodic box side (> 0) */
  double eta;            /* viscosity (> 0) */
  double kT;             /* thermal energy */
  double tol_ewald;      /* Ewald / NUFFT tolerance epsilon */
  double tol_gmres;      /* GMRES relative residual ||b - A x|| <= tol ||b|| */
  double tol_lanczos;    /* Lanczos stop: ||y_k - y_{k-1}|| <= tol ||y_k|| */
  double xi;             /* Ewald splitting parameter (0: derive) */
  double tau_spurious;   /* eigenvalues <= tau * lambda_max treated as spurious (default 1e-8) */
  int32_t alpert_order;  /* 4 or 8 */
  int32_t n_box;         /* cells per side; r_c = L / n_box (0: derive); must be >= 3,
                            and xi r_c <= 8 (the real-space series covers xi^2 r^2 <= 64,
                            where the Stokeslet's real part is below 1e-28) */
  int32_t grid_M;        /* Fourier grid M (even; 0: derive) */
  int32_t P;             /* spreading support (odd; 0: derive) */
  int32_t precision;     /* FBIM_PREC_FP64 or FBIM_PREC_MIXED */
  int32_t gmres_restart; /* Krylov dimension before restart (0: 100) */
  int32_t gmres_maxiter; /* total GMRES iteration limit (0: 1000) */
  int32_t lanczos_maxiter; /* Lanczos iteration limit (0: 200) */
  int32_t tile;          /* spreading tile edge in grid points (0: choose) */
  uint32_t flags;        /* FBIM_FLAG_* bits */
  uint64_t seed;         /* key of the context's noise generator (fbim_noise_normals) */
  double tol_rfd;        /* GMRES tolerance of the two random-finite-difference solves of
                            a time step (0: tol_gmres); the paper runs them at 1e-3 with
                            1e-6 for the other solves (Section 4.4, spring-pair runs) */
} fbim_params;

/* Derived quantities reported back by fbim_get_derived. */
typedef struct {
  double xi, r_c, h, eta_s, r_alpert;
  int32_t n_box, grid_M, P, tile;
  int32_t alpert_j, alpert_a;    /* rule size and dropped-point count */
  int32_t n_bodies, n_nodes;
} fbim_derived;

/* Per-call solver report. */
typedef struct {
  int32_t gmres_iters;        /* total GMRES iterations of the call (all solves) */
  int32_t gmres_solves;
  int32_t lanczos_iters;
  int32_t status;             /* fbim_status of the last solver */
  double gmres_residual;      /* largest final true relative residual over the solves */
  double lanczos_change;      /* final relative change of the Lanczos iterate */
  double ms_total;            /* wall time of the call (host clock, stream synchronised) */
} fbim_info;

typedef struct fbim_ctx fbim_ctx;

/* Create a context on the current HIP device.  Parameters are validated and
 * derived (Section 3.2); the Alpert rule of the requested order is derived
 * from its moment conditions.  Returns FBIM_EINVAL for inconsistent values
 * (n_box < 3, odd grid, (P-1)/2 larger than a spreading tile, ...). */
fbim_status fbim_create(const fbim_params *params, fbim_ctx **out);
void fbim_destroy(fbim_ctx *ctx);
const char *fbim_last_error(const fbim_ctx *ctx);  /* never NULL */
const char *fbim_status_string(fbim_status s);

/* Stream for all subsequent work (a hipStream_t passed as void*; NULL = the
 * null stream). */
fbim_status fbim_set_stream(fbim_ctx *ctx, void *stream);

/* Add a body shape given by HOST ref_xy[2*n_p]: the node positions of the
 * reference configuration (theta = 0, tracking point at the origin) at
 * s_j = 2 pi j / n_p, j = 0..n_p-1 (Section 3.1).  Off-node points needed by
 * the Alpert rule are obtained by trigonometric interpolation of ref_xy, so
 * the curve must be resolved by its nodes.  Precomputes, in FP64 on the host,
 * the symmetrised Alpert block M^(a)_ref (Sections 3.2-3.3), the reference
 * self block M_ref and its pseudo-inverse for the block-diagonal
 * preconditioner (eqs. 3.31-3.37), and G_ref = V (Sigma^+)^(1/2) V^T,
 * G_ref^+ = V Sigma^(1/2) V^T from M^(r)_ref (eqs. 3.40-3.41, symmetric
 * reading).  n_p must be even, 16 <= n_p <= 512. */
fbim_status fbim_add_shape(fbim_ctx *ctx, int32_t n_p, const double *ref_xy, int32_t *shape_id);

/* Helper: ref_xy of the starfish r(s) = r_s (1 + b cos(n_arm s)) (Section 4.4.1). */
void fbim_starfish(double r_s, double b, int32_t n_arm, int32_t n_p, double *ref_xy);

/* Set the bodies (HOST arrays): shape_id[n], q[2n] tracking points, theta[n].
 * Builds node positions, the cell list (cells of side L/n_box) and the
 * spreading tile lists on the device.  Returns FBIM_EOVERLAP if two nodes of
 * distinct bodies are closer than 0.05 of the smaller node spacing, and
 * FBIM_EINVAL for more than 2^26 - 2 nodes or more than 4096 nodes in one
 * cutoff cell (the neighbour lists address a source by its place in its cell;
 * a larger n_box makes the cells smaller). */
fbim_status fbim_set_bodies(fbim_ctx *ctx, int32_t n, const int32_t *shape_id, const double *q,
                            const double *theta);

fbim_status fbim_get_derived(const fbim_ctx *ctx, fbim_derived *out);

/* DEVICE out[2N] <- node positions (wrapped into [0, L)^2), node order. */
fbim_status fbim_get_nodes(fbim_ctx *ctx, double *x);

/* DEVICE out[2N] = M mu (Section 3.2, eq. 3.20) restricted to `parts`
 * (FBIM_PART_REAL: trapezoid pairs within r_c, FBIM_PART_ALPERT: symmetrised
 * Alpert correction, FBIM_PART_WAVE: spectral-Ewald M^(w)).  mu, out: DEVICE,
 * 2N doubles, must not alias.  Precision follows the context: in a mixed
 * context the real-space pair sum and the wave-space part run in FP32 (the
 * mixed solver's inner operator). */
fbim_status fbim_apply_M(fbim_ctx *ctx, const double *mu, double *out, uint32_t parts);

/* DEVICE out[2N] = (M^(w))^(1/2) W^(w) by eq. 3.30 from DEVICE W_grid[2 M M]
 * standard normals laid out [component][y][x]: W(kappa) = FFT(W_grid)/M,
 * scaled by V^(-1/2) sqrt(H(k))/k (I - k k^T/k^2), inverse FFT keeping the
 * real part, Gaussian interpolation.  Excludes the sqrt(2 kT/dt) factor. */
fbim_status fbim_random_field(fbim_ctx *ctx, const double *W_grid, double *out);

/* DEVICE out[2N] = G^+ (G M^(r) G^T)^(1/2) W_r (eq. 3.38) by Lanczos with
 * full reorthogonalisation, from DEVICE W_r[2N]. */
fbim_status fbim_sqrt_Mr(fbim_ctx *ctx, const double *W_r, double *out, fbim_info *info);

/* DEVICE y[2N + 3n] = P^-1 z for DEVICE z[2N + 3n] = [a (node vector); c (body
 * vector)]: the block-diagonal preconditioner of the saddle system (Section
 * 3.4, eqs. 3.31-3.37).  Per body b, with M_bb^+ = R_b M_ref^+ R_b^T (the
 * pseudo-inverse of the body's self block, eigenvalues |lambda| <= tau
 * lambda_max dropped) and N_b = (K_b^T M_bb^+ K_b)^-1:
 *   U_b = -N_b (c_b + K_b^T M_bb^+ a_b),  mu_b = M_bb^+ (a_b + K_b U_b);
 * with the learned correction in use (fbim_mlp_use), U_b -= C_b c_b where C_b
 * is the body's correction dN rotated into the lab frame.  z, y must not alias. */
fbim_status fbim_apply_precond(fbim_ctx *ctx, const double *z, double *y);

/* Mobility solve of eq. 3.8: [M -K; -K^T 0][mu; U] = -[slip; F].
 * DEVICE F[3n]; DEVICE slip[2N] or NULL (zero slip); DEVICE U[3n];
 * DEVICE mu_out[2N] or NULL.  FBIM_ENOCONV still writes U and mu. */
fbim_status fbim_mobility(fbim_ctx *ctx, const double *F, const double *slip, double *U,
                          double *mu_out, fbim_info *info);

/* U = N F + sqrt(2 kT/dt) N^(1/2) W (eqs. 2.4 and 3.9), with the slip
 * sqrt(2 kT/dt) (v^(r) + v^(w)) built from DEVICE W_r[2N] and W_grid[2 M M]
 * standard normals (eq. 3.27).  A NULL W_r or W_grid is drawn by the
 * context's generator (fbim_noise_normals, streams FBIM_NOISE_W_R and
 * FBIM_NOISE_W_GRID) at the draw counter fbim_noise_counter reports, which the
 * call then advances by one. */
fbim_status fbim_brownian_velocity(fbim_ctx *ctx, double dt, const double *F, const double *W_r,
                                   const double *W_grid, double *U, fbim_info *info);

/* One Euler-Maruyama step with the centred random finite difference (eq. 4.3)
 * (noise pointers that are NULL are drawn as in fbim_brownian_velocity, W_tilde
 * from stream FBIM_NOISE_W_TILDE, all at one draw counter):
 *   dQ = dt U0 + dt kT/delta [N(Q + delta/2 Wt) Wt - N(Q - delta/2 Wt) Wt]
 * with U0 from fbim_brownian_velocity at Q.  Without FBIM_FLAG_BATCH_RFD the solve
 * at Q - delta/2 Wt starts from the solution at Q + delta/2 Wt (same right-hand
 * side, configurations delta apart); every solve stops on its own true residual.  DEVICE F[3n], W_r[2N],
 * W_grid[2MM], W_tilde[3n]; DEVICE dQ[3n] = (dq_x, dq_y, dtheta) per body.
 * If apply != 0 the bodies are moved by dQ afterwards; otherwise the
 * configuration is restored to Q.  The two RFD solves stop at
 * fbim_params.tol_rfd when it is set.  delta = 0 drops the RFD term (dQ = dt U0:
 * the scheme without the stochastic drift of Section 4.4.1, whose equilibrium
 * is biased by 1 / N_theta,theta; W_tilde is then neither read nor drawn). */
fbim_status fbim_step_em_rfd(fbim_ctx *ctx, double dt, double delta, const double *F,
                             const double *W_r, const double *W_grid, const double *W_tilde,
                             double *dQ, int32_t apply, fbim_info *info);

/* One step of the Adams-Bashforth scheme with the random finite difference
 * (Section 4.4, the AB2-RFD equation):
 *   dQ = dt (3/2 N^n F^n - 1/2 N^(n-1) F^(n-1)) + sqrt(2 kT dt) (N^n)^(1/2) W
 *        + dt kT/delta [N(Q + delta/2 Wt) Wt - N(Q - delta/2 Wt) Wt],
 * computed as the EM-RFD displacement of fbim_step_em_rfd plus
 * dt/2 (N^n F^n - N^(n-1) F^(n-1)), where N^n F^n is a fourth mobility solve
 * (F alone, zero slip) at Q.  DEVICE NF_hist[3n]: on entry N^(n-1) F^(n-1) when
 * have_hist != 0 (else the step is the EM step: the usual start of the scheme);
 * on return N^n F^n for the next step.  Other arguments, noise draws, delta = 0
 * and apply as fbim_step_em_rfd. */
fbim_status fbim_step_ab2_rfd(fbim_ctx *ctx, double dt, double delta, const double *F,
                              const double *W_r, const double *W_grid, const double *W_tilde,
                              double *NF_hist, int32_t have_hist, double *dQ, int32_t apply,
                              fbim_info *info);

/* ---- Completed second-kind formulation (Appendix B) --------------------------
 * The exterior flow as a double-layer potential of a density phi plus, per body,
 * a Stokeslet with its force and a rotlet with its torque at its tracking point
 * (the Power-Miranda completion).  On the boundary, with u and omega tied to phi,
 *   u_b + omega_b (x - q_b)^perp = phi/2 + D phi + sum_c [G(x - q_c) f_c + R(x - q_c) tau_c] + slip,
 *   u_b = (1/|Gamma_b|) int phi dS,  omega_b = (1/W_b) int phi . (x - q_b)^perp dS,
 * W_b = int |x - q_b|^2 dS, trapezoid rule in the curve parameter (spectrally
 * accurate in two dimensions: the stresslet is smooth on the curve).  The
 * periodic stresslet, Stokeslet and rotlet sums are Ewald-split with the
 * context's xi: real space over the neighbour lists / cutoff r_c, wave space by
 * the spectral-Ewald steps (rocFFT), the stresslet's mean term and the
 * trapezoid diagonal 2 kappa t t^T ds.  Curve normals, tangents and curvature
 * come from trigonometric interpolation of each shape's reference nodes (either
 * orientation).  Solved by the context's GMRES (tol_gmres, restart, iteration
 * limit) without a preconditioner, FP64 in every context; ENOCONV still writes
 * the outputs.  perp is counterclockwise, (-x_2, x_1), as in fbim_mobility.
 * The first call in a configuration builds per-node curve data; the state lives
 * with the context. */
/* DEVICE F[3n] (forces, torques), slip[2N] or NULL, U[3n], phi_out[2N] or NULL. */
fbim_status fbim_mobility_second_kind(fbim_ctx *ctx, const double *F, const double *slip, double *U,
                                      double *phi_out, fbim_info *info);
/* DEVICE out[2N] = D phi (the formulation's double layer, including the mean and
 * diagonal terms), for checking the operator. */
fbim_status fbim_apply_double_layer(fbim_ctx *ctx, const double *phi, double *out);
/* The mixed first/second-kind Brownian velocity (the closing remark of Appendix
 * B): the slip sqrt(2 kT/dt) (v^(r) + v^(w)) of the first-kind formulation (as in
 * fbim_brownian_velocity: Lanczos on M^(r), random Fourier field; NULL noise drawn
 * by the generator) with the second-kind solve.  Discrete fluctuation-dissipation
 * balance holds only to the difference of the two discretisations. */
fbim_status fbim_brownian_velocity_mixed(fbim_ctx *ctx, double dt, const double *F, const double *W_r,
                                         const double *W_grid, double *U, fbim_info *info);

/* ---- Noise ----------------------------------------------------------------
 * The method consumes independent standard normals (W^(r), W^(w): Sections
 * 3.1 and 3.3; W, W~: Section 4.4).  Each context carries a counter-based
 * generator keyed by fbim_params.seed: element i of stream s at draw counter k
 * is a pure function of (seed, s, k, i), so draws are reproducible on any
 * device and in any order.  Definition: Philox4x32-10 (Salmon, Moraes, Dror,
 * Shaw, SC'11) with counter words (i / 2, s, k mod 2^32, k / 2^32) and key
 * words (seed mod 2^32, seed / 2^32) gives (x0, x1, x2, x3);
 * u1 = ((x0 2^32 + x1) / 2^11 (integer division) + 1) 2^-53 in (0, 1],
 * u2 = ((x2 2^32 + x3) / 2^11) 2^-53 in [0, 1);
 * element 2j = sqrt(-2 ln u1) cos(2 pi u2), element 2j + 1 = sqrt(-2 ln u1)
 * sin(2 pi u2) for pair j (Box-Muller).  n / 2 must stay below 2^32. */
enum { FBIM_NOISE_W_R = 0, FBIM_NOISE_W_GRID = 1, FBIM_NOISE_W_TILDE = 2 };
/* DEVICE out[n] <- standard normals of stream `stream` at draw `counter`. */
fbim_status fbim_noise_normals(fbim_ctx *ctx, uint32_t stream, uint64_t counter, size_t n, double *out);
/* DEVICE out[4 n_pairs] <- the raw Philox words (x0, x1, x2, x3) of pairs
 * j < n_pairs behind those normals (for verification of the generator). */
fbim_status fbim_noise_words(fbim_ctx *ctx, uint32_t stream, uint64_t counter, size_t n_pairs, uint32_t *out);
/* HOST *counter <- the draw counter the next call with NULL noise will use
 * (0 for a new context); fbim_set_noise_counter sets it (to resume a run). */
fbim_status fbim_noise_counter(const fbim_ctx *ctx, uint64_t *counter);
fbim_status fbim_set_noise_counter(fbim_ctx *ctx, uint64_t counter);

/* Host utility (no device needed): derive parameters as fbim_create does.
 * Writes the derived values into *out; returns FBIM_EINVAL on bad input. */
fbim_status fbim_derive_params(const fbim_params *in, fbim_derived *out);

/* Host utility: the Alpert log-singular end correction of the given order
 * (4 or 8) derived from its moment conditions (Section 3.1): j nodes chi[j]
 * and weights w[j] replacing the a - 1 trapezoid points next to the
 * singularity.  HOST chi, w must hold 8 doubles. */
fbim_status fbim_alpert_rule(int32_t order, int32_t *j, int32_t *a, double *chi, double *w);

/* ---- Batches of independent systems ------------------------------------------
 * A batch advances S independent systems (suspensions of any sizes, same
 * precision) together: every stage of the matvec (gathers, pair sum, Alpert
 * band, spreading, multiplier, interpolation), the rigid-body terms, the
 * preconditioner and the Krylov vector operations of all systems run as one
 * launch per stage, with the FFTs batched per grid size; GMRES runs in
 * lockstep, each system with its own Krylov space, Hessenberg matrix and
 * stopping test, and leaves the batch when it converges.  With
 * FBIM_BATCH_GRAPH the preconditioner + saddle-operator launch sequence of a
 * GMRES iteration is captured once into a HIP graph and replayed.
 * Members are ordinary contexts owned by the batch (fbim_batch_member): give
 * them shapes and bodies with fbim_add_shape / fbim_set_bodies; every
 * single-system call keeps working on them.  All members use the batch's
 * stream. */
typedef struct fbim_batch fbim_batch;
enum { FBIM_BATCH_GRAPH = 1u };

/* HOST params[S] (one per system).  Fails with FBIM_EINVAL if the precisions differ. */
fbim_status fbim_batch_create(int32_t S, const fbim_params *params, fbim_batch **out);
void fbim_batch_destroy(fbim_batch *batch);
const char *fbim_batch_last_error(const fbim_batch *batch);  /* never NULL */
fbim_ctx *fbim_batch_member(fbim_batch *batch, int32_t s);  /* NULL if s is out of range */
fbim_status fbim_batch_set_stream(fbim_batch *batch, void *stream);
fbim_status fbim_batch_set_flags(fbim_batch *batch, uint32_t flags);  /* FBIM_BATCH_* bits */

/* out[s] = M_s mu[s] (all parts) for every member: HOST arrays of S DEVICE
 * pointers, each 2 N_s doubles. */
fbim_status fbim_batch_apply_M(fbim_batch *batch, const double *const *mu, double *const *out);

/* Mobility solves of eq. 3.8 for every member at once: HOST arrays of S DEVICE
 * pointers F[s] (3 n_s), slip[s] (2 N_s, or NULL entries / NULL array for zero
 * slip), U[s] (3 n_s); HOST info[S] or NULL.  Returns FBIM_ENOCONV if any
 * system hit its iteration limit (all outputs still written). */
fbim_status fbim_batch_mobility(fbim_batch *batch, const double *const *F, const double *const *slip,
                                double *const *U, fbim_info *info);

/* One EM-RFD step (eq. 4.3) of every member, with the three mobility solves of
 * every member (at Q, Q + delta/2 Wt, Q - delta/2 Wt) in one batched GMRES.
 * Arguments as fbim_step_em_rfd, as HOST arrays of S DEVICE pointers; a NULL
 * noise array, or a NULL entry, is drawn by that member's generator. */
fbim_status fbim_batch_step_em_rfd(fbim_batch *batch, double dt, double delta, const double *const *F,
                                   const double *const *W_r, const double *const *W_grid,
                                   const double *const *W_tilde, double *const *dQ, int32_t apply,
                                   fbim_info *info);

/* One AB2-RFD step (fbim_step_ab2_rfd) of every member: the EM-RFD solves as in
 * fbim_batch_step_em_rfd, then the members' N^n F^n solves in one more batched
 * GMRES.  HOST arrays of S DEVICE pointers; NF_hist[s] as NF_hist of
 * fbim_step_ab2_rfd (have_hist applies to every member). */
fbim_status fbim_batch_step_ab2_rfd(fbim_batch *batch, double dt, double delta, const double *const *F,
                                    const double *const *W_r, const double *const *W_grid,
                                    const double *const *W_tilde, double *const *NF_hist, int32_t have_hist,
                                    double *const *dQ, int32_t apply, fbim_info *info);

/* ---- Learned correction of the block-diagonal preconditioner ----------------
 * A per-body MLP 32 -> 128 -> 128 -> 6 with tanh hidden layers maps features
 * of a body's neighbourhood (in its body frame) to a symmetric correction dN
 * of the isolated-body mobility N_ref that the preconditioner of Section 3.4
 * (eqs. 3.31-3.37) applies.  GMRES's true residual still decides convergence:
 * the correction changes iteration counts, not solutions.  Matrix products
 * run on the MFMA units in BF16 with FP32 accumulation; weights are FP32.
 *
 * Weights: FBIM_MLP_NPARAM floats, flat, in the order W1 (32 x 128, row-major
 * input x output), b1 (128), W2 (128 x 128), b2 (128), W3 (128 x 6), b3 (6).
 * Features (FBIM_MLP_IN per body).  Neighbours of body b are the other bodies
 * whose tracking points lie closer than R = 3 r_max (minimum image; r_max =
 * largest distance of a reference node from its tracking point over all
 * shapes), nearest first, ties by index, at most 6.  For slot k < 6 (zeros
 * when empty): [5k, 5k+1] = neighbour offset rotated into b's frame / R;
 * 5k+2 = r_max / distance; [5k+3, 5k+4] = cos, sin of sym (theta_c - theta_b).
 * 30 = neighbour count / 6; 31 = clamp((d_min - 2 r_max) / r_max, -2, 2) with
 * d_min the nearest distance (R if none).
 * Output y (6 per body) gives, in the body frame,
 *   dN = [[y0 sx, y3 sxy, y4 sxt], [y3 sxy, y1 sy, y5 syt], [y4 sxt, y5 syt, y2 st]],
 * s. the diagonal of N_ref and sxy = sqrt(sx sy), sxt = sqrt(sx st), syt = sqrt(sy st).
 * Training target: for forces with independent standard-normal components the
 * solve gives U = N F, and E[U_b F_b^T] = N_bb, so the loss
 *   mean over samples s and bodies b of sum_i (r_i / N_ref,ii)^2,
 *   r = (N_ref + dN_b) R_b^T F_b - R_b^T U_b   (R_b rotates the translational part)
 * is minimised by dN_b = N_bb - N_ref in expectation. */
#define FBIM_MLP_IN 32
#define FBIM_MLP_HID 128
#define FBIM_MLP_OUT 6
#define FBIM_MLP_NPARAM (32 * 128 + 128 + 128 * 128 + 128 + 128 * 6 + 6)

typedef struct {
  int32_t n_solves; /* random-force mobility solves on the current configuration (>= 1) */
  int32_t epochs;   /* Adam steps over those samples (>= 0) */
  float lr;         /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
  uint64_t seed;    /* forces: independent standard normals from this seed (host generator) */
} fbim_train_cfg;

typedef struct {
  float loss_first;     /* loss before the first Adam step */
  float loss_last;      /* loss after the last Adam step */
  int32_t gmres_iters;  /* GMRES iterations of the sample solves */
  int32_t samples;      /* body samples used (n_solves x bodies) */
} fbim_train_info;

/* Initialise the weights (Glorot-uniform from a host generator seeded with
 * `seed`; biases zero; last layer scaled by 1e-2 so that dN starts near 0)
 * and set the angular symmetry order used by the features (5 for a five-arm
 * starfish; 1 for a shape without rotational symmetry). */
fbim_status fbim_mlp_init(fbim_ctx *ctx, uint64_t seed, int32_t sym_order);
/* HOST w[n], n == FBIM_MLP_NPARAM. */
fbim_status fbim_mlp_set_weights(fbim_ctx *ctx, const float *w, size_t n);
fbim_status fbim_mlp_get_weights(fbim_ctx *ctx, float *w, size_t n);
/* DEVICE X[n_bodies][FBIM_MLP_IN] <- features of the current bodies. */
fbim_status fbim_mlp_features(fbim_ctx *ctx, float *X);
/* DEVICE Y[n][6] = MLP(DEVICE X[n][32]) with the current weights. */
fbim_status fbim_mlp_forward(fbim_ctx *ctx, const float *X, int32_t n, float *Y);
/* fbim_mlp_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels, with the hidden activations in a static device array of
 * 2 x 128 x FBIM_NOALLOC_MAX_BODIES floats (8 MiB) that each GPU holds for the
 * life of the process; the call itself allocates and frees nothing.
 * n <= FBIM_NOALLOC_MAX_BODIES, else FBIM_EINVAL.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other
 * host threads, other contexts) race and must be serialised by the caller.
 * Requires fbim_mlp_init (the weights are the context's). */
#define FBIM_NOALLOC_MAX_BODIES 8192
fbim_status fbim_mlp_forward_noalloc(fbim_ctx *ctx, const float *X, int32_t n, float *Y);
/* DEVICE grad[FBIM_MLP_NPARAM] = d (sum_ij dY_ij Y_ij) / d w at DEVICE X[n][32],
 * DEVICE dY[n][6] (grad is overwritten, same layout as the weights). */
fbim_status fbim_mlp_backward(fbim_ctx *ctx, const float *X, const float *dY, int32_t n, float *grad);
/* Loss above for the current bodies from DEVICE Y[n][6] and ns samples of
 * DEVICE F[ns][3n], U[ns][3n]; HOST *loss, DEVICE dY[n][6] = d loss / d Y. */
fbim_status fbim_mlp_loss(fbim_ctx *ctx, const float *Y, int32_t ns, const double *F, const double *U,
                          float *loss, float *dY);
/* Generate cfg->n_solves random-force solves on the current configuration
 * (with the preconditioner currently in use) and take cfg->epochs Adam steps
 * on the loss over them. */
fbim_status fbim_mlp_train(fbim_ctx *ctx, const fbim_train_cfg *cfg, fbim_train_info *info);
/* on != 0: the preconditioner applies N_ref + dN_b (recomputed whenever the
 * bodies change); 0: the plain block-diagonal preconditioner. */
fbim_status fbim_mlp_use(fbim_ctx *ctx, int32_t on);

/* Kernel timing (for measurement): when enabled, device events bracket each
 * launch of the named kernel class; fbim_kernel_time returns the summed
 * milliseconds and launch count since the last reset.  Classes: "pair",
 * "alpert", "spread", "interp", "fft", "multiplier", "precond", "blas", "mlp"; in a mixed
 * context the FP32 launches are counted separately as "pair32", "spread32",
 * "interp32", "fft32" and "multiplier32". */
fbim_status fbim_set_timing(fbim_ctx *ctx, int32_t enable);
fbim_status fbim_kernel_time(fbim_ctx *ctx, const char *name, double *ms, int64_t *count);

/* ---- Autotuner ----------------------------------------------------------------
 * Not a step of the paper's method: a throughput choice among parameters that
 * the method leaves free.  Times the single-layer matvec (fbim_apply_M, all
 * parts, in the context's own precision; median of 5 after 2 untimed) of the
 * context's current configuration for each candidate, on the context's stream,
 * and returns the context's parameters with the fastest admissible candidate
 * filled in (explicit n_box, grid_M, tile); the caller creates a context with
 * them.  Candidates:
 *   FBIM_TUNE_TILE   every spreading tile edge T <= 32 with T | M, M / T >= 3 and
 *                    T >= (P - 1)/2 (results agree to round-off: the spread sums
 *                    are fixed point per tile);
 *   FBIM_TUNE_SPLIT  the Ewald split of Section 3.2: n_box (r_c = L / n_box) at
 *                    0.6 ... 1.3 times the given one, each with the grid of the
 *                    parameter rule for tol_ewald and with the next power of two;
 *                    a candidate whose shapes break r_Alpert <= 0.6 r_c is not
 *                    admissible.  Results change within the Ewald tolerance.
 *                    Needs params.n_box given and grid_M = xi = 0.
 * cache_path (may be NULL): a JSON-lines file, one object per line
 *   {"key": "<key>", "n_box": ., "grid_M": ., "tile": ., "ms": .}; a line whose key
 *   matches (device architecture and compute-unit count, precision, node count,
 *   nodes per body and body count per shape, L, tolerance, Alpert order, the
 *   given grid_M / n_box / xi / P, the tuning set) is used without timing (the
 *   last such line wins; malformed lines are skipped); otherwise the choice is
 *   appended.  Host file I/O is serialised within the process.
 * The call allocates two node vectors and each candidate's context; it
 * synchronises the context's stream.  FBIM_EINVAL: no bodies set, invalid set,
 * SPLIT without a free split, or no admissible candidate. */
#define FBIM_TUNE_TILE 1u
#define FBIM_TUNE_SPLIT 2u
typedef struct {
  int32_t candidates;  /* candidates timed (0 when taken from the cache) */
  int32_t from_cache;  /* 1 when the cache answered */
  int32_t cache_error; /* 1 when the choice could not be appended to the cache */
  int32_t reserved;
  double ms_best;      /* median matvec time of the choice (cached value if from_cache) */
  double ms_default;   /* median matvec time of the context's own parameters (-1 if from_cache) */
} fbim_tune_report;
fbim_status fbim_autotune(fbim_ctx *ctx, uint32_t what, const char *cache_path, fbim_params *out,
                          fbim_tune_report *report);
/* The cache key fbim_autotune uses for ctx and `what` (NUL-terminated into
 * buf[len]; FBIM_EINVAL if it does not fit). */
fbim_status fbim_autotune_key(const fbim_ctx *ctx, uint32_t what, char *buf, int32_t len);
/* Host only: 1 and the cached choice when cache_path holds `key`, else 0. */
int32_t fbim_autotune_lookup(const char *cache_path, const char *key, int32_t *n_box, int32_t *grid_M,
                             int32_t *tile);

#ifdef __cplusplus
}
#endif
#endif /* FBIM_H */
