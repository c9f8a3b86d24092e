"""FP64 oracle for the FBIM hot path (test infrastructure only).

Plain, slow definitions following the paper (arXiv:1709.01480):

  geometry            nodes x_{b,j} = q_b + R(theta_b) gamma(s_j), s_j = j ds
                      (Section 3.1); starfish gamma (Section 4.4.1)
  K, K^T              rigid-motion map and its trapezoid adjoint (Section 3.1)
  parameters          xi, r_c, M, P, Gaussian shape (Section 3.2, eq. 3.26)
  G^(r), G^(w)        Hasimoto split of the periodic Stokeslet
                      (eqs. 3.13-3.16); G^(w) as the plain k-sum
  M = M^(t)+M^(a)+M^(w)  single-layer matrix (eqs. 3.17-3.20): trapezoid
                      pairs inside the cutoff, Alpert correction built per body
                      directly (no rotation shortcut) and symmetrised
                      (Section 3.3), all k-space pairs including m = n
  mobility            dense saddle-point solve (eq. 3.8) -> U, mu
  M^(r)^(1/2) W       G^+ (G M^(r) G^T)^(1/2) W with G from the reference body
                      (eqs. 3.38-3.42), dense eigen square root
  (M^(w))^(1/2) W     the spreading / FFT / multiplier / interpolation steps of
                      eq. 3.30 in the paper's order
  EM-RFD step         eq. 4.3

Layout shared with the device library: node vectors are 2N long with (x, y)
interleaved per node, bodies in order, nodes j = 0..N_p-1 within a body;
body vectors are 3n long, (u_x, u_y, omega) per body.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .alpert import alpert_rule, lagrange_stencil
from .special import e1

C_R = 100.0   # real-space error constant (Section 3.2)
C_W = 1.0     # wave-space error constant (Section 3.2)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
@dataclass
class Shape:
    r_s: float
    b: float
    n_arm: int
    n_p: int

    def gamma(self, s):
        """Reference curve (theta = 0, tracking point at the origin)."""
        s = np.asarray(s, dtype=np.float64)
        r = self.r_s * (1.0 + self.b * np.cos(self.n_arm * s))
        return np.stack([r * np.cos(s), r * np.sin(s)], axis=-1)


@dataclass
class Geometry:
    L: float
    shapes: list          # list[Shape]
    shape_id: np.ndarray  # (n,)
    q: np.ndarray         # (n, 2)
    theta: np.ndarray     # (n,)

    @property
    def n(self):
        return len(self.theta)

    def offsets(self):
        npb = np.array([self.shapes[s].n_p for s in self.shape_id])
        return np.concatenate([[0], np.cumsum(npb)])

    @property
    def N(self):
        return int(self.offsets()[-1])


def geometry_from_workload(wl) -> Geometry:
    sh = Shape(wl.r_s, wl.b, wl.n_arm, wl.n_p)
    return Geometry(wl.L, [sh], np.zeros(wl.n_bodies, dtype=int),
                    np.array(wl.q, dtype=np.float64), np.array(wl.theta, dtype=np.float64))


def rot(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def body_points(geo: Geometry, b: int, s):
    """Points gamma_b(s) = q_b + R(theta_b) gamma(s) (not wrapped)."""
    sh = geo.shapes[geo.shape_id[b]]
    return geo.q[b] + sh.gamma(s) @ rot(geo.theta[b]).T


def nodes(geo: Geometry):
    """Node positions X (N, 2) (not wrapped) and the body index of each node."""
    X, body = [], []
    for b in range(geo.n):
        sh = geo.shapes[geo.shape_id[b]]
        s = 2 * np.pi * np.arange(sh.n_p) / sh.n_p
        X.append(body_points(geo, b, s))
        body.append(np.full(sh.n_p, b))
    return np.concatenate(X), np.concatenate(body)


def K_matrix(geo: Geometry):
    """Dense K (2N x 3n): (K U)_{b,j} = u_b + omega_b x (x_{b,j} - q_b),
    with omega x r = omega (-r_y, r_x) in two dimensions."""
    X, body = nodes(geo)
    N, n = len(X), geo.n
    K = np.zeros((2 * N, 3 * n))
    for i in range(N):
        b = body[i]
        r = X[i] - geo.q[b]
        K[2 * i, 3 * b] = 1.0
        K[2 * i + 1, 3 * b + 1] = 1.0
        K[2 * i, 3 * b + 2] = -r[1]
        K[2 * i + 1, 3 * b + 2] = r[0]
    return K


# ----------------------------------------------------------------------------
# parameters (Section 3.2)
# ----------------------------------------------------------------------------
def derive_params(L, eps, n_box=0, grid_M=0, xi=0.0, P=0):
    """Choose r_c, xi, M, P and the Gaussian shape from the truncation estimates
    C_r exp(-xi^2 r_c^2) <= eps, C_w exp(-k_max^2 / 4 xi^2) <= eps and
    exp(-pi P / 2) <= eps, with r_c = L / N_box and m = sqrt(pi P).
    If the grid is fixed first, N_box is the largest box count whose xi still
    meets the wave-space estimate."""
    lr = math.sqrt(math.log(C_R / eps))
    lw = math.sqrt(math.log(C_W / eps))
    if xi == 0.0:
        if n_box == 0:
            if grid_M == 0:
                raise ValueError("need one of n_box, grid_M, xi")
            xi_max = (math.pi * grid_M / L) / (2 * lw)
            n_box = int(math.floor(L * xi_max / lr))
        xi = lr * n_box / L
    if n_box == 0:
        n_box = int(math.floor(L * xi / lr))
    if n_box < 2:
        raise ValueError("cutoff would exceed half the box (N_box < 2)")
    r_c = L / n_box
    if grid_M == 0:
        kmax = 2 * xi * lw
        grid_M = int(math.ceil(kmax * L / math.pi))
        grid_M += grid_M % 2
    if P == 0:
        P = int(math.ceil(2 * math.log(1 / eps) / math.pi))
        P += 1 - P % 2
    h = L / grid_M
    w = P * h / 2
    m = math.sqrt(math.pi * P)
    eta_s = (2 * w * xi / m) ** 2
    return dict(L=L, eps=eps, n_box=n_box, r_c=r_c, xi=xi, grid_M=grid_M, P=P,
                h=h, eta_s=eta_s)


# ----------------------------------------------------------------------------
# Ewald-split Stokeslet kernels (eqs. 3.13-3.16)
# ----------------------------------------------------------------------------
def G_real(r, xi, eta=1.0):
    """G^(r)(r) = 1/(4 pi eta) [ E1(xi^2 r^2)/2 I + (r r^T / r^2 - I) exp(-xi^2 r^2) ];
    r has shape (..., 2), result (..., 2, 2)."""
    r = np.asarray(r, dtype=np.float64)
    r2 = np.sum(r * r, axis=-1)
    z = xi * xi * r2
    a = 0.5 * e1(z)
    ez = np.exp(-z)
    rr = r[..., :, None] * r[..., None, :] / r2[..., None, None]
    I = np.eye(2)
    return (a[..., None, None] * I + (rr - I) * ez[..., None, None]) / (4 * np.pi * eta)


def hasimoto(k2, xi):
    u = k2 / (4 * xi * xi)
    return (1 + u) * np.exp(-u)


def wave_vectors(L, xi, u_max=40.0):
    """All k = 2 pi kappa / L != 0 with k^2 / 4 xi^2 <= u_max (terms beyond are
    below e^-40 relative)."""
    kmax = 2 * xi * math.sqrt(u_max)
    kap = int(math.ceil(kmax * L / (2 * np.pi)))
    g = np.arange(-kap, kap + 1)
    KX, KY = np.meshgrid(g, g, indexing="ij")
    kv = 2 * np.pi / L * np.stack([KX.ravel(), KY.ravel()], axis=-1)
    k2 = np.sum(kv * kv, axis=-1)
    keep = (k2 > 0) & (k2 <= kmax * kmax)
    return kv[keep], k2[keep]


def wave_multiplier(kv, k2, xi, L, eta=1.0):
    """B(k) entries (xx, xy, yy) including the 1/(eta V) factor of eq. 3.14."""
    s = hasimoto(k2, xi) / k2 / (eta * L * L)
    return np.stack([s * (1 - kv[:, 0] ** 2 / k2), s * (-kv[:, 0] * kv[:, 1] / k2),
                     s * (1 - kv[:, 1] ** 2 / k2)], axis=-1)


def G_wave_direct(r, xi, L, eta=1.0):
    """G^(w)(r) as the plain k-sum of eq. 3.14 (real, even in r)."""
    kv, k2 = wave_vectors(L, xi)
    B = wave_multiplier(kv, k2, xi, L, eta)
    r = np.atleast_2d(r)
    c = np.cos(r @ kv.T)  # e^{-i k.r} summed over +-k is real
    out = np.empty((len(r), 2, 2))
    out[:, 0, 0] = c @ B[:, 0]
    out[:, 0, 1] = out[:, 1, 0] = c @ B[:, 1]
    out[:, 1, 1] = c @ B[:, 2]
    return out


def min_image(d, L):
    return d - L * np.round(d / L)


# ----------------------------------------------------------------------------
# single-layer matrix (eqs. 3.17-3.20)
# ----------------------------------------------------------------------------
def _blocks_to_dense(Gb):
    """(N, N, 2, 2) block array -> (2N, 2N)."""
    N = Gb.shape[0]
    return Gb.transpose(0, 2, 1, 3).reshape(2 * N, 2 * N)


def M_trap(X, L, xi, r_c, eta=1.0):
    """M^(t): G^(r) between distinct nodes closer than r_c (minimum image)."""
    N = len(X)
    D = min_image(X[:, None, :] - X[None, :, :], L)
    r2 = np.sum(D * D, axis=-1)
    mask = (r2 <= r_c * r_c)
    np.fill_diagonal(mask, False)
    Gb = np.zeros((N, N, 2, 2))
    Gb[mask] = G_real(D[mask], xi, eta)
    return _blocks_to_dense(Gb)


def M_wave_direct(X, L, xi, eta=1.0):
    """M^(w)_{mn} = G^(w)(x_m - x_n) for all m, n (including m = n)."""
    kv, k2 = wave_vectors(L, xi)
    B = wave_multiplier(kv, k2, xi, L, eta)
    ph = X @ kv.T
    C, S = np.cos(ph), np.sin(ph)
    N = len(X)
    out = np.zeros((N, N, 2, 2))
    for (i, j), col in (((0, 0), 0), ((0, 1), 1), ((1, 1), 2)):
        blk = (C * B[:, col]) @ C.T + (S * B[:, col]) @ S.T
        out[:, :, i, j] = blk
        if i != j:
            out[:, :, j, i] = blk
    return _blocks_to_dense(out)


def alpert_body(geo: Geometry, b: int, xi, r_c, order, eta=1.0, kernel=None):
    """Alpert correction block M^(a)_bb (2Np x 2Np), built directly for body b:
    for target t, the trapezoid pairs with 0 < |l - t| < a are removed and the
    auxiliary nodes s_t +- chi_k ds are added with kernel values evaluated
    exactly and the force density Lagrange-interpolated from the nodes."""
    if kernel is None:
        kernel = lambda r: G_real(r, xi, eta)
    sh = geo.shapes[geo.shape_id[b]]
    n_p = sh.n_p
    ds = 2 * np.pi / n_p
    chi, w, a = alpert_rule(order)
    s_nodes = ds * np.arange(n_p)
    xb = body_points(geo, b, s_nodes)
    Ma = np.zeros((n_p, n_p, 2, 2))
    for t in range(n_p):
        for k in range(len(chi)):
            for sgn in (1.0, -1.0):
                y = body_points(geo, b, np.array([s_nodes[t] + sgn * chi[k] * ds]))[0]
                Gk = kernel((xb[t] - y)[None, :])[0]
                offs, lw = lagrange_stencil(sgn * chi[k], order)
                for m in range(len(offs)):
                    # mu = phi ds: interpolating phi = mu / ds and weighting by
                    # the rule's w_k ds leaves w_k times the Lagrange weight times mu
                    Ma[t, (t + offs[m]) % n_p] += w[k] * lw[m] * Gk
        for i in range(1, a):
            for l in ((t + i) % n_p, (t - i) % n_p):
                d = xb[t] - xb[l]
                if d @ d <= r_c * r_c:
                    Ma[t, l] -= kernel(d[None, :])[0]
    return _blocks_to_dense(Ma)


def M_alpert(geo: Geometry, xi, r_c, order, eta=1.0, symmetric=True):
    """Block-diagonal M^(a), symmetrised per body (Section 3.3)."""
    N = geo.N
    off = geo.offsets()
    Ma = np.zeros((2 * N, 2 * N))
    for b in range(geo.n):
        blk = alpert_body(geo, b, xi, r_c, order, eta)
        if symmetric:
            blk = 0.5 * (blk + blk.T)
        sl = slice(2 * off[b], 2 * off[b + 1])
        Ma[sl, sl] = blk
    return Ma


def single_layer(geo: Geometry, prm: dict, order=4, eta=1.0):
    """Dense parts of M: dict with Mt, Ma (symmetrised), Mw, Mr = Mt + Ma, M."""
    X, _ = nodes(geo)
    Mt = M_trap(X, geo.L, prm["xi"], prm["r_c"], eta)
    Ma = M_alpert(geo, prm["xi"], prm["r_c"], order, eta)
    Mw = M_wave_direct(X, geo.L, prm["xi"], eta)
    return dict(Mt=Mt, Ma=Ma, Mw=Mw, Mr=Mt + Ma, M=Mt + Ma + Mw)


# ----------------------------------------------------------------------------
# mobility (eq. 3.8) and body mobility (eq. 3.9)
# ----------------------------------------------------------------------------
def saddle_solve(M, K, F, slip=None):
    """Solve [M -K; -K^T 0][mu; U] = -[slip; F] densely; returns (U, mu)."""
    N2, n3 = K.shape
    A = np.block([[M, -K], [-K.T, np.zeros((n3, n3))]])
    rhs = -np.concatenate([np.zeros(N2) if slip is None else slip, F])
    sol = np.linalg.solve(A, rhs)
    return sol[N2:], sol[:N2]


def body_mobility(M, K):
    """N = (K^T M^-1 K)^-1 (eq. 3.9)."""
    return np.linalg.inv(K.T @ np.linalg.solve(M, K))


# ----------------------------------------------------------------------------
# Brownian slip: real-space part (eqs. 3.38-3.42)
# ----------------------------------------------------------------------------
def sym_funcs(A, tau):
    """Eigen-decompose a symmetric matrix and return (V, lam, keep) where keep
    marks eigenvalues above tau * max(lam); the others are treated as spurious."""
    lam, V = np.linalg.eigh(0.5 * (A + A.T))
    keep = lam > tau * lam.max()
    return V, lam, keep


def reference_geometry(sh: Shape, L):
    return Geometry(L, [sh], np.zeros(1, dtype=int), np.array([[0.5 * L, 0.5 * L]]),
                    np.zeros(1))


def G_reference(sh: Shape, L, prm, order, tau, eta=1.0):
    """Symmetric preconditioner for the reference body:
    G_ref = V (Sigma^+)^(1/2) V^T, G_ref^+ = V Sigma^(1/2) V^T with
    Sigma from M^(r)_ref and spurious eigenvalues set to zero."""
    geo = reference_geometry(sh, L)
    X, _ = nodes(geo)
    Mr = M_trap(X, L, prm["xi"], prm["r_c"], eta) + M_alpert(geo, prm["xi"], prm["r_c"], order, eta)
    V, lam, keep = sym_funcs(Mr, tau)
    s_inv = np.where(keep, 1.0 / np.sqrt(np.where(keep, lam, 1.0)), 0.0)
    s = np.where(keep, np.sqrt(np.where(keep, lam, 0.0)), 0.0)
    return (V * s_inv) @ V.T, (V * s) @ V.T


def block_rotation(geo: Geometry):
    N = geo.N
    off = geo.offsets()
    R = np.zeros((2 * N, 2 * N))
    for b in range(geo.n):
        Rb = rot(geo.theta[b])
        for i in range(off[b], off[b + 1]):
            R[2 * i:2 * i + 2, 2 * i:2 * i + 2] = Rb
    return R


def G_blocks(geo: Geometry, prm, order, tau, eta=1.0):
    """Block-diagonal G and G^+ with G_bb = R_b G_ref R_b^T (single shape)."""
    Gref, Gref_p = G_reference(geo.shapes[0], geo.L, prm, order, tau, eta)
    R = block_rotation(geo)
    nb = geo.n
    G = np.kron(np.eye(nb), Gref)
    Gp = np.kron(np.eye(nb), Gref_p)
    return R @ G @ R.T, R @ Gp @ R.T


def sqrt_psd(A):
    """Principal square root with negative eigenvalues clamped to zero."""
    lam, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.sqrt(np.clip(lam, 0.0, None))) @ V.T


def slip_real(Mr, G, Gp, W_r):
    """v^(r) = G^+ (G M^(r) G^T)^(1/2) W^(r) (eq. 3.38), dense."""
    return Gp @ (sqrt_psd(G @ Mr @ G.T) @ W_r)


# ----------------------------------------------------------------------------
# Spectral Ewald pieces (Section 3.2, eqs. 3.21-3.25, 3.28-3.30)
# ----------------------------------------------------------------------------
def _gauss(prm):
    xi, eta_s = prm["xi"], prm["eta_s"]
    c = 2 * xi * xi / (np.pi * eta_s)
    a = 2 * xi * xi / eta_s
    return c, a


def stencil(x, prm):
    """P nearest grid indices (periodic) and offsets to node coordinate x."""
    h, M, P = prm["h"], prm["grid_M"], prm["P"]
    i_near = np.floor(x / h + 0.5).astype(np.int64)
    idx = i_near[:, None] + np.arange(P)[None, :] - (P - 1) // 2
    d = x[:, None] - idx * h
    return np.mod(idx, M), d


def spread(X, mu, prm):
    """H_c(x_g) = sum_n mu_{n,c} g(x_g - x_n) on the M x M grid ([c][y][x])."""
    M = prm["grid_M"]
    c, a = _gauss(prm)
    Xw = np.mod(X, prm["L"])
    ix, dx = stencil(Xw[:, 0], prm)
    iy, dy = stencil(Xw[:, 1], prm)
    gx = np.exp(-a * dx * dx)
    gy = np.exp(-a * dy * dy)
    H = np.zeros((2, M, M))
    mu2 = mu.reshape(-1, 2)
    for p in range(prm["P"]):
        for q in range(prm["P"]):
            wgt = c * gx[:, p] * gy[:, q]
            for comp in range(2):
                np.add.at(H[comp], (iy[:, q], ix[:, p]), wgt * mu2[:, comp])
    return H


def interpolate(X, U, prm):
    """v_{n,c} = h^2 sum_g g(x_n - x_g) U_c(x_g)."""
    c, a = _gauss(prm)
    Xw = np.mod(X, prm["L"])
    ix, dx = stencil(Xw[:, 0], prm)
    iy, dy = stencil(Xw[:, 1], prm)
    gx = np.exp(-a * dx * dx)
    gy = np.exp(-a * dy * dy)
    out = np.zeros((len(X), 2))
    for p in range(prm["P"]):
        for q in range(prm["P"]):
            wgt = c * gx[:, p] * gy[:, q]
            for comp in range(2):
                out[:, comp] += wgt * U[comp][iy[:, q], ix[:, p]]
    return (prm["h"] ** 2 * out).ravel()


def grid_wavenumbers(prm):
    M, L = prm["grid_M"], prm["L"]
    kap = np.fft.fftfreq(M, 1.0 / M)  # 0..M/2-1, -M/2..-1
    ky, kx = np.meshgrid(2 * np.pi * kap / L, 2 * np.pi * kap / L, indexing="ij")
    return kx, ky


def wave_se(X, mu, prm, eta=1.0):
    """M^(w) mu by spreading, FFT, multiplier (with deconvolution), inverse FFT and
    interpolation; the inverse transform keeps the real part."""
    M, L, xi, eta_s = prm["grid_M"], prm["L"], prm["xi"], prm["eta_s"]
    H = spread(X, mu, prm)
    Hh = np.fft.fft2(H, axes=(1, 2)) * prm["h"] ** 2
    kx, ky = grid_wavenumbers(prm)
    k2 = kx * kx + ky * ky
    k2s = np.where(k2 > 0, k2, 1.0)
    u = k2 / (4 * xi * xi)
    s = np.where(k2 > 0, (1 + u) * np.exp(-(1 - eta_s) * u) / k2s, 0.0) / (eta * L * L)
    Fx, Fy = Hh
    Ux = s * ((1 - kx * kx / k2s) * Fx - kx * ky / k2s * Fy)
    Uy = s * (-kx * ky / k2s * Fx + (1 - ky * ky / k2s) * Fy)
    Ug = np.real(np.fft.ifft2(np.stack([Ux, Uy]), axes=(1, 2))) * M * M
    return interpolate(X, Ug, prm)


def random_field(X, W_grid, prm, eta=1.0):
    """(M^(w))^(1/2) W^(w) by eq. 3.30: W(kappa) = FFT(W_grid)/M; project and
    scale by V^-1/2 sqrt(H)/k with the spreading Gaussian divided out; inverse
    FFT (real part); interpolate.  Excludes the sqrt(2 kT / dt) factor."""
    M, L, xi, eta_s = prm["grid_M"], prm["L"], prm["xi"], prm["eta_s"]
    Wg = W_grid.reshape(2, M, M)
    Z = np.fft.fft2(Wg, axes=(1, 2)) / M
    kx, ky = grid_wavenumbers(prm)
    k2 = kx * kx + ky * ky
    k2s = np.where(k2 > 0, k2, 1.0)
    u = k2 / (4 * xi * xi)
    s = np.where(k2 > 0, np.sqrt(1 + u) * np.exp(-0.5 * (1 - eta_s) * u) / np.sqrt(k2s), 0.0)
    s = s / math.sqrt(eta * L * L)
    Zx, Zy = Z
    Ux = s * ((1 - kx * kx / k2s) * Zx - kx * ky / k2s * Zy)
    Uy = s * (-kx * ky / k2s * Zx + (1 - ky * ky / k2s) * Zy)
    Ug = np.real(np.fft.ifft2(np.stack([Ux, Uy]), axes=(1, 2))) * M * M
    return interpolate(X, Ug, prm)


# ----------------------------------------------------------------------------
# velocities and the EM-RFD step (eqs. 2.4, 3.8, 3.27, 4.3)
# ----------------------------------------------------------------------------
class DenseFBIM:
    """Everything assembled densely for one configuration (small N only)."""

    def __init__(self, geo: Geometry, prm: dict, order=4, eta=1.0, tau=1e-8):
        self.geo, self.prm, self.order, self.eta, self.tau = geo, prm, order, eta, tau
        self.X, _ = nodes(geo)
        self.mats = single_layer(geo, prm, order, eta)
        self.K = K_matrix(geo)

    def mobility(self, F, slip=None):
        return saddle_solve(self.mats["M"], self.K, F, slip)

    def real_root(self):
        """A_r = G^+ (G M^(r) G^T)^(1/2), the dense map W^(r) -> v^(r) of eq. 3.38
        (computed once per configuration)."""
        if not hasattr(self, "_Ar"):
            G, Gp = G_blocks(self.geo, self.prm, self.order, self.tau, self.eta)
            self._Ar = Gp @ sqrt_psd(G @ self.mats["Mr"] @ G.T)
        return self._Ar

    def slip(self, W_r, W_grid, kT, dt):
        """v = sqrt(2 kT / dt) (v^(r) + v^(w)) (eq. 3.27) with independent W^(r), W^(w)."""
        vr = self.real_root() @ W_r
        vw = random_field(self.X, W_grid, self.prm, self.eta)
        return math.sqrt(2 * kT / dt) * (vr + vw), vr, vw

    def brownian_velocity(self, F, W_r, W_grid, kT, dt):
        slip, _, _ = self.slip(W_r, W_grid, kT, dt)
        U, _ = self.mobility(F, slip)
        return U


def moved(geo: Geometry, dQ):
    dQ = dQ.reshape(-1, 3)
    return Geometry(geo.L, geo.shapes, geo.shape_id, geo.q + dQ[:, :2], geo.theta + dQ[:, 2])


def em_rfd_step(geo: Geometry, prm, F, W_r, W_grid, W_tilde, kT, dt, delta, order=4,
                eta=1.0, tau=1e-8):
    """Displacement of one Euler-Maruyama step with the centred random finite
    difference drift (eq. 4.3):
      dQ = dt U0 + dt kT/delta [N(Q + delta/2 Wt) Wt - N(Q - delta/2 Wt) Wt]
    with U0 = N F + sqrt(2 kT/dt) N^(1/2) W from the saddle solve with slip.
    delta = 0: the scheme without the drift term, dQ = dt U0 (Section 4.4.1)."""
    U0 = DenseFBIM(geo, prm, order, eta, tau).brownian_velocity(F, W_r, W_grid, kT, dt)
    if delta == 0:
        return dt * U0, U0, None, None
    h = 0.5 * delta * W_tilde
    Up, _ = DenseFBIM(moved(geo, h), prm, order, eta, tau).mobility(W_tilde)
    Um, _ = DenseFBIM(moved(geo, -h), prm, order, eta, tau).mobility(W_tilde)
    return dt * U0 + dt * kT / delta * (Up - Um), U0, Up, Um


def ab2_rfd_step(geo: Geometry, prm, F, W_r, W_grid, W_tilde, kT, dt, delta, NF_prev=None, order=4,
                 eta=1.0, tau=1e-8):
    """Displacement of one step of the stochastic Adams-Bashforth scheme with the
    random finite difference (Section 4.4, the AB2-RFD equation):
      dQ = dt (3/2 N^n F^n - 1/2 N^(n-1) F^(n-1)) + sqrt(2 kT dt) (N^n)^(1/2) W
           + dt kT/delta [N(Q + delta/2 Wt) Wt - N(Q - delta/2 Wt) Wt],
    where sqrt(2 kT dt) N^(1/2) W = dt times the response to the slip alone
    (eq. 3.27) and the deterministic and stochastic velocities are separate solves.
    NF_prev = None: the first step, where N^(n-1) F^(n-1) is taken as N^n F^n.
    delta = 0 drops the drift term.  Returns (dQ, N^n F^n)."""
    D = DenseFBIM(geo, prm, order, eta, tau)
    NF, _ = D.mobility(F)
    slip, _, _ = D.slip(W_r, W_grid, kT, dt)
    Us, _ = D.mobility(np.zeros_like(F), slip)
    prev = NF if NF_prev is None else NF_prev
    dQ = dt * (1.5 * NF - 0.5 * prev) + dt * Us
    if delta != 0:
        h = 0.5 * delta * W_tilde
        Up, _ = DenseFBIM(moved(geo, h), prm, order, eta, tau).mobility(W_tilde)
        Um, _ = DenseFBIM(moved(geo, -h), prm, order, eta, tau).mobility(W_tilde)
        dQ = dQ + dt * kT / delta * (Up - Um)
    return dQ, NF
