"""Completed second-kind boundary integral formulation of the periodic mobility
problem (Appendix B), dense and direct, FP64 (TEST INFRASTRUCTURE ONLY).

The exterior velocity is a double-layer potential of a density phi plus, for
every body, a Stokeslet with the body's force f and a rotlet with its torque tau
at its tracking point q (the Power-Miranda completion).  On the boundary
(jump relation) and with the closure of u and omega by phi, the unknowns
(phi, u, omega) solve

    u_b + omega_b (x - q_b)^perp = phi(x)/2 + (D phi)(x) + sum_c [G(x - q_c) f_c + R(x - q_c) tau_c]
    u_b = (1/|Gamma_b|) int phi dS,   omega_b = (1/W_b) int phi . (x - q_b)^perp dS,
    W_b = int |x - q_b|^2 dS,

with the trapezoid rule in the curve parameter.  Periodic sums (Appendix B):

  stresslet  T^(r) over images + (1/V) sum_k T^(w)(k) sin(k.(x_t - x_s)) + the
             mean term (4 pi / V) x_s,j (phi . n)_s ds_s, times 1/(4 pi eta), plus
             the trapezoid rule's diagonal entry: the kernel's limit on the curve,
             2 kappa t t^T ds for the outward normal (read from the limit; the
             printed factor is garbled).  The double layer takes the normal pointing
             into the body, the orientation for which 1/2 + D annihilates rigid
             motions (with the outward normal a constant density gives D c = c/2)
  rotlet     [R^(r) over images + (1/V) sum_k R^(w)(k) sin(k.(x_t - q))] tau / (4 pi eta):
             the wave part inside the 1/(4 pi eta), as for the stresslet (with the
             printed 1/(eta V) the two parts do not add up to a xi-independent sum;
             R^(r) is the gradient of the screened stream function
             (exp(-xi^2 r^2) - E1(xi^2 r^2))/2 and R^(w) its complement)
  Stokeslet  the periodic Stokeslet of the first-kind oracle (eqs. 3.13-3.15)

Real-space sums run over every image with xi |r| <= 6.5 and wave sums over every
k with k^2 / 4 xi^2 <= 40, so each periodic sum is exact to ~1e-15 relative
whatever xi is: xi only splits the work.  The perpendicular is taken
counterclockwise, x^perp = (-x_2, x_1), so omega and tau have the orientation of
the first-kind formulation (with the printed (x_2, -x_1) both change sign
together and N is unchanged).
"""
from __future__ import annotations

import math

import numpy as np

from . import fbim as F

REAL_CUT = 6.5   # xi |r| beyond which exp(-xi^2 r^2) < 1e-18
WAVE_UMAX = 40.0


def perp(v):
    """Counterclockwise perpendicular (-v_y, v_x)."""
    return np.stack([-v[..., 1], v[..., 0]], axis=-1)


# ----------------------------------------------------------------------------
# geometry: nodes, normals, curvature, weights
# ----------------------------------------------------------------------------
def curve_data(geo: F.Geometry):
    """Per node: position x (unwrapped), outward unit normal n, unit tangent t,
    curvature kappa, trapezoid weight ds = |gamma'(s_j)| 2 pi / N_p, and the body."""
    xs, ns, ts, ks, ws, body = [], [], [], [], [], []
    for b in range(geo.n):
        sh = geo.shapes[geo.shape_id[b]]
        s = 2 * np.pi * np.arange(sh.n_p) / sh.n_p
        m = sh.n_arm
        r = sh.r_s * (1 + sh.b * np.cos(m * s))
        r1 = -sh.r_s * sh.b * m * np.sin(m * s)
        r2 = -sh.r_s * sh.b * m * m * np.cos(m * s)
        c, si = np.cos(s), np.sin(s)
        g1 = np.stack([r1 * c - r * si, r1 * si + r * c], -1)
        g2 = np.stack([r2 * c - 2 * r1 * si - r * c, r2 * si + 2 * r1 * c - r * si], -1)
        sp = np.linalg.norm(g1, axis=-1)
        R = F.rot(geo.theta[b])
        t = (g1 / sp[:, None]) @ R.T
        n = np.stack([t[:, 1], -t[:, 0]], -1)  # outward for a counterclockwise curve
        kappa = (g1[:, 0] * g2[:, 1] - g1[:, 1] * g2[:, 0]) / sp ** 3
        xs.append(F.body_points(geo, b, s))
        ns.append(n)
        ts.append(t)
        ks.append(kappa)
        ws.append(sp * 2 * np.pi / sh.n_p)
        body.append(np.full(sh.n_p, b))
    return (np.concatenate(xs), np.concatenate(ns), np.concatenate(ts), np.concatenate(ks), np.concatenate(ws),
            np.concatenate(body))


def _images(L, xi):
    m = int(math.ceil(REAL_CUT / (xi * L))) + 1
    g = np.arange(-m, m + 1)
    P = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2) * L
    return P


def _waves(L, xi):
    return F.wave_vectors(L, xi, WAVE_UMAX)


# ----------------------------------------------------------------------------
# periodic kernels (Appendix B)
# ----------------------------------------------------------------------------
def stresslet_real(r, xi):
    """T^(r)_jlm(r; xi) for r of shape (..., 2): array (..., 2, 2, 2) [j, l, m]."""
    r2 = np.sum(r * r, -1)
    z = xi * xi * r2
    e = np.exp(-z)
    I = np.eye(2)
    rrr = r[..., :, None, None] * r[..., None, :, None] * r[..., None, None, :]
    a = (-4.0 * (1 + z) / (r2 * r2) * e)[..., None, None, None] * rrr
    b = 2 * xi * xi * e[..., None, None, None] * (I[None, :, :] * r[..., :, None, None]
                                                  + np.einsum("mj,...l->...jlm", I, r))
    return a + b


def stresslet_wave(kv, k2, xi):
    """T^(w)_jlm(k; xi): (K, 2, 2, 2) [j, l, m]."""
    I = np.eye(2)
    e = np.exp(-k2 / (4 * xi * xi))
    h = (1 + k2 / (4 * xi * xi)) * e
    kj = kv[:, :, None, None]
    kl = kv[:, None, :, None]
    km = kv[:, None, None, :]
    # k^2 (k_j delta_lm + k_l delta_mj) - 2 k_j k_l k_m
    t1 = k2[:, None, None, None] * (kj * I[None, None, :, :] + kl * I.T[None, :, None, :]) - 2 * kj * kl * km
    t2 = k2[:, None, None, None] * km * I[None, :, :, None]
    return -4 * np.pi / (k2 * k2)[:, None, None, None] * (h[:, None, None, None] * t1 + e[:, None, None, None] * t2)


def rotlet_real(r, xi):
    """R^(r)_j(r; xi) = r^perp_j / r^2 (1 - xi^2 r^2) exp(-xi^2 r^2)."""
    r2 = np.sum(r * r, -1)
    z = xi * xi * r2
    return perp(r) * ((1 - z) * np.exp(-z) / r2)[..., None]


def rotlet_wave(kv, k2, xi):
    """R^(w)_j(k; xi) = 2 pi k^perp_j / k^2 (1 + k^2/4xi^2) exp(-k^2/4xi^2)."""
    u = k2 / (4 * xi * xi)
    return 2 * np.pi * perp(kv) * ((1 + u) * np.exp(-u) / k2)[:, None]


def periodic_rotlet(r, L, xi, eta=1.0):
    """Velocity per unit torque at separations r (M, 2): (M, 2)."""
    out = np.zeros_like(r)
    for p in _images(L, xi):
        d = r + p
        d2 = np.sum(d * d, -1)
        ok = (d2 > 0) & (xi * xi * d2 <= REAL_CUT ** 2)
        out[ok] += rotlet_real(d[ok], xi) / (4 * np.pi * eta)
    kv, k2 = _waves(L, xi)
    Rw = rotlet_wave(kv, k2, xi)
    out += np.sin(r @ kv.T) @ Rw / (4 * np.pi * eta * L * L)
    return out


def periodic_stokeslet(r, L, xi, eta=1.0):
    """The periodic Stokeslet of eqs. 3.13-3.15 at separations r (M, 2): (M, 2, 2)."""
    out = np.zeros((len(r), 2, 2))
    for p in _images(L, xi):
        d = r + p
        d2 = np.sum(d * d, -1)
        ok = (d2 > 0) & (xi * xi * d2 <= REAL_CUT ** 2)
        out[ok] += F.G_real(d[ok], xi, eta)
    return out + F.G_wave_direct(r, xi, L, eta)


def double_layer_matrix(geo: F.Geometry, xi, eta=1.0):
    """D (2N x 2N): (D phi)_t = sum_s D_ts phi_s, the periodic double layer with
    the trapezoid rule, entries [2t + j, 2s + l]."""
    X, n, t, kappa, ds, _ = curve_data(geo)
    N, L, V = len(X), geo.L, geo.L ** 2
    D = np.zeros((N, 2, N, 2))
    R = X[:, None, :] - X[None, :, :]  # x_t - x_s
    # real space over images (the self pair at p = 0 is the diagonal term below)
    for p in _images(L, xi):
        d = R + p
        d2 = np.sum(d * d, -1)
        ok = (d2 > 0) & (xi * xi * d2 <= REAL_CUT ** 2)
        T = stresslet_real(d[ok], xi)  # (M, j, l, m)
        ii, jj = np.nonzero(ok)
        D[ii, :, jj, :] += np.einsum("ajlm,am->ajl", T, n[jj]) * ds[jj][:, None, None]
    # wave space: (1/V) sum_k T^(w)_jlm(k) n_m sin(k.(x_t - x_s))
    kv, k2 = _waves(L, xi)
    Tw = stresslet_wave(kv, k2, xi)  # (K, j, l, m)
    Twn = np.einsum("kjlm,sm->ksjl", Tw, n)  # (K, s, j, l)
    for c0 in range(0, len(kv), 256):
        sl = slice(c0, c0 + 256)
        S = np.sin(np.einsum("tsd,kd->kts", R, kv[sl]))  # (k, t, s)
        D += np.einsum("kts,ksjl->tjsl", S, Twn[sl]) / V * ds[None, None, :, None]
    # mean term (4 pi / V) delta_lm x_s,j S_lm
    D += (4 * np.pi / V) * np.einsum("sj,sl->jsl", X, n)[None, :, :, :] * ds[None, None, :, None]
    # trapezoid diagonal: the kernel's limit on the curve, 2 kappa t t^T (outward n)
    for s in range(N):
        D[s, :, s, :] += 2 * kappa[s] * np.outer(t[s], t[s]) * ds[s]
    # so far with the outward normal, for which a constant density gives D c = c / 2
    # on the curve; the formulation's 1/2 + D has the rigid motions in its null space,
    # i.e. its double layer takes the normal pointing into the body: the sign flips
    return -D.reshape(2 * N, 2 * N) / (4 * np.pi * eta)


def completion_matrix(geo: F.Geometry, xi, eta=1.0):
    """C (2N x 3n): velocity at every node from the periodic Stokeslet (force) and
    rotlet (torque) at every body's tracking point."""
    X, _, _, _, _, _ = curve_data(geo)
    N, n = len(X), geo.n
    C = np.zeros((N, 2, n, 3))
    for c in range(n):
        r = X - geo.q[c]
        C[:, :, c, :2] = periodic_stokeslet(r, geo.L, xi, eta)
        C[:, :, c, 2] = periodic_rotlet(r, geo.L, xi, eta)
    return C.reshape(2 * N, 3 * n)


class SecondKind:
    """The discrete completed second-kind system of one configuration."""

    def __init__(self, geo: F.Geometry, xi, eta=1.0):
        self.geo, self.xi, self.eta = geo, xi, eta
        X, n, t, kappa, ds, body = curve_data(geo)
        self.X, self.ds, self.body = X, ds, body
        N, nb = len(X), geo.n
        self.D = double_layer_matrix(geo, xi, eta)
        self.C = completion_matrix(geo, xi, eta)
        # rigid motion of the nodes: u_b + omega_b (x - q_b)^perp
        K = np.zeros((N, 2, nb, 3))
        # closure rows: u_b = (1/|Gamma_b|) sum phi ds, omega_b = (1/W_b) sum phi . (x - q_b)^perp ds
        Z = np.zeros((nb, 3, N, 2))
        for b in range(nb):
            idx = np.nonzero(body == b)[0]
            r = X[idx] - geo.q[b]
            K[idx, 0, b, 0] = 1.0
            K[idx, 1, b, 1] = 1.0
            K[idx, :, b, 2] = perp(r)
            per = ds[idx].sum()
            W = np.sum(np.sum(r * r, -1) * ds[idx])
            Z[b, 0, idx, 0] = ds[idx] / per
            Z[b, 1, idx, 1] = ds[idx] / per
            Z[b, 2, idx, :] = perp(r) * (ds[idx] / W)[:, None]
        self.K = K.reshape(2 * N, 3 * nb)
        self.Z = Z.reshape(3 * nb, 2 * N)
        # unknowns [phi; U]: rows  K U - (1/2 + D) phi = C F  and  U - Z phi = 0
        self.A = np.block([[-(0.5 * np.eye(2 * N) + self.D), self.K], [-self.Z, np.eye(3 * nb)]])

    def mobility(self, Fb, slip=None):
        """U for body forces and torques F (3n) and an optional surface slip (2N)
        added to the completion flow (u + omega r^perp = phi/2 + D phi + C F + slip);
        returns (U, phi)."""
        N2 = 2 * len(self.X)
        top = self.C @ Fb if slip is None else self.C @ Fb + slip
        rhs = np.concatenate([top, np.zeros(3 * self.geo.n)])
        sol = np.linalg.solve(self.A, rhs)
        return sol[N2:], sol[:N2]

    def body_mobility(self):
        n3 = 3 * self.geo.n
        return np.stack([self.mobility(e)[0] for e in np.eye(n3)], axis=1)


def brownian_velocity_mixed(geo, prm, F_b, W_r, W_grid, kT, dt, order=4, eta=1.0, tau=1e-8):
    """The mixed first/second-kind Brownian velocity (closing remark of Appendix B):
    the first-kind slip sqrt(2 kT/dt) (v^(r) + v^(w)) of eq. 3.27 (dense first-kind
    oracle) with the second-kind solve at the first-kind parameters' xi.
    Parity unpinned beyond its two parts: it is the composition of the pinned
    first-kind slip and the pinned second-kind solve."""
    slip, _, _ = F.DenseFBIM(geo, prm, order, eta, tau).slip(W_r, W_grid, kT, dt)
    U, _ = SecondKind(geo, prm["xi"], eta).mobility(F_b, slip)
    return U
