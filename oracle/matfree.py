"""Matrix-free FP64 oracle of the Brownian step for suspensions too large to
assemble densely (TEST INFRASTRUCTURE ONLY).

The same definitions as oracle/fbim.py, applied without forming M:

  M mu      = M^(t) mu (direct O(N^2) real-space sum in C, eqs. 3.13-3.17)
            + M^(a) mu (per-body Alpert blocks built directly, symmetrised,
              Section 3.3)
            + M^(w) mu (spectral Ewald: spread, FFT, multiplier with the
              Gaussian divided out, inverse FFT, interpolate; Section 3.2)
  mobility  the saddle system [M -K; -K^T 0][mu; U] = -[slip; F] (eq. 3.8)
            by right-preconditioned GMRES with the paper's block-diagonal
            preconditioner built on the rotated reference block (Section 3.4)
  v^(r)     G^+ (G M^(r) G^T)^(1/2) W^(r) (eq. 3.38) with the square root
            applied by Lanczos (Section 3.3): y_k = ||w|| V_k T_k^(1/2) e_1,
            full reorthogonalisation, stop when the iterates agree to tol
  v^(w)     the random Fourier field of eq. 3.30
  step      the EM-RFD displacement of eq. 4.3

Differences from the dense oracle, both within the method's own error
budget: the wave part is the spectral-Ewald approximation (error ~ the Ewald
tolerance) instead of the plain k-sum, and the two solves stop at a residual
tolerance instead of a direct factorisation.  Pinned against DenseFBIM on
small suspensions by the CPU tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.sparse.linalg import LinearOperator

from . import direct as D
from . import fbim as F
from . import precond as P


def gmres(A, rhs, Pinv, tol=1e-10, restart=100, maxit=2000):
    """Right-preconditioned restarted GMRES(restart) with x0 = 0: each cycle
    runs P.gmres on the current true residual and adds its correction; returns
    (x, iterations, ||rhs - A x|| / ||rhs||)."""
    nb = np.linalg.norm(rhs)
    x = np.zeros_like(rhs)
    if nb == 0.0:
        return x, 0, 0.0
    its = 0
    r = rhs.copy()
    while its < maxit:
        dx, k = P.gmres(A, r, Pinv, tol=tol * nb / np.linalg.norm(r), maxit=restart)
        x += dx
        its += k
        r = rhs - A @ x
        if np.linalg.norm(r) <= tol * nb:
            break
    return x, its, np.linalg.norm(r) / nb


def lanczos_sqrt(A, w, tol=1e-10, maxit=400):
    """A^(1/2) w for symmetric positive semi-definite A (a callable), by the
    Lanczos process with full reorthogonalisation; negative Ritz values from
    round-off are clamped to zero.  Returns (y, iterations)."""
    nw = np.linalg.norm(w)
    if nw == 0.0:
        return np.zeros_like(w), 0
    V = [w / nw]
    alpha, beta = [], []
    y_old = None
    for k in range(maxit):
        v = A(V[k])
        a = V[k] @ v
        v = v - a * V[k] - (beta[-1] * V[k - 1] if k > 0 else 0.0)
        Vm = np.array(V)
        for _ in range(2):
            v = v - Vm.T @ (Vm @ v)
        alpha.append(a)
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        lam, S = np.linalg.eigh(T)
        f = S @ (np.sqrt(np.clip(lam, 0.0, None)) * S[0, :])
        y = nw * (Vm.T @ f)
        if y_old is not None and np.linalg.norm(y - y_old) <= tol * np.linalg.norm(y):
            return y, k + 1
        y_old = y
        b = np.linalg.norm(v)
        if b == 0.0:
            return y, k + 1
        beta.append(b)
        V.append(v / b)
    return y, maxit


class MatrixFreeFBIM:
    """One configuration: nodes, Alpert blocks and preconditioner built once,
    M applied matrix-free."""

    def __init__(self, geo: F.Geometry, prm: dict, order=4, eta=1.0, tau=1e-8):
        self.geo, self.prm, self.order, self.eta, self.tau = geo, prm, order, eta, tau
        self.X, _ = F.nodes(geo)
        self.N2, self.n3 = 2 * geo.N, 3 * geo.n
        self.K = F.K_matrix(geo)
        off = geo.offsets()
        self.alp = []
        for b in range(geo.n):
            blk = F.alpert_body(geo, b, prm["xi"], prm["r_c"], order, eta)
            self.alp.append((slice(2 * off[b], 2 * off[b + 1]), 0.5 * (blk + blk.T)))
        self.pinv, _ = P.reference_preconditioner(geo, prm, order=order, tau=tau, eta=eta)
        self.matvecs = 0

    def apply_Mr(self, mu):
        """M^(r) mu = M^(t) mu + M^(a) mu."""
        out = D.real_space(self.X, mu, self.geo.L, self.prm["xi"], self.prm["r_c"], eta=self.eta)
        for sl, blk in self.alp:
            out[sl] += blk @ mu[sl]
        return out

    def apply_M(self, mu):
        self.matvecs += 1
        return self.apply_Mr(mu) + F.wave_se(self.X, mu, self.prm, self.eta)

    def saddle(self):
        N2, n3, K = self.N2, self.n3, self.K

        def mv(z):
            mu, U = z[:N2], z[N2:]
            return np.concatenate([self.apply_M(mu) - K @ U, -K.T @ mu])
        return LinearOperator((N2 + n3, N2 + n3), matvec=mv, dtype=np.float64)

    def mobility(self, Fb, slip=None, tol=1e-10):
        """Solve [M -K; -K^T 0][mu; U] = -[slip; F]; returns (U, mu, iterations, relres)."""
        rhs = -np.concatenate([np.zeros(self.N2) if slip is None else slip, Fb])
        x, its, rr = gmres(self.saddle(), rhs, self.pinv, tol=tol)
        return x[self.N2:], x[:self.N2], its, rr

    def real_slip(self, W_r, tol=1e-10):
        """v^(r) = G^+ (G M^(r) G^T)^(1/2) W^(r) (eq. 3.38), G = R G_ref R^T per body."""
        Gref, Gref_p = F.G_reference(self.geo.shapes[0], self.geo.L, self.prm, self.order, self.tau, self.eta)
        off = self.geo.offsets()
        Rb = []
        for b in range(self.geo.n):
            m = off[b + 1] - off[b]
            Rb.append((slice(2 * off[b], 2 * off[b + 1]), np.kron(np.eye(m), F.rot(self.geo.theta[b]))))

        def blockwise(B, v):
            out = np.empty_like(v)
            for sl, R in Rb:
                out[sl] = R @ (B @ (R.T @ v[sl]))
            return out

        A = lambda v: blockwise(Gref, self.apply_Mr(blockwise(Gref, v)))  # noqa: E731  (G symmetric)
        y, its = lanczos_sqrt(A, W_r, tol)
        return blockwise(Gref_p, y), its

    def brownian_velocity(self, Fb, W_r, W_grid, kT, dt, tol=1e-10):
        """U = N F + sqrt(2 kT/dt) N^(1/2) W through the saddle solve with slip
        v = sqrt(2 kT/dt)(v^(r) + v^(w)) (eqs. 3.27, 3.8)."""
        vr, lits = self.real_slip(W_r, tol)
        vw = F.random_field(self.X, W_grid, self.prm, self.eta)
        slip = math.sqrt(2 * kT / dt) * (vr + vw)
        U, _, its, rr = self.mobility(Fb, slip, tol)
        return U, dict(lanczos_iters=lits, gmres_iters=its, relres=rr)


def em_rfd_step(geo: F.Geometry, prm, Fb, W_r, W_grid, W_tilde, kT, dt, delta, order=4, eta=1.0, tau=1e-8,
                tol=1e-10):
    """The EM-RFD displacement of eq. 4.3 with every solve matrix-free:
      dQ = dt U0 + dt kT/delta [N(Q + delta/2 Wt) Wt - N(Q - delta/2 Wt) Wt].
    Returns (dQ, U0, U+, U-, info)."""
    U0, info = MatrixFreeFBIM(geo, prm, order, eta, tau).brownian_velocity(Fb, W_r, W_grid, kT, dt, tol)
    h = 0.5 * delta * W_tilde
    Up, _, itp, rrp = MatrixFreeFBIM(F.moved(geo, h), prm, order, eta, tau).mobility(W_tilde, tol=tol)
    Um, _, itm, rrm = MatrixFreeFBIM(F.moved(geo, -h), prm, order, eta, tau).mobility(W_tilde, tol=tol)
    info.update(gmres_iters_rfd=(itp, itm), relres_rfd=(rrp, rrm))
    return dt * U0 + dt * kT / delta * (Up - Um), U0, Up, Um, info
