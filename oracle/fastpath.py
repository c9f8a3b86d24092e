"""FP64 CPU fast path of the single-layer matvec (TEST INFRASTRUCTURE ONLY):
the CPU baseline the GPU is timed beside, for suspensions where the direct
sums of oracle/direct.py are out of reach.

Same operator as the oracle, M mu = M^(t) mu + M^(a) mu + M^(w) mu
(eqs. 3.17-3.20), computed with

  M^(t)  the real-space sum over a cell list (cells of side >= r_c, 3 x 3
         neighbourhood, OpenMP; oracle/direct.c);
  M^(a)  the Alpert correction of the reference body, built once per shape by
         oracle/fbim.py and applied to every body as R_b A_ref R_b^T: the
         correction only involves the body's own points, and G^(r) is
         rotation covariant, G(R r) = R G(r) R^T (Section 3.3);
  M^(w)  spectral Ewald (Section 3.2): Gaussian spreading and interpolation in C
         (OpenMP), FFTs by scipy.fft on all cores, the multiplier of eq. 3.28
         with the Gaussian divided out, in the oracle's order.

Validated against the direct oracle (oracle/direct.py, oracle/fbim.py) by the
CPU tests; nothing here is tuned beyond the cell list and the shared Alpert
block, and it shares no code with the HIP library.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft

from . import direct as D
from . import fbim as F


def _workers():
    return os.cpu_count() or 1


class FastFBIM:
    """One configuration with a single body shape."""

    def __init__(self, geo: F.Geometry, prm: dict, order=4, eta=1.0):
        if len(geo.shapes) != 1:
            raise ValueError("one body shape")
        self.geo, self.prm, self.order, self.eta = geo, prm, order, eta
        self.X, _ = F.nodes(geo)
        self.n_p = geo.shapes[0].n_p
        ref = F.reference_geometry(geo.shapes[0], geo.L)
        blk = F.alpert_body(ref, 0, prm["xi"], prm["r_c"], order, eta)
        self.A_ref = 0.5 * (blk + blk.T)
        c, s = np.cos(geo.theta), np.sin(geo.theta)
        self.R = np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)  # [n, 2, 2]
        M = prm["grid_M"]
        kap = np.fft.fftfreq(M, 1.0 / M)
        ky, kx = np.meshgrid(2 * np.pi * kap / geo.L, 2 * np.pi * kap / geo.L, indexing="ij")
        k2 = kx * kx + ky * ky
        k2s = np.where(k2 > 0, k2, 1.0)
        u = k2 / (4 * prm["xi"] ** 2)
        sc = np.where(k2 > 0, (1 + u) * np.exp(-(1 - prm["eta_s"]) * u) / k2s, 0.0) / (eta * geo.L ** 2)
        # the multiplier on the half spectrum of the real transforms
        h = M // 2 + 1
        self.Bxx = (sc * (1 - kx * kx / k2s))[:, :h]
        self.Bxy = (-sc * kx * ky / k2s)[:, :h]
        self.Byy = (sc * (1 - ky * ky / k2s))[:, :h]
        xi, eta_s = prm["xi"], prm["eta_s"]
        self.gc, self.ga = 2 * xi * xi / (math.pi * eta_s), 2 * xi * xi / eta_s

    def apply_real(self, mu):
        return D.real_space_cells(self.X, mu, self.geo.L, self.prm["xi"], self.prm["r_c"], self.eta)

    def apply_alpert(self, mu):
        n, n_p = self.geo.n, self.n_p
        m = mu.reshape(n, n_p, 2)
        body = np.einsum("bji,bpj->bpi", self.R, m).reshape(n, 2 * n_p)  # R^T mu, body frame
        out = (body @ self.A_ref.T).reshape(n, n_p, 2)
        return np.einsum("bij,bpj->bpi", self.R, out).reshape(-1)

    def apply_wave(self, mu):
        prm, L = self.prm, self.geo.L
        M, P, h = prm["grid_M"], prm["P"], prm["h"]
        H = D.spread(self.X, mu, L, h, M, P, self.gc, self.ga)
        Hh = scipy.fft.rfft2(H, axes=(1, 2), workers=_workers()) * h * h
        Ux = self.Bxx * Hh[0] + self.Bxy * Hh[1]
        Uy = self.Bxy * Hh[0] + self.Byy * Hh[1]
        Ug = scipy.fft.irfft2(np.stack([Ux, Uy]), s=(M, M), axes=(1, 2), workers=_workers()) * M * M
        return h * h * D.interp(self.X, Ug, L, h, M, P, self.gc, self.ga)

    def apply_Mr(self, mu):
        return self.apply_real(mu) + self.apply_alpert(mu)

    def apply_M(self, mu):
        return self.apply_Mr(mu) + self.apply_wave(mu)
