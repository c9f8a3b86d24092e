"""Seeded synthetic workloads: starfish suspensions in a periodic square box.

This module is shared by the oracle, the tests and the benchmark.  It holds
no arithmetic of the boundary-integral method itself: it only places bodies
(tracking points and angles), draws applied forces/torques and the standard
normal noise arrays the method consumes, and records the numerical
parameters of each workload.  Node positions, kernels, quadrature, solvers
and everything else are computed independently by each consumer.

Shape family (Section 4.4.1, starfish):  r(s) = r_s (1 + b cos(n_arm s)),
(x, y) = r(s) (cos s, sin s).  The paper's single-body experiments use four
arms; the suspension workloads use five.

Noise layout (shared by every consumer):
  W_r     : 2N standard normals, one per node component, body-major,
            (x, y) interleaved;
  W_grid  : 2*M*M standard normals, component-major, then row y, then x;
  W_tilde : 3n standard normals, per body (x, y, theta).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = ["Workload", "CONFIGS", "make", "noise", "noise_key", "starfish_area",
           "disk_lattice", "single_starfish", "uneven_suspensions"]


@dataclasses.dataclass
class Workload:
    name: str
    n_bodies: int
    n_p: int              # nodes per body
    r_s: float            # starfish base radius
    b: float              # arm amplitude
    n_arm: int
    L: float              # periodic box side
    tol_ewald: float
    grid_M: int = 0       # 0: derive from tol_ewald
    xi: float = 0.0       # 0: derive
    n_box: int = 0        # 0: derive
    P: int = 0            # 0: derive
    alpert_order: int = 4
    eta: float = 1.0
    kT: float = 1.0
    dt: float = 1e-3
    tol_gmres: float = 1e-6
    tol_lanczos: float = 1e-6
    tau_spurious: float = 1e-8
    placement: str = "auto"   # "rsa", "lattice" (jittered square lattice) or "auto" (lattice from 2000 bodies)
    gap: float = -1.0         # minimum gap between bounding circles / r_s (negative: two node spacings)
    # filled by make()
    q: Optional[np.ndarray] = None       # (n, 2)
    theta: Optional[np.ndarray] = None   # (n,)
    F: Optional[np.ndarray] = None       # (3n,)

    @property
    def n_nodes(self) -> int:
        return self.n_bodies * self.n_p

    @property
    def a(self) -> float:
        """Maximum radius of the starfish (characteristic length)."""
        return self.r_s * (1.0 + self.b)

    def params(self) -> dict:
        return dict(L=self.L, eta=self.eta, kT=self.kT, tol_ewald=self.tol_ewald,
                    tol_gmres=self.tol_gmres, tol_lanczos=self.tol_lanczos,
                    alpert_order=self.alpert_order, n_box=self.n_box,
                    grid_M=self.grid_M, P=self.P, xi=self.xi,
                    tau_spurious=self.tau_spurious)


def starfish_area(r_s: float, b: float) -> float:
    """Area enclosed by r = r_s (1 + b cos(n s)) for any n >= 1."""
    return math.pi * r_s * r_s * (1.0 + 0.5 * b * b)


def _box_for_fraction(n, r_s, b, phi):
    return math.sqrt(n * starfish_area(r_s, b) / phi)


def _rs_for_fraction(n, L, b, phi):
    return math.sqrt(phi * L * L / (n * math.pi * (1.0 + 0.5 * b * b)))


CONFIGS = {
    # 4 five-arm starfish, r_s = 0.05, 64 nodes each, unit box, xi = 20, grid 64^2.
    "starfish4": dict(n_bodies=4, n_p=64, r_s=0.05, b=0.3, n_arm=5, L=1.0,
                      tol_ewald=1e-9, xi=20.0, n_box=4, grid_M=64, P=15),
    # 100 five-arm starfish, r_s = 0.02, 128 nodes each, area fraction 0.2, grid 256^2.
    "starfish100": dict(n_bodies=100, n_p=128, r_s=0.02, b=0.3, n_arm=5,
                        L=_box_for_fraction(100, 0.02, 0.3, 0.2),
                        tol_ewald=1e-8, grid_M=256),
    # 10,000 five-arm starfish x 64 nodes (640k nodes), area fraction 0.3, grid 2048^2.
    # Time step of the Brownian dynamics runs: with kT = eta = 1 a body of this size has a
    # translational mobility ~0.36 and a rotational one ~9e3, so dt = 2.5e-9 moves it by
    # ~1.4% of its radius and turns it by ~7e-3 rad (RMS) per step.
    "starfish10k": dict(n_bodies=10000, n_p=64, r_s=_rs_for_fraction(10000, 1.0, 0.3, 0.3),
                        b=0.3, n_arm=5, L=1.0, tol_ewald=1e-6, grid_M=2048,
                        alpert_order=4, dt=2.5e-9),
    # dense suspensions (area fraction 0.4, bounding-circle gaps down to 0.05 r_s) for the
    # learned preconditioner: 1000 x 128 nodes, grid 1024^2, and a 200 x 64 training size
    "dense1000": dict(n_bodies=1000, n_p=128, r_s=_rs_for_fraction(1000, 1.0, 0.3, 0.4), b=0.3, n_arm=5,
                      L=1.0, tol_ewald=1e-6, grid_M=1024, alpert_order=4, placement="lattice", gap=0.05),
    "dense200": dict(n_bodies=200, n_p=64, r_s=_rs_for_fraction(200, 1.0, 0.3, 0.4), b=0.3, n_arm=5,
                     L=1.0, tol_ewald=1e-6, grid_M=256, alpert_order=4, placement="lattice", gap=0.05),
    # small cases for fast tests
    "tiny2": dict(n_bodies=2, n_p=32, r_s=0.08, b=0.3, n_arm=5, L=1.0,
                  tol_ewald=1e-8, xi=14.0, n_box=3, grid_M=48, P=13),
    "small12": dict(n_bodies=12, n_p=48, r_s=0.04, b=0.3, n_arm=5, L=1.0,
                    tol_ewald=1e-8, n_box=6, grid_M=0),
}

_SEEDS = {"starfish4": 0, "starfish100": 1, "small12": 10, "tiny2": 11,
          "starfish10k": 4, "dense1000": 3, "dense200": 12}


def _node_spacing(r_s, b, n_p):
    # largest arc length between consecutive nodes (arc speed <= r_s*(1+b*n_arm)-ish bound)
    return 2.0 * math.pi / n_p * r_s * math.sqrt((1 + b) ** 2 + (5 * b) ** 2)


def _place_rsa(rng, n, L, dmin, max_tries=2_000_000):
    """Random sequential addition of n points in the periodic box with minimum
    periodic distance dmin, accelerated by a cell grid."""
    nc = max(1, int(L // dmin))
    cell = L / nc
    grid = {}
    pts = np.empty((n, 2))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA placement failed; packing too dense")
        p = rng.uniform(0.0, L, 2)
        ci, cj = int(p[0] // cell) % nc, int(p[1] // cell) % nc
        ok = True
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for idx in grid.get(((ci + di) % nc, (cj + dj) % nc), ()):
                    d = p - pts[idx]
                    d -= L * np.round(d / L)
                    if d @ d < dmin * dmin:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[k] = p
            grid.setdefault((ci, cj), []).append(k)
            k += 1
    return pts


def _place_lattice(rng, n, L, dmin):
    """Jittered square lattice (for dense large suspensions)."""
    side = int(math.ceil(math.sqrt(n)))
    sp = L / side
    jit = 0.5 * (sp - dmin)
    if jit < 0:
        raise RuntimeError("lattice too dense for dmin")
    ij = np.array([(i, j) for j in range(side) for i in range(side)][:n], dtype=float)
    pts = (ij + 0.5) * sp + rng.uniform(-jit, jit, (n, 2))
    return np.mod(pts, L)


def make(name: str, seed: Optional[int] = None, **overrides) -> Workload:
    """Build a workload with seeded geometry and forces (geometry seed 1709+i)."""
    spec = dict(CONFIGS[name])
    spec.update(overrides)
    wl = Workload(name=name, **spec)
    s = 1709 + (_SEEDS.get(name, 99) if seed is None else seed)
    rng = np.random.default_rng(s)
    a = wl.a
    dmin = 2 * a + (2 * _node_spacing(wl.r_s, wl.b, wl.n_p) if wl.gap < 0 else wl.gap * wl.r_s)
    if wl.placement == "lattice" or (wl.placement == "auto" and wl.n_bodies >= 2000):
        wl.q = _place_lattice(rng, wl.n_bodies, wl.L, dmin)
    else:
        wl.q = _place_rsa(rng, wl.n_bodies, wl.L, dmin)
    wl.theta = rng.uniform(0.0, 2 * math.pi, wl.n_bodies)
    wl.F = rng.standard_normal(3 * wl.n_bodies)
    return wl


def uneven_suspensions(count: int, seed: int = 0, n_min: int = 16, n_max: int = 512,
                       n_ps=(64, 128, 256), phi: float = 0.2, tol: float = 1e-6) -> list:
    """Independent suspensions of uneven size for batches: bodies per suspension
    log-uniform in [n_min, n_max], nodes per body drawn from n_ps, unit box,
    area fraction phi, Ewald parameters derived from tol; suspension k uses
    geometry seed 3000 + 97 seed + k.  The cell count per side gives about 16 nodes
    per cell (at least 3); the grid is the power of two at or above the one the
    parameter rule needs for that cutoff (xi L ~ n_box sqrt(ln(C_r / tol)),
    k_max = pi M / L with exp(-k_max^2 / 4 xi^2) <= tol)."""
    rng = np.random.default_rng(0xB47C + seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n_p = int(rng.choice(n_ps))
        n_box = max(3, int(math.sqrt(n * n_p / 16.0)))
        xi = n_box * math.sqrt(math.log(100.0 / tol))
        m_need = 2.0 * xi * math.sqrt(math.log(1.0 / tol)) / math.pi
        grid_M = 1 << max(6, int(math.ceil(math.log2(m_need))))
        out.append(make("starfish4", seed=3000 + 97 * seed + k, n_bodies=n, n_p=n_p,
                        r_s=_rs_for_fraction(n, 1.0, 0.3, phi), tol_ewald=tol, xi=0.0, n_box=n_box,
                        grid_M=grid_M, P=0))
    return out


def noise_key(wl: Workload, seed: Optional[int] = None) -> int:
    """Key of the noise of workload i (0xF81A + i): numpy draws below, and the seed
    of the device generator when the library draws the noise itself."""
    return 0xF81A + (_SEEDS.get(wl.name, 99) if seed is None else seed)


def noise(wl: Workload, grid_M: int, seed: Optional[int] = None):
    """Standard normal arrays (W_r, W_grid, W_tilde); noise key 0xF81A+i."""
    rng = np.random.default_rng(noise_key(wl, seed))
    W_r = rng.standard_normal(2 * wl.n_nodes)
    W_grid = rng.standard_normal(2 * grid_M * grid_M)
    W_tilde = rng.standard_normal(3 * wl.n_bodies)
    return W_r, W_grid, W_tilde


def disk_lattice(l: float, n_p: int, tol: float = 1e-9, n_box: int = 4, a: float = 1.0) -> Workload:
    """One disk of radius a in a periodic square cell of side l (square array)."""
    wl = Workload(name="disk_lattice", n_bodies=1, n_p=n_p, r_s=a, b=0.0, n_arm=1,
                  L=l, tol_ewald=tol, n_box=n_box)
    wl.q = np.array([[0.5 * l, 0.5 * l]])
    wl.theta = np.zeros(1)
    wl.F = np.array([1.0, 0.0, 0.0])
    return wl


def starfish_pair(n_p: int = 48, tol: float = 1e-6, n_box: int = 6) -> Workload:
    """Two four-arm starfish (b = 0.3, a = 1.3 r_s = l/12) in a periodic box of side
    l = 2, tracking points 5a apart along x, angles pi/4 and pi/2 (the spring-pair
    configuration of Section 4.4.2)."""
    l = 2.0
    a = l / 12.0
    # the parameter rule asks for a 62^2 grid; 64^2 admits a spreading tile
    wl = Workload(name="starfish_pair", n_bodies=2, n_p=n_p, r_s=a / 1.3, b=0.3, n_arm=4, L=l,
                  tol_ewald=tol, n_box=n_box, grid_M=64)
    wl.q = np.array([[0.5 * l - 2.5 * a, 0.5 * l], [0.5 * l + 2.5 * a, 0.5 * l]])
    wl.theta = np.array([0.25 * math.pi, 0.5 * math.pi])
    wl.F = np.zeros(6)
    return wl


def single_starfish(theta: float = 0.0, n_p: int = 64, tol: float = 1e-7,
                    n_box: int = 3) -> Workload:
    """One four-arm starfish, b = 0.3, a = 1.3 r_s = 0.45, in the unit box."""
    wl = Workload(name="single_starfish", n_bodies=1, n_p=n_p, r_s=0.45 / 1.3, b=0.3,
                  n_arm=4, L=1.0, tol_ewald=tol, n_box=n_box)
    wl.q = np.array([[0.5, 0.5]])
    wl.theta = np.array([theta])
    wl.F = np.zeros(3)
    return wl
