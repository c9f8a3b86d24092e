"""Pins of the matrix-free oracle (oracle/matfree.py) against the dense oracle
on small suspensions, and of the stored 100-starfish golden's inputs.

  - M^(r) mu matrix-free equals the assembled M^(t) + M^(a) to round-off, and
    M mu differs from the dense (plain k-sum) M only by the spectral-Ewald error;
  - the Lanczos square root reproduces the dense G^+ (G M^(r) G^T)^(1/2) W of
    eq. 3.38;
  - restarted GMRES reaches the dense saddle solution (eq. 3.8) even when each
    cycle is cut short;
  - the whole EM-RFD displacement (eq. 4.3) agrees with the dense oracle's;
  - a planted mistake (the RFD difference with delta instead of delta / 2 in the
    moved configurations) fails the comparison.
"""
import hashlib
import os

import numpy as np
import pytest

import workloads as W
from oracle import fbim as OF
from oracle import matfree as MF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "starfish100_em_rfd.txt")


def _setup(name):
    wl = W.make(name)
    prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
    return wl, OF.geometry_from_workload(wl), prm


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def tiny():
    wl, geo, prm = _setup("tiny2")
    D = OF.DenseFBIM(geo, prm, wl.alpert_order, tau=wl.tau_spurious)
    m = MF.MatrixFreeFBIM(geo, prm, wl.alpert_order, tau=wl.tau_spurious)
    return wl, geo, prm, D, m


def test_operator_parts_match_dense(tiny):
    wl, geo, prm, D, m = tiny
    mu = np.random.default_rng(3).standard_normal(2 * geo.N)
    assert _rel(m.apply_Mr(mu), D.mats["Mr"] @ mu) < 1e-13
    # spectral Ewald against the plain k-sum: the Ewald tolerance of the workload
    assert _rel(m.apply_M(mu), D.mats["M"] @ mu) < 10 * wl.tol_ewald


def test_lanczos_root_matches_dense_root(tiny):
    wl, geo, prm, D, m = tiny
    Wr, _, _ = W.noise(wl, prm["grid_M"])
    vr, its = m.real_slip(Wr, tol=1e-12)
    assert its >= 2
    assert _rel(vr, D.real_root() @ Wr) < 1e-11


def test_lanczos_sqrt_of_a_known_matrix():
    # A = Q diag(lam) Q^T: A^(1/2) w is known in closed form
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.linspace(0.1, 4.0, 60)
    A = (Q * lam) @ Q.T
    w = rng.standard_normal(60)
    y, its = MF.lanczos_sqrt(lambda v: A @ v, w, tol=1e-13)
    assert _rel(y, (Q * np.sqrt(lam)) @ (Q.T @ w)) < 1e-11


def test_restarted_gmres_reaches_dense_solution(tiny):
    wl, geo, prm, D, m = tiny
    U_ref, mu_ref = OF.saddle_solve(D.mats["M"], D.K, wl.F)
    # short cycles: the restart path must carry the solution across cycles
    rhs = -np.concatenate([np.zeros(2 * geo.N), wl.F])
    x, its, rr = MF.gmres(m.saddle(), rhs, m.pinv, tol=1e-11, restart=3)
    assert rr <= 1e-11 and its > 3
    assert _rel(x[2 * geo.N:], U_ref) < 10 * wl.tol_ewald


@pytest.mark.parametrize("name", ["tiny2", "starfish4"])
def test_step_matches_dense_oracle(name):
    wl, geo, prm = _setup(name)
    noise = W.noise(wl, prm["grid_M"])
    delta = wl.a * 1e-2
    ref, _, _, _ = OF.em_rfd_step(geo, prm, wl.F, *noise, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                  tau=wl.tau_spurious)
    dQ, _, _, _, info = MF.em_rfd_step(geo, prm, wl.F, *noise, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                       tau=wl.tau_spurious, tol=1e-11)
    assert info["relres"] <= 1e-11
    # the two differ by the spectral-Ewald error of the wave part only
    assert _rel(dQ, ref) < 1e-6


def test_planted_rfd_half_step_mistake_fails():
    wl, geo, prm = _setup("starfish4")
    noise = W.noise(wl, prm["grid_M"])
    delta = wl.a * 1e-2
    ref, _, _, _ = OF.em_rfd_step(geo, prm, wl.F, *noise, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                  tau=wl.tau_spurious)
    Wt = noise[2]
    U0, _ = MF.MatrixFreeFBIM(geo, prm, wl.alpert_order, tau=wl.tau_spurious).brownian_velocity(
        wl.F, noise[0], noise[1], wl.kT, wl.dt, tol=1e-11)
    # mistake: configurations moved by +- delta Wt instead of +- delta / 2 Wt
    Up = MF.MatrixFreeFBIM(OF.moved(geo, delta * Wt), prm, wl.alpert_order, tau=wl.tau_spurious).mobility(Wt)[0]
    Um = MF.MatrixFreeFBIM(OF.moved(geo, -delta * Wt), prm, wl.alpert_order, tau=wl.tau_spurious).mobility(Wt)[0]
    wrong = wl.dt * U0 + wl.dt * wl.kT / delta * (Up - Um)
    assert _rel(wrong, ref) > 1e-3


def test_golden_inputs_are_regenerated_exactly():
    # the stored 100-starfish step was computed from these seeded inputs
    wl, geo, prm = _setup("starfish100")
    noise = W.noise(wl, prm["grid_M"])
    h = hashlib.sha256()
    for a in (wl.q, wl.theta, wl.F) + tuple(noise):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    with open(GOLDEN) as f:
        lines = f.read().splitlines()
    digest = [ln.split()[-1] for ln in lines if ln.startswith("# inputs sha256")][0]
    assert digest == h.hexdigest()
    rows = np.array([[float(v) for v in ln.split()] for ln in lines if not ln.startswith("#")])
    assert rows.shape == (wl.n_bodies, 7) and np.all(np.isfinite(rows))
