"""Pins of the oracle's Brownian velocity and EM-RFD step against what the paper
fixes (Section 3.1, discrete fluctuation-dissipation balance, eq. 3.11;
Section 4.4, the EM-RFD update eq. 4.3).

Each check is built so that a plausible slip in the oracle fails it:
  - the slip amplitude sqrt(2 kT / dt) (a sqrt(kT / dt) gives half the
    covariance): the linear map (W_r, W_grid) -> U, taken column by column
    through DenseFBIM.brownian_velocity, must have covariance (2 kT / dt) N;
  - a seeded statistical check: the sample covariance of U tends to
    (2 kT / dt) N and the mean of the chi^2 statistic U^T N^-1 U dt / (2 kT)
    is 3n;
  - the random finite difference: with F = 0 and zero W, em_rfd_step with
    W~ = e_i returns dt kT times the derivative of the i-th column of N along
    Q_i, compared with a central difference of the body mobility at another
    step (a wrong sign, a delta in place of delta/2, or a missing dt fails);
    translational directions give zero for one body in a periodic box;
  - moved() turns the body rigidly: x' - q' = R(dtheta) (x - q).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fbim as F


@pytest.fixture(scope="module")
def tiny():
    # two five-arm starfish (32 nodes each); a 32^2 grid keeps the noise map small
    wl = W.make("tiny2", grid_M=32, P=11)
    geo = F.geometry_from_workload(wl)
    prm = F.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
    return wl, geo, prm, F.DenseFBIM(geo, prm, order=4)


KT, DT = 1.0, 1e-3


def brownian_map(wl, prm, d):
    """B: (W_r, W_grid) -> U with F = 0, one column per unit noise vector,
    each through DenseFBIM.brownian_velocity."""
    n2, nw = 2 * wl.n_nodes, 2 * prm["grid_M"] ** 2
    F0 = np.zeros(3 * wl.n_bodies)
    B = np.zeros((3 * wl.n_bodies, n2 + nw))
    zr, zw = np.zeros(n2), np.zeros(nw)
    for j in range(n2):
        e = zr.copy()
        e[j] = 1.0
        B[:, j] = d.brownian_velocity(F0, e, zw, KT, DT)
    for j in range(nw):
        e = zw.copy()
        e[j] = 1.0
        B[:, n2 + j] = d.brownian_velocity(F0, zr, e, KT, DT)
    return B


def fdb_error(B, d):
    """max |B B^T - (2 kT/dt) N| / max |(2 kT/dt) N| (eqs. 3.11, 3.27)."""
    target = 2 * KT / DT * F.body_mobility(d.mats["M"], d.K)
    return np.max(np.abs(B @ B.T - target)) / np.max(np.abs(target))


@pytest.fixture(scope="module")
def noise_map(tiny):
    wl, geo, prm, d = tiny
    return brownian_map(wl, prm, d), KT, DT


def test_brownian_map_covariance_is_scaled_mobility(tiny, noise_map):
    # eq. 3.11 with the slip amplitude of eq. 3.27: B B^T = (2 kT / dt) N
    wl, geo, prm, d = tiny
    B, kT, dt = noise_map
    Nm = F.body_mobility(d.mats["M"], d.K)
    rel = fdb_error(B, d)
    assert rel < 1e-4, rel
    # the map is linear in the noise and F enters additively
    rng = np.random.default_rng(5)
    Wr, Wg = rng.standard_normal(2 * wl.n_nodes), rng.standard_normal(2 * prm["grid_M"] ** 2)
    Fv = rng.standard_normal(3 * wl.n_bodies)
    U = d.brownian_velocity(Fv, Wr, Wg, kT, dt)
    ref = B @ np.concatenate([Wr, Wg]) + Nm @ Fv
    assert np.max(np.abs(U - ref)) < 1e-9 * np.max(np.abs(ref))


def test_brownian_velocity_statistics(tiny, noise_map):
    # seeded statistical check of discrete FDB: sample covariance -> (2 kT/dt) N,
    # chi^2 = U^T N^-1 U dt / (2 kT) has mean 3n and variance 6n
    wl, geo, prm, d = tiny
    B, kT, dt = noise_map
    Nm = F.body_mobility(d.mats["M"], d.K)
    n3 = 3 * wl.n_bodies
    S = 4000
    Wn = np.random.default_rng(1709).standard_normal((B.shape[1], S))
    U = B @ Wn
    Ninv = np.linalg.inv(Nm)
    chi2 = np.einsum("is,ij,js->s", U, Ninv, U) * dt / (2 * kT)
    assert abs(chi2.mean() - n3) < 4 * math.sqrt(2 * n3 / S), chi2.mean()
    assert abs(chi2.var() / (2 * n3) - 1.0) < 0.15, chi2.var()
    C = U @ U.T / S
    target = 2 * kT / dt * Nm
    # each entry within 5 standard errors of its Wishart spread
    se = np.sqrt((target ** 2 + np.outer(np.diag(target), np.diag(target))) / S)
    assert np.all(np.abs(C - target) < 5 * se)


@pytest.fixture(scope="module")
def starfish_one():
    wl = W.single_starfish(theta=0.3, n_p=64, tol=1e-9, n_box=3)
    geo = F.geometry_from_workload(wl)
    prm = F.derive_params(1.0, 1e-9, n_box=3)
    return wl, geo, prm


@pytest.fixture(scope="module")
def mobility_derivative(starfish_one):
    """dt kT dN/dtheta by a central difference of the body mobility (eq. 3.9) at
    theta +- h, a step unrelated to the RFD's delta."""
    wl, geo, prm = starfish_one

    def N_at(dth):
        g = F.Geometry(geo.L, geo.shapes, geo.shape_id, geo.q.copy(), geo.theta + dth)
        dd = F.DenseFBIM(g, prm, order=4)
        return F.body_mobility(dd.mats["M"], dd.K)

    h = 1e-3
    return KT * DT * (N_at(h) - N_at(-h)) / (2 * h)


def rfd_rotation_error(starfish_one, ref):
    """em_rfd_step with F = 0, W = 0, Wt = e_theta against dt kT dN e_theta / dtheta."""
    wl, geo, prm = starfish_one
    M = prm["grid_M"]
    e = np.array([0.0, 0.0, 1.0])
    dQ, U0, _, _ = F.em_rfd_step(geo, prm, np.zeros(3), np.zeros(2 * wl.n_nodes), np.zeros(2 * M * M), e,
                                 KT, DT, 4e-3)
    assert np.max(np.abs(U0)) == 0.0
    return np.max(np.abs(dQ - ref[:, 2])) / np.max(np.abs(ref))


def test_rfd_drift_is_divergence_of_mobility(starfish_one, mobility_derivative):
    # eq. 4.3: with F = 0 and W = 0, dQ = dt kT / delta [N(Q + delta/2 Wt) - N(Q - delta/2 Wt)] Wt,
    # which for Wt = e_i is dt kT d N e_i / d Q_i + O(delta^2)
    wl, geo, prm = starfish_one
    kT, dt, delta = KT, DT, 4e-3
    M = prm["grid_M"]
    zr, zw = np.zeros(2 * wl.n_nodes), np.zeros(2 * M * M)
    F0 = np.zeros(3)
    scale = np.max(np.abs(mobility_derivative))
    assert scale > 0
    assert rfd_rotation_error(starfish_one, mobility_derivative) < 1e-3
    # one body in a periodic box: N does not depend on its position
    for i in (0, 1):
        e = np.zeros(3)
        e[i] = 1.0
        dQt, _, _, _ = F.em_rfd_step(geo, prm, F0, zr, zw, e, kT, dt, delta)
        assert np.max(np.abs(dQt)) < 1e-6 * scale, dQt


def test_moved_is_a_rigid_motion(tiny):
    wl, geo, prm, d = tiny
    rng = np.random.default_rng(3)
    dQ = rng.standard_normal(3 * wl.n_bodies) * np.tile([0.01, 0.01, 0.2], wl.n_bodies)
    g2 = F.moved(geo, dQ)
    X, body = F.nodes(geo)
    X2, _ = F.nodes(g2)
    dq = dQ.reshape(-1, 3)
    for b in range(wl.n_bodies):
        c, s = math.cos(dq[b, 2]), math.sin(dq[b, 2])
        Rb = np.array([[c, -s], [s, c]])
        sel = body == b
        assert np.allclose(g2.q[b], geo.q[b] + dq[b, :2], rtol=0, atol=1e-15)
        assert np.allclose(X2[sel] - g2.q[b], (X[sel] - geo.q[b]) @ Rb.T, rtol=0, atol=1e-14)


# ---------------------------------------------------- planted mistakes (oracle, CPU)
def test_planted_half_slip_variance_fails_fdb(tiny, monkeypatch):
    # sqrt(kT / dt) in place of sqrt(2 kT / dt) halves the covariance
    wl, geo, prm, d = tiny

    def slip(self, W_r, W_grid, kT, dt):
        vr = self.real_root() @ W_r
        vw = F.random_field(self.X, W_grid, self.prm, self.eta)
        return math.sqrt(kT / dt) * (vr + vw), vr, vw

    monkeypatch.setattr(F.DenseFBIM, "slip", slip)
    assert fdb_error(brownian_map(wl, prm, d), d) > 0.3


@pytest.mark.parametrize("factor", [2.0, -1.0])
def test_planted_rfd_displacement_mistakes_fail(starfish_one, mobility_derivative, monkeypatch, factor):
    # configurations at Q +- delta Wt (factor 2) or with the sign of the difference
    # swapped (factor -1) instead of Q +- delta/2 Wt
    real = F.moved
    monkeypatch.setattr(F, "moved", lambda geo, dQ: real(geo, factor * np.asarray(dQ)))
    assert rfd_rotation_error(starfish_one, mobility_derivative) > 0.5


def test_ab2_step_reduces_to_em_and_carries_the_force_history(tiny):
    # AB2-RFD (Section 4.4): with N^(n-1) F^(n-1) = N^n F^n it is the EM-RFD step;
    # otherwise it differs from it by exactly dt/2 (N^n F^n - N^(n-1) F^(n-1)), and
    # the deterministic and stochastic parts, solved separately, add up to U0
    wl, geo, prm, _ = tiny
    Wr, Wg, Wt = W.noise(wl, prm["grid_M"])
    delta = 1e-2 * wl.a
    em, U0, _, _ = F.em_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, order=wl.alpert_order)
    ab, NF = F.ab2_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, order=wl.alpert_order)
    assert np.linalg.norm(ab - em) <= 1e-12 * np.linalg.norm(em)
    NF_prev = np.random.default_rng(3).standard_normal(NF.size)
    ab2, NF2 = F.ab2_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, NF_prev=NF_prev,
                               order=wl.alpert_order)
    assert np.allclose(NF2, NF, rtol=0, atol=1e-14 * np.abs(NF).max())
    assert np.allclose(ab2 - em, 0.5 * wl.dt * (NF - NF_prev), rtol=1e-10, atol=1e-14 * np.abs(em).max())
    # planted mistake: weights (1, 0) instead of (3/2, -1/2) fails
    wrong = em + 0.0 * (NF - NF_prev)
    assert np.linalg.norm(wrong - ab2) > 1e-3 * np.linalg.norm(ab2)


def test_em_step_without_the_drift_term(tiny):
    # delta = 0: the biased scheme dQ = dt U0 of Section 4.4.1
    wl, geo, prm, _ = tiny
    Wr, Wg, Wt = W.noise(wl, prm["grid_M"])
    dQ, U0, Up, Um = F.em_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, 0.0, order=wl.alpert_order)
    U = F.DenseFBIM(geo, prm, wl.alpert_order).brownian_velocity(wl.F, Wr, Wg, wl.kT, wl.dt)
    assert Up is None and Um is None and np.allclose(dQ, wl.dt * U, rtol=1e-13, atol=0)
