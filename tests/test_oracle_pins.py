"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, a
printed value, an invariant, or a textbook routine, chosen so that a dropped
term, a wrong sign/index or a transposed operand fails at least one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import workloads as W
from conftest import golden
from oracle import fbim as F
from oracle.alpert import (alpert_rule, periodic_log_quadrature,
                           periodic_log_quadrature_interp)
from oracle.special import e1

PAPER = golden("paper_values.txt")


# ----------------------------------------------------------------- E1 (eq. 3.16)
def test_e1_against_mpmath():
    z = np.concatenate([np.logspace(-14, 0, 60), np.linspace(1.0, 64.0, 300)])
    ref = np.array([float(mp.e1(mp.mpf(float(x)))) for x in z])
    assert np.max(np.abs(e1(z) - ref) / ref) < 3e-15


def test_e1_small_argument_limit():
    # E1(z) = -gamma - log z + O(z) (Section 3.2)
    z = np.array([1e-10, 1e-8])
    assert np.allclose(e1(z), -np.euler_gamma - np.log(z), rtol=0, atol=2e-8)


# --------------------------------------------------------- Alpert rules (Sec. 3.1)
@pytest.mark.parametrize("order,min_rate", [(4, 3.6), (8, 7.5)])
def test_alpert_log_integral_convergence(order, min_rate):
    # int_0^{2pi} ln(4 sin^2(s/2)) cos(n s) ds = -2 pi / n
    nmode = 3
    errs = []
    ns = (64, 128, 256) if order == 4 else (32, 48, 64)
    for n in ns:
        f = lambda s: np.log(4 * np.sin(s / 2) ** 2) * np.cos(nmode * s)
        errs.append(abs(periodic_log_quadrature(f, n, order) + 2 * np.pi / nmode))
    rates = [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    assert min(rates) > min_rate, (errs, rates)


@pytest.mark.parametrize("order,min_rate", [(4, 3.6), (8, 7.0)])
def test_alpert_with_lagrange_interpolation(order, min_rate):
    # same closed form, singularity at s_t = t ds, density known only at nodes:
    # int ln(4 sin^2((s - s_t)/2)) cos(n s) ds = -(2 pi / n) cos(n s_t)
    nmode = 2
    errs = []
    ns = (64, 128, 256) if order == 4 else (64, 96, 128)
    for n in ns:
        st = 2 * np.pi * 5 / n
        dens = np.cos(nmode * 2 * np.pi * np.arange(n) / n)
        v = periodic_log_quadrature_interp(lambda s: np.log(4 * np.sin((s - st) / 2) ** 2),
                                           dens, n, order, t=5)
        exact = -2 * np.pi / nmode * np.cos(nmode * st)
        errs.append(abs(v - exact))
    rates = [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    assert min(rates) > min_rate, (errs, rates)


def test_alpert_weights_sum():
    # the one-sided weights replace a - 1/2 dropped unit-spaced points
    for order in (4, 8):
        chi, w, a = alpert_rule(order)
        assert abs(w.sum() - (a - 0.5)) < 1e-13
        assert np.all(w > 0) and np.all((chi > 0) & (chi < a))


# ------------------------------------------------ kernels (eqs. 3.13-3.15, 3.26)
def test_ewald_split_is_xi_independent():
    L = 1.0
    rng = np.random.default_rng(3)
    pts = rng.uniform(-0.5, 0.5, (6, 2))

    def total(xi):
        acc = np.zeros((len(pts), 2, 2))
        for px in range(-3, 4):
            for py in range(-3, 4):
                acc += F.G_real(pts + np.array([px, py]) * L, xi)
        return acc + F.G_wave_direct(pts, xi, L)

    t0 = total(6.0)
    for xi in (9.0, 14.0):
        assert np.max(np.abs(total(xi) - t0)) < 1e-14


def test_real_kernel_log_singularity():
    # G^(r) ~ -(1/8 pi)(gamma + log(xi^2 r^2)) I + (1/4 pi)(r r^T/r^2 - I) as r -> 0
    xi, r = 7.0, 1e-6
    g = F.G_real(np.array([[r, 0.0]]), xi)[0]
    lead = -(np.euler_gamma + math.log(xi * xi * r * r)) / (8 * math.pi)
    assert abs(g[0, 0] - lead) < 1e-9
    assert abs(g[1, 1] - (lead - 1 / (4 * math.pi))) < 1e-9


def test_parameter_rule_printed_values():
    p4 = F.derive_params(1.0, 1e-9, n_box=4)
    v, tol, _ = PAPER["xiL_nbox4_eps1e-9"]
    assert abs(p4["xi"] * 1.0 - v) / v < tol
    p10 = F.derive_params(1.0, 1e-9, n_box=10)
    v, tol, _ = PAPER["xi_nbox10_eps1e-9"]
    assert abs(p10["xi"] - v) / v < tol
    # spreading width from exp(-pi P / 2) <= eps, P odd
    assert F.derive_params(1.0, 1e-6, n_box=4)["P"] == 9
    assert F.derive_params(1.0, 1e-8, n_box=4)["P"] == 13


def test_starfish_packing_fraction():
    v, tol, _ = PAPER["starfish_phi_a045_b03"]
    assert abs(W.starfish_area(0.45 / 1.3, 0.3) - v) / v < tol
    v, tol, _ = PAPER["phi_max_square_lattice"]
    assert abs(math.pi / 4 - v) / v < tol


# --------------------------------------------- spectral Ewald (eqs. 3.21-3.30)
def _small_points(n=7, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (n, 2)), rng.standard_normal(2 * n)


def test_spectral_ewald_matches_direct_ksum():
    prm = F.derive_params(1.0, 1e-10, xi=5.0, n_box=2, grid_M=48, P=15)
    X, mu = _small_points()
    ref = F.M_wave_direct(X, 1.0, prm["xi"]) @ mu
    assert np.max(np.abs(F.wave_se(X, mu, prm) - ref)) / np.max(np.abs(ref)) < 2e-9


def test_random_field_covariance_is_Mwave():
    prm = F.derive_params(1.0, 1e-10, xi=5.0, n_box=2, grid_M=32, P=15)
    X, _ = _small_points(5, 1)
    M = prm["grid_M"]
    A = np.zeros((10, 2 * M * M))
    for j in range(2 * M * M):
        e = np.zeros(2 * M * M)
        e[j] = 1.0
        A[:, j] = F.random_field(X, e, prm)
    Mw = F.M_wave_direct(X, 1.0, prm["xi"])
    assert np.max(np.abs(A @ A.T - Mw)) / np.max(np.abs(Mw)) < 1e-8


# ------------------------------------------------------- single-layer matrix
@pytest.fixture(scope="module")
def small_dense():
    wl = W.make("tiny2")
    geo = F.geometry_from_workload(wl)
    prm = F.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
    return wl, geo, prm, F.DenseFBIM(geo, prm, order=4)


def test_M_symmetric_and_wave_psd(small_dense):
    _, _, _, d = small_dense
    M, Mw = d.mats["M"], d.mats["Mw"]
    assert np.max(np.abs(M - M.T)) < 1e-13 * np.max(np.abs(M))
    lam = np.linalg.eigvalsh(Mw)
    assert lam.min() > -1e-12 * lam.max()


def test_M_annihilates_normals(small_dense):
    # the single-layer operator has the normal densities in its null space
    # (Section 2.2); mu = n |gamma'| ds
    wl, geo, prm, d = small_dense
    s = 2 * np.pi * np.arange(wl.n_p) / wl.n_p
    mu = []
    for b in range(wl.n_bodies):
        ds = 1e-6
        t = (F.body_points(geo, b, s + ds) - F.body_points(geo, b, s - ds)) / (2 * ds)
        nrm = np.stack([t[:, 1], -t[:, 0]], axis=1) * (2 * np.pi / wl.n_p)
        mu.append(nrm)
    mu = np.concatenate(mu).ravel()
    out = d.mats["M"] @ mu
    scale = np.max(np.abs(d.mats["M"] @ np.ones_like(mu))) * np.max(np.abs(mu))
    assert np.max(np.abs(out)) < 2e-3 * scale  # quadrature error at N_p = 32


def test_M_independent_of_xi(small_dense):
    # M mu = (M^(r) + M^(w)) mu does not depend on xi up to eps and the quadrature
    # error (Sec. 4.3); checked on a smooth force density
    wl, geo, prm, d = small_dense
    s = 2 * np.pi * np.arange(wl.n_p) / wl.n_p
    mu = np.stack([np.cos(s) + 0.3, np.sin(2 * s)], axis=1) * (2 * np.pi / wl.n_p)
    mu = np.concatenate([mu, 0.5 * mu[::-1]]).ravel()
    ref = d.mats["M"] @ mu
    for nb in (2, 4):
        prm2 = F.derive_params(wl.L, 1e-10, n_box=nb)
        M2 = F.single_layer(geo, prm2, order=4)["M"]
        assert np.max(np.abs(M2 @ mu - ref)) / np.max(np.abs(ref)) < 1e-4
    # and exactly (to eps) between different bodies, where no quadrature correction acts
    prm2 = F.derive_params(wl.L, 1e-10, n_box=2)
    M2 = F.single_layer(geo, prm2, order=4)["M"]
    n2 = 2 * wl.n_p
    assert np.max(np.abs(M2[:n2, n2:] - d.mats["M"][:n2, n2:])) < 1e-9


def test_K_adjoint_and_normals(small_dense):
    wl, geo, prm, d = small_dense
    K = d.K
    rng = np.random.default_rng(5)
    U = rng.standard_normal(3 * wl.n_bodies)
    mu = rng.standard_normal(2 * wl.n_nodes)
    # torque tau = r_x f_y - r_y f_x is the adjoint of omega x r
    X, body = F.nodes(geo)
    r = X - geo.q[body]
    tau = np.array([np.sum((r[:, 0] * mu[1::2] - r[:, 1] * mu[0::2])[body == b])
                    for b in range(wl.n_bodies)])
    assert np.allclose((K.T @ mu)[2::3], tau, atol=1e-14)
    assert abs(mu @ (K @ U) - (K.T @ mu) @ U) < 1e-12


# ------------------------------------------------------------- mobility (eq. 4.1)
def hasimoto_drag(phi):
    c0 = PAPER["hasimoto_c0"][0]
    c2 = PAPER["hasimoto_c2"][0]
    c3 = PAPER["hasimoto_c3"][0]
    return 4 * math.pi / (-math.log(math.sqrt(phi)) - c0 + phi + c2 * phi ** 2 + c3 * phi ** 3)


@pytest.mark.parametrize("phi,tol", [(0.01, 4e-4), (0.05, 4e-4), (0.1, 1.5e-3)])
def test_square_array_drag_matches_hasimoto(phi, tol):
    # the printed coefficients carry 3 decimals, which limits the agreement
    l = math.sqrt(math.pi / phi)
    wl = W.disk_lattice(l, 64, tol=1e-9, n_box=4)
    geo = F.geometry_from_workload(wl)
    prm = F.derive_params(l, 1e-9, n_box=4)
    U, _ = F.DenseFBIM(geo, prm, order=4).mobility(np.array([1.0, 0.0, 0.0]))
    drag = 1.0 / U[0]
    assert abs(drag - hasimoto_drag(phi)) / hasimoto_drag(phi) < tol


def test_rotational_mobility_of_dilute_disk():
    # isolated rotating disk: torque = 4 pi eta a^2 omega (periodic correction O(phi))
    phi = 1e-3
    l = math.sqrt(math.pi / phi)
    wl = W.disk_lattice(l, 64, tol=1e-9, n_box=4)
    geo = F.geometry_from_workload(wl)
    prm = F.derive_params(l, 1e-9, n_box=4)
    d = F.DenseFBIM(geo, prm, order=4)
    Nm = F.body_mobility(d.mats["M"], d.K)
    assert abs(Nm[2, 2] * 4 * math.pi - 1.0) < 2 * phi
    assert abs(Nm[0, 1]) < 1e-12 and abs(Nm[0, 0] - Nm[1, 1]) < 1e-10


def starfish_averages(order=4, n_theta=16, n_p=64):
    nxx, nyy, ntt = [], [], []
    for th in np.arange(n_theta) * (math.pi / 2) / n_theta:
        wl = W.single_starfish(theta=th, n_p=n_p, tol=1e-9, n_box=3)
        geo = F.geometry_from_workload(wl)
        prm = F.derive_params(1.0, 1e-9, n_box=3)
        d = F.DenseFBIM(geo, prm, order=order)
        Nm = F.body_mobility(d.mats["M"], d.K)
        nxx.append(Nm[0, 0])
        nyy.append(Nm[1, 1])
        ntt.append(Nm[2, 2])
    return np.mean(nxx), np.mean(nyy), np.mean(ntt)


def test_starfish_diffusion_coefficients():
    # Section 4.4.1: kT<N_xx> ~ 2.47e-3, kT<N_thth> ~ 0.2081 (uniform theta average)
    nxx, nyy, ntt = starfish_averages()
    v, tol, _ = PAPER["chi_trans_starfish"]
    assert abs(nxx - v) / v < tol
    v, tol, _ = PAPER["chi_rot_starfish"]
    assert abs(ntt - v) / v < tol
    assert abs(nxx - nyy) < 1e-9  # four-fold body in a square box


def test_planted_mistake_dropping_alpert_fails_pin(monkeypatch):
    # the starfish pin has teeth: without the singular correction it fails
    monkeypatch.setattr(F, "M_alpert", lambda geo, *a, **k: np.zeros((2 * geo.N, 2 * geo.N)))
    nxx, _, ntt = starfish_averages(n_theta=4)
    v, tol, _ = PAPER["chi_rot_starfish"]
    assert abs(ntt - v) / v > 10 * tol


# ------------------------------------------------ fluctuation-dissipation (eq. 3.11)
def test_discrete_fdb(small_dense):
    # the linear map from (W_r, W_grid) to the Brownian velocity has covariance N
    wl, geo, prm, d = small_dense
    G, Gp = F.G_blocks(geo, prm, 4, 1e-8)
    Ar = Gp @ F.sqrt_psd(G @ d.mats["Mr"] @ G.T)
    M = prm["grid_M"]
    Aw = np.zeros((2 * wl.n_nodes, 2 * M * M))
    for j in range(2 * M * M):
        e = np.zeros(2 * M * M)
        e[j] = 1.0
        Aw[:, j] = F.random_field(d.X, e, prm)
    Nm = F.body_mobility(d.mats["M"], d.K)
    B = Nm @ d.K.T @ np.linalg.solve(d.mats["M"], np.hstack([Ar, Aw]))
    rel = np.max(np.abs(B @ B.T - Nm)) / np.max(np.abs(Nm))
    assert rel < 1e-4, rel
