"""Pins of the completed second-kind oracle (oracle/secondkind.py, Appendix B).

  - each Ewald-split periodic sum (stresslet, rotlet, Stokeslet) is independent
    of the splitting parameter xi;
  - 1/2 + D annihilates rigid motions of a body (the reason the completion flow
    is needed), with spectral convergence in the number of nodes;
  - the mobility is symmetric (the reciprocal theorem of Appendix A);
  - it agrees with the first-kind formulation, two independent discretisations
    of the same problem, to 2e-11 against 8th-order Alpert at 256 nodes;
  - the paper's printed free-starfish diffusion coefficients (Section 4.4.1,
    computed there with this formulation);
  - planted mistakes (no mean term, the printed rotlet prefactor, the diagonal
    term dropped) fail.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fbim as F
from oracle import secondkind as SK

from test_oracle_pins import PAPER


def _pair(n_p):
    sh = F.Shape(0.08, 0.3, 5, n_p)
    return F.Geometry(1.0, [sh, sh], np.zeros(2, dtype=int), np.array([[0.3, 0.4], [0.62, 0.55]]),
                      np.array([0.2, 1.1]))


def test_periodic_sums_are_independent_of_xi():
    r = np.random.default_rng(0).uniform(-0.5, 0.5, (5, 2))
    rot = [SK.periodic_rotlet(r, 1.0, xi) for xi in (4.0, 7.0, 12.0)]
    sto = [SK.periodic_stokeslet(r, 1.0, xi) for xi in (4.0, 7.0, 12.0)]
    for a in rot[1:]:
        assert np.abs(a - rot[0]).max() < 1e-12 * np.abs(rot[0]).max()
    for a in sto[1:]:
        assert np.abs(a - sto[0]).max() < 1e-12 * np.abs(sto[0]).max()
    geo = _pair(32)
    D1, D2 = SK.double_layer_matrix(geo, 6.0), SK.double_layer_matrix(geo, 10.0)
    assert np.abs(D1 - D2).max() < 1e-12 * np.abs(D1).max()


@pytest.mark.parametrize("n_p,bar", [(64, 5e-4), (128, 5e-8), (256, 1e-12)])
def test_rigid_motions_span_the_null_space(n_p, bar):
    geo = _pair(n_p)
    X, n, t, kappa, ds, body = SK.curve_data(geo)
    D = SK.double_layer_matrix(geo, 8.0)
    c = np.tile([0.3, -0.7], len(X))
    rot = np.zeros(2 * len(X))
    idx = np.nonzero(body == 1)[0]
    rot.reshape(-1, 2)[idx] = SK.perp(X[idx] - geo.q[1])
    for phi in (c, rot):
        assert np.abs(0.5 * phi + D @ phi).max() < bar * np.abs(phi).max()


@pytest.fixture(scope="module")
def second_kind_pair():
    return SK.SecondKind(_pair(256), 8.0).body_mobility()


def test_mobility_is_symmetric(second_kind_pair):
    N = second_kind_pair
    assert np.abs(N - N.T).max() < 1e-11 * np.abs(N).max()
    assert np.all(np.linalg.eigvalsh(0.5 * (N + N.T)) > 0)


def test_agrees_with_the_first_kind_formulation(second_kind_pair):
    geo = _pair(256)
    prm = F.derive_params(1.0, 1e-12, n_box=4)
    d = F.DenseFBIM(geo, prm, order=8)
    N1 = F.body_mobility(d.mats["M"], d.K)
    assert np.abs(N1 - second_kind_pair).max() < 1e-9 * np.abs(second_kind_pair).max()


def test_free_starfish_diffusion_coefficients():
    # Section 4.4.1: kT <N_xx> ~ 2.47e-3, kT <N_thth> ~ 0.2081 (uniform theta average
    # over a period, 16 angles), the values the paper computed with the second-kind solver
    nxx, ntt = [], []
    for th in np.arange(16) * (math.pi / 2) / 16:
        wl = W.single_starfish(theta=th, n_p=128)
        N = SK.SecondKind(F.geometry_from_workload(wl), 8.0).body_mobility()
        nxx.append(N[0, 0])
        ntt.append(N[2, 2])
    v, tol, _ = PAPER["chi_trans_starfish"]
    assert abs(np.mean(nxx) - v) / v < tol
    v, tol, _ = PAPER["chi_rot_starfish"]
    assert abs(np.mean(ntt) - v) / v < tol


def test_planted_mistakes_fail(monkeypatch):
    # the rotlet's wave part with the printed 1/(eta V) prefactor: the sum is no
    # longer independent of xi
    r = np.random.default_rng(1).uniform(-0.5, 0.5, (5, 2))

    def printed(xi):
        kv, k2 = SK._waves(1.0, xi)
        wave = np.sin(r @ kv.T) @ SK.rotlet_wave(kv, k2, xi)
        return SK.periodic_rotlet(r, 1.0, xi) + (1 - 1 / (4 * math.pi)) * wave
    a, b = printed(4.0), printed(9.0)
    assert np.abs(a - b).max() > 1e-3 * np.abs(a).max()
    # without the trapezoid diagonal term rigid motions leave the null space
    geo = _pair(128)
    X = SK.curve_data(geo)[0]
    c = np.tile([0.3, -0.7], len(X))
    good = np.abs(0.5 * c + SK.double_layer_matrix(geo, 8.0) @ c).max()
    orig = SK.curve_data
    monkeypatch.setattr(SK, "curve_data", lambda g: (lambda x: (x[0], x[1], x[2], 0 * x[3], x[4], x[5]))(orig(g)))
    bad = np.abs(0.5 * c + SK.double_layer_matrix(geo, 8.0) @ c).max()
    assert bad > 1e3 * good
    # without the mean term the periodic double layer of a constant is off by (A/V) c
    monkeypatch.setattr(SK, "curve_data", orig)
    D = SK.double_layer_matrix(geo, 8.0)
    X, n, t, kappa, ds, body = orig(geo)
    mean = -(4 * np.pi / geo.L ** 2) * np.einsum("sj,sl->jsl", X, n) * ds[None, :, None] / (4 * np.pi)
    Dm = D - np.broadcast_to(mean[None], (len(X),) + mean.shape).reshape(D.shape)
    assert np.abs(0.5 * c + Dm @ c).max() > 1e3 * good
