"""Pins of the FP64 reference of the learned preconditioner correction
(oracle/mlp.py) against finite differences, invariances and hand-checked
values -- nothing here calls the library."""
import math

import numpy as np
import pytest

from oracle import mlp as OM


def _net(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, OM.N_PARAM)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    w = _net(1)
    X = rng.standard_normal((5, OM.N_IN))
    dY = rng.standard_normal((5, OM.N_OUT))
    g = OM.backward(w, X, dY)
    f = lambda ww: float(np.sum(dY * OM.forward(ww, X)[0]))  # noqa: E731
    # every bias and every W3 entry, and a random subset of W1 / W2
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in OM.SIZES])
    idx = list(range(offs[1], offs[2])) + list(range(offs[3], offs[6]))
    idx += list(rng.choice(offs[1], 300, replace=False)) + list(offs[2] + rng.choice(offs[3] - offs[2], 300,
                                                                                           replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(w)
        e[i] = h
        fd = (f(w + e) - f(w - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), i


def _bodies(n, seed):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0, 2 * np.pi, n)
    A = rng.standard_normal((n, 3, 3))
    Nref = np.einsum("bij,bkj->bik", A, A) + 3 * np.eye(3)
    return theta, Nref


def test_loss_gradient_matches_central_differences():
    n, ns = 4, 3
    theta, Nref = _bodies(n, 2)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((ns, n, 3))
    U = rng.standard_normal((ns, n, 3))
    Y = 0.1 * rng.standard_normal((n, 6))
    g = OM.loss_grad(Y, Nref, theta, F, U)
    h = 1e-6
    for b in range(n):
        for k in range(6):
            e = np.zeros_like(Y)
            e[b, k] = h
            fd = (OM.loss(Y + e, Nref, theta, F, U) - OM.loss(Y - e, Nref, theta, F, U)) / (2 * h)
            assert abs(fd - g[b, k]) <= 1e-7 * max(1.0, abs(fd))


def test_loss_vanishes_at_the_exact_self_mobility():
    """Block-diagonal N: U_b = N_bb F_b exactly, so dN = N_bb - N_ref (body
    frame) gives zero loss and zero gradient."""
    n, ns = 5, 4
    theta, Nref = _bodies(n, 4)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((n, 3, 3))
    Nbody = Nref + 0.2 * (B + B.transpose(0, 2, 1))  # N_bb in the body frame
    F = rng.standard_normal((ns, n, 3))
    # lab frame U = R N_bb R^T F (R acts on the translational part only)
    c, s = np.cos(theta), np.sin(theta)
    R = np.zeros((n, 3, 3))
    R[:, 0, 0], R[:, 0, 1], R[:, 1, 0], R[:, 1, 1], R[:, 2, 2] = c, -s, s, c, 1.0
    Nlab = np.einsum("bij,bjk,blk->bil", R, Nbody, R)
    U = np.einsum("bij,sbj->sbi", Nlab, F)
    D = Nbody - Nref
    sx, sy, st = Nref[:, 0, 0], Nref[:, 1, 1], Nref[:, 2, 2]
    Y = np.stack([D[:, 0, 0] / sx, D[:, 1, 1] / sy, D[:, 2, 2] / st, D[:, 0, 1] / np.sqrt(sx * sy),
                  D[:, 0, 2] / np.sqrt(sx * st), D[:, 1, 2] / np.sqrt(sy * st)], axis=1)
    assert OM.loss(Y, Nref, theta, F, U) < 1e-24
    assert np.max(np.abs(OM.loss_grad(Y, Nref, theta, F, U))) < 1e-12
    assert OM.loss(np.zeros_like(Y), Nref, theta, F, U) > 1e-3


def test_features_hand_checked_three_bodies():
    r, d, sym = 0.1, 0.25, 5
    R = 3 * r
    q = np.array([[0.5, 0.5], [0.5 + d, 0.5], [0.5, 0.5 + 1.1 * d]])
    theta = np.array([math.pi / 2, 0.1, 0.0])
    X = OM.features(q, theta, 10.0, r, sym)
    # body 0 (rotated by pi/2): neighbour 1 at lab (d, 0) -> body frame (0, -d); neighbour 2 at (0, 1.1 d) -> (1.1 d, 0)
    assert np.allclose(X[0, 0:5], [0.0, -d / R, r / d, math.cos(sym * (0.1 - math.pi / 2)),
                                   math.sin(sym * (0.1 - math.pi / 2))], atol=1e-15)
    assert np.allclose(X[0, 5:10], [1.1 * d / R, 0.0, r / (1.1 * d), math.cos(sym * (-math.pi / 2)),
                                    math.sin(sym * (-math.pi / 2))], atol=1e-15)
    assert np.all(X[0, 10:30] == 0.0)
    assert X[0, 30] == pytest.approx(2 / 6)
    assert X[0, 31] == pytest.approx((d - 2 * r) / r)
    # body 1 sees body 0 at distance d; body 2 at sqrt(d^2 + (1.1 d)^2) > R: one neighbour
    d12 = math.hypot(d, 1.1 * d)
    assert d12 > R
    assert X[1, 30] == pytest.approx(1 / 6)
    assert np.allclose(X[1, 0:3], [-d * math.cos(0.1) / R, d * math.sin(0.1) / R, r / d], atol=1e-15)


def test_features_invariant_under_translation_and_rotation():
    rng = np.random.default_rng(7)
    n, r = 40, 0.02
    q = rng.uniform(0, 0.3, (n, 2)) + 5.0
    theta = rng.uniform(0, 2 * np.pi, n)
    L = 100.0
    X = OM.features(q, theta, L, r, 5)
    assert np.max(X[:, 30]) > 0.3  # the configuration has neighbours
    # translation (with periodic wrap of a shifted copy)
    X2 = OM.features(np.mod(q + np.array([47.3, -81.9]), L), theta, L, r, 5)
    assert np.max(np.abs(X2 - X)) < 1e-10  # positions of size ~50 carry ~1e-14 absolute rounding
    # rigid rotation of the whole configuration about a point, bodies turning with it
    a = 0.7
    Rm = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    q3 = (q - 5.0) @ Rm.T + 50.0
    X3 = OM.features(q3, theta + a, L, r, 5)
    assert np.max(np.abs(X3 - X)) < 1e-10
