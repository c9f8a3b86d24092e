"""The oracle's C direct sums agree with its dense numpy assembly, and the
oracle's spectral-Ewald steps converge to the direct k-sum as P and M grow."""
import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle import fbim as F


@pytest.fixture(scope="module")
def small12():
    wl = W.make("small12")
    geo = F.geometry_from_workload(wl)
    prm = F.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box)
    X, _ = F.nodes(geo)
    mu = np.random.default_rng(1).standard_normal(2 * len(X))
    return wl, geo, prm, X, mu


def test_c_real_space_matches_dense(small12):
    wl, geo, prm, X, mu = small12
    ref = F.M_trap(X, wl.L, prm["xi"], prm["r_c"]) @ mu
    out = D.real_space(X, mu, wl.L, prm["xi"], prm["r_c"])
    assert np.max(np.abs(out - ref)) < 1e-13 * np.max(np.abs(ref))
    tg = np.array([3, 100, 7])
    sub = D.real_space(X, mu, wl.L, prm["xi"], prm["r_c"], targets=tg)
    assert np.allclose(sub.reshape(-1, 2), ref.reshape(-1, 2)[tg], rtol=0, atol=1e-15)


def test_c_wave_space_matches_dense(small12):
    wl, geo, prm, X, mu = small12
    ref = F.M_wave_direct(X, wl.L, prm["xi"]) @ mu
    out = D.wave_space(X, mu, wl.L, prm["xi"])
    assert np.max(np.abs(out - ref)) < 1e-13 * np.max(np.abs(ref))


def test_c_e1_matches_python():
    from oracle.special import e1
    for z in (1e-9, 0.3, 1.0, 2.5, 17.0, 40.0):
        assert abs(D.lib().oracle_e1(z) - e1(np.array([z]))[0]) <= 1e-15 * abs(e1(np.array([z]))[0])


def test_spectral_ewald_error_decreases_with_support(small12):
    wl, geo, prm, X, mu = small12
    ref = D.wave_space(X, mu, wl.L, prm["xi"])
    errs = []
    for M, P in ((80, 13), (96, 17), (128, 21)):
        p = F.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=M, P=P)
        errs.append(np.max(np.abs(F.wave_se(X, mu, p) - ref)) / np.max(np.abs(ref)))
    assert errs[0] < 1e-6 and errs[1] < errs[0] / 10 and errs[2] < 1e-11
