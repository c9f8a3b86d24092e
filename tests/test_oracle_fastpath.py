"""The CPU fast path (oracle/fastpath.py) against the direct oracle: the
cell-list real-space sum against the all-pairs sum (eqs. 3.15, 3.17), the
shared-block Alpert correction against blocks built body by body (Section 3.3),
and the C gridding with real transforms against the oracle's spectral Ewald
(Section 3.2), on the 4- and 100-starfish suspensions and on points that sit
on cell and box edges."""
import numpy as np
import pytest

import workloads as W
from oracle import direct as OD
from oracle import fastpath as FP
from oracle import fbim as OF


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _setup(name):
    wl = W.make(name)
    prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
    geo = OF.geometry_from_workload(wl)
    return wl, prm, geo, FP.FastFBIM(geo, prm, wl.alpert_order)


@pytest.mark.parametrize("name", ["tiny2", "starfish4", "starfish100"])
def test_fast_path_matches_direct_oracle(name):
    wl, prm, geo, f = _setup(name)
    mu = np.random.default_rng(4).standard_normal(2 * geo.N)
    assert _rel(f.apply_real(mu), OD.real_space(f.X, mu, wl.L, prm["xi"], prm["r_c"])) < 1e-14
    # spectral Ewald with real transforms against the oracle's complex ones: they
    # differ only in how the (negligible) Nyquist modes are symmetrised
    assert _rel(f.apply_wave(mu), OF.wave_se(f.X, mu, prm)) < 1e-10
    off = geo.offsets()
    alp = f.apply_alpert(mu)
    for b in range(min(geo.n, 6)):
        blk = OF.alpert_body(geo, b, prm["xi"], prm["r_c"], wl.alpert_order)
        sl = slice(2 * off[b], 2 * off[b + 1])
        assert _rel(alp[sl], 0.5 * (blk + blk.T) @ mu[sl]) < 1e-12


def test_cell_list_on_cell_and_box_edges():
    # points on cell boundaries, at 0 and just below L, and outside [0, L): the cell
    # list must find every in-range pair the direct sum finds
    L, xi, r_c = 1.0, 9.0, 0.2  # 5 cells of side 0.2 = r_c
    rng = np.random.default_rng(9)
    edge = np.array([0.0, 0.2, 0.4, 0.6, 0.8, 1.0 - 1e-15, 0.2 - 1e-15, 0.4 + 1e-15])
    X = np.concatenate([rng.uniform(-1.0, 2.0, (300, 2)),
                        np.stack(np.meshgrid(edge, edge), -1).reshape(-1, 2)])
    mu = rng.standard_normal(2 * len(X))
    ref = OD.real_space(X, mu, L, xi, r_c)
    assert _rel(OD.real_space_cells(X, mu, L, xi, r_c), ref) < 1e-14


def test_too_few_cells_falls_back_to_the_direct_sum():
    rng = np.random.default_rng(10)
    X = rng.uniform(0, 1, (50, 2))
    mu = rng.standard_normal(100)
    r_c = 0.45  # floor(1 / 0.45) = 2 cells per side
    assert np.array_equal(OD.real_space_cells(X, mu, 1.0, 6.0, r_c), OD.real_space(X, mu, 1.0, 6.0, r_c))
