"""The 640,000-node workload (10,000 five-arm starfish x 64 nodes, grid
2048^2, tol 1e-6) in the launch configuration the benchmark times.

The dense oracle cannot run at this size, so outputs are checked where the
oracle can compute them one by one: the real-space sum at sampled targets
(direct O(N) sums), the Alpert correction of sampled bodies, and the
wave-space part against the oracle's own spectral-Ewald steps over the full
grid.  Every part must also be repeatable: the operator handed to the Krylov
solvers has to be the same matrix on every application."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, host, log, make_ctx, oracle_params, relerr, zeros
from oracle import direct as OD
from oracle import fbim as OF

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import paper_1709_01480_amd as fb
    wl = W.make("starfish10k")
    log("case starfish10k: %d nodes" % wl.n_nodes)
    ctx = make_ctx(wl)
    geo = OF.geometry_from_workload(wl)
    X, _ = OF.nodes(geo)
    mu = np.random.default_rng(1).standard_normal(2 * wl.n_nodes)
    parts = {}
    for name, p in (("real", fb.PART_REAL), ("alpert", fb.PART_ALPERT), ("wave", fb.PART_WAVE)):
        a, b = zeros(mu.size), zeros(mu.size)
        ctx.apply_M(dev(mu), a, p)
        ctx.apply_M(dev(mu), b, p)
        parts[name] = (host(a), host(b))
    return wl, ctx, geo, oracle_params(wl), X, mu, parts


def test_parts_repeatable(big):
    wl, ctx, geo, prm, X, mu, parts = big
    for name, (a, b) in parts.items():
        scale = np.max(np.abs(a))
        assert np.max(np.abs(a - b)) <= 1e-13 * scale, name


def test_real_space_sampled(big):
    wl, ctx, geo, prm, X, mu, parts = big
    tg = np.random.default_rng(2).choice(wl.n_nodes, 256, replace=False)
    ref = OD.real_space(X, mu, wl.L, prm["xi"], prm["r_c"], targets=tg)
    got = parts["real"][0].reshape(-1, 2)[tg].ravel()
    assert relerr(got, ref) < 1e-12


def test_alpert_sampled_bodies(big):
    wl, ctx, geo, prm, X, mu, parts = big
    off = geo.offsets()
    for b in (0, 4321, 9999):
        blk = OF.alpert_body(geo, b, prm["xi"], prm["r_c"], wl.alpert_order)
        blk = 0.5 * (blk + blk.T)
        sl = slice(2 * off[b], 2 * off[b + 1])
        assert relerr(parts["alpert"][0][sl], blk @ mu[sl]) < 1e-11


def test_wave_full_grid(big):
    wl, ctx, geo, prm, X, mu, parts = big
    ref = OF.wave_se(X, mu, prm)
    assert relerr(parts["wave"][0], ref) < 1e-10


def test_mixed_matvec_close_to_fp64(big):
    import paper_1709_01480_amd as fb
    wl, ctx, geo, prm, X, mu, parts = big
    cm = make_ctx(wl, precision=fb.PREC_MIXED)
    out = zeros(mu.size)
    cm.apply_M(dev(mu), out, fb.PART_ALL)
    ref = parts["real"][0] + parts["alpert"][0] + parts["wave"][0]
    assert relerr(host(out), ref) < 1e-5
    cm.close()


def test_mobility_converges_deterministically(big):
    wl, ctx, geo, prm, X, mu, parts = big
    U1, U2 = zeros(3 * wl.n_bodies), zeros(3 * wl.n_bodies)
    i1 = ctx.mobility(dev(wl.F), U1)
    i2 = ctx.mobility(dev(wl.F), U2)
    log("mobility at 640k nodes: %s / %s" % (i1, i2))
    assert i1["gmres_residual"] <= wl.tol_gmres and i2["gmres_residual"] <= wl.tol_gmres
    assert i1["gmres_iters"] == i2["gmres_iters"]
    # every reduction of the path has a fixed order (spreading sums are exact
    # fixed-point integers), so two solves agree bit for bit
    assert np.array_equal(host(U1), host(U2))
