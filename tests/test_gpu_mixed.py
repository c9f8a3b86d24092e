"""Mixed precision (FP32 pair sum / spreading / FFT / interpolation with FP64
Krylov) against the FP64 oracle.  The bar is 1e-4 relative on the Brownian
displacement; the matvec itself is checked at FP32 round-off level."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, host, log, make_ctx, oracle_params, relerr, workload, zeros
from oracle import fbim as OF

pytestmark = pytest.mark.gpu


def _ctx(wl, **kw):
    import paper_1709_01480_amd as fb
    return make_ctx(wl, precision=fb.PREC_MIXED, **kw)


@pytest.mark.parametrize("name", ["tiny2", "small12"])
def test_mixed_matvec(name):
    import paper_1709_01480_amd as fb
    wl = workload(name)
    log("mixed matvec %s" % name)
    ctx = _ctx(wl)
    geo = OF.geometry_from_workload(wl)
    prm = oracle_params(wl)
    X, _ = OF.nodes(geo)
    mu = np.random.default_rng(2).standard_normal(2 * wl.n_nodes)
    out = zeros(mu.size)
    ctx.apply_M(dev(mu), out, fb.PART_REAL)
    assert relerr(host(out), OF.M_trap(X, wl.L, prm["xi"], prm["r_c"]) @ mu) < 2e-6
    ctx.apply_M(dev(mu), out, fb.PART_WAVE)
    assert relerr(host(out), OF.wave_se(X, mu, prm)) < 2e-6
    ctx.apply_M(dev(mu), out, fb.PART_ALL)
    M = OF.single_layer(geo, prm, order=wl.alpert_order)["M"]
    assert relerr(host(out), M @ mu) < 2e-6 + 50 * wl.tol_ewald


@pytest.mark.parametrize("name", ["tiny2", "starfish4"])
def test_mixed_em_rfd_step(name):
    wl = workload(name)
    log("mixed em-rfd %s" % name)
    ctx = _ctx(wl, tol_gmres=1e-8, tol_lanczos=1e-8)
    geo = OF.geometry_from_workload(wl)
    prm = oracle_params(wl)
    Wr, Wg, Wt = W.noise(wl, prm["grid_M"])
    delta = wl.a * 1e-2
    dQ = zeros(3 * wl.n_bodies)
    info = ctx.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), dQ)
    ref, _, _, _ = OF.em_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                  tau=wl.tau_spurious)
    log("mixed em-rfd %s: rel err %.3e info %s" % (name, relerr(host(dQ), ref), info))
    assert relerr(host(dQ), ref) < 1e-4
