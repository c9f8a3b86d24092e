"""The time-stepping variants of Section 4.4 on the GPU against the oracle:
the Euler-Maruyama step without the drift term (delta = 0, Section 4.4.1), the
stochastic Adams-Bashforth step with the random finite difference (the AB2-RFD
equation) carrying N F from one step to the next, sequential and batched, and
RFD solves at their own looser GMRES tolerance (the spring-pair runs)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, host, log, make_ctx, oracle_params, relerr, workload, zeros
from oracle import fbim as OF

pytestmark = pytest.mark.gpu
TIGHT = dict(tol_gmres=1e-11, tol_lanczos=1e-11)


def _inputs(wl, ctx):
    return W.noise(wl, ctx.get_derived()["grid_M"])


@pytest.mark.parametrize("mode", ["sequential", "batch_rfd_flag"])
def test_step_without_drift_matches_oracle(mode):
    import paper_1709_01480_amd as fb
    wl = workload("starfish4")
    log("EM without RFD, %s" % mode)
    flags = (fb.FLAG_BATCH_RFD | fb.FLAG_GRAPH) if mode == "batch_rfd_flag" else 0
    ctx = make_ctx(wl, flags=flags, **TIGHT)
    Wr, Wg, Wt = _inputs(wl, ctx)
    dQ = zeros(3 * wl.n_bodies)
    info = ctx.step_em_rfd(wl.dt, 0.0, dev(wl.F), dev(Wr), dev(Wg), None, dQ)
    assert info["gmres_solves"] == 1
    ref, _, _, _ = OF.em_rfd_step(OF.geometry_from_workload(wl), oracle_params(wl), wl.F, Wr, Wg, Wt, wl.kT,
                                  wl.dt, 0.0, order=wl.alpert_order, tau=wl.tau_spurious)
    assert relerr(host(dQ), ref) < 1e-6


def test_ab2_steps_match_oracle():
    wl = workload("starfish4")
    log("AB2-RFD sequential")
    ctx = make_ctx(wl, **TIGHT)
    geo, prm = OF.geometry_from_workload(wl), oracle_params(wl)
    Wr, Wg, Wt = _inputs(wl, ctx)
    delta = 1e-2 * wl.a
    hist, dQ = zeros(3 * wl.n_bodies), zeros(3 * wl.n_bodies)
    # first step: no history, the EM-RFD step; the history becomes N F
    info = ctx.step_ab2_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), hist, False, dQ)
    assert info["gmres_solves"] == 4
    ref1, NF1 = OF.ab2_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                tau=wl.tau_spurious)
    assert relerr(host(dQ), ref1) < 1e-6 and relerr(host(hist), NF1) < 1e-8
    # second step with another force: 3/2 N F2 - 1/2 N F1
    F2 = np.random.default_rng(31).standard_normal(3 * wl.n_bodies)
    ctx.step_ab2_rfd(wl.dt, delta, dev(F2), dev(Wr), dev(Wg), dev(Wt), hist, True, dQ)
    ref2, NF2 = OF.ab2_rfd_step(geo, prm, F2, Wr, Wg, Wt, wl.kT, wl.dt, delta, NF_prev=NF1,
                                order=wl.alpert_order, tau=wl.tau_spurious)
    assert relerr(host(dQ), ref2) < 1e-6 and relerr(host(hist), NF2) < 1e-8


@pytest.mark.parametrize("delta_scale", [1e-2, 0.0])
def test_batched_ab2_step_matches_oracle(delta_scale):
    import paper_1709_01480_amd as fb
    wls = [workload("starfish4"), workload("tiny2")]
    log("AB2-RFD batch, delta %g a" % delta_scale)
    prms = []
    for wl in wls:
        p = wl.params()
        p.update(TIGHT)
        prms.append(p)
    b = fb.Batch(prms, graph=True)
    for m, wl in zip(b.members, wls):
        sid = m.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
        m.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    noise = [_inputs(wl, m) for wl, m in zip(wls, b.members)]
    delta = delta_scale * min(wl.a for wl in wls)
    hists = [dev(np.random.default_rng(40 + k).standard_normal(3 * wl.n_bodies)) for k, wl in enumerate(wls)]
    prev = [host(h).copy() for h in hists]
    dQs = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.step_ab2_rfd(wls[0].dt, delta, [dev(wl.F) for wl in wls], [dev(n[0]) for n in noise],
                           [dev(n[1]) for n in noise], [dev(n[2]) for n in noise], hists, True, dQs)
    for wl, nz, dQ, h, p, info in zip(wls, noise, dQs, hists, prev, infos):
        assert info["gmres_solves"] == (4 if delta > 0 else 2)
        ref, NF = OF.ab2_rfd_step(OF.geometry_from_workload(wl), oracle_params(wl), wl.F, *nz, wl.kT, wl.dt,
                                  delta, NF_prev=p, order=wl.alpert_order, tau=wl.tau_spurious)
        assert relerr(host(dQ), ref) < 1e-6, wl.name
        assert relerr(host(h), NF) < 1e-8, wl.name


@pytest.mark.parametrize("batch", [False, True])
def test_loose_rfd_tolerance(batch):
    # RFD solves at 1e-3, the Brownian solve at 1e-8: fewer iterations, every solve
    # within its own tolerance
    import paper_1709_01480_amd as fb
    wl = workload("small12")
    log("loose RFD tolerance, batch %s" % batch)
    flags = (fb.FLAG_BATCH_RFD | fb.FLAG_GRAPH) if batch else 0
    tight = make_ctx(wl, flags=flags, tol_gmres=1e-8, tol_lanczos=1e-8)
    loose = make_ctx(wl, flags=flags, tol_gmres=1e-8, tol_lanczos=1e-8, tol_rfd=1e-3)
    Wr, Wg, Wt = _inputs(wl, tight)
    delta = 1e-2 * wl.a
    d0, d1 = zeros(3 * wl.n_bodies), zeros(3 * wl.n_bodies)
    i0 = tight.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), d0)
    i1 = loose.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), d1)
    log("iterations tight %d loose %d; residual tight %.2e loose %.2e"
        % (i0["gmres_iters"], i1["gmres_iters"], i0["gmres_residual"], i1["gmres_residual"]))
    assert i1["gmres_iters"] < i0["gmres_iters"]
    assert i0["gmres_residual"] <= 1e-8 and i1["gmres_residual"] <= 1e-3
    # the Brownian displacement is unchanged: with Wt = 0 the RFD solves are trivial
    z = np.zeros(3 * wl.n_bodies)
    tight.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(z), d0)
    loose.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(z), d1)
    assert relerr(host(d1), host(d0)) < 1e-12
