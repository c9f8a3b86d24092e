"""GPU parity of the batched entry points: several independent systems of
different sizes (and grid sizes) through one launch per stage must give each
system's own single-system results.

Bars: the batched matvec runs the same per-system arithmetic (the spreading's
sums are exact fixed-point integers, so the order of its LDS atomics does not
matter), so 1e-12 relative; batched GMRES runs
each system's own Krylov iteration, so solutions agree to the solver
tolerance (GMRES at 1e-10 here: 1e-8 relative); the EM-RFD step as the
single-system step (1e-6, the step's parity bar against the oracle)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, host, log, make_ctx, relerr, zeros

pytestmark = pytest.mark.gpu

NAMES = ["tiny2", "starfish4", "small12"]


def _setup_member(ctx, wl):
    import paper_1709_01480_amd as fb
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)


def _batch(wls, graph=False, **over):
    import paper_1709_01480_amd as fb
    prms = []
    for wl in wls:
        p = wl.params()
        p.update(over)
        prms.append(p)
    b = fb.Batch(prms, graph=graph)
    for m, wl in zip(b.members, wls):
        _setup_member(m, wl)
    return b


def test_batched_matvec_matches_each_system():
    wls = [W.make(n) for n in NAMES]
    log("batch matvec %s" % NAMES)
    b = _batch(wls)
    rng = np.random.default_rng(3)
    mus = [dev(rng.standard_normal(2 * wl.n_nodes)) for wl in wls]
    outs = [zeros(2 * wl.n_nodes) for wl in wls]
    b.apply_M(mus, outs)
    for wl, mu, out in zip(wls, mus, outs):
        ctx = make_ctx(wl)
        ref = zeros(2 * wl.n_nodes)
        ctx.apply_M(mu, ref)
        assert relerr(host(out), host(ref)) < 1e-12, wl.name


@pytest.mark.parametrize("graph", [False, True])
def test_batched_mobility_matches_each_system(graph):
    wls = [W.make(n) for n in NAMES]
    log("batch mobility graph=%s" % graph)
    b = _batch(wls, graph=graph, tol_gmres=1e-10)
    Fs = [dev(wl.F) for wl in wls]
    for rep in range(2):  # the second call replays the captured graph
        Us = [zeros(3 * wl.n_bodies) for wl in wls]
        infos = b.mobility(Fs, Us)
        log("rep %d infos %s" % (rep, [(i["gmres_iters"], i["gmres_residual"]) for i in infos]))
        for wl, U, info in zip(wls, Us, infos):
            ctx = make_ctx(wl, tol_gmres=1e-10)
            ref = zeros(3 * wl.n_bodies)
            ri = ctx.mobility(dev(wl.F), ref)
            assert info["gmres_residual"] <= 1e-10
            assert abs(info["gmres_iters"] - ri["gmres_iters"]) <= 1
            assert relerr(host(U), host(ref)) < 1e-8, wl.name


def test_uneven_suspensions_batched_mobility():
    """Eight suspensions of 6..40 bodies with 32..64 nodes per body, different
    grids, in one batch."""
    rng = np.random.default_rng(11)
    wls = []
    for k in range(8):
        n = int(rng.integers(6, 41))
        n_p = int(rng.choice([32, 48, 64]))
        r_s = float(np.sqrt(0.15 / (n * np.pi * 1.045)))
        wls.append(W.make("small12", seed=50 + k, n_bodies=n, n_p=n_p, r_s=r_s,
                          n_box=4, grid_M=int(rng.choice([64, 96, 128])), tol_ewald=1e-8))
    log("uneven batch %s" % [(w.n_bodies, w.n_p, w.grid_M) for w in wls])
    b = _batch(wls, tol_gmres=1e-10)
    Fs = [dev(wl.F) for wl in wls]
    Us = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.mobility(Fs, Us)
    for wl, U, info in zip(wls, Us, infos):
        ctx = make_ctx(wl, tol_gmres=1e-10)
        ref = zeros(3 * wl.n_bodies)
        ctx.mobility(dev(wl.F), ref)
        assert info["gmres_residual"] <= 1e-10
        assert relerr(host(U), host(ref)) < 1e-8


@pytest.mark.parametrize("basis32,graph,lagged", [(False, False, False), (True, False, False), (True, True, False),
                                                  (False, False, True), (True, True, True)])
def test_batched_mixed_mobility_reaches_fp64_tolerance(basis32, graph, lagged):
    """Relaxed-matvec GMRES, with the Krylov basis in FP64 or FP32, with two
    Gram-Schmidt passes per step or the second one delayed (FBIM_FLAG_LAGGED_REORTH):
    the FP64 restart residual meets the tolerance, and the solution matches the FP64
    context's to the accuracy that tolerance allows.  Each system switches to the
    FP32 operator on its own and leaves the lockstep launches when it converges (the
    delayed passes then take the remaining systems' lags in the new order); with
    graphs on (three systems) the launch sets of mixed groupings run eagerly, the
    others from graphs."""
    import paper_1709_01480_amd as fb
    wls = [W.make(n) for n in NAMES]
    flags = (fb.FLAG_BASIS32 if basis32 else 0) | (fb.FLAG_LAGGED_REORTH if lagged else 0)
    b = _batch(wls, graph=graph, precision=fb.PREC_MIXED, tol_gmres=1e-8, flags=flags)
    Fs = [dev(wl.F) for wl in wls]
    Us = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.mobility(Fs, Us)
    log("basis32 %s lagged %s iterations %s" % (basis32, lagged, [i["gmres_iters"] for i in infos]))
    for wl, U, info in zip(wls, Us, infos):
        assert info["status"] == 0
        assert info["gmres_residual"] <= 1e-8
        ctx = make_ctx(wl, tol_gmres=1e-10)
        ref = zeros(3 * wl.n_bodies)
        ctx.mobility(dev(wl.F), ref)
        assert relerr(host(U), host(ref)) < 1e-6


@pytest.mark.parametrize("lagged", [False, True])
def test_batched_mobility_with_short_restarts(lagged):
    """Restart length 6, so every solve restarts several times (with the delayed
    Gram-Schmidt pass each cycle starts its lags afresh): the FP64 restart residual
    meets the tolerance and the solution matches each system solved alone with the
    default restart length."""
    import paper_1709_01480_amd as fb
    wls = [W.make(n) for n in NAMES]
    b = _batch(wls, tol_gmres=1e-10, gmres_restart=6, flags=fb.FLAG_LAGGED_REORTH if lagged else 0)
    Fs = [dev(wl.F) for wl in wls]
    Us = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.mobility(Fs, Us)
    log("restart 6 lagged %s iterations %s" % (lagged, [i["gmres_iters"] for i in infos]))
    for wl, U, info in zip(wls, Us, infos):
        assert info["status"] == 0
        assert info["gmres_residual"] <= 1e-10
        ctx = make_ctx(wl, tol_gmres=1e-10, flags=fb.FLAG_LAGGED_REORTH if lagged else 0)
        ref = zeros(3 * wl.n_bodies)
        ctx.mobility(dev(wl.F), ref)
        assert relerr(host(U), host(ref)) < 1e-8
        ctx.close()


def test_batched_em_rfd_matches_each_system():
    wls = [W.make(n) for n in NAMES[:2]]
    log("batch em-rfd")
    b = _batch(wls, tol_gmres=1e-10, tol_lanczos=1e-10)
    args = []
    for m, wl in zip(b.members, wls):
        M = m.get_derived()["grid_M"]
        Wr, Wg, Wt = W.noise(wl, M)
        args.append((dev(wl.F), dev(Wr), dev(Wg), dev(Wt)))
    dQs = [zeros(3 * wl.n_bodies) for wl in wls]
    delta = 1e-2 * wls[0].a
    infos = b.step_em_rfd(1e-3, delta, [a[0] for a in args], [a[1] for a in args], [a[2] for a in args],
                          [a[3] for a in args], dQs)
    for wl, a, dQ, info in zip(wls, args, dQs, infos):
        assert info["gmres_solves"] == 3
        ctx = make_ctx(wl, tol_gmres=1e-10, tol_lanczos=1e-10)
        ref = zeros(3 * wl.n_bodies)
        ctx.step_em_rfd(1e-3, delta, a[0], a[1], a[2], a[3], ref)
        assert relerr(host(dQ), host(ref)) < 1e-6, wl.name


@pytest.mark.parametrize("graph", [False, True])
def test_single_context_batched_rfd_flag(graph):
    import paper_1709_01480_amd as fb
    wl = W.make("starfish4")
    ctx0 = make_ctx(wl, tol_gmres=1e-10, tol_lanczos=1e-10)
    ctx1 = make_ctx(wl, tol_gmres=1e-10, tol_lanczos=1e-10,
                    flags=fb.FLAG_BATCH_RFD | (fb.FLAG_GRAPH if graph else 0))
    Wr, Wg, Wt = W.noise(wl, ctx0.get_derived()["grid_M"])
    d0, d1 = zeros(3 * wl.n_bodies), zeros(3 * wl.n_bodies)
    delta = 1e-2 * wl.a
    i0 = ctx0.step_em_rfd(1e-3, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), d0)
    for rep in range(2):  # with a graph the second step replays the captured graph
        i1 = ctx1.step_em_rfd(1e-3, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), d1)
        assert i1["gmres_solves"] == 3
        assert relerr(host(d1), host(d0)) < 1e-6
    # the configuration is restored in both
    U0, U1 = zeros(3 * wl.n_bodies), zeros(3 * wl.n_bodies)
    ctx0.mobility(dev(wl.F), U0)
    ctx1.mobility(dev(wl.F), U1)
    assert relerr(host(U1), host(U0)) < 1e-8
    del i0


def test_uneven_suspension_batch_of_sixteen():
    """Sixteen independent suspensions drawn as the uneven-batch workload (bodies
    log-uniform in [16, 512], 64 / 128 / 256 nodes per body, area fraction 0.2,
    tol 1e-6; ~3.7e5 nodes, grids 128..1024 on the fused transform path): one
    batched mobility solve against each suspension's own context."""
    wls = W.uneven_suspensions(16)
    log("cfg3-style batch: %s" % [(w.n_bodies, w.n_p, w.grid_M) for w in wls])
    b = _batch(wls, tol_gmres=1e-8)
    Us = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.mobility([dev(wl.F) for wl in wls], Us)
    log("iterations %s" % [i["gmres_iters"] for i in infos])
    for wl, U, info in zip(wls, Us, infos):
        assert info["gmres_residual"] <= 1e-8
        ctx = make_ctx(wl, tol_gmres=1e-8)
        ref = zeros(3 * wl.n_bodies)
        ctx.mobility(dev(wl.F), ref)
        assert relerr(host(U), host(ref)) < 1e-6, (wl.n_bodies, wl.n_p)


def test_uneven_suspension_batch_full_size():
    """The uneven-suspension batch at full size: 64 suspensions (bodies
    log-uniform in [16, 512], 64 / 128 / 256 nodes per body, area fraction 0.2;
    9824 bodies, 1.42e6 nodes, grids 128..1024), graphs on, one batched mobility
    solve.  Every suspension meets the tolerance on its FP64 true residual, and
    the smallest, the largest and two other suspensions match their own contexts."""
    wls = W.uneven_suspensions(64)
    log("full uneven batch: %d suspensions, %d nodes" % (len(wls), sum(w.n_nodes for w in wls)))
    b = _batch(wls, graph=True, tol_gmres=1e-8)
    Us = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.mobility([dev(wl.F) for wl in wls], Us)
    log("iterations min %d max %d" % (min(i["gmres_iters"] for i in infos), max(i["gmres_iters"] for i in infos)))
    for info in infos:
        assert info["status"] == 0 and info["gmres_residual"] <= 1e-8
    sizes = [wl.n_nodes for wl in wls]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 40})
    for k in pick:
        wl = wls[k]
        ctx = make_ctx(wl, tol_gmres=1e-8)
        ref = zeros(3 * wl.n_bodies)
        ctx.mobility(dev(wl.F), ref)
        assert relerr(host(Us[k]), host(ref)) < 1e-6, (k, wl.n_bodies, wl.n_p)


@pytest.mark.parametrize("basis32", [False, True])
def test_mixed_batched_rfd_step_matches_sequential(basis32):
    """Mixed contexts: the EM-RFD step with the batched solves (U0 and U+ in one
    lockstep solve, then U- from U+), graphs on, with an FP64 or FP32 Krylov
    basis, against the same context type solving one system after another."""
    import paper_1709_01480_amd as fb
    wl = W.make("small12")
    flags = fb.FLAG_BATCH_RFD | fb.FLAG_GRAPH | (fb.FLAG_BASIS32 if basis32 else 0)
    ctx0 = make_ctx(wl, precision=fb.PREC_MIXED, tol_gmres=1e-9, tol_lanczos=1e-10)
    ctx1 = make_ctx(wl, precision=fb.PREC_MIXED, tol_gmres=1e-9, tol_lanczos=1e-10, flags=flags)
    Wr, Wg, Wt = W.noise(wl, ctx0.get_derived()["grid_M"])
    d0, d1 = zeros(3 * wl.n_bodies), zeros(3 * wl.n_bodies)
    delta = 1e-2 * wl.a
    i0 = ctx0.step_em_rfd(1e-3, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), d0)
    for rep in range(3):  # replays of the captured graphs
        i1 = ctx1.step_em_rfd(1e-3, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), d1)
        log("basis32 %s rep %d iterations %d (sequential %d)" % (basis32, rep, i1["gmres_iters"], i0["gmres_iters"]))
        assert i1["status"] == 0 and i1["gmres_solves"] == 3
        assert i1["gmres_residual"] <= 1e-9
        assert relerr(host(d1), host(d0)) < 1e-6


def test_uneven_batch_em_rfd_step_against_oracle():
    """The uneven-suspension workload as a batched EM-RFD step: 64 suspensions,
    mixed precision with the FP32 Krylov basis, graphs on, three right-hand sides
    per suspension (U0 at Q, U+- at Q +- delta/2 Wt) in lockstep launch sets.
    Every member meets the GMRES tolerance on its FP64 true residual; the two
    smallest suspensions' displacements match the matrix-free FP64 oracle's step
    (eq. 4.3) at the mixed-precision bar 1e-4."""
    import paper_1709_01480_amd as fb
    from gpu_util import oracle_params
    from oracle import fbim as OF
    from oracle import matfree as MF
    wls = W.uneven_suspensions(64)
    log("uneven batch EM-RFD: %d suspensions, %d nodes" % (len(wls), sum(w.n_nodes for w in wls)))
    b = _batch(wls, graph=True, precision=fb.PREC_MIXED, flags=fb.FLAG_BASIS32, tol_gmres=1e-8, tol_lanczos=1e-8)
    noise = [W.noise(wl, m.get_derived()["grid_M"]) for wl, m in zip(wls, b.members)]
    delta = min(wl.a for wl in wls) * 1e-2
    dt = 1e-3
    dQs = [zeros(3 * wl.n_bodies) for wl in wls]
    infos = b.step_em_rfd(dt, delta, [dev(wl.F) for wl in wls], [dev(n[0]) for n in noise],
                          [dev(n[1]) for n in noise], [dev(n[2]) for n in noise], dQs)
    log("iterations min %d max %d" % (min(i["gmres_iters"] for i in infos), max(i["gmres_iters"] for i in infos)))
    for info in infos:
        assert info["status"] == 0 and info["gmres_solves"] == 3 and info["gmres_residual"] <= 1e-8
    sizes = [wl.n_nodes for wl in wls]
    for k in np.argsort(sizes)[:2]:
        wl, m = wls[k], b.members[k]
        prm = oracle_params(wl)
        d = m.get_derived()
        assert prm["grid_M"] == d["grid_M"] and prm["P"] == d["P"] and abs(prm["xi"] / d["xi"] - 1) < 1e-12
        ref, _, _, _, _ = MF.em_rfd_step(OF.geometry_from_workload(wl), prm, wl.F, *noise[k], wl.kT, dt, delta,
                                         order=wl.alpert_order, tau=wl.tau_spurious, tol=1e-10)
        err = relerr(host(dQs[k]), ref)
        log("member %d (%d x %d): rel err %.3e" % (k, wl.n_bodies, wl.n_p, err))
        assert err < 1e-4
