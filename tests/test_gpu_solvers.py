"""GPU parity of the solvers built on the matvec: GMRES mobility (eq. 3.8),
Lanczos (M^(r))^(1/2) (eqs. 3.38-3.42), Brownian velocity (eqs. 2.4, 3.27) and
the EM-RFD step (eq. 4.3), against dense FP64 oracle solves on the same
seeded inputs.  Solver tolerances are tightened to 1e-10..1e-12 so that solver
error does not mask kernel error; the remaining difference is the method's
own spectral-Ewald error (the oracle uses the exact k-sum in M)."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import golden
from gpu_util import dev, host, log, make_ctx, oracle_params, relerr, workload, zeros
from oracle import fbim as OF

pytestmark = pytest.mark.gpu
PAPER = golden("paper_values.txt")
TIGHT = dict(tol_gmres=1e-12, tol_lanczos=1e-12)


def _dense(wl):
    geo = OF.geometry_from_workload(wl)
    return geo, oracle_params(wl), OF.DenseFBIM(geo, oracle_params(wl), order=wl.alpert_order)


@pytest.mark.parametrize("name", ["tiny2", "starfish4"])
def test_mobility_matches_dense_solve(name):
    wl = workload(name)
    log("mobility %s" % name)
    ctx = make_ctx(wl, **TIGHT)
    geo, prm, d = _dense(wl)
    U = zeros(3 * wl.n_bodies)
    info = ctx.mobility(dev(wl.F), U)
    Uo, _ = d.mobility(wl.F)
    assert info["gmres_residual"] <= 1e-12
    assert relerr(host(U), Uo) < 1e-6


@pytest.mark.parametrize("name,prec", [("tiny2", "fp64"), ("starfish4", "fp64"), ("starfish4", "mixed")])
def test_lagged_reorthogonalisation_matches_dense_solve(name, prec):
    """FBIM_FLAG_LAGGED_REORTH (delayed second Gram-Schmidt pass): the mobility solve
    against the dense oracle, and the iteration count against the two-pass default."""
    import paper_1709_01480_amd as fb
    wl = workload(name)
    log("lagged reorth %s %s" % (name, prec))
    over = dict(TIGHT) if prec == "fp64" else dict(tol_gmres=1e-8, tol_lanczos=1e-8, precision=fb.PREC_MIXED)
    geo, prm, d = _dense(wl)
    Uo, _ = d.mobility(wl.F)
    its = {}
    for flags in (0, fb.FLAG_LAGGED_REORTH):
        ctx = make_ctx(wl, flags=flags, **over)
        U = zeros(3 * wl.n_bodies)
        info = ctx.mobility(dev(wl.F), U)
        its[flags] = info["gmres_iters"]
        assert info["gmres_residual"] <= over["tol_gmres"]
        assert relerr(host(U), Uo) < (1e-6 if prec == "fp64" else 1e-5)
        ctx.close()
    log("iterations two-pass %d lagged %d" % (its[0], its[fb.FLAG_LAGGED_REORTH]))
    assert abs(its[fb.FLAG_LAGGED_REORTH] - its[0]) <= 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lagged_reorthogonalisation_with_short_restarts(prec):
    """Restart length 6 with the delayed Gram-Schmidt pass (every solve restarts
    several times and each cycle starts its lags afresh): the mobility solve against
    the dense oracle."""
    import paper_1709_01480_amd as fb
    wl = workload("starfish4")
    log("lagged reorth restart 6 %s" % prec)
    over = dict(TIGHT) if prec == "fp64" else dict(tol_gmres=1e-8, tol_lanczos=1e-8, precision=fb.PREC_MIXED)
    geo, prm, d = _dense(wl)
    Uo, _ = d.mobility(wl.F)
    ctx = make_ctx(wl, flags=fb.FLAG_LAGGED_REORTH, gmres_restart=6, **over)
    U = zeros(3 * wl.n_bodies)
    info = ctx.mobility(dev(wl.F), U)
    log("iterations %d" % info["gmres_iters"])
    assert info["gmres_residual"] <= over["tol_gmres"]
    assert relerr(host(U), Uo) < (1e-6 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("name", ["starfish4", "small12"])
def test_lagged_reorthogonalisation_batched_step(name):
    """The batched mixed EM-RFD step (lockstep solves, graphs, FP32 basis) with the
    delayed second Gram-Schmidt pass: the displacement against the oracle's step, and
    the iteration count against the same step with two passes per Arnoldi step."""
    import paper_1709_01480_amd as fb
    wl = workload(name)
    log("lagged batched step %s" % name)
    geo, prm, _ = _dense(wl)
    Wr, Wg, Wt = W.noise(wl, prm["grid_M"])
    delta = wl.a * 1e-2
    ref, _, _, _ = OF.em_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                  tau=wl.tau_spurious)
    base = fb.FLAG_BATCH_RFD | fb.FLAG_GRAPH | fb.FLAG_BASIS32
    its = {}
    for flags in (base, base | fb.FLAG_LAGGED_REORTH):
        ctx = make_ctx(wl, precision=fb.PREC_MIXED, flags=flags, tol_gmres=1e-8, tol_lanczos=1e-8)
        for rep in range(2):  # the second step replays the captured graphs
            dQ = zeros(3 * wl.n_bodies)
            info = ctx.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), dQ)
            assert info["gmres_solves"] == 3 and info["gmres_residual"] <= 1e-8
            assert relerr(host(dQ), ref) < 1e-4
        its[flags] = info["gmres_iters"]
        ctx.close()
    log("iterations two-pass %d lagged %d" % (its[base], its[base | fb.FLAG_LAGGED_REORTH]))
    assert abs(its[base | fb.FLAG_LAGGED_REORTH] - its[base]) <= 2


def test_mobility_with_slip_matches_dense_solve():
    wl = workload("tiny2")
    ctx = make_ctx(wl, **TIGHT)
    geo, prm, d = _dense(wl)
    slip = np.random.default_rng(11).standard_normal(2 * wl.n_nodes)
    U = zeros(3 * wl.n_bodies)
    mu = zeros(2 * wl.n_nodes)
    ctx.mobility(dev(wl.F), U, slip=dev(slip), mu_out=mu)
    Uo, muo = d.mobility(wl.F, slip)
    assert relerr(host(U), Uo) < 1e-6
    # mu is determined only up to the near-null normal densities: check (a) the
    # saddle equations with the device's own operator, to the solver tolerance, and
    # (b) M mu, which does not see those modes, against the oracle's M mu (each side
    # with its own operator: the spectral-Ewald M differs from the exact k-sum by
    # the split's truncation error, which |mu| ~ 100 would amplify)
    muh = host(mu)
    Mmu = zeros(2 * wl.n_nodes)
    ctx.apply_M(mu, Mmu)
    Kx = d.K
    r1 = host(Mmu) - Kx @ host(U) + slip
    r2 = -Kx.T @ muh + wl.F
    nb = np.linalg.norm(np.concatenate([slip, wl.F]))
    assert np.linalg.norm(np.concatenate([r1, r2])) < 1e-10 * nb
    M = d.mats["M"]
    assert relerr(host(Mmu), M @ muo) < 1e-6


@pytest.mark.parametrize("phi", [0.01, 0.05])
def test_square_array_drag_on_gpu(phi):
    """Eq. 4.1 (Sangani-Acrivos dilute expansion) through the GPU mobility solve."""
    l = math.sqrt(math.pi / phi)
    wl = W.disk_lattice(l, 64, tol=1e-9, n_box=4)
    ctx = make_ctx(wl, **TIGHT)
    U = zeros(3)
    ctx.mobility(dev(np.array([1.0, 0.0, 0.0])), U)
    drag = 1.0 / host(U)[0]
    c0, c2, c3 = PAPER["hasimoto_c0"][0], PAPER["hasimoto_c2"][0], PAPER["hasimoto_c3"][0]
    th = 4 * math.pi / (-math.log(math.sqrt(phi)) - c0 + phi + c2 * phi ** 2 + c3 * phi ** 3)
    assert abs(drag - th) / th < 4e-4


def test_starfish_rotational_mobility_on_gpu():
    """Section 4.4.1: kT <N_thth> ~ 0.2081 for the four-arm starfish (16 angles)."""
    ntt = []
    for th in np.arange(16) * (math.pi / 2) / 16:
        wl = W.single_starfish(theta=th, n_p=64, tol=1e-9, n_box=3)
        ctx = make_ctx(wl, **TIGHT)
        U = zeros(3)
        ctx.mobility(dev(np.array([0.0, 0.0, 1.0])), U)
        ntt.append(host(U)[2])
        ctx.close()
    v, tol, _ = PAPER["chi_rot_starfish"]
    assert abs(np.mean(ntt) - v) / v < tol


def test_random_field_is_real_part_definition():
    wl = workload("tiny2")
    ctx = make_ctx(wl)
    geo, prm, d = _dense(wl)
    M = prm["grid_M"]
    Wg = np.random.default_rng(5).standard_normal(2 * M * M)
    out = zeros(2 * wl.n_nodes)
    ctx.random_field(dev(Wg), out)
    assert relerr(host(out), OF.random_field(d.X, Wg, prm)) < 1e-9


@pytest.mark.parametrize("name", ["tiny2", "starfish4"])
def test_lanczos_sqrt_matches_dense(name):
    wl = workload(name)
    log("lanczos %s" % name)
    ctx = make_ctx(wl, **TIGHT)
    geo, prm, d = _dense(wl)
    Wr = np.random.default_rng(9).standard_normal(2 * wl.n_nodes)
    out = zeros(2 * wl.n_nodes)
    info = ctx.sqrt_Mr(dev(Wr), out)
    G, Gp = OF.G_blocks(geo, prm, wl.alpert_order, wl.tau_spurious)
    ref = OF.slip_real(d.mats["Mr"], G, Gp, Wr)
    assert info["lanczos_iters"] < 200
    assert relerr(host(out), ref) < 1e-8


@pytest.mark.parametrize("name", ["tiny2", "starfish4"])
def test_brownian_velocity_matches_dense(name):
    wl = workload(name)
    log("brownian %s" % name)
    ctx = make_ctx(wl, **TIGHT)
    geo, prm, d = _dense(wl)
    Wr, Wg, _ = W.noise(wl, prm["grid_M"])
    U = zeros(3 * wl.n_bodies)
    ctx.brownian_velocity(wl.dt, dev(wl.F), dev(Wr), dev(Wg), U)
    Uo = d.brownian_velocity(wl.F, Wr, Wg, wl.kT, wl.dt)
    assert relerr(host(U), Uo) < 1e-6


@pytest.mark.parametrize("name", ["tiny2", "starfish4"])
def test_em_rfd_step_matches_oracle(name):
    wl = workload(name)
    log("em-rfd %s" % name)
    ctx = make_ctx(wl, **TIGHT)
    geo, prm, _ = _dense(wl)
    Wr, Wg, Wt = W.noise(wl, prm["grid_M"])
    delta = wl.a * 1e-2
    dQ = zeros(3 * wl.n_bodies)
    info = ctx.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), dQ)
    ref, _, _, _ = OF.em_rfd_step(geo, prm, wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                  tau=wl.tau_spurious)
    assert info["gmres_solves"] == 3
    assert relerr(host(dQ), ref) < 1e-6
    # the configuration is restored afterwards
    U = zeros(3 * wl.n_bodies)
    ctx.mobility(dev(wl.F), U)
    Uo, _ = OF.DenseFBIM(geo, prm, order=wl.alpert_order).mobility(wl.F)
    assert relerr(host(U), Uo) < 1e-6


@pytest.mark.parametrize("shift", [3e-7, 1e-4])
def test_overlap_detection(shift):
    """Two copies of one body a tiny shift apart: their nodes are closer than 5% of
    the node spacing, which set_bodies refuses (EOVERLAP); the same copies one
    body diameter apart are accepted.  (The check rides on the count pass of the
    neighbour lists.)"""
    import paper_1709_01480_amd as fb
    wl = workload("starfish4")
    ctx = fb.Context(**wl.params())
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    q = np.array([[0.3, 0.3], [0.3 + shift, 0.3]])
    with pytest.raises(fb.FbimError) as e:
        ctx.set_bodies(np.full(2, sid), q, np.zeros(2))
    assert e.value.status == 3
    q[1] = [0.3 + 3.0 * wl.r_s, 0.3]
    ctx.set_bodies(np.full(2, sid), q, np.zeros(2))
