"""The device noise generator against the oracle's re-implementation of the
same published definition (Philox4x32-10 + Box-Muller): raw words bit for
bit, normals to the last bits of the transcendental functions, and steps that
draw their own noise against steps given the oracle's draw."""
import math

import numpy as np
import pytest

from gpu_util import dev, host, log, make_ctx, oracle_params, relerr, workload, zeros
from oracle import fbim as OF
from oracle import philox as PH

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,stream,counter,npairs", [(0, 0, 0, 1), (1709, 1, 3, 4097),
                                                        (0xFEDCBA9876543210, 2, (5 << 32) + 11, 257)])
def test_words_bit_exact(seed, stream, counter, npairs):
    import torch
    log("philox words seed=%x stream=%d counter=%d n=%d" % (seed, stream, counter, npairs))
    ctx = make_ctx(workload("tiny2"), seed=seed)
    out = torch.zeros(4 * npairs, dtype=torch.int32, device="cuda")
    ctx.noise_words(stream, counter, out)
    got = out.cpu().numpy().view(np.uint32).reshape(npairs, 4).T.astype(np.uint64)
    ref = PH.raw_words(seed, stream, counter, npairs)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [1, 2, 1001, 1 << 20])
def test_normals_match_oracle(n):
    log("normals n=%d" % n)
    ctx = make_ctx(workload("tiny2"), seed=42)
    out = zeros(n)
    ctx.noise_normals(1, 9, out)
    z = host(out)
    ref = PH.normals(42, 1, 9, n)
    # same uniforms; log, sqrt and sincos of the two math libraries agree to a few ulp
    assert np.max(np.abs(z - ref)) < 1e-14 * max(1.0, np.max(np.abs(ref)))
    if n >= 1 << 20:
        assert abs(z.mean()) < 5 / math.sqrt(n) and abs(z.var() - 1) < 5 * math.sqrt(2 / n)


def test_step_draws_its_own_noise_reproducibly():
    # a step with NULL noise equals a step given the generator's draw at the
    # reported counter; the counter advances by one per step
    wl = workload("starfish4")
    ctx = make_ctx(wl, seed=77, tol_gmres=1e-10, tol_lanczos=1e-10)
    M = ctx.get_derived()["grid_M"]
    k = ctx.noise_counter()
    assert k == 0
    delta = wl.a * 1e-2
    dQ1 = zeros(3 * wl.n_bodies)
    ctx.step_em_rfd(wl.dt, delta, dev(wl.F), None, None, None, dQ1)
    assert ctx.noise_counter() == k + 1
    Wr = PH.normals(77, PH.STREAM_W_R, k, 2 * wl.n_nodes)
    Wg = PH.normals(77, PH.STREAM_W_GRID, k, 2 * M * M)
    Wt = PH.normals(77, PH.STREAM_W_TILDE, k, 3 * wl.n_bodies)
    dQ2 = zeros(3 * wl.n_bodies)
    # the explicit call is given the oracle's draw (a few ulp from the device's)
    ctx.step_em_rfd(wl.dt, delta, dev(wl.F), dev(Wr), dev(Wg), dev(Wt), dQ2)
    assert ctx.noise_counter() == k + 1
    assert relerr(host(dQ1), host(dQ2)) < 1e-9
    geo = OF.geometry_from_workload(wl)
    ref, _, _, _ = OF.em_rfd_step(geo, oracle_params(wl), wl.F, Wr, Wg, Wt, wl.kT, wl.dt, delta,
                                  order=wl.alpert_order, tau=wl.tau_spurious)
    assert relerr(host(dQ1), ref) < 1e-6
    # the next step draws new noise
    dQ3 = zeros(3 * wl.n_bodies)
    ctx.step_em_rfd(wl.dt, delta, dev(wl.F), None, None, None, dQ3)
    assert ctx.noise_counter() == k + 2
    assert relerr(host(dQ3), host(dQ1)) > 1e-3


def test_brownian_velocity_with_drawn_noise():
    wl = workload("tiny2")
    ctx = make_ctx(wl, seed=5, tol_gmres=1e-12, tol_lanczos=1e-12)
    ctx.set_noise_counter(40)
    M = ctx.get_derived()["grid_M"]
    U = zeros(3 * wl.n_bodies)
    ctx.brownian_velocity(wl.dt, dev(wl.F), None, None, U)
    assert ctx.noise_counter() == 41
    Wr = PH.normals(5, PH.STREAM_W_R, 40, 2 * wl.n_nodes)
    Wg = PH.normals(5, PH.STREAM_W_GRID, 40, 2 * M * M)
    geo = OF.geometry_from_workload(wl)
    d = OF.DenseFBIM(geo, oracle_params(wl), order=wl.alpert_order)
    assert relerr(host(U), d.brownian_velocity(wl.F, Wr, Wg, wl.kT, wl.dt)) < 1e-6
