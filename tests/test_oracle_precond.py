"""Pins of the reference block preconditioner (oracle/precond.py), and the
measured effect of correcting each body's mobility block on GMRES.

The learned preconditioner correction of the library targets N_bb, the
exact self-mobility of each body inside the suspension.  The last test
records what even the exact target buys: on a dense suspension (area fraction
0.4) the iteration count is unchanged, because the iterations are spent
resolving the densities of nearly touching bodies (the mu block), which the
rigid-body correction leaves untouched by construction."""
import math

import numpy as np

import workloads as W
from oracle import fbim as OF
from oracle import precond as OP


def _system(n, n_p, phi, seed):
    r_s = math.sqrt(phi / (n * math.pi * (1 + 0.5 * 0.3 ** 2)))
    wl = W.make("dense200", seed=seed, n_bodies=n, n_p=n_p, r_s=r_s, grid_M=0, n_box=4, tol_ewald=1e-6)
    geo = OF.geometry_from_workload(wl)
    prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=4)
    M = OF.single_layer(geo, prm, order=4)["M"]
    K = OF.K_matrix(geo)
    N2 = M.shape[0]
    A = np.block([[M, -K], [-K.T, np.zeros((K.shape[1], K.shape[1]))]])
    return wl, geo, M, K, A, N2


def test_block_preconditioner_inverts_a_single_body():
    wl, geo, M, K, A, N2 = _system(1, 32, 0.05, 1)
    P, _ = OP.block_preconditioner(M, K, geo.offsets())
    z = np.random.default_rng(0).standard_normal(A.shape[0])
    # exact up to the spurious (near-null) density modes of M: compare the
    # rigid-body velocities and the velocity residual
    y = P(z)
    r = A @ y - z
    assert np.linalg.norm(r) < 1e-6 * np.linalg.norm(z)
    _, its = OP.gmres(A, z, P, tol=1e-10)
    assert its <= 3


def test_corrected_block_is_the_exact_inverse_of_the_modified_block():
    wl, geo, M, K, A, N2 = _system(1, 32, 0.05, 2)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((3, 3))
    C = 1e-3 * (B + B.T)
    P, Nref = OP.block_preconditioner(M, K, geo.offsets(), C=C[None])
    Am = A.copy()
    Am[:N2, :N2] += K @ C @ K.T
    z = rng.standard_normal(A.shape[0])
    assert np.linalg.norm(Am @ P(z) - z) < 1e-6 * np.linalg.norm(z)
    # the modified block's body mobility is N_ref + C
    Nm = np.linalg.inv(K.T @ OP.pinv_sym(Am[:N2, :N2]) @ K)
    assert np.max(np.abs(Nm - (Nref[0] + C))) < 1e-8 * np.max(np.abs(Nref[0]))


def test_exact_self_mobility_correction_leaves_iterations_unchanged():
    wl, geo, M, K, A, N2 = _system(16, 32, 0.4, 5)
    off = geo.offsets()
    P0, Nref = OP.block_preconditioner(M, K, off)
    Nfull = OF.body_mobility(M, K)
    n = wl.n_bodies
    C = np.array([Nfull[3 * b:3 * b + 3, 3 * b:3 * b + 3] - Nref[b] for b in range(n)])
    # the correction is far from small in this dense suspension ...
    rel = [np.linalg.norm(C[b]) / np.linalg.norm(Nref[b]) for b in range(n)]
    assert np.mean(rel) > 0.2
    P1, _ = OP.block_preconditioner(M, K, off, C=C)
    rhs = -np.concatenate([np.zeros(N2), np.random.default_rng(2).standard_normal(3 * n)])
    x0, i0 = OP.gmres(A, rhs, P0, tol=1e-8)
    x1, i1 = OP.gmres(A, rhs, P1, tol=1e-8)
    # ... yet GMRES takes (within one) the same number of iterations, to the same solution
    assert abs(i1 - i0) <= 1
    assert np.max(np.abs(x1[N2:] - x0[N2:])) < 1e-6 * np.max(np.abs(x0[N2:]))


def test_reference_preconditioner_is_exact_for_the_reference_orientation():
    # one body at theta = 0 is its own reference configuration: the rotated
    # reference block is the body's block, so both constructions coincide
    wl, geo, M, K, A, N2 = _system(1, 32, 0.05, 1)
    geo.theta[:] = 0.0
    prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=4)
    M = OF.single_layer(geo, prm, order=4)["M"]
    K = OF.K_matrix(geo)
    P_ref, N_ref = OP.reference_preconditioner(geo, prm)
    P_blk, N_blk = OP.block_preconditioner(M, K, geo.offsets())
    z = np.random.default_rng(2).standard_normal(N2 + 3)
    assert np.allclose(P_ref(z), P_blk(z), rtol=0, atol=1e-8 * np.max(np.abs(P_blk(z))))
    assert np.max(np.abs(N_ref[0] - N_blk[0])) < 1e-10 * np.max(np.abs(N_blk[0]))


def test_reference_preconditioner_rotates_with_the_body():
    # the rotated reference block approximates each body's own block (the
    # periodic lattice's anisotropy is small for a body much smaller than the
    # box); planting the transposed rotation breaks the density part
    wl, geo, M, K, A, N2 = _system(3, 32, 0.05, 4)
    prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=4)
    P_ref, N_ref = OP.reference_preconditioner(geo, prm)
    P_blk, N_blk = OP.block_preconditioner(M, K, geo.offsets())
    for b in range(3):
        assert np.max(np.abs(N_ref[b] - N_blk[b])) < 1e-4 * np.max(np.abs(N_blk[b]))
    z = np.random.default_rng(3).standard_normal(A.shape[0])
    yr, yb = P_ref(z), P_blk(z)
    assert np.max(np.abs(yr - yb)) < 1e-3 * np.max(np.abs(yb))
    _, its_ref = OP.gmres(A, z, P_ref, tol=1e-8)
    _, its_blk = OP.gmres(A, z, P_blk, tol=1e-8)
    assert abs(its_ref - its_blk) <= 2
    g2 = OF.Geometry(geo.L, geo.shapes, geo.shape_id, geo.q, -geo.theta)  # planted: R^T in place of R
    P_bad, _ = OP.reference_preconditioner(g2, prm)
    Kb = OF.K_matrix(geo)
    # same K (the body's own nodes), wrongly rotated reference block
    y_bad = P_bad(z)
    assert np.max(np.abs(y_bad[:N2] - yb[:N2])) > 1e-1 * np.max(np.abs(yb[:N2]))


def test_cluster_blocks_of_close_bodies_bound_what_a_local_correction_can_gain():
    # the iteration ceiling of any correction local to close bodies: the exact
    # inverse of the saddle block of each cluster of nearly touching bodies (up to
    # four, gaps below four node spacings) in place of the single-body blocks
    wl, geo, M, K, A, N2 = _system(16, 32, 0.4, 5)
    off = geo.offsets()
    n = wl.n_bodies
    h = 2 * math.pi * wl.r_s * (1 + wl.b) / wl.n_p  # largest node spacing
    G = OP.surface_gaps(geo)
    rhs = -np.concatenate([np.zeros(N2), np.random.default_rng(2).standard_normal(3 * n)])
    singles = [[b] for b in range(n)]
    P1 = OP.cluster_preconditioner(M, K, off, singles)
    P0, _ = OP.block_preconditioner(M, K, off)
    z = np.random.default_rng(4).standard_normal(A.shape[0])
    # one-body groups are the block-diagonal preconditioner
    assert np.linalg.norm(P1(z) - P0(z)) < 1e-8 * np.linalg.norm(P0(z))
    _, i0 = OP.gmres(A, rhs, P0, tol=1e-8)
    pairs = OP.close_clusters(G, 4 * h, 2)
    clusters = OP.close_clusters(G, 4 * h, 4)
    assert any(len(g) == 2 for g in pairs) and any(len(g) > 2 for g in clusters)
    _, ip = OP.gmres(A, rhs, OP.cluster_preconditioner(M, K, off, pairs), tol=1e-8)
    _, ic = OP.gmres(A, rhs, OP.cluster_preconditioner(M, K, off, clusters), tol=1e-8)
    # measured 38 -> 34 (pairs) -> 33 (clusters): the near-contact blocks are worth
    # about a tenth of the iterations; the rest is the suspension's long-range coupling
    assert ic <= ip <= i0
    assert ic >= 0.75 * i0
