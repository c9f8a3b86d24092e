"""FP64 reference of the block-diagonal preconditioner of the saddle system
(Section 3.4, eqs. 3.31-3.37) and of its corrected form, with a plain
right-preconditioned GMRES (TEST INFRASTRUCTURE).

Block inverse per body b for the system [M -K; -K^T 0][mu; U] = [a; c]:
  g = c_b + K_b^T M_bb^+ a_b,  U_b = -N_b g,  mu_b = M_bb^+ (a_b + K_b U_b),
  N_b = (K_b^T M_bb^+ K_b)^-1  (= N_ref of the body).
Corrected form: the exact inverse of the block with M_bb replaced by
M_bb + K_b C K_b^T for a symmetric 3 x 3 C; by the Woodbury identity the
body's mobility becomes N_b + C, mu_b is unchanged and U_b gains -C c_b.

Two forms of the blocks: block_preconditioner takes M_bb, the body's own
diagonal block of the dense M; reference_preconditioner follows the paper's
construction, M_bb^+ ~ R_b M_ref^+ R_b^T with M_ref the self block of the
shape in its reference configuration (theta = 0) in the same periodic box
(Section 3.4, the equation after eq. 3.37).  The two differ because the
periodic lattice of images is not rotation invariant.
"""
import math

import numpy as np

from . import fbim as F


def pinv_sym(A, tau=1e-8):
    lam, V = np.linalg.eigh(0.5 * (A + A.T))
    keep = np.abs(lam) > tau * np.max(np.abs(lam))
    return (V[:, keep] / lam[keep]) @ V[:, keep].T


def block_preconditioner(M, K, offsets, C=None, tau=1e-8):
    """Returns z -> P^-1 z for the saddle vector z = [a (2N); c (3n)].
    offsets: node offsets per body (n + 1); C: optional [n, 3, 3] corrections."""
    n = len(offsets) - 1
    N2 = 2 * offsets[-1]
    blocks = []
    for b in range(n):
        sl = slice(2 * offsets[b], 2 * offsets[b + 1])
        Mp = pinv_sym(M[sl, sl], tau)
        Kb = K[sl, 3 * b:3 * b + 3]
        blocks.append((sl, Mp, Kb, np.linalg.inv(Kb.T @ Mp @ Kb)))

    def apply(z):
        a, c = z[:N2], z[N2:]
        mu, U = np.zeros(N2), np.zeros(3 * n)
        for b, (sl, Mp, Kb, Nb) in enumerate(blocks):
            cb = c[3 * b:3 * b + 3]
            u = -Nb @ (cb + Kb.T @ (Mp @ a[sl]))
            mu[sl] = Mp @ (a[sl] + Kb @ u)
            if C is not None:
                u = u - C[b] @ cb
            U[3 * b:3 * b + 3] = u
        return np.concatenate([mu, U])

    return apply, [bl[3] for bl in blocks]


def gmres(A, rhs, Pinv, tol=1e-8, maxit=500):
    """Right-preconditioned GMRES (x0 = 0, no restart, CGS2 Arnoldi); returns
    (x, iterations) with ||rhs - A x|| <= tol ||rhs||."""
    n = len(rhs)
    nb = np.linalg.norm(rhs)
    V = np.zeros((n, maxit + 1))
    Z = np.zeros((n, maxit))
    H = np.zeros((maxit + 1, maxit))
    V[:, 0] = rhs / nb
    for j in range(maxit):
        Z[:, j] = Pinv(V[:, j])
        w = A @ Z[:, j]
        for _ in range(2):
            h = V[:, :j + 1].T @ w
            w -= V[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0:
            V[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(j + 2)
        e1[0] = nb
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
        if np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y) <= tol * nb or H[j + 1, j] == 0:
            return Z[:, :j + 1] @ y, j + 1
    return Z @ y, maxit


def reference_preconditioner(geo, prm, order=4, C=None, tau=1e-8, eta=1.0):
    """z -> P^-1 z with every body block built from the reference configuration:
    M_bb^+ = R_b M_ref^+ R_b^T, K_b from the body's own nodes (single shape).
    C: optional [n, 3, 3] lab-frame corrections as in block_preconditioner.
    Returns (apply, [N_b])."""
    sh = geo.shapes[0]
    ref = F.reference_geometry(sh, geo.L)
    Mref = F.single_layer(ref, prm, order, eta)["M"]
    Mref_p = pinv_sym(Mref, tau)
    K = F.K_matrix(geo)
    off = geo.offsets()
    n = geo.n
    N2 = 2 * off[-1]
    blocks = []
    for b in range(n):
        sl = slice(2 * off[b], 2 * off[b + 1])
        c, s = math.cos(geo.theta[b]), math.sin(geo.theta[b])
        Rb = np.kron(np.eye(off[b + 1] - off[b]), np.array([[c, -s], [s, c]]))
        Mp = Rb @ Mref_p @ Rb.T
        Kb = K[sl, 3 * b:3 * b + 3]
        blocks.append((sl, Mp, Kb, np.linalg.inv(Kb.T @ Mp @ Kb)))

    def apply(z):
        a, cz = z[:N2], z[N2:]
        mu, U = np.zeros(N2), np.zeros(3 * n)
        for b, (sl, Mp, Kb, Nb) in enumerate(blocks):
            cb = cz[3 * b:3 * b + 3]
            u = -Nb @ (cb + Kb.T @ (Mp @ a[sl]))
            mu[sl] = Mp @ (a[sl] + Kb @ u)
            if C is not None:
                u = u - C[b] @ cb
            U[3 * b:3 * b + 3] = u
        return np.concatenate([mu, U])

    return apply, [bl[3] for bl in blocks]


def surface_gaps(geo):
    """Smallest node-to-node distance (minimum image) between every two bodies."""
    X, body = F.nodes(geo)
    n, L = geo.n, geo.L
    G = np.full((n, n), np.inf)
    for b in range(n):
        for c in range(b + 1, n):
            d = X[body == b][:, None, :] - X[body == c][None, :, :]
            d -= L * np.round(d / L)
            G[b, c] = G[c, b] = np.sqrt((d ** 2).sum(-1)).min()
    return G


def close_clusters(G, threshold, cap):
    """Groups of bodies joined while their gap is below `threshold`, closest pairs
    first, no group larger than `cap` (cap = 2: a matching of the closest pairs)."""
    n = len(G)
    parent = list(range(n))
    size = [1] * n

    def root(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for g, b, c in sorted((G[b, c], b, c) for b in range(n) for c in range(b + 1, n) if G[b, c] < threshold):
        rb, rc = root(b), root(c)
        if rb != rc and size[rb] + size[rc] <= cap:
            parent[rb] = rc
            size[rc] += size[rb]
    groups = {}
    for b in range(n):
        groups.setdefault(root(b), []).append(b)
    return list(groups.values())


def cluster_preconditioner(M, K, offsets, groups):
    """z -> P^-1 z with P the saddle operator restricted to each group of bodies
    (the exact inverse of the group's block [M_gg -K_g; -K_g^T 0]); groups of one
    body give the block-diagonal preconditioner with each body's own block."""
    N2 = 2 * offsets[-1]
    blocks = []
    for g in groups:
        idx = np.concatenate([np.arange(2 * offsets[b], 2 * offsets[b + 1]) for b in g])
        cidx = np.concatenate([np.arange(3 * b, 3 * b + 3) for b in g])
        Kg = K[np.ix_(idx, cidx)]
        Ag = np.block([[M[np.ix_(idx, idx)], -Kg], [-Kg.T, np.zeros((len(cidx), len(cidx)))]])
        blocks.append((idx, cidx, np.linalg.pinv(Ag, rcond=1e-12)))

    def apply(z):
        out = np.zeros_like(z)
        for idx, cidx, Ai in blocks:
            y = Ai @ np.concatenate([z[idx], z[N2 + cidx]])
            out[idx] = y[:len(idx)]
            out[N2 + cidx] = y[len(idx):]
        return out
    return apply
