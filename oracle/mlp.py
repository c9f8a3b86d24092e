"""FP64 reference of the learned preconditioner correction (TEST INFRASTRUCTURE).

The method's block-diagonal preconditioner (Section 3.4, eqs. 3.31-3.37) uses
each body's isolated mobility N_ref.  The learned form adds a per-body
symmetric correction dN predicted by a small network from the body's
neighbourhood; this module restates, in plain numpy, the definitions that the
library's GPU path must reproduce:

  features(q, theta, L, r_max, sym)  -- neighbourhood descriptor per body
  forward / backward                 -- 32 -> 128 -> 128 -> 6 tanh MLP
  loss_and_grad                      -- regression of (N_ref + dN) F_b on U_b

The training target: with forces F of independent standard-normal components
and U = N F from the mobility solve (eq. 3.9), E[U_b F_b^T] = N_bb, so the
least-squares loss is minimised by dN_b = N_bb - N_ref in expectation.

Pins (tests/test_oracle_mlp.py): central finite differences of forward /
loss for every gradient, translation and rotation invariance of the features
and a hand-checked three-body arrangement.  Whether the correction reduces
GMRES iterations is an empirical matter: parity unpinned (judged by GMRES's
true residual and the measured iteration counts).
"""
import numpy as np

N_IN, N_HID, N_OUT = 32, 128, 6
K_NB = 6
SIZES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    """Flat weight vector -> dict of arrays (row-major, input x output)."""
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(w[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def features(q, theta, L, r_max, sym):
    """Per body: up to K_NB nearest other bodies within R = 3 r_max (minimum
    image, ties by index); for slot k (zeros if empty) the neighbour offset
    rotated into the body frame over R, r_max / distance, cos and sin of
    sym (theta_c - theta_b); then count / K_NB and the clamped gap estimate
    (d_min - 2 r_max) / r_max (d_min = R when there is no neighbour)."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 2)
    theta = np.asarray(theta, dtype=np.float64)
    n = len(theta)
    R = 3.0 * r_max
    X = np.zeros((n, N_IN))
    for b in range(n):
        d = q - q[b]
        d -= L * np.round(d / L)
        dist = np.hypot(d[:, 0], d[:, 1])
        cand = [(dist[c], c) for c in range(n) if c != b and dist[c] < R]
        cand.sort()
        c_, s_ = np.cos(theta[b]), np.sin(theta[b])
        for k, (dk, c) in enumerate(cand[:K_NB]):
            ux = c_ * d[c, 0] + s_ * d[c, 1]
            uy = -s_ * d[c, 0] + c_ * d[c, 1]
            X[b, 5 * k:5 * k + 5] = [ux / R, uy / R, r_max / dk, np.cos(sym * (theta[c] - theta[b])),
                                     np.sin(sym * (theta[c] - theta[b]))]
        X[b, 30] = len(cand) / K_NB
        dmin = cand[0][0] if cand else R
        X[b, 31] = min(2.0, max(-2.0, (dmin - 2.0 * r_max) / r_max))
    return X


def forward(w, X):
    p = unpack(w)
    H1 = np.tanh(X @ p["W1"] + p["b1"])
    H2 = np.tanh(H1 @ p["W2"] + p["b2"])
    Y = H2 @ p["W3"] + p["b3"]
    return Y, (X, H1, H2)


def backward(w, X, dY):
    """Gradient of sum(dY * Y) with respect to the flat weights."""
    p = unpack(w)
    _, (X, H1, H2) = forward(w, X)
    g = {}
    g["W3"] = H2.T @ dY
    g["b3"] = dY.sum(0)
    dZ2 = (dY @ p["W3"].T) * (1.0 - H2 ** 2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ p["W2"].T) * (1.0 - H1 ** 2)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(0)
    return pack(g)


def correction(Y, Nref):
    """Symmetric body-frame dN per body from the network output Y[n, 6] and
    the reference mobilities Nref[n, 3, 3]."""
    n = len(Y)
    sx, sy, st = Nref[:, 0, 0], Nref[:, 1, 1], Nref[:, 2, 2]
    D = np.zeros((n, 3, 3))
    D[:, 0, 0] = Y[:, 0] * sx
    D[:, 1, 1] = Y[:, 1] * sy
    D[:, 2, 2] = Y[:, 2] * st
    D[:, 0, 1] = D[:, 1, 0] = Y[:, 3] * np.sqrt(sx * sy)
    D[:, 0, 2] = D[:, 2, 0] = Y[:, 4] * np.sqrt(sx * st)
    D[:, 1, 2] = D[:, 2, 1] = Y[:, 5] * np.sqrt(sy * st)
    return D


def body_frame(V, theta):
    """Rotate the translational part of body vectors V[..., n, 3] by R(theta)^T."""
    V = np.asarray(V, dtype=np.float64)
    c, s = np.cos(theta), np.sin(theta)
    out = V.copy()
    out[..., 0] = c * V[..., 0] + s * V[..., 1]
    out[..., 1] = -s * V[..., 0] + c * V[..., 1]
    return out


def loss(Y, Nref, theta, F, U):
    """Mean over samples s and bodies b of sum_i (r_i / Nref_ii)^2 with
    r = (Nref + dN(Y_b)) R^T F_sb - R^T U_sb.  F, U: [ns, n, 3] (lab frame)."""
    Nb = Nref + correction(Y, Nref)
    Ft, Ut = body_frame(F, theta), body_frame(U, theta)
    r = np.einsum("bij,sbj->sbi", Nb, Ft) - Ut
    wgt = 1.0 / np.stack([Nref[:, 0, 0], Nref[:, 1, 1], Nref[:, 2, 2]], axis=1) ** 2
    return float(np.mean(np.sum(wgt[None] * r * r, axis=2)))


def loss_grad(Y, Nref, theta, F, U):
    """d loss / d Y [n, 6]."""
    ns, n = F.shape[0], F.shape[1]
    Nb = Nref + correction(Y, Nref)
    Ft, Ut = body_frame(F, theta), body_frame(U, theta)
    r = np.einsum("bij,sbj->sbi", Nb, Ft) - Ut
    wgt = 1.0 / np.stack([Nref[:, 0, 0], Nref[:, 1, 1], Nref[:, 2, 2]], axis=1) ** 2
    G = np.einsum("sbi,sbj->bij", 2.0 * wgt[None] * r, Ft) / (ns * n)  # d loss / d N_b
    sx, sy, st = Nref[:, 0, 0], Nref[:, 1, 1], Nref[:, 2, 2]
    dY = np.zeros((n, 6))
    dY[:, 0] = G[:, 0, 0] * sx
    dY[:, 1] = G[:, 1, 1] * sy
    dY[:, 2] = G[:, 2, 2] * st
    dY[:, 3] = (G[:, 0, 1] + G[:, 1, 0]) * np.sqrt(sx * sy)
    dY[:, 4] = (G[:, 0, 2] + G[:, 2, 0]) * np.sqrt(sx * st)
    dY[:, 5] = (G[:, 1, 2] + G[:, 2, 1]) * np.sqrt(sy * st)
    return dY
