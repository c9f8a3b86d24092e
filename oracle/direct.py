"""ctypes front end of the oracle's direct C sums (test infrastructure only).

build() compiles oracle/direct.c with gcc into oracle/_direct.so; the
sums themselves are documented in direct.c.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import fbim as F

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_direct.so")


def build():
    src = os.path.join(HERE, "direct.c")
    tmp = SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, SO)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        _lib = ctypes.CDLL(SO)
        d, i = ctypes.c_double, ctypes.c_int
        p = ctypes.c_void_p
        _lib.oracle_e1.restype = d
        _lib.oracle_e1.argtypes = [d]
        _lib.oracle_real_space.argtypes = [i, p, p, d, d, d, d, i, p, p]
        _lib.oracle_wave_space.argtypes = [i, p, p, i, p, p, i, p, p]
        _lib.oracle_real_space_cells.restype = i
        _lib.oracle_real_space_cells.argtypes = [i, p, p, d, d, d, d, p]
        _lib.oracle_spread.argtypes = [i, p, p, d, d, i, i, d, d, p]
        _lib.oracle_interp.argtypes = [i, p, p, d, d, i, i, d, d, p]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def real_space(X, mu, L, xi, r_c, targets=None, eta=1.0):
    X = np.ascontiguousarray(X, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    N = len(X)
    tg = np.arange(N, dtype=np.int32) if targets is None else np.ascontiguousarray(targets, dtype=np.int32)
    out = np.zeros(2 * len(tg))
    lib().oracle_real_space(N, _ptr(X), _ptr(mu), L, xi, eta, r_c, len(tg), _ptr(tg), _ptr(out))
    return out


def wave_space(X, mu, L, xi, targets=None, eta=1.0):
    X = np.ascontiguousarray(X, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    kv, k2 = F.wave_vectors(L, xi)
    B = np.ascontiguousarray(F.wave_multiplier(kv, k2, xi, L, eta))
    kv = np.ascontiguousarray(kv)
    N = len(X)
    tg = np.arange(N, dtype=np.int32) if targets is None else np.ascontiguousarray(targets, dtype=np.int32)
    out = np.zeros(2 * len(tg))
    lib().oracle_wave_space(N, _ptr(X), _ptr(mu), len(kv), _ptr(kv), _ptr(B), len(tg), _ptr(tg), _ptr(out))
    return out


def real_space_cells(X, mu, L, xi, r_c, eta=1.0):
    """M^(t) mu over the 3 x 3 cells around each target (cells of side >= r_c);
    the direct sum where the box holds fewer than 3 cells per side."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    out = np.zeros(2 * len(X))
    if lib().oracle_real_space_cells(len(X), _ptr(X), _ptr(mu), L, xi, eta, r_c, _ptr(out)) != 0:
        return real_space(X, mu, L, xi, r_c, eta=eta)
    return out


def spread(X, mu, L, h, M, P, c, a):
    """H[2, M, M] = sum_n c e^{-a |x_g - x_n|^2} mu_n over the P x P stencils."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    if P > 32:
        raise ValueError("P > 32")
    H = np.zeros((2, M, M))
    lib().oracle_spread(len(X), _ptr(X), _ptr(mu), L, h, M, P, c, a, _ptr(H))
    return H


def interp(X, U, L, h, M, P, c, a):
    """v_n = sum_g c e^{-a |x_n - x_g|^2} U(x_g) (without the h^2 factor)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    if P > 32:
        raise ValueError("P > 32")
    out = np.zeros(2 * len(X))
    lib().oracle_interp(len(X), _ptr(X), _ptr(U), L, h, M, P, c, a, _ptr(out))
    return out
