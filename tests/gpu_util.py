"""Shared helpers of the GPU parity tests: build a library context and the
matching oracle objects for a workload, and move arrays to and from the GPU."""
import sys

import numpy as np

import workloads as W
from oracle import fbim as OF


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device="cuda")


def oracle_params(wl):
    return OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)


def make_ctx(wl, **over):
    import paper_1709_01480_amd as fb
    prm = wl.params()
    prm.update(over)
    ctx = fb.Context(**prm)
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    return ctx


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def workload(name, **kw):
    return W.make(name, **kw)
