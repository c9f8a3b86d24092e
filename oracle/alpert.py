"""Alpert hybrid Gauss-trapezoid end corrections for a log singularity
(oracle; test infrastructure only).

Section 3.1 discretises the single-layer operator with the periodic
trapezoid rule plus Alpert's correction for the logarithmic singularity of
the Stokeslet; Section 4.1 uses rules of 4th and 8th order.  The paper does
not print nodes or weights, so they are derived here from the defining
moment conditions.  With unit spacing, a one-sided rule that drops the
trapezoid points 0 < i < a and adds j nodes chi_k with weights w_k must
integrate x^p and x^p ln x (p < j) exactly near the end point; with the
zeta-regularised value of the discarded trapezoid sums this reads

  sum_k w_k chi_k^p        = -zeta(-p)  + sum_{0<i<a} i^p
  sum_k w_k chi_k^p ln chi_k =  zeta'(-p) + sum_{0<i<a} i^p ln i

The (j, a) pairs are (3, 2) for order 4 and (7, 5) for order 8; both have
positive weights and nodes inside (0, a).  The system is solved with
mpmath at 40 digits from fixed seeded starts.

The density at the auxiliary parameters s_t +- chi_k ds is obtained by
Lagrange interpolation from the ell = order trapezoid nodes centred on the
auxiliary point (reading of Section 3.2, which only says "local Lagrangian
interpolation").
"""
import functools

import mpmath as mp
import numpy as np

RULES = {4: (3, 2), 8: (7, 5)}


@functools.lru_cache(maxsize=None)
def alpert_rule(order):
    """Return (chi, w, a) for the log-singular end correction of given order."""
    j, a = RULES[order]
    with mp.workdps(40):
        r1 = [-mp.zeta(-p) + sum(mp.mpf(i) ** p for i in range(1, a)) for p in range(j)]
        r2 = [mp.zeta(-p, derivative=1) + sum(mp.mpf(i) ** p * mp.log(i) for i in range(1, a))
              for p in range(j)]

        def F(*v):
            chi = [mp.exp(v[k]) for k in range(j)]
            w = v[j:]
            eqs = [sum(w[k] * chi[k] ** p for k in range(j)) - r1[p] for p in range(j)]
            eqs += [sum(w[k] * chi[k] ** p * mp.log(chi[k]) for k in range(j)) - r2[p]
                    for p in range(j)]
            return eqs

        # starting points: nodes clustered quadratically towards the end point,
        # weights equal to the local node spacing; then seeded perturbations
        # (the last a-1 nodes sit near the dropped integers 1..a-1, the
        # remaining ones cluster geometrically towards 0)
        n_small = j - (a - 1)
        base = np.concatenate([0.4 * 0.2 ** np.arange(n_small - 1, -1, -1.0),
                               np.arange(1.0, a)])
        rng = np.random.default_rng(12345)
        for attempt in range(200):
            x0 = base if attempt == 0 else np.sort(base * np.exp(rng.normal(0.0, 0.3, j)))
            w0 = np.gradient(x0) if attempt == 0 else rng.uniform(0.1, 1.0, j)
            w0 = np.minimum(w0, 1.0)
            try:
                v = mp.findroot(F, [mp.log(x) for x in x0] + list(w0), tol=1e-32, maxsteps=100)
            except Exception:  # singular Jacobian or no convergence from this start
                continue
            chi = np.array([float(mp.exp(v[k])) for k in range(j)])
            w = np.array([float(v[j + k]) for k in range(j)])
            if np.all(w > 0) and np.all(chi > 0) and np.all(chi < a):
                o = np.argsort(chi)
                return chi[o], w[o], a
    raise RuntimeError("no admissible Alpert rule found")


def lagrange_stencil(x, ell):
    """Offsets (ell consecutive integers centred on x) and Lagrange weights
    interpolating a function known at integer points to the point x."""
    i0 = int(np.floor(x)) - ell // 2 + 1
    nodes = np.arange(i0, i0 + ell)
    wts = np.ones(ell)
    for m in range(ell):
        for q in range(ell):
            if q != m:
                wts[m] *= (x - nodes[q]) / (nodes[m] - nodes[q])
    return nodes, wts


def periodic_log_quadrature(f_at, n, order, t=0):
    """Apply the corrected periodic trapezoid rule on [0, 2 pi) with n nodes to an
    integrand f(s) with a log singularity at s_t = t*ds.  f_at(s) evaluates the
    integrand anywhere (the auxiliary nodes use exact values)."""
    chi, w, a = alpert_rule(order)
    ds = 2 * np.pi / n
    st = t * ds
    total = 0.0
    for i in range(a, n - a + 1):
        total += f_at(st + i * ds)
    for k in range(len(chi)):
        total += w[k] * (f_at(st + chi[k] * ds) + f_at(st - chi[k] * ds))
    return total * ds


def periodic_log_quadrature_interp(kernel_at, density, n, order, t=0):
    """Same rule, but the smooth density is only known at the trapezoid nodes and
    is Lagrange-interpolated to the auxiliary nodes; kernel_at(s) is evaluated
    exactly.  This is the form used to build the single-layer correction."""
    chi, w, a = alpert_rule(order)
    ds = 2 * np.pi / n
    st = t * ds
    total = 0.0
    for i in range(a, n - a + 1):
        total += kernel_at(st + i * ds) * density[(t + i) % n]
    for k in range(len(chi)):
        for sgn in (1.0, -1.0):
            offs, lw = lagrange_stencil(sgn * chi[k], order)
            dens = sum(lw[m] * density[(t + offs[m]) % n] for m in range(len(offs)))
            total += w[k] * kernel_at(st + sgn * chi[k] * ds) * dens
    return total * ds
