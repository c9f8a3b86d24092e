"""Write the FP64 oracle's EM-RFD displacement for the 100-starfish suspension
(100 bodies x 128 nodes, area fraction 0.2, grid 256^2, Ewald tolerance 1e-8)
to tests/golden/starfish100_em_rfd.txt.

Calls only oracle/ (the matrix-free step of eq. 4.3: direct real-space sum,
per-body Alpert blocks, spectral-Ewald wave part, GMRES and Lanczos to 1e-11)
and the seeded input generators of workloads/.  Run from the repository root:

    python tests/golden/make_starfish100_step.py

It takes a few minutes on 8 cores.
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fbim as OF  # noqa: E402
from oracle import matfree as MF  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "starfish100_em_rfd.txt")
TOL = 1e-11
DELTA_OVER_A = 1e-2


def input_digest(wl, noise):
    """SHA-256 of the step's inputs (configuration, forces, noise), so a reader can
    check that regenerated inputs are the ones this file was computed from."""
    h = hashlib.sha256()
    for a in (wl.q, wl.theta, wl.F) + tuple(noise):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def main():
    wl = W.make("starfish100")
    prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
    noise = W.noise(wl, prm["grid_M"])
    geo = OF.geometry_from_workload(wl)
    delta = wl.a * DELTA_OVER_A
    t0 = time.time()
    dQ, U0, Up, Um, info = MF.em_rfd_step(geo, prm, wl.F, *noise, wl.kT, wl.dt, delta, order=wl.alpert_order,
                                          tau=wl.tau_spurious, tol=TOL)
    el = time.time() - t0
    with open(OUT, "w") as f:
        f.write("# EM-RFD displacement (eq. 4.3) of the FP64 matrix-free oracle, written by\n")
        f.write("# tests/golden/make_starfish100_step.py (calls only oracle/ and workloads/).\n")
        f.write("# workload starfish100: %d bodies x %d nodes, L = %.16g, grid %d, P %d, xi %.16g, r_c %.16g\n"
                % (wl.n_bodies, wl.n_p, wl.L, prm["grid_M"], prm["P"], prm["xi"], prm["r_c"]))
        f.write("# kT %.16g dt %.16g delta %.16g (a x %g), alpert order %d, tau %.3g, solver tol %.1e\n"
                % (wl.kT, wl.dt, delta, DELTA_OVER_A, wl.alpert_order, wl.tau_spurious, TOL))
        f.write("# inputs sha256 %s\n" % input_digest(wl, noise))
        f.write("# GMRES iterations %d (+ RFD %d, %d), Lanczos %d, relres %.2e; %.0f s\n"
                % (info["gmres_iters"], info["gmres_iters_rfd"][0], info["gmres_iters_rfd"][1],
                   info["lanczos_iters"], max(info["relres"], *info["relres_rfd"]), el))
        f.write("# columns: body  dQ_x  dQ_y  dQ_theta  U0_x  U0_y  U0_theta\n")
        for b in range(wl.n_bodies):
            f.write("%d %s %s\n" % (b, " ".join("%.17e" % v for v in dQ[3 * b:3 * b + 3]),
                                    " ".join("%.17e" % v for v in U0[3 * b:3 * b + 3])))
    print("wrote %s (%.0f s)" % (OUT, el))


if __name__ == "__main__":
    main()
