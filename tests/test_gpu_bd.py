"""Brownian-dynamics validation on the GPU (Section 4.4): short versions of the
bench's validation runs, with statistical bars of four standard errors (the
runs are seeded, so each outcome is reproducible).

  - one four-arm starfish diffusing freely: with the RFD term the angle's
    equilibrium is uniform (<cos 4 theta> = 0); without it the angle follows the
    biased density proportional to 1 / N_theta,theta (Section 4.4.1), and the two
    runs are told apart; the translational MSD follows 4 kT <N_xx> t;
  - the spring-coupled pair (Section 4.4.2) with AB2-RFD and RFD solves at 1e-3:
    the means of theta_1, theta_2 and the distance d match the Gibbs-Boltzmann
    distribution."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def test_single_starfish_equilibrium_with_and_without_rfd():
    import torch

    import bench
    import paper_1709_01480_amd as fb
    import workloads as W
    r = bench.run_bd_starfish(fb, W, np, torch, n_traj=64, steps=500, burn=50, lags=(0.2,), progress=log)
    th = r["theory"]
    log("cos4: rfd %.4f +- %.4f (theory %.4f); no rfd %.4f +- %.4f (theory %.4f)"
        % (r["rfd"]["cos4"], r["rfd"]["cos4_se"], th["rfd"]["cos4"], r["no_rfd"]["cos4"], r["no_rfd"]["cos4_se"],
           th["no_rfd"]["cos4"]))
    for lab in ("rfd", "no_rfd"):
        assert abs(r[lab]["cos4"] - th[lab]["cos4"]) < 4 * r[lab]["cos4_se"], lab
        m = r[lab]["msd"]["0.2"]
        log("MSD(0.2) %s: %.4e +- %.1e, Einstein %.4e" % (lab, m["msd"], m["se"], m["einstein"]))
        assert abs(m["msd"] - m["einstein"]) < 4 * m["se"], lab
    # without the drift the uniform equilibrium is rejected
    assert r["no_rfd"]["cos4"] > 3 * r["no_rfd"]["cos4_se"]
    # the biased density itself: 1 / N_theta,theta varies by a factor ~1.8 over the period
    assert max(th["no_rfd"]["hist"]) / min(th["no_rfd"]["hist"]) > 1.4


def test_spring_pair_equilibrium_means_ab2():
    import torch

    import bench
    import paper_1709_01480_amd as fb
    import workloads as W
    r = bench.run_bd_pair(fb, W, np, torch, scheme="ab2", n_traj=16, T=6.0, dt=0.0149, tol_rfd=1e-3, progress=log)
    log("pair means %s +- %s, theory %s" % (r["mean"], r["mean_se"], r["theory"]["mean"]))
    for k in range(3):
        assert abs(r["mean"][k] - r["theory"]["mean"][k]) < 4 * r["mean_se"][k] + 1e-12, k
