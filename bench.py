"""Benchmark: Brownian EM-RFD steps/s (and the single-layer matvec) on one MI355X.

Workload: 10,000 five-arm starfish x 64 nodes (640,000 nodes), area fraction
0.3, unit periodic box, grid 2048^2, tol_ewald 1e-6, 4th-order Alpert, GMRES and
Lanczos tolerance 1e-6.  Inputs (geometry, forces, noise) are synthetic and
seeded, and resident in HBM before timing starts.  One step = one
Euler-Maruyama random-finite-difference step (Lanczos square root, random
Fourier field, three GMRES mobility solves, geometry rebuilds).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Stokeslet matvec Mnodes/s + Brownian steps/s @640k nodes; mixed+learned vs FP64"
PEAK = {"hbm": 8000.0, "fp64_vec": 78.6, "fp32_vec": 157.3}  # GB/s, TFLOP/s
FLOP_PER_PAIR = 60.0       # kernel evaluation per in-range pair (E1, exp, 2x2 apply)
FLOP_PER_CANDIDATE = 6.0   # distance test per culled candidate


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def count_pairs(x, L, r_c, nb):
    """In-range pairs (ordered, i != j) and 3x3-cell candidates of the node set,
    for the algorithmic flop count of the real-space kernel."""
    import numpy as np
    from scipy.spatial import cKDTree
    x = np.mod(x.reshape(-1, 2), L)
    tree = cKDTree(x, boxsize=L)
    inrange = int(tree.count_neighbors(tree, r_c)) - len(x)
    cell = np.minimum((x / (L / nb)).astype(np.int64), nb - 1)
    cnt = np.bincount(cell[:, 1] * nb + cell[:, 0], minlength=nb * nb).reshape(nb, nb)
    nbr = sum(np.roll(np.roll(cnt, dy, 0), dx, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    cand = int(np.sum(cnt * nbr))
    return inrange, cand


def cpu_baseline(wl, X_nodes, prm, matvecs_per_step, budget_s=20.0):
    """Time the FP64 oracle on a bounded sample of the same workload and scale to
    steps/s: real-space direct sums for a sample of targets, the Alpert blocks of
    a sample of bodies and one full spectral-Ewald wave-space application."""
    import numpy as np

    from oracle import direct as OD
    from oracle import fbim as OF
    N = len(X_nodes)
    rng = np.random.default_rng(0)
    mu = rng.standard_normal(2 * N)
    geo = OF.geometry_from_workload(wl)
    t0 = time.time()
    ntg = 256
    OD.real_space(X_nodes, mu, wl.L, prm["xi"], prm["r_c"], targets=rng.choice(N, ntg, replace=False))
    t_real = (time.time() - t0) / ntg * N
    t0 = time.time()
    nbod = 20
    for b in range(nbod):
        OF.alpert_body(geo, b, prm["xi"], prm["r_c"], wl.alpert_order)
    t_alp = (time.time() - t0) / nbod * wl.n_bodies
    t0 = time.time()
    OF.wave_se(X_nodes, mu, prm)
    t_wave = time.time() - t0
    t_mv = t_real + t_alp + t_wave
    return {
        "value": 1.0 / (matvecs_per_step * t_mv), "unit": "steps/s", "cores": os.cpu_count(),
        "kind": "oracle",
        "sample": "FP64 oracle on the 640k-node workload: direct real-space sums for %d sampled targets "
                  "(x N/%d), Alpert blocks of %d bodies (x n/%d), one full spectral-Ewald M^(w) mu; "
                  "matvec %.2f s, times %d matvecs per step measured on the GPU run"
                  % (ntg, ntg, nbod, nbod, t_mv, matvecs_per_step),
        "matvec_s": t_mv,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--config", default="starfish10k")
    ap.add_argument("--matvecs", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="step", choices=["step", "matvec", "copy"],
                    help="step: the EM-RFD benchmark; matvec: only single-layer matvecs "
                         "(short runs for counter collection); copy: a plain 1 GiB device copy "
                         "used to calibrate the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_01480_amd as fb
    import workloads as W

    torch.cuda.set_device(0)
    if args.mode == "copy":
        n = (1 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "copies": args.steps}))
        return
    wl = W.make(args.config)
    prec = fb.PREC_FP64 if args.precision == "fp64" else fb.PREC_MIXED
    log("workload %s: %d bodies x %d nodes" % (args.config, wl.n_bodies, wl.n_p))
    ctx = fb.Context(**wl.params(), precision=prec)
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    d = ctx.get_derived()
    M = d["grid_M"]
    N = d["n_nodes"]
    log("derived: %s" % d)
    W_r, W_grid, W_t = W.noise(wl, M)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    F, Wr, Wg, Wt = dev(wl.F), dev(W_r), dev(W_grid), dev(W_t)
    dQ = torch.zeros(3 * wl.n_bodies, dtype=torch.float64, device="cuda")
    delta = wl.a * wl.tol_gmres ** (1.0 / 3.0)

    # ---- matvec throughput
    mu = dev(np.random.default_rng(1).standard_normal(2 * N))
    out = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    for _ in range(3):
        ctx.apply_M(mu, out, fb.PART_ALL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.matvecs):
        ctx.apply_M(mu, out, fb.PART_ALL)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / args.matvecs
    log("matvec: %.3f ms (%.1f Mnodes/s)" % (1e3 * t_mv, N / t_mv / 1e6))
    if args.mode == "matvec":
        print(json.dumps({"mode": "matvec", "nodes": N, "ms": 1e3 * t_mv, "Mnodes/s": N / t_mv / 1e6}))
        ctx.close()
        return

    # ---- EM-RFD steps
    for i in range(args.warmup):
        info = ctx.step_em_rfd(wl.dt, delta, F, Wr, Wg, Wt, dQ)
        log("warmup step %d: %s" % (i, info))
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(ctx.step_em_rfd(wl.dt, delta, F, Wr, Wg, Wt, dQ))
        log("step %d: %s" % (i, infos[-1]))
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    kt = {k: ctx.kernel_time(k) for k in ("pair", "alpert", "spread", "interp", "fft", "multiplier",
                                          "precond", "blas")}
    ctx.set_timing(False)
    matvecs = (sum(i["gmres_iters"] + i["gmres_solves"] + 1 for i in infos) + sum(i["lanczos_iters"] for i in infos))
    matvecs_per_step = matvecs / args.steps
    log("kernel ms per step: %s" % {k: round(v[0] / args.steps, 3) for k, v in kt.items()})

    # ---- roofline of the dominant kernel
    dom = max(kt, key=lambda k: kt[k][0])
    ms, cnt = kt[dom]
    avg_s = ms / max(cnt, 1) / 1e3
    x = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    ctx.get_nodes(x)
    xh = x.cpu().numpy()
    roof = None
    if dom == "pair":
        npair, ncand = count_pairs(xh, wl.L, d["r_c"], d["n_box"])
        flops = FLOP_PER_PAIR * npair + FLOP_PER_CANDIDATE * ncand
        peak = PEAK["fp64_vec"] if prec == fb.PREC_FP64 else PEAK["fp32_vec"]
        ach = flops / avg_s / 1e12
        roof = {"kernel": "pair", "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": None, "avg_launch_ms": avg_s * 1e3,
                "pairs": npair, "candidates": ncand}
    else:
        wb = 8 if prec == fb.PREC_FP64 else 4
        grid_bytes = 2 * M * M * wb
        per = {"spread": 2 * N * 2 * wb + 2 * N * 4 + grid_bytes,     # positions, mu, anchors in; grid out
               "interp": grid_bytes + 2 * N * 2 * wb + 2 * N * 4 + 2 * N * 8 * 2,
               "fft": 2 * grid_bytes + 2 * grid_bytes,
               "multiplier": 2 * 2 * M * (M // 2 + 1) * 2 * wb,
               "precond": 4 * (2 * N + 3 * wl.n_bodies) * 8,
               "blas": 2 * (2 * N + 3 * wl.n_bodies) * 8,
               "alpert": 2 * N * 8 * 3}
        b = per.get(dom, 0)
        ach = b / avg_s / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s",
                "frac": ach / PEAK["hbm"], "traffic": None, "avg_launch_ms": avg_s * 1e3}

    res = {
        "metric": METRIC, "value": 1.0 / t_step, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == fb.PREC_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "%s: %d five-arm starfish x %d nodes (%d nodes), area fraction 0.3, grid %d^2, "
                               "tol 1e-6, EM-RFD step (Lanczos + random field + 3 GMRES solves)"
                               % (args.config, wl.n_bodies, wl.n_p, N, M),
                   "precision": args.precision, "gmres_tol": wl.tol_gmres, "lanczos_tol": wl.tol_lanczos},
        "matvec": {"value": N / t_mv / 1e6, "unit": "Mnodes/s", "ms": 1e3 * t_mv},
        "solver": {"gmres_iters_per_solve": sum(i["gmres_iters"] for i in infos) / max(1, sum(i["gmres_solves"] for i in infos)),
                   "lanczos_iters": sum(i["lanczos_iters"] for i in infos) / args.steps,
                   "matvecs_per_step": matvecs_per_step},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import fbim as OF
        prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
        geo = OF.geometry_from_workload(wl)
        Xn, _ = OF.nodes(geo)
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(wl, Xn, prm, matvecs_per_step)
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
