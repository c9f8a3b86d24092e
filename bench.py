"""Benchmark: Brownian EM-RFD steps/s (and the single-layer matvec) on one MI355X.

Workload: 10,000 five-arm starfish x 64 nodes (640,000 nodes), area fraction
0.3, unit periodic box, grid 2048^2, tol_ewald 1e-6, 4th-order Alpert, GMRES and
Lanczos tolerance 1e-6.  Inputs (geometry, forces, noise) are synthetic and
seeded, and resident in HBM before timing starts.  One step = one
Brownian-dynamics step: Euler-Maruyama with the random finite difference
(fresh noise drawn by the library, Lanczos square root, random Fourier field,
three GMRES mobility solves, geometry of the two RFD configurations) and the
move of the bodies to Q + dQ (geometry rebuild, learned-correction refresh).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp64,mixed+batched+learned]

Two forms are timed on the same inputs: the plain FP64 method and the
mixed-precision form with batched EM-RFD solves and the learned preconditioner
correction (trained, untimed, on other seeded configurations of the workload).
`value` is the second form's steps/s; both forms are reported under "forms".
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# autotuner cache (JSON lines); the first run on a device times the candidates
TUNE_CACHE = os.environ.get("FBIM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fbim",
                                                            "tune_cache.jsonl"))
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


def cpu_baseline(wl, prm, gmres_mv, lanczos_mv, reps=3):
    """Time the FP64 CPU fast path of the oracle (cell-list real space, shared
    Alpert block, spectral Ewald with C gridding and multi-threaded FFTs) on the
    full workload: the configuration set-up once, M mu (median of `reps`) and
    M^(r) mu (median of 2), then scale to steps/s with the matvec counts of one
    GPU step (`gmres_mv` full matvecs, `lanczos_mv` real-space matvecs)."""
    import numpy as np

    from oracle import fastpath as FP
    from oracle import fbim as OF
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    geo = OF.geometry_from_workload(wl)
    t0 = time.perf_counter()
    f = FP.FastFBIM(geo, prm, wl.alpert_order)
    t_setup = time.perf_counter() - t0
    mu = np.random.default_rng(0).standard_normal(2 * geo.N)

    def med(fn, k):
        ts = []
        for _ in range(k):
            t = time.perf_counter()
            fn(mu)
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))
    t_M = med(f.apply_M, reps)
    t_Mr = med(f.apply_Mr, 2)
    t_step = t_setup + gmres_mv * t_M + lanczos_mv * t_Mr
    return {
        "value": 1.0 / t_step, "unit": "steps/s", "cores": threads, "kind": "oracle",
        "sample": "FP64 CPU fast path of the oracle on the full %d-node workload, %d threads: set-up %.2f s, "
                  "M mu %.2f s (median of %d), M^(r) mu %.2f s (median of 2), measured; steps/s = 1 / (set-up + "
                  "%.1f M mu + %.1f M^(r) mu), the matvec counts of one GPU step"
                  % (geo.N, threads, t_setup, t_M, reps, t_Mr, gmres_mv, lanczos_mv),
        "matvec": {"value": geo.N / t_M / 1e6, "unit": "Mnodes/s", "s": t_M},
        "real_matvec_s": t_Mr, "setup_s": t_setup,
    }


# every form runs GMRES with the second Gram-Schmidt pass of each Arnoldi step delayed
# into the next step's read of the basis (FBIM_FLAG_LAGGED_REORTH)
FORMS = {
    # plain method: FP64 everywhere, block-diagonal preconditioner, solves one after another
    "fp64": dict(precision="fp64", batch_rfd=False, learned=False),
    # mixed precision only (FP32 matvecs in FP64 Krylov), solves one after another
    "mixed": dict(precision="mixed", batch_rfd=False, learned=False),
    # relaxed-matvec GMRES (FP32 operator once the residual is small) with an FP32 Krylov basis and
    # the EM-RFD solves in batched launch sets
    "mixed+batched": dict(precision="mixed", batch_rfd=True, graph=True, learned=False, basis32=True),
    # the same with the learned preconditioner correction, trained beforehand on solves
    "mixed+batched+learned": dict(precision="mixed", batch_rfd=True, graph=True, learned=True, basis32=True),
}


def run_form(name, form, wl, args, fb, W, np, torch):
    prec = fb.PREC_FP64 if form["precision"] == "fp64" else fb.PREC_MIXED
    flags = ((fb.FLAG_BATCH_RFD if form["batch_rfd"] else 0) | (fb.FLAG_GRAPH if form.get("graph") else 0)
             | (fb.FLAG_BASIS32 if form.get("basis32") else 0) | fb.FLAG_LAGGED_REORTH)
    prm = dict(wl.params(), precision=prec, flags=flags, seed=W.noise_key(wl))
    ctx = fb.Context(**prm)
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    # untimed: the spreading tile from the autotuner (the grid is part of the workload)
    tuned, tune_rep = ctx.autotune(fb.TUNE_TILE, TUNE_CACHE)
    if tuned["tile"] != ctx.get_derived()["tile"]:
        ctx.close()
        prm["tile"] = tuned["tile"]
        ctx = fb.Context(**prm)
        sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
        ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    log("%s: spreading tile %d (%s)" % (name, ctx.get_derived()["tile"], tune_rep))
    d = ctx.get_derived()
    M, N = d["grid_M"], d["n_nodes"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    train = None
    if form["learned"]:
        # untimed: train the correction on random-force solves of other configurations of the workload
        ctx.mlp_init(seed=7, sym_order=wl.n_arm)
        t0 = time.perf_counter()
        for k in range(args.train_configs):
            w2 = W.make(args.config, seed=500 + k)
            ctx.set_bodies(np.full(w2.n_bodies, sid), w2.q, w2.theta)
            train = ctx.mlp_train(n_solves=2, epochs=20, lr=2e-3, seed=k)
        ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
        ctx.mlp_use(True)
        log("%s: trained on %d configurations in %.1f s (last: %s)"
            % (name, args.train_configs, time.perf_counter() - t0, train))
    F = dev(wl.F)
    dQ = torch.zeros(3 * wl.n_bodies, dtype=torch.float64, device="cuda")
    delta = wl.a * wl.tol_gmres ** (1.0 / 3.0)
    # matvec throughput
    mu = dev(np.random.default_rng(1).standard_normal(2 * N))
    out = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    for _ in range(3):
        ctx.apply_M(mu, out, fb.PART_ALL)
    ctx.set_timing(True)  # per-kernel events of single-system launches (roofline)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.matvecs):
        ctx.apply_M(mu, out, fb.PART_ALL)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / args.matvecs
    kt_mv = {k: ctx.kernel_time(k) for k in KERNEL_CLASSES}
    log("%s matvec: %.3f ms (%.1f Mnodes/s)" % (name, 1e3 * t_mv, N / t_mv / 1e6))
    # Brownian dynamics: every step draws fresh noise in the library (W_r, W_grid, W~ from
    # the context's generator), solves, and moves the bodies to Q + dQ (geometry rebuild and,
    # with the learned correction, its refresh).  Warm-up steps run the same way, untimed
    # (graphs are captured there).
    ctx.set_timing(False)
    for i in range(args.warmup):
        info = ctx.step_em_rfd(wl.dt, delta, F, None, None, None, dQ, apply=True)
        log("%s warmup step %d: %s" % (name, i, info))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(ctx.step_em_rfd(wl.dt, delta, F, None, None, None, dQ, apply=True))
        log("%s step %d: %s" % (name, i, infos[-1]))
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    dq = dQ.cpu().numpy().reshape(-1, 3)
    rms_move = float(np.sqrt(np.mean(dq[:, :2] ** 2)) / wl.a)
    # one more step with per-kernel events for the breakdown (outside the timed steps;
    # events bracket every launch and keep graphs off)
    ctx.set_timing(True)
    ctx.step_em_rfd(wl.dt, delta, F, None, None, None, dQ, apply=True)
    kt = {k: ctx.kernel_time(k) for k in KERNEL_CLASSES}
    ctx.set_timing(False)
    gmres_mv = sum(i["gmres_iters"] + i["gmres_solves"] + 1 for i in infos)
    lanczos_mv = sum(i["lanczos_iters"] for i in infos)
    matvecs = gmres_mv + lanczos_mv
    log("%s kernel ms per step: %s" % (name, {k: round(v[0], 3) for k, v in kt.items()}))
    x = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    ctx.get_nodes(x)
    res = {
        "steps_per_s": 1.0 / t_step, "ms_per_step": 1e3 * t_step,
        "tuning": dict(tune_rep, tile=d["tile"]),
        "matvec": {"value": N / t_mv / 1e6, "unit": "Mnodes/s", "ms": 1e3 * t_mv},
        "solver": {"gmres_iters_per_solve": sum(i["gmres_iters"] for i in infos)
                   / max(1, sum(i["gmres_solves"] for i in infos)),
                   "gmres_iters_per_step": [i["gmres_iters"] for i in infos],
                   "lanczos_iters_per_step": [i["lanczos_iters"] for i in infos],
                   "rms_displacement_over_a": rms_move,
                   "lanczos_iters": sum(i["lanczos_iters"] for i in infos) / args.steps,
                   "matvecs_per_step": matvecs / args.steps,
                   "full_matvecs_per_step": gmres_mv / args.steps,
                   "real_matvecs_per_step": lanczos_mv / args.steps,
                   "max_residual": max(i["gmres_residual"] for i in infos)},
        "kernel_ms_per_step": {k: v[0] for k, v in kt.items()},
        "dtype": "f64" if prec == fb.PREC_FP64 else "f32+f64",
    }
    if train:
        res["training"] = train
    ctx.close()
    return res, kt_mv, x.cpu().numpy(), d


def kernel_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    the kernel source is unchanged since the counters were taken (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", COUNTER_FILE)
    if not os.path.exists(path) or kernel not in KERNEL_SOURCE:
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch\[%s\]:\s*([0-9.eE+]+)" % re.escape(kernel), txt)
    h = re.search(r"source_sha256\[%s\]:\s*([0-9a-f]+)" % re.escape(KERNEL_SOURCE[kernel]), txt)
    src = os.path.join(ROOT, "paper_1709_01480_amd", "csrc", KERNEL_SOURCE[kernel])
    if not (m and h and os.path.exists(src)):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != h.group(1):
        return None
    return float(m.group(1))


COUNTER_FILE = "matvec_kernels_starfish10k_counters.md"
KERNEL_CLASSES = ("pair", "pair32", "alpert", "spread", "spread32", "interp", "interp32", "fft", "fft32",
                  "multiplier", "multiplier32", "precond", "blas", "mlp")
# classes timed as exactly one kernel (candidates for the roofline line) and their sources
KERNEL_SOURCE = {"pair": "kernels_real.hip", "pair32": "kernels_real.hip", "spread": "kernels_wave.hip",
                 "spread32": "kernels_wave.hip", "interp": "kernels_wave.hip", "interp32": "kernels_wave.hip",
                 "alpert": "kernels_real.hip", "precond": "kernels_la.hip", "multiplier": "kernels_wave.hip",
                 "multiplier32": "kernels_wave.hip"}


def roofline(kt, xh, wl, d):
    """Dominant single kernel of the single-layer matvec (one system per launch,
    HIP events on the context's stream around every launch of the timed matvecs)."""
    N, M = d["n_nodes"], d["grid_M"]
    dom = max(KERNEL_SOURCE, key=lambda k: kt[k][0])
    f32 = dom.endswith("32")
    ms, cnt = kt[dom]
    avg_s = ms / max(cnt, 1) / 1e3
    traffic = kernel_traffic(dom)
    if dom.startswith("pair"):
        npair, ncand = count_pairs(xh, wl.L, d["r_c"], d["n_box"])
        flops = FLOP_PER_PAIR * npair + FLOP_PER_CANDIDATE * ncand
        peak = PEAK["fp32_vec"] if f32 else PEAK["fp64_vec"]
        ach = flops / avg_s / 1e12
        return {"kernel": "%s (k_pair_ell<%s>)" % (dom, "float, 9" if f32 else "double, 16"), "bound": "alu",
                "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic,
                "avg_launch_ms": avg_s * 1e3, "pairs": npair, "candidates": ncand,
                "flop_per_launch": flops}
    wb = 4 if f32 else 8
    grid_bytes = 2 * M * M * wb
    per = {"spread": 2 * N * 2 * wb + 2 * N * 4 + grid_bytes,
           "interp": grid_bytes + 2 * N * 2 * wb + 2 * N * 4 + 2 * N * 8 * 2,
           "multiplier": 2 * 2 * M * (M // 2 + 1) * 2 * wb,
           "precond": 4 * (2 * N + 3 * wl.n_bodies) * 8,
           "alpert": 2 * N * 8 * 3}
    b = per[dom.rstrip("32")]
    ach = b / avg_s / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s",
            "frac": ach / PEAK["hbm"], "traffic": traffic, "avg_launch_ms": avg_s * 1e3, "bytes_per_launch": b}


def run_batch(args, fb, W, np, torch):
    """The uneven-suspension batch: 64 independent suspensions, bodies per
    suspension log-uniform in [16, 512], 64 / 128 / 256 nodes per body, mixed
    precision with the FP32 Krylov basis and the delayed second Gram-Schmidt pass.
    One batched EM-RFD step of all of them
    (three mobility solves per suspension in lockstep launch sets, preconditioner
    and saddle operator replayed from graphs, noise drawn by each member, bodies
    moved) against the same member contexts stepping one after another.  One
    JSON line on stdout."""
    wls = W.uneven_suspensions(64)
    prms = []
    for k, wl in enumerate(wls):
        p = wl.params()
        p.update(precision=fb.PREC_MIXED, flags=fb.FLAG_BASIS32 | fb.FLAG_LAGGED_REORTH, seed=W.noise_key(wl, 100 + k))
        prms.append(p)
    b = fb.Batch(prms, graph=True)
    for m, wl in zip(b.members, wls):
        sid = m.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
        m.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    Fs = [dev(wl.F) for wl in wls]
    dQs = [torch.zeros(3 * wl.n_bodies, dtype=torch.float64, device="cuda") for wl in wls]
    delta = min(wl.a for wl in wls) * 1e-2
    dt = 1e-7  # RMS move ~2% of the smallest bodies' radius per step
    nw = [None] * len(wls)
    for _ in range(max(1, args.warmup)):
        b.step_em_rfd(dt, delta, Fs, nw, nw, nw, dQs, apply=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    binfo = []
    for _ in range(args.steps):
        binfo.append(b.step_em_rfd(dt, delta, Fs, nw, nw, nw, dQs, apply=True))
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / args.steps
    # the members one after another (same contexts, sequential EM-RFD step each)
    for m, F, dQ in zip(b.members, Fs, dQs):
        m.step_em_rfd(dt, delta, F, None, None, None, dQ, apply=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for _ in range(args.steps):
        for m, F, dQ in zip(b.members, Fs, dQs):
            its += m.step_em_rfd(dt, delta, F, None, None, None, dQ, apply=True)["gmres_iters"]
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"mode": "batch", "workload": "64 uneven suspensions, bodies log-uniform in [16, 512], "
                      "64/128/256 nodes per body, area fraction 0.2, tol 1e-6; EM-RFD step, 3 RHS each",
                      "precision": "mixed+basis32+lagged", "suspensions": len(wls), "bodies": sum(w.n_bodies for w in wls),
                      "nodes": sum(w.n_nodes for w in wls), "steps": args.steps,
                      "ms_per_step_batched": 1e3 * t_b, "ms_per_step_one_after_another": 1e3 * t_s,
                      "speedup": t_s / t_b,
                      "gmres_iters_batched": sum(i["gmres_iters"] for st in binfo for i in st) / args.steps,
                      "gmres_iters_one_after_another": its / args.steps,
                      "max_residual": max(i["gmres_residual"] for st in binfo for i in st)}), flush=True)
    b.close()


def _batch_of(fb, wl, count, seed0, **over):
    """`count` independent copies of workload wl as members of one batch (graphs
    on), member k with noise seed seed0 + k."""
    import numpy as np
    prms = []
    for k in range(count):
        p = wl.params()
        p.update(over)
        p["seed"] = seed0 + k
        prms.append(p)
    b = fb.Batch(prms, graph=True)
    for m in b.members:
        sid = m.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
        m.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    return b


def single_starfish_mobility(fb, W, np, thetas):
    """N_xx and N_theta,theta of the single four-arm starfish at each angle
    (FP64 solves to 1e-10 with forces e_x and e_theta)."""
    import torch
    wl = W.single_starfish()
    ctx = fb.Context(**dict(wl.params(), tol_gmres=1e-10))
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    out = []
    U = torch.zeros(3, dtype=torch.float64, device="cuda")
    for th in thetas:
        ctx.set_bodies(np.full(1, sid), wl.q, np.array([th]))
        row = []
        for e in (0, 2):
            F = torch.zeros(3, dtype=torch.float64, device="cuda")
            F[e] = 1.0
            ctx.mobility(F, U)
            row.append(float(U[e]))
        out.append(row)
    ctx.close()
    return np.array(out)


def run_bd_starfish(fb, W, np, torch, n_traj=64, steps=1500, burn=250, dt=0.02, lags=(0.2, 1.0, 2.0),
                    progress=log):
    """Free diffusion of one four-arm starfish (b = 0.3, a = 0.45, 64 nodes,
    tolerance 1e-7) in the unit periodic box, Section 4.4.1: n_traj independent
    trajectories (one batch), EM with the RFD term and EM without it (delta = 0),
    angles uniform at the start.  After `burn` steps: the histogram of theta mod
    pi/2 and <cos 4 theta> against the Gibbs-Boltzmann distribution (uniform) and
    the biased one (proportional to 1 / N_theta,theta), and the translational MSD
    against 4 kT <N_xx> t under each.  Standard errors from the spread over
    trajectories."""
    wl = W.single_starfish()
    delta = wl.a * wl.tol_ewald ** (1.0 / 3.0)
    fine = (np.arange(256) + 0.5) * (0.5 * math.pi / 256)  # midpoints over one period
    Nf = single_starfish_mobility(fb, W, np, fine)
    w_b = 1.0 / Nf[:, 1]
    w_b /= w_b.sum()
    nb = 8
    edges = np.linspace(0, 0.5 * math.pi, nb + 1)
    binof = np.minimum((fine / (0.5 * math.pi) * nb).astype(int), nb - 1)
    theory = {"rfd": {"hist": [1.0 / nb] * nb, "cos4": float(np.mean(np.cos(4 * fine))),
                      "Nxx": float(np.mean(Nf[:, 0]))},
              "no_rfd": {"hist": [float(w_b[binof == k].sum()) for k in range(nb)],
                         "cos4": float(np.sum(w_b * np.cos(4 * fine))), "Nxx": float(np.sum(w_b * Nf[:, 0]))}}
    rng = np.random.default_rng(0x5F5)
    th0 = rng.uniform(0, 2 * math.pi, n_traj)
    out = {"workload": "single four-arm starfish, b 0.3, a 0.45, 64 nodes, unit box, tol 1e-7, kT 1",
           "dt": dt, "delta": delta, "trajectories": n_traj, "steps": steps, "burn_in": burn, "theory": theory}
    for label, dl in (("rfd", delta), ("no_rfd", 0.0)):
        b = _batch_of(fb, wl, n_traj, 1000 if dl else 2000)
        for k, m in enumerate(b.members):
            m.set_bodies(np.zeros(1, dtype=np.int64), wl.q, th0[k:k + 1])
        Q = np.zeros((steps + 1, n_traj, 3))
        Q[0, :, :2] = wl.q[0]
        Q[0, :, 2] = th0
        Fs = [torch.zeros(3, dtype=torch.float64, device="cuda") for _ in range(n_traj)]
        dQs = [torch.zeros(3, dtype=torch.float64, device="cuda") for _ in range(n_traj)]
        nw = [None] * n_traj
        t0 = time.perf_counter()
        for t in range(steps):
            b.step_em_rfd(dt, dl, Fs, nw, nw, nw, dQs, apply=True)
            Q[t + 1] = Q[t] + torch.stack(dQs).cpu().numpy()
            if progress and (t + 1) % 250 == 0:
                progress("bd-starfish %s: step %d / %d (%.1f s)" % (label, t + 1, steps, time.perf_counter() - t0))
        b.close()
        th = np.mod(Q[burn + 1:, :, 2], 0.5 * math.pi)  # [time, traj]
        h = np.stack([np.histogram(th[:, k], bins=edges)[0] / th.shape[0] for k in range(n_traj)])
        c4 = np.cos(4 * th).mean(axis=0)
        msd = {}
        for lag in lags:
            L = int(round(lag / dt))
            if L >= steps - burn:
                continue
            d = Q[burn + 1 + L:, :, :2] - Q[burn + 1:-L, :, :2]
            per = (d ** 2).sum(axis=2).mean(axis=0)  # per trajectory
            msd["%g" % lag] = {"msd": float(per.mean()), "se": float(per.std(ddof=1) / math.sqrt(n_traj)),
                               "einstein": 4 * wl.kT * theory[label]["Nxx"] * lag}
        out[label] = {"hist": h.mean(axis=0).tolist(), "hist_se": (h.std(axis=0, ddof=1) / math.sqrt(n_traj)).tolist(),
                      "cos4": float(c4.mean()), "cos4_se": float(c4.std(ddof=1) / math.sqrt(n_traj)), "msd": msd,
                      "s_per_step": (time.perf_counter() - t0) / steps}
    return out


def run_bd_pair(fb, W, np, torch, scheme="ab2", n_traj=16, T=14.86, dt=0.0149, tol_rfd=1e-3, progress=log):
    """A pair of four-arm starfish (a = l/12, 48 nodes, box l = 2) joined by a
    Hookean spring between the tracking points (rest length 5a, k_s = 81) with
    each angle held by a harmonic potential (k_theta = 2.446, preferred angles
    pi/4 and pi/2), Section 4.4.2: n_traj independent trajectories (one batch),
    EM-RFD or AB2-RFD, deterministic solves at 1e-6 and RFD solves at tol_rfd.
    Mean and covariance of theta_1, theta_2 and d = |q_1 - q_2| against the
    Gibbs-Boltzmann distribution, the separation with density proportional to
    exp(-k_s (d - l_s)^2 / 2 kT) on the periodic cell (d its minimum-image length)."""
    wl = W.starfish_pair()
    a, L = wl.a, wl.L
    ls, ks, kth = 5 * a, 81.0, 2.446
    pref = np.array([0.25 * math.pi, 0.5 * math.pi])
    delta = a * 1e-6 ** (1.0 / 3.0)
    steps = int(round(T / dt))
    b = _batch_of(fb, wl, n_traj, 3000 if scheme == "ab2" else 4000, tol_gmres=1e-6, tol_rfd=tol_rfd)
    Q = np.tile(np.concatenate([wl.q, wl.theta[:, None]], axis=1).ravel(), (n_traj, 1))  # [traj, 6]
    dQs = [torch.zeros(6, dtype=torch.float64, device="cuda") for _ in range(n_traj)]
    hists = [torch.zeros(6, dtype=torch.float64, device="cuda") for _ in range(n_traj)]
    nw = [None] * n_traj

    def forces(Q):
        F = np.zeros_like(Q)
        r = Q[:, 0:2] - Q[:, 3:5]
        r -= L * np.round(r / L)
        d = np.linalg.norm(r, axis=1)
        f = -ks * (d - ls)[:, None] * r / d[:, None]
        F[:, 0:2], F[:, 3:5] = f, -f
        F[:, 2] = -kth * (Q[:, 2] - pref[0])
        F[:, 5] = -kth * (Q[:, 5] - pref[1])
        return F, d
    rec = []
    t0 = time.perf_counter()
    for t in range(steps):
        F, d = forces(Q)
        rec.append(np.stack([Q[:, 2], Q[:, 5], d], axis=1))
        Fs = [torch.as_tensor(F[k]).cuda() for k in range(n_traj)]
        if scheme == "ab2":
            b.step_ab2_rfd(dt, delta, Fs, nw, nw, nw, hists, t > 0, dQs, apply=True)
        else:
            b.step_em_rfd(dt, delta, Fs, nw, nw, nw, dQs, apply=True)
        Q = Q + torch.stack(dQs).cpu().numpy()
        if progress and (t + 1) % 200 == 0:
            progress("bd-pair %s: step %d / %d (%.1f s)" % (scheme, t + 1, steps, time.perf_counter() - t0))
    b.close()
    R = np.array(rec)  # [time, traj, 3]: theta1, theta2, d
    burn = int(round(1.0 / dt))  # ~8 relaxation times
    R = R[burn:]
    # Gibbs-Boltzmann: theta_i ~ N(pref_i, kT/k_theta); the separation q_1 - q_2 lives
    # on the periodic cell with density exp(-k_s (d - l_s)^2 / 2 kT), d its minimum-image
    # length (the ring of radius l_s + 3 sd reaches past l/2, so the planar density
    # d exp(...) would overstate <d> by 0.007): midpoint rule on the cell
    g = (np.arange(4000) + 0.5) * (L / 4000) - 0.5 * L
    dd = np.hypot(*np.meshgrid(g, g))
    pw = np.exp(-ks * (dd - ls) ** 2 / 2)
    md = float((dd * pw).sum() / pw.sum())
    vd = float(((dd - md) ** 2 * pw).sum() / pw.sum())
    theory = {"mean": [float(pref[0]), float(pref[1]), md], "var": [1 / kth, 1 / kth, vd]}
    per_mean = R.mean(axis=0)  # [traj, 3]
    per_cov = np.stack([np.cov(R[:, k, :].T) for k in range(n_traj)])  # [traj, 3, 3]
    se = lambda x: (x.std(axis=0, ddof=1) / math.sqrt(n_traj)).tolist()  # noqa: E731
    return {"workload": "starfish pair, a = l/12, 48 nodes, l = 2, k_s 81, l_s 5a, k_theta 2.446",
            "scheme": scheme, "dt": dt, "T": T, "steps": steps, "trajectories": n_traj, "tol_rfd": tol_rfd,
            "delta": delta, "theory": theory,
            "mean": per_mean.mean(axis=0).tolist(), "mean_se": se(per_mean),
            "cov": per_cov.mean(axis=0).tolist(), "cov_se": se(per_cov),
            "s_per_step": (time.perf_counter() - t0) / steps}


def run_learned(fb, W, np, torch, n_train=100, solves=100, epochs=4, n_test=6, progress=log):
    """The learned-correction study on dense suspensions: 1000 five-arm starfish x
    128 nodes, area fraction 0.35-0.45 (five values, one body shape each), jittered
    lattice with bounding-circle gaps down to 0.05 r_s, grid 1024^2, mixed
    precision.  Training: n_train configurations x `solves` random-force solves
    (the method's own solves, GMRES at 1e-6), `epochs` Adam steps per
    configuration.  Evaluation on n_test held-out configurations: GMRES iterations
    and solve time of three random-force mobility solves, plain block-diagonal
    preconditioner against the learned correction."""
    phis = [0.35, 0.375, 0.4, 0.425, 0.45]
    base = W.make("dense1000")
    ctx = fb.Context(**dict(base.params(), precision=fb.PREC_MIXED))
    sids = {}
    for phi in phis:
        r_s = W._rs_for_fraction(base.n_bodies, base.L, base.b, phi)
        sids[phi] = (ctx.add_shape(fb.starfish(r_s, base.b, base.n_arm, base.n_p)), r_s)
    ctx.mlp_init(seed=11, sym_order=base.n_arm)

    def config(seed, phi):
        w = W.make("dense1000", seed=seed, r_s=sids[phi][1])
        ctx.set_bodies(np.full(w.n_bodies, sids[phi][0]), w.q, w.theta)
        return w
    t0 = time.perf_counter()
    losses = []
    for k in range(n_train):
        phi = phis[k % len(phis)]
        config(600 + k, phi)
        info = ctx.mlp_train(n_solves=solves, epochs=epochs, lr=1e-3, seed=k)
        losses.append((info["loss_first"], info["loss_last"]))
        if progress and (k + 1) % 10 == 0:
            progress("learned: trained on %d configurations, %d solves (%.0f s), loss %.4g -> %.4g"
                     % (k + 1, (k + 1) * solves, time.perf_counter() - t0, info["loss_first"], info["loss_last"]))
    t_train = time.perf_counter() - t0
    rng = np.random.default_rng(77)
    rows = []
    for k in range(n_test):
        phi = phis[k % len(phis)]
        w = W.make("dense1000", seed=900 + k, r_s=sids[phi][1])
        Fs = [torch.as_tensor(rng.standard_normal(3 * w.n_bodies)).cuda() for _ in range(3)]
        U = torch.zeros(3 * w.n_bodies, dtype=torch.float64, device="cuda")
        row = {"phi": phi, "seed": 900 + k}
        for on in (False, True):
            ctx.mlp_use(on)
            ctx.set_bodies(np.full(w.n_bodies, sids[phi][0]), w.q, w.theta)
            torch.cuda.synchronize()
            t = time.perf_counter()
            its = [ctx.mobility(F, U)["gmres_iters"] for F in Fs]
            torch.cuda.synchronize()
            row["learned" if on else "plain"] = {"iters": its, "ms": 1e3 * (time.perf_counter() - t) / len(Fs)}
        rows.append(row)
        if progress:
            progress("learned: held-out %d (phi %.3f): plain %s, learned %s"
                     % (k, phi, row["plain"]["iters"], row["learned"]["iters"]))
    ctx.close()
    ip = sum(sum(r["plain"]["iters"]) for r in rows)
    il = sum(sum(r["learned"]["iters"]) for r in rows)
    return {"workload": "1000 five-arm starfish x 128 nodes, area fraction 0.35-0.45, grid 1024^2, mixed, tol 1e-6",
            "train_configurations": n_train, "train_solves": n_train * solves, "train_s": t_train,
            "loss_first_last": [losses[0], losses[-1]], "held_out": rows,
            "iters_plain": ip, "iters_learned": il, "iteration_ratio": il / ip}


def run_second_kind(fb, W, np, torch, reps=5):
    """The completed second-kind solver against the first-kind one on the
    100-starfish suspension (12,800 nodes, grid 256^2, FP64, GMRES 1e-8): time per
    operator application (HIP events around `reps` applications), iterations and
    time per mobility solve, and the two mobilities' difference."""
    wl = W.make("starfish100")
    ctx = fb.Context(**dict(wl.params(), tol_gmres=1e-8))
    sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
    ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    N = wl.n_nodes
    phi = torch.as_tensor(np.random.default_rng(3).standard_normal(2 * N)).cuda()
    out = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
    F = torch.as_tensor(wl.F).cuda()
    U1 = torch.zeros(3 * wl.n_bodies, dtype=torch.float64, device="cuda")
    U2 = torch.zeros_like(U1)
    res = {"workload": "starfish100: 100 five-arm starfish x 128 nodes, grid 256^2, FP64, GMRES tol 1e-8"}
    for name, fn in (("single_layer_matvec_ms", lambda: ctx.apply_M(phi, out, fb.PART_ALL)),
                     ("double_layer_matvec_ms", lambda: ctx.apply_double_layer(phi, out))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    for name, fn, U in (("first_kind", lambda: ctx.mobility(F, U1), U1),
                        ("second_kind", lambda: ctx.mobility_second_kind(F, U2), U2)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fn()
        torch.cuda.synchronize()
        res[name] = {"ms": 1e3 * (time.perf_counter() - t0), "gmres_iters": info["gmres_iters"],
                     "residual": info["gmres_residual"]}
    u1, u2 = U1.cpu().numpy(), U2.cpu().numpy()
    res["mobility_difference"] = float(np.linalg.norm(u1 - u2) / np.linalg.norm(u2))
    ctx.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default=",".join(FORMS), help="comma-separated subset of %s" % list(FORMS))
    ap.add_argument("--config", default="starfish10k")
    ap.add_argument("--matvecs", type=int, default=20)
    ap.add_argument("--train-configs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="step", choices=["step", "matvec", "copy", "batch", "bd-starfish", "bd-pair", "learned",
                             "second-kind"],
                    help="step: the EM-RFD benchmark; matvec: only single-layer matvecs of the first form "
                         "(short runs for counter collection); copy: a plain 1 GiB device copy "
                         "used to calibrate the HBM byte counters; batch: EM-RFD steps of the "
                         "64-suspension uneven batch, batched against one after another; bd-starfish / bd-pair: "
                         "the Brownian-dynamics validation runs (single starfish with and without the "
                         "RFD term; spring-coupled pair with EM-RFD and AB2-RFD at three time steps); learned: the "
                         "learned-correction study on 1000-body dense suspensions; second-kind: the completed "
                         "second-kind solver against the first-kind one on 100 bodies")
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
    os.makedirs(os.path.dirname(TUNE_CACHE), exist_ok=True)
    if args.mode == "copy":
        n = (1 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "copies": args.steps}))
        return
    if args.mode == "batch":
        run_batch(args, fb, W, np, torch)
        return
    if args.mode == "bd-starfish":
        print(json.dumps(dict(mode="bd-starfish", **run_bd_starfish(fb, W, np, torch))), flush=True)
        return
    if args.mode == "bd-pair":
        for dt in (0.0297, 0.0149, 0.00743):  # tau_s / 4, / 8, / 16
            for scheme in ("em", "ab2"):
                print(json.dumps(dict(mode="bd-pair", **run_bd_pair(fb, W, np, torch, scheme=scheme, dt=dt))),
                      flush=True)
        return
    if args.mode == "second-kind":
        print(json.dumps(dict(mode="second-kind", **run_second_kind(fb, W, np, torch))), flush=True)
        return
    if args.mode == "learned":
        print(json.dumps(dict(mode="learned", **run_learned(fb, W, np, torch))), flush=True)
        return
    wl = W.make(args.config)
    names = [f for f in args.forms.split(",") if f]
    log("workload %s: %d bodies x %d nodes" % (args.config, wl.n_bodies, wl.n_p))
    if args.mode == "matvec":
        form = FORMS[names[0]]
        prec = fb.PREC_FP64 if form["precision"] == "fp64" else fb.PREC_MIXED
        ctx = fb.Context(**wl.params(), precision=prec)
        sid = ctx.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
        ctx.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
        N = ctx.get_derived()["n_nodes"]
        mu = torch.as_tensor(np.random.default_rng(1).standard_normal(2 * N)).cuda()
        out = torch.zeros(2 * N, dtype=torch.float64, device="cuda")
        for _ in range(args.matvecs):
            ctx.apply_M(mu, out, fb.PART_ALL)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "matvec", "form": names[0], "nodes": N, "matvecs": args.matvecs}))
        ctx.close()
        return
    results, kts = {}, {}
    for nm in names:
        results[nm], kts[nm], xh, d = run_form(nm, FORMS[nm], wl, args, fb, W, np, torch)
    head = names[-1]
    N, M = d["n_nodes"], d["grid_M"]
    res = {
        "metric": METRIC, "value": results[head]["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": results[head]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": results[head]["dtype"],
        "data": "synthetic",
        "config": {"workload": "%s: %d five-arm starfish x %d nodes (%d nodes), area fraction 0.3, grid %d^2, "
                               "tol 1e-6, EM-RFD step (Lanczos + random field + 3 GMRES solves)"
                               % (args.config, wl.n_bodies, wl.n_p, N, M),
                   "form": head, "gmres_tol": wl.tol_gmres, "lanczos_tol": wl.tol_lanczos},
        "matvec": results[head]["matvec"],
        "forms": results,
        "roofline": roofline(kts[head], xh, wl, d),
        "cpu_baseline": None,
    }
    if "fp64" in results and head != "fp64":
        res["speedup_vs_fp64_form"] = results[head]["steps_per_s"] / results["fp64"]["steps_per_s"]
    if not args.no_cpu_baseline:
        from oracle import fbim as OF
        prm = OF.derive_params(wl.L, wl.tol_ewald, n_box=wl.n_box, grid_M=wl.grid_M, xi=wl.xi, P=wl.P)
        # the FP64 form's iteration counts when it ran (the CPU path is FP64)
        sol = results["fp64" if "fp64" in results else head]["solver"]
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(wl, prm, sol["full_matvecs_per_step"], sol["real_matvecs_per_step"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
