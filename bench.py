"""Throughput benchmark of the SSD hot path on one MI355X.

Workload: inviscid flow (Mach 0.3) past an ellipse (semi-axes 0.5 x 0.1)
spinning at omega = 1 inside a rotating disk r < 3, in a stationary box
[-30, 30]^2; 4096 x (64 + 180) = 999,424 quadrilaterals, N = 4 solution
points per direction (63,963,136 DOF), 4096 sliding-interface faces per
side, SSP-RK3; the initial state is the far field with a seeded 1% density
perturbation (SplitMix64, seed 20150307).

One "step" is one SSP-RK3 step (three residual evaluations, each with its
mortar rebuild and projection).  `value` is DOF-updates per second per RK
stage: 4 N^2 E x 3 x steps / seconds, with the state resident in HBM.

Prints one JSON line.  `--gpus` above 1 is refused: the library runs one
mesh on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per RK stage at stated L2 error; learned-coarse vs plain speedup"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_ellipse_n4.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1503_02198_amd", "csrc", f)
                  for f in ("ssd_kernels.hip", "ssd_tiles.h", "ssd_device.h", "ssd_internal.h")]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(args):
    from workloads import cases as C
    from workloads import meshes as M
    if getattr(args, "viscous", False):
        # Navier-Stokes on the same mesh: isothermal ellipse wall, Mach 0.3,
        # Re 1000 on the major axis
        mesh = M.ellipse_mesh(K=args.K, n_in=args.n_in, n_out=args.n_out,
                              wall=M.FACE_WALL_ISOTHERMAL)
        case = C.ellipse_viscous_case(mach=0.3, reynolds=1000.0)
    else:
        mesh = M.ellipse_mesh(K=args.K, n_in=args.n_in, n_out=args.n_out)
        case = C.ellipse_case()
    N = args.N
    E = len(mesh["zone"])
    Q0 = C.perturbed_farfield_state(case, N, E).astype(np.float32)
    # time step from the smallest corner-to-corner edge and the fastest
    # signal (|u| + c + omega r_max), CFL 0.1 per solution-point spacing
    xy = mesh["xy"][:, [0, 3, 6, 9]]
    edges = np.linalg.norm(xy - np.roll(xy, 1, axis=1), axis=-1)
    h = edges.min()
    rho, u, v, p = case["farfield"]
    lam = np.hypot(u, v) + np.sqrt(case["gamma"] * p / rho) + abs(case["omega"]) * mesh["radius"]
    dt = 0.1 * h / (lam * N * N)
    return mesh, case, N, E, Q0, dt


def batch_workload(seed=20150307, n=64):
    """The many-case workload: n instances, Taylor-Couette or vortex with
    equal odds, cell count log-uniform in [1k, 50k] (nearest mesh of the
    family), N uniform in 2..5, omega uniform in [0.1, 2], all drawn from one
    seed.  Initial states are the far field with a seeded 1% density
    perturbation; each case steps at its own CFL 0.1 time step."""
    from workloads import cases as C
    from workloads import meshes as M
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n):
        kind = "couette" if rng.random() < 0.5 else "vortex"
        E_target = float(np.exp(rng.uniform(np.log(1000.0), np.log(50000.0))))
        N = int(rng.integers(2, 6))
        omega = float(rng.uniform(0.1, 2.0))
        if kind == "vortex":
            f = int(min(11, max(2, round(np.sqrt(E_target / 384.0)))))
            mesh = M.vortex_mesh(f)
            case = C.vortex_case(omega=omega)
        else:
            nr = int(min(112, max(16, 2 * round(np.sqrt(E_target / 4.0) / 2.0))))
            mesh = M.couette_mesh(nr, 4 * nr, phi_offset=0.37 * 2 * np.pi / (4 * nr))
            case = C.couette_case(omega=omega)
        E = len(mesh["zone"])
        Q0 = C.perturbed_farfield_state(case, N, E, seed=seed + c).astype(np.float32)
        xy = mesh["xy"][:, [0, 3, 6, 9]]
        h = np.linalg.norm(xy - np.roll(xy, 1, axis=1), axis=-1).min()
        rho, u, v, p = case["farfield"]
        r_max = float(np.abs(mesh["xy"]).max())
        lam = np.hypot(u, v) + np.sqrt(case["gamma"] * p / rho) + abs(omega) * r_max
        out.append(dict(kind=kind, mesh=mesh, case=case, N=N, E=E, Q0=Q0,
                        dt=0.1 * h / (lam * N * N)))
    return out


def batched_main(args):
    """Aggregate throughput of the many-case workload: one batch (graphs,
    then eager launches) against stepping every case on its own."""
    import torch
    from paper_1503_02198_amd import Batch, Mesh, pack_state
    ws = batch_workload()
    meshes = [Mesh(w["mesh"], w["case"], w["N"], device=0) for w in ws]
    qs = [torch.from_numpy(pack_state(w["Q0"])).to("cuda:0") for w in ws]
    works = [torch.empty(m.info["work_len"], dtype=torch.float32, device="cuda:0") for m in meshes]
    dts = [w["dt"] for w in ws]
    dof = sum(4 * w["N"] ** 2 * w["E"] for w in ws)
    steps = args.steps
    batch = Batch(meshes)
    res = {}
    for mode in ("graph", "eager"):
        graph = mode == "graph"
        batch.rk_steps(qs, works, [0.0] * len(ws), dts, args.warmup, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.rk_steps(qs, works, [0.0] * len(ws), dts, steps, graph=graph)
        torch.cuda.synchronize()
        res[mode] = time.perf_counter() - t0
    # every case on its own, one after the other on the same stream
    for m, q, wk, w in zip(meshes, qs, works, ws):
        m.rk_steps(q, wk, 0.0, w["dt"], args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m, q, wk, w in zip(meshes, qs, works, ws):
        m.rk_steps(q, wk, 0.0, w["dt"], steps)
    torch.cuda.synchronize()
    res["separate"] = time.perf_counter() - t0
    for m in meshes:
        m.check()
    groups = batch.groups()
    rate = {k: dof * 3 * steps / v for k, v in res.items()}
    print(json.dumps({
        "metric": "aggregate DOF-updates/s per RK stage, 64-case batch",
        "value": rate["graph"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 Taylor-Couette and vortex instances, cells log-uniform in "
                               "[1k, 50k], N in 2..5, omega in [0.1, 2], seed 20150307, SSP-RK3",
                   "cells": sum(w["E"] for w in ws), "dof": dof,
                   "kinds": {k: sum(w["kind"] == k for w in ws) for k in ("vortex", "couette")},
                   "groups": groups},
        "batched_graph": rate["graph"], "batched_eager": rate["eager"],
        "separate": rate["separate"], "speedup_vs_separate": rate["graph"] / rate["separate"],
        "seconds": res}), flush=True)


def mlp_kernels_main(args):
    """Throughput of the learned-correction kernels alone, on seeded random
    rows: the normalisation fit, 200 Adam steps on minibatches of 4096 rows
    with input noise 0.1, one forward pass over all rows, then 200 SSP-RK3
    steps of the coarse viscous ellipse mesh (64 x (8 + 16) cells, N = 3)
    with the network attached.  Only library entry points are called."""
    import torch
    from paper_1503_02198_amd import MLP
    from paper_1503_02198_amd import subgrid as G
    from workloads import cases as C
    meshes = G.ellipse_pair(64, 8, 16)
    P = G.Pair(meshes, C.ellipse_viscous_case(omega=0.2))
    net = MLP(3)
    net.set_params(G.init_params(np.random.default_rng(1), net.n_in, net.n_out))
    rows, batch, steps = P.Ec * 64, 4096, 200
    g = torch.Generator().manual_seed(20150307)
    X = torch.randn(rows * net.n_in, generator=g).to("cuda:0")
    T = torch.randn(rows * net.n_out, generator=g).to("cuda:0")
    net.fit_normalization(X, T, min_rel=1e-2)
    rng = np.random.default_rng(2)
    idx = [torch.tensor(rng.integers(0, rows, batch).astype(np.int32), device="cuda:0")
           for _ in range(steps)]
    Y = torch.empty(rows * net.n_out, device="cuda:0")
    q, w = P.uniform(P.coarse), P.work(P.coarse)
    P.coarse.attach(net)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    t_train = timed(lambda: [net.train_step(X, T, i, 1e-3, 0.1, 7) for i in idx])
    t_fwd = timed(lambda: net.forward(X, Y))
    t_rk = timed(lambda: P.coarse.rk_steps(q, w, 0.0, P.dt_c, steps))
    P.coarse.check()
    print(json.dumps({"metric": "learned-correction kernels", "rows": rows,
                      "train_samples_per_s": steps * batch / t_train,
                      "forward_samples_per_s": rows / t_fwd,
                      "corrected_rk3_steps_per_s": steps / t_rk,
                      "cells": P.Ec, "N": 3}), flush=True)


def subgrid_main(args):
    """The learned-correction workload end to end: fine runs for training
    data, training, rounds of training on rows taken along the corrected
    coarse runs (a posteriori), then plain SSD runs and the corrected coarse
    run over one evaluation interval, with the speedup at equal error on the
    plain runs' cost-error front."""
    import torch
    from paper_1503_02198_amd import MLP
    from paper_1503_02198_amd import subgrid as G
    from workloads import cases as C
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)
    cfg = dict(K=64, n_in=8, n_out=16, runs=4, snapshots=500, window=(0.5, 1.0), epochs=40,
               batch=4096, lr=2e-3, noise=0.1, eval_window=(args.eval_t0, args.eval_t1),
               seed=20150307, per_step=True, rounds=args.aposteriori_rounds,
               traj_snapshots=250, relax_rate=args.relax_rate, retrain=args.retrain,
               resync=args.resync, zero_free_stream=not args.no_zero_free_stream,
               ft_epochs=args.ft_epochs, ft_lr=1e-3)
    meshes = G.ellipse_pair(cfg["K"], cfg["n_in"], cfg["n_out"])
    rng = np.random.default_rng(cfg["seed"])
    rates = rng.uniform(0.5, 2.0, cfg["runs"])
    rate_eval = float(rng.uniform(0.5, 2.0))
    X, T, gen_s = G.generate(meshes, G.convective_omega(rates), cfg["window"][0], cfg["window"][1],
                             cfg["snapshots"], log=log)
    rows = X.numel() // 84
    net = MLP(3)
    losses, train_s = G.train(net, X, T, cfg["epochs"], cfg["batch"], cfg["lr"], seed=7,
                              noise=cfg["noise"])
    # the free stream is the same at every rate: any rate's pair serves
    calib = (G.Pair(meshes, C.ellipse_viscous_case(omega=G.convective_omega(rate_eval)))
             if cfg["zero_free_stream"] else None)
    if calib is not None:
        G.zero_at_free_stream(net, calib)
    log(f"training loss {losses[0]:.4e} -> {losses[-1]:.4e} in {train_s:.2f} s")
    steps = cfg["epochs"] * (rows // cfg["batch"])
    rounds = []
    if cfg["rounds"]:
        # the network trained on the fine runs alone, evaluated for comparison
        res0 = G.evaluate(meshes, net, G.convective_omega(rate_eval), *cfg["eval_window"],
                          weights=(1.0,), per_step=cfg["per_step"])
        rounds.append({"round": 0, "err": res0["learned"][0]["err"],
                       "fallback": res0["learned"][0]["fallback"], "training_rows": rows})
    # a posteriori rounds: rows along the corrected coarse runs, added to the
    # data, and training continued on all of it
    for r in range(cfg["rounds"]):
        Xt, Tt, gs, restarts = G.generate_trajectory(
            meshes, G.convective_omega(rates), net, cfg["window"][0], cfg["window"][1],
            cfg["traj_snapshots"], cfg["relax_rate"], per_step=cfg["per_step"], log=log,
            resync=cfg["resync"])
        X, T = torch.cat([X, Xt]), torch.cat([T, Tt])
        del Xt, Tt
        rows = X.numel() // 84
        gen_s += gs
        if cfg["retrain"]:    # fresh weights and normalisation on all rows so far
            ls, ts = G.train(net, X, T, cfg["epochs"], cfg["batch"], cfg["lr"], seed=11 + r,
                             noise=cfg["noise"])
        else:                 # continue from the current weights
            ls, ts = G.train(net, X, T, cfg["ft_epochs"], cfg["batch"], cfg["ft_lr"],
                             seed=11 + r, noise=cfg["noise"], resume=True)
        train_s += ts
        if calib is not None:
            G.zero_at_free_stream(net, calib)
        steps += (cfg["epochs"] if cfg["retrain"] else cfg["ft_epochs"]) * (rows // cfg["batch"])
        log(f"round {r + 1}: {rows} rows, loss {ls[0]:.4e} -> {ls[-1]:.4e} in {ts:.2f} s")
        rounds.append({"round": r + 1, "training_rows": rows, "restarts": restarts,
                       "loss_last_epoch": ls[-1]})
    res = G.evaluate(meshes, net, G.convective_omega(rate_eval), *cfg["eval_window"],
                     weights=(1.0,), per_step=cfg["per_step"])
    sp = G.speedup_at_equal_error(res)[0]
    if rounds:
        rounds[-1]["err"] = res["learned"][0]["err"]
    print(json.dumps({
        "metric": "learned-coarse vs plain SSD: wall-clock speedup at equal error (interpolated "
                  "on the plain runs' cost-error front)",
        "value": sp["speedup_interpolated"], "unit": "x", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32 state, bf16 network products (f32 accumulate)", "data": "synthetic",
        "config": {"workload": "viscous rotating ellipse (axes 1 x 0.2, isothermal wall, Mach 0.2, "
                               "Re 1000), coarse 64 x (8 + 16) cells N=3, nested fine mesh N=6; "
                               "rotation rates uniform [0.5, 2] in the convective unit",
                   **{k: v for k, v in cfg.items()}, "rates": rates.tolist(),
                   "rate_eval": rate_eval, "training_rows": rows},
        "speedup_vs_cheapest_plain_run_at_most_that_error": sp["speedup"],
        "learned_err": sp["err"], "plain_run_at_most_that_error": sp["plain_run"],
        "plain_run_err": sp["plain_err"],
        "runs": [{k: r[k] for k in ("run", "s", "err", "dof")} for r in res["plain"] + res["learned"]],
        "fallback": res["learned"][0]["fallback"],
        "training": {"loss_first_epoch": losses[0], "loss_last_epoch": losses[-1],
                     "steps": steps, "seconds": train_s,
                     "samples_per_s": steps * cfg["batch"] / train_s,
                     "aposteriori_rounds": rounds},
        "data_generation_s": gen_s}), flush=True)


def contraction_probe_main(args):
    """The per-cell contractions (interpolation to the flux points, a
    pointwise flux, the derivative back) on the stage kernel's layout, as
    vector fused multiply-adds and on the matrix cores (FP32 MFMA), for the
    choice between the two: time per launch and agreement of the results."""
    import torch
    from paper_1503_02198_amd import Mesh
    from workloads import cases as C
    from workloads import meshes as M
    gm = Mesh(M.box_mesh(2, 2), C.vortex_case(), 4, device=0)   # supplies the N = 4 operators
    cells, reps = 999424, args.probe_reps
    g = torch.Generator().manual_seed(20150307)
    q = (1.0 + 0.1 * torch.rand(64 * cells, generator=g)).to("cuda:0")
    outs, ms = [], []
    for variant in (0, 1):
        out = torch.empty_like(q)
        for _ in range(3):
            gm.probe_contraction(variant, cells, reps, q, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = args.probe_launches
        e0.record()
        for _ in range(n):
            gm.probe_contraction(variant, cells, reps, q, out)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1) / n)
        outs.append(out)
    diff = float(((outs[1] - outs[0]).abs().max() / outs[0].abs().max()).item())
    # useful flops per launch: per cell, line and variable and round, 5 x 4
    # multiply-adds to interpolate, 5 products, 4 x 5 to differentiate
    flops = cells * 4 * 4 * reps * (2 * 20 + 5 + 2 * 20)
    print(json.dumps({"metric": "contraction probe (N = 4, FP32)", "cells": cells, "reps": reps,
                      "valu_us": 1e3 * ms[0], "mfma_us": 1e3 * ms[1],
                      "valu_tflops": flops / (ms[0] * 1e-3) / 1e12,
                      "mfma_tflops": flops / (ms[1] * 1e-3) / 1e12,
                      "mfma_over_valu_time": ms[1] / ms[0], "max_rel_diff": diff}), flush=True)


def stream_probe_main(args):
    """Bandwidth ceiling of the stage kernel's state traffic: c = 0.75 a +
    0.25 b over arrays the size of the benchmark's state (63,963,136
    floats), two read and one written, with 16-byte plain, 16-byte
    non-temporal, and the stage kernel's own 4-byte non-temporal buffer
    accesses (variants 0, 1, 2)."""
    import torch
    from paper_1503_02198_amd import Mesh
    from workloads import cases as C
    from workloads import meshes as M
    gm = Mesh(M.box_mesh(2, 2), C.vortex_case(), 4, device=0)   # supplies the device handle
    n = 4 * 16 * 999424
    g = torch.Generator().manual_seed(20150307)
    a = torch.rand(n, generator=g).to("cuda:0")
    b = torch.rand(n, generator=g).to("cuda:0")
    c = torch.empty_like(a)
    t_end = time.perf_counter() + args.settle_s   # settle the clocks
    while time.perf_counter() < t_end:
        for _ in range(100):
            gm.probe_stream(2, n, a, b, c)
        torch.cuda.synchronize()
    res = {}
    for variant in (0, 1, 2):
        for _ in range(5):
            gm.probe_stream(variant, n, a, b, c)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.probe_launches)]
        for k in range(args.probe_launches):
            ev[2 * k].record()
            gm.probe_stream(variant, n, a, b, c)
            ev[2 * k + 1].record()
        torch.cuda.synchronize()
        us = sorted(1e3 * ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.probe_launches))
        avg = sum(us) / len(us)
        err = float((c - (0.75 * a + 0.25 * b)).abs().max().item())
        res[("x4_plain", "x4_nontemporal", "rows_nontemporal")[variant]] = {
            "avg_us": avg, "median_us": us[len(us) // 2], "TB_s": 12.0 * n / (avg * 1e-6) / 1e12,
            "max_abs_err": err}
    print(json.dumps({"metric": "stream probe: two FP32 arrays read, one written",
                      "floats_per_array": n, "bytes_per_launch": 12 * n, "launches": args.probe_launches,
                      "variants": res}), flush=True)


def traffic_for(kind_hash, E, N):
    """HBM bytes per stage launch from the committed rocprofv3 counter runs,
    or None when the kernels changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != kind_hash or t.get("n_elem") != E or t.get("N") != N:
        return None
    return t.get("bytes_per_launch")


def _usable_cores():
    """Host cores this process may run on, at most 16 (the CPU share of one
    GPU on the measurement machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_step_timed(mesh, case, N, Q0, dt, cells, depth=3):
    """One SSP-RK3 step of the FP64 oracle on the sub-mesh around `cells`
    (mesh build and set-up excluded from the time): (seconds, sub-mesh
    cells, sub-mesh state after the step, global indices)."""
    from oracle.ssd import SSD, submesh
    sub, idx = submesh(mesh, cells, depth=depth)
    ora = SSD(sub, case, N)
    Qs = Q0[..., idx].astype(np.float64)
    t0 = time.perf_counter()
    Q1 = ora.ssprk3_step(Qs, 0.0, dt)
    return time.perf_counter() - t0, len(idx), Q1, idx


def _cpu_worker(rank, lo, hi, runs, viscous, barrier, out):
    """One process of the all-cores oracle timing: rebuilds the workload,
    then times `runs` oracle steps on the sub-mesh of cells [lo, hi), each
    started together with the other processes."""
    from threadpoolctl import threadpool_limits

    from oracle.ssd import SSD, submesh

    class A:
        N, K, n_in, n_out = 4, 4096, 64, 180
    A.viscous = viscous
    mesh, case, N, E, Q0, dt = workload(A)
    with threadpool_limits(1):
        sub, idx = submesh(mesh, np.arange(lo, hi), depth=3)
        ora = SSD(sub, case, N)
        Qs = Q0[..., idx].astype(np.float64)
        times = []
        for _ in range(runs):
            barrier.wait()
            t0 = time.perf_counter()
            ora.ssprk3_step(Qs, 0.0, dt)
            times.append(time.perf_counter() - t0)
    out.put((rank, len(idx), times))


def cpu_baseline(mesh, case, N, Q0, dt, q_gpu_step, target_s, runs=3):
    """The FP64 oracle timed on the host, on 1 core and on every usable core
    (the median of `runs` steps each), on bounded samples of the workload;
    also the oracle-vs-GPU errors of one step on the sampled cells."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from tests.parity_utils import change_error, state_error
    E = len(mesh["zone"])
    n = 8192
    with threadpool_limits(1):
        while True:
            sample = np.arange(min(n, E))
            el, ncell, Q1, idx = _oracle_step_timed(mesh, case, N, Q0, dt, sample)
            # one step of the sample takes between 2/3 of the target and about the target
            if el > target_s / 1.5 or n >= E:
                break
            n = int(n * min(8.0, max(1.5, target_s / max(el, 1e-3))))
        one = [el] + [_oracle_step_timed(mesh, case, N, Q0, dt, sample)[0]
                      for _ in range(runs - 1)]
    loc = np.searchsorted(idx, sample)
    err = state_error(q_gpu_step[..., sample], Q1[..., loc])
    ch, bound = change_error(q_gpu_step[..., sample], Q1[..., loc], Q0[..., sample])
    t1 = float(np.median(one))
    rate1 = 4 * N * N * ncell * 3 / t1

    # all cores: one process per core, each on its own slice of the cells
    P = _usable_cores()
    per = min(len(sample), E // P)
    ctx = mp.get_context("spawn")
    barrier, out = ctx.Barrier(P), ctx.Queue()
    procs = [ctx.Process(target=_cpu_worker, args=(r, r * per, (r + 1) * per, runs,
                                                    case["mu"] > 0.0, barrier, out))
             for r in range(P)]
    for pr in procs:
        pr.start()
    res = sorted(out.get() for _ in range(P))
    for pr in procs:
        pr.join()
    cells_all = sum(r[1] for r in res)
    wall = [max(r[2][k] for r in res) for k in range(runs)]
    tP = float(np.median(wall))
    rateP = 4 * N * N * cells_all * 3 / tP
    rec = dict(value=rateP, unit="DOF-updates/s", cores=P, kind="oracle",
               sample=(f"FP64 numpy oracle, one SSP-RK3 step (3 stages), median of {runs}: "
                       f"{P} processes, one per core, each on the sub-mesh of {per} cells of the "
                       f"workload (with every interface cell and 3 neighbour layers; "
                       f"{cells_all} cells in all), {tP:.2f} s; on 1 core the sub-mesh of cells "
                       f"0..{len(sample) - 1} ({ncell} cells), {t1:.2f} s"),
               value_1core=rate1, seconds_1core=one, seconds_all_cores=wall)
    return rec, err, ch, bound


def _counter_means(csv_path, counter):
    """Mean value of one counter per kernel name in a rocprofv3 counter CSV."""
    import csv
    acc = {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            k = r["Kernel_Name"]
            acc.setdefault(k, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def ingest_counters(fetch_csv, write_csv, calib_fetch_csv, calib_write_csv, E, N):
    """Write the stage kernel's measured HBM bytes per launch from rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch), each scaled by what the
    same counter reads for a plain 1 GiB device copy."""
    def pick(d, key):
        vals = [v for k, v in d.items() if key in k]
        if not vals:
            raise SystemExit(f"no {key} dispatches in the counter file")
        return max(vals)
    copy = float(1 << 30)
    f_scale = copy / (pick(_counter_means(calib_fetch_csv, "FETCH_SIZE"), "copyBuffer") * 1024)
    w_scale = copy / (pick(_counter_means(calib_write_csv, "WRITE_SIZE"), "copyBuffer") * 1024)
    fetch = pick(_counter_means(fetch_csv, "FETCH_SIZE"), "k_stage<") * 1024 * f_scale
    write = pick(_counter_means(write_csv, "WRITE_SIZE"), "k_stage<") * 1024 * w_scale
    rec = {"kernel": "k_stage", "kernel_hash": kernel_hash(), "n_elem": E, "N": N,
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write, "fetch_scale": f_scale, "write_scale": w_scale,
           "note": "mean over the stage launches of a short run (stages 1-3 averaged)"}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def calib_copy(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling rocprofv3 counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": nbytes, "calib_copy_bytes_written": nbytes,
                      "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--N", type=int, default=4)
    ap.add_argument("--K", type=int, default=4096)
    ap.add_argument("--n-in", type=int, default=64)
    ap.add_argument("--n-out", type=int, default=180)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--viscous", action="store_true",
                    help="Navier-Stokes on the same mesh (isothermal ellipse wall, Mach 0.3, "
                         "Re 1000), reported alongside the Euler headline")
    ap.add_argument("--scheme", choices=("rk3", "rk54"), default="rk3",
                    help="time integrator of the headline run (SSP-RK3, the benchmark "
                         "configuration; SSPRK54, the paper's scheme, reported alongside)")
    ap.add_argument("--cpu-seconds", type=float, default=4.0)
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed steps before the warm-up steps (clock settling)")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="the 64-case batch workload instead of the headline run")
    ap.add_argument("--subgrid", action="store_true",
                    help="the learned-correction workload (training data, training, evaluation)")
    ap.add_argument("--aposteriori-rounds", type=int, default=2,
                    help="learned-correction workload: rounds of training on rows taken along "
                         "the corrected coarse runs")
    ap.add_argument("--relax-rate", type=float, default=0.0,
                    help="relaxation rate towards the restricted fine state in the a posteriori "
                         "targets (0: none)")
    ap.add_argument("--retrain", action="store_true",
                    help="a posteriori rounds train afresh on all rows instead of continuing "
                         "from the current weights")
    ap.add_argument("--resync", type=float, default=0.2,
                    help="a posteriori rows: restart the corrected coarse runs from the restricted "
                         "fine state every RESYNC time units (0: only on failure)")
    ap.add_argument("--no-zero-free-stream", action="store_true",
                    help="learned-correction workload: keep the network's output offset at the "
                         "free stream (by default it is shifted to zero after each training)")
    ap.add_argument("--ft-epochs", type=int, default=15)
    ap.add_argument("--eval-t0", type=float, default=0.5)
    ap.add_argument("--eval-t1", type=float, default=0.7)
    ap.add_argument("--mlp-kernels", action="store_true",
                    help="throughput of the learned-correction kernels on seeded random rows")
    ap.add_argument("--contraction-probe", action="store_true",
                    help="vector-ALU vs matrix-core (FP32 MFMA) per-cell contractions")
    ap.add_argument("--stream-probe", action="store_true",
                    help="bandwidth ceiling of the stage kernel's state traffic")
    ap.add_argument("--probe-reps", type=int, default=16)
    ap.add_argument("--probe-launches", type=int, default=20)
    ap.add_argument("--ingest-counters", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV",
                                                          "CALIB_FETCH_CSV", "CALIB_WRITE_CSV"))
    args = ap.parse_args()
    if args.ingest_counters:
        E = args.K * (args.n_in + args.n_out)
        ingest_counters(*args.ingest_counters, E=E, N=args.N)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "method over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return
    if args.batched:
        batched_main(args)
        return
    if args.subgrid:
        subgrid_main(args)
        return
    if args.mlp_kernels:
        mlp_kernels_main(args)
        return
    if args.contraction_probe:
        contraction_probe_main(args)
        return
    if args.stream_probe:
        stream_probe_main(args)
        return

    from paper_1503_02198_amd import Mesh, pack_state, unpack_state
    t_setup = time.perf_counter()
    mesh, case, N, E, Q0, dt = workload(args)
    gm = Mesh(mesh, case, N, device=0)
    q = torch.from_numpy(pack_state(Q0)).to("cuda:0")
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0")
    setup_s = time.perf_counter() - t_setup
    print(f"# setup {setup_s:.1f} s: E={E} N={N} K={gm.info['K']} cubic={gm.info['n_cubic']} "
          f"dt={dt:.3e}", file=sys.stderr, flush=True)

    t = 0.0
    scheme = args.scheme
    # Clock settling: after an idle spell the GPU's clocks and power state
    # need a few hundred stage launches to settle (measured: launches 13-25
    # of a cold start run 230-245 us, later ones 170-190 us).  The path is
    # stepped for `--settle-s` seconds before the `--warmup` steps, so that
    # the timed steps see the state a long run runs in.
    settle_steps = 0
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < args.settle_s:
        gm.rk_steps(q, work, t, dt, 50, scheme=scheme)
        torch.cuda.synchronize()
        t += 50 * dt
        settle_steps += 50
    if args.warmup:
        gm.rk_steps(q, work, t, dt, args.warmup, scheme=scheme)
        t += args.warmup * dt
    gm.check()
    torch.cuda.synchronize()
    # timed region: only the stage kernel is timed, by events attached to
    # its dispatch
    gm.timing_enable(kernels=["stage"])
    gm.timing_reset()
    t0 = time.perf_counter()
    gm.rk_steps(q, work, t, dt, args.steps, scheme=scheme)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t += args.steps * dt
    ms, n = gm.timing_read("stage")
    per = 1e3 * gm.timing_samples("stage")
    kern = {"stage": dict(launches=n, avg_us=1e3 * ms / n, total_ms=ms,
                          median_us=float(np.median(per)), p10_us=float(np.percentile(per, 10)),
                          p90_us=float(np.percentile(per, 90)), min_us=float(per.min()),
                          max_us=float(per.max()))}
    # the other kernels, from a short run after the timed region
    others = ("traces", "mortar") + (("grad",) if args.viscous else ())
    gm.timing_enable(kernels=list(others))
    gm.timing_reset()
    gm.rk_steps(q, work, t, dt, 20, scheme=scheme)
    for k in others:
        ms, n = gm.timing_read(k)
        kern[k] = dict(launches=n, avg_us=(1e3 * ms / n) if n else None, total_ms=ms)
    gm.timing_enable(False)
    gm.check()
    print(f"# timed {args.steps} steps in {el:.3f} s", file=sys.stderr, flush=True)

    dof = 4 * N * N * E
    stages = (3 if scheme == "rk3" else 5) * args.steps
    value = dof * stages / el
    # algorithmic bytes of one stage launch: the state it must read and
    # write, on average per DOF, and the cell geometry as the FP64 node
    # coordinates read once per cell (4 nodes, 64 bytes, for a bilinear
    # cell; 12 nodes, 192 bytes, for a cubic one).  SSP-RK3: Q_k and, in
    # stages 2-3, Q^n, then Q_{k+1}: (8 + 12 + 12) / 3 bytes.  SSPRK54:
    # stage 1 8, stages 2 and 3 12, stage 4 20 (it also reads U2 and writes
    # the last stage's increment over it), stage 5 16 (it reads that
    # increment): 13.6 bytes.
    n_cubic = gm.info["n_cubic"]
    alg_bytes = (((32.0 / 3.0) if scheme == "rk3" else 13.6) * dof
                 + 64.0 * (E - n_cubic) + 192.0 * n_cubic)
    if args.viscous:
        # the viscous stage also reads the SP gradients (8 values per point,
        # 8 B/DOF); the gradient pass is a kernel of its own
        alg_bytes += 8.0 * dof
    stage_us = kern["stage"]["avg_us"]
    achieved = alg_bytes / (stage_us * 1e-6) / 1e9
    hsh = kernel_hash()
    # the stored counters are those of the SSP-RK3 run
    traffic = traffic_for(hsh, E, N) if scheme == "rk3" and not args.viscous else None

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rotating-ellipse Euler on a sliding mesh: 999,424 quads "
                               "(4096 x (64+180)), N=4, 4096 interface faces per side, "
                               + ("SSP-RK3" if scheme == "rk3" else "SSPRK54 (five stages)")
                               + (", Navier-Stokes (Mach 0.3, Re 1000, isothermal ellipse wall)"
                                  if args.viscous else "")
                               + ", seeded 1% density perturbation",
                   "n_elem": E, "N": N, "dof": dof, "dt": dt, "K": gm.info["K"],
                   "n_cubic": gm.info["n_cubic"], "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_stage (element residual + RK stage update)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": stage_us},
        "kernels": kern,
        "kernel_hash": hsh,
        "settle": {"steps": settle_steps, "seconds": args.settle_s},
    }
    if not args.no_cpu_baseline and scheme == "rk3" and not args.viscous:
        # one GPU step from the same initial state for the sampled parity check
        q1 = torch.from_numpy(pack_state(Q0)).to("cuda:0")
        gm.rk_step(q1, work, 0.0, dt)
        gm.check()
        q1h = unpack_state(q1.cpu().numpy(), N, E).astype(np.float64)
        cb, err, ch, bound = cpu_baseline(mesh, case, N, Q0, dt, q1h, args.cpu_seconds)
        result["cpu_baseline"] = cb
        # one GPU step from the same state against the oracle's on the
        # sampled cells: the state error, and the error of the step's change
        # (the step moves the state by about 2e-5 of its norm)
        result["l2_rel_vs_oracle"] = [float(x) for x in err]
        result["step_change_err_vs_oracle"] = {"value": float(ch), "bound": float(bound)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
