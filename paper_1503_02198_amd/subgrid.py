"""Learned per-element subgrid correction: training data from fine runs of the
solver, training, and the coarse run it serves (an extension of the method;
not in the paper).

The steps are calls of the HIP library (include/ssd.h) in sequence: fine
time steps, residuals, the restriction of the nested fine mesh to the coarse
one, features and targets, minibatch gradient and Adam steps, and coarse
SSP-RK3 with the network attached.  This module only orders those calls and
draws the seeded random numbers the procedure needs (rotation rates, initial
weights, minibatch order), which it passes in.

Workload (the geometry of the rotating-ellipse benchmark, made viscous):
  * ellipse of axes 1 x 0.2 (isothermal no-slip wall) turning at omega in a
    disk r < 3 inside the far-field box [-30, 30]^2; Mach 0.2, Re 1000 on
    the major axis;
  * coarse mesh K x (n_in + n_out) cells at N = 3; the fine mesh splits every
    coarse cell 2 x 2 and runs at N = 6;
  * both start from the uniform free stream at t = 0 (impulsive start of
    the rotation) and step SSP-RK3 at CFL 0.1 of their own meshes.
"""
import time

import numpy as np

from .ssd import MLP, Mesh, pack_state, restrict, subgrid_nudge, subgrid_targets, unpack_state


def ellipse_pair(K=64, n_in=8, n_out=16, first_in=0.01, first_out=0.02):
    """Coarse mesh, its 2 x 2 refinement and the child table."""
    from workloads import meshes as M
    return M.ellipse_mesh(K=K, n_in=n_in, n_out=n_out, first_in=first_in, first_out=first_out,
                          wall=M.FACE_WALL_ISOTHERMAL, nested=True)


def cfl_dt(mesh, case, N, cfl=0.1):
    """Time step of an SD run: the smallest over cells of cfl h / (lam N^2),
    h the cell's shortest edge and lam = |u| + c + the grid speed at the
    cell's outermost corner (rotating cells), and the viscous bound
    cfl h^2 / (nu N^4)."""
    xy = np.asarray(mesh["xy"])[:, [0, 3, 6, 9]]
    h = np.linalg.norm(xy - np.roll(xy, 1, axis=1), axis=-1).min(axis=1)
    r = np.linalg.norm(xy - np.asarray(mesh["center"]), axis=-1).max(axis=1)
    rho, u, v, p = case["farfield"]
    rot = np.asarray(mesh["zone"]) == 1
    lam = np.hypot(u, v) + np.sqrt(case["gamma"] * p / rho) + np.where(rot, abs(case["omega"]) * r, 0)
    dt = cfl * np.min(h / lam) / (N * N)
    if case["mu"] > 0:
        dt = min(dt, cfl * h.min() ** 2 / (case["mu"] / rho * N ** 4))
    return float(dt)


class Pair:
    """Coarse and fine meshes of one rotation rate on the GPU."""

    def __init__(self, meshes, case, Nc=3, Nf=6, device=0):
        import torch
        coarse, fine, children = meshes
        self.case = case
        self.coarse = Mesh(coarse, case, Nc, device)
        self.fine = Mesh(fine, case, Nf, device)
        self.children = torch.tensor(np.ascontiguousarray(children, np.int32).ravel(),
                                     device=f"cuda:{device}")
        self.dt_c = cfl_dt(coarse, case, Nc)
        self.dt_f = cfl_dt(fine, case, Nf)
        self.Nc, self.Nf = Nc, Nf
        self.Ec = self.coarse.info["n_elem"]
        self.device = device

    def uniform(self, mesh):
        import torch
        N, E = mesh.info["N"], mesh.info["n_elem"]
        rho, u, v, p = self.case["farfield"]
        q = np.array([rho, rho * u, rho * v, p / (self.case["gamma"] - 1) + 0.5 * rho * (u * u + v * v)])
        Q = np.broadcast_to(q.astype(np.float32)[:, None, None, None], (4, N, N, E))
        return torch.tensor(pack_state(Q), device=f"cuda:{self.device}")

    def work(self, mesh):
        import torch
        return torch.empty(mesh.info["work_len"], dtype=torch.float32, device=f"cuda:{self.device}")

    def theta(self, t):
        return self.case.get("theta0", 0.0) + self.case["omega"] * t

    def restrict(self, qf):
        import torch
        qc = torch.empty(self.coarse.info["state_len"], dtype=torch.float32, device=qf.device)
        restrict(self.fine, self.coarse, self.children, qf, qc)
        return qc

    def sample(self, qf, t, X, T, qc=None, rate=0.0):
        """Features into X and targets into T (views of Ec rows each): at the
        restricted state (qc None), or at the coarse state qc (trajectory
        targets), with rate > 0 also the relaxation towards the restricted
        state."""
        import torch
        th, om = self.theta(t), self.case["omega"]
        rf = torch.empty_like(qf)
        self.fine.set_rotation(th, om)
        self.fine.mortar_rebuild()
        self.fine.residual(qf, rf)
        qr = self.restrict(qf)
        if qc is None:
            qc = qr
        rc = torch.empty_like(qc)
        self.coarse.set_rotation(th, om)
        self.coarse.mortar_rebuild()
        self.coarse.residual(qc, rc)
        subgrid_targets(self.fine, self.coarse, self.children, rf, rc, T)
        if rate:
            subgrid_nudge(self.coarse, qr, qc, rate, T)
        self.coarse.features(qc, X)


def advance(mesh, q, work, t, dt, t_end):
    """SSP-RK3 from t to t_end (the last step shortened to land on it)."""
    n = int(np.floor((t_end - t) / dt + 1e-9))
    if n > 0:
        mesh.rk_steps(q, work, t, dt, n)
        t += n * dt
    if t_end - t > 1e-12 * max(1.0, abs(t_end)):
        mesh.rk_steps(q, work, t, t_end - t, 1)
    return t_end


def convective_omega(omega, case_mach=0.2):
    """Rotation rate in the solver's unit (major axis / speed of sound) of a
    rate given in the free-stream convective unit (major axis / U)."""
    return omega * case_mach


def generate(meshes, omegas, t_start, t_end, n_snap, Nc=3, Nf=6, log=None):
    """Training rows from fine runs, one per rotation rate (solver units),
    stepped together as one batch with a common time step (the smallest of
    the runs): n_snap snapshots per run, equally spaced in [t_start, t_end].
    Returns (X, T) on the GPU and the seconds spent."""
    import torch
    from workloads import cases as C
    from .ssd import Batch
    Ec = len(meshes[0]["zone"])
    n_in, n_out = 4 * Nc * Nc + 16 * Nc, 4 * Nc * Nc
    rows = len(omegas) * n_snap * Ec
    X = torch.empty(rows * n_in, dtype=torch.float32, device="cuda:0")
    T = torch.empty(rows * n_out, dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    pairs = [Pair(meshes, C.ellipse_viscous_case(omega=om), Nc, Nf) for om in omegas]
    dt = min(P.dt_f for P in pairs)
    batch = Batch([P.fine for P in pairs])
    qs = [P.uniform(P.fine) for P in pairs]
    ws = [P.work(P.fine) for P in pairs]
    n = len(pairs)
    warm = int(round(t_start / dt))
    gap = max(1, int(round((t_end - t_start) / (max(n_snap - 1, 1) * dt))))
    if warm:
        batch.rk_steps(qs, ws, [0.0] * n, [dt] * n, warm)
    t = warm * dt
    k = 0
    for s in range(n_snap):
        if s:
            batch.rk_steps(qs, ws, [t] * n, [dt] * n, gap)
            t += gap * dt
        for P, q in zip(pairs, qs):
            P.sample(q, t, X[k * Ec * n_in:(k + 1) * Ec * n_in],
                     T[k * Ec * n_out:(k + 1) * Ec * n_out])
            k += 1
    for P in pairs:
        P.fine.check()
    torch.cuda.synchronize()
    if log:
        log(f"{n} fine runs to t = {t:.3f} (dt {dt:.3e}, {warm + (n_snap - 1) * gap} steps), "
            f"{n_snap} snapshots each, {time.perf_counter() - t0:.1f} s")
    batch.close()
    return X, T, time.perf_counter() - t0


def generate_trajectory(meshes, omegas, net, t_start, t_end, n_snap, rate=0.0, weight=1.0,
                        per_step=True, Nc=3, Nf=6, log=None, resync=0.0):
    """Training rows along corrected coarse runs (a posteriori training): the
    fine runs, one per rotation rate, stepped together as one batch as in
    `generate`, and beside each the coarse run with `net` attached, started
    from the restriction of the fine state at t_start.  At n_snap times
    equally spaced in [t_start, t_end]: the coarse run's features, with the
    targets restrict(R_f(Q_f)) - R_c(Q_c) + rate (restrict(Q_f) - Q_c), the
    correction that gives the coarse run the restricted fine dQ/dt at its
    own state (and, with rate > 0, pulls it back to the restricted fine
    state).  A coarse run that fails its check (ssd_check) restarts from
    the restricted fine state, and with resync > 0 every coarse run restarts
    from it each resync time units (the rows then come from coarse states no
    older than that).  Returns (X, T) on the GPU, the seconds spent and the
    number of restarts."""
    import torch
    from workloads import cases as C
    from .ssd import Batch, SSDError
    Ec = len(meshes[0]["zone"])
    n_in, n_out = 4 * Nc * Nc + 16 * Nc, 4 * Nc * Nc
    rows = len(omegas) * n_snap * Ec
    X = torch.empty(rows * n_in, dtype=torch.float32, device="cuda:0")
    T = torch.empty(rows * n_out, dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    pairs = [Pair(meshes, C.ellipse_viscous_case(omega=om), Nc, Nf) for om in omegas]
    dt = min(P.dt_f for P in pairs)
    batch = Batch([P.fine for P in pairs])
    qs = [P.uniform(P.fine) for P in pairs]
    ws = [P.work(P.fine) for P in pairs]
    n = len(pairs)
    warm = int(round(t_start / dt))
    gap = max(1, int(round((t_end - t_start) / (max(n_snap - 1, 1) * dt))))
    if warm:
        batch.rk_steps(qs, ws, [0.0] * n, [dt] * n, warm)
    t = warm * dt
    qcs = [P.restrict(q) for P, q in zip(pairs, qs)]
    wcs = [P.work(P.coarse) for P in pairs]
    k, restarts = 0, 0
    t_sync = t
    try:
        for P in pairs:
            P.coarse.attach(net, weight, per_step=per_step)
        for snap in range(n_snap):
            if snap:
                batch.rk_steps(qs, ws, [t] * n, [dt] * n, gap)
                for j, P in enumerate(pairs):
                    try:
                        advance(P.coarse, qcs[j], wcs[j], t, P.dt_c, t + gap * dt)
                        P.coarse.check()
                    except SSDError:
                        qcs[j] = P.restrict(qs[j])
                        restarts += 1
                t += gap * dt
                if resync > 0.0 and t - t_sync >= resync - 1e-12:
                    qcs = [P.restrict(q) for P, q in zip(pairs, qs)]
                    t_sync = t
            for j, P in enumerate(pairs):
                P.sample(qs[j], t, X[k * Ec * n_in:(k + 1) * Ec * n_in],
                         T[k * Ec * n_out:(k + 1) * Ec * n_out], qc=qcs[j], rate=rate)
                k += 1
    finally:
        for P in pairs:
            P.coarse.attach(None)
    for P in pairs:
        P.fine.check()
    torch.cuda.synchronize()
    batch.close()
    if log:
        log(f"{n} corrected coarse runs beside their fine runs to t = {t:.3f}, {n_snap} snapshots "
            f"each, {restarts} restarts, {time.perf_counter() - t0:.1f} s")
    return X, T, time.perf_counter() - t0, restarts


def init_params(rng, n_in, n_out, H=MLP.HIDDEN):
    """Glorot-uniform weights and zero biases, drawn from rng."""
    def glorot(o, i):
        a = np.sqrt(6.0 / (i + o))
        return rng.uniform(-a, a, size=(o, i)).astype(np.float32)
    return dict(W1=glorot(H, n_in), b1=np.zeros(H, np.float32), W2=glorot(H, H),
                b2=np.zeros(H, np.float32), W3=glorot(n_out, H), b3=np.zeros(n_out, np.float32))


def zero_at_free_stream(net, pair):
    """Shift the network's output bias so that its correction of the
    uniform free stream of pair's case is zero.  A uniform flow has no
    subgrid scales (both meshes preserve it), so the corrected scheme then
    keeps it too; otherwise the fit's small offset there acts as a source in
    every far-field cell.  Every element of a uniform state has the same
    features; the output scale of each component is measured as the
    response to a unit change of its bias.  Resets the Adam moments (as
    set_params does).  Returns the correction of the free stream before the
    shift."""
    import torch
    q = pair.uniform(pair.coarse)
    X = torch.empty(pair.Ec * net.n_in, dtype=torch.float32, device=q.device)
    pair.coarse.features(q, X)
    x = X[:net.n_in].clone()
    y = torch.empty(net.n_out, dtype=torch.float32, device=q.device)
    p = net.get_params()
    net.forward(x, y)
    y0 = y.cpu().numpy().astype(np.float64)
    bumped = dict(p, b3=(p["b3"] + 1.0).astype(np.float32))
    net.set_params(bumped)
    net.forward(x, y)
    scale = y.cpu().numpy().astype(np.float64) - y0
    p["b3"] = (p["b3"] - y0 / scale).astype(np.float32)
    net.set_params(p)
    return y0


def train(net, X, T, epochs, batch, lr, seed, log=None, min_rel=1e-2, noise=0.0, resume=False):
    """Adam over shuffled minibatches with input noise of standard deviation
    `noise` (normalised units); the learning rate decays as a cosine to a
    tenth.  resume: continue from the network's weights and normalisation
    (new Adam moments) instead of fresh weights.  Returns the per-epoch mean
    losses and the seconds spent."""
    import torch
    rows = X.numel() // net.n_in
    rng = np.random.default_rng(seed)
    if resume:
        net.set_params(net.get_params())      # same weights, fresh Adam moments
    else:
        net.set_params(init_params(rng, net.n_in, net.n_out))
        net.fit_normalization(X, T, min_rel=min_rel)
    per = rows // batch
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(rows)[:per * batch].astype(np.int32), device="cuda:0")
        a = lr * (0.55 + 0.45 * np.cos(np.pi * ep / max(epochs - 1, 1)))
        for b in range(per):
            net.train_step(X, T, perm[b * batch:(b + 1) * batch], a, noise, seed)
        losses.append(net.loss()[0])
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e} lr {a:.2e}")
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def evaluate(meshes, net, omega, t0, t1, Nc=3, Nf=6, fine_orders=(5, 4, 3), coarse_orders=(4,),
             weights=(1.0,), chunks=10, per_step=True):
    """Plain SSD runs and the corrected coarse run over [t0, t1], all from the
    state at t0 of a fine run (N = Nf) from the free stream at t = 0.

    Runs (each timed over [t0, t1], GPU synchronised):
      * the fine mesh at N = Nf: the reference;
      * the fine mesh at each N in fine_orders, from the projection of the
        fine state onto that order;
      * the coarse mesh at N = Nc, plain, from the restriction of the fine
        state, and at each N in coarse_orders (higher orders on the coarse
        mesh, the other plain way to buy accuracy);
      * the coarse mesh with the network attached, once per weight, its
        correction evaluated once per step (per_step) or in every stage;
        checked after each of `chunks` parts of the interval, and if it
        fails the plain coarse run stands in (fallback) and the failure time
        is kept.
    Error of a run: its state restricted to the coarse mesh at N = Nc minus
    the restricted reference, in L2 over all variables, relative to the
    restricted reference's departure from the free stream."""
    import torch
    from workloads import cases as C
    from .ssd import SSDError
    case = C.ellipse_viscous_case(omega=omega)
    P = Pair(meshes, case, Nc, Nf)
    qf, wf = P.uniform(P.fine), P.work(P.fine)
    advance(P.fine, qf, wf, 0.0, P.dt_f, t0)
    q_start = qf.clone()
    qc0 = P.restrict(qf)

    def timed(fn):
        torch.cuda.synchronize()
        s = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - s

    runs = []
    s_ref = timed(lambda: advance(P.fine, qf, wf, t0, P.dt_f, t1))
    P.fine.check()
    Nc, Ec = P.Nc, P.Ec
    ref = unpack_state(P.restrict(qf).cpu().numpy(), Nc, Ec).astype(np.float64).reshape(4, -1)
    dev = np.sum((ref - uniform_ref(P)) ** 2)

    def err(qc):
        q = unpack_state(qc.cpu().numpy(), Nc, Ec).astype(np.float64).reshape(4, -1)
        return float(np.sqrt(np.sum((q - ref) ** 2) / dev))

    runs.append(dict(run=f"fine mesh N={Nf} (reference)", s=s_ref, err=0.0, dt=P.dt_f,
                     dof=P.fine.info["state_len"]))
    fine_mesh = meshes[1]
    for k in fine_orders:
        m = Mesh(fine_mesh, case, k, P.device)
        q = torch.empty(m.info["state_len"], dtype=torch.float32, device=qf.device)
        restrict(P.fine, m, None, q_start, q)
        w = P.work(m)
        dt = cfl_dt(fine_mesh, case, k)
        s = timed(lambda: advance(m, q, w, t0, dt, t1))
        m.check()
        qc = torch.empty(P.coarse.info["state_len"], dtype=torch.float32, device=qf.device)
        restrict(m, P.coarse, P.children, q, qc)
        runs.append(dict(run=f"fine mesh N={k}", s=s, err=err(qc), dt=dt,
                         dof=m.info["state_len"]))
        m.close()
    coarse_mesh = meshes[0]
    for k in coarse_orders:
        m = Mesh(coarse_mesh, case, k, P.device)
        q = torch.empty(m.info["state_len"], dtype=torch.float32, device=qf.device)
        restrict(P.fine, m, P.children, q_start, q)
        w = P.work(m)
        dt = cfl_dt(coarse_mesh, case, k)
        s = timed(lambda: advance(m, q, w, t0, dt, t1))
        m.check()
        qc = torch.empty(P.coarse.info["state_len"], dtype=torch.float32, device=qf.device)
        restrict(m, P.coarse, None, q, qc)
        runs.append(dict(run=f"coarse mesh N={k}", s=s, err=err(qc), dt=dt,
                         dof=m.info["state_len"]))
        m.close()
    wc = P.work(P.coarse)
    edges = np.linspace(t0, t1, chunks + 1)

    def coarse_run(net_w):
        q = qc0.clone()
        if net_w:
            P.coarse.attach(*net_w, per_step=per_step)
        spent, t = 0.0, t0
        try:
            for te in edges[1:]:
                spent += timed(lambda: advance(P.coarse, q, wc, t, P.dt_c, te))
                t = te
                P.coarse.check()
        except SSDError:
            return None, spent, t
        finally:
            P.coarse.attach(None)
        return q, spent, None

    qp, s_plain, _ = coarse_run(None)
    plain = dict(run=f"coarse mesh N={Nc}", s=s_plain, err=err(qp), dt=P.dt_c,
                 dof=P.coarse.info["state_len"])
    runs.append(plain)
    learned = []
    for wgt in weights:
        ql, s, failed = coarse_run((net, wgt))
        r = dict(run=f"coarse mesh N={Nc} + learned correction (weight {wgt})", s=s,
                 dt=P.dt_c, dof=P.coarse.info["state_len"], weight=wgt)
        if ql is None:
            r.update(err=plain["err"], fallback=True, failed_at=failed)
        else:
            r.update(err=err(ql), fallback=False)
        learned.append(r)
    return dict(omega=omega, t0=t0, t1=t1, plain=runs, learned=learned)


def speedup_at_equal_error(result):
    """For each corrected run: the cheapest plain run whose error is at most
    the corrected run's, and its time over the corrected run's (`speedup`);
    and the time of a plain run of exactly that error on the plain runs'
    cost-error front, interpolated log-linearly between the two neighbouring
    plain runs, over the corrected run's time (`speedup_interpolated`)."""
    out = []
    plain = sorted(result["plain"], key=lambda p: p["s"])
    for r in result["learned"]:
        ok = [p for p in plain if p["err"] <= r["err"]]
        best = min(ok, key=lambda p: p["s"])
        interp = None
        for a, b in zip(plain, plain[1:]):
            if a["err"] >= r["err"] >= b["err"] > 0.0:
                f = np.log(a["err"] / r["err"]) / np.log(a["err"] / b["err"])
                interp = float(np.exp(np.log(a["s"]) + f * np.log(b["s"] / a["s"]))) / r["s"]
        out.append(dict(weight=r["weight"], err=r["err"], plain_run=best["run"],
                        plain_err=best["err"], speedup=best["s"] / r["s"],
                        speedup_interpolated=interp))
    return out


def uniform_ref(P):
    """The free-stream state per variable as a column (4, 1)."""
    rho, u, v, p = P.case["farfield"]
    g = P.case["gamma"]
    return np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])[:, None]
