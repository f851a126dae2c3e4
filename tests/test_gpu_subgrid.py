"""Learned subgrid correction on the GPU (features, restriction, targets, the
BF16-MFMA network and its training step, and SSP-RK3 with the correction
attached) against the FP64 oracle (oracle/subgrid.py) on the same seeded
inputs, through the C ABI.

Tolerances:
  features, restriction   FP32 sums of at most 4 N^2 products of O(1)
                          values: 1e-5 of the largest magnitude;
  targets                 differences of two residuals: 1e-5 of the
                          residuals' largest magnitude (the residual bar);
  network                 the oracle rounds the same operands to bfloat16
                          and sums in FP64, the kernels sum in FP32.  Where
                          an FP32 pre-activation lies within its rounding of
                          a bfloat16 rounding boundary, the two round one
                          activation to neighbouring bfloat16 values (one
                          unit, 2^-8 relative): rare, and a few such events
                          move an output by far less than 1e-2 of the
                          largest output.  So the bound is 1e-2 on the
                          largest deviation and 1e-5 on the median one.

Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

from oracle import subgrid as S
from oracle.ssd import SSD
from tests.parity_utils import TOL, from_gpu, state_error, to_gpu
from workloads import cases as C
from workloads import meshes as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def nested():
    coarse, fine, ch = M.ellipse_mesh(K=16, n_in=4, n_out=4, radius=1.5, box_half=4.0,
                                      first_in=0.05, first_out=0.1,
                                      wall=M.FACE_WALL_ISOTHERMAL, nested=True)
    return coarse, fine, ch


def _smooth_state(ssd, case, theta=0.0):
    x, y = ssd.sp_coords(theta)
    g = case["gamma"]
    rho = 1.0 + 0.05 * np.sin(0.9 * x) * np.cos(0.7 * y)
    u = case["farfield"][1] + 0.03 * np.sin(0.8 * y + 0.2)
    v = 0.03 * np.cos(0.6 * x - 0.1)
    p = case["farfield"][3] * (1.0 + 0.04 * np.cos(0.5 * x + 0.4 * y))
    return np.stack([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


def _close(a, b, rel, what):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    print(what, "max error relative to the largest value", err, flush=True)
    assert err <= rel, (what, err)


def _net(rng, N, scale=0.25):
    nin, nout, H = 4 * N * N + 16 * N, 4 * N * N, 64
    p = dict(W1=rng.normal(size=(H, nin)) * scale / np.sqrt(nin) * 4,
             b1=rng.normal(size=H) * 0.1,
             W2=rng.normal(size=(H, H)) * scale / np.sqrt(H) * 4,
             b2=rng.normal(size=H) * 0.1,
             W3=rng.normal(size=(nout, H)) * scale / np.sqrt(H) * 4,
             b3=rng.normal(size=nout) * 0.1)
    p = {k: v.astype(np.float32) for k, v in p.items()}
    norm = dict(mu_x=rng.normal(size=nin).astype(np.float32),
                sig_x=rng.uniform(0.5, 2.0, nin).astype(np.float32),
                mu_y=rng.normal(size=nout).astype(np.float32),
                sig_y=rng.uniform(0.5, 2.0, nout).astype(np.float32))
    return p, norm


def _gpu_net(N, p, norm):
    from paper_1503_02198_amd import MLP
    net = MLP(N)
    net.set_params(p)
    net.set_normalization(norm["mu_x"], norm["sig_x"], norm["mu_y"], norm["sig_y"])
    return net


def _oracle_net(p, norm):
    return S.MLP(p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"], **norm)


def _net_close(y_gpu, y_ora, what):
    d = np.abs(np.asarray(y_gpu, np.float64) - y_ora)
    top = np.abs(y_ora).max()
    print(what, "largest and median deviation relative to the largest value",
          d.max() / top, np.median(d) / top, flush=True)
    assert d.max() <= 1e-2 * top and np.median(d) <= 1e-5 * top, what


# ---------------------------------------------------------------------------
def test_features(torch_cuda, nested):
    from paper_1503_02198_amd import Mesh
    print("case: features, coarse ellipse N=3 and relabelled box N=2", flush=True)
    coarse = nested[0]
    box = M.box_mesh(6, 5, L=(2.0, 1.5), distort=0.1, zone=0)
    box = M.relabel(box, np.random.default_rng(2).integers(0, 4, len(box["zone"])))
    for mesh, case, N in ((coarse, C.ellipse_viscous_case(), 3), (box, C.vortex_case(), 2)):
        ora = SSD(mesh, case, N)
        Q = _smooth_state(ora, case) * (1 + 0.01 * np.random.default_rng(N).normal(
            size=(4, N, N, ora.E)))
        gm = Mesh(mesh, case, N)
        X = torch_cuda.empty(ora.E * S.n_features(N), dtype=torch_cuda.float32, device="cuda:0")
        gm.features(to_gpu(Q), X)
        Xg = X.cpu().numpy().reshape(ora.E, -1)
        _close(Xg, S.features(ora, Q), 1e-6, f"features N={N}")


@pytest.mark.parametrize("Nc,Nf,split", [(3, 6, True), (2, 4, True), (3, 5, True), (4, 6, True),
                                         (3, 6, False), (5, 6, False), (2, 3, False),
                                         (3, 4, False)])
def test_restrict(torch_cuda, nested, Nc, Nf, split):
    """Nested fine mesh to the coarse one, or one mesh to a lower order."""
    from paper_1503_02198_amd import Mesh, restrict
    print(f"case: restriction N {Nf} -> {Nc}, nested {split}", flush=True)
    coarse, fine, ch = nested
    case = C.ellipse_viscous_case()
    of = SSD(fine, case, Nf)
    Qf = _smooth_state(of, case) * (1 + 0.01 * np.random.default_rng(1).normal(
        size=(4, Nf, Nf, of.E)))
    gf = Mesh(fine, case, Nf)
    gc = Mesh(coarse if split else fine, case, Nc)
    qc = torch_cuda.empty(gc.info["state_len"], dtype=torch_cuda.float32, device="cuda:0")
    chd = torch_cuda.tensor(ch.ravel(), device="cuda:0") if split else None
    restrict(gf, gc, chd, to_gpu(Qf), qc)
    want = S.restrict(Qf, ch if split else None, Nc)
    _close(from_gpu(qc, Nc, gc.info["n_elem"]), want, 1e-6, "restriction")


def test_targets(torch_cuda, nested):
    """Restricted fine dQ/dt minus the coarse residual of the restricted
    state, on the viscous ellipse pair (isothermal wall, sliding interface)."""
    from paper_1503_02198_amd import Mesh, restrict, subgrid_targets
    from tests.parity_utils import gpu_residual
    print("case: targets, viscous ellipse N 6 -> 3", flush=True)
    coarse, fine, ch = nested
    case = C.ellipse_viscous_case(omega=1.3)
    of, oc = SSD(fine, case, 6), SSD(coarse, case, 3)
    theta = 0.3
    Qf = _smooth_state(of, case, theta)
    T_ora, Qc_ora = S.targets(of, oc, ch, Qf, theta, case["omega"])
    gf, gc = Mesh(fine, case, 6), Mesh(coarse, case, 3)
    chd = torch_cuda.tensor(ch.ravel(), device="cuda:0")
    Rf = to_gpu(gpu_residual(gf, Qf, theta, case["omega"]))
    qc = torch_cuda.empty(gc.info["state_len"], dtype=torch_cuda.float32, device="cuda:0")
    restrict(gf, gc, chd, to_gpu(Qf), qc)
    Rc = to_gpu(gpu_residual(gc, from_gpu(qc, 3, gc.info["n_elem"]), theta, case["omega"]))
    T = torch_cuda.empty_like(qc)
    subgrid_targets(gf, gc, chd, Rf, Rc, T)
    Tg = T.cpu().numpy().reshape(gc.info["n_elem"], -1)
    scale = np.abs(S.restrict(of.residual(Qf, theta, case["omega"]), ch, 3)).max()
    err = np.abs(Tg - T_ora).max() / scale
    print("target error relative to the restricted residual", err, flush=True)
    assert err <= 1e-5


def test_trajectory_targets(torch_cuda, nested):
    """Targets at a coarse state off the restricted fine state (a corrected
    run's state): restricted fine dQ/dt minus the coarse residual at that
    state plus the relaxation rate (restrict(Qf) - Qc), against the oracle."""
    from paper_1503_02198_amd import Mesh, restrict, subgrid_nudge, subgrid_targets
    from tests.parity_utils import gpu_residual
    print("case: trajectory targets, viscous ellipse N 6 -> 3", flush=True)
    coarse, fine, ch = nested
    case = C.ellipse_viscous_case(omega=0.9)
    of, oc = SSD(fine, case, 6), SSD(coarse, case, 3)
    theta, rate = 0.21, 40.0
    Qf = _smooth_state(of, case, theta)
    Qr = S.restrict(Qf, ch, 3)
    # a coarse state that differs from the restricted one by a smooth field
    x, y = oc.sp_coords(theta)
    Qc = Qr * (1.0 + 0.01 * np.sin(0.7 * x + 0.3 * y)[None])
    T_ora = S.trajectory_targets(of, oc, ch, Qf, Qc, theta, case["omega"], rate)
    gf, gc = Mesh(fine, case, 6), Mesh(coarse, case, 3)
    chd = torch_cuda.tensor(ch.ravel(), device="cuda:0")
    Rf = to_gpu(gpu_residual(gf, Qf, theta, case["omega"]))
    qr = torch_cuda.empty(gc.info["state_len"], dtype=torch_cuda.float32, device="cuda:0")
    restrict(gf, gc, chd, to_gpu(Qf), qr)
    qc = to_gpu(Qc)
    Rc = to_gpu(gpu_residual(gc, Qc, theta, case["omega"]))
    T = torch_cuda.empty_like(qc)
    subgrid_targets(gf, gc, chd, Rf, Rc, T)
    subgrid_nudge(gc, qr, qc, rate, T)
    Tg = T.cpu().numpy().reshape(gc.info["n_elem"], -1)
    scale = np.abs(S.restrict(of.residual(Qf, theta, case["omega"]), ch, 3)).max()
    relax = rate * np.abs(Qr - Qc).max()
    err = np.abs(Tg - T_ora).max() / scale
    print("target error relative to the restricted residual", err, "relaxation term", relax,
          "residual scale", scale, flush=True)
    # the relaxation term is far above the tolerance: leaving it out fails
    assert relax > 100 * 1e-5 * scale
    assert err <= 1e-5


@pytest.mark.parametrize("N,n", [(3, 200), (2, 64), (4, 77)])
def test_mlp_forward(torch_cuda, N, n):
    print(f"case: network forward N={N} rows={n}", flush=True)
    rng = np.random.default_rng(10 + N)
    p, norm = _net(rng, N)
    net = _gpu_net(N, p, norm)
    X = rng.normal(size=(n, net.n_in)) * 1.5 + norm["mu_x"]
    Y = torch_cuda.empty(n * net.n_out, dtype=torch_cuda.float32, device="cuda:0")
    net.forward(torch_cuda.tensor(X.astype(np.float32), device="cuda:0").reshape(-1), Y)
    y_ora = _oracle_net(p, norm).predict(X.astype(np.float32), bf=True)
    _net_close(Y.cpu().numpy().reshape(n, -1), y_ora, "forward")
    got = net.get_params()
    assert all(np.array_equal(got[k], p[k]) for k in p)


@pytest.mark.parametrize("N,batch", [(3, 200), (2, 64)])
def test_mlp_gradient(torch_cuda, N, batch):
    print(f"case: network gradient N={N} batch={batch}", flush=True)
    rng = np.random.default_rng(20 + N)
    p, norm = _net(rng, N)
    net = _gpu_net(N, p, norm)
    n = 300
    X = (rng.normal(size=(n, net.n_in)) * 1.5 + norm["mu_x"]).astype(np.float32)
    T = (rng.normal(size=(n, net.n_out)) + norm["mu_y"]).astype(np.float32)
    idx = rng.integers(0, n, batch).astype(np.int32)
    Xd = torch_cuda.tensor(X, device="cuda:0").reshape(-1)
    Td = torch_cuda.tensor(T, device="cuda:0").reshape(-1)
    loss, G = net.gradient(Xd, Td, torch_cuda.tensor(idx, device="cuda:0"))
    L_ora, G_ora = _oracle_net(p, norm).loss_grads(X[idx], T[idx], bf=True)
    print("loss", loss, L_ora, flush=True)
    assert abs(loss - L_ora) <= 1e-5 * abs(L_ora)
    for k in G_ora:
        rel = np.linalg.norm(G[k] - G_ora[k]) / np.linalg.norm(G_ora[k])
        print("gradient", k, "relative error", rel, flush=True)
        assert rel <= 2e-3, k
    # with input noise (step 1 after the parameters were set)
    loss_n, G_n = net.gradient(Xd, Td, torch_cuda.tensor(idx, device="cuda:0"), noise=0.3,
                               seed=99)
    nz = S.training_noise(99, 1, batch, net.n_in, 0.3)
    L_n, G_no = _oracle_net(p, norm).loss_grads(X[idx], T[idx], bf=True, noise=nz)
    print("loss with noise", loss_n, L_n, flush=True)
    assert abs(loss_n - L_n) <= 1e-5 * abs(L_n) and abs(L_n - L_ora) > 1e-3 * L_ora
    for k in G_no:
        assert np.linalg.norm(G_n[k] - G_no[k]) <= 2e-3 * np.linalg.norm(G_no[k]), k
    # an index outside the rows contributes nothing; the mean is still
    # taken over the whole minibatch
    bad = idx.copy()
    bad[::7] = -1
    bad[3] = n + 5
    keep = (bad >= 0) & (bad < n)
    loss_b, G_b = net.gradient(Xd, Td, torch_cuda.tensor(bad, device="cuda:0"))
    # the oracle on the same minibatch, a skipped row given the network's own
    # output as its target (so it adds nothing, and the mean keeps its size)
    ora = _oracle_net(p, norm)
    Xm = X[np.where(keep, bad, 0)]
    Tm = np.where(keep[:, None], T[np.where(keep, bad, 0)], ora.predict(Xm, bf=True))
    L_m, G_m = ora.loss_grads(Xm, Tm, bf=True)
    assert abs(loss_b - L_m) <= 1e-5 * abs(L_m)
    for k in G_m:
        assert np.linalg.norm(G_b[k] - G_m[k]) <= 2e-3 * np.linalg.norm(G_m[k]), k


def test_mlp_adam_and_training(torch_cuda):
    """The first Adam step moves every parameter by lr against the sign of
    its gradient; a few hundred steps fit a teacher network."""
    import torch
    print("case: network training N=3", flush=True)
    rng = np.random.default_rng(31)
    N = 3
    p, norm = _net(rng, N)
    net = _gpu_net(N, p, norm)
    n = 4096
    X = (rng.normal(size=(n, net.n_in)) * 1.5 + norm["mu_x"]).astype(np.float32)
    teacher, _ = _net(np.random.default_rng(32), N, scale=0.4)
    T = _oracle_net(teacher, norm).predict(X).astype(np.float32)
    Xd = torch.tensor(X, device="cuda:0").reshape(-1)
    Td = torch.tensor(T, device="cuda:0").reshape(-1)
    idx = torch.tensor(rng.integers(0, n, 256).astype(np.int32), device="cuda:0")
    _, G = _oracle_net(p, norm).loss_grads(X[idx.cpu().numpy()], T[idx.cpu().numpy()], bf=True)
    lr = 1e-3
    net.train_step(Xd, Td, idx, lr)
    q = net.get_params()
    for k in p:
        g = G[k]
        big = np.abs(g) > 1e-3 * np.abs(g).max()
        step = (q[k] - p[k])[big]
        assert np.allclose(step, -lr * np.sign(g[big]), rtol=1e-3, atol=1e-7), k
    # fit the normalisation to the data and train
    net.set_params(p)
    net.fit_normalization(Xd, Td)
    first = None
    for it in range(400):
        idx = torch.tensor(rng.integers(0, n, 256).astype(np.int32), device="cuda:0")
        net.train_step(Xd, Td, idx, 3e-3)
        if it == 19:
            first, _ = net.loss()
    last, steps = net.loss()
    print("training loss", first, "->", last, "over", steps, "steps", flush=True)
    assert steps == 380 and last < 0.5 * first


def test_attached_correction_rk3(torch_cuda, nested):
    """SSP-RK3 of dQ/dt = R(Q) + C(Q) on the coarse viscous ellipse mesh,
    and plain SSD again once the network is detached."""
    import torch
    from paper_1503_02198_amd import Mesh
    print("case: SSP-RK3 with the learned correction, coarse ellipse N=3", flush=True)
    coarse = nested[0]
    case = C.ellipse_viscous_case(omega=0.8)
    N = 3
    ora = SSD(coarse, case, N)
    Q = _smooth_state(ora, case)
    F = S.features(ora, Q)
    rng = np.random.default_rng(41)
    p, _ = _net(rng, N)
    sd = F.std(0)
    norm = dict(mu_x=F.mean(0).astype(np.float32),
                sig_x=np.where(sd > 1e-6, sd, 1.0).astype(np.float32),
                mu_y=np.zeros(4 * N * N, np.float32), sig_y=np.full(4 * N * N, 0.05, np.float32))
    net = _gpu_net(N, p, norm)
    gm = Mesh(coarse, case, N)
    gm.attach(net)
    dt, steps = 2e-3, 4
    q = to_gpu(Q)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0")
    gm.rk_steps(q, work, 0.0, dt, steps)
    gm.check()
    Qg = from_gpu(q, N, ora.E)
    Qo = S.corrected_rk3(ora, _oracle_net(p, norm), Q, 0.0, dt, steps, bf=True)
    Qp = ora.run(Q, 0.0, dt, steps)
    err = state_error(Qg, Qo)
    print("state error", err, "; the correction moved the state by",
          state_error(Qo, Qp), flush=True)
    assert np.all(err <= TOL)
    assert np.all(state_error(Qo, Qp) > 100 * err)
    with pytest.raises(Exception):
        gm.rk_steps(q, work, 0.0, dt, 1, scheme="rk54")
    # the correction of Q^n held for the step's three stages
    gm.attach(net, per_step=True)
    q = to_gpu(Q)
    gm.rk_steps(q, work, 0.0, dt, steps)
    gm.check()
    Qs = S.corrected_rk3(ora, _oracle_net(p, norm), Q, 0.0, dt, steps, bf=True, per_step=True)
    err_s = state_error(from_gpu(q, N, ora.E), Qs)
    print("per-step state error", err_s, "; per-step vs per-stage", state_error(Qs, Qo), flush=True)
    assert np.all(err_s <= TOL)
    assert np.all(state_error(Qs, Qo) > 10 * err_s)
    # detached: plain SSD, bitwise equal to a mesh that never had a network
    gm.attach(None)
    q1, q2 = to_gpu(Q), to_gpu(Q)
    gm.rk_steps(q1, work, 0.0, dt, 2)
    plain = Mesh(coarse, case, N)
    plain.rk_steps(q2, work, 0.0, dt, 2)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)


def test_trained_network_reduces_coarse_error(torch_cuda):
    """End to end on a small viscous ellipse pair: fine runs (N=6) at two
    seeded rates give the training rows, the network is trained on the GPU,
    and at a third rate the corrected coarse run (N=3) ends closer to the
    fine run than the plain coarse run over a short interval."""
    from paper_1503_02198_amd import MLP
    from paper_1503_02198_amd import subgrid as G
    print("case: trained correction vs plain coarse, K=32 ellipse pair", flush=True)
    meshes = G.ellipse_pair(32, 4, 8, first_in=0.02, first_out=0.04)
    rates = G.convective_omega(np.array([0.8, 1.6]))
    X, T, _ = G.generate(meshes, rates, 0.3, 0.5, 100)
    net = MLP(3)
    losses, _ = G.train(net, X, T, 30, 1024, 2e-3, seed=7, noise=0.1)
    print("training loss", losses[0], "->", losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    res = G.evaluate(meshes, net, G.convective_omega(1.2), 0.3, 0.31, fine_orders=(),
                     coarse_orders=())
    plain = [r for r in res["plain"] if r["run"] == "coarse mesh N=3"][0]
    learned = res["learned"][0]
    print("coarse error plain", plain["err"], "corrected", learned["err"], flush=True)
    assert not learned["fallback"]
    assert learned["err"] < 0.8 * plain["err"]


def test_zero_at_free_stream(torch_cuda, nested):
    """zero_at_free_stream shifts the output bias so that the correction of
    the uniform free stream vanishes: the network's output there drops from
    O(1) to rounding, and an SSP-RK3 step from the free stream with the
    correction taken at the step's start then equals the plain step (later
    steps see the sliding interface's small free-stream error, to which the
    network responds)."""
    import torch
    from paper_1503_02198_amd import subgrid as G
    print("case: free-stream calibration of the correction, coarse ellipse N=3", flush=True)
    case = C.ellipse_viscous_case(omega=0.8)
    P = G.Pair(nested, case, 3, 6)
    p, norm = _net(np.random.default_rng(43), 3)
    norm["sig_y"] = np.full(36, 0.05, np.float32)
    norm["mu_y"] = np.full(36, 0.01, np.float32)
    net = _gpu_net(3, p, norm)
    q = P.uniform(P.coarse)
    X = torch.empty(P.Ec * net.n_in, dtype=torch.float32, device="cuda:0")
    P.coarse.features(q, X)
    y = torch.empty(net.n_out, dtype=torch.float32, device="cuda:0")
    w = P.work(P.coarse)

    def step_gap():
        qa, qb = q.clone(), q.clone()
        P.coarse.attach(net, per_step=True)
        P.coarse.rk_steps(qa, w, 0.0, 1e-3, 1)
        P.coarse.attach(None)
        P.coarse.rk_steps(qb, w, 0.0, 1e-3, 1)
        return float((qa - qb).abs().max())

    before = step_gap()
    y0 = G.zero_at_free_stream(net, P)
    net.forward(X[:net.n_in].clone(), y)
    after_y = float(y.abs().max())
    after = step_gap()
    print("free-stream correction", np.abs(y0).max(), "->", after_y,
          "; corrected minus plain after one step", before, "->", after, flush=True)
    assert np.abs(y0).max() > 1e-3
    assert after_y <= 1e-4 * np.abs(y0).max()
    assert after <= 1e-3 * before
