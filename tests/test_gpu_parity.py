"""HIP path vs the FP64 oracle on identical seeded inputs (through the C ABI).

Every case prints its name before touching the GPU so a failure names it.
"""
import numpy as np
import pytest

from oracle.exact import vortex_state
from oracle.ssd import SSD
from tests.parity_utils import (ELEM_TOL, TOL, change_error, element_max_error, gpu_residual,
                                gpu_run, interface_cells, residual_error, state_error, to_gpu)
from workloads import cases as C
from workloads import meshes as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mesh(mesh, case, N):
    from paper_1503_02198_amd import Mesh
    return Mesh(mesh, case, N, device=0)


def _vortex(N=3, f=1, omega=0.5, theta0=0.0):
    case = C.vortex_case(omega=omega, theta0=theta0)
    mesh = M.vortex_mesh(f)
    ora = SSD(mesh, case, N)
    x, y = ora.sp_coords(theta0)
    return mesh, case, ora, vortex_state(x, y, 0.0, case)


@pytest.mark.parametrize("theta", [0.0, 0.05, 0.1963495408, -0.4, 2.0])
def test_residual_vortex(torch_cuda, theta):
    print(f"case: vortex residual N=3 theta={theta}", flush=True)
    mesh, case, ora, Q = _vortex()
    gm = _mesh(mesh, case, 3)
    Rg = gpu_residual(gm, Q, theta, case["omega"])
    Ro, diag = ora.residual(Q, theta, case["omega"], diag=True)
    err = residual_error(Rg, Ro, diag["flux_scale"])
    emax = element_max_error(Rg, Ro, diag["flux_scale"], interface_cells(mesh))
    print("residual error", err, "interface cells, element maximum", emax)
    assert np.all(err <= TOL), err
    assert np.all(emax <= ELEM_TOL), emax


@pytest.mark.parametrize("N", [2, 4, 5, 6])
def test_residual_vortex_sliding_all_orders(torch_cuda, N):
    """The inviscid sliding mortar at every other order, at a zero offset,
    a mid-face offset and just below a whole face width; the interface
    cells are compared element by element."""
    mesh, case, ora, Q = _vortex(N=N)
    gm = _mesh(mesh, case, N)
    sl = interface_cells(mesh)
    for theta in (0.0, 0.083, 2 * np.pi / 32 - 1e-3):
        print(f"case: vortex residual N={N} theta={theta}", flush=True)
        Rg = gpu_residual(gm, Q, theta, case["omega"])
        Ro, diag = ora.residual(Q, theta, case["omega"], diag=True)
        err = residual_error(Rg, Ro, diag["flux_scale"])
        emax = element_max_error(Rg, Ro, diag["flux_scale"], sl)
        eall = element_max_error(Rg, Ro, diag["flux_scale"])
        print("residual error", err, "interface element maximum", emax, "all cells", eall)
        assert np.all(err <= TOL), err
        assert np.all(emax <= ELEM_TOL) and np.all(eall <= ELEM_TOL), (emax, eall)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("curved", [False, True])
def test_residual_box_all_orders(torch_cuda, N, curved):
    print(f"case: box residual N={N} curved={curved}", flush=True)
    case = C.vortex_case()
    mesh = M.box_mesh(7, 5, L=(3.0, 2.0), distort=0.15, curved=0.06 if curved else 0.0, zone=1)
    ora = SSD(mesh, case, N)
    x, y = ora.sp_coords(0.0)
    case["vortex"]["period"] = 100.0
    case["vortex"]["center"] = (1.5, 1.0)
    Q = vortex_state(x, y, 0.0, case)
    gm = _mesh(mesh, case, N)
    Rg = gpu_residual(gm, Q, 0.3, 0.8)
    Ro, diag = ora.residual(Q, 0.3, 0.8, diag=True)
    err = residual_error(Rg, Ro, diag["flux_scale"])
    print("residual error", err)
    assert np.all(err <= TOL), err


@pytest.mark.parametrize("N", [3, 4])
def test_residual_relabelled_sliding_mesh(torch_cuda, N):
    """Random corner relabelling flips face parameters on the interface."""
    print(f"case: relabelled vortex residual N={N}", flush=True)
    case = C.vortex_case(omega=0.5)
    mesh = M.relabel(M.vortex_mesh(1), np.random.default_rng(11).integers(0, 4, 384))
    ora = SSD(mesh, case, N)
    x, y = ora.sp_coords(0.0)
    Q = vortex_state(x, y, 0.0, case)
    gm = _mesh(mesh, case, N)
    for th in (0.0, 0.137):
        Rg = gpu_residual(gm, Q, th, 0.5)
        Ro, diag = ora.residual(Q, th, 0.5, diag=True)
        err = residual_error(Rg, Ro, diag["flux_scale"])
        emax = element_max_error(Rg, Ro, diag["flux_scale"], interface_cells(mesh))
        print("theta", th, "residual error", err, "interface element maximum", emax)
        assert np.all(err <= TOL), err
        assert np.all(emax <= ELEM_TOL), emax


def test_rk3_vortex_100_steps(torch_cuda):
    """The vortex workload: 384 cells, N=3, SSP-RK3, dt = 1e-3, 100 steps."""
    print("case: vortex SSP-RK3 100 steps", flush=True)
    mesh, case, ora, Q = _vortex()
    gm = _mesh(mesh, case, 3)
    Qg = gpu_run(gm, Q, 0.0, 1e-3, 100)
    Qo = ora.run(Q, 0.0, 1e-3, 100)
    err = state_error(Qg, Qo)
    ch, bound = change_error(Qg, Qo, Q)
    # interface cells, element by element, against the largest change
    sl = interface_cells(mesh)
    dmax = np.abs(Qg[..., sl] - Qo[..., sl]).max() / np.abs(Qo - Q).max()
    print("state error", err, "error of the change", ch, "bound", bound,
          "interface cells, largest error / largest change", dmax)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)
    assert dmax <= 1e-3, dmax


@pytest.mark.parametrize("N", [3, 4])
def test_rk3_relabelled_vortex_steps(torch_cuda, N):
    """SSP-RK3 on the vortex mesh with random corner relabelling (384 cells,
    six 64-cell blocks): block-internal faces of mixed direction or reversed
    point order go through the trace buffer, which the stage's export pass
    must then write; same-direction ones through the block's exchange
    array."""
    print(f"case: relabelled vortex SSP-RK3 20 steps N={N}", flush=True)
    case = C.vortex_case(omega=0.5)
    mesh = M.relabel(M.vortex_mesh(1), np.random.default_rng(17).integers(0, 4, 384))
    ora = SSD(mesh, case, N)
    x, y = ora.sp_coords(0.0)
    Q = vortex_state(x, y, 0.0, case)
    gm = _mesh(mesh, case, N)
    dt = 1e-3 if N == 3 else 6e-4
    Qg = gpu_run(gm, Q, 0.0, dt, 20)
    Qo = ora.run(Q, 0.0, dt, 20)
    err = state_error(Qg, Qo)
    ch, bound = change_error(Qg, Qo, Q)
    dmax = np.abs(Qg - Qo).max() / np.abs(Qo - Q).max()
    print("state error", err, "error of the change", ch, "bound", bound,
          "largest element error / largest change", dmax, flush=True)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)
    assert dmax <= 1e-3, dmax


def test_rk3_vortex_offset_wraps(torch_cuda):
    """Start just below a face-width offset so the mortars wrap mid-run."""
    print("case: vortex SSP-RK3 wrap", flush=True)
    mesh, case, ora, Q = _vortex(theta0=2 * np.pi / 32 - 0.02)
    gm = _mesh(mesh, case, 3)
    Qg = gpu_run(gm, Q, 0.0, 2e-3, 30)
    Qo = ora.run(Q, 0.0, 2e-3, 30)
    err = state_error(Qg, Qo)
    ch, bound = change_error(Qg, Qo, Q)
    print("state error", err, "error of the change", ch, "bound", bound)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)


def test_deterministic_and_restartable(torch_cuda):
    import torch
    print("case: determinism / restart", flush=True)
    mesh, case, ora, Q = _vortex()
    gm = _mesh(mesh, case, 3)
    a = gpu_run(gm, Q, 0.0, 1e-3, 20)
    b = gpu_run(gm, Q, 0.0, 1e-3, 20)
    assert np.array_equal(a, b)
    half = gpu_run(gm, Q, 0.0, 1e-3, 10)
    c = gpu_run(gm, half, 10e-3, 1e-3, 10)
    # the state carries everything: a restart from a host copy continues the
    # run (the restart time 10e-3 and 0 + 10 * 1e-3 may differ in the last
    # bit, which moves the rotor angle by an ulp)
    assert np.all(state_error(c, a) < 1e-6)


@pytest.mark.parametrize("viscous", [False, True])
def test_tile_order_does_not_change_the_step(torch_cuda, viscous):
    """Blocks share nothing within a launch, so the order in which a launch
    takes the 64-cell tiles cannot change its result.  The single-mesh path
    runs every Euler stage in tile order and every viscous stage in reverse
    order after its lead tiles; the batched path takes successive stages of
    a viscous group in opposite orders and an inviscid group's in order.
    With the rotor at rest at angle 0 (so that both paths form the same
    rotation exactly), one SSP-RK3 step by each agrees bit for bit, and so
    do repeated residual evaluations.  A rotating-ellipse mesh of two tiles,
    the last one ragged (112 cells); viscous: isothermal wall, Re 1000."""
    import torch
    from paper_1503_02198_amd import Batch
    print(f"case: tile order (single-mesh step, batched step), viscous={viscous}", flush=True)
    case = C.ellipse_viscous_case(omega=0.0) if viscous else C.ellipse_case(omega=0.0)
    mesh = M.ellipse_mesh(K=16, n_in=3, n_out=4, radius=1.5, box_half=4.0, first_in=0.1,
                          first_out=0.2, tile=None,
                          wall=M.FACE_WALL_ISOTHERMAL if viscous else M.FACE_WALL_SLIP)
    gm, gb = _mesh(mesh, case, 4), _mesh(mesh, case, 4)
    Q = C.perturbed_farfield_state(case, 4, gm.info["n_elem"], amplitude=0.05)
    E = gm.info["n_elem"]
    assert E > 64 and E % 64 != 0, E
    q = to_gpu(Q)
    r = [torch.empty_like(q) for _ in range(3)]
    gm.set_rotation(0.0, 0.0)
    gm.mortar_rebuild()
    for k in range(3):
        gm.residual(q, r[k])
    torch.cuda.synchronize()
    assert torch.equal(r[0], r[1]) and torch.equal(r[1], r[2])
    assert bool(torch.isfinite(r[0]).all()) and float(r[0].abs().max()) > 0
    dt = 2e-3
    qa, qb = to_gpu(Q), to_gpu(Q)
    wa = torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0")
    wb = torch.empty(gb.info["work_len"], dtype=torch.float32, device="cuda:0")
    gm.rk_steps(qa, wa, 0.0, dt, 1)
    batch = Batch([gb])
    batch.rk_steps([qb], [wb], [0.0], [dt], 1, graph=False)
    torch.cuda.synchronize()
    batch.close()
    moved = float((qa - q).abs().max())
    diff = float((qa - qb).abs().max())
    print("step moved the state by", moved, "; single minus batched", diff, flush=True)
    assert moved > 1e-4
    assert torch.equal(qa, qb)


def test_error_paths(torch_cuda):
    import torch
    from paper_1503_02198_amd.ssd import SSDError
    print("case: error paths", flush=True)
    mesh, case, ora, Q = _vortex()
    gm = _mesh(mesh, case, 3)
    n = gm.info["state_len"]
    q = torch.zeros(n, device="cuda:0")
    r = torch.zeros(n, device="cuda:0")
    gm.set_rotation(0.1, 0.5)
    with pytest.raises(SSDError) as ei:
        gm.residual(q, r)
    assert ei.value.status == -3
    with pytest.raises(SSDError) as ei:
        gm.rk_step(q, torch.zeros(gm.info["work_len"], device="cuda:0"), 0.0, -1.0)
    assert ei.value.status == -1
    # a negative density is reported by ssd_check
    Qb = Q.copy()
    Qb[0, 1, 1, 7] = -1.0
    from tests.parity_utils import to_gpu
    qb = to_gpu(Qb)
    work = torch.zeros(gm.info["work_len"], device="cuda:0")
    gm.rk_step(qb, work, 0.0, 1e-3)
    with pytest.raises(SSDError) as ei:
        gm.check()
    assert ei.value.status == -6
    gm.check()     # flag cleared


def test_mesh_validation(torch_cuda):
    from paper_1503_02198_amd import Mesh
    from paper_1503_02198_amd.ssd import SSDError
    print("case: mesh validation", flush=True)
    case = C.vortex_case()
    mesh = M.vortex_mesh(1)
    bad = dict(mesh)
    bad["nbr"] = mesh["nbr"].copy()
    e = int(np.nonzero(mesh["face_kind"][:, 0] == 0)[0][0])
    bad["nbr"][e, 0] = (bad["nbr"][e, 0] + 5) % 384
    with pytest.raises(SSDError) as ei:
        Mesh(bad, case, 3)
    assert ei.value.status == -2
    bad = dict(mesh)
    bad["xy"] = mesh["xy"].copy()
    bad["xy"][10] = bad["xy"][10][::-1]         # clockwise cell: |J| < 0
    with pytest.raises(SSDError) as ei:
        Mesh(bad, case, 3)
    assert ei.value.status == -2
    bad = dict(mesh)
    kind = mesh["face_kind"].copy()
    sl = np.argwhere(kind == M.FACE_SLIDING)
    kind[sl[0][0], sl[0][1]] = M.FACE_WALL_SLIP    # one side loses a face
    bad["face_kind"] = kind
    with pytest.raises(SSDError) as ei:
        Mesh(bad, case, 3)
    assert ei.value.status == -2
    with pytest.raises(SSDError) as ei:
        Mesh(mesh, case, 7)
    assert ei.value.status == -1


def test_rk_steps_equals_repeated_rk_step(torch_cuda):
    """ssd_rk_steps reuses the last stage's traces; it must reproduce the
    same number of single steps at the same times t0 + k dt."""
    import torch
    from tests.parity_utils import from_gpu, to_gpu
    print("case: rk_steps vs rk_step", flush=True)
    mesh, case, ora, Q = _vortex(theta0=2 * np.pi / 32 - 0.01)
    gm = _mesh(mesh, case, 3)
    a = gpu_run(gm, Q, 0.0, 2e-3, 12)
    q = to_gpu(Q)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    gm.rk_steps(q, work, 0.0, 2e-3, 12)
    gm.check()
    b = from_gpu(q, 3, gm.info["n_elem"])
    print("bitwise equal:", np.array_equal(a, b), "max rel", state_error(b, a))
    assert np.all(state_error(b, a) < 1e-6)


def test_ssprk54_vortex_steps(torch_cuda):
    """SSPRK54 (the paper's integrator) on the vortex workload, through a
    mortar wrap, against the oracle's SSPRK54."""
    print("case: vortex SSPRK54 40 steps", flush=True)
    mesh, case, ora, Q = _vortex(theta0=2 * np.pi / 32 - 0.02)
    gm = _mesh(mesh, case, 3)
    Qg = gpu_run(gm, Q, 0.0, 2e-3, 40, scheme="rk54")
    Qo = ora.run(Q, 0.0, 2e-3, 40, scheme="rk54")
    err = state_error(Qg, Qo)
    ch, bound = change_error(Qg, Qo, Q)
    print("state error", err, "error of the change", ch, "bound", bound, flush=True)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)


def test_ssprk54_rk_steps_equals_repeated(torch_cuda):
    import torch
    from tests.parity_utils import from_gpu, to_gpu
    print("case: SSPRK54 rk_steps vs rk_step", flush=True)
    mesh, case, ora, Q = _vortex()
    gm = _mesh(mesh, case, 3)
    a = gpu_run(gm, Q, 0.0, 2e-3, 8, scheme="rk54")
    q = to_gpu(Q)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    gm.rk_steps(q, work, 0.0, 2e-3, 8, scheme="rk54")
    gm.check()
    b = from_gpu(q, 3, gm.info["n_elem"])
    assert np.all(state_error(b, a) < 1e-6)
