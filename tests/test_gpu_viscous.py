"""Viscous HIP path (BR1 gradient pass, viscous mortar, viscous fluxes in the
stage kernel) vs the FP64 oracle on identical seeded inputs, through the C ABI.

Every case prints its name before touching the GPU so a failure names it.
"""
import numpy as np
import pytest

from oracle.exact import Couette, vortex_state
from oracle.ssd import SSD
from tests.parity_utils import (TOL, change_error, gpu_residual, gpu_run, residual_error,
                                state_error)
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


def _couette_state(ora, case, theta, seed=3):
    """Exact Couette state with a smooth seeded perturbation, so that every
    gradient component and every face jump is non-zero."""
    x, y = ora.sp_coords(theta)
    Q = Couette(case).state(x, y)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, size=(4, 3))
    for v in range(4):
        Q[v] *= 1.0 + 0.02 * np.sin(a[v, 0] * x + a[v, 1] * y + a[v, 2])
    return Q


def _check_residual(gm, ora, Q, theta, omega, label):
    Rg = gpu_residual(gm, Q, theta, omega)
    Ro, diag = ora.residual(Q, theta, omega, diag=True)
    err = residual_error(Rg, Ro, diag["flux_scale"])
    print(label, "residual error", err, flush=True)
    assert np.all(err <= TOL), err


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_residual_couette(torch_cuda, N):
    """Isothermal rotating and fixed walls, sliding interface at a non-zero
    offset delta, cubic cells on walls and interface."""
    print(f"case: couette residual N={N}", flush=True)
    case = C.couette_case()
    mesh = M.couette_mesh(4, 16, phi_offset=0.3 * 2 * np.pi / 16)
    ora = SSD(mesh, case, N)
    gm = _mesh(mesh, case, N)
    for th in (0.0, 0.21, -1.3):
        Q = _couette_state(ora, case, th)
        _check_residual(gm, ora, Q, th, case["omega"], f"theta={th}")


@pytest.mark.parametrize("N", [3, 4])
def test_residual_couette_relabelled(torch_cuda, N):
    """Corner relabelling reverses face parameters on walls and interface."""
    print(f"case: relabelled couette residual N={N}", flush=True)
    case = C.couette_case()
    base = M.couette_mesh(4, 16, phi_offset=0.17)
    mesh = M.relabel(base, np.random.default_rng(5).integers(0, 4, len(base["zone"])))
    ora = SSD(mesh, case, N)
    gm = _mesh(mesh, case, N)
    for th in (0.05, 0.9):
        Q = _couette_state(ora, case, th, seed=9)
        _check_residual(gm, ora, Q, th, case["omega"], f"theta={th}")


@pytest.mark.parametrize("N", [2, 4, 6])
@pytest.mark.parametrize("curved", [False, True])
def test_residual_viscous_box(torch_cuda, N, curved):
    """Periodic conforming box turning as a whole: conforming and periodic
    BR1 faces, in-block and cross-block neighbours, straight and cubic cells."""
    print(f"case: viscous box residual N={N} curved={curved}", flush=True)
    case = C.vortex_case()
    case["mu"] = 0.05
    mesh = M.box_mesh(9, 8, L=(3.0, 2.0), distort=0.15, curved=0.06 if curved else 0.0, zone=1)
    ora = SSD(mesh, case, N)
    x, y = ora.sp_coords(0.0)
    case["vortex"]["period"] = 100.0
    case["vortex"]["center"] = (1.5, 1.0)
    Q = vortex_state(x, y, 0.0, case)
    gm = _mesh(mesh, case, N)
    _check_residual(gm, ora, Q, 0.3, 0.8, "box")


@pytest.mark.parametrize("wall", ["slip", "isothermal"])
@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_residual_viscous_ellipse(torch_cuda, N, wall):
    """Slip or isothermal no-slip wall, far field and the sliding interface
    with viscosity, at every order (N >= 5 takes every gradient trace
    through the trace buffer)."""
    print(f"case: viscous ellipse residual N={N} wall={wall}", flush=True)
    case = C.ellipse_case()
    case["mu"] = 0.02
    mesh = M.ellipse_mesh(K=32, n_in=4, n_out=4, radius=1.5, box_half=4.0, first_in=0.05,
                          first_out=0.1,
                          wall=M.FACE_WALL_SLIP if wall == "slip" else M.FACE_WALL_ISOTHERMAL)
    ora = SSD(mesh, case, N)
    E = len(mesh["zone"])
    Q = C.perturbed_farfield_state(case, N, E, amplitude=0.02)
    gm = _mesh(mesh, case, N)
    for th in (0.0, 0.07):
        _check_residual(gm, ora, Q, th, case["omega"], f"theta={th}")


def test_rk3_couette_steps(torch_cuda):
    """SSP-RK3 on the viscous Couette mesh through several mortar offsets."""
    print("case: couette SSP-RK3 40 steps", flush=True)
    case = C.couette_case()
    mesh = M.couette_mesh(4, 16, phi_offset=0.11)
    N = 3
    ora = SSD(mesh, case, N)
    Q = _couette_state(ora, case, 0.0)
    gm = _mesh(mesh, case, N)
    dt = 2e-3
    Qg = gpu_run(gm, Q, 0.0, dt, 40)
    Qo = ora.run(Q, 0.0, dt, 40)
    err = state_error(Qg, Qo)
    print("state error", err, "relative to the change",
          np.linalg.norm(Qg - Qo) / np.linalg.norm(Qo - Q), flush=True)
    assert np.all(err <= TOL), err


def test_rk3_couette_relabelled_steps(torch_cuda):
    """SSP-RK3 on a relabelled 8 x 32 Couette mesh (four 64-cell blocks): the
    BR1 gradient traces of block-internal faces of mixed direction or
    reversed order go through the gradient-trace buffer, the rest through
    the stage's exchange array."""
    print("case: relabelled couette SSP-RK3 10 steps N=3", flush=True)
    case = C.couette_case()
    base = M.couette_mesh(8, 32, phi_offset=0.07)
    mesh = M.relabel(base, np.random.default_rng(23).integers(0, 4, len(base["zone"])))
    N = 3
    ora = SSD(mesh, case, N)
    Q = _couette_state(ora, case, 0.0, seed=4)
    gm = _mesh(mesh, case, N)
    dt = 1e-3
    Qg = gpu_run(gm, Q, 0.0, dt, 10)
    Qo = ora.run(Q, 0.0, dt, 10)
    err = state_error(Qg, Qo)
    rel = np.linalg.norm(Qg - Qo) / np.linalg.norm(Qo - Q)
    print("state error", err, "relative to the change", rel, flush=True)
    assert np.all(err <= TOL), err
    assert rel <= 1e-2, rel


def test_rk_steps_viscous_equals_repeated(torch_cuda):
    import torch
    from tests.parity_utils import from_gpu, to_gpu
    print("case: viscous rk_steps vs rk_step", flush=True)
    case = C.couette_case()
    mesh = M.couette_mesh(4, 16, phi_offset=0.11)
    ora = SSD(mesh, case, 3)
    Q = _couette_state(ora, case, 0.0)
    gm = _mesh(mesh, case, 3)
    a = gpu_run(gm, Q, 0.0, 2e-3, 10)
    q = to_gpu(Q)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    gm.rk_steps(q, work, 0.0, 2e-3, 10)
    gm.check()
    b = from_gpu(q, 3, gm.info["n_elem"])
    assert np.all(state_error(b, a) < 1e-6)


@pytest.mark.parametrize("N", [3, 5, 6])
def test_ssprk54_couette_steps(torch_cuda, N):
    """SSPRK54 on the viscous Couette mesh (the fourth stage forms the last
    stage's increment in the same kernel, at N = 5 and 6 too), asserting
    the state and the error of the run's change."""
    print(f"case: couette SSPRK54 15 steps N={N}", flush=True)
    case = C.couette_case()
    mesh = M.couette_mesh(4, 16, phi_offset=0.11)
    ora = SSD(mesh, case, N)
    Q = _couette_state(ora, case, 0.0)
    gm = _mesh(mesh, case, N)
    dt = 3e-3 * (3.0 / N) ** 2
    Qg = gpu_run(gm, Q, 0.0, dt, 15, scheme="rk54")
    Qo = ora.run(Q, 0.0, dt, 15, scheme="rk54")
    err = state_error(Qg, Qo)
    ch, bound = change_error(Qg, Qo, Q)
    print("state error", err, "error of the change", ch, "bound", bound, flush=True)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)
