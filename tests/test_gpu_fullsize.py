"""Parity at the benchmark's full size (999,424-cell rotating-ellipse mesh,
N = 4, the launch configuration bench.py times): the GPU's residual and one
SSP-RK3 or SSPRK54 step, Euler and Navier-Stokes, are compared with the FP64
oracle on sampled cells, which the oracle evaluates on sub-meshes around
them (every interface cell included).
"""
import numpy as np
import pytest

from oracle.ssd import SSD, submesh
from tests.parity_utils import (ELEM_TOL, TOL, change_error, element_max_error, from_gpu,
                                residual_error, state_error, to_gpu)
from workloads import cases as C
from workloads import meshes as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    from paper_1503_02198_amd import Mesh

    class A:
        N, K, n_in, n_out = 4, 4096, 64, 180
    mesh, case, N, E, Q0, dt = bench.workload(A)
    gm = Mesh(mesh, case, N, device=0)
    return mesh, case, N, E, Q0, dt, gm


def _samples(E, rng):
    # the ellipse wall, both interface rings' neighbourhoods (tile-ordered
    # blocks), the far field, and random cells
    fixed = np.array([0, 1, 63, 64, 4095, 262080, 262143, 262144, 262200, E - 1])
    return np.unique(np.concatenate([fixed, rng.choice(E, 200, replace=False)]))


def test_fullsize_residual_sampled(c3):
    import torch
    mesh, case, N, E, Q0, dt, gm = c3
    theta = 0.0123
    print(f"case: full-size residual E={E} N={N} theta={theta}", flush=True)
    q = to_gpu(Q0)
    r = torch.empty_like(q)
    gm.set_rotation(theta, case["omega"])
    gm.mortar_rebuild()
    gm.residual(q, r)
    Rg = from_gpu(r, N, E)
    pick = _samples(E, np.random.default_rng(5))
    sub, idx = submesh(mesh, pick, depth=1)
    ora = SSD(sub, case, N)
    Ro, diag = ora.residual(Q0[..., idx].astype(np.float64), theta, case["omega"], diag=True)
    loc = np.searchsorted(idx, pick)
    err = residual_error(Rg[..., pick], Ro[..., loc], diag["flux_scale"][..., loc])
    print("sampled residual error", err)
    assert np.all(err <= TOL), err
    # interface cells (all in the sub-mesh) are compared in full
    sl = np.nonzero(np.any(mesh["face_kind"] == M.FACE_SLIDING, axis=1))[0]
    locs = np.searchsorted(idx, sl)
    err = residual_error(Rg[..., sl], Ro[..., locs], diag["flux_scale"][..., locs])
    emax = element_max_error(Rg[..., sl], Ro[..., locs], diag["flux_scale"][..., locs])
    print("interface-cell residual error", err, "element maximum", emax)
    assert np.all(err <= TOL), err
    assert np.all(emax <= ELEM_TOL), emax


def test_fullsize_rk3_step_sampled(c3):
    import torch
    mesh, case, N, E, Q0, dt, gm = c3
    print(f"case: full-size SSP-RK3 step E={E} dt={dt:.3e}", flush=True)
    q = to_gpu(Q0)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    gm.rk_step(q, work, 0.0, dt)
    gm.check()
    Qg = from_gpu(q, N, E)
    pick = _samples(E, np.random.default_rng(6))
    sub, idx = submesh(mesh, pick, depth=3)
    ora = SSD(sub, case, N)
    Qo = ora.ssprk3_step(Q0[..., idx].astype(np.float64), 0.0, dt)
    loc = np.searchsorted(idx, pick)
    err = state_error(Qg[..., pick], Qo[..., loc])
    # one step at this dt moves the state by about 2e-5 of its norm, so the
    # state error alone would pass a kernel that applied half the increment:
    # the error of the change is asserted too
    ch, bound = change_error(Qg[..., pick], Qo[..., loc], Q0[..., pick])
    print("sampled state error", err, "error of the change", ch, "bound", bound)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)


def test_fullsize_ssprk54_step_sampled(c3):
    """One SSPRK54 step (five residual evaluations, the fourth stage forming
    the last stage's increment) on the full mesh, against the oracle on a
    sub-mesh five neighbour layers deep around the sampled cells."""
    import torch
    mesh, case, N, E, Q0, dt, gm = c3
    print(f"case: full-size SSPRK54 step E={E} dt={dt:.3e}", flush=True)
    q = to_gpu(Q0)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    gm.rk_step(q, work, 0.0, dt, scheme="rk54")
    gm.check()
    Qg = from_gpu(q, N, E)
    pick = _samples(E, np.random.default_rng(7))
    sub, idx = submesh(mesh, pick, depth=5)
    ora = SSD(sub, case, N)
    Qo = ora.ssprk54_step(Q0[..., idx].astype(np.float64), 0.0, dt)
    loc = np.searchsorted(idx, pick)
    err = state_error(Qg[..., pick], Qo[..., loc])
    ch, bound = change_error(Qg[..., pick], Qo[..., loc], Q0[..., pick])
    print("sampled state error", err, "error of the change", ch, "bound", bound)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)


@pytest.fixture(scope="module")
def c3_viscous():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    from paper_1503_02198_amd import Mesh

    class A:
        N, K, n_in, n_out, viscous = 4, 4096, 64, 180, True
    mesh, case, N, E, Q0, dt = bench.workload(A)
    gm = Mesh(mesh, case, N, device=0)
    return mesh, case, N, E, Q0, dt, gm


def test_fullsize_viscous_residual_sampled(c3_viscous):
    """The viscous residual on the full mesh of `bench.py --viscous`
    (isothermal ellipse wall, Mach 0.3, Re 1000), against the oracle on a
    sub-mesh two neighbour layers deep (BR1 gradients reach two layers)."""
    import torch
    mesh, case, N, E, Q0, dt, gm = c3_viscous
    theta = 0.0371
    print(f"case: full-size viscous residual E={E} N={N} theta={theta}", flush=True)
    q = to_gpu(Q0)
    r = torch.empty_like(q)
    gm.set_rotation(theta, case["omega"])
    gm.mortar_rebuild()
    gm.residual(q, r)
    Rg = from_gpu(r, N, E)
    pick = _samples(E, np.random.default_rng(8))
    sub, idx = submesh(mesh, pick, depth=2)
    ora = SSD(sub, case, N)
    Ro, diag = ora.residual(Q0[..., idx].astype(np.float64), theta, case["omega"], diag=True)
    loc = np.searchsorted(idx, pick)
    err = residual_error(Rg[..., pick], Ro[..., loc], diag["flux_scale"][..., loc])
    print("sampled viscous residual error", err)
    assert np.all(err <= TOL), err


def test_fullsize_viscous_rk3_step_sampled(c3_viscous):
    """One viscous SSP-RK3 step on the full mesh of `bench.py --viscous`,
    the launch sequence it times (mortar, gradient pass, viscous mortar,
    stage, three times), against the oracle on a sub-mesh six neighbour
    layers deep (two per stage: the BR1 common solution and gradient)."""
    import torch
    mesh, case, N, E, Q0, dt, gm = c3_viscous
    print(f"case: full-size viscous SSP-RK3 step E={E} dt={dt:.3e}", flush=True)
    q = to_gpu(Q0)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    gm.rk_step(q, work, 0.0, dt)
    gm.check()
    Qg = from_gpu(q, N, E)
    pick = _samples(E, np.random.default_rng(9))
    sub, idx = submesh(mesh, pick, depth=6)
    ora = SSD(sub, case, N)
    Qo = ora.ssprk3_step(Q0[..., idx].astype(np.float64), 0.0, dt)
    loc = np.searchsorted(idx, pick)
    err = state_error(Qg[..., pick], Qo[..., loc])
    ch, bound = change_error(Qg[..., pick], Qo[..., loc], Q0[..., pick])
    print("sampled state error", err, "error of the change", ch, "bound", bound)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)
