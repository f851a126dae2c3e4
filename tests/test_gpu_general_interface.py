"""General sliding interface on the GPU (sides of different face counts,
non-uniform faces) against the oracle's general interface, through the C
ABI.  Inviscid rotating-ellipse meshes; tolerances as in the parity tests
(tests/parity_utils.py).  Every case prints its name before touching the
GPU."""
import numpy as np
import pytest

from oracle.ssd import SSD, GeneralInterface
from tests.parity_utils import (ELEM_TOL, TOL, change_error, element_max_error, from_gpu,
                                gpu_residual, gpu_run, interface_cells, residual_error, state_error,
                                to_gpu)
from workloads import cases as C
from workloads import meshes as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mesh(K, K_out, warp):
    return M.ellipse_mesh(K=K, n_in=2, n_out=2, radius=1.5, box_half=4.0, first_in=0.1,
                          first_out=0.2, tile=None, K_out=K_out, warp=warp)


@pytest.mark.parametrize("K,K_out,warp,N", [(16, 24, 0.3, 3), (24, 16, -0.4, 4), (16, 16, 0.5, 2),
                                            (32, 48, 0.0, 5), (16, 24, 0.2, 6)])
def test_residual(torch_cuda, K, K_out, warp, N):
    from paper_1503_02198_amd import Mesh
    print(f"case: general interface residual K={K} K_out={K_out} warp={warp} N={N}", flush=True)
    case = C.ellipse_case()
    mesh = _mesh(K, K_out, warp)
    ora = SSD(mesh, case, N)
    assert isinstance(ora.iface, GeneralInterface)
    gm = Mesh(mesh, case, N)
    Q = C.perturbed_farfield_state(case, N, ora.E, amplitude=0.05)
    for th in (0.0, 0.37, -2.1, 5.0):
        Rg = gpu_residual(gm, Q, th, case["omega"])
        Ro, diag = ora.residual(Q, th, case["omega"], diag=True)
        err = residual_error(Rg, Ro, diag["flux_scale"])
        emax = element_max_error(Rg, Ro, diag["flux_scale"], interface_cells(mesh))
        print("theta", th, "residual error", err, "interface-cell maximum", emax, flush=True)
        assert np.all(err <= TOL), err
        assert np.all(emax <= ELEM_TOL), emax


def test_rk3_steps(torch_cuda):
    """40 steps at 0.8 of the CFL-0.1 step of the mesh (1.5e-4)."""
    from paper_1503_02198_amd import Mesh
    print("case: general interface SSP-RK3 40 steps", flush=True)
    case = C.ellipse_case(omega=2.0)
    mesh = _mesh(16, 24, 0.3)
    N = 3
    ora = SSD(mesh, case, N)
    gm = Mesh(mesh, case, N)
    Q = C.perturbed_farfield_state(case, N, ora.E, amplitude=0.05)
    Qg = gpu_run(gm, Q, 0.4, 1.2e-4, 40)
    Qo = ora.run(Q, 0.4, 1.2e-4, 40)
    err = state_error(Qg, Qo)
    ch, bound = change_error(Qg, Qo, Q)
    print("state error", err, "error of the change", ch, "bound", bound, flush=True)
    assert np.all(err <= TOL), err
    assert ch <= bound, (ch, bound)


@pytest.mark.parametrize("K,K_out,warp,N", [(16, 24, 0.3, 3), (24, 16, -0.4, 4), (16, 16, 0.5, 2),
                                            (32, 48, 0.0, 5)])
def test_viscous_residual(torch_cuda, K, K_out, warp, N):
    """BR1 common solution and viscous flux through the general mortars."""
    from paper_1503_02198_amd import Mesh
    print(f"case: general interface viscous residual K={K} K_out={K_out} N={N}", flush=True)
    case = C.ellipse_case()
    case["mu"] = 0.02
    mesh = _mesh(K, K_out, warp)
    ora = SSD(mesh, case, N)
    gm = Mesh(mesh, case, N)
    Q = C.perturbed_farfield_state(case, N, ora.E, amplitude=0.05)
    for th in (0.0, 0.81, -2.6):
        Rg = gpu_residual(gm, Q, th, case["omega"])
        Ro, diag = ora.residual(Q, th, case["omega"], diag=True)
        err = residual_error(Rg, Ro, diag["flux_scale"])
        print("theta", th, "residual error", err, flush=True)
        assert np.all(err <= TOL), err


@pytest.mark.parametrize("scheme", ["rk3", "rk54"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_with_general_rings(torch_cuda, scheme, graph):
    """A batch mixing general-ring meshes (inviscid N = 3 and 4, viscous
    N = 3) with a uniform-ring mesh of the same N steps like each mesh
    alone.  The batch reads each stage's rotor angle from its device step
    counter, the single mesh gets it from the host, so the two agree to
    rounding (relative 1e-6), not bit for bit."""
    import torch
    from paper_1503_02198_amd import Batch, Mesh
    print(f"case: batch with general rings, {scheme}, graph={graph}", flush=True)
    cv = C.ellipse_case(omega=2.0)
    cv["mu"] = 0.02
    specs = [(_mesh(16, 24, 0.3), C.ellipse_case(omega=2.0), 3, 0.4),
             (_mesh(24, 16, -0.4), C.ellipse_case(omega=-1.5), 4, 0.1),
             (_mesh(16, 16, 0.0), C.ellipse_case(omega=1.0), 3, 0.0),   # uniform rings
             (_mesh(16, 24, 0.3), cv, 3, 0.2)]
    meshes = [Mesh(m, c, N) for m, c, N, _ in specs]
    assert [g.info["K"] for g in meshes] == [24, 24, 16, 24]
    dt, nsteps = 6.0e-5, 6
    Qs = [C.perturbed_farfield_state(c, N, g.info["n_elem"], amplitude=0.05, seed=k)
          for k, ((m, c, N, _), g) in enumerate(zip(specs, meshes))]
    ref = []
    for g, Q, (m, c, N, t0) in zip(meshes, Qs, specs):
        ref.append(gpu_run(g, Q, t0, dt, nsteps, scheme=scheme))
    batch = Batch(meshes)
    qs = [to_gpu(Q) for Q in Qs]
    ws = [torch.empty(g.info["work_len"], dtype=torch.float32, device="cuda:0") for g in meshes]
    batch.rk_steps(qs, ws, [s[3] for s in specs], [dt] * len(specs), nsteps, scheme=scheme,
                   graph=graph)
    for g in meshes:
        g.check()
    assert sorted((g["N"], g["viscous"]) for g in batch.groups()) == [(3, 0), (3, 1), (4, 0)]
    for k, (g, (m, c, N, t0)) in enumerate(zip(meshes, specs)):
        err = state_error(from_gpu(qs[k], N, g.info["n_elem"]), ref[k])
        print(k, "N", N, "relative difference", err, flush=True)
        assert np.all(err < 1e-6), (k, err)
    batch.close()
