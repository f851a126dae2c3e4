"""General sliding interface on the GPU (sides of different face counts,
non-uniform faces) against the oracle's general interface, through the C
ABI.  Inviscid rotating-ellipse meshes; tolerances as in the parity tests
(tests/parity_utils.py).  Every case prints its name before touching the
GPU."""
import numpy as np
import pytest

from oracle.ssd import SSD, GeneralInterface
from tests.parity_utils import TOL, gpu_residual, gpu_run, residual_error, state_error
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
                                            (32, 48, 0.0, 5)])
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
        print("theta", th, "residual error", err, flush=True)
        assert np.all(err <= TOL), err


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
    print("state error", err, flush=True)
    assert np.all(err <= TOL), err


@pytest.mark.parametrize("K,K_out,warp,N", [(16, 24, 0.3, 3), (24, 16, -0.4, 4)])
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


def test_batch_rejects_general_rings(torch_cuda):
    from paper_1503_02198_amd import Batch, Mesh, SSDError
    print("case: batch rejects general rings", flush=True)
    gm = Mesh(_mesh(16, 24, 0.3), C.ellipse_case(), 3)
    with pytest.raises(SSDError):
        Batch([gm])
