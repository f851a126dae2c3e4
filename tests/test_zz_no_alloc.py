"""ssd_rk_steps_noalloc (work arrays in the library's fixed per-GPU array)
against ssd_rk_steps with a caller's work tensor, through the C ABI: two
calls in a row on different meshes, the second smaller than the first, so
the second runs on what the first left in the array.  Both paths run the
same kernels on the same inputs, so the results must agree bit for bit (and
therefore within the parity bar of the oracle comparisons)."""
import numpy as np
import pytest

from oracle.exact import vortex_state
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


def _case(f, N, scheme):
    case = C.vortex_case(omega=0.5, theta0=0.01)
    mesh = M.vortex_mesh(f)
    x, y = SSD(mesh, case, N).sp_coords(case["theta0"])
    return mesh, case, N, vortex_state(x, y, 0.0, case), scheme


def test_noalloc_matches_rk_steps_twice(torch_cuda):
    import torch
    from paper_1503_02198_amd import Mesh
    # larger first (1,536 cells, N = 4, SSPRK54: 3 work arrays), then
    # smaller (384 cells, N = 3, SSP-RK3: 2 work arrays)
    for mesh, case, N, Q, scheme in (_case(2, 4, "rk54"), _case(1, 3, "rk3")):
        E = len(mesh["zone"])
        print(f"case: noalloc vs rk_steps E={E} N={N} {scheme}", flush=True)
        gm = Mesh(mesh, case, N, device=0)
        q_ref = to_gpu(Q)
        work = torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0")
        gm.rk_steps(q_ref, work, 0.0, 1e-3, 7, scheme=scheme)
        gm.check()
        q = to_gpu(Q)
        gm.rk_steps_noalloc(q, 0.0, 1e-3, 7, scheme=scheme)
        gm.check()
        a, b = from_gpu(q, N, E), from_gpu(q_ref, N, E)
        err = state_error(a, b)
        print("relative difference", err, "bitwise equal", np.array_equal(a, b), flush=True)
        assert np.all(err <= TOL), err
        assert np.array_equal(a, b)
        gm.close()


def test_noalloc_refuses_oversized_meshes_and_timing(torch_cuda):
    from paper_1503_02198_amd import Mesh
    from paper_1503_02198_amd.ssd import SSDError
    print("case: noalloc size limit and timing refusal", flush=True)
    case = C.vortex_case(omega=0.0)
    # 200 x 200 cells at N = 6: a state is 4 * 36 * 40,000 floats (23.0 MB),
    # SSPRK54's three work arrays 69.1 MB > 64 MiB (67.1 MB)
    mesh = M.box_mesh(200, 200, L=(2.0, 2.0))
    gm = Mesh(mesh, case, 6, device=0)
    import torch
    q = torch.ones(gm.info["state_len"], dtype=torch.float32, device="cuda:0")
    with pytest.raises(SSDError) as ei:
        gm.rk_steps_noalloc(q, 0.0, 1e-4, 1, scheme="rk54")
    assert ei.value.status == -1
    gm.close()
    small = Mesh(M.vortex_mesh(1), C.vortex_case(), 3, device=0)
    q = torch.ones(small.info["state_len"], dtype=torch.float32, device="cuda:0")
    small.timing_enable(kernels=["stage"])
    with pytest.raises(SSDError) as ei:
        small.rk_steps_noalloc(q, 0.0, 1e-4, 1)
    assert ei.value.status == -3
    small.timing_enable(False)
    small.close()
