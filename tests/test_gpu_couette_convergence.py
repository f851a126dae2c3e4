"""Steady Taylor-Couette on the GPU against the analytic profile (Sec. 4.2,
Tables 5-6): x-velocity L1/L2 errors on two annulus refinements, and their
order.

The run starts from the exact steady state and marches with SSPRK54 (the
paper's integrator) to t = 2, long enough for the discrete steady state to
form.  The state is FP32: at this Mach number (0.1 at the inner wall) the
energy is about 180 times the kinetic energy, and the velocity error of an
FP32 steady state levels off near 3e-6 (L2).  The levels used here keep the
errors well above that floor: N = 2 on the 8 x 32 and 16 x 64 annuli,
N = 3, 4 and 5 on the 4 x 16 and 8 x 32 annuli (at N = 4 and 5 the 8 x 32
errors, 2-3e-5, are ten times the floor; the 2 x 8 annulus is not yet in the
asymptotic range, order 2.8-2.9).  At N = 5 the errors are close to N = 4's:
the cubic (serendipity) wall and interface cells carry an O(h^4) geometric
error, so the order stays near 4.5 rather than 5.
"""
import json
import os

import numpy as np
import pytest

from oracle.exact import Couette
from oracle.ssd import SSD
from workloads import cases as C
from workloads import meshes as M

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _couette_error(N, nr, nt, T=2.0, cfl=0.2):
    import torch
    from paper_1503_02198_amd import Mesh
    from tests.parity_utils import from_gpu, to_gpu
    case = C.couette_case()
    ex = Couette(case)
    mesh = M.couette_mesh(nr, nt, phi_offset=0.37 * 2 * np.pi / nt)
    geo = SSD(mesh, case, N)          # solution-point coordinates and |J| only
    E = len(mesh["zone"])
    x, y = geo.sp_coords(0.0)
    gm = Mesh(mesh, case, N, device=0)
    q = to_gpu(ex.state(x, y))
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    h = min(2 * np.pi / nt, 1.0 / nr)
    lam = 1.0 + np.sqrt(case["gamma"] * case["farfield"][3])
    n = int(np.ceil(T / (cfl * h / (lam * N * N))))
    dt = T / n
    done = 0
    while done < n:                     # bounded chunks, progress per chunk
        k = min(4000, n - done)
        gm.rk_steps(q, work, done * dt, dt, k, scheme="rk54")
        done += k
        gm.check()
        print(f"  N={N} {nr}x{nt}: {done}/{n} steps", flush=True)
    Q = from_gpu(q, N, E)
    xT, yT = geo.sp_coords(case["omega"] * T)
    e = Q[1] / Q[0] - ex.u(xT, yT)
    w = geo.ops.w
    W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(geo.geo.detJ, 0, 2)
    return (W * np.abs(e)).sum() / W.sum(), np.sqrt((W * e * e).sum() / W.sum())


@pytest.mark.parametrize("N,nr,min_order", [(2, 8, 1.6), (3, 4, 2.6), (4, 4, 3.5), (5, 4, 3.5)])
def test_couette_steady_convergence(torch_cuda, N, nr, min_order):
    print(f"case: Couette steady state N={N}, {nr}x{4 * nr} and {2 * nr}x{8 * nr}", flush=True)
    e1 = _couette_error(N, nr, 4 * nr)
    e2 = _couette_error(N, 2 * nr, 8 * nr)
    order = np.log2(np.array(e1) / np.array(e2))
    print("L1, L2:", e1, e2, "orders", order, flush=True)
    assert np.all(order > min_order), order
    assert e2[1] > 1e-5          # above the FP32 floor: the order is the method's
    if N in (3, 4):
        key = {3: "table5_couette_N3", 4: "table6_couette_N4"}[N]
        with open(GOLD) as fh:
            paper = [r["L2_order"] for r in json.load(fh)[key]["rows"] if r["L2_order"] is not None]
        assert order[1] > min(paper) - 0.6, (order, paper)
