"""Batched stepping (ssd_batch_*) of meshes with different N, viscosity,
sizes and rotation rates against stepping each mesh alone with
ssd_rk_steps: eager launches and graph replays, SSP-RK3 and SSPRK54, an odd
number of steps (a two-step graph plus a one-step graph).

The batch forms each stage's rotor angle on the device from t + (n + c) dt
with a device step counter, the single-mesh path on the host from t + n dt +
c dt; the results agree to rounding (relative 1e-6), not bit for bit.
"""
import numpy as np
import pytest

from oracle.exact import Couette, vortex_state
from oracle.ssd import SSD
from tests.parity_utils import from_gpu, state_error, to_gpu
from workloads import cases as C
from workloads import meshes as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cases():
    """(mesh, case, N, initial state, t0, dt) for a mixed batch."""
    out = []
    for N, omega, th0, f in ((3, 0.5, 0.0, 1), (3, 1.3, 0.2, 1), (5, 0.7, 0.1, 1)):
        case = C.vortex_case(omega=omega, theta0=th0)
        mesh = M.vortex_mesh(f)
        x, y = SSD(mesh, case, N).sp_coords(th0)
        out.append((mesh, case, N, vortex_state(x, y, 0.0, case), 0.0, 1e-3))
    for N, nr in ((2, 4), (3, 4)):
        case = C.couette_case()
        mesh = M.couette_mesh(nr, 4 * nr, phi_offset=0.23)
        x, y = SSD(mesh, case, N).sp_coords(0.0)
        out.append((mesh, case, N, Couette(case).state(x, y), 0.1, 2e-3))
    case = C.vortex_case(omega=0.8)
    case["vortex"]["period"] = 100.0
    case["vortex"]["center"] = (1.5, 1.0)
    mesh = M.box_mesh(7, 5, L=(3.0, 2.0), distort=0.15, zone=1)
    x, y = SSD(mesh, case, 4).sp_coords(0.0)
    out.append((mesh, case, 4, vortex_state(x, y, 0.0, case), 0.05, 1.5e-3))
    return out


@pytest.mark.parametrize("scheme", ["rk3", "rk54"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_single_meshes(torch_cuda, scheme, graph):
    import torch
    from paper_1503_02198_amd import Batch, Mesh
    print(f"case: batch of 6 meshes, {scheme}, graph={graph}", flush=True)
    cs = _cases()
    meshes = [Mesh(m, c, N, device=0) for m, c, N, _, _, _ in cs]
    nsteps = 5
    ref = []
    for gm, (m, c, N, Q, t0, dt) in zip(meshes, cs):
        q = to_gpu(Q)
        w = torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0")
        gm.rk_steps(q, w, t0, dt, nsteps, scheme=scheme)
        gm.check()
        ref.append(from_gpu(q, N, gm.info["n_elem"]))
    batch = Batch(meshes)
    qs = [to_gpu(Q) for _, _, _, Q, _, _ in cs]
    ws = [torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0") for gm in meshes]
    batch.rk_steps(qs, ws, [c[4] for c in cs], [c[5] for c in cs], nsteps, scheme=scheme,
                   graph=graph)
    for gm in meshes:
        gm.check()
    groups = batch.groups()
    print("groups", groups, flush=True)
    assert sorted((g["N"], g["viscous"]) for g in groups) == [(2, 1), (3, 0), (3, 1), (4, 0), (5, 0)]
    assert all(g["tuned"] and 0 <= g["stream"] < g["n_streams"] <= 4 and g["stage_us"] > 0
               for g in groups)
    for k, (gm, (m, c, N, Q, t0, dt)) in enumerate(zip(meshes, cs)):
        got = from_gpu(qs[k], N, gm.info["n_elem"])
        err = state_error(got, ref[k])
        print(k, "N", N, "relative difference", err, flush=True)
        assert np.all(err < 1e-6), (k, err)
    # a second call reuses the graphs and the tuned grids, from the new state
    for k in range(len(cs)):
        ref[k] = from_gpu(qs[k], cs[k][2], meshes[k].info["n_elem"])
    batch.rk_steps(qs, ws, [c[4] + nsteps * c[5] for c in cs], [c[5] for c in cs], 2,
                   scheme=scheme, graph=graph)
    for gm in meshes:
        gm.check()
    for k, gm in enumerate(meshes):
        q = to_gpu(ref[k])
        w = torch.empty(gm.info["work_len"], dtype=torch.float32, device="cuda:0")
        gm.rk_steps(q, w, cs[k][4] + nsteps * cs[k][5], cs[k][5], 2, scheme=scheme)
        err = state_error(from_gpu(qs[k], cs[k][2], gm.info["n_elem"]),
                          from_gpu(q, cs[k][2], gm.info["n_elem"]))
        assert np.all(err < 1e-6), (k, err)
    batch.close()
