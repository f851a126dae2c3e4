"""Helpers shared by the GPU parity tests: run the HIP path through the C
ABI binding and the FP64 oracle on the same inputs, and the error norms.

Tolerances (FP32 state and fluxes, FP64 metrics and mortar projections):
  residual  per variable, ||R_gpu - R_oracle||_2 / ||S||_2 <= 1e-5, where S
            is the oracle's flux-derivative scale sum_k |D_ik||F~_k| / |J|
            (the residual is a small difference of O(|S|) terms, so FP32
            rounding is bounded relative to S, not to R);
  state     per variable, ||Q_gpu - Q_oracle||_2 / ||Q_oracle||_2 <= 1e-5,
            with both momentum components measured against the norm of
            the momentum vector.
  change    ||dQ_gpu - dQ_oracle||_2 / ||dQ_oracle||_2 over all variables,
            dQ = Q_end - Q_start: the error of the update itself.  Storing
            Q in FP32 rounds each value by up to 6e-8 |Q|, and the stored
            stage values add their own roundings, so the bound is
            CHANGE_TOL + 1.2e-7 ||Q|| / ||dQ|| (one FP32 ulp; a step that
            moves Q by 2e-5 of its norm allows 7e-3); half the increment, or
            none, gives 0.5 or 1.
  element   per element and variable, max |R_gpu - R_oracle| over the
            element's points divided by the largest S of that element and
            variable, <= ELEM_TOL = 1e-4.  FP32 rounding of the O(10^2)
            operations behind one residual value bounds it by about 1e-5; the
            L2 norm above would dilute an error confined to a few cells (the
            64 interface cells of a 384-cell mesh by a factor of 2.4).
"""
import numpy as np

TOL = 1e-5
ELEM_TOL = 1e-4
CHANGE_TOL = 1e-3
FP32_ROUND = 1.2e-7


def residual_error(R_gpu, R_ora, scale):
    R_gpu = np.asarray(R_gpu, dtype=np.float64)
    out = []
    for v in range(4):
        out.append(np.linalg.norm(R_gpu[v] - R_ora[v]) / np.linalg.norm(scale[v]))
    return np.array(out)


def state_error(Q_gpu, Q_ora):
    Q_gpu = np.asarray(Q_gpu, dtype=np.float64)
    mom = np.sqrt(np.linalg.norm(Q_ora[1]) ** 2 + np.linalg.norm(Q_ora[2]) ** 2)
    den = [np.linalg.norm(Q_ora[0]), mom, mom, np.linalg.norm(Q_ora[3])]
    return np.array([np.linalg.norm(Q_gpu[v] - Q_ora[v]) / den[v] for v in range(4)])


def element_max_error(R_gpu, R_ora, scale, cells=None):
    """Per variable, the largest over the given cells (all by default) of
    max |R_gpu - R_ora| / max S within the cell."""
    R_gpu = np.asarray(R_gpu, dtype=np.float64)
    if cells is None:
        cells = np.arange(R_ora.shape[-1])
    d = np.abs(R_gpu[..., cells] - R_ora[..., cells]).max(axis=(1, 2))
    s = np.abs(scale[..., cells]).max(axis=(1, 2))
    return (d / s).max(axis=1)


def change_error(Q_gpu, Q_ora, Q_start):
    """(error of the change, its bound): ||dQ_gpu - dQ_ora|| / ||dQ_ora||
    over all variables, and CHANGE_TOL + the FP32 rounding of Q relative to
    the change."""
    Q_gpu = np.asarray(Q_gpu, dtype=np.float64)
    do = Q_ora - Q_start
    err = np.linalg.norm((Q_gpu - Q_start) - do) / np.linalg.norm(do)
    bound = CHANGE_TOL + FP32_ROUND * np.linalg.norm(Q_ora) / np.linalg.norm(do)
    return err, bound


def interface_cells(mesh):
    """Elements with a sliding face."""
    from workloads.meshes import FACE_SLIDING
    return np.nonzero(np.any(mesh["face_kind"] == FACE_SLIDING, axis=1))[0]


def to_gpu(Q, device=0):
    import torch
    from paper_1503_02198_amd.ssd import pack_state
    return torch.tensor(pack_state(np.asarray(Q, dtype=np.float32)), device=f"cuda:{device}")


def from_gpu(t, N, E):
    import torch
    torch.cuda.synchronize()
    from paper_1503_02198_amd.ssd import unpack_state
    return unpack_state(t.detach().cpu().numpy(), N, E).astype(np.float64)


def gpu_residual(gm, Q, theta, omega):
    import torch
    N, E = gm.info["N"], gm.info["n_elem"]
    q = to_gpu(Q, gm.device)
    r = torch.empty_like(q)
    gm.set_rotation(theta, omega)
    gm.mortar_rebuild()
    gm.residual(q, r)
    return from_gpu(r, N, E)


def gpu_run(gm, Q, t0, dt, nsteps, check=True, scheme="rk3"):
    import torch
    N, E = gm.info["N"], gm.info["n_elem"]
    q = to_gpu(Q, gm.device)
    work = torch.empty(gm.info["work_len"], dtype=torch.float32, device=q.device)
    for k in range(nsteps):
        gm.rk_step(q, work, t0 + k * dt, dt, scheme=scheme)
    if check:
        gm.check()
    return from_gpu(q, N, E)
