"""Pins of two oracle readings that the residual pins leave open.

* Galilean pin of the ALE Rusanov flux (Sec. 2.2 moving-grid fluxes, Sec.
  3.1 Rusanov solver).  On a face moving with velocity u_g, the ALE flux of
  the state Q equals the fixed-face flux of the state seen from the moving
  frame, Q' (velocity u - u_g), mapped back by the Galilean transformation
  G(u_g) of conservative variables:
      rho = rho',  m = m' + rho' u_g,  E = E' + u_g . m' + |u_g|^2 rho' / 2.
  G is linear, and the wave speed |u.n - u_g.n| + c equals |u'.n| + c, so
  the whole Rusanov flux obeys f*(QL, QR; n, u_g) = G f*(QL', QR'; n, 0).
  A wave speed that drops the grid velocity, or a flux that drops the
  u_g Q term, breaks it.

* Point-reflection pin of the viscous far field (Sec. 2.1 viscous fluxes,
  BR1 common values).  The reading: common solution Q_inf, common gradient
  the interior one.  Take the box [0, Lx] x [0, Ly] with far-field faces at
  x = 0 and x = Lx (periodic in y) and a state that depends on x only.
  Extend it to [-Lx, Lx] by the point reflection Q(-x) = 2 Q_inf - Q(x):
  all of the doubled box's faces at x = 0 are then conforming, and the
  discrete scheme is symmetric under the reflection, so there the mean of
  the two traces is exactly Q_inf and the mean of the two gradients is
  exactly the interior gradient.  The inviscid common fluxes differ
  (Rusanov against Q_inf, or against the reflected trace), so the pin
  compares the viscous part alone, R(mu) - R(0), on the cells of [0, Lx].
  The doubled box only uses the interior-face path, which the residual pins
  cover.

Each pin is shown to fail when a plausible mistake is planted in a copy of
the oracle.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle.ssd as ossd
from oracle import physics as ph
from oracle.ssd import SSD
from workloads import cases as C
from workloads import meshes as M


# ---------------------------------------------------------------- Galilean pin
def _galilean(F, ug, vg):
    """G(u_g) applied to conservative values (or fluxes) F."""
    return np.stack([F[0], F[1] + ug * F[0], F[2] + vg * F[0],
                     F[3] + ug * F[1] + vg * F[2] + 0.5 * (ug * ug + vg * vg) * F[0]])


def _random_faces(n=400, seed=3):
    rng = np.random.default_rng(seed)
    g = 1.4

    def state():
        return ph.conservative(rng.uniform(0.4, 2.0, n), rng.normal(0, 0.8, n),
                               rng.normal(0, 0.8, n), rng.uniform(0.3, 3.0, n), g)
    QL, QR = state(), state()
    nx, ny = rng.normal(0, 1.5, n), rng.normal(0, 1.5, n)   # not unit normals
    ug, vg = rng.normal(0, 0.7, n), rng.normal(0, 0.7, n)
    return g, QL, QR, nx, ny, ug, vg


def _shift(Q, ug, vg, g):
    rho, u, v, p = ph.primitives(Q, g)
    return ph.conservative(rho, u - ug, v - vg, p, g)


def _galilean_defect(rusanov):
    g, QL, QR, nx, ny, ug, vg = _random_faces()
    f_ale = rusanov(QL, QR, nx, ny, ug * nx + vg * ny, g)
    f_fix = rusanov(_shift(QL, ug, vg, g), _shift(QR, ug, vg, g), nx, ny, 0.0 * nx, g)
    return np.abs(f_ale - _galilean(f_fix, ug, vg)).max() / np.abs(f_ale).max()


def test_galilean_transformation_maps_conservative_values():
    """G(u_g) takes the state seen from the moving frame back to Q."""
    g, QL, _, _, _, ug, vg = _random_faces()
    assert np.abs(_galilean(_shift(QL, ug, vg, g), ug, vg) - QL).max() < 1e-13


def test_ale_rusanov_is_galilean_invariant():
    assert _galilean_defect(ph.rusanov) < 1e-13


def test_galilean_pin_catches_planted_mistakes():
    """The pin fails for a wave speed without the grid velocity and for a
    flux without the u_g Q term."""

    def no_grid_speed(QL, QR, nx, ny, vgn, gamma):
        mag = np.sqrt(nx * nx + ny * ny)
        fl = ph.normal_inviscid_flux(QL, nx, ny, vgn, gamma)
        fr = ph.normal_inviscid_flux(QR, nx, ny, vgn, gamma)
        _, ul, vl, _ = ph.primitives(QL, gamma)
        _, ur, vr, _ = ph.primitives(QR, gamma)
        lam = np.maximum(np.abs(ul * nx + vl * ny) + ph.sound_speed(QL, gamma) * mag,
                         np.abs(ur * nx + vr * ny) + ph.sound_speed(QR, gamma) * mag)
        return 0.5 * (fl + fr) - 0.5 * lam * (QR - QL)

    def no_grid_flux(QL, QR, nx, ny, vgn, gamma):
        return ph.rusanov(QL, QR, nx, ny, vgn, gamma) + 0.5 * vgn * (QL + QR)

    assert _galilean_defect(no_grid_speed) > 1e-3
    assert _galilean_defect(no_grid_flux) > 1e-3


# ---------------------------------------------------------------- far-field pin
def _viscous_case(mu):
    case = C.ellipse_viscous_case(omega=0.0)
    case["mu"] = mu
    return case


def _far_field_x(mesh):
    """The box with its x-periodic faces (local faces 1, 3) made far field."""
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in mesh.items()}
    kind, nbr, nf = out["face_kind"], out["nbr"], out["nbr_face"]
    for f in (1, 3):
        sel = kind[:, f] == M.FACE_PERIODIC
        kind[sel, f] = M.FACE_FARFIELD
        nbr[sel, f] = -1
        nf[sel, f] = -1
    return out


def _odd_state(x, case, Lx):
    """Q_inf + d(|x|) sign(x): the point reflection about (x = 0, Q_inf) of
    a smooth x-dependent state whose trace at x = 0 is not Q_inf."""
    g = case["gamma"]
    Qinf = ph.conservative(*case["farfield"], g)
    s = np.abs(x) / Lx
    rho0, u0, _, p0 = case["farfield"]
    d = np.stack([0.05 * rho0 * np.cos(1.3 * s + 0.4),
                  0.08 * np.sin(2.1 * s + 0.7),
                  0.06 * np.cos(1.7 * s - 0.2),
                  0.07 * p0 / (g - 1.0) * np.sin(1.1 * s + 1.0)])
    return Qinf[:, None, None, None] + np.sign(x)[None] * d


def _viscous_part(cls, mesh, N, Lx, shift=0.0):
    R = []
    for mu in (0.04, 0.0):
        case = _viscous_case(mu)
        o = cls(mesh, case, N)
        x, _ = o.sp_coords(0.0)
        R.append(o.residual(_odd_state(x + shift, case, Lx), 0.0, 0.0))
    return R[0] - R[1], o


def _far_field_defect(cls, N):
    nx, ny, Lx, Ly = 3, 2, 1.5, 1.0
    half = _far_field_x(M.box_mesh(nx, ny, L=(Lx, Ly)))
    full = _far_field_x(M.box_mesh(2 * nx, ny, L=(2 * Lx, Ly)))
    # the doubled box spans [-Lx, Lx]: its state is evaluated at x - Lx
    Vh, oh = _viscous_part(cls, half, N, Lx)
    Vf, of = _viscous_part(cls, full, N, Lx, shift=-Lx)
    ch, cf = oh.sp_coords(0.0), of.sp_coords(0.0)
    keyh = np.round(np.stack([ch[0].mean((0, 1)), ch[1].mean((0, 1))], 1), 9)
    keyf = {tuple(k): e for e, k in enumerate(np.round(np.stack([cf[0].mean((0, 1)) - Lx,
                                                                  cf[1].mean((0, 1))], 1), 9))}
    match = np.array([keyf[tuple(k)] for k in keyh])
    scale = np.abs(Vf[..., match]).max()
    assert scale > 1e-3   # the viscous terms carry weight
    return np.abs(Vh - Vf[..., match]).max() / scale


@pytest.mark.parametrize("N", [2, 3, 4])
def test_viscous_far_field_equals_point_reflection(N):
    assert _far_field_defect(SSD, N) < 1e-11


def _mutant(old, new):
    """A subclass of the oracle whose viscous pass has `old` replaced by
    `new` (a mistake planted in a copy, on the CPU)."""
    src = textwrap.dedent(inspect.getsource(SSD._viscous))
    assert old in src
    ns = dict(vars(ossd))
    exec(src.replace(old, new), ns)
    return type("Mutant", (SSD,), {"_viscous": ns["_viscous"]})


@pytest.mark.parametrize("old,new", [
    # common solution: the interior trace, or its mean with Q_inf
    ("Qc = np.where(far, Qinf, Qc)", "Qc = np.where(far, T, Qc)"),
    ("Qc = np.where(far, Qinf, Qc)", "Qc = np.where(far, 0.5 * (T + Qinf), Qc)"),
    # common gradient: the mean with a zero exterior gradient
    ("GXc = np.where(inter, 0.5 * (GX + GXn), GX)",
     "GXc = np.where(inter, 0.5 * (GX + GXn), np.where(far, 0.5 * GX, GX))"),
    # no viscous flux through the far field
    ("fv = np.where(slip, 0.0, fv)", "fv = np.where(slip | far, 0.0, fv)"),
])
def test_far_field_pin_catches_planted_mistakes(old, new):
    assert _far_field_defect(_mutant(old, new), 3) > 1e-4
