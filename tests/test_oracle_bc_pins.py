"""Pins of the oracle's viscous slip-wall and far-field readings (Sec. 2,
BR1 viscous treatment) against paths pinned elsewhere.

* Mirror pin (slip wall).  Take a periodic box and a flow with v = 0, u a
  function of y alone, and rho, p even about the lines y = 0 and y = Ly.
  On those lines the exact shear stress, normal stress and heat flux
  vanish, and the discrete scheme is symmetric.  So the lower half of the
  doubled, all-interior box [0, Lx] x [0, 2 Ly] (periodic both ways) must
  give the same residual as the box [0, Lx] x [0, Ly] whose y = 0 and
  y = Ly faces are slip walls.  The doubled box only uses the
  interior-face path, which the residual pins cover.
* Free-stream pins.  A uniform flow tangent to straight slip walls, with
  far-field ends carrying the same state, is an exact steady solution of
  the Navier-Stokes equations; the residual is zero to roundoff.
"""
import numpy as np
import pytest

from oracle import physics as ph
from oracle.ssd import SSD
from workloads import cases as C
from workloads import meshes as M


def _viscous_case(mu=0.05):
    case = C.ellipse_viscous_case(omega=0.0)
    case["mu"] = mu
    return case


def _with_boundaries(mesh, y_kind, x_kind=None):
    """The box with its y-periodic faces (local faces 0, 2) turned into
    y_kind boundaries and, with x_kind, its x-periodic faces (1, 3) too."""
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in mesh.items()}
    kind, nbr, nf = out["face_kind"], out["nbr"], out["nbr_face"]
    for faces, k in (((0, 2), y_kind), ((1, 3), x_kind)):
        if k is None:
            continue
        for f in faces:
            sel = kind[:, f] == M.FACE_PERIODIC
            kind[sel, f] = k
            nbr[sel, f] = -1
            nf[sel, f] = -1
    return out


def _state(ora, case, Lx, Ly, a=0.08, b=0.05, c=0.04):
    """v = 0; rho and u functions of y alone, even about y = 0 and y = Ly
    (so rho u is constant along x and the discrete du/dx, hence the normal
    viscous stress on those lines, is exactly zero); p, and with it the
    temperature, also varies along x."""
    x, y = ora.sp_coords(0.0)
    rho0, u0, _, p0 = case["farfield"]
    ey = np.cos(np.pi * y / Ly)
    rho = rho0 * (1.0 + b * ey)
    u = u0 * (1.0 + a * ey)
    p = p0 * (1.0 + c * np.cos(2 * np.pi * x / Lx) * np.cos(2 * np.pi * y / Ly))
    return ph.conservative(rho, u, np.zeros_like(u), p, case["gamma"])


@pytest.mark.parametrize("N", [2, 3, 4])
def test_slip_wall_equals_mirror_plane(N):
    case = _viscous_case()
    nx, ny, Lx, Ly = 4, 3, 2.0, 1.5
    half = _with_boundaries(M.box_mesh(nx, ny, L=(Lx, Ly)), M.FACE_WALL_SLIP)
    full = M.box_mesh(nx, 2 * ny, L=(Lx, 2 * Ly))
    oh, of = SSD(half, case, N), SSD(full, case, N)
    Rh = oh.residual(_state(oh, case, Lx, Ly), 0.0, 0.0)
    Rf = of.residual(_state(of, case, Lx, Ly), 0.0, 0.0)
    # element of the doubled box at the same place as each element of the half box
    ch = oh.sp_coords(0.0)
    cf = of.sp_coords(0.0)
    keyh = np.round(np.stack([ch[0].mean((0, 1)), ch[1].mean((0, 1))], 1), 9)
    keyf = {tuple(k): e for e, k in enumerate(np.round(np.stack([cf[0].mean((0, 1)),
                                                                  cf[1].mean((0, 1))], 1), 9))}
    match = np.array([keyf[tuple(k)] for k in keyh])
    scale = np.abs(Rf).max()
    assert scale > 1e-3   # the flow is not steady: the comparison has content
    err = np.abs(Rh - Rf[..., match]).max() / scale
    assert err < 1e-11, err


def test_mirror_pin_sees_the_viscous_terms():
    """The same comparison with mu = 0 differs from the viscous one: the
    viscous terms carry weight in the mirror pin."""
    nx, ny, Lx, Ly, N = 4, 3, 2.0, 1.5, 3
    mesh = _with_boundaries(M.box_mesh(nx, ny, L=(Lx, Ly)), M.FACE_WALL_SLIP)
    R = []
    for mu in (0.05, 0.0):
        case = _viscous_case(mu)
        o = SSD(mesh, case, N)
        R.append(o.residual(_state(o, case, Lx, Ly), 0.0, 0.0))
    assert np.abs(R[0] - R[1]).max() > 1e-3 * np.abs(R[0]).max()


@pytest.mark.parametrize("N", [2, 4])
@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_free_stream_between_slip_walls_and_far_field(N, mu):
    case = _viscous_case(mu)
    mesh = _with_boundaries(M.box_mesh(5, 4, L=(2.0, 1.0), distort=0.2), M.FACE_WALL_SLIP,
                            M.FACE_FARFIELD)
    ora = SSD(mesh, case, N)
    rho0, u0, v0, p0 = case["farfield"]
    assert v0 == 0.0 and u0 != 0.0
    x, _ = ora.sp_coords(0.0)
    one = np.ones_like(x)
    Q = ph.conservative(rho0 * one, u0 * one, 0.0 * one, p0 * one, case["gamma"])
    R, diag = ora.residual(Q, 0.0, 0.0, diag=True)
    assert np.abs(R).max() < 1e-12 * max(1.0, np.abs(diag["flux_scale"]).max())


def test_slip_state_properties():
    """The slip common solution is fixed by what it must satisfy: zero
    velocity normal to the wall relative to the wall, with density, pressure
    and the tangential relative velocity unchanged.  It is idempotent, does
    not depend on the normal's length or sign, and leaves a state that
    already moves with the wall unchanged."""
    rng = np.random.default_rng(11)
    g = 1.4
    n = 200
    rho = rng.uniform(0.5, 2.0, n)
    u, v = rng.normal(0, 1, n), rng.normal(0, 1, n)
    p = rng.uniform(0.3, 3.0, n)
    Q = ph.conservative(rho, u, v, p, g)
    nx, ny = rng.normal(0, 1, n), rng.normal(0, 1, n)
    ug, vg = rng.normal(0, 0.5, n), rng.normal(0, 0.5, n)
    S = ph.slip_state(Q, nx, ny, ug, vg, g)
    r2, u2, v2, p2 = ph.primitives(S, g)
    mag = np.hypot(nx, ny)
    tx, ty = -ny / mag, nx / mag
    assert np.allclose(((u2 - ug) * nx + (v2 - vg) * ny) / mag, 0.0, atol=1e-13)
    assert np.allclose(r2, rho, rtol=1e-14) and np.allclose(p2, p, rtol=1e-12)
    assert np.allclose((u2 - ug) * tx + (v2 - vg) * ty, (u - ug) * tx + (v - vg) * ty, atol=1e-13)
    assert np.allclose(ph.slip_state(S, nx, ny, ug, vg, g), S, atol=1e-13)
    assert np.allclose(ph.slip_state(Q, -3.0 * nx, -3.0 * ny, ug, vg, g), S, atol=1e-13)
    # a state moving with the wall plus any tangential velocity is unchanged
    w = rng.normal(0, 1, n)
    Qt = ph.conservative(rho, ug + w * tx, vg + w * ty, p, g)
    assert np.allclose(ph.slip_state(Qt, nx, ny, ug, vg, g), Qt, atol=1e-13)
