"""Pins of the oracle's flux functions (Sec. 2.1, 2.2, 3.1).

Checks are consistency and symmetry properties and closed-form special
cases: a consistent Rusanov flux, its antisymmetry, rotation covariance of
the Euler flux, zero viscous stress for rigid rotation, the stress of a pure
dilatation and a simple shear, and the Fourier heat flux.
"""
import numpy as np
import pytest

from oracle import physics as ph

G = 1.4


def _rand_state(rng, n):
    rho = rng.uniform(0.5, 2.0, n)
    u = rng.uniform(-1, 1, n)
    v = rng.uniform(-1, 1, n)
    p = rng.uniform(0.5, 2.0, n)
    return ph.conservative(rho, u, v, p, G)


def test_rusanov_consistency_and_antisymmetry():
    rng = np.random.default_rng(0)
    QL, QR = _rand_state(rng, 50), _rand_state(rng, 50)
    nx, ny = rng.standard_normal(50), rng.standard_normal(50)
    vgn = rng.standard_normal(50) * 0.3
    f_same = ph.rusanov(QL, QL, nx, ny, vgn, G)
    assert np.allclose(f_same, ph.normal_inviscid_flux(QL, nx, ny, vgn, G), atol=1e-13)
    a = ph.rusanov(QL, QR, nx, ny, vgn, G)
    b = ph.rusanov(QR, QL, -nx, -ny, -vgn, G)
    assert np.allclose(a, -b, atol=1e-13)
    # scaling of the normal scales the flux (per unit face parameter)
    c = ph.rusanov(QL, QR, 3 * nx, 3 * ny, 3 * vgn, G)
    assert np.allclose(c, 3 * a, atol=1e-12)


def test_euler_flux_closed_form_and_rotation():
    Q = ph.conservative(np.array([1.2]), np.array([0.3]), np.array([-0.4]), np.array([0.9]), G)
    F, Gf = ph.inviscid_flux(Q, G)
    E = 0.9 / 0.4 + 0.5 * 1.2 * 0.25
    assert np.allclose(F[:, 0], [1.2 * 0.3, 1.2 * 0.09 + 0.9, 1.2 * 0.3 * -0.4, (E + 0.9) * 0.3])
    assert np.allclose(Gf[:, 0], [1.2 * -0.4, 1.2 * 0.3 * -0.4, 1.2 * 0.16 + 0.9, (E + 0.9) * -0.4])
    # rotating the state and the normal rotates the normal flux's momentum
    rng = np.random.default_rng(1)
    Q = _rand_state(rng, 20)
    a = 0.7
    ca, sa = np.cos(a), np.sin(a)
    Qr = Q.copy()
    Qr[1], Qr[2] = ca * Q[1] - sa * Q[2], sa * Q[1] + ca * Q[2]
    nx, ny = rng.standard_normal(20), rng.standard_normal(20)
    f = ph.normal_inviscid_flux(Q, nx, ny, 0.0, G)
    fr = ph.normal_inviscid_flux(Qr, ca * nx - sa * ny, sa * nx + ca * ny, 0.0, G)
    assert np.allclose(fr[[0, 3]], f[[0, 3]], atol=1e-13)
    assert np.allclose(fr[1], ca * f[1] - sa * f[2], atol=1e-13)
    assert np.allclose(fr[2], sa * f[1] + ca * f[2], atol=1e-13)


def _grad_of(rho, u, v, p, drho, du, dv, dp):
    """Conservative gradient from primitive values and gradients."""
    E_d = dp / (G - 1) + 0.5 * drho * (u * u + v * v) + rho * (u * du + v * dv)
    return np.array([drho, drho * u + rho * du, drho * v + rho * dv, E_d])


@pytest.mark.parametrize("mu", [0.1, 2.0])
def test_viscous_flux_special_cases(mu):
    R, Pr = 3.0, 0.72
    rho, u, v, p = 1.3, 0.4, -0.2, 2.0
    Q = ph.conservative(np.array(rho), np.array(u), np.array(v), np.array(p), G)
    # rigid rotation u = -W y, v = W x: no strain, no stress
    W = 0.8
    Qx = _grad_of(rho, u, v, p, 0.0, 0.0, W, 0.0)
    Qy = _grad_of(rho, u, v, p, 0.0, -W, 0.0, 0.0)
    F, Gf = ph.viscous_flux(Q, Qx, Qy, G, R, mu, Pr)
    assert np.allclose(F, 0.0, atol=1e-13) and np.allclose(Gf, 0.0, atol=1e-13)
    # pure dilatation u_x = v_y = a at constant T: tau_xx = tau_yy = 2 mu a - 4/3 mu a
    a = 0.5
    Qx = _grad_of(rho, u, v, p, 0.0, a, 0.0, 0.0)
    Qy = _grad_of(rho, u, v, p, 0.0, 0.0, a, 0.0)
    # keep T constant: p_x = R T rho_x = 0 with rho_x = 0
    F, Gf = ph.viscous_flux(Q, Qx, Qy, G, R, mu, Pr)
    t = 2.0 / 3.0 * mu * a
    assert np.allclose(F, -np.array([0, t, 0, u * t]), atol=1e-13)
    assert np.allclose(Gf, -np.array([0, 0, t, v * t]), atol=1e-13)
    # simple shear u_y = s: tau_xy = mu s
    s = 1.7
    Qx = _grad_of(rho, u, v, p, 0.0, 0.0, 0.0, 0.0)
    Qy = _grad_of(rho, u, v, p, 0.0, s, 0.0, 0.0)
    F, Gf = ph.viscous_flux(Q, Qx, Qy, G, R, mu, Pr)
    assert np.allclose(F, -np.array([0, 0, mu * s, v * mu * s]), atol=1e-13)
    assert np.allclose(Gf, -np.array([0, mu * s, 0, u * mu * s]), atol=1e-13)
    # heat conduction: grad T = (Tx, 0) via a pressure gradient at fixed rho
    Tx = 0.25
    Qx = _grad_of(rho, u, v, p, 0.0, 0.0, 0.0, rho * R * Tx)
    Qy = _grad_of(rho, u, v, p, 0.0, 0.0, 0.0, 0.0)
    F, Gf = ph.viscous_flux(Q, Qx, Qy, G, R, mu, Pr)
    k = mu * G * R / ((G - 1) * Pr)
    assert np.allclose(F, -np.array([0, 0, 0, k * Tx]), atol=1e-12)
    assert np.allclose(Gf, 0.0, atol=1e-13)
