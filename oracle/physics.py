"""Fluxes of the 2-D compressible Navier-Stokes equations (Sec. 2).

State Q = [rho, rho u, rho v, E] with E = p/(gamma-1) + rho (u^2+v^2)/2
(eq. Q).  Arrays carry the 4 conservative variables on axis 0 and any
trailing shape.

Sec. 2.1: inviscid fluxes F_inv, G_inv; viscous fluxes
F_vis = -[0, tau_xx, tau_yx, u tau_xx + v tau_yx + k T_x] (and G_vis alike),
tau_ij = mu (u_i,j + u_j,i) + lambda delta_ij u_k,k with lambda = -2 mu / 3,
p = rho R T.  Sec. 2.2: on the rotating zone the inviscid fluxes lose
u_g Q and v_g Q.  Sec. 3.1: the common inviscid flux is the Rusanov flux.
"""
import numpy as np


def primitives(Q, gamma):
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho
    p = (gamma - 1.0) * (Q[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def inviscid_flux(Q, gamma):
    """(F_inv, G_inv), each shaped like Q."""
    rho, u, v, p = primitives(Q, gamma)
    F = np.stack([Q[1], Q[1] * u + p, Q[1] * v, (Q[3] + p) * u])
    G = np.stack([Q[2], Q[2] * u, Q[2] * v + p, (Q[3] + p) * v])
    return F, G


def normal_inviscid_flux(Q, nx, ny, vgn, gamma):
    """(F_inv - u_g Q) nx + (G_inv - v_g Q) ny, with vgn = u_g nx + v_g ny.

    (nx, ny) need not be a unit vector: the result scales with its length.
    """
    F, G = inviscid_flux(Q, gamma)
    return F * nx + G * ny - vgn * Q


def sound_speed(Q, gamma):
    rho, u, v, p = primitives(Q, gamma)
    return np.sqrt(gamma * p / rho)


def rusanov(QL, QR, nx, ny, vgn, gamma):
    """Rusanov flux along the (scaled) normal (nx, ny), from L towards R.

    f = (f_n(QL) + f_n(QR))/2 - lam |n| (QR - QL)/2, where
    lam = max over both sides of |u.n_hat - u_g.n_hat| + c.
    """
    mag = np.sqrt(nx * nx + ny * ny)
    fl = normal_inviscid_flux(QL, nx, ny, vgn, gamma)
    fr = normal_inviscid_flux(QR, nx, ny, vgn, gamma)
    _, ul, vl, _ = primitives(QL, gamma)
    _, ur, vr, _ = primitives(QR, gamma)
    lam_l = np.abs(ul * nx + vl * ny - vgn) + sound_speed(QL, gamma) * mag
    lam_r = np.abs(ur * nx + vr * ny - vgn) + sound_speed(QR, gamma) * mag
    lam = np.maximum(lam_l, lam_r)
    return 0.5 * (fl + fr) - 0.5 * lam * (QR - QL)


def primitive_gradients(Q, Qx, Qy, gamma, gas_R):
    """Gradients of u, v, T from conservative values and gradients."""
    rho, u, v, p = primitives(Q, gamma)
    out = []
    for d in (Qx, Qy):
        ud = (d[1] - u * d[0]) / rho
        vd = (d[2] - v * d[0]) / rho
        pd = (gamma - 1.0) * (d[3] - u * d[1] - v * d[2] + 0.5 * (u * u + v * v) * d[0])
        Td = (pd - p / rho * d[0]) / (rho * gas_R)
        out.append((ud, vd, Td))
    return out


def viscous_flux(Q, Qx, Qy, gamma, gas_R, mu, prandtl):
    """(F_vis, G_vis) of Sec. 2.1 with constant mu and k = mu cp / Pr."""
    rho, u, v, p = primitives(Q, gamma)
    (ux, vx, Tx), (uy, vy, Ty) = primitive_gradients(Q, Qx, Qy, gamma, gas_R)
    k = mu * gamma * gas_R / ((gamma - 1.0) * prandtl)
    lam = -2.0 / 3.0 * mu
    div = ux + vy
    txx = 2.0 * mu * ux + lam * div
    tyy = 2.0 * mu * vy + lam * div
    txy = mu * (uy + vx)
    z = np.zeros_like(rho)
    F = -np.stack([z, txx, txy, u * txx + v * txy + k * Tx])
    G = -np.stack([z, txy, tyy, u * txy + v * tyy + k * Ty])
    return F, G


def slip_state(Q, nx, ny, ug, vg, gamma):
    """Common solution of a slip wall (BR1 reading, Sec. 2): the trace Q
    with the velocity component normal to the wall, relative to the wall's
    own velocity (ug, vg), removed; density and pressure unchanged.  (nx,
    ny) is any nonzero normal."""
    rho, u, v, p = primitives(Q, gamma)
    mag = np.sqrt(nx * nx + ny * ny)
    nhx, nhy = nx / mag, ny / mag
    urel = (u - ug) * nhx + (v - vg) * nhy
    return conservative(rho, u - urel * nhx, v - urel * nhy, p, gamma)


def conservative(rho, u, v, p, gamma):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
