"""Physical parameters of the workloads and seeded initial states.

A case dict carries the gas constants, the motion of the rotating zone and
the boundary data:

  gamma, gas_R, mu, prandtl   ratio of specific heats, gas constant,
                              dynamic viscosity (0 -> Euler), Prandtl number
  T_wall                      temperature of isothermal walls
  farfield                    (rho, u, v, p) of far-field faces
  omega, theta0               rotation rate of zone 1 and its angle at t=0

Nondimensionalisation: reference density, speed and temperature are 1,
so p_ref = 1 / (gamma M^2) and gas_R = p_ref.
"""
import numpy as np

from .rng import uniform_pm1

GAMMA = 1.4


def vortex_case(omega=0.5, theta0=0.0):
    """Isentropic vortex transport on the periodic square with a rotating
    disk: freestream Mach 0.5 along x, rho = p = 1 (so T = 1, R = 1)."""
    return dict(gamma=GAMMA, gas_R=1.0, mu=0.0, prandtl=0.72, T_wall=1.0,
                farfield=(1.0, 0.5 * np.sqrt(GAMMA), 0.0, 1.0),
                omega=float(omega), theta0=float(theta0),
                vortex=dict(beta=5.0, mach=0.5, center=(0.0, 0.0), period=10.0))


def paper_vortex_case(omega=1.0, theta0=0.0, mach=0.3, epsilon=1.0, direction=np.arctan(0.5)):
    """The paper's own vortex test (Sec. 4.1): U = rho = 1, Mach 0.3, mean
    flow at angle arctan(1/2), strength epsilon = 1, r_c = 1, period 10,
    inner disk rotating at omega = 1.  The printed p = 1 would make the
    Mach number 0.85; p = 1 / (gamma M^2) keeps M = 0.3 (so T = 1 with
    R = p)."""
    p = 1.0 / (GAMMA * mach ** 2)
    return dict(gamma=GAMMA, gas_R=p, mu=0.0, prandtl=0.72, T_wall=1.0,
                farfield=(1.0, float(np.cos(direction)), float(np.sin(direction)), p),
                omega=float(omega), theta0=float(theta0),
                vortex=dict(epsilon=float(epsilon), center=(0.0, 0.0), period=10.0))


def couette_case(mach_wall=0.1, reynolds=10.0, prandtl=0.72, omega=1.0, r_in=1.0):
    """Taylor-Couette flow: inner wall speed omega*r_in = 1 at Mach
    `mach_wall`, Re based on r_in and the wall speed, constant viscosity."""
    u_wall = omega * r_in
    p_ref = 1.0 / (GAMMA * mach_wall ** 2) * u_wall ** 2
    return dict(gamma=GAMMA, gas_R=p_ref, mu=u_wall * r_in / reynolds, prandtl=prandtl,
                T_wall=1.0, farfield=(1.0, 0.0, 0.0, p_ref), omega=float(omega), theta0=0.0)


def ellipse_case(mach=0.3, omega=1.0):
    """Inviscid flow past the rotating ellipse: rho = 1, u = M, c = 1."""
    return dict(gamma=GAMMA, gas_R=1.0 / GAMMA, mu=0.0, prandtl=0.72, T_wall=1.0,
                farfield=(1.0, mach, 0.0, 1.0 / GAMMA), omega=float(omega), theta0=0.0)


def ellipse_viscous_case(mach=0.2, reynolds=1000.0, omega=1.0, prandtl=0.72):
    """Viscous flow past the rotating ellipse: far field (1, mach, 0, 1/gamma),
    so that the speed of sound is 1; Re based on the major axis (length 1)
    and the free-stream speed; isothermal walls at the free-stream
    temperature."""
    return dict(gamma=GAMMA, gas_R=1.0 / GAMMA, mu=mach / reynolds, prandtl=prandtl, T_wall=1.0,
                farfield=(1.0, mach, 0.0, 1.0 / GAMMA), omega=float(omega), theta0=0.0)


def perturbed_farfield_state(case, N, E, seed=20150307, amplitude=0.01):
    """Conservative state [4][N][N][E] (float64): the far-field state with
    density scaled by (1 + amplitude * u), u uniform on [-1, 1) drawn by
    SplitMix64 from `seed` at counter (e*N + j)*N + i for solution point
    (i, j) of element e.  Velocity and pressure are left unchanged."""
    rho0, u, v, p = case["farfield"]
    g = case["gamma"]
    e = np.arange(E, dtype=np.uint64)
    jj, ii = np.meshgrid(np.arange(N, dtype=np.uint64), np.arange(N, dtype=np.uint64), indexing="ij")
    idx = (e[None, None, :] * np.uint64(N) + jj[:, :, None]) * np.uint64(N) + ii[:, :, None]
    rho = rho0 * (1.0 + amplitude * uniform_pm1(seed, idx))
    Q = np.empty((4, N, N, E))
    Q[0] = rho
    Q[1] = rho * u
    Q[2] = rho * v
    Q[3] = p / (g - 1.0) + 0.5 * rho * (u * u + v * v)
    return Q


def uniform_state(case, N, E, rho=None, u=None, v=None, p=None):
    """Uniform conservative state [4][N][N][E] (float64)."""
    r0, u0, v0, p0 = case["farfield"]
    rho = r0 if rho is None else rho
    u = u0 if u is None else u
    v = v0 if v is None else v
    p = p0 if p is None else p
    g = case["gamma"]
    Q = np.empty((4, N, N, E))
    Q[0] = rho
    Q[1] = rho * u
    Q[2] = rho * v
    Q[3] = p / (g - 1.0) + 0.5 * rho * (u * u + v * v)
    return Q
