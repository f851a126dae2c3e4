"""Pins of the oracle's residual, mortar and time stepping (Sec. 3, Sec. 4).

- free-stream preservation on fixed, distorted and rotating cells;
- conservation across the sliding interface (Sec. 3.2; Kopriva's mortar
  argument): the integral of dQ/dt vanishes on a periodic domain;
- invariance under relabelling of element corners (orientation bookkeeping)
  and covariance under a rigid rotation of the whole problem;
- the mortar at zero offset reduces to a pointwise Rusanov flux across the
  matching faces; continuity of the residual as the offset wraps;
- truncation error of the exact vortex and Taylor-Couette solutions decays
  with refinement; the exact vortex (the workload's and the paper's own
  parameters) solves the Euler equations;
- on the paper's own vortex test (Sec. 4.1) the oracle converges at the
  orders of Table 1 and Table 2 (tests/golden/paper_tables.json) to within
  0.2, on three levels;
- SSP-RK3 is third order.
"""
import json
import os

import numpy as np
import pytest

from oracle import physics as ph
from oracle.exact import Couette, vortex_state
from oracle.ssd import SSD, submesh
from workloads import cases as C
from workloads import meshes as M

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _wl2(s, e):
    w = s.ops.w
    W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(s.geo.detJ, 0, 2)
    return np.array([np.sqrt((W * e[v] ** 2).sum() / W.sum()) for v in range(4)])


# ---------------------------------------------------------------- free stream
@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_freestream_fixed_box(N):
    case = C.vortex_case()
    mesh = M.box_mesh(6, 5, distort=0.2)
    s = SSD(mesh, case, N)
    R = s.residual(C.uniform_state(case, N, s.E, v=0.2), 0.0, 0.0)
    assert np.abs(R).max() < 1e-11
    if N >= 3:   # cubic cells: metrics of degree 3 <= N
        mesh = M.box_mesh(6, 5, distort=0.2, curved=0.08)
        s = SSD(mesh, case, N)
        R = s.residual(C.uniform_state(case, N, s.E, v=0.2), 0.0, 0.0)
        assert np.abs(R).max() < 1e-11


@pytest.mark.parametrize("N", [2, 3, 4])
def test_freestream_rotating_box(N):
    """A whole rotating zone of bilinear cells (2 p_g <= N)."""
    case = C.vortex_case()
    mesh = M.box_mesh(6, 5, distort=0.2, zone=1)
    s = SSD(mesh, case, N)
    R = s.residual(C.uniform_state(case, N, s.E, v=-0.3), 0.4, 1.3)
    assert np.abs(R).max() < 1e-11


@pytest.mark.parametrize("N", [2, 3, 4])
def test_freestream_sliding_mesh(N):
    """Exact in every cell away from the interface; at interface cells the
    exact-circle mortar differs from the cells' cubic faces by a geometric
    error that converges with refinement: at the order of the face
    polynomials' fit to the circle, measured 1.0-1.1 in the residual at
    N = 2 and 2.0-2.1 at N = 3, 4 (h -> h/2 -> h/4).  A geometry error that
    does not shrink with h (a wrong mortar angle or offset) fails this."""
    case = C.vortex_case(omega=0.5)
    errs = []
    for f in (1, 4):
        mesh = M.vortex_mesh(f)
        s = SSD(mesh, case, N)
        R = s.residual(C.uniform_state(case, N, s.E), 0.17, 0.5)
        em = np.abs(R).max(axis=(0, 1, 2))
        sl = np.any(mesh["face_kind"] == M.FACE_SLIDING, axis=1)
        assert em[~sl].max() < 1e-11
        errs.append(em[sl].max())
    order = np.log(errs[0] / errs[1]) / np.log(4.0)
    assert order >= (0.9 if N == 2 else 1.8), (errs, order)


# ---------------------------------------------------------------- conservation
def _vortex_setup(N, f=1, omega=0.5, theta0=0.0):
    case = C.vortex_case(omega=omega, theta0=theta0)
    s = SSD(M.vortex_mesh(f), case, N)
    x, y = s.sp_coords(theta0)
    return case, s, vortex_state(x, y, 0.0, case)


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("theta", [0.0, 0.05, 0.1963495408, 0.31, -0.77])
def test_conservation_across_interface(N, theta):
    case, s, Q = _vortex_setup(N)
    R = s.residual(Q, theta, 0.5)
    tot = s.integrate(R)
    scale = s.integrate(np.abs(R))
    assert np.all(np.abs(tot) <= 1e-12 * scale)


def test_conservation_over_rk_steps():
    case, s, Q = _vortex_setup(3, omega=0.5, theta0=2 * np.pi / 32 - 0.02)
    m0 = s.integrate(Q)
    Q = s.run(Q, 0.0, 2e-2, 5)           # delta wraps within these steps
    assert np.allclose(s.integrate(Q), m0, rtol=0, atol=1e-13 * np.abs(m0).max())


# ---------------------------------------------------------- orientation, frame
def _relabel_state(Q, shifts):
    """State on the relabelled mesh.  One quarter-turn relabelling gives old
    coordinates xi = 1 - eta', eta = xi'; it is applied `shift` times."""
    out = Q.copy()
    for e, k in enumerate(shifts):
        a = Q[:, :, :, e]
        for _ in range(k % 4):
            # new[j', i'] = old[i', N-1-j']  (old xi = 1 - eta', old eta = xi')
            a = np.transpose(a, (0, 2, 1))[:, ::-1, :]
        out[:, :, :, e] = a
    return out


@pytest.mark.parametrize("meshname", ["vortex", "couette"])
def test_relabel_invariance(meshname):
    rng = np.random.default_rng(3)
    if meshname == "vortex":
        case, s, Q = _vortex_setup(3, omega=0.5)
        mesh = M.vortex_mesh(1)
    else:
        case = C.couette_case()
        mesh = M.couette_mesh(4, 16, phi_offset=0.4 * 2 * np.pi / 16)
        s = SSD(mesh, case, 3)
        x, y = s.sp_coords(0.0)
        Q = Couette(case).state(x, y)
        Q[0] *= 1 + 0.01 * np.sin(3 * x) * np.cos(2 * y)
    shifts = rng.integers(0, 4, s.E)
    m2 = M.relabel(mesh, shifts)
    s2 = SSD(m2, case, 3)
    Q2 = _relabel_state(Q, shifts)
    for th in (0.0, 0.123):
        R = s.residual(Q, th, case["omega"])
        R2 = s2.residual(Q2, th, case["omega"])
        assert np.allclose(_relabel_state(R, shifts), R2, rtol=0, atol=1e-10 * np.abs(R).max())


def test_rotation_covariance():
    case, s, Q = _vortex_setup(3, omega=0.7)
    a = 0.37
    mesh2 = M.rotate_mesh(M.vortex_mesh(1), a)
    s2 = SSD(mesh2, case, 3)
    ca, sa = np.cos(a), np.sin(a)

    def rot(A):
        B = A.copy()
        B[1], B[2] = ca * A[1] - sa * A[2], sa * A[1] + ca * A[2]
        return B
    R = s.residual(Q, 0.21, 0.7)
    R2 = s2.residual(rot(Q), 0.21, 0.7)
    assert np.allclose(rot(R), R2, rtol=0, atol=1e-10 * np.abs(R).max())


# ------------------------------------------------------------- mortar special
def test_mortar_zero_offset_is_pointwise_rusanov():
    case, s, Q = _vortex_setup(3, omega=0.5)
    itf = s.iface
    m, dlt, thL, thR = itf.placement(0.0)
    assert dlt == 0.0 or dlt > 1 - 1e-12 or dlt < 1e-12
    _, diag = s.residual(Q, 0.0, 0.5, diag=True)
    fs = diag["face_flux"]
    # traces: re-interpolate each side's face values directly
    q = np.moveaxis(Q, 3, 1)
    I = s.ops.I
    qxi = np.einsum("ki,veji->vejk", I, q)
    qeta = np.einsum("kj,veji->veki", I, q)
    T = s._faces(qxi, qeta, s.N)
    TL, TR = itf.canon(itf.L, T), itf.canon(itf.Rt, T)
    if dlt > 0.5:
        m = (m + 1) % itf.K
    TRm = TR[:, (np.arange(itf.K) + m) % itf.K]
    phi = itf.face_angles(itf.L, thL)
    sc = itf.R * itf.delta
    f = ph.rusanov(TL, TRm, np.cos(phi) * sc, np.sin(phi) * sc, 0.0, case["gamma"])
    got = itf.canon(itf.L, fs)
    assert np.allclose(got, f, rtol=0, atol=1e-11)


def test_residual_continuous_across_wrap():
    case, s, Q = _vortex_setup(3, omega=0.5)
    D = s.iface.delta
    R1 = s.residual(Q, D * (1 - 1e-9), 0.5)
    R2 = s.residual(Q, D * (1 + 1e-9), 0.5)
    m1 = s.iface.placement(D * (1 - 1e-9))[0]
    m2 = s.iface.placement(D * (1 + 1e-9))[0]
    assert m1 != m2
    assert np.abs(R1 - R2).max() < 1e-6 * np.abs(R1).max()


# ------------------------------------------------------------ exact vortex
@pytest.mark.parametrize("case_fn", [C.vortex_case, C.paper_vortex_case])
def test_vortex_state_solves_euler(case_fn):
    """The exact vortex (Sec. 4.1) with the workload's parameters and with
    the paper's own (epsilon = 1, Mach 0.3, mean flow at arctan(1/2)): the
    Euler equations dQ/dt + dF/dx + dG/dy = 0 hold at random points, by
    fourth-order central differences in x, y and t of the closed form."""
    case = case_fn()
    g = case["gamma"]
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-2.5, 2.5, (2, 200))
    t, h = 0.37, 1e-3

    def d(fn, k):
        e = np.zeros(3)
        e[k] = h
        a = lambda s: fn(x + s * e[0], y + s * e[1], t + s * e[2])
        return (8 * (a(1) - a(-1)) - (a(2) - a(-2))) / (12 * h)
    Q = lambda xx, yy, tt: vortex_state(xx, yy, tt, case)
    F = lambda xx, yy, tt: ph.inviscid_flux(Q(xx, yy, tt), g)[0]
    G = lambda xx, yy, tt: ph.inviscid_flux(Q(xx, yy, tt), g)[1]
    res = d(Q, 2) + d(F, 0) + d(G, 1)
    scale = np.abs(d(F, 0)).max(axis=1)
    assert np.all(np.abs(res).max(axis=1) < 1e-7 * scale), np.abs(res).max(axis=1) / scale
    # the vortex moves with the mean flow: at the centre after time t the
    # velocity is the far-field velocity and the density is at its minimum
    rho_inf, u_inf, v_inf, _ = case["farfield"]
    xc, yc = np.array(case["vortex"]["center"]) + t * np.array([u_inf, v_inf])
    q = Q(np.array([xc]), np.array([yc]), t)
    assert abs(q[1, 0] / q[0, 0] - u_inf) < 1e-12 and abs(q[2, 0] / q[0, 0] - v_inf) < 1e-12
    ring = Q(xc + 0.3 * np.cos(np.linspace(0, 6, 7)), yc + 0.3 * np.sin(np.linspace(0, 6, 7)), t)
    assert np.all(ring[0] > q[0, 0])


# ------------------------------------------------------------ truncation error
@pytest.mark.parametrize("N,min_order", [(3, 1.4), (4, 2.2)])
def test_vortex_truncation_error_decays(N, min_order):
    case = C.vortex_case(omega=1.0)
    errs = []
    for f in (1, 2):
        s = SSD(M.vortex_mesh(f), case, N)
        t, h = 0.3, 1e-5

        def qat(tt):
            x, y = s.sp_coords(s.theta(tt))
            return vortex_state(x, y, tt, case)
        dQ = (qat(t + h) - qat(t - h)) / (2 * h)     # d/dt following the SPs
        R = s.residual(qat(t), s.theta(t), case["omega"])
        errs.append(_wl2(s, R - dQ))
    order = np.log2(errs[0] / errs[1])
    assert np.all(order > min_order), order
    assert np.all(errs[1] < 3e-3)


@pytest.mark.parametrize("N,min_order", [(2, 0.6), (3, 2.0), (4, 2.2)])
def test_couette_truncation_error_decays(N, min_order):
    """Exact steady compressible Couette state (viscous path, isothermal
    walls, viscous mortar at a non-zero offset)."""
    case = C.couette_case()
    ex = Couette(case)
    errs = []
    for nr in (4, 8):
        mesh = M.couette_mesh(nr, 4 * nr, phi_offset=0.3 * 2 * np.pi / (4 * nr))
        s = SSD(mesh, case, N)
        th, h = 0.2, 1e-5

        def qat(tt):
            x, y = s.sp_coords(tt)
            return ex.state(x, y)
        dQ = (qat(th + h) - qat(th - h)) / (2 * h)
        R = s.residual(qat(th), th, case["omega"])
        errs.append(_wl2(s, R - dQ))
    order = np.log2(errs[0] / errs[1])
    assert np.all(order > min_order), order


def test_couette_mass_conservation():
    case = C.couette_case()
    mesh = M.couette_mesh(4, 16, phi_offset=0.27)
    s = SSD(mesh, case, 3)
    x, y = s.sp_coords(0.0)
    Q = Couette(case).state(x, y)
    Q[0] *= 1 + 0.02 * np.sin(2 * x + y)
    R = s.residual(Q, 0.31, 1.0)
    tot = s.integrate(R)
    assert abs(tot[0]) < 1e-12 * s.integrate(np.abs(R))[0]


# ------------------------------------------------------------------ time order
def test_ssprk3_third_order():
    class Lin(SSD):
        def __init__(self, lam):
            self.lam = lam
            self.case = dict(theta0=0.0, omega=0.0)

        def residual(self, Q, theta, omega, diag=False):
            return self.lam * Q
    lam = -1.3
    s = Lin(lam)
    errs = []
    for n in (10, 20, 40):
        Q = np.array([1.0])
        Q = s.run(Q, 0.0, 1.0 / n, n)
        errs.append(abs(Q[0] - np.exp(lam)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.15), orders


class _Riccati(SSD):
    """y' = -2 t y^2, y(0) = 1: y = 1 / (1 + t^2).  Nonlinear and explicitly
    time dependent (through the rotor angle theta = t), so it checks the
    nonlinear order conditions and the stage times of a scheme."""

    def __init__(self):
        self.case = dict(theta0=0.0, omega=1.0)

    def residual(self, Q, theta, omega, diag=False):
        return -2.0 * theta * Q * Q


@pytest.mark.parametrize("scheme,order", [("rk3", 3.0), ("rk54", 4.0)])
def test_ssprk_order_nonlinear_time_dependent(scheme, order):
    s = _Riccati()
    errs = []
    for n in (8, 16, 32, 64):
        Q = s.run(np.array([1.0]), 0.0, 2.0 / n, n, scheme=scheme)
        errs.append(abs(Q[0] - 1.0 / 5.0))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders[1:] - order) < 0.25), orders


def test_ssprk54_coefficients():
    """Consistency of the Shu-Osher form: each stage is a convex combination
    plus a time step, the final combination sums to one, and the stage
    times lie in [0, 1]."""
    from oracle.ssd import SSPRK54, ssprk54_stage_times
    a, c = SSPRK54["a"], SSPRK54["c"]
    for k in (1, 2, 3):
        assert abs(a[k][0] + a[k][1] - 1.0) < 1e-14
    assert abs(c[0] + c[1] + c[3] - 1.0) < 1e-14
    assert all(x >= 0.0 for row in a for x in row) and all(x >= 0.0 for x in c)
    tau = ssprk54_stage_times()
    assert all(0.0 <= x <= 1.0 for x in tau)
    # the update is exact for L = 1 (dU/dt = 1): U^{n+1} = U + dt
    U = 0.0
    L = lambda V: 1.0
    U1 = U + a[0][2] * L(U)
    U2 = a[1][0] * U + a[1][1] * U1 + a[1][2] * L(U1)
    U3 = a[2][0] * U + a[2][1] * U2 + a[2][2] * L(U2)
    U4 = a[3][0] * U + a[3][1] * U3 + a[3][2] * L(U3)
    U5 = c[0] * U2 + c[1] * U3 + c[2] * L(U3) + c[3] * U4 + c[4] * L(U4)
    assert abs(U5 - 1.0) < 1e-14
    # the stage values are the stage times for dU/dt = 1
    assert np.allclose([U1, U2, U3, U4], tau[1:], atol=1e-14)


# ---------------------------------------------------------------- convergence
def _vortex_errors(N, fs, T, dt0):
    case = C.vortex_case(omega=1.0)
    out = []
    for f in fs:
        s = SSD(M.vortex_mesh(f), case, N)
        x, y = s.sp_coords(0.0)
        Q = vortex_state(x, y, 0.0, case)
        n = int(round(T / (dt0 / f)))
        Q = s.run(Q, 0.0, T / n, n)
        xT, yT = s.sp_coords(s.theta(T))
        e = Q[0] - vortex_state(xT, yT, T, case)[0]
        w = s.ops.w
        W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(s.geo.detJ, 0, 2)
        out.append(((W * np.abs(e)).sum() / W.sum(), np.sqrt((W * e * e).sum() / W.sum())))
    return np.array(out)


def _paper_orders(table):
    with open(GOLD) as fh:
        g = json.load(fh)[table]
    return np.array([[r["L1_order"], r["L2_order"]] for r in g["rows"] if r["L1_order"] is not None])


@pytest.mark.parametrize("N,table,T,dt0,slack", [(3, "table1_vortex_N3", 0.2, 0.01, 0.75),
                                                  (4, "table2_vortex_N4", 0.2, 0.004, 1.1)])
def test_vortex_convergence_two_levels(N, table, T, dt0, slack):
    """Density error order on 384 -> 1536 cells against Table 1 / Table 2."""
    e = _vortex_errors(N, (1, 2), T, dt0)
    order = np.log2(e[0] / e[1])
    paper = _paper_orders(table).min(axis=0)
    assert np.all(order > paper - slack), (order, paper)


# The paper's own vortex test (Sec. 4.1: epsilon 1, Mach 0.3, mean flow at
# arctan(1/2), omega 1, errors at t = 2) on three levels of the vortex mesh
# family, from tests/golden/paper_vortex_errors_oracle.json (written by
# tests/golden/make_paper_vortex_errors.py from the oracle alone, about 40
# minutes of CPU); the cheapest level is recomputed here to pin the file to
# the oracle as it stands.
PAPER_ORACLE = os.path.join(os.path.dirname(__file__), "golden", "paper_vortex_errors_oracle.json")


def _paper_runs():
    with open(PAPER_ORACLE) as fh:
        return json.load(fh)


def _paper_vortex_orders(N):
    runs = sorted((r for r in _paper_runs()["runs"] if r["N"] == N), key=lambda r: r["f"])
    assert [r["f"] for r in runs] == [1, 2, 3]
    e = np.array([[r["L1"], r["L2"]] for r in runs])
    f = np.array([r["f"] for r in runs], dtype=float)
    pairs = np.log(e[:-1] / e[1:]) / np.log(f[1:] / f[:-1])[:, None]
    whole = np.log(e[0] / e[-1]) / np.log(f[-1] / f[0])
    return pairs, whole


def test_paper_vortex_orders_n3():
    """N = 3 on 384, 1,536 and 3,456 cells: both refinements' orders, L1 and
    L2, within 0.2 of Table 1's two."""
    pairs, _ = _paper_vortex_orders(3)
    paper = _paper_orders("table1_vortex_N3")
    print("orders (L1, L2):", pairs.tolist(), "Table 1:", paper.tolist())
    assert np.all(np.abs(pairs - paper) <= 0.2), (pairs, paper)


def test_paper_vortex_orders_n4():
    """N = 4 on the same levels: the order over the whole range (384 to
    3,456 cells) within 0.2 of both of Table 2's orders.  Refinement by
    refinement it is not: the 384-cell level is not yet asymptotic at N = 4,
    so the first refinement falls short of 4 and the second exceeds it (3.91
    and 4.43 in L1, 3.65 and 4.46 in L2); the pairs are printed, not
    asserted."""
    pairs, whole = _paper_vortex_orders(4)
    paper = _paper_orders("table2_vortex_N4")
    print("orders (L1, L2):", pairs.tolist(), "whole range:", whole.tolist(),
          "Table 2:", paper.tolist())
    assert np.all(np.abs(whole - paper) <= 0.2), (whole, paper)


def test_paper_vortex_stored_level_reproduces():
    """N = 3 on 384 cells to t = 2 (500 SSP-RK3 steps) gives the stored
    errors."""
    from oracle.exact import vortex_state as vs
    g = _paper_runs()
    r = [r for r in g["runs"] if r["N"] == 3 and r["f"] == 1][0]
    case = C.paper_vortex_case()
    s = SSD(M.vortex_mesh(1), case, 3)
    x, y = s.sp_coords(0.0)
    T = g["T"]
    n = r["steps"]
    Q = s.run(vs(x, y, 0.0, case), 0.0, T / n, n)
    xT, yT = s.sp_coords(s.theta(T))
    e = Q[0] - vs(xT, yT, T, case)[0]
    w = s.ops.w
    W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(s.geo.detJ, 0, 2)
    l1 = (W * np.abs(e)).sum() / W.sum()
    l2 = np.sqrt((W * e * e).sum() / W.sum())
    assert np.allclose([l1, l2], [r["L1"], r["L2"]], rtol=1e-9, atol=0), ([l1, l2], r)


# ---------------------------------------------------------------- sub-meshes
def test_submesh_matches_full_residual():
    case, s, Q = _vortex_setup(3, omega=0.5)
    R = s.residual(Q, 0.08, 0.5)
    mesh = M.vortex_mesh(1)
    pick = np.array([0, 17, 100, 250, 300, 383])
    sub, idx = submesh(mesh, pick, depth=1)
    s2 = SSD(sub, case, 3)
    R2 = s2.residual(Q[..., idx], 0.08, 0.5)
    loc = np.searchsorted(idx, pick)
    assert np.allclose(R2[..., loc], R[..., pick], rtol=0, atol=1e-12)
