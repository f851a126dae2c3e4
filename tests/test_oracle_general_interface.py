"""Pins of the oracle's general sliding interface (rings of different face
counts, non-uniform faces): on uniform rings it equals the uniform
(m, delta) construction; its mortars tile the circle within their faces; it
conserves flux across the interface; and for a smooth state continuous
across the interface its face fluxes converge to the exact normal flux."""
import numpy as np
import pytest

from oracle import physics as ph
from oracle.ssd import SSD, GeneralInterface
from workloads import cases as C
from workloads import meshes as M


def _mesh(K=16, K_out=24, warp=0.3, n=2):
    return M.ellipse_mesh(K=K, n_in=n, n_out=n, radius=1.5, box_half=4.0, first_in=0.1,
                          first_out=0.2, tile=None, K_out=K_out, warp=warp)


def test_equals_uniform_construction_on_uniform_rings():
    case = C.ellipse_case()
    mesh = _mesh(K_out=16, warp=0.0)
    Q = C.perturbed_farfield_state(case, 3, len(mesh["zone"]), amplitude=0.05)
    uni, gen = SSD(mesh, case, 3), SSD(mesh, case, 3, general_interface=True)
    assert isinstance(gen.iface, GeneralInterface) and not isinstance(uni.iface, GeneralInterface)
    for th in (0.0, 0.21, 1.7, -2.9):
        Ru, Rg = uni.residual(Q, th, 1.0), gen.residual(Q, th, 1.0)
        assert np.abs(Ru - Rg).max() <= 1e-12 * np.abs(Ru).max()


@pytest.mark.parametrize("theta", [0.0, 0.4, 2.2])
def test_mortars_tile_the_circle(theta):
    itf = SSD(_mesh(), C.ellipse_case(), 3).iface
    recs = itf.mortars(theta)
    assert len(recs) == 16 + 24
    assert abs(sum(r["w"] for r in recs) - 2 * np.pi) < 1e-12
    for r in recs:
        for k in ("L", "R"):
            assert -1e-12 <= r["o" + k] and r["o" + k] + r["s" + k] <= 1 + 1e-12
    # each face is covered exactly by its mortars
    for key, side, n in (("L", itf.L, 16), ("R", itf.Rt, 24)):
        cover = np.zeros(n)
        for r in recs:
            cover[r["i" + key]] += r["s" + key]
        assert np.allclose(cover, 1.0, atol=1e-12)


def test_flux_is_conserved_across_the_interface():
    case = C.ellipse_case()
    mesh = _mesh()
    ssd = SSD(mesh, case, 4)
    Q = C.perturbed_farfield_state(case, 4, ssd.E, amplitude=0.1)
    q = np.moveaxis(Q, 3, 1)
    qxi = np.einsum("ki,veji->vejk", ssd.ops.I, q)
    qeta = np.einsum("kj,veji->veki", ssd.ops.I, q)
    T = SSD._faces(qxi, qeta, 4)
    itf = ssd.iface
    FL, FR = itf.common_flux(T, 0.83, case["gamma"])
    w = ssd.ops.w
    totL = np.einsum("p,vkp->v", w, FL)
    totR = np.einsum("p,vkp->v", w, FR)
    assert np.allclose(totL, totR, rtol=1e-12, atol=1e-12 * np.abs(totL).max())


def test_face_flux_converges_to_the_normal_flux():
    """Traces of one smooth field on both sides: the mortar face flux tends
    to F(q) . n R width at the face points as the rings are refined."""
    case = C.ellipse_case()
    gam = case["gamma"]
    errs = []
    for K, Ko in ((16, 24), (32, 48), (64, 96)):
        ssd = SSD(_mesh(K, Ko), case, 3)
        itf = ssd.iface
        th = 0.3
        X = ssd.ops.X

        def field(phi):
            rho = 1.0 + 0.1 * np.sin(phi)
            u, v, p = 0.3 + 0.05 * np.cos(2 * phi), 0.1 * np.sin(phi), 1 / gam
            return np.stack([rho, rho * u, rho * v, p / (gam - 1) + 0.5 * rho * (u * u + v * v)])

        T = np.zeros((4, ssd.E, 4, 3))
        worst = 0.0
        for side, rot in ((itf.L, itf.rotL), (itf.Rt, itf.rotR)):
            phi = (side["start"][:, None] + (th if rot else 0.0)
                   + side["width"][:, None] * X[None, :])
            vals = field(phi)                                            # (4, k, N)
            d = np.where(side["flip"][None, :, None], vals[:, :, ::-1], vals)
            T[:, side["e"], side["f"], :] = d
        FL, FR = itf.common_flux(T, th, gam)
        for side, rot, F in ((itf.L, itf.rotL, FL), (itf.Rt, itf.rotR, FR)):
            phi = (side["start"][:, None] + (th if rot else 0.0)
                   + side["width"][:, None] * X[None, :])
            q = field(phi)
            s = itf.R * side["width"][:, None]
            exact = ph.normal_inviscid_flux(q, np.cos(phi) * s, np.sin(phi) * s, 0.0, gam)
            worst = max(worst, np.abs(F - exact).max() / np.abs(exact).max())
        errs.append(worst)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-4 and np.all(rates > 2.5), (errs, rates)


def test_viscous_equals_uniform_construction_on_uniform_rings():
    """BR1 common solution and viscous mortar flux through the general
    interface equal the uniform construction's on uniform rings."""
    case = C.ellipse_case()
    case["mu"] = 0.02
    mesh = _mesh(K_out=16, warp=0.0)
    Q = C.perturbed_farfield_state(case, 3, len(mesh["zone"]), amplitude=0.05)
    uni, gen = SSD(mesh, case, 3), SSD(mesh, case, 3, general_interface=True)
    for th in (0.0, 0.43, -1.2):
        Ru, Rg = uni.residual(Q, th, 1.0), gen.residual(Q, th, 1.0)
        assert np.abs(Ru - Rg).max() <= 1e-12 * np.abs(Ru).max()


def test_viscous_general_residual_conserves():
    """On unequal, non-uniform rings the viscous residual's interface terms
    still cancel: the total of |J| dQ/dt over the mesh equals the boundary
    flux through the walls and the far field only, as on a conforming mesh;
    checked as the change of the totals under a change of the state that is
    zero away from the interface."""
    case = C.ellipse_case()
    case["mu"] = 0.02
    ssd = SSD(_mesh(n=4), case, 3)   # BR1 reaches two cells: keep walls and far field 3 away
    Q = C.perturbed_farfield_state(case, 3, ssd.E, amplitude=0.05)
    R1 = ssd.residual(Q, 0.3, 1.0)
    Q2 = Q.copy()
    ring = np.unique(np.concatenate([ssd.iface.L["e"], ssd.iface.Rt["e"]]))
    Q2[..., ring] *= 1.0 + 0.02 * np.random.default_rng(3).normal(size=(4, 3, 3, len(ring)))
    R2 = ssd.residual(Q2, 0.3, 1.0)
    w = ssd.ops.w
    J = ssd.geo.detJ                                                   # (E, N, N) [e, j, i]
    tot = lambda R: np.einsum("j,i,eji,vjie->v", w, w, J, R)
    # the ring cells touch no wall and no far field, so the totals may only
    # differ by roundoff
    assert np.allclose(tot(R1), tot(R2), rtol=0, atol=1e-10 * np.abs(R1).max())
