"""The sliding-mesh SD residual, the dynamic mortars and SSP-RK3 (Sec. 3).

State layout at the interface: Q[v, j, i, e], the 4 conservative variables
at solution point (X_i, X_j) of element e.  The state is the physical Q at
the SPs; since |J| of a rigidly rotating or fixed cell does not change in
time, dQ~/dt = |J| dQ/dt and residual() returns dQ/dt.

Per residual evaluation (Sec. 3.1, Sec. 3.2):
  1. Q at the FPs by Lagrange interpolation along each line (eq. Qt).
  2. Transformed fluxes F~ = |J| J^-1 (F, G) at interior FPs
     (eq. transform_relation) with the ALE grid-velocity terms (Sec. 2.2).
  3. Common normal fluxes at element-boundary FPs: Rusanov on conforming
     and periodic faces, boundary fluxes on walls and far field, and the
     curved dynamic mortar on the sliding interface (eqs. xz, prjQ2, prjF2).
  4. With viscosity, BR1-style common solution and common gradient
     (Sec. 3.1 refers the viscous details elsewhere; Sec. 3.2 gives the
     mortar steps for them).
  5. dQ~/dt = -(dF~/dxi + dG~/deta) at the SPs from the degree-N flux
     polynomials (eqs. Ft, Gt).
"""
import numpy as np

from workloads.meshes import (FACE_CORNERS, FACE_INTERIOR, FACE_PERIODIC, FACE_SLIDING,
                              FACE_WALL_ISOTHERMAL, FACE_WALL_SLIP, FACE_FARFIELD)
from .basis import Operators
from .geometry import Geometry
from . import physics as ph

FACE_EXTERNAL = 100   # face of a sub-mesh whose neighbour lies outside it


# SSPRK54 (five stages, fourth order, strong-stability preserving), Shu-Osher
# form: U1 = U + a[0][2] dt L(U); U_k = a[k-1][0] U + a[k-1][1] U_{k-1} +
# a[k-1][2] dt L(U_{k-1}) for k = 2, 3, 4; U^{n+1} = c[0] U2 + c[1] U3 +
# c[2] dt L(U3) + c[3] U4 + c[4] dt L(U4).  The published SSPRK(5,4)
# coefficients of Spiteri and Ruuth; tests check fourth order on a
# nonlinear, time-dependent ODE.
SSPRK54 = {
    "a": [[0.0, 1.0, 0.391752226571890],
          [0.444370493651235, 0.555629506348765, 0.368410593050371],
          [0.620101851488403, 0.379898148511597, 0.251891774271694],
          [0.178079954393132, 0.821920045606868, 0.544974750228521]],
    "c": [0.517231671970585, 0.096059710526147, 0.063692468666290,
          0.386708617503269, 0.226007483236906],
}


def ssprk54_stage_times():
    """Times (in units of dt after t) at which SSPRK54 evaluates L: the
    time of each stage value, following the same combinations as U."""
    a = SSPRK54["a"]
    tau = [0.0, a[0][2]]
    for k in (1, 2, 3):
        tau.append(a[k][1] * tau[-1] + a[k][2])
    return tau


def _wrap_pi(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


class Interface:
    """The two rings of faces on the circular sliding interface (Sec. 3.2).

    Inner cells are the left (L) side, outer cells the right (R) side; faces
    on each side are sorted counter-clockwise.  Each face gets a canonical
    coordinate that increases counter-clockwise (its own parameter, or the
    reverse when `flip`), so face j of a side spans the angles
    phi0 + theta_side + [j, j+1] * Delta, Delta = 2 pi / K.
    """

    def __init__(self, mesh, ops):
        self.ops = ops
        self.c = np.asarray(mesh["center"], dtype=float)
        self.R = float(mesh["radius"])
        xy = mesh["xy"]
        e, f = np.nonzero(mesh["face_kind"] == FACE_SLIDING)
        st = xy[e, FACE_CORNERS[f, 0]] - self.c
        en = xy[e, FACE_CORNERS[f, 1]] - self.c
        a0 = np.arctan2(st[:, 1], st[:, 0])
        a1 = np.arctan2(en[:, 1], en[:, 0])
        d = _wrap_pi(a1 - a0)
        flip = d < 0
        start = np.where(flip, a1, a0) % (2 * np.pi)
        cen = xy[e][:, [0, 3, 6, 9]].mean(axis=1) - self.c
        inner = np.hypot(cen[:, 0], cen[:, 1]) < self.R
        sides = []
        for sel in (inner, ~inner):
            order = np.argsort(start[sel])
            sides.append(dict(e=e[sel][order], f=f[sel][order], flip=flip[sel][order],
                              start=start[sel][order], zone=mesh["zone"][e[sel][order]]))
        self.L, self.Rt = sides
        K = len(self.L["e"])
        if K == 0 or len(self.Rt["e"]) != K:
            raise ValueError("sliding interface needs the same number of faces on both sides")
        self.K = K
        self.delta = 2 * np.pi / K
        for s in sides:
            steps = _wrap_pi(np.diff(np.concatenate([s["start"], s["start"][:1] + 2 * np.pi])))
            if np.max(np.abs(steps - self.delta)) > 1e-9:
                raise ValueError("sliding interface faces are not uniform")
            if len(set(s["zone"].tolist())) != 1:
                raise ValueError("one side of the interface spans two zones")
        self.rotL = int(self.L["zone"][0]) == 1
        self.rotR = int(self.Rt["zone"][0]) == 1

    def placement(self, theta):
        """(m, delta_frac, thL, thR): L face j overlaps R faces j+m and j+m+1;
        its first (1 - delta_frac) lies on R face j+m."""
        thL = theta if self.rotL else 0.0
        thR = theta if self.rotR else 0.0
        a = (self.L["start"][0] + thL) - (self.Rt["start"][0] + thR)
        x = a / self.delta
        fl = np.floor(x)
        dlt = x - fl
        m = int(fl) % self.K
        if dlt >= 1.0:
            dlt, m = 0.0, (m + 1) % self.K
        return m, float(dlt), thL, thR

    def operators(self, dlt):
        """(o, s) of the two mortars seen from an L face and from an R face,
        with their forward and backward projections (eqs. prjQ2, prjF2)."""
        ops = self.ops
        osL = [(0.0, 1.0 - dlt), (1.0 - dlt, dlt)]
        osR = [(dlt, 1.0 - dlt), (0.0, dlt)]
        PfL = [ops.forward(o, s) for o, s in osL]
        PbL = [ops.backward(o, s) for o, s in osL]
        PfR = [ops.forward(o, s) for o, s in osR]
        PbR = [ops.backward(o, s) for o, s in osR]
        return osL, PfL, PbL, PfR, PbR

    def canon(self, side, arr):
        """Face data (4, E, 4, N) -> canonical ring data (4, K, N)."""
        d = arr[:, side["e"], side["f"], :]
        return np.where(side["flip"][None, :, None], d[:, :, ::-1], d)

    def scatter(self, side, ring, out, sign):
        """Canonical ring data (4, K, N) -> element faces of `out`."""
        d = np.where(side["flip"][None, :, None], ring[:, :, ::-1], ring)
        out[:, side["e"], side["f"], :] = sign * d

    def mortar_angles(self, theta_side_L, osL):
        """Angles of the mortar SPs, (2, K, N), from the L faces."""
        j = np.arange(self.K)[:, None]
        X = self.ops.X[None, :]
        return [self.L["start"][0] + theta_side_L + self.delta * (j + o + s * X) for o, s in osL]

    def face_angles(self, side, theta_side):
        j = np.arange(self.K)[:, None]
        return side["start"][0] + theta_side + self.delta * (j + self.ops.X[None, :])

    def to_mortars(self, qL, qR, m, PfL, PfR):
        """Project canonical L and R face data onto the 2K mortars."""
        K = self.K
        r1 = (np.arange(K) + m) % K
        r2 = (np.arange(K) + m + 1) % K
        out = []
        for k, rr in ((0, r1), (1, r2)):
            aL = np.einsum("ab,vjb->vja", PfL[k], qL)
            aR = np.einsum("ab,vjb->vja", PfR[k], qR[:, rr, :])
            out.append((aL, aR))
        return out

    def to_faces(self, mort, m, PbL, PbR):
        """Back-project per-mortar data (2 x (4, K, N)) to L and R faces."""
        K = self.K
        FL = (np.einsum("ab,vjb->vja", PbL[0], mort[0])
              + np.einsum("ab,vjb->vja", PbL[1], mort[1]))
        r = np.arange(K)
        FR = (np.einsum("ab,vjb->vja", PbR[0], mort[0][:, (r - m) % K, :])
              + np.einsum("ab,vjb->vja", PbR[1], mort[1][:, (r - m - 1) % K, :]))
        return FL, FR

    def common_flux(self, T, theta, gam):
        """Interface fluxes per unit face coordinate, canonical (4, K, N) for
        the L and R faces, from the face traces T (4, E, 4, N)."""
        m, dlt, thL, thR = self.placement(theta)
        osL, PfL, PbL, PfR, PbR = self.operators(dlt)
        TL, TR = self.canon(self.L, T), self.canon(self.Rt, T)
        proj = self.to_mortars(TL, TR, m, PfL, PfR)
        ang = self.mortar_angles(thL, osL)
        scale = self.R * self.delta
        fm = []
        for (aL, aR), phi in zip(proj, ang):
            nx, ny = np.cos(phi) * scale, np.sin(phi) * scale
            fm.append(ph.rusanov(aL, aR, nx, ny, 0.0, gam))
        return self.to_faces(fm, m, PbL, PbR)


    def common_solution(self, T, theta):
        """BR1 common solution on the interface faces, canonical (4, K, N):
        the mean of both sides' projections on each mortar, projected back."""
        m, dlt, thL, thR = self.placement(theta)
        osL, PfL, PbL, PfR, PbR = self.operators(dlt)
        TL, TR = self.canon(self.L, T), self.canon(self.Rt, T)
        proj = self.to_mortars(TL, TR, m, PfL, PfR)
        return self.to_faces([0.5 * (aL + aR) for aL, aR in proj], m, PbL, PbR)

    def viscous_common_flux(self, Qc, GX, GY, theta, flux):
        """Viscous interface flux per unit face coordinate, canonical: each
        side's face viscous flux along the radial normal (from the faces'
        common solution and own gradients; flux(q, gx, gy) -> (F, G)),
        projected onto the mortars, averaged, projected back."""
        m, dlt, thL, thR = self.placement(theta)
        osL, PfL, PbL, PfR, PbR = self.operators(dlt)
        scale = self.R * self.delta

        def side_flux(side, th):
            phi = self.face_angles(side, th)
            nx, ny = np.cos(phi) * scale, np.sin(phi) * scale
            Fs, Gs = flux(self.canon(side, Qc), self.canon(side, GX), self.canon(side, GY))
            return Fs * nx + Gs * ny

        proj = self.to_mortars(side_flux(self.L, thL), side_flux(self.Rt, thR), m, PfL, PfR)
        return self.to_faces([0.5 * (aL + aR) for aL, aR in proj], m, PbL, PbR)


class GeneralInterface:
    """A sliding interface whose two rings need not have the same number of
    faces nor uniform faces (more than two mortars per face; the extension
    named at the end of Sec. 3.2 and in the conclusions).

    Each side's faces are sorted counter-clockwise, face i spanning the
    angles start_i + theta_side + [0, width_i].  At a rotor angle the two
    sides' face end points, merged in angular order, cut the circle into
    mortars; each mortar lies on exactly one L face and one R face, at face
    coordinate offset o and length s on each (eqs. xz, prjQ2, prjF2 with a
    separate (o, s) per mortar).  Fluxes: Rusanov on the exact circle at
    each mortar's solution points, as flux per unit angle times R, projected
    back to a face with s M^-1 A^T and scaled by the face's width (flux per
    unit face coordinate).
    """

    def __init__(self, mesh, ops):
        self.ops = ops
        self.c = np.asarray(mesh["center"], dtype=float)
        self.R = float(mesh["radius"])
        xy = mesh["xy"]
        e, f = np.nonzero(mesh["face_kind"] == FACE_SLIDING)
        st = xy[e, FACE_CORNERS[f, 0]] - self.c
        en = xy[e, FACE_CORNERS[f, 1]] - self.c
        a0 = np.arctan2(st[:, 1], st[:, 0])
        a1 = np.arctan2(en[:, 1], en[:, 0])
        d = _wrap_pi(a1 - a0)
        flip = d < 0
        start = np.where(flip, a1, a0) % (2 * np.pi)
        cen = xy[e][:, [0, 3, 6, 9]].mean(axis=1) - self.c
        inner = np.hypot(cen[:, 0], cen[:, 1]) < self.R
        sides = []
        for sel in (inner, ~inner):
            order = np.argsort(start[sel])
            s = dict(e=e[sel][order], f=f[sel][order], flip=flip[sel][order],
                     start=start[sel][order], width=np.abs(d[sel][order]),
                     zone=mesh["zone"][e[sel][order]])
            nxt = np.concatenate([s["start"][1:], s["start"][:1] + 2 * np.pi])
            if np.max(np.abs(nxt - s["start"] - s["width"])) > 1e-9:
                raise ValueError("sliding interface faces do not tile the circle")
            if len(set(s["zone"].tolist())) != 1:
                raise ValueError("one side of the interface spans two zones")
            sides.append(s)
        self.L, self.Rt = sides
        self.rotL = int(self.L["zone"][0]) == 1
        self.rotR = int(self.Rt["zone"][0]) == 1

    def mortars(self, theta):
        """Per mortar: L face, R face, (o, s) on each, start angle, width."""
        thL = theta if self.rotL else 0.0
        thR = theta if self.rotR else 0.0
        pts = []
        for side, th, tag in ((self.L, thL, 0), (self.Rt, thR, 1)):
            for i, a in enumerate(side["start"]):
                pts.append(((a + th) % (2 * np.pi), tag, i))
        pts.sort(key=lambda p: (p[0], p[1]))
        out = []
        M = len(pts)
        cur = {}
        # the face of each side in force at the first merged point
        for tag, side, th in ((0, self.L, thL), (1, self.Rt, thR)):
            a = (side["start"] + th) % (2 * np.pi)
            before = np.nonzero(a <= pts[0][0])[0]
            cur[tag] = int(before[np.argmax(a[before])]) if len(before) else int(np.argmax(a))
        for k in range(M):
            b0, tag, i = pts[k]
            cur[tag] = i
            b1 = pts[(k + 1) % M][0] + (2 * np.pi if k + 1 == M else 0.0)
            w = b1 - b0
            rec = dict(b0=b0, w=w, iL=cur[0], iR=cur[1])
            for key, side, th, idx in (("L", self.L, thL, cur[0]), ("R", self.Rt, thR, cur[1])):
                a = (side["start"][idx] + th) % (2 * np.pi)
                off = (b0 - a) % (2 * np.pi)
                rec["o" + key] = off / side["width"][idx]
                rec["s" + key] = w / side["width"][idx]
            out.append(rec)
        return out

    def canon(self, side, arr):
        d = arr[:, side["e"], side["f"], :]
        return np.where(side["flip"][None, :, None], d[:, :, ::-1], d)

    def scatter(self, side, ring, out, sign):
        d = np.where(side["flip"][None, :, None], ring[:, :, ::-1], ring)
        out[:, side["e"], side["f"], :] = sign * d

    def _per_mortar(self, VL, VR, theta, combine, widths):
        """For every mortar: project side data VL, VR (4, K_side, N) onto it,
        combine(aL, aR, rec) -> (4, N) mortar values, project back onto both
        faces (times the face width when `widths`)."""
        ops = self.ops
        FL = np.zeros((VL.shape[0],) + VL.shape[1:])
        FR = np.zeros((VR.shape[0],) + VR.shape[1:])
        for r in self.mortars(theta):
            if r["w"] <= 0.0:
                continue
            aL = (ops.forward(r["oL"], r["sL"]) @ VL[:, r["iL"], :].T).T       # (4, N)
            aR = (ops.forward(r["oR"], r["sR"]) @ VR[:, r["iR"], :].T).T
            fm = combine(aL, aR, r)
            wL = self.L["width"][r["iL"]] if widths else 1.0
            wR = self.Rt["width"][r["iR"]] if widths else 1.0
            FL[:, r["iL"], :] += (ops.backward(r["oL"], r["sL"]) @ fm.T).T * wL
            FR[:, r["iR"], :] += (ops.backward(r["oR"], r["sR"]) @ fm.T).T * wR
        return FL, FR

    def common_flux(self, T, theta, gam):
        def rus(aL, aR, r):
            phi = r["b0"] + r["w"] * self.ops.X
            return ph.rusanov(aL, aR, np.cos(phi) * self.R, np.sin(phi) * self.R, 0.0, gam)
        return self._per_mortar(self.canon(self.L, T), self.canon(self.Rt, T), theta, rus, True)

    def common_solution(self, T, theta):
        return self._per_mortar(self.canon(self.L, T), self.canon(self.Rt, T), theta,
                                lambda aL, aR, r: 0.5 * (aL + aR), False)

    def viscous_common_flux(self, Qc, GX, GY, theta, flux):
        X = self.ops.X

        def side_flux(side, rot):
            th = theta if rot else 0.0
            phi = side["start"][:, None] + th + side["width"][:, None] * X[None, :]
            nx, ny = np.cos(phi) * self.R, np.sin(phi) * self.R          # per unit angle
            Fs, Gs = flux(self.canon(side, Qc), self.canon(side, GX), self.canon(side, GY))
            return Fs * nx + Gs * ny

        return self._per_mortar(side_flux(self.L, self.rotL), side_flux(self.Rt, self.rotR), theta,
                                lambda aL, aR, r: 0.5 * (aL + aR), True)


def make_interface(mesh, ops, general=None):
    """The uniform interface (K equal faces per side) when the rings allow
    it, else the general one; general=True forces the general one."""
    if general:
        return GeneralInterface(mesh, ops)
    try:
        return Interface(mesh, ops)
    except ValueError:
        if general is False:
            raise
        return GeneralInterface(mesh, ops)


class SSD:
    """FP64 residual of the SSD method on one mesh (Sec. 3)."""

    def __init__(self, mesh, case, N, general_interface=None):
        self.mesh = mesh
        self.case = case
        self.N = N
        self.ops = Operators(N)
        self.geo = Geometry(mesh, self.ops)
        self.E = len(mesh["zone"])
        self.kind = np.asarray(mesh["face_kind"])
        self.nbr = np.asarray(mesh["nbr"])
        self.nbf = np.asarray(mesh["nbr_face"])
        xy = mesh["xy"]
        ends = xy[:, FACE_CORNERS]                          # (E,4,2,2)
        tang = ends[:, :, 1] - ends[:, :, 0]
        has = self.nbr >= 0
        nb = np.where(has, self.nbr, 0)
        nf = np.where(has, self.nbf, 0)
        self.rev = has & (np.einsum("efc,efc->ef", tang, tang[nb, nf]) < 0)
        self.iface = (make_interface(mesh, self.ops, general_interface)
                      if np.any(self.kind == FACE_SLIDING) else None)
        self.zone1 = np.asarray(mesh["zone"]) == 1

    # ------------------------------------------------------------------
    def _neighbor(self, T):
        """Neighbour traces (.., E, 4, N) aligned with each face's parameter."""
        nb = np.where(self.nbr >= 0, self.nbr, np.arange(self.E)[:, None])
        nf = np.where(self.nbr >= 0, self.nbf, np.arange(4)[None, :])
        Tn = T[..., nb, nf, :]
        return np.where(self.rev[..., :, :, None], Tn[..., ::-1], Tn)

    @staticmethod
    def _faces(axi, aeta, N):
        """Face values (.., E, 4, N) from xi-FP (.., E, N, N+1) and eta-FP
        (.., E, N+1, N) arrays, in each face's own parameter order."""
        return np.stack([aeta[..., 0, :], axi[..., :, N], aeta[..., N, :], axi[..., :, 0]], axis=-2)

    def residual(self, Q, theta, omega, diag=False):
        """dQ/dt at the SPs for state Q[v, j, i, e] with zone 1 at angle
        theta turning at rate omega."""
        ops, N, E = self.ops, self.N, self.E
        cs = self.case
        gam = cs["gamma"]
        visc = cs["mu"] > 0.0
        q = np.moveaxis(np.asarray(Q, dtype=float), 3, 1)            # (4,E,N,N) [v,e,j,i]
        g = self.geo.at(theta)
        cx, cy = self.geo.center
        rot = self.zone1

        qxi = np.einsum("ki,veji->vejk", ops.I, q)                  # (4,E,N,N+1)
        qeta = np.einsum("kj,veji->veki", ops.I, q)                 # (4,E,N+1,N)

        def gridvel(d):
            m = rot.reshape((-1,) + (1,) * (d["x"].ndim - 1))
            ug = np.where(m, -omega * (d["y"] - cy), 0.0)
            vg = np.where(m, omega * (d["x"] - cx), 0.0)
            return ug, vg

        gx, ge = g["fxi"], g["feta"]
        ugx, vgx = gridvel(gx)
        uge, vge = gridvel(ge)
        # scaled contravariant normals of the FP lines: (y_eta, -x_eta), (-y_xi, x_xi)
        nxi = (gx["y_eta"], -gx["x_eta"])
        neta = (-ge["y_xi"], ge["x_xi"])
        vgn_xi = ugx * nxi[0] + vgx * nxi[1]
        vgn_eta = uge * neta[0] + vge * neta[1]
        Ft = ph.normal_inviscid_flux(qxi, nxi[0], nxi[1], vgn_xi, gam)     # (4,E,N,N+1)
        Gt = ph.normal_inviscid_flux(qeta, neta[0], neta[1], vgn_eta, gam)  # (4,E,N+1,N)

        # ---- faces: traces, outward scaled normals, grid velocity --------
        T = self._faces(qxi, qeta, N)                                    # (4,E,4,N)
        sgn = np.array([-1.0, 1.0, 1.0, -1.0])[None, :, None]
        fnx = self._faces(nxi[0], neta[0], N) * sgn
        fny = self._faces(nxi[1], neta[1], N) * sgn
        fug = self._faces(ugx, uge, N)
        fvg = self._faces(vgx, vge, N)
        fvgn = fug * fnx + fvg * fny
        Tn = self._neighbor(T)
        kind = self.kind[:, :, None]
        inter = (kind == FACE_INTERIOR) | (kind == FACE_PERIODIC)
        wall = (kind == FACE_WALL_ISOTHERMAL) | (kind == FACE_WALL_SLIP)
        far = kind == FACE_FARFIELD
        ext = kind == FACE_EXTERNAL
        Qinf = ph.conservative(*cs["farfield"], gam)[:, None, None, None] * np.ones_like(T)

        fs = np.zeros_like(T)
        rus = ph.rusanov(T, Tn, fnx, fny, fvgn, gam)
        fs = np.where(inter, rus, fs)
        _, _, _, pT = ph.primitives(T, gam)
        zero = np.zeros_like(pT)
        fwall = np.stack([zero, pT * fnx, pT * fny, pT * fvgn])
        fs = np.where(wall, fwall, fs)
        fs = np.where(far, ph.rusanov(T, Qinf, fnx, fny, fvgn, gam), fs)
        fs = np.where(ext, ph.normal_inviscid_flux(T, fnx, fny, fvgn, gam), fs)

        itf = self.iface
        if itf is not None:
            FL, FR = itf.common_flux(T, theta, gam)
            itf.scatter(itf.L, FL, fs, 1.0)
            itf.scatter(itf.Rt, FR, fs, -1.0)

        if visc:
            fv, Ftv, Gtv = self._viscous(q, qxi, qeta, T, Tn, g, fnx, fny, fug, fvg,
                                         nxi, neta, theta)
            fs = fs + fv
            Ft = Ft + Ftv
            Gt = Gt + Gtv

        # common fluxes at the element-boundary FPs (sign: outward -> F~, G~)
        Ft[..., 0] = -fs[:, :, 3, :]
        Ft[..., N] = fs[:, :, 1, :]
        Gt[:, :, 0, :] = -fs[:, :, 0, :]
        Gt[:, :, N, :] = fs[:, :, 2, :]

        dF = np.einsum("ik,vejk->veji", ops.D, Ft)
        dG = np.einsum("jk,veki->veji", ops.D, Gt)
        R = -(dF + dG) / self.geo.detJ[None]
        Rapi = np.moveaxis(R, 1, 3)
        if not diag:
            return Rapi
        absD = np.abs(ops.D)
        scale = (np.einsum("ik,vejk->veji", absD, np.abs(Ft))
                 + np.einsum("jk,veki->veji", absD, np.abs(Gt))) / np.abs(self.geo.detJ[None])
        return Rapi, dict(flux_scale=np.moveaxis(scale, 1, 3), face_flux=fs)

    # ------------------------------------------------------------------
    def _viscous(self, q, qxi, qeta, T, Tn, g, fnx, fny, fug, fvg, nxi, neta, theta):
        """Viscous parts (BR1 reading): face common viscous flux (outward,
        per unit face parameter) and interior transformed viscous fluxes."""
        ops, N = self.ops, self.N
        cs = self.case
        gam, Rg, mu, Pr = cs["gamma"], cs["gas_R"], cs["mu"], cs["prandtl"]
        kind = self.kind[:, :, None]
        inter = (kind == FACE_INTERIOR) | (kind == FACE_PERIODIC)
        iso = kind == FACE_WALL_ISOTHERMAL
        slip = kind == FACE_WALL_SLIP
        far = kind == FACE_FARFIELD

        # common solution at the faces
        rho, u, v, p = ph.primitives(T, gam)
        Qc = T.copy()
        Qc = np.where(inter, 0.5 * (T + Tn), Qc)
        rb = p / (Rg * cs["T_wall"])
        Qiso = ph.conservative(rb, fug, fvg, p, gam)
        Qc = np.where(iso, Qiso, Qc)
        Qc = np.where(slip, ph.slip_state(T, fnx, fny, fug, fvg, gam), Qc)
        Qinf = ph.conservative(*cs["farfield"], gam)[:, None, None, None] * np.ones_like(T)
        Qc = np.where(far, Qinf, Qc)

        itf = self.iface
        if itf is not None:
            QcL, QcR = itf.common_solution(T, theta)
            itf.scatter(itf.L, QcL, Qc, 1.0)
            itf.scatter(itf.Rt, QcR, Qc, 1.0)

        # gradients at the SPs from FP values with common boundary values
        qxs = qxi.copy()
        qxs[..., 0] = Qc[:, :, 3, :]
        qxs[..., N] = Qc[:, :, 1, :]
        qes = qeta.copy()
        qes[:, :, 0, :] = Qc[:, :, 0, :]
        qes[:, :, N, :] = Qc[:, :, 2, :]
        Qxi = np.einsum("ik,vejk->veji", ops.D, qxs)
        Qeta = np.einsum("jk,veki->veji", ops.D, qes)
        sp = g["sp"]
        J = self.geo.detJ[None]
        Qx = (sp["y_eta"][None] * Qxi - sp["y_xi"][None] * Qeta) / J
        Qy = (-sp["x_eta"][None] * Qxi + sp["x_xi"][None] * Qeta) / J

        # gradients at the FPs
        gx_xi = np.einsum("ki,veji->vejk", ops.I, Qx)
        gy_xi = np.einsum("ki,veji->vejk", ops.I, Qy)
        gx_eta = np.einsum("kj,veji->veki", ops.I, Qx)
        gy_eta = np.einsum("kj,veji->veki", ops.I, Qy)
        GX = self._faces(gx_xi, gx_eta, N)
        GY = self._faces(gy_xi, gy_eta, N)
        GXn, GYn = self._neighbor(GX), self._neighbor(GY)
        GXc = np.where(inter, 0.5 * (GX + GXn), GX)
        GYc = np.where(inter, 0.5 * (GY + GYn), GY)

        Fv, Gv = ph.viscous_flux(Qc, GXc, GYc, gam, Rg, mu, Pr)
        fv = Fv * fnx + Gv * fny
        fv = np.where(slip, 0.0, fv)

        if itf is not None:
            FvL, FvR = itf.viscous_common_flux(
                Qc, GX, GY, theta, lambda q, gx, gy: ph.viscous_flux(q, gx, gy, gam, Rg, mu, Pr))
            itf.scatter(itf.L, FvL, fv, 1.0)
            itf.scatter(itf.Rt, FvR, fv, -1.0)

        Fx, Gx = ph.viscous_flux(qxi, gx_xi, gy_xi, gam, Rg, mu, Pr)
        Fe, Ge = ph.viscous_flux(qeta, gx_eta, gy_eta, gam, Rg, mu, Pr)
        Ftv = Fx * nxi[0] + Gx * nxi[1]
        Gtv = Fe * neta[0] + Ge * neta[1]
        return fv, Ftv, Gtv

    # ------------------------------------------------------------------
    def theta(self, t):
        return self.case["theta0"] + self.case["omega"] * t

    def ssprk3_step(self, Q, t, dt):
        """Three-stage SSP Runge-Kutta step (Shu-Osher form); the rotor angle
        and the mortars follow the stage times t, t+dt, t+dt/2."""
        w = self.case["omega"]
        Q1 = Q + dt * self.residual(Q, self.theta(t), w)
        Q2 = 0.75 * Q + 0.25 * (Q1 + dt * self.residual(Q1, self.theta(t + dt), w))
        return Q / 3.0 + 2.0 / 3.0 * (Q2 + dt * self.residual(Q2, self.theta(t + 0.5 * dt), w))

    def ssprk54_step(self, Q, t, dt):
        """Five-stage fourth-order SSP Runge-Kutta step (the explicit SSP
        scheme the paper uses for all its tests, Sec. 4), in Shu-Osher form
        with the coefficients of SSPRK54; every stage evaluates the
        residual (and rebuilds the mortars) at its own stage time."""
        a, c = SSPRK54["a"], SSPRK54["c"]
        w = self.case["omega"]

        def L(U, tau):
            return dt * self.residual(U, self.theta(t + tau * dt), w)
        tau = ssprk54_stage_times()
        U1 = Q + a[0][2] * L(Q, 0.0)
        U2 = a[1][0] * Q + a[1][1] * U1 + a[1][2] * L(U1, tau[1])
        U3 = a[2][0] * Q + a[2][1] * U2 + a[2][2] * L(U2, tau[2])
        L3 = L(U3, tau[3])
        U4 = a[3][0] * Q + a[3][1] * U3 + a[3][2] * L3
        return c[0] * U2 + c[1] * U3 + c[2] * L3 + c[3] * U4 + c[4] * L(U4, tau[4])

    def run(self, Q, t0, dt, nsteps, scheme="rk3"):
        step = {"rk3": self.ssprk3_step, "rk54": self.ssprk54_step}[scheme]
        Q = np.array(Q, dtype=float)
        t = t0
        for _ in range(nsteps):
            Q = step(Q, t, dt)
            t += dt
        return Q

    # ------------------------------------------------------------------
    def sp_coords(self, theta=0.0):
        """Physical coordinates of the SPs at angle theta, each (N, N, E)."""
        sp = self.geo.at(theta)["sp"]
        return np.moveaxis(sp["x"], 0, 2), np.moveaxis(sp["y"], 0, 2)

    def integrate(self, Q):
        """sum_e sum_ij w_i w_j |J|_ij Q_ij for each variable (4,)."""
        w = self.ops.w
        W = (w[:, None] * w[None, :])[:, :, None] * np.moveaxis(self.geo.detJ, 0, 2)
        return np.einsum("vjie,jie->v", np.asarray(Q), W)


def submesh(mesh, elems, depth=2):
    """Sub-mesh around `elems` for sampled evaluation.

    Holds `elems`, every cell with a sliding face, and `depth` layers of
    neighbours around both.  Faces whose neighbour is left out become
    FACE_EXTERNAL; residuals are exact for cells at least `depth` faces away
    from such faces.  Returns (sub_mesh, global indices of its cells).
    """
    E = len(mesh["zone"])
    keep = np.zeros(E, bool)
    keep[np.asarray(elems)] = True
    keep[np.any(mesh["face_kind"] == FACE_SLIDING, axis=1)] = True
    for _ in range(depth):
        nb = mesh["nbr"][keep]
        keep[nb[nb >= 0]] = True
    idx = np.nonzero(keep)[0]
    remap = np.full(E, -1, np.int64)
    remap[idx] = np.arange(len(idx))
    nb = mesh["nbr"][idx]
    newnb = np.where(nb >= 0, remap[np.maximum(nb, 0)], -1)
    kind = mesh["face_kind"][idx].copy()
    lost = (nb >= 0) & (newnb < 0)
    kind[lost] = FACE_EXTERNAL
    sub = dict(mesh)
    sub.update(xy=mesh["xy"][idx], geom=mesh["geom"][idx], zone=mesh["zone"][idx],
               nbr=newnb.astype(np.int32),
               nbr_face=np.where(newnb >= 0, mesh["nbr_face"][idx], -1).astype(np.int32),
               face_kind=kind)
    return sub, idx
