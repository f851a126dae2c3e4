"""Iso-parametric element maps and metric terms (Sec. 2.3, Sec. 3.1).

Each cell is mapped to the standard square 0 <= xi, eta <= 1.  Sec. 3.1 uses
4-node linear cells, and 12-node cubic cells along curved boundaries; the
12-node cell is read as the cubic serendipity element, whose shape functions
here come straight from their definition: the unique combination of the 12
serendipity monomials that is 1 at its own node and 0 at the other 11.

Metrics (Sec. 2.3): x_xi, x_eta, y_xi, y_eta are the exact derivatives of the
map, |J| = x_xi y_eta - x_eta y_xi.  In the rotating zone the coordinates are
updated analytically (Sec. 2.2): a rigid rotation by theta about the centre
rotates positions and the derivative vectors and leaves |J| unchanged.
"""
import numpy as np

from workloads.meshes import NODE_REF, GEOM_CUBIC

_MONO = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2),
         (3, 0), (2, 1), (1, 2), (0, 3), (3, 1), (1, 3)]


def _mono(xi, eta, dx=0, dy=0):
    """Monomials (or their derivatives) at points: (P, 12)."""
    cols = []
    for a, b in _MONO:
        if a < dx or b < dy:
            cols.append(np.zeros_like(xi))
            continue
        ca = 1.0
        for t in range(dx):
            ca *= (a - t)
        cb = 1.0
        for t in range(dy):
            cb *= (b - t)
        cols.append(ca * cb * xi ** (a - dx) * eta ** (b - dy))
    return np.stack(cols, axis=-1)


_COEF = np.linalg.solve(_mono(NODE_REF[:, 0], NODE_REF[:, 1]), np.eye(12))


def serendipity(xi, eta):
    """Cubic serendipity shape functions and derivatives: 3 x (P, 12)."""
    return (_mono(xi, eta) @ _COEF, _mono(xi, eta, 1, 0) @ _COEF, _mono(xi, eta, 0, 1) @ _COEF)


def bilinear(xi, eta):
    """Bilinear shape functions on the corner nodes 0, 3, 6, 9: 3 x (P, 12)."""
    P = len(xi)
    Nf = np.zeros((P, 12))
    Nx = np.zeros((P, 12))
    Ny = np.zeros((P, 12))
    Nf[:, 0], Nf[:, 3], Nf[:, 6], Nf[:, 9] = (1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta
    Nx[:, 0], Nx[:, 3], Nx[:, 6], Nx[:, 9] = -(1 - eta), (1 - eta), eta, -eta
    Ny[:, 0], Ny[:, 3], Ny[:, 6], Ny[:, 9] = -(1 - xi), -xi, xi, (1 - xi)
    return Nf, Nx, Ny


def point_sets(ops):
    """Reference coordinates of the SP grid and both FP grids.

    sp  : (N, N)   index [j, i] -> (X_i, X_j)
    fxi : (N, N+1) index [j, k] -> (Xf_k, X_j)    (xi-direction FPs)
    feta: (N+1, N) index [k, i] -> (X_i, Xf_k)    (eta-direction FPs)
    """
    X, Xf = ops.X, ops.Xf
    sp = np.meshgrid(X, X, indexing="xy")          # [j][i]: xi = X[i], eta = X[j]
    fxi = np.meshgrid(Xf, X, indexing="xy")        # [j][k]: xi = Xf[k], eta = X[j]
    feta = np.meshgrid(X, Xf, indexing="xy")       # [k][i]: xi = X[i], eta = Xf[k]
    return {"sp": sp, "fxi": fxi, "feta": feta}


class Geometry:
    """Body-frame positions and metric terms at the SPs and FPs.

    For each point set s in ('sp', 'fxi', 'feta'), self.data[s] holds arrays
    x, y, x_xi, x_eta, y_xi, y_eta of shape (E,) + grid shape.
    """

    def __init__(self, mesh, ops):
        self.ops = ops
        self.zone = np.asarray(mesh["zone"])
        self.center = np.asarray(mesh["center"], dtype=float)
        xy = np.asarray(mesh["xy"], dtype=float)
        cubic = np.asarray(mesh["geom"]) == GEOM_CUBIC
        self.data = {}
        for name, (gxi, geta) in point_sets(ops).items():
            shape = gxi.shape
            xi, eta = gxi.ravel(), geta.ravel()
            out = {}
            for sel, fun in ((~cubic, bilinear), (cubic, serendipity)):
                if not np.any(sel):
                    continue
                Nf, Nx, Ny = fun(xi, eta)
                sub = xy[sel]
                for key, Nm in (("", Nf), ("_xi", Nx), ("_eta", Ny)):
                    for c, cn in ((0, "x"), (1, "y")):
                        arr = out.setdefault(cn + key, np.zeros((len(xy), len(xi))))
                        arr[sel] = sub[:, :, c] @ Nm.T
            self.data[name] = {k: v.reshape((len(xy),) + shape) for k, v in out.items()}
        sp = self.data["sp"]
        self.detJ = sp["x_xi"] * sp["y_eta"] - sp["x_eta"] * sp["y_xi"]

    def at(self, theta):
        """Positions and metrics with zone 1 rotated by theta about the centre."""
        c, s = np.cos(theta), np.sin(theta)
        rot = self.zone == 1
        out = {}
        for name, d in self.data.items():
            o = dict(d)
            if np.any(rot) and theta != 0.0:
                rshape = (-1,) + (1,) * (d["x"].ndim - 1)
                m = rot.reshape(rshape)
                dx = d["x"] - self.center[0]
                dy = d["y"] - self.center[1]
                o["x"] = np.where(m, self.center[0] + c * dx - s * dy, d["x"])
                o["y"] = np.where(m, self.center[1] + s * dx + c * dy, d["y"])
                for a in ("_xi", "_eta"):
                    vx, vy = d["x" + a], d["y" + a]
                    o["x" + a] = np.where(m, c * vx - s * vy, vx)
                    o["y" + a] = np.where(m, s * vx + c * vy, vy)
            out[name] = o
        return out
