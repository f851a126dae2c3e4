"""Points, Lagrange bases and mortar matrices of the SD method.

Sec. 3.1: an N-th order scheme uses N solution points (SPs) per direction at
the Chebyshev-Gauss points and N+1 flux points (FPs): the N-1 Legendre-Gauss
points plus the two ends of [0,1].  eq. (hbasis) and eq. (lbasis) define the
Lagrange bases h_i on the SPs and l_{k+1/2} on the FPs.

Sec. 3.2, eqs. (mortarM), (mortarS): M_ij = int_0^1 h_i h_j dz and the
overlap integrals of a face basis against a mortar basis.  The integrals are
done exactly by polynomial algebra (Legendre series on [0,1]; the paper
evaluates the same integrals analytically).
"""
import numpy as np
from numpy.polynomial import Legendre, Polynomial
from numpy.polynomial import legendre as nleg


def solution_points(N):
    """Chebyshev-Gauss points on [0,1]: X_s = (1 - cos((2s-1) pi / 2N)) / 2."""
    s = np.arange(1, N + 1)
    return 0.5 * (1.0 - np.cos((2 * s - 1) * np.pi / (2 * N)))


def flux_points(N):
    """0, the N-1 Legendre-Gauss points mapped to [0,1], and 1."""
    if N == 1:
        return np.array([0.0, 1.0])
    g, _ = nleg.leggauss(N - 1)
    return np.concatenate([[0.0], 0.5 * (g + 1.0), [1.0]])


def lagrange(nodes, i, x):
    """Cardinal polynomial of `nodes` for node i evaluated at x (product form)."""
    x = np.asarray(x, dtype=float)
    out = np.ones_like(x)
    for s, xs in enumerate(nodes):
        if s != i:
            out = out * (x - xs) / (nodes[i] - xs)
    return out


def lagrange_deriv(nodes, i, x):
    """d/dx of the cardinal polynomial: sum over the dropped factor m."""
    x = np.asarray(x, dtype=float)
    out = np.zeros_like(x)
    for m, xm in enumerate(nodes):
        if m == i:
            continue
        term = np.full_like(x, 1.0 / (nodes[i] - xm))
        for s, xs in enumerate(nodes):
            if s != i and s != m:
                term = term * (x - xs) / (nodes[i] - xs)
        out = out + term
    return out


def lagrange_poly(nodes, i):
    """Cardinal polynomial of `nodes` for node i as a Legendre series on the
    domain [0, 1] (well conditioned for exact products and integrals)."""
    others = [x for s, x in enumerate(nodes) if s != i]
    p = Legendre.fromroots(others, domain=[0.0, 1.0]) if others else Legendre([1.0], domain=[0.0, 1.0])
    return p / p(nodes[i])


def _integrate01(p):
    ip = p.integ()
    return ip(1.0) - ip(0.0)


class Operators:
    """1-D operator tables for order N.

    X   (N,)     SPs          Xf (N+1,) FPs
    I   (N+1, N) I[k, i] = h_i(Xf_k)       (SP -> FP interpolation, eq. Qt)
    D   (N, N+1) D[i, k] = l'_{k+1/2}(X_i) (FP -> SP derivative, eqs. Ft, Gt)
    w   (N,)     w_i = int_0^1 h_i        (interpolatory quadrature weights)
    M   (N, N)   M_ij = int_0^1 h_i h_j   (eq. mortarM)
    """

    def __init__(self, N):
        self.N = N
        self.X = solution_points(N)
        self.Xf = flux_points(N)
        self.I = np.array([[lagrange(self.X, i, xk) for i in range(N)] for xk in self.Xf])
        self.D = np.array([[lagrange_deriv(self.Xf, k, xi) for k in range(N + 1)] for xi in self.X])
        self.hp = [lagrange_poly(self.X, i) for i in range(N)]
        self.w = np.array([_integrate01(p) for p in self.hp])
        self.M = np.array([[_integrate01(a * b) for b in self.hp] for a in self.hp])
        self.Minv = np.linalg.inv(self.M)

    def overlap(self, o, s):
        """A[i, j] = int_0^1 h_i(z) h_j(o + s z) dz.

        Row i is the mortar basis, column j the face basis: with a face
        coordinate xi = o + s z on the mortar (eq. xz), the unweighted L2
        projection of eq. (prjQ1) reads M q_mortar = A q_face.  The paper's
        eq. (mortarS) prints the same integral with the index roles swapped;
        eq. (prjQ1) fixes which index is the test function.
        """
        N = self.N
        lin = Legendre.cast(Polynomial([o, s]), domain=[0.0, 1.0])
        comp = [h(lin) for h in self.hp]          # h_j(o + s z) as a series in z
        return np.array([[_integrate01(self.hp[i] * comp[j]) for j in range(N)]
                         for i in range(N)])

    def forward(self, o, s):
        """Face -> mortar projection, eq. (prjQ2): M^-1 A."""
        return self.Minv @ self.overlap(o, s)

    def backward(self, o, s):
        """Mortar -> face projection of one mortar, eq. (prjF2): s M^-1 A^T."""
        return s * (self.Minv @ self.overlap(o, s).T)
