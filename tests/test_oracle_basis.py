"""Pins of the oracle's 1-D operators against what the mathematics fixes.

Point sets and bases (Sec. 3.1, eqs. hbasis, lbasis), mortar matrices
(Sec. 3.2, eqs. mortarM, mortarS, prjQ2, prjF2).  Reference values come from
high-precision quadrature (mpmath) of the product-form cardinal
polynomials, and from exact Legendre polynomials (sympy), never from the
oracle's own polynomial algebra.
"""
import mpmath as mp
import numpy as np
import pytest
import sympy as sp

from oracle.basis import Operators, flux_points, solution_points

NS = [2, 3, 4, 5, 6]


@pytest.mark.parametrize("N", NS)
def test_point_sets(N):
    X = solution_points(N)
    # Chebyshev-Gauss: roots of T_N(2X-1), symmetric about 1/2
    t = sp.chebyshevt(N, sp.Symbol("z"))
    for x in X:
        assert abs(float(t.subs("z", 2 * x - 1))) < 1e-12
    assert np.allclose(X + X[::-1], 1.0, atol=1e-15)
    Xf = flux_points(N)
    assert Xf[0] == 0.0 and Xf[-1] == 1.0 and len(Xf) == N + 1
    P = sp.legendre(N - 1, sp.Symbol("z"))
    for x in Xf[1:-1]:
        assert abs(float(P.subs("z", 2 * x - 1))) < 1e-12
    assert np.all(np.diff(Xf) > 0)
    # staggering: every SP lies strictly between consecutive FPs
    assert np.all((X > Xf[:-1]) & (X < Xf[1:]))


@pytest.mark.parametrize("N", NS)
def test_interpolation_and_derivative_exactness(N):
    ops = Operators(N)
    # cardinal + partition of unity of the SP basis at the FPs
    assert np.allclose(ops.I.sum(axis=1), 1.0, atol=1e-13)
    # I interpolates polynomials of degree <= N-1 exactly
    for m in range(N):
        assert np.allclose(ops.I @ ops.X ** m, ops.Xf ** m, atol=1e-13)
    # D differentiates degree <= N exactly (flux polynomial degree, eq. Ft)
    for m in range(N + 1):
        d = m * ops.X ** (m - 1) if m else np.zeros(N)
        assert np.allclose(ops.D @ ops.Xf ** m, d, atol=1e-11)
    assert np.allclose(ops.D.sum(axis=1), 0.0, atol=1e-12)


@pytest.mark.parametrize("N", NS)
def test_weights_and_mass(N):
    ops = Operators(N)
    assert abs(ops.w.sum() - 1.0) < 1e-14
    assert np.allclose(ops.M @ np.ones(N), ops.w, atol=1e-14)
    # quadrature exact for degree N-1 (interpolatory on N points)
    for m in range(N):
        assert abs(ops.w @ ops.X ** m - 1.0 / (m + 1)) < 1e-13
    assert np.allclose(ops.M, ops.M.T)
    assert np.all(np.linalg.eigvalsh(ops.M) > 0)


def _mp_basis(N):
    mp.mp.dps = 40
    X = [(1 - mp.cos((2 * s - 1) * mp.pi / (2 * N))) / 2 for s in range(1, N + 1)]

    def h(i, x):
        r = mp.mpf(1)
        for s in range(N):
            if s != i:
                r *= (x - X[s]) / (X[i] - X[s])
        return r
    return h


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("o,s", [(0.0, 1.0), (0.0, 0.375), (0.375, 0.625), (0.2, 0.8),
                                 (0.9, 0.1), (0.0, 0.0)])
def test_mortar_matrices_high_precision(N, o, s):
    """M and A(o,s) against 40-digit quadrature of the product-form bases."""
    ops = Operators(N)
    h = _mp_basis(N)
    M = np.array([[float(mp.quad(lambda z: h(i, z) * h(j, z), [0, 1])) for j in range(N)]
                  for i in range(N)])
    assert np.allclose(ops.M, M, rtol=0, atol=1e-12)
    A = np.array([[float(mp.quad(lambda z: h(i, z) * h(j, o + s * z), [0, 1])) for j in range(N)]
                  for i in range(N)])
    assert np.allclose(ops.overlap(o, s), A, rtol=0, atol=5e-12)


@pytest.mark.parametrize("N", NS)
def test_overlap_special_cases(N):
    ops = Operators(N)
    assert np.allclose(ops.overlap(0.0, 1.0), ops.M, atol=1e-14)
    # a mortar of zero length samples the face at one point: A = w h(o)^T
    o = 0.3
    h_o = np.array([np.prod([(o - ops.X[t]) / (ops.X[j] - ops.X[t]) for t in range(N) if t != j])
                    for j in range(N)])
    assert np.allclose(ops.overlap(o, 0.0), np.outer(ops.w, h_o), atol=1e-13)
    # rows of A sum to w (the face basis sums to one)
    A = ops.overlap(0.25, 0.5)
    assert np.allclose(A.sum(axis=1), ops.w, atol=1e-14)


@pytest.mark.parametrize("N", NS)
@pytest.mark.parametrize("dlt", [0.0, 0.1, 0.5, 0.77, 1.0 - 1e-9])
def test_projection_identities(N, dlt):
    """Forward projection reproduces polynomials of degree N-1 on the mortar
    (eq. prjQ1 is an L2 projection); the two back-projections invert the two
    forward ones; integrals are preserved with the s factor of eq. prjF2."""
    ops = Operators(N)
    pairs = [(0.0, 1.0 - dlt), (1.0 - dlt, dlt)]
    rng = np.random.default_rng(N)
    c = rng.standard_normal(N)
    q = np.polynomial.polynomial.polyval(ops.X, c)
    for o, s in pairs:
        Pf = ops.forward(o, s)
        assert np.allclose(Pf @ q, np.polynomial.polynomial.polyval(o + s * ops.X, c), atol=1e-10)
        assert np.allclose(Pf @ np.ones(N), 1.0, atol=1e-12)
        # integral over the mortar in face units equals s * integral in z
        f = rng.standard_normal(N)
        assert abs(ops.w @ (ops.backward(o, s) @ f) - s * (ops.w @ f)) < 1e-12
    Rt = sum(ops.backward(o, s) @ ops.forward(o, s) for o, s in pairs)
    assert np.allclose(Rt, np.eye(N), atol=1e-9)
