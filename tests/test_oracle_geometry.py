"""Pins of the oracle's element maps and metrics (Sec. 2.3, Sec. 3.1).

The serendipity shape functions are checked for the nodal (cardinal)
property and for reproducing the serendipity polynomial space; metrics of
an element whose nodes sample a known map must equal that map's exact
derivatives; cell areas integrated from |J| must add up to the domain.
"""
import numpy as np
import pytest

from oracle.basis import Operators
from oracle.geometry import Geometry, bilinear, serendipity
from workloads import meshes as M
from workloads.meshes import NODE_REF, GEOM_CUBIC, GEOM_LINEAR


def test_shape_functions_cardinal():
    Nf, _, _ = serendipity(NODE_REF[:, 0], NODE_REF[:, 1])
    assert np.allclose(Nf, np.eye(12), atol=1e-13)
    rng = np.random.default_rng(0)
    xi, eta = rng.uniform(0, 1, 30), rng.uniform(0, 1, 30)
    for fun in (serendipity, bilinear):
        Nf, Nx, Ny = fun(xi, eta)
        assert np.allclose(Nf.sum(axis=1), 1.0, atol=1e-13)
        assert np.allclose(Nx.sum(axis=1), 0.0, atol=1e-12)
        assert np.allclose(Ny.sum(axis=1), 0.0, atol=1e-12)


def _element_from_map(fx, fy, geom):
    xy = np.stack([fx(NODE_REF[:, 0], NODE_REF[:, 1]), fy(NODE_REF[:, 0], NODE_REF[:, 1])], axis=-1)
    return dict(xy=xy[None], geom=np.array([geom]), zone=np.array([0]), center=np.zeros(2))


@pytest.mark.parametrize("N", [2, 4])
def test_cubic_map_reproduced(N):
    """x = xi + 0.1 xi^3 eta + 0.05 eta^3, y = eta + 0.2 xi^2 eta - 0.1 xi eta^3
    lies in the serendipity space, so the 12-node map is exact."""
    fx = lambda a, b: a + 0.1 * a ** 3 * b + 0.05 * b ** 3
    fy = lambda a, b: b + 0.2 * a * a * b - 0.1 * a * b ** 3
    dx = (lambda a, b: 1 + 0.3 * a * a * b, lambda a, b: 0.1 * a ** 3 + 0.15 * b * b)
    dy = (lambda a, b: 0.4 * a * b - 0.1 * b ** 3, lambda a, b: 1 + 0.2 * a * a - 0.3 * a * b * b)
    ops = Operators(N)
    geo = Geometry(_element_from_map(fx, fy, GEOM_CUBIC), ops)
    from oracle.geometry import point_sets
    for name, (gxi, geta) in point_sets(ops).items():
        d = geo.data[name]
        assert np.allclose(d["x"][0], fx(gxi, geta), atol=1e-13)
        assert np.allclose(d["y"][0], fy(gxi, geta), atol=1e-13)
        assert np.allclose(d["x_xi"][0], dx[0](gxi, geta), atol=1e-12)
        assert np.allclose(d["x_eta"][0], dx[1](gxi, geta), atol=1e-12)
        assert np.allclose(d["y_xi"][0], dy[0](gxi, geta), atol=1e-12)
        assert np.allclose(d["y_eta"][0], dy[1](gxi, geta), atol=1e-12)


def test_bilinear_map_and_rotation():
    fx = lambda a, b: 1.0 + 2.0 * a + 0.5 * b + 0.3 * a * b
    fy = lambda a, b: -1.0 + 0.2 * a + 1.5 * b - 0.1 * a * b
    ops = Operators(3)
    el = _element_from_map(fx, fy, GEOM_LINEAR)
    el["zone"] = np.array([1])
    el["center"] = np.array([0.3, -0.2])
    geo = Geometry(el, ops)
    sp = geo.data["sp"]
    gxi, geta = np.meshgrid(ops.X, ops.X, indexing="xy")
    J = (2.0 + 0.3 * geta) * (1.5 - 0.1 * gxi) - (0.5 + 0.3 * gxi) * (0.2 - 0.1 * geta)
    assert np.allclose(geo.detJ[0], J, atol=1e-13)
    th = 0.9
    r = geo.at(th)["sp"]
    Jr = r["x_xi"] * r["y_eta"] - r["x_eta"] * r["y_xi"]
    assert np.allclose(Jr, geo.detJ, atol=1e-13)
    c = el["center"]
    x0, y0 = sp["x"] - c[0], sp["y"] - c[1]
    assert np.allclose(r["x"], c[0] + np.cos(th) * x0 - np.sin(th) * y0, atol=1e-13)
    assert np.allclose(np.hypot(r["x"] - c[0], r["y"] - c[1]), np.hypot(x0, y0), atol=1e-13)


@pytest.mark.parametrize("N", [3, 4])
def test_areas(N):
    ops = Operators(N)
    W = np.outer(ops.w, ops.w)[None]
    box = M.box_mesh(5, 4, L=(2.0, 3.0), distort=0.15, curved=0.05)
    g = Geometry(box, ops)
    # cubic cells with N >= 3: |J| has degree <= 2N-2 ... integrated exactly
    # only up to the quadrature degree; areas still sum to the box exactly
    # because interior edge bends cancel between neighbours.
    assert abs((W * g.detJ).sum() - 6.0) < 1e-3
    box = M.box_mesh(5, 4, L=(2.0, 3.0), distort=0.15)
    g = Geometry(box, ops)
    assert abs((W * g.detJ).sum() - 6.0) < 1e-12
    cm = M.couette_mesh(8, 32)
    g = Geometry(cm, ops)
    area = (W * g.detJ).sum()
    assert abs(area - np.pi * 3.0) < 2e-4          # cubic arcs, Delta = 11.25 deg
    assert np.all(g.detJ > 0)
    cm2 = M.couette_mesh(16, 64)
    area2 = (W * Geometry(cm2, ops).detJ).sum()
    assert abs(area2 - np.pi * 3.0) < abs(area - np.pi * 3.0) / 8
