"""Pins of the subgrid-correction oracle (oracle/subgrid.py) against what
mathematics fixes: bfloat16 rounding of known values, polynomial exactness
and the orthogonality of the L2 restriction, continuity of the neighbour
traces, finite differences of the loss, the small-weight linearisation of
the MLP and the first Adam step.  CPU only."""
import numpy as np
import pytest
from numpy.polynomial import legendre as nleg

from oracle import subgrid as S
from oracle.basis import solution_points
from oracle.ssd import SSD
from workloads import cases as C
from workloads import meshes as M


def test_bf16_known_values():
    one = 1.0
    u = 2.0 ** -7                                                   # bf16 spacing at 1
    vals = np.array([one, one + u / 2, one + 3 * u / 2, one + u / 2 + 2.0 ** -20, -2.5, 0.0,
                     3.0e38, 1.0e-39])
    want = np.array([one, one, one + 2 * u, one + u, -2.5, 0.0, None, None], dtype=object)
    got = S.bf16(vals)
    for g, w in zip(got[:6], want[:6]):
        assert g == w
    # the largest finite values round up into the FP32 overflow like FP32 does
    assert S.bf16(np.float32(3.0e38)) > 2.9e38
    # results are representable: rounding twice changes nothing
    r = np.random.default_rng(1).normal(size=1000) * 10.0 ** np.random.default_rng(2).integers(-8, 8, 1000)
    assert np.array_equal(S.bf16(S.bf16(r)), S.bf16(r))
    assert np.all(np.abs(S.bf16(r) - r) <= 2.0 ** -8 * np.abs(r) * (1 + 1e-7))


@pytest.mark.parametrize("Nc,Nf", [(3, 6), (2, 4), (3, 3)])
def test_restriction_reproduces_coarse_polynomials(Nc, Nf):
    """A polynomial of degree < Nc sampled on both child halves restricts to
    its own values at the coarse solution points."""
    R = S.restriction_1d(Nc, Nf)
    Xc, Xf = solution_points(Nc), solution_points(Nf)
    rng = np.random.default_rng(Nc * 10 + Nf)
    for _ in range(3):
        c = rng.normal(size=Nc)
        u = lambda x: np.polyval(c, x)
        got = R[0] @ u(Xf / 2) + R[1] @ u((1 + Xf) / 2)
        assert np.allclose(got, u(Xc), atol=1e-12)


@pytest.mark.parametrize("Nc,Nf", [(3, 6), (2, 5)])
def test_restriction_is_orthogonal_projection(Nc, Nf):
    """For a fine piecewise polynomial u (independent on each half), u - Pu is
    orthogonal to every coarse polynomial, by Gauss-Legendre quadrature on
    each half (exact for these degrees)."""
    R = S.restriction_1d(Nc, Nf)
    Xc, Xf = solution_points(Nc), solution_points(Nf)
    rng = np.random.default_rng(5)
    vals = rng.normal(size=(2, Nf))                                # fine nodal values per half
    coarse = R[0] @ vals[0] + R[1] @ vals[1]                      # coarse nodal values
    g, w = nleg.leggauss(Nc + Nf + 2)
    z, w = 0.5 * (g + 1.0), 0.5 * w

    def lag(nodes, vals, x):
        out = np.zeros_like(x)
        for i in range(len(nodes)):
            li = np.ones_like(x)
            for s in range(len(nodes)):
                if s != i:
                    li *= (x - nodes[s]) / (nodes[i] - nodes[s])
            out += vals[i] * li
        return out

    for k in range(Nc):
        test_fn = np.zeros(Nc)
        test_fn[k] = 1.0
        tot = 0.0
        for a in range(2):
            x = 0.5 * (a + z)
            u = lag(Xf, vals[a], z)
            pu = lag(Xc, coarse, x)
            tot += 0.5 * np.sum(w * lag(Xc, test_fn, x) * (u - pu))
        assert abs(tot) < 1e-14


@pytest.fixture(scope="module")
def nested():
    return M.ellipse_mesh(K=32, n_in=4, n_out=4, radius=1.5, box_half=4.0, first_in=0.05,
                          first_out=0.1, nested=True)


def test_nested_mesh_children_cover_parents(nested):
    coarse, fine, ch = nested
    assert len(fine["zone"]) == 4 * len(coarse["zone"])
    assert sorted(ch.ravel().tolist()) == list(range(len(fine["zone"])))
    # child (a, b) holds the parent's corner (a, b)
    for a in range(2):
        for b in range(2):
            corner = [0, 3, 9, 6][a + 2 * b]
            assert np.allclose(fine["xy"][ch[:, a + 2 * b], corner], coarse["xy"][:, corner],
                               atol=1e-12)
    assert np.all(fine["zone"][ch] == coarse["zone"][:, None])


def test_restrict_linear_field(nested):
    """A field linear in x and y is bilinear on bilinear cells, so it
    restricts exactly there; on cubic cells to the cell's curvature."""
    coarse, fine, ch = nested
    case = C.ellipse_case()
    sf, sc = SSD(fine, case, 6), SSD(coarse, case, 3)
    xf, yf = sf.sp_coords(0.0)
    xc, yc = sc.sp_coords(0.0)
    f = lambda x, y: np.stack([1 + 0.3 * x - 0.2 * y, 0.5 * y, -x, 2 + x + y])
    Qc = S.restrict(f(xf, yf), ch, 3)
    err = np.abs(Qc - f(xc, yc)).max(axis=(0, 1, 2))
    lin = coarse["geom"] == M.GEOM_LINEAR
    assert err[lin].max() < 1e-12
    assert err[~lin].max() < 1e-3


def test_features_uniform_and_continuous():
    """Uniform state: every feature is that state.  A linear field on a
    relabelled straight-sided box: across interior faces the neighbour trace
    at each face point equals the field at the point (continuity, reversal;
    the field jumps across the periodic cuts)."""
    case = C.vortex_case()
    box = M.box_mesh(5, 4, L=(2.0, 1.5), distort=0.1, zone=0)
    mesh = M.relabel(box, np.random.default_rng(3).integers(0, 4, len(box["zone"])))
    N = 3
    ssd = SSD(mesh, case, N)
    E = ssd.E
    q0 = np.array([1.1, 0.2, -0.3, 2.5])
    F = S.features(ssd, np.broadcast_to(q0[:, None, None, None], (4, N, N, E)))
    assert F.shape == (E, S.n_features(N))
    assert np.allclose(F[:, :36], np.repeat(q0, 9)[None, :])
    assert np.allclose(F[:, 36:], np.tile(q0, 12)[None, :])
    # linear field: neighbour traces of interior faces = field at own face points
    x, y = ssd.sp_coords(0.0)
    lin = lambda x, y: np.stack([1 + 0.3 * x, 0.5 * y - x, 0.2 + y, 3 - x + 2 * y])
    F = S.features(ssd, lin(x, y))
    g = ssd.geo.at(0.0)
    fx = np.stack([g["feta"]["x"][:, 0, :], g["fxi"]["x"][:, :, N],
                   g["feta"]["x"][:, N, :], g["fxi"]["x"][:, :, 0]], axis=1)   # (E, 4, N)
    fy = np.stack([g["feta"]["y"][:, 0, :], g["fxi"]["y"][:, :, N],
                   g["feta"]["y"][:, N, :], g["fxi"]["y"][:, :, 0]], axis=1)
    want = lin(fx, fy).transpose(1, 2, 3, 0).reshape(E, 48)     # (e, f, p, v)
    inner = np.repeat(np.asarray(mesh["face_kind"]) == M.FACE_INTERIOR, 12, axis=1)
    assert np.abs(F[:, 36:] - want)[inner].max() < 1e-12
    assert ssd.rev.sum() > 0


def _mlp(rng, n_in=7, H=5, n_out=3, scale=0.7):
    return S.MLP(rng.normal(size=(H, n_in)) * scale, rng.normal(size=H) * 0.1,
                 rng.normal(size=(H, H)) * scale, rng.normal(size=H) * 0.1,
                 rng.normal(size=(n_out, H)) * scale, rng.normal(size=n_out) * 0.1,
                 mu_x=rng.normal(size=n_in), sig_x=rng.uniform(0.5, 2, n_in),
                 mu_y=rng.normal(size=n_out), sig_y=rng.uniform(0.5, 2, n_out))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(11)
    net = _mlp(rng)
    X = rng.normal(size=(9, 7))
    T = rng.normal(size=(9, 3))
    L, G = net.loss_grads(X, T)
    h = 1e-6
    for k, P in net.p.items():
        flat = P.reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = net.loss_grads(X, T)
            flat[idx] = old - h
            Lm, _ = net.loss_grads(X, T)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - G[k].reshape(-1)[idx]) < 1e-7 * (1 + abs(fd)), (k, idx)


def test_mlp_small_weight_linearisation_and_symmetry():
    """With weights scaled by eps and zero biases the network is W3 W2 W1 xn
    to relative O(eps^2); with zero biases it is odd in xn."""
    rng = np.random.default_rng(4)
    W1, W2, W3 = rng.normal(size=(6, 5)), rng.normal(size=(6, 6)), rng.normal(size=(2, 6))
    z6, z2 = np.zeros(6), np.zeros(2)
    X = rng.normal(size=(4, 5))
    rel = []
    for eps in (1e-2, 1e-3):
        net = S.MLP(eps * W1, z6, eps * W2, z6, eps * W3, z2)
        yn, _ = net.forward(X)
        lin = eps ** 3 * X @ W1.T @ W2.T @ W3.T
        rel.append(np.abs(yn - lin).max() / np.abs(lin).max())
    # tanh z = z - z^3/3 + ...: the relative deviation falls as eps^2
    assert rel[0] < 1e-2 and 70 < rel[0] / rel[1] < 130
    net = S.MLP(W1, z6, W2, z6, W3, z2)
    assert np.allclose(net.forward(-X)[0], -net.forward(X)[0], atol=1e-14)


def test_mlp_bf16_forward_within_rounding():
    """BF16 operands change each layer by a few units of 2^-8."""
    rng = np.random.default_rng(8)
    net = _mlp(rng, n_in=84, H=64, n_out=36, scale=0.15)
    X = rng.normal(size=(64, 84))
    y64 = net.predict(X)
    y16 = net.predict(X, bf=True)
    assert np.abs(y16 - y64).max() < 0.05 * np.abs(y64).max()
    assert np.abs(y16 - y64).max() > 0.0


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(2)
    p = {"w": rng.normal(size=10)}
    g = {"w": rng.normal(size=10)}
    m = {"w": np.zeros(10)}
    v = {"w": np.zeros(10)}
    w0 = p["w"].copy()
    S.adam_step(p, g, m, v, 1, lr=1e-3)
    assert np.allclose(p["w"] - w0, -1e-3 * np.sign(g["w"]), rtol=1e-6)


def test_targets_vanish_on_free_stream(nested):
    """A uniform flow is preserved by both meshes (free-stream preservation
    on the moving mesh), so the correction target is zero there."""
    coarse, fine, ch = nested
    case = C.ellipse_case()
    sf, sc = SSD(fine, case, 4), SSD(coarse, case, 2)
    Qf = C.uniform_state(case, 4, len(fine["zone"]))
    T, Qc = S.targets(sf, sc, ch, Qf, 0.3, case["omega"])
    assert np.abs(Qc - C.uniform_state(case, 2, len(coarse["zone"]))).max() < 1e-12
    # on bilinear cells, whose metrics the flux polynomials hold exactly (the
    # cubic cells on the wall and the interface preserve a uniform flow only
    # to their metric error at these orders)
    lin = coarse["geom"] == M.GEOM_LINEAR
    assert lin.sum() > len(lin) // 2
    assert np.abs(T[lin]).max() < 1e-10


def test_training_noise_is_uniform_unit_variance():
    """The training noise is uniform on [-sqrt(3), sqrt(3)) std, so it has
    mean 0 and standard deviation std; distinct steps give distinct noise."""
    z = S.training_noise(7, 3, 256, 84, 0.5).astype(np.float64)
    assert z.shape == (256, 84)
    assert np.all(np.abs(z) <= 0.5 * np.sqrt(3.0))
    assert abs(z.mean()) < 0.01 and abs(z.std() - 0.5) < 0.01
    h, _ = np.histogram(z, bins=8, range=(-0.5 * np.sqrt(3), 0.5 * np.sqrt(3)))
    assert h.min() > 0.9 * h.mean()
    assert not np.array_equal(z, S.training_noise(7, 4, 256, 84, 0.5))
    assert np.array_equal(z, S.training_noise(7, 3, 256, 84, 0.5))


@pytest.mark.parametrize("Nc,Nf", [(3, 6), (5, 6), (4, 4)])
def test_projection_reproduces_and_is_orthogonal(Nc, Nf):
    """Same-mesh order lowering: polynomials of degree < Nc are kept, and the
    remainder is orthogonal to the coarse polynomials (Gauss-Legendre)."""
    P = S.projection_1d(Nc, Nf)
    Xc, Xf = solution_points(Nc), solution_points(Nf)
    rng = np.random.default_rng(Nc + 7 * Nf)
    c = rng.normal(size=Nc)
    assert np.allclose(P @ np.polyval(c, Xf), np.polyval(c, Xc), atol=1e-12)
    vals = rng.normal(size=Nf)
    coarse = P @ vals
    g, w = nleg.leggauss(Nf + 2)
    z, w = 0.5 * (g + 1.0), 0.5 * w
    from oracle.basis import lagrange
    u = sum(vals[m] * lagrange(Xf, m, z) for m in range(Nf))
    pu = sum(coarse[k] * lagrange(Xc, k, z) for k in range(Nc))
    for k in range(Nc):
        assert abs(np.sum(w * lagrange(Xc, k, z) * (u - pu))) < 1e-14
    if Nc == Nf:
        assert np.allclose(P, np.eye(Nc), atol=1e-13)
