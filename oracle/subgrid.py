"""Learned per-element subgrid correction: the per-element features, the
fine-to-coarse restriction of nested meshes, and a small MLP with its loss
gradient and Adam step.  FP64 test infrastructure: only the tests,
__graft_entry__.smoke() and bench.py's CPU-baseline leg import it.

This extension is not in the paper.  It reuses the paper's ingredients:
  * the element state Q at the solution points and the face traces, the
    solution interpolated to the flux points on the element boundary
    (Sec. 3.1, eq. Qt);
  * the nodal Lagrange basis h_i on the solution points (eq. hbasis), with
    which a coarse element's polynomial is formed.

Features of element e (4 N^2 + 16 N values, 84 at N = 3):
  * first Q[v, j, i, e] in (v, j, i) order;
  * then, for each local face f and each face point p in the face's own
    parameter order, the 4 variables of the neighbour's trace at that face
    point.  An interior or periodic face takes the neighbour's trace; a
    boundary or sliding face takes the element's own.

Restriction (nested meshes): every coarse cell is split 2 x 2 in its own
reference square, so child (a, b) covers xi in [a/2, (a+1)/2] and
eta in [b/2, (b+1)/2].  The coarse state is the L2 projection, in the
parent's reference coordinates, of the fine piecewise polynomial onto the
coarse degree-(Nc-1) polynomials, evaluated at the coarse solution points.
The projection is a tensor product of 1-D operators R[a] (Nc x Nf), one per
child half, with integrals exact by Gauss-Legendre quadrature.

MLP: x -> tanh(W1 xn + b1) -> tanh(W2 . + b2) -> W3 . + b3 = yn, with
xn = (x - mu_x) / sig_x and y = yn sig_y + mu_y.  The loss is the mean
over samples and outputs of (yn - tn)^2 with tn = (t - mu_y) / sig_y.
With bf16=True the matrix-product operands are rounded to bfloat16 (round
to nearest, ties to even) where a BF16 matrix engine rounds them.  The
products and sums stay in FP64.
"""
import numpy as np
from .basis import lagrange, solution_points
from .ssd import SSD


# ----------------------------------------------------------------------------
# bfloat16 rounding
# ----------------------------------------------------------------------------
def bf16(x):
    """Round to bfloat16 (8 significant bits, FP32 exponent range), nearest
    with ties to even, from the FP32 value of x; returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------
def n_features(N):
    return 4 * N * N + 16 * N


def features(ssd, Q):
    """(E, 4N^2 + 16N) features of every element of state Q[v, j, i, e]."""
    ops, N, E = ssd.ops, ssd.N, ssd.E
    q = np.moveaxis(np.asarray(Q, dtype=float), 3, 1)            # (4, E, N, N) [v, e, j, i]
    qxi = np.einsum("ki,veji->vejk", ops.I, q)                    # xi-FPs (4, E, N, N+1)
    qeta = np.einsum("kj,veji->veki", ops.I, q)                   # eta-FPs (4, E, N+1, N)
    T = SSD._faces(qxi, qeta, N)                                  # (4, E, 4, N)
    Tn = ssd._neighbor(T)                                         # neighbour's, face-aligned
    own = q.transpose(1, 0, 2, 3).reshape(E, 4 * N * N)           # (v, j, i)
    nbr = Tn.transpose(1, 2, 3, 0).reshape(E, 16 * N)             # (f, p, v)
    return np.concatenate([own, nbr], axis=1)


# ----------------------------------------------------------------------------
# restriction of a nested fine mesh to its coarse parent mesh
# ----------------------------------------------------------------------------
def restriction_1d(Nc, Nf):
    """R[a] (Nc x Nf): coarse SP values of the L2 projection onto degree
    Nc-1 polynomials on [0, 1] of the fine basis function m of child half a
    (h^f_m(2 xi - a) on [a/2, (a+1)/2], zero on the other half).  The
    integrands are polynomials of degree at most Nc + Nf - 2, integrated
    exactly by Gauss-Legendre quadrature of Nc + Nf points per half."""
    Xc, Xf = solution_points(Nc), solution_points(Nf)
    g, w = np.polynomial.legendre.leggauss(Nc + Nf)
    z, w = 0.5 * (g + 1.0), 0.5 * w                               # on [0, 1]
    hc = np.array([lagrange(Xc, k, z) for k in range(Nc)])        # (Nc, Q)
    M = (hc * w) @ hc.T
    R = np.empty((2, Nc, Nf))
    for a in range(2):
        xi = 0.5 * (a + z)                                        # quadrature on the half
        hck = np.array([lagrange(Xc, k, xi) for k in range(Nc)])
        hfm = np.array([lagrange(Xf, m, z) for m in range(Nf)])   # h^f_m(2 xi - a) = h^f_m(z)
        b = 0.5 * (hck * w) @ hfm.T
        R[a] = np.linalg.solve(M, b)
    return R


def projection_1d(Nc, Nf):
    """P (Nc x Nf): coarse SP values of the L2 projection onto degree Nc-1
    polynomials on [0, 1] of the basis function m of Nf points on the same
    interval (lowering the order on one mesh)."""
    Xc, Xf = solution_points(Nc), solution_points(Nf)
    g, w = np.polynomial.legendre.leggauss(Nc + Nf)
    z, w = 0.5 * (g + 1.0), 0.5 * w
    hc = np.array([lagrange(Xc, k, z) for k in range(Nc)])
    hf = np.array([lagrange(Xf, m, z) for m in range(Nf)])
    return np.linalg.solve((hc * w) @ hc.T, (hc * w) @ hf.T)


def restrict(Qf, children, Nc):
    """Coarse state Qc[v, j, i, c] from the fine state Qf[v, j, i, e] of the
    nested mesh; children[c, a + 2 b] is the fine element of child (a, b).
    children None: the same mesh at a lower order (projection per element)."""
    Qf = np.asarray(Qf, dtype=float)
    Nf = Qf.shape[1]
    if children is None:
        P = projection_1d(Nc, Nf)
        return np.einsum("JF,IG,vFGc->vJIc", P, P, Qf)
    R = restriction_1d(Nc, Nf)
    ch = np.asarray(children)
    out = np.zeros((Qf.shape[0], Nc, Nc, len(ch)))
    for b in range(2):
        for a in range(2):
            q = Qf[..., ch[:, a + 2 * b]]                         # (4, Nf, Nf, Ec)
            out += np.einsum("JF,IG,vFGc->vJIc", R[b], R[a], q)
    return out


def targets(ssd_f, ssd_c, children, Qf, theta, omega):
    """Per-element correction that makes the coarse residual of the
    restricted state equal the restriction of the fine residual:
    restrict(R_f(Qf)) - R_c(restrict(Qf)), as (Ec, 4 Nc^2) rows."""
    Nc = ssd_c.N
    Rf = ssd_f.residual(Qf, theta, omega)
    Qc = restrict(Qf, children, Nc)
    d = restrict(Rf, children, Nc) - ssd_c.residual(Qc, theta, omega)
    return d.transpose(3, 0, 1, 2).reshape(ssd_c.E, 4 * Nc * Nc), Qc


def trajectory_targets(ssd_f, ssd_c, children, Qf, Qc, theta, omega, rate):
    """Targets along a corrected coarse run (a posteriori training): at the
    coarse run's state Qc, the correction that makes its dQ/dt the
    restricted fine dQ/dt and also relaxes Qc towards the restricted fine
    state at `rate`:  restrict(R_f(Qf)) - R_c(Qc) + rate (restrict(Qf) - Qc),
    as (Ec, 4 Nc^2) rows.  At Qc = restrict(Qf) it is the a priori target."""
    Nc = ssd_c.N
    Rf = ssd_f.residual(Qf, theta, omega)
    Qr = restrict(Qf, children, Nc)
    d = restrict(Rf, children, Nc) - ssd_c.residual(Qc, theta, omega) + rate * (Qr - Qc)
    return d.transpose(3, 0, 1, 2).reshape(ssd_c.E, 4 * Nc * Nc)


# ----------------------------------------------------------------------------
# the MLP
# ----------------------------------------------------------------------------
class MLP:
    """Two tanh hidden layers of width H between n_in inputs and n_out
    outputs, in FP64, with the input and output normalisation."""

    def __init__(self, W1, b1, W2, b2, W3, b3, mu_x=None, sig_x=None, mu_y=None, sig_y=None):
        self.p = {k: np.asarray(v, dtype=float) for k, v in
                  dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3).items()}
        n_in, n_out = self.p["W1"].shape[1], self.p["W3"].shape[0]
        self.mu_x = np.zeros(n_in) if mu_x is None else np.asarray(mu_x, dtype=float)
        self.sig_x = np.ones(n_in) if sig_x is None else np.asarray(sig_x, dtype=float)
        self.mu_y = np.zeros(n_out) if mu_y is None else np.asarray(mu_y, dtype=float)
        self.sig_y = np.ones(n_out) if sig_y is None else np.asarray(sig_y, dtype=float)

    def _in(self, X, bf, noise=None):
        X = np.asarray(X, dtype=float)
        if not bf:
            xn = (X - self.mu_x) / self.sig_x
            return xn if noise is None else xn + noise
        # as a kernel does it: FP32 difference times the FP32 reciprocal
        f32 = np.float32
        xn = (X.astype(f32) - self.mu_x.astype(f32)) * (f32(1.0) / self.sig_x.astype(f32))
        if noise is not None:
            xn = xn + np.asarray(noise, dtype=f32)
        return bf16(xn)

    def forward(self, X, bf=False, noise=None):
        """Normalised outputs yn and the activations (a1, h1, a2, h2, a3);
        `noise` (rows x n_in) is added to the normalised inputs."""
        p = self.p
        r = bf16 if bf else (lambda v: v)
        a1 = self._in(X, bf, noise)
        h1 = np.tanh(a1 @ r(p["W1"]).T + p["b1"])
        a2 = r(h1)
        h2 = np.tanh(a2 @ r(p["W2"]).T + p["b2"])
        a3 = r(h2)
        yn = a3 @ r(p["W3"]).T + p["b3"]
        return yn, (a1, h1, a2, h2, a3)

    def predict(self, X, bf=False):
        yn, _ = self.forward(X, bf)
        return yn * self.sig_y + self.mu_y

    def loss_grads(self, X, T, bf=False, noise=None):
        """Loss and its gradient with respect to every parameter (inputs
        perturbed by `noise` in normalised units, if given)."""
        p = self.p
        r = bf16 if bf else (lambda v: v)
        yn, (a1, h1, a2, h2, a3) = self.forward(X, bf, noise)
        tn = (np.asarray(T, dtype=float) - self.mu_y) / self.sig_y
        B, n_out = yn.shape
        d = yn - tn
        L = np.mean(d * d)
        g3 = 2.0 * d / (B * n_out)                                # dL/dyn
        G = {}
        G["W3"] = r(g3).T @ a3
        G["b3"] = g3.sum(0)
        gz2 = (r(g3) @ r(p["W3"])) * (1.0 - h2 * h2)
        G["W2"] = r(gz2).T @ a2
        G["b2"] = gz2.sum(0)
        gz1 = (r(gz2) @ r(p["W2"])) * (1.0 - h1 * h1)
        G["W1"] = r(gz1).T @ a1
        G["b1"] = gz1.sum(0)
        return L, G


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), in place, at step count t >= 1."""
    for k in params:
        g = grads[k]
        m[k] = beta1 * m[k] + (1.0 - beta1) * g
        v[k] = beta2 * v[k] + (1.0 - beta2) * g * g
        mh = m[k] / (1.0 - beta1 ** t)
        vh = v[k] / (1.0 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def corrected_rk3(ssd, mlp, Q, t, dt, nsteps, bf=False, per_step=False):
    """SSP-RK3 of dQ/dt = R(Q) + C, C the MLP output laid back out as
    [v, j, i, e] (the correction of the coarse run): C(Q) of each stage's
    input, or (per_step) C(Q^n) of the step's start for all its stages."""
    N = ssd.N

    def corr(U):
        C = mlp.predict(features(ssd, U), bf)                     # (E, 4 N^2)
        return C.reshape(ssd.E, 4, N, N).transpose(1, 2, 3, 0)

    U = np.asarray(Q, dtype=float).copy()
    for s in range(nsteps):
        tn = t + s * dt
        Cn = corr(U) if per_step else None

        def rhs(V, tau):
            return ssd.residual(V, ssd.theta(tau), ssd.case["omega"]) + (
                Cn if per_step else corr(V))

        U1 = U + dt * rhs(U, tn)
        U2 = 0.75 * U + 0.25 * (U1 + dt * rhs(U1, tn + dt))
        U = U / 3.0 + 2.0 / 3.0 * (U2 + dt * rhs(U2, tn + 0.5 * dt))
    return U


def training_noise(seed, step, batch, n_in, std):
    """Input noise of one training step: std * (2u - 1) sqrt(3) for
    minibatch position s and input i, u the top 24 bits (times 2^-24) of
    SplitMix64 of stream `seed` at counter (step << 32) + s n_in + i; in FP32
    as the kernels form it."""
    from workloads.rng import splitmix64
    s = np.arange(batch, dtype=np.uint64)[:, None]
    i = np.arange(n_in, dtype=np.uint64)[None, :]
    z = splitmix64(seed, (np.uint64(step) << np.uint64(32)) + s * np.uint64(n_in) + i)
    f32 = np.float32
    u = (z >> np.uint64(40)).astype(f32) * f32(2.0 ** -24)
    eps = (f32(2.0) * u - f32(1.0)) * f32(1.7320508075688772)
    return f32(std) * eps
