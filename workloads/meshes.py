"""Quadrilateral mesh descriptions for the sliding-mesh workloads.

A mesh is a dict of numpy arrays:

  xy         (E, 12, 2) float64  element nodes, see NODE_REF below
  geom       (E,)  int32   GEOM_LINEAR (4 corners, bilinear map) or
                           GEOM_CUBIC (all 12 nodes, cubic serendipity map)
  zone       (E,)  int32   0 stationary, 1 rotating
  nbr        (E, 4) int32  neighbour element across each local face, or -1
  nbr_face   (E, 4) int32  the neighbour's local face index, or -1
  face_kind  (E, 4) int32  FACE_* tag of each local face
  center     (2,)  float64 rotation centre of zone 1
  radius     float         radius of the circular sliding interface (0: none)

Element nodes run counter-clockwise around the reference square [0,1]^2:

  index  0     1      2      3     4      5      6     7      8      9     10     11
  (xi,eta) (0,0) (1/3,0) (2/3,0) (1,0) (1,1/3) (1,2/3) (1,1) (2/3,1) (1/3,1) (0,1) (0,2/3) (0,1/3)

Local faces: 0 is eta=0 (parameter xi), 1 is xi=1 (parameter eta),
2 is eta=1 (parameter xi), 3 is xi=0 (parameter eta).  A face's parameter
runs from its FACE_CORNERS[f][0] node to its FACE_CORNERS[f][1] node.

Nothing here evaluates the spectral-difference method: the generators place
nodes on lines, circles and an ellipse and match faces by their end points.
"""
import numpy as np

FACE_INTERIOR = 0
FACE_PERIODIC = 1
FACE_SLIDING = 2
FACE_WALL_ISOTHERMAL = 3
FACE_WALL_SLIP = 4
FACE_FARFIELD = 5

GEOM_LINEAR = 0
GEOM_CUBIC = 1

NODE_REF = np.array([[0, 0], [1 / 3, 0], [2 / 3, 0], [1, 0], [1, 1 / 3], [1, 2 / 3],
                     [1, 1], [2 / 3, 1], [1 / 3, 1], [0, 1], [0, 2 / 3], [0, 1 / 3]])
FACE_CORNERS = np.array([[0, 3], [3, 6], [9, 6], [0, 9]])
FACE_NODES = np.array([[0, 1, 2, 3], [3, 4, 5, 6], [9, 8, 7, 6], [0, 11, 10, 9]])


# ----------------------------------------------------------------------------
# structured blocks
# ----------------------------------------------------------------------------
def _block(P, curves=None, zone=0, tile=None):
    """Elements of a structured block of nodes P (ni+1, nj+1, 2).

    Element (i, j) has corners P[i,j], P[i+1,j], P[i+1,j+1], P[i,j+1] as its
    (0,0), (1,0), (1,1), (0,1) nodes; xi runs along i and eta along j.
    `curves` maps a line index i to fn(j, t) giving the point a fraction t
    of the way along the j-th edge of that line (edges along eta); those
    edges get curved edge nodes and their elements become GEOM_CUBIC.
    Elements are numbered with j fastest, or, with tile = (tj, ti), in
    consecutive tiles of tj x ti elements (j fastest inside a tile, tiles
    j-major), so that neighbours mostly share a tile.
    """
    curves = curves or {}
    ni, nj = P.shape[0] - 1, P.shape[1] - 1
    c00 = P[:-1, :-1]
    c10 = P[1:, :-1]
    c11 = P[1:, 1:]
    c01 = P[:-1, 1:]
    xy = np.empty((ni, nj, 12, 2))
    xy[:, :, 0] = c00
    xy[:, :, 3] = c10
    xy[:, :, 6] = c11
    xy[:, :, 9] = c01
    xy[:, :, 1] = c00 + (c10 - c00) / 3.0
    xy[:, :, 2] = c00 + 2.0 * (c10 - c00) / 3.0
    xy[:, :, 7] = c01 + 2.0 * (c11 - c01) / 3.0
    xy[:, :, 8] = c01 + (c11 - c01) / 3.0
    xy[:, :, 11] = c00 + (c01 - c00) / 3.0
    xy[:, :, 10] = c00 + 2.0 * (c01 - c00) / 3.0
    xy[:, :, 4] = c10 + (c11 - c10) / 3.0
    xy[:, :, 5] = c10 + 2.0 * (c11 - c10) / 3.0
    geom = np.full((ni, nj), GEOM_LINEAR, np.int32)
    jj = np.arange(nj)
    for line, fn in curves.items():
        if line < ni:      # inner edge (face 3) of elements in row `line`
            xy[line, :, 11] = fn(jj, 1.0 / 3.0)
            xy[line, :, 10] = fn(jj, 2.0 / 3.0)
            geom[line, :] = GEOM_CUBIC
        if line >= 1:      # outer edge (face 1) of elements in row `line`-1
            xy[line - 1, :, 4] = fn(jj, 1.0 / 3.0)
            xy[line - 1, :, 5] = fn(jj, 2.0 / 3.0)
            geom[line - 1, :] = GEOM_CUBIC
    out = dict(xy=xy.reshape(-1, 12, 2), geom=geom.reshape(-1),
               zone=np.full(ni * nj, zone, np.int32), sid=np.arange(ni * nj))
    if tile is not None:
        tj, ti = tile
        # full bands of ti rows use tj x ti tiles; a last band of r < ti rows
        # uses (tj ti / r) x r tiles, so every tile keeps tj ti elements
        r = ni % ti
        tjr = (tj * ti) // r if r else tj
        if nj % tj or (r and ((tj * ti) % r or nj % tjr)):
            raise ValueError("block size does not split into whole tiles")
        ii, jj = np.meshgrid(np.arange(ni), np.arange(nj), indexing="ij")
        band, il = ii // ti, ii % ti
        last = (ni - r) if r else ni
        w = np.where(ii >= last, tjr, tj)       # tile width along j
        h = np.where(ii >= last, r if r else ti, ti)
        key = ((band * (nj // w) + jj // w) * h + il) * w + jj % w
        order = np.argsort(key.ravel(), kind="stable")
        out = {k: v[order] for k, v in out.items()}
    return out


def _refine_block(P, curves=None):
    """Nodes and curves of the block whose cells are the 2 x 2 children of
    the cells of block (P, curves), each child an exact piece of its
    parent's map.  A parent with a curved edge is its bilinear map plus the
    curve's deviation from the chord blended linearly across the cell, so
    the line through the parent's middle is a curve too: the average of the
    curved edge and the opposite chord.  Returns (Pf, curves_f)."""
    curves = curves or {}
    ni, nj = P.shape[0] - 1, P.shape[1] - 1
    Pf = np.empty((2 * ni + 1, 2 * nj + 1, 2))
    Pf[0::2, 0::2] = P
    Pf[1::2, 0::2] = 0.5 * (P[:-1] + P[1:])
    Pf[0::2, 1::2] = 0.5 * (P[:, :-1] + P[:, 1:])
    Pf[1::2, 1::2] = 0.25 * (P[:-1, :-1] + P[1:, :-1] + P[:-1, 1:] + P[1:, 1:])

    def chord(line, j, t):
        j = np.asarray(j)
        t = np.asarray(t, dtype=float)[..., None]
        return (1.0 - t) * P[line, j] + t * P[line, j + 1]

    def fine_fn(fn):
        def g(jf, t):
            jf = np.asarray(jf)
            return fn(jf // 2, (jf % 2 + np.asarray(t, dtype=float)) / 2.0)
        return g

    def mid_fn(fn, opposite):
        def g(jf, t):
            jf = np.asarray(jf)
            eta = (jf % 2 + np.asarray(t, dtype=float)) / 2.0
            j = jf // 2
            return 0.5 * (fn(j, eta) + chord(opposite, j, eta))
        return g

    curves_f = {}
    jj = np.arange(nj)
    for line, fn in curves.items():
        curves_f[2 * line] = fine_fn(fn)
        Pf[2 * line, 1::2] = fn(jj, 0.5)
        for mid, opp in ((2 * line + 1, line + 1), (2 * line - 1, line - 1)):
            if 0 < mid < 2 * ni:
                if mid in curves_f:
                    raise ValueError("a cell with two curved edges cannot be refined")
                curves_f[mid] = mid_fn(fn, opp)
                Pf[mid, 1::2] = curves_f[mid](2 * jj, 1.0)
    return Pf, curves_f


def _children(coarse_blocks, fine_blocks):
    """children[c, a + 2 b]: the fine element of child (a, b) of coarse
    element c, for blocks refined by _refine_block and concatenated in the
    same order (a along xi = the block's i, b along eta = its j)."""
    out, off_c, off_f = [], 0, 0
    for (bc, nj), bf in zip(coarse_blocks, fine_blocks):
        pos = np.empty(len(bf["sid"]), np.int64)
        pos[bf["sid"]] = np.arange(len(bf["sid"]))
        i, j = bc["sid"] // nj, bc["sid"] % nj
        ch = np.empty((len(bc["sid"]), 4), np.int64)
        for b in range(2):
            for a in range(2):
                ch[:, a + 2 * b] = pos[(2 * i + a) * (2 * nj) + 2 * j + b] + off_f
        out.append(ch)
        off_c += len(bc["sid"])
        off_f += len(bf["sid"])
    return np.concatenate(out).astype(np.int32)


def _concat(blocks):
    return dict(xy=np.concatenate([b["xy"] for b in blocks]),
                geom=np.concatenate([b["geom"] for b in blocks]),
                zone=np.concatenate([b["zone"] for b in blocks]))


def _face_ends(xy):
    """(E, 4, 2, 2): start and end corner of each local face."""
    return xy[:, FACE_CORNERS, :]


def _match(keys_a, keys_b):
    """Pairs (ia, ib) of rows with identical integer keys between two sets."""
    ka = np.ascontiguousarray(keys_a)
    kb = np.ascontiguousarray(keys_b)
    allk = np.concatenate([ka, kb])
    src = np.concatenate([np.zeros(len(ka), np.int8), np.ones(len(kb), np.int8)])
    idx = np.concatenate([np.arange(len(ka)), np.arange(len(kb))])
    order = np.lexsort(allk.T[::-1])
    sk = allk[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    i = np.nonzero(same)[0]
    a, b = order[i], order[i + 1]
    # keep cross-set pairs only, oriented (set A, set B)
    sa, sb = src[a], src[b]
    keep = sa != sb
    a, b, sa = a[keep], b[keep], sa[keep]
    ia = np.where(sa == 0, idx[a], idx[b])
    ib = np.where(sa == 0, idx[b], idx[a])
    return ia, ib


def _quant(p, scale):
    return np.round(p / scale).astype(np.int64)


def connect(mesh, classify, periodic=None, tol=1e-9):
    """Fill nbr, nbr_face and face_kind.

    Faces of the same zone sharing both end points are neighbours.  Faces
    left unmatched are tagged by `classify(ends, zone)` -> FACE_* (vector
    over faces).  `periodic` is an optional list of translation vectors T:
    unmatched faces whose ends + T coincide with another unmatched face's
    ends are paired as FACE_PERIODIC.
    """
    xy, zone = mesh["xy"], mesh["zone"]
    E = xy.shape[0]
    ends = _face_ends(xy).reshape(E * 4, 2, 2)
    fzone = np.repeat(zone, 4)
    scale = tol * max(1.0, np.abs(xy).max())

    def keyset(en, z):
        q = _quant(en, scale).reshape(-1, 4)
        # orientation-free key: sort the two end points lexicographically
        a, b = q[:, :2], q[:, 2:]
        swap = (a[:, 0] > b[:, 0]) | ((a[:, 0] == b[:, 0]) & (a[:, 1] > b[:, 1]))
        lo = np.where(swap[:, None], b, a)
        hi = np.where(swap[:, None], a, b)
        return np.column_stack([z, lo, hi])

    nbr = np.full(E * 4, -1, np.int64)
    kind = np.full(E * 4, -1, np.int32)
    keys = keyset(ends, fzone)
    order = np.lexsort(keys.T[::-1])
    sk = keys[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    i = np.nonzero(same)[0]
    a, b = order[i], order[i + 1]
    if len(i) and np.any(np.diff(i) == 1):
        raise ValueError("a face is shared by more than two elements")
    nbr[a], nbr[b] = b, a
    kind[a] = FACE_INTERIOR
    kind[b] = FACE_INTERIOR

    free = np.nonzero(nbr < 0)[0]
    for T in (periodic or []):
        free = np.nonzero(nbr < 0)[0]
        ka = keyset(ends[free] + np.asarray(T)[None, None, :], fzone[free])
        kb = keyset(ends[free], fzone[free])
        ia, ib = _match(ka, kb)
        fa, fb = free[ia], free[ib]
        nbr[fa], nbr[fb] = fb, fa
        kind[fa] = FACE_PERIODIC
        kind[fb] = FACE_PERIODIC
    free = np.nonzero(nbr < 0)[0]
    if len(free):
        kind[free] = classify(ends[free], fzone[free])
    if np.any(kind < 0):
        raise ValueError("unclassified boundary face")
    nb = np.where(nbr >= 0, nbr // 4, -1)
    nf = np.where(nbr >= 0, nbr % 4, -1)
    mesh["nbr"] = nb.reshape(E, 4).astype(np.int32)
    mesh["nbr_face"] = nf.reshape(E, 4).astype(np.int32)
    mesh["face_kind"] = kind.reshape(E, 4)
    return mesh


def _on_circle(ends, c, r, tol=1e-9):
    d = np.hypot(ends[..., 0] - c[0], ends[..., 1] - c[1])
    return np.all(np.abs(d - r) <= tol * max(1.0, r), axis=-1)


# ----------------------------------------------------------------------------
# the vortex workload: periodic square with a rotating disk
# ----------------------------------------------------------------------------
def _square_perimeter(s):
    """Counter-clockwise perimeter points of the square with side coordinates
    s[0..n] (ascending), starting at the (s[-1], s[0]) corner: 4n points."""
    n = len(s) - 1
    hi, lo = s[-1], s[0]
    right = np.column_stack([np.full(n, hi), s[:-1]])
    top = np.column_stack([s[::-1][:-1], np.full(n, hi)])
    left = np.column_stack([np.full(n, lo), s[::-1][:-1]])
    bottom = np.column_stack([s[:-1], np.full(n, lo)])
    return np.concatenate([right, top, left, bottom])


def _circle_fn(c, r, phi0, dphi):
    def fn(j, t):
        a = phi0 + (np.asarray(j) + t) * dphi
        return np.column_stack([c[0] + r * np.cos(a), c[1] + r * np.sin(a)])
    return fn


def _wrap(P):
    """Append the first column to close an azimuthally periodic block."""
    return np.concatenate([P, P[:, :1]], axis=1)


def vortex_mesh(refine=1, core_half=0.8, radius=2.0, box_half=5.0):
    """Periodic square [-B,B]^2 with a rotating disk r < radius.

    The disk is an (8f x 8f) square core plus 6f blended rings of 32f cells;
    the stationary part is 4f blended rings of 32f cells from the circle to
    the box.  refine=1 gives 64 + 192 + 128 = 384 cells, K = 32 interface
    faces per side.  Cells with an edge on the circle are cubic.
    """
    f = int(refine)
    nc, nrr, nro = 8 * f, 6 * f, 4 * f
    K = 4 * nc
    c = np.zeros(2)
    s_core = np.linspace(-core_half, core_half, nc + 1)
    s_core[nc // 2] = 0.0
    gx, gy = np.meshgrid(s_core, s_core, indexing="ij")
    core = _block(np.stack([gx, gy], axis=-1), zone=1)

    S = _square_perimeter(s_core)
    dphi = 2 * np.pi / K
    phi = -np.pi / 4 + dphi * np.arange(K)
    C = np.column_stack([radius * np.cos(phi), radius * np.sin(phi)])
    t = np.arange(nrr + 1) / nrr
    Pr = (1 - t)[:, None, None] * S[None] + t[:, None, None] * C[None]
    Pr[0] = S
    Pr[-1] = C
    circ = _circle_fn(c, radius, -np.pi / 4, dphi)
    rot = _block(_wrap(Pr), curves={nrr: circ}, zone=1)

    s_box = np.linspace(-box_half, box_half, nc + 1)
    s_box[nc // 2] = 0.0
    B = _square_perimeter(s_box)
    t = np.arange(nro + 1) / nro
    Po = (1 - t)[:, None, None] * C[None] + t[:, None, None] * B[None]
    Po[0] = C
    Po[-1] = B
    out = _block(_wrap(Po), curves={0: circ}, zone=0)

    mesh = _concat([core, rot, out])
    mesh["center"] = c
    mesh["radius"] = float(radius)

    def classify(ends, z):
        return np.where(_on_circle(ends, c, radius), FACE_SLIDING, -1).astype(np.int32)

    L = 2 * box_half
    return connect(mesh, classify, periodic=[(L, 0.0), (0.0, L)])


# ----------------------------------------------------------------------------
# the Taylor-Couette workload: annulus, rotating inner half
# ----------------------------------------------------------------------------
def couette_mesh(nr=8, nt=32, r_in=1.0, r_out=2.0, r_s=1.5, phi_offset=0.0):
    """Annulus r_in < r < r_out cut at r_s; nr radial x nt azimuthal cells.

    The inner nr/2 layers rotate.  Node lines are circles; element edges are
    straight chords except on the two walls and the interface, whose
    adjacent cells are cubic.  The outer zone's azimuthal nodes are shifted
    by `phi_offset` radians.
    """
    if nr % 2:
        raise ValueError("nr must be even")
    c = np.zeros(2)
    dphi = 2 * np.pi / nt
    h = nr // 2

    def ring(r_lo, r_hi, nl, phi0, zone):
        r = r_lo + (r_hi - r_lo) * np.arange(nl + 1) / nl
        r[0], r[-1] = r_lo, r_hi
        phi = phi0 + dphi * np.arange(nt)
        P = np.stack([r[:, None] * np.cos(phi)[None], r[:, None] * np.sin(phi)[None]], axis=-1)
        curves = {0: _circle_fn(c, r_lo, phi0, dphi), nl: _circle_fn(c, r_hi, phi0, dphi)}
        return _block(_wrap(P), curves=curves, zone=zone)

    mesh = _concat([ring(r_in, r_s, h, 0.0, 1), ring(r_s, r_out, nr - h, phi_offset, 0)])
    mesh["center"] = c
    mesh["radius"] = float(r_s)

    def classify(ends, z):
        k = np.full(len(ends), -1, np.int32)
        k[_on_circle(ends, c, r_s)] = FACE_SLIDING
        k[_on_circle(ends, c, r_in) | _on_circle(ends, c, r_out)] = FACE_WALL_ISOTHERMAL
        return k

    return connect(mesh, classify)


# ----------------------------------------------------------------------------
# the rotating-ellipse workload: O-grids around an ellipse inside a box
# ----------------------------------------------------------------------------
def _geometric(n, first):
    """n+1 fractions from 0 to 1 whose spacings grow geometrically from
    `first` (as a fraction of the total)."""
    if first * n >= 1.0:
        return np.linspace(0.0, 1.0, n + 1)
    lo, hi = 1.0, 2.0
    while first * (hi ** n - 1) / (hi - 1) < 1.0:
        hi *= 2.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        if first * (q ** n - 1) / (q - 1) < 1.0:
            lo = q
        else:
            hi = q
    q = 0.5 * (lo + hi)
    x = np.concatenate([[0.0], np.cumsum(first * q ** np.arange(n))])
    x /= x[-1]
    x[-1] = 1.0
    return x


def ellipse_mesh(K=4096, n_in=64, n_out=180, semi=(0.5, 0.1), radius=3.0,
                 box_half=30.0, first_in=2e-3, first_out=4e-3, tile=(16, 4),
                 wall=FACE_WALL_SLIP, nested=False, K_out=None, warp=0.0):
    """Ellipse wall (slip, or `wall`) in a rotating disk r < radius inside a
    stationary box [-B,B]^2 with far-field sides.  K azimuthal cells, n_in
    rotating and n_out stationary layers (defaults: 4096 x (64 + 180) =
    999,424 cells), numbered in tiles of 16 azimuthal x 4 radial cells
    (tile=None: ring by ring).  nested=True returns (coarse, fine, children):
    the fine mesh splits every cell 2 x 2 in its reference square (2K
    faces per interface side) and children[c, a + 2 b] is the fine element
    of child (a, b) of coarse element c.

    K_out (default K) sets the number of stationary azimuthal cells, so the
    two sides of the sliding interface may have different face counts; warp
    (|warp| < 1) spaces the rotating side's K faces non-uniformly, at angles
    2 pi s + warp sin(2 pi s) for s = j / K."""
    K_out = K if K_out is None else K_out
    if K % 4 or K_out % 4:
        raise ValueError("K and K_out must be multiples of 4")
    if not abs(warp) < 1.0:
        raise ValueError("need |warp| < 1")
    c = np.zeros(2)
    a, b = semi

    def ang_in(s):
        s = np.asarray(s, dtype=float)
        return 2 * np.pi * s + warp * np.sin(2 * np.pi * s)

    tt = ang_in(np.arange(K) / K)
    Ell = np.column_stack([a * np.cos(tt), b * np.sin(tt)])
    Cin = np.column_stack([radius * np.cos(tt), radius * np.sin(tt)])
    f = _geometric(n_in, first_in)
    Pin = (1 - f)[:, None, None] * Ell[None] + f[:, None, None] * Cin[None]
    Pin[0], Pin[-1] = Ell, Cin

    def ell_fn(j, t):
        ang = ang_in((np.asarray(j) + t) / K)
        return np.column_stack([a * np.cos(ang), b * np.sin(ang)])

    def circ_in(j, t):
        ang = ang_in((np.asarray(j) + t) / K)
        return np.column_stack([c[0] + radius * np.cos(ang), c[1] + radius * np.sin(ang)])

    inner_P = _wrap(Pin)
    inner_curves = {0: ell_fn, n_in: circ_in}
    inner = _block(inner_P, curves=inner_curves, zone=1, tile=tile)

    dphi = 2 * np.pi / K_out
    phi = -np.pi / 4 + dphi * np.arange(K_out)
    Cout = np.column_stack([radius * np.cos(phi), radius * np.sin(phi)])
    s_box = np.linspace(-box_half, box_half, K_out // 4 + 1)
    Bx = _square_perimeter(s_box)
    g = _geometric(n_out, first_out)
    Pout = (1 - g)[:, None, None] * Cout[None] + g[:, None, None] * Bx[None]
    Pout[0], Pout[-1] = Cout, Bx
    outer_P = _wrap(Pout)
    outer_curves = {0: _circle_fn(c, radius, -np.pi / 4, dphi)}
    outer = _block(outer_P, curves=outer_curves, zone=0, tile=tile)
    tol = 1e-9 * box_half

    def classify(ends, z):
        k = np.full(len(ends), -1, np.int32)
        k[_on_circle(ends, c, radius)] = FACE_SLIDING
        on_box = np.all((np.abs(np.abs(ends[..., 0]) - box_half) <= tol)
                        | (np.abs(np.abs(ends[..., 1]) - box_half) <= tol), axis=-1)
        k[on_box] = FACE_FARFIELD
        r2 = (ends[..., 0] / a) ** 2 + (ends[..., 1] / b) ** 2
        k[np.all(np.abs(r2 - 1.0) < 1e-9, axis=-1)] = wall
        return k

    def finish(blocks):
        mesh = _concat(blocks)
        mesh["center"] = c
        mesh["radius"] = float(radius)
        return connect(mesh, classify)

    coarse = finish([inner, outer])
    if not nested:
        return coarse
    fine_blocks = []
    for P, cv, z in ((inner_P, inner_curves, 1), (outer_P, outer_curves, 0)):
        Pf, cf = _refine_block(P, cv)
        fine_blocks.append(_block(Pf, curves=cf, zone=z, tile=tile))
    fine = finish(fine_blocks)
    children = _children([(inner, K), (outer, K_out)], fine_blocks)
    return coarse, fine, children


# ----------------------------------------------------------------------------
# conforming periodic box (no interface), optionally distorted
# ----------------------------------------------------------------------------
def box_mesh(nx=6, ny=5, L=(2.0, 2.0), distort=0.0, curved=0.0, zone=0, seed=7):
    """Periodic box [0,Lx] x [0,Ly] of nx x ny cells.

    `distort` moves interior nodes by a smooth periodic field (fraction of a
    cell); `curved` bends every cell's edges by a smooth periodic field
    (fraction of a cell) and makes all cells cubic.
    """
    Lx, Ly = L
    x = np.linspace(0.0, Lx, nx + 1)
    y = np.linspace(0.0, Ly, ny + 1)
    gx, gy = np.meshgrid(x, y, indexing="ij")
    hx, hy = Lx / nx, Ly / ny

    def field(px, py):
        dx = np.sin(2 * np.pi * px / Lx) * np.sin(2 * np.pi * py / Ly)
        dy = np.sin(4 * np.pi * px / Lx + 1.0) * np.sin(2 * np.pi * py / Ly)
        return dx, dy

    dx, dy = field(gx, gy)
    P = np.stack([gx + distort * hx * dx, gy + distort * hy * dy], axis=-1)
    blk = _block(P, zone=zone)
    if curved:
        # bend every non-corner node by a smooth field that vanishes on the
        # box boundary lines, so periodic partners stay translates
        ref = blk["xy"]
        bx = np.sin(np.pi * ref[..., 0] / Lx * 2) * np.sin(np.pi * ref[..., 1] / Ly * 2)
        by = np.sin(np.pi * ref[..., 0] / Lx * 2 + 0.5) * np.sin(np.pi * ref[..., 1] / Ly * 2)
        mid = np.ones(12, bool)
        mid[[0, 3, 6, 9]] = False
        blk["xy"][:, mid, 0] += curved * hx * bx[:, mid]
        blk["xy"][:, mid, 1] += curved * hy * by[:, mid]
        blk["geom"][:] = GEOM_CUBIC
    blk["center"] = np.array([0.5 * Lx, 0.5 * Ly])
    blk["radius"] = 0.0

    def classify(ends, z):
        return np.full(len(ends), -1, np.int32)

    return connect(blk, classify, periodic=[(Lx, 0.0), (0.0, Ly)])


# ----------------------------------------------------------------------------
# mesh transforms used by invariance tests
# ----------------------------------------------------------------------------
def relabel(mesh, shifts):
    """Cyclically relabel each element's corners by shifts[e] in {0,1,2,3}
    quarter turns (the element and its map are unchanged; local face f of
    the new labelling is old face (f + shift) % 4).  Returns the new mesh;
    node order stays counter-clockwise."""
    shifts = np.asarray(shifts) % 4
    E = len(shifts)
    out = dict(mesh)
    xy = mesh["xy"]
    perm = np.array([(np.arange(12) + 3 * s) % 12 for s in range(4)])
    out["xy"] = xy[np.arange(E)[:, None], perm[shifts]]
    old_of_new = (np.arange(4)[None, :] + shifts[:, None]) % 4      # (E,4)
    new_of_old = (np.arange(4)[None, :] - shifts[:, None]) % 4
    nb = mesh["nbr"][np.arange(E)[:, None], old_of_new]
    nf_old = mesh["nbr_face"][np.arange(E)[:, None], old_of_new]
    nf = np.where(nb >= 0, new_of_old[np.maximum(nb, 0), np.maximum(nf_old, 0)], -1)
    out["nbr"] = nb.astype(np.int32)
    out["nbr_face"] = nf.astype(np.int32)
    out["face_kind"] = mesh["face_kind"][np.arange(E)[:, None], old_of_new]
    return out


def rotate_mesh(mesh, angle):
    """Rigidly rotate a whole mesh about its centre by `angle` radians."""
    out = dict(mesh)
    c = np.asarray(mesh["center"])
    ca, sa = np.cos(angle), np.sin(angle)
    d = mesh["xy"] - c
    out["xy"] = np.stack([c[0] + ca * d[..., 0] - sa * d[..., 1],
                          c[1] + sa * d[..., 0] + ca * d[..., 1]], axis=-1)
    return out
