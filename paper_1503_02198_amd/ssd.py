"""ctypes binding of libssd.so (include/ssd.h).

Argument marshalling only: every step of the residual and the time step
runs in the library's HIP kernels.  Device arrays are torch float32 CUDA
(HIP) tensors; streams are torch streams.  The binding fails loudly when
the library is not built; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssd.so")

SSD_OK = 0
STATUS = {0: "SSD_OK", -1: "SSD_ERR_INVALID_ARG", -2: "SSD_ERR_MESH", -3: "SSD_ERR_STATE",
          -4: "SSD_ERR_DEVICE", -5: "SSD_ERR_NOMEM", -6: "SSD_ERR_NUMERIC"}
KERNELS = {"stage": 0, "traces": 1, "mortar": 2, "rebuild": 3, "grad": 4}
SCHEMES = {"rk3": 0, "rk54": 1}   # ssd_rk
EXPORTS = ["ssd_create_mesh", "ssd_destroy_mesh", "ssd_query", "ssd_set_rotation",
           "ssd_mortar_rebuild", "ssd_residual", "ssd_rk_step", "ssd_rk_steps",
           "ssd_rk_steps_noalloc", "ssd_check",
           "ssd_last_error", "ssd_timing_enable", "ssd_timing_reset", "ssd_timing_read",
           "ssd_timing_samples", "ssd_probe_contraction", "ssd_probe_stream",
           "ssd_batch_create", "ssd_batch_destroy", "ssd_batch_rk_steps", "ssd_batch_query",
           "ssd_mlp_create", "ssd_mlp_destroy", "ssd_mlp_dims", "ssd_mlp_set_params",
           "ssd_mlp_get_params", "ssd_mlp_set_normalization", "ssd_mlp_fit_normalization",
           "ssd_mlp_forward", "ssd_mlp_gradient", "ssd_mlp_train_step", "ssd_mlp_loss",
           "ssd_subgrid_features", "ssd_restrict", "ssd_subgrid_targets", "ssd_subgrid_nudge",
           "ssd_subgrid_attach"]


# -- cell-blocked state layout (include/ssd.h) ------------------------------
# Elements in blocks of CB consecutive elements (the last holds the
# remainder); block b stores plane after plane, each plane a row of its
# elements.  These two helpers only reorder values (numpy arrays or torch
# tensors, on any device); no step of the method is computed here.
CB = 64


def _swap01(a, shape):
    a = a.reshape(shape)
    return a.transpose(1, 0, 2) if isinstance(a, np.ndarray) else a.permute(1, 0, 2)


def _cat(parts, axis):
    if isinstance(parts[0], np.ndarray):
        return np.concatenate(parts, axis=axis)
    import torch
    return torch.cat(parts, dim=axis)


def pack_state(Q):
    """Flat cell-blocked array of Q [..., n_elem] (the leading axes are the
    planes: [4, N, N, n_elem] for a state)."""
    if Q.ndim < 2:
        raise ValueError("pack_state needs planes x elements (e.g. [4, N, N, n_elem])")
    E = Q.shape[-1]
    P = int(np.prod(Q.shape[:-1]))
    Q2 = Q.reshape(P, E)
    nb = E // CB
    head = _swap01(Q2[:, :nb * CB], (P, nb, CB)).reshape(-1)
    tail = Q2[:, nb * CB:].reshape(-1)
    return _cat([head, tail], 0)


def unpack_state(q, N, n_elem, nvar=4):
    """[nvar, N, N, n_elem] view of a flat cell-blocked array."""
    E, P = n_elem, nvar * N * N
    if q.ndim != 1 or q.shape[0] != P * E:
        raise ValueError(f"expected a flat array of {P * E} values, got shape {tuple(q.shape)}")
    nb = E // CB
    head = _swap01(q[:P * nb * CB], (nb, P, CB)).reshape(P, nb * CB)
    tail = q[P * nb * CB:P * E].reshape(P, E - nb * CB)
    return _cat([head, tail], 1).reshape(nvar, N, N, E)


class SSDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n_elem", ctypes.c_int32),
                ("elem_xy", ctypes.POINTER(ctypes.c_double)),
                ("elem_geom", ctypes.POINTER(ctypes.c_int32)),
                ("elem_zone", ctypes.POINTER(ctypes.c_int32)),
                ("nbr_elem", ctypes.POINTER(ctypes.c_int32)),
                ("nbr_face", ctypes.POINTER(ctypes.c_int32)),
                ("face_kind", ctypes.POINTER(ctypes.c_int32)),
                ("rot_center", ctypes.c_double * 2), ("iface_radius", ctypes.c_double),
                ("omega", ctypes.c_double), ("theta0", ctypes.c_double),
                ("gamma", ctypes.c_double), ("gas_R", ctypes.c_double), ("mu", ctypes.c_double),
                ("prandtl", ctypes.c_double), ("T_wall", ctypes.c_double),
                ("farfield", ctypes.c_double * 4)]


class BatchGroup(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("N", ctypes.c_int32), ("viscous", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("stream", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("tuned", ctypes.c_int32), ("stage_us", ctypes.c_float),
                ("tiles_per_block", ctypes.c_int32), ("stage_us_tpb", ctypes.c_float * 2)]


class Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n_elem", ctypes.c_int32), ("K", ctypes.c_int32),
                ("n_cubic", ctypes.c_int32), ("viscous", ctypes.c_int32),
                ("device", ctypes.c_int32), ("state_len", ctypes.c_int64),
                ("work_len", ctypes.c_int64)]


_lib = None


def lib():
    """Load libssd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1503_02198_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "ssd_create_mesh": (i32, [ctypes.POINTER(MeshDesc), ctypes.c_int, ctypes.POINTER(vp)]),
            "ssd_destroy_mesh": (i32, [vp]),
            "ssd_query": (i32, [vp, ctypes.POINTER(Info)]),
            "ssd_set_rotation": (i32, [vp, dbl, dbl]),
            "ssd_mortar_rebuild": (i32, [vp, vp]),
            "ssd_residual": (i32, [vp, vp, vp, vp]),
            "ssd_rk_step": (i32, [vp, vp, vp, dbl, dbl, ctypes.c_int, vp]),
            "ssd_rk_steps": (i32, [vp, vp, vp, dbl, dbl, i32, ctypes.c_int, vp]),
            "ssd_rk_steps_noalloc": (i32, [vp, vp, dbl, dbl, i32, ctypes.c_int, vp]),
            "ssd_check": (i32, [vp, vp]),
            "ssd_last_error": (ctypes.c_char_p, []),
            "ssd_timing_enable": (i32, [vp, ctypes.c_int]),
            "ssd_timing_reset": (i32, [vp]),
            "ssd_timing_read": (i32, [vp, ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
            "ssd_timing_samples": (i32, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_float), i64,
                                         ctypes.POINTER(i64)]),
            "ssd_probe_contraction": (i32, [vp, i32, i32, i32, vp, vp, vp]),
            "ssd_probe_stream": (i32, [vp, i32, i64, vp, vp, vp, vp]),
            "ssd_batch_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]),
            "ssd_batch_destroy": (i32, [vp]),
            "ssd_batch_rk_steps": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(dbl), ctypes.POINTER(dbl), i32,
                                         ctypes.c_int, i32, vp]),
            "ssd_batch_query": (i32, [vp, i32, ctypes.POINTER(BatchGroup)]),
            "ssd_mlp_create": (i32, [i32, i32, ctypes.POINTER(vp)]),
            "ssd_mlp_destroy": (i32, [vp]),
            "ssd_mlp_dims": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "ssd_mlp_set_params": (i32, [vp] + [ctypes.POINTER(ctypes.c_float)] * 6),
            "ssd_mlp_get_params": (i32, [vp] + [ctypes.POINTER(ctypes.c_float)] * 6),
            "ssd_mlp_set_normalization": (i32, [vp] + [ctypes.POINTER(ctypes.c_float)] * 4),
            "ssd_mlp_fit_normalization": (i32, [vp, vp, vp, i64, ctypes.c_float, vp]),
            "ssd_mlp_forward": (i32, [vp, vp, i64, vp, vp]),
            "ssd_mlp_gradient": (i32, [vp, vp, vp, i64, vp, i32, ctypes.c_float, ctypes.c_uint64]
                                 + [ctypes.POINTER(ctypes.c_float)] * 6
                                 + [ctypes.POINTER(dbl), vp]),
            "ssd_mlp_train_step": (i32, [vp, vp, vp, i64, vp, i32, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_uint64, vp]),
            "ssd_mlp_loss": (i32, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
            "ssd_subgrid_features": (i32, [vp, vp, vp, vp]),
            "ssd_restrict": (i32, [vp, vp, vp, vp, vp, vp]),
            "ssd_subgrid_targets": (i32, [vp, vp, vp, vp, vp, vp, vp]),
            "ssd_subgrid_nudge": (i32, [vp, vp, vp, ctypes.c_float, vp, vp]),
            "ssd_subgrid_attach": (i32, [vp, vp, ctypes.c_float, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != SSD_OK:
        raise SSDError(status, lib().ssd_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_desc(mesh, case, N):
    """Fill an ssd_mesh_desc from a mesh dict and a case dict.  Returns the
    descriptor and the numpy arrays it points into (keep them alive)."""
    keep = dict(
        xy=np.ascontiguousarray(mesh["xy"], dtype=np.float64),
        geom=np.ascontiguousarray(mesh["geom"], dtype=np.int32),
        zone=np.ascontiguousarray(mesh["zone"], dtype=np.int32),
        nbr=np.ascontiguousarray(mesh["nbr"], dtype=np.int32),
        nf=np.ascontiguousarray(mesh["nbr_face"], dtype=np.int32),
        kind=np.ascontiguousarray(mesh["face_kind"], dtype=np.int32))
    d = MeshDesc()
    d.N = int(N)
    d.n_elem = int(keep["zone"].shape[0])
    d.elem_xy = _ptr(keep["xy"], ctypes.c_double)
    d.elem_geom = _ptr(keep["geom"], ctypes.c_int32)
    d.elem_zone = _ptr(keep["zone"], ctypes.c_int32)
    d.nbr_elem = _ptr(keep["nbr"], ctypes.c_int32)
    d.nbr_face = _ptr(keep["nf"], ctypes.c_int32)
    d.face_kind = _ptr(keep["kind"], ctypes.c_int32)
    c = mesh.get("center", (0.0, 0.0))
    d.rot_center[0], d.rot_center[1] = float(c[0]), float(c[1])
    d.iface_radius = float(mesh.get("radius", 0.0))
    d.omega = float(case["omega"])
    d.theta0 = float(case.get("theta0", 0.0))
    d.gamma = float(case["gamma"])
    d.gas_R = float(case["gas_R"])
    d.mu = float(case["mu"])
    d.prandtl = float(case["prandtl"])
    d.T_wall = float(case["T_wall"])
    for i, v in enumerate(case["farfield"]):
        d.farfield[i] = float(v)
    return d, keep


def _stream_ptr(stream, device):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(int(s.cuda_stream))


class Mesh:
    """One SSD mesh on one GPU (a handle of the C library)."""

    def __init__(self, mesh, case, N, device=0):
        d, keep = make_desc(mesh, case, N)
        h = ctypes.c_void_p()
        _check(lib().ssd_create_mesh(ctypes.byref(d), int(device), ctypes.byref(h)))
        del keep
        self._h = h
        self.device = int(device)
        self.info = self.query()

    def query(self):
        inf = Info()
        _check(lib().ssd_query(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ssd_destroy_mesh(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _tensor(self, t, n, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be contiguous float32 with {n} elements")
        if t.device.index != self.device:
            raise ValueError(f"{name} lives on device {t.device.index}, mesh on {self.device}")
        return ctypes.c_void_p(t.data_ptr())

    def set_rotation(self, theta, omega):
        _check(lib().ssd_set_rotation(self._h, float(theta), float(omega)))

    def mortar_rebuild(self, stream=None):
        _check(lib().ssd_mortar_rebuild(self._h, _stream_ptr(stream, self.device)))

    def residual(self, q, r, stream=None):
        n = self.info["state_len"]
        _check(lib().ssd_residual(self._h, self._tensor(q, n, "q"), self._tensor(r, n, "r"),
                                  _stream_ptr(stream, self.device)))

    def rk_step(self, q, work, t, dt, stream=None, scheme="rk3"):
        n = self.info["state_len"]
        _check(lib().ssd_rk_step(self._h, self._tensor(q, n, "q"),
                                 self._tensor(work, self.info["work_len"], "work"),
                                 float(t), float(dt), SCHEMES[scheme],
                                 _stream_ptr(stream, self.device)))

    def rk_steps(self, q, work, t, dt, nsteps, stream=None, scheme="rk3"):
        n = self.info["state_len"]
        _check(lib().ssd_rk_steps(self._h, self._tensor(q, n, "q"),
                                  self._tensor(work, self.info["work_len"], "work"),
                                  float(t), float(dt), int(nsteps), SCHEMES[scheme],
                                  _stream_ptr(stream, self.device)))

    def rk_steps_noalloc(self, q, t, dt, nsteps, stream=None, scheme="rk3"):
        """rk_steps with the library's fixed per-GPU work array instead of a
        caller's work tensor (ssd_rk_steps_noalloc)."""
        _check(lib().ssd_rk_steps_noalloc(self._h, self._tensor(q, self.info["state_len"], "q"),
                                          float(t), float(dt), int(nsteps), SCHEMES[scheme],
                                          _stream_ptr(stream, self.device)))

    def probe_contraction(self, variant, n_cells, reps, q, out, stream=None):
        """The VALU (0) or MFMA (1) contraction probe (ssd_probe_contraction)."""
        n = 64 * n_cells
        _check(lib().ssd_probe_contraction(self._h, int(variant), int(n_cells), int(reps),
                                           self._tensor(q, n, "q"), self._tensor(out, n, "out"),
                                           _stream_ptr(stream, self.device)))

    def probe_stream(self, variant, n, a, b, c, stream=None):
        """The stream probe c = 0.75 a + 0.25 b over n floats (ssd_probe_stream)."""
        _check(lib().ssd_probe_stream(self._h, int(variant), int(n), self._tensor(a, n, "a"),
                                      self._tensor(b, n, "b"), self._tensor(c, n, "c"),
                                      _stream_ptr(stream, self.device)))

    def check(self, stream=None):
        _check(lib().ssd_check(self._h, _stream_ptr(stream, self.device)))

    def features(self, q, X, stream=None):
        """Rows X [E][4N^2 + 16N] of the learned correction's features of q."""
        n_in = 4 * self.info["N"] ** 2 + 16 * self.info["N"]
        _check(lib().ssd_subgrid_features(self._h, self._tensor(q, self.info["state_len"], "q"),
                                          self._tensor(X, self.info["n_elem"] * n_in, "X"),
                                          _stream_ptr(stream, self.device)))

    def attach(self, net, weight=1.0, per_step=False):
        """Add weight x the learned correction of `net` to dQ/dt in every
        SSP-RK3 stage, evaluated per stage or (per_step) once per step at the
        step's start (None: plain SSD).  The network must outlive the
        attachment."""
        _check(lib().ssd_subgrid_attach(self._h, net._h if net is not None else None,
                                        float(weight), int(bool(per_step))))
        self._net = net

    def timing_enable(self, on=True, kernels=None):
        """Bracket launches with HIP events: every kernel class, or only
        `kernels` (names from KERNELS), or none (on=False)."""
        if not on:
            mask = 0
        elif kernels is None:
            mask = (1 << len(KERNELS)) - 1
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << KERNELS[k]
        _check(lib().ssd_timing_enable(self._h, mask))

    def timing_reset(self):
        _check(lib().ssd_timing_reset(self._h))

    def timing_read(self, kernel):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().ssd_timing_read(self._h, KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def timing_samples(self, kernel):
        """Durations (ms) of the timed launches of one kernel class since
        the last reset, in launch order."""
        n = ctypes.c_int64()
        _check(lib().ssd_timing_samples(self._h, KERNELS[kernel], None, 0, ctypes.byref(n)))
        buf = (ctypes.c_float * max(1, n.value))()
        _check(lib().ssd_timing_samples(self._h, KERNELS[kernel], buf, n.value, ctypes.byref(n)))
        return np.frombuffer(buf, dtype=np.float32, count=n.value).astype(np.float64)


class Batch:
    """Several meshes of one GPU stepped together (ssd_batch_*).  The meshes
    must outlive the batch."""

    def __init__(self, meshes):
        self.meshes = list(meshes)
        n = len(self.meshes)
        arr = (ctypes.c_void_p * n)(*[m._h.value for m in self.meshes])
        h = ctypes.c_void_p()
        _check(lib().ssd_batch_create(arr, n, ctypes.byref(h)))
        self._h = h
        self.device = self.meshes[0].device

    def rk_steps(self, qs, works, ts, dts, nsteps, scheme="rk3", graph=True, stream=None):
        n = len(self.meshes)
        if not (len(qs) == len(works) == len(ts) == len(dts) == n):
            raise ValueError("one state, work array, t and dt per mesh")
        q = (ctypes.c_void_p * n)(*[m._tensor(x, m.info["state_len"], "q").value
                                    for m, x in zip(self.meshes, qs)])
        w = (ctypes.c_void_p * n)(*[m._tensor(x, m.info["work_len"], "work").value
                                    for m, x in zip(self.meshes, works)])
        t = (ctypes.c_double * n)(*[float(x) for x in ts])
        d = (ctypes.c_double * n)(*[float(x) for x in dts])
        _check(lib().ssd_batch_rk_steps(self._h, q, w, t, d, int(nsteps), SCHEMES[scheme],
                                        int(bool(graph)), _stream_ptr(stream, self.device)))

    def groups(self):
        out, g = [], 0
        while True:
            inf = BatchGroup()
            _check(lib().ssd_batch_query(self._h, g, ctypes.byref(inf)))
            out.append({f: (list(getattr(inf, f)) if f == "stage_us_tpb" else getattr(inf, f))
                        for f, _ in BatchGroup._fields_ if f != "n_groups"})
            g += 1
            if g >= inf.n_groups:
                return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ssd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f32(a, n, name):
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.size != n:
        raise ValueError(f"{name} must hold {n} values")
    return a


def _dev(t, n, name, dtype="float32", device=None):
    import torch
    want = getattr(torch, dtype)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != want or not t.is_contiguous() or (n is not None and t.numel() != n):
        raise ValueError(f"{name} must be contiguous {dtype}"
                         + (f" with {n} elements" if n is not None else ""))
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} lives on device {t.device.index}, expected {device}")
    return ctypes.c_void_p(t.data_ptr())


class MLP:
    """Network of the learned per-element correction (a handle of the C
    library): n_in = 4N^2 + 16N features, two tanh layers of HIDDEN, n_out =
    4N^2 outputs, BF16 matrix products with FP32 accumulation."""

    HIDDEN = 64

    def __init__(self, N, device=0):
        h = ctypes.c_void_p()
        _check(lib().ssd_mlp_create(int(N), int(device), ctypes.byref(h)))
        self._h = h
        self.N = int(N)
        self.device = int(device)
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ssd_mlp_dims(self._h, ctypes.byref(a), ctypes.byref(b)))
        self.n_in, self.n_out = a.value, b.value

    def shapes(self):
        H = self.HIDDEN
        return dict(W1=(H, self.n_in), b1=(H,), W2=(H, H), b2=(H,), W3=(self.n_out, H),
                    b3=(self.n_out,))

    def set_params(self, p):
        arrs = [_f32(p[k], int(np.prod(sh)), k) for k, sh in self.shapes().items()]
        _check(lib().ssd_mlp_set_params(self._h, *[_ptr(a, ctypes.c_float) for a in arrs]))

    def get_params(self):
        out = {k: np.empty(sh, np.float32) for k, sh in self.shapes().items()}
        _check(lib().ssd_mlp_get_params(self._h, *[_ptr(out[k], ctypes.c_float) for k in out]))
        return out

    def set_normalization(self, mu_x, sig_x, mu_y, sig_y):
        a = [_f32(mu_x, self.n_in, "mu_x"), _f32(sig_x, self.n_in, "sig_x"),
             _f32(mu_y, self.n_out, "mu_y"), _f32(sig_y, self.n_out, "sig_y")]
        _check(lib().ssd_mlp_set_normalization(self._h, *[_ptr(x, ctypes.c_float) for x in a]))

    def fit_normalization(self, X, T, min_rel=0.0, stream=None):
        n = X.numel() // self.n_in
        _check(lib().ssd_mlp_fit_normalization(
            self._h, _dev(X, n * self.n_in, "X", device=self.device),
            _dev(T, n * self.n_out, "T", device=self.device), int(n), float(min_rel),
            _stream_ptr(stream, self.device)))

    def forward(self, X, Y, stream=None):
        n = X.numel() // self.n_in
        _check(lib().ssd_mlp_forward(self._h, _dev(X, n * self.n_in, "X", device=self.device),
                                     int(n), _dev(Y, n * self.n_out, "Y", device=self.device),
                                     _stream_ptr(stream, self.device)))

    def gradient(self, X, T, idx, noise=0.0, seed=0, stream=None):
        """Loss and its gradient (host arrays) on the rows idx of X, T."""
        n = X.numel() // self.n_in
        out = {k: np.empty(sh, np.float32) for k, sh in self.shapes().items()}
        loss = ctypes.c_double()
        _check(lib().ssd_mlp_gradient(
            self._h, _dev(X, n * self.n_in, "X", device=self.device),
            _dev(T, n * self.n_out, "T", device=self.device), int(n),
            _dev(idx, None, "idx", "int32", self.device), int(idx.numel()), float(noise),
            int(seed), *[_ptr(out[k], ctypes.c_float) for k in out], ctypes.byref(loss),
            _stream_ptr(stream, self.device)))
        return loss.value, out

    def train_step(self, X, T, idx, lr, noise=0.0, seed=0, stream=None):
        n = X.numel() // self.n_in
        _check(lib().ssd_mlp_train_step(
            self._h, _dev(X, n * self.n_in, "X", device=self.device),
            _dev(T, n * self.n_out, "T", device=self.device), int(n),
            _dev(idx, None, "idx", "int32", self.device), int(idx.numel()), float(lr),
            float(noise), int(seed), _stream_ptr(stream, self.device)))

    def loss(self):
        """Mean loss of the steps since the last call, and their count."""
        s, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().ssd_mlp_loss(self._h, ctypes.byref(s), ctypes.byref(n)))
        return (s.value / n.value if n.value else float("nan")), n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ssd_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def restrict(fine, coarse, children, qf, qc, stream=None):
    """qc = restriction of the fine state qf to the coarse parent mesh
    (children None: the same mesh at the lower order of `coarse`)."""
    _check(lib().ssd_restrict(fine._h, coarse._h,
                              None if children is None else
                              _dev(children, 4 * coarse.info["n_elem"], "children", "int32",
                                   coarse.device),
                              fine._tensor(qf, fine.info["state_len"], "qf"),
                              coarse._tensor(qc, coarse.info["state_len"], "qc"),
                              _stream_ptr(stream, coarse.device)))


def subgrid_targets(fine, coarse, children, Rf, Rc, T, stream=None):
    """T rows = restriction of the fine dQ/dt Rf minus the coarse Rc."""
    _check(lib().ssd_subgrid_targets(fine._h, coarse._h,
                                     _dev(children, 4 * coarse.info["n_elem"], "children",
                                          "int32", coarse.device),
                                     fine._tensor(Rf, fine.info["state_len"], "Rf"),
                                     coarse._tensor(Rc, coarse.info["state_len"], "Rc"),
                                     coarse._tensor(T, coarse.info["state_len"], "T"),
                                     _stream_ptr(stream, coarse.device)))


def subgrid_nudge(coarse, q_ref, q, rate, T, stream=None):
    """T rows += rate (q_ref - q), both states of the coarse mesh
    (ssd_subgrid_nudge)."""
    n = coarse.info["state_len"]
    _check(lib().ssd_subgrid_nudge(coarse._h, coarse._tensor(q_ref, n, "q_ref"),
                                   coarse._tensor(q, n, "q"), float(rate),
                                   coarse._tensor(T, n, "T"), _stream_ptr(stream, coarse.device)))
