"""ctypes marshalling for libfsib.so (argument checks and pointer passing only)."""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libfsib.so"
DIAG_COUNT = 11

FSIB_F64, FSIB_F32 = 0, 1
FSIB_STOKES, FSIB_NAVIER_STOKES = 0, 1
FSIB_FORCE_CURVE_TENSION, FSIB_FORCE_SURFACE_TENSION, FSIB_FORCE_EDGE_SPRINGS, FSIB_FORCE_TARGET = 0, 1, 2, 3


class FSIBError(RuntimeError):
    def __init__(self, status, name, message):
        super().__init__(f"{name}: {message} (status {status})")
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_modes", ctypes.c_int64 * 3), ("L", ctypes.c_double),
                ("prec", ctypes.c_int), ("tol", ctypes.c_double), ("upsampfac", ctypes.c_double),
                ("ntrans", ctypes.c_int), ("max_points", ctypes.c_int64), ("fluid", ctypes.c_int),
                ("navier_stokes", ctypes.c_int), ("ninst", ctypes.c_int), ("deterministic", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int), ("beta", ctypes.c_double), ("degree", ctypes.c_int),
                ("n_fine", ctypes.c_int64 * 3), ("n_dealias", ctypes.c_int64 * 3), ("tile", ctypes.c_int64 * 3),
                ("workspace_bytes", ctypes.c_int64)]


class _Params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("rho", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
                ("body", ctypes.c_double * 3)]


class _Tuning(ctypes.Structure):
    _fields_ = [("xcd_chunk_interp", ctypes.c_int), ("xcd_chunk_spread", ctypes.c_int), ("split", ctypes.c_int),
                ("overlap", ctypes.c_int), ("interp_points", ctypes.c_int), ("spread_threads", ctypes.c_int),
                ("nl_stages", ctypes.c_int)]


class _Force(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("K", ctypes.c_double), ("tris", ctypes.c_void_p), ("ntris", ctypes.c_int64),
                ("v2t_ptr", ctypes.c_void_p), ("v2t_idx", ctypes.c_void_p), ("aux", ctypes.c_void_p)]


_SIGS = {
    "fsib_version": (ctypes.c_char_p, []),
    "fsib_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fsib_last_error": (ctypes.c_char_p, []),
    "fsib_device_count": (ctypes.c_int, []),
    "fsib_plan_create": (ctypes.c_int, [ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_void_p)]),
    "fsib_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fsib_plan_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning), ctypes.c_int]),
    "fsib_plan_set_instances": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "fsib_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Info)]),
    "fsib_plan_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_plan_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "fsib_plan_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "fsib_spread": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_double, ctypes.c_void_p]),
    "fsib_spread_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "fsib_interp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "fsib_spectral_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_grad_combine": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "fsib_force_spread": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "fsib_velocity_interp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_fluid_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_compute_force": (ctypes.c_int, [ctypes.POINTER(_Force), ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_force_jvp": (ctypes.c_int, [ctypes.POINTER(_Force), ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_spring_stiffness": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_pressure": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_velocity": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_Force), ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_Force), ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fsib_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_Force), ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "fsib_group_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "fsib_group_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fsib_group_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_Force),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.c_void_p]),
}

_lib = None


def library_path():
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load libfsib.so (built in-tree by paper_2302_08694_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run `python -m paper_2302_08694_amd.build` "
                              "(the FSIB path has no CPU fallback)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status, name):
    if status != 0:
        lib = load_library()
        raise FSIBError(status, name, lib.fsib_last_error().decode())


def version():
    return load_library().fsib_version().decode()


def device_count():
    return int(load_library().fsib_device_count())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor (the FSIB path runs on the GPU only)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class FluidParams:
    def __init__(self, model="navier_stokes", rho=1.0, mu=1.0, dt=1e-3, body=(0.0, 0.0, 0.0)):
        m = {"stokes": FSIB_STOKES, "navier_stokes": FSIB_NAVIER_STOKES}[model]
        b = tuple(float(x) for x in body) + (0.0,) * (3 - len(body))
        self._s = _Params(m, float(rho), float(mu), float(dt), (ctypes.c_double * 3)(*b[:3]))
        self.model, self.rho, self.mu, self.dt, self.body = model, rho, mu, dt, b[:3]


class Force:
    """Built-in force law.

    kind "tension2d" (closed curve), "surface3d" (triangulated surface: tris (T,3) and the
    vertex->triangle CSR (ptr, idx)), "springs" (edge springs: the vertex->neighbour CSR as (ptr, idx)
    and the stiffness of every CSR entry as `aux`, double; tris optional, used by the volume
    diagnostic) or "target" (target points: `aux` = targets, double (M, dim)).  Index arrays are int32
    device tensors.
    """

    KINDS = {"tension2d": FSIB_FORCE_CURVE_TENSION, "surface3d": FSIB_FORCE_SURFACE_TENSION,
             "springs": FSIB_FORCE_EDGE_SPRINGS, "target": FSIB_FORCE_TARGET}

    def __init__(self, kind, K, tris=None, v2t_ptr=None, v2t_idx=None, aux=None):
        k = self.KINDS[kind]
        self.kind = kind
        self._keep = (tris, v2t_ptr, v2t_idx, aux)
        ntris = 0
        if kind == "surface3d":
            _need(tris, "tris", torch.int32)
        if kind in ("surface3d", "springs"):
            _need(v2t_ptr, "v2t_ptr", torch.int32)
            _need(v2t_idx, "v2t_idx", torch.int32)
        if kind in ("springs", "target"):
            _need(aux, "aux", torch.float64)
        if tris is not None:
            _need(tris, "tris", torch.int32)
            ntris = tris.shape[0]
        p = lambda t: _ptr(t).value if t is not None else None
        self._s = _Force(k, float(K), p(tris), ntris, p(v2t_ptr), p(v2t_idx), p(aux))


def spring_stiffness(X0, tris, v2t_ptr, v2t_idx, nbr_ptr, nbr_idx):
    """Edge-spring stiffness per neighbour-CSR entry (sigma = 1) of the reference mesh X0 (device)."""
    lib = load_library()
    _need(X0, "X0", torch.float64)
    for t, n in ((tris, "tris"), (v2t_ptr, "v2t_ptr"), (v2t_idx, "v2t_idx"), (nbr_ptr, "nbr_ptr"), (nbr_idx, "nbr_idx")):
        _need(t, n, torch.int32)
    kij = torch.empty(nbr_idx.shape[0], dtype=torch.float64, device=X0.device)
    _check(lib.fsib_spring_stiffness(X0.shape[0], _ptr(X0), _ptr(tris), _ptr(v2t_ptr), _ptr(v2t_idx), _ptr(nbr_ptr),
                                     _ptr(nbr_idx), _ptr(kij)), "fsib_spring_stiffness")
    return kij


def compute_force(force, X):
    """Nodal force F(X) (double, same shape as X) of a built-in force law."""
    lib = load_library()
    dim = X.shape[1]
    _need(X, "X", torch.float64)
    F = torch.empty_like(X)
    _check(lib.fsib_compute_force(ctypes.byref(force._s), dim, X.shape[0], _ptr(X), _ptr(F), _stream()),
           "fsib_compute_force")
    return F


def force_jvp(force, X, V):
    """dF(X)[V] (double, same shape as X) of a built-in force law; also dF(X)^T V (symmetric)."""
    lib = load_library()
    dim = X.shape[1]
    _need(X, "X", torch.float64)
    _need(V, "V", torch.float64, X.shape)
    out = torch.empty_like(X)
    _check(lib.fsib_force_jvp(ctypes.byref(force._s), dim, X.shape[0], _ptr(X), _ptr(V), _ptr(out), _stream()),
           "fsib_force_jvp")
    return out


class Plan:
    def __init__(self, dim, n_modes, L=1.0, prec="f64", tol=1e-6, ntrans=1, max_points=1 << 16, fluid=False,
                 navier_stokes=False, upsampfac=0.0, ninst=1, deterministic=False):
        lib = load_library()
        nm = list(n_modes) + [1] * (3 - len(n_modes))
        self.dim = int(dim)
        self.n_modes = tuple(int(n) for n in n_modes[:dim])
        self.L = float(L)
        self.prec = prec
        self.rdtype = {"f64": torch.float64, "f32": torch.float32}[prec]
        self.cdtype = {"f64": torch.complex128, "f32": torch.complex64}[prec]
        self.ntrans = int(ntrans)
        self.max_points = int(max_points)
        opts = _Opts(self.dim, (ctypes.c_int64 * 3)(*nm), self.L, FSIB_F64 if prec == "f64" else FSIB_F32,
                     float(tol), float(upsampfac), self.ntrans, self.max_points, int(bool(fluid)),
                     int(bool(navier_stokes)), int(ninst), int(bool(deterministic)))
        self.ninst = max(1, int(ninst))
        h = ctypes.c_void_p()
        _check(lib.fsib_plan_create(ctypes.byref(opts), ctypes.byref(h)), "fsib_plan_create")
        self._h = h
        self._lib = lib

    @property
    def field_shape(self):
        """Shape of the half spectra of the plan's real fields: (dim, ...) or (ninst, dim, ...)."""
        return ((self.dim,) if self.ninst == 1 else (self.ninst, self.dim)) + self.half_shape

    def tuning(self, **changes):
        """Launch-shape knobs (fsib_plan_tuning): with no arguments returns them as a dict; keyword
        arguments (xcd_chunk_interp, xcd_chunk_spread, split, overlap, interp_points, spread_threads,
        nl_stages) set them and return the new dict."""
        t = _Tuning()
        _check(self._lib.fsib_plan_tuning(self._h, ctypes.byref(t), 1), "fsib_plan_tuning")
        if changes:
            names = {k for k, _ in _Tuning._fields_}
            for k, v in changes.items():
                if k not in names:
                    raise ValueError(f"unknown tuning knob {k!r}")
                setattr(t, k, int(v))
            _check(self._lib.fsib_plan_tuning(self._h, ctypes.byref(t), 0), "fsib_plan_tuning")
        return {k: getattr(t, k) for k, _ in _Tuning._fields_}

    def set_instances(self, counts):
        """Point counts of the instances of a multi-instance plan (fsib_plan_set_instances); points are
        then passed instance after instance."""
        counts = [int(c) for c in counts]
        if len(counts) != self.ninst:
            raise ValueError(f"need {self.ninst} counts, got {len(counts)}")
        off = (ctypes.c_int64 * (self.ninst + 1))()
        for i, c in enumerate(counts):
            off[i + 1] = off[i] + c
        _check(self._lib.fsib_plan_set_instances(self._h, off), "fsib_plan_set_instances")
        self.instance_offsets = list(off)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fsib_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes
    @property
    def spectral_shape(self):
        return tuple(reversed(self.n_modes))

    @property
    def half_shape(self):
        s = list(reversed(self.n_modes))
        s[-1] = self.n_modes[0] // 2 + 1
        return tuple(s)

    def info(self):
        inf = _Info()
        _check(self._lib.fsib_plan_info(self._h, ctypes.byref(inf)), "fsib_plan_info")
        return dict(w=inf.w, beta=inf.beta, degree=inf.degree, n_fine=tuple(inf.n_fine)[: self.dim],
                    n_dealias=tuple(inf.n_dealias)[: self.dim], tile=tuple(inf.tile)[: self.dim],
                    workspace_bytes=inf.workspace_bytes)

    def check(self):
        _check(self._lib.fsib_plan_check(self._h, _stream()), "fsib_plan_check")

    PROF_CLASSES = {"fft_strided": 1, "spread": 2, "interp": 3, "fft_x": 4, "nl_x": 5}

    def profile(self, kernel_class, max_launches=4096):
        """Time every launch of one kernel class with HIP events (None disables)."""
        cls = -1 if kernel_class is None else self.PROF_CLASSES[kernel_class]
        _check(self._lib.fsib_plan_profile(self._h, cls, int(max_launches)), "fsib_plan_profile")

    def profile_read(self):
        """(total_ms, launches, algorithmic_bytes) of the launches recorded since the last read."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(self._lib.fsib_plan_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
               "fsib_plan_profile_read")
        return ms.value, n.value, b.value

    def _X(self, X):
        _need(X, "X", torch.float64)
        if X.dim() != 2 or X.shape[1] != self.dim:
            raise ValueError(f"X must have shape (M, {self.dim})")
        return X.shape[0]

    def spread(self, X, c, scale=1.0, out=None):
        M = self._X(X)
        c = _need(c, "c", self.cdtype)
        if tuple(c.shape) not in ((self.ntrans, M),) + (((M,),) if self.ntrans == 1 else ()):
            raise ValueError("c must have shape (ntrans, M) (or (M,) with ntrans = 1)")
        shp = ((self.ntrans,) if self.ntrans > 1 or c.dim() == 2 else ()) + self.spectral_shape
        out = torch.empty(shp, dtype=self.cdtype, device=X.device) if out is None else _need(out, "fhat", self.cdtype, shp)
        _check(self._lib.fsib_spread(self._h, M, _ptr(X), _ptr(c), _ptr(out), float(scale), _stream()), "fsib_spread")
        return out

    def spread_noalloc(self, X, c, out, scale=1.0):
        """Type-1 as spread() through the library's static per-GPU scratch (fsib_spread_noalloc): the
        call allocates nothing; `out` must be given.  M may exceed max_points within the scratch."""
        M = self._X(X)
        c = _need(c, "c", self.cdtype)
        if tuple(c.shape) not in ((self.ntrans, M),) + (((M,),) if self.ntrans == 1 else ()):
            raise ValueError("c must have shape (ntrans, M) (or (M,) with ntrans = 1)")
        shp = ((self.ntrans,) if self.ntrans > 1 or c.dim() == 2 else ()) + self.spectral_shape
        _need(out, "fhat", self.cdtype, shp)
        _check(self._lib.fsib_spread_noalloc(self._h, M, _ptr(X), _ptr(c), _ptr(out), float(scale), _stream()),
               "fsib_spread_noalloc")
        return out

    def interp(self, X, fhat, out=None):
        M = self._X(X)
        fhat = _need(fhat, "fhat", self.cdtype)
        if fhat.numel() != self.ntrans * int(torch.tensor(self.spectral_shape).prod()):
            raise ValueError("fhat must hold ntrans full spectral arrays")
        shp = (self.ntrans, M) if (self.ntrans > 1 or fhat.dim() == self.dim + 1) else (M,)
        out = torch.empty(shp, dtype=self.cdtype, device=X.device) if out is None else _need(out, "c", self.cdtype, shp)
        _check(self._lib.fsib_interp(self._h, M, _ptr(X), _ptr(fhat), _ptr(out), _stream()), "fsib_interp")
        return out

    def spectral_scale(self, fhat, axis=-1, scale=1.0, out=None, half=False):
        """scale * fhat (axis = -1) or scale * i k_axis * fhat (fsib_spectral_scale); full spectra
        (ntrans arrays) or, with half=True, the dim half spectra of real fields."""
        fhat = _need(fhat, "fhat", self.cdtype)
        if half:
            _need(fhat, "fhat", self.cdtype, (self.dim,) + self.half_shape)
        out = torch.empty_like(fhat) if out is None else _need(out, "out", self.cdtype, tuple(fhat.shape))
        _check(self._lib.fsib_spectral_scale(self._h, 1 if half else 0, int(axis), float(scale), _ptr(fhat), _ptr(out),
                                             _stream()), "fsib_spectral_scale")
        return out

    def grad_combine(self, u, v, gX, axis, scale=1.0, u2=None, v2=None):
        """gX[:, axis] = scale * sum_t Re(conj(u) v) for complex (ntrans, M) u, v, or
        scale * sum_a (u v + u2 v2) for real (M, dim) u, v (u2, v2 optional) (fsib_grad_combine)."""
        M = gX.shape[0]
        _need(gX, "gX", torch.float64, (M, self.dim))
        real = not u.is_complex()
        dt = self.rdtype if real else self.cdtype
        u = _need(u, "u", dt)
        v = _need(v, "v", dt)
        n = M * self.dim if real else M * self.ntrans
        if u.numel() != n or v.numel() != n:
            raise ValueError("u and v must hold (M, dim) real or ntrans x M complex values")
        if (u2 is None) != (v2 is None) or (u2 is not None and not real):
            raise ValueError("u2 and v2 go together, for real u, v only")
        if u2 is not None:
            _need(u2, "u2", dt, tuple(u.shape))
            _need(v2, "v2", dt, tuple(u.shape))
        _check(self._lib.fsib_grad_combine(self._h, M, 1 if real else 0, _ptr(u), _ptr(v), _ptr(u2), _ptr(v2),
                                           float(scale), _ptr(gX), int(axis), _stream()), "fsib_grad_combine")
        return gX

    def force_spread(self, X, S, scale, out=None):
        M = self._X(X)
        _need(S, "S", self.rdtype, (M, self.dim))
        shp = self.field_shape
        out = torch.empty(shp, dtype=self.cdtype, device=X.device) if out is None else _need(out, "fhat", self.cdtype, shp)
        _check(self._lib.fsib_force_spread(self._h, M, _ptr(X), _ptr(S), _ptr(out), float(scale), _stream()),
               "fsib_force_spread")
        return out

    def velocity_interp(self, X, uhat, out=None):
        M = self._X(X)
        _need(uhat, "uhat", self.cdtype, self.field_shape)
        out = torch.empty((M, self.dim), dtype=self.rdtype, device=X.device) if out is None else \
            _need(out, "U", self.rdtype, (M, self.dim))
        _check(self._lib.fsib_velocity_interp(self._h, M, _ptr(X), _ptr(uhat), _ptr(out), _stream()),
               "fsib_velocity_interp")
        return out

    def fluid_step(self, params, fhat, uhat, uhat_mid=None):
        shp = self.field_shape
        _need(fhat, "fhat", self.cdtype, shp)
        _need(uhat, "uhat", self.cdtype, shp)
        if uhat_mid is not None:
            _need(uhat_mid, "uhat_mid", self.cdtype, shp)
        _check(self._lib.fsib_fluid_step(self._h, ctypes.byref(params._s), _ptr(fhat), _ptr(uhat), _ptr(uhat_mid),
                                         _stream()), "fsib_fluid_step")
        return uhat

    def pressure(self, params, fhat, uhat=None, out=None):
        """Half spectrum of the pressure (fsib_pressure); uhat is needed for Navier-Stokes."""
        shp = (self.dim,) + self.half_shape
        _need(fhat, "fhat", self.cdtype, shp)
        if uhat is not None:
            _need(uhat, "uhat", self.cdtype, shp)
        out = torch.empty(self.half_shape, dtype=self.cdtype, device=fhat.device) if out is None else \
            _need(out, "phat", self.cdtype, self.half_shape)
        _check(self._lib.fsib_pressure(self._h, ctypes.byref(params._s), _ptr(fhat), _ptr(uhat), _ptr(out),
                                       _stream()), "fsib_pressure")
        return out

    def velocity(self, params, force, X, uhat, out=None):
        M = self._X(X)
        _need(uhat, "uhat", self.cdtype, self.field_shape)
        out = torch.empty((M, self.dim), dtype=self.rdtype, device=X.device) if out is None else \
            _need(out, "U", self.rdtype, (M, self.dim))
        _check(self._lib.fsib_velocity(self._h, ctypes.byref(params._s), ctypes.byref(force._s) if force else None, M,
                                       _ptr(X), _ptr(out), _ptr(uhat), _stream()), "fsib_velocity")
        return out

    def step(self, params, force, X, U, uhat, diag=None):
        M = self._X(X)
        _need(U, "U", self.rdtype, (M, self.dim))
        _need(uhat, "uhat", self.cdtype, self.field_shape)
        if diag is not None:
            _need(diag, "diag", torch.float64, (DIAG_COUNT,))
        _check(self._lib.fsib_step(self._h, ctypes.byref(params._s), ctypes.byref(force._s), M, _ptr(X), _ptr(U),
                                   _ptr(uhat), _ptr(diag), _stream()), "fsib_step")

    def steps(self, params, force, X, U, uhat, nsteps, diag=None):
        """nsteps steps of Alg. 1 in one call (fsib_steps): as nsteps calls of step(), with the
        interpolation of each step's U on the plan's second stream beside the next step's products."""
        M = self._X(X)
        _need(U, "U", self.rdtype, (M, self.dim))
        _need(uhat, "uhat", self.cdtype, self.field_shape)
        if diag is not None:
            _need(diag, "diag", torch.float64, (DIAG_COUNT,))
        _check(self._lib.fsib_steps(self._h, ctypes.byref(params._s), ctypes.byref(force._s), M, _ptr(X), _ptr(U),
                                    _ptr(uhat), int(nsteps), _ptr(diag), _stream()), "fsib_steps")


class Group:
    """Stokes simulations of several plans (different N, each plan with its own instances) stepped
    together (fsib_group_create / fsib_group_steps): every stage of a step is one launch over all plans.
    The plans must stay open while the group is used."""

    def __init__(self, plans):
        lib = load_library()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.fsib_group_create(len(self.plans), arr, ctypes.byref(h)), "fsib_group_create")
        self._h = h
        self._lib = lib

    def steps(self, params, forces, X, U, uhat, nsteps=1):
        """nsteps steps; params, forces, X, U, uhat: one entry per plan, as for Plan.step."""
        n = len(self.plans)
        if not all(len(a) == n for a in (params, forces, X, U, uhat)):
            raise ValueError(f"need {n} entries per operand")
        Ms = []
        for p, x, u, uh in zip(self.plans, X, U, uhat):
            M = p._X(x)
            _need(u, "U", p.rdtype, (M, p.dim))
            _need(uh, "uhat", p.cdtype, p.field_shape)
            Ms.append(M)
        prm = (_Params * n)(*[q._s for q in params])
        frc = (_Force * n)(*[f._s for f in forces])
        vp = lambda ts: (ctypes.c_void_p * n)(*[_ptr(t).value for t in ts])
        _check(self._lib.fsib_group_steps(self._h, prm, frc, (ctypes.c_int64 * n)(*Ms), vp(X), vp(U), vp(uhat),
                                          int(nsteps), _stream()), "fsib_group_steps")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fsib_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
