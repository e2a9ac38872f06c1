"""ctypes binding of the HIP library ``_lisaresp.so`` (C ABI in include/lisaresp.h).

Argument marshalling only: every step of the response runs in the library's
kernels.  Arrays are torch CUDA tensors (float64, contiguous); the stream is
torch's current stream unless one is given.  A missing library raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# LISARESP_LIB selects another build of the same library (tuning variants).
LIB_PATH = os.environ.get("LISARESP_LIB") or os.path.join(_HERE, "_lisaresp.so")
# LR_ABI_VERSION of include/lisaresp.h that the argument lists below follow
ABI_VERSION = 5

LR_XYZ, LR_AET, LR_XYZ_AET = 0, 1, 2
CHANNELS = {"XYZ": LR_XYZ, "AET": LR_AET, "XYZAET": LR_XYZ_AET}


class LisaRespError(RuntimeError):
    def __init__(self, status, where, message):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (where, message, _status_name(status)))


# status codes of include/lisaresp.h
LR_OK, LR_E_ARG, LR_E_RANGE, LR_E_UNSUPPORTED, LR_E_WORKSPACE, LR_E_HIP = range(6)


class lr_orbits(ctypes.Structure):
    _fields_ = [("t0", ctypes.c_double), ("dt", ctypes.c_double), ("n", ctypes.c_int64),
                ("coef", ctypes.c_void_p), ("L_min", ctypes.c_double),
                ("L_max", ctypes.c_double), ("R_max", ctypes.c_double)]


_lib = None


def _status_name(s):
    try:
        return lib().lr_status_str(int(s)).decode()
    except Exception:  # noqa: BLE001 - only used to decorate an error message
        return str(s)


def lib():
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is missing; build it with "
                           "`python -m paper_2204_06633_amd.csrc.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    d, i32, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    P = ctypes.POINTER
    po = P(lr_orbits)
    L.lr_status_str.restype = ctypes.c_char_p
    L.lr_status_str.argtypes = [i32]
    L.lr_last_error.restype = ctypes.c_char_p
    L.lr_abi_version.restype = i32
    if L.lr_abi_version() != ABI_VERSION:
        raise RuntimeError("%s has ABI version %d, this binding expects %d: rebuild it "
                           "(python -m paper_2204_06633_amd.csrc.build)"
                           % (LIB_PATH, L.lr_abi_version(), ABI_VERSION))
    L.lr_build_config.restype = ctypes.c_char_p
    L.lr_build_config.argtypes = []
    L.lr_orbits_bytes.restype = ctypes.c_size_t
    L.lr_orbits_bytes.argtypes = [i64]
    L.lr_orbits_init.argtypes = [d, d, i64, vp, vp, vp, ctypes.c_size_t, po, vp]
    L.lr_orbits_bounds.argtypes = [d, d, i64, vp, vp, po]
    L.lr_projection_padding.argtypes = [po, i32, d, P(i64), P(i64)]
    L.lr_tdi_padding.argtypes = [po, i32, i32, d, P(i64), P(i64)]
    L.lr_project_links.argtypes = [po, d, d, i64, vp, vp, vp, i32, i64, i64, vp, vp]
    L.lr_tdi_combine.argtypes = [po, d, d, i64, vp, i32, i32, i32, i64, i64, vp, vp]
    L.lr_tdi_adjoint.argtypes = [po, d, d, i64, i32, i32, i32, i64, i64, vp, vp, vp]
    L.lr_project_adjoint_workspace.restype = ctypes.c_size_t
    L.lr_project_adjoint_workspace.argtypes = [i64]
    L.lr_project_adjoint.argtypes = [po, d, d, i64, vp, vp, vp, i32, i64, i64, vp, vp, vp, vp,
                                     vp, ctypes.c_size_t, vp]
    L.lr_loglike_workspace.restype = ctypes.c_size_t
    L.lr_loglike.argtypes = [vp, vp, i64, d, vp, vp, vp, ctypes.c_size_t, vp]
    L.lr_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.lr_noalloc_scratch_bytes.argtypes = []
    L.lr_project_adjoint_noalloc.argtypes = [po, d, d, i64, vp, vp, vp, i32, i64, i64, vp, vp, vp,
                                             vp, vp]
    for name in ("lr_orbits_init", "lr_orbits_bounds", "lr_projection_padding", "lr_tdi_padding",
                 "lr_project_links", "lr_tdi_combine", "lr_tdi_adjoint", "lr_project_adjoint",
                 "lr_loglike", "lr_project_adjoint_noalloc"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def build_config():
    """The tuning switches the loaded library was compiled with (a dict of
    name -> int, from lr_build_config)."""
    text = lib().lr_build_config().decode()
    return {k: int(v) for k, v in (item.split("=") for item in text.split(";") if item)}


def _check(status, where):
    if status != 0:
        raise LisaRespError(status, where, lib().lr_last_error().decode())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _size(t, name, shape=None, numel=None, min_numel=None):
    """Check a tensor argument's extent against what the kernels will touch
    (before any pointer is handed to the library): exact ``shape``, exact
    ``numel`` or at least ``min_numel`` elements.  Raises ValueError."""
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if shape is not None and tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError("%s has shape %s, the call needs %s" % (name, tuple(t.shape),
                                                                  tuple(int(v) for v in shape)))
    if numel is not None and t.numel() != int(numel):
        raise ValueError("%s has %d elements, the call needs %d" % (name, t.numel(), int(numel)))
    if min_numel is not None and t.numel() < int(min_numel):
        raise ValueError("%s has %d elements, the call needs at least %d"
                         % (name, t.numel(), int(min_numel)))


def _same_device(*named):
    """All given tensors (None skipped) on one device."""
    devs = {(n, t.device) for n, t in named if t is not None}
    if len({d for _, d in devs}) > 1:
        raise ValueError("arguments on different devices: %s"
                         % ", ".join("%s on %s" % (n, d) for n, d in sorted(devs, key=str)))


# ---------------------------------------------------------------------------
# Orbits
# ---------------------------------------------------------------------------

class Orbits:
    """Orbit splines resident on the GPU (lr_orbits_init).

    ``x`` [n][3][3] m and ``ltt`` [n][6] s are host arrays on the coarse grid
    t0 + k*dt."""

    def __init__(self, t0, dt, x, ltt, device="cuda", stream=None):
        import numpy as np
        import torch
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3, 3))
        ltt = np.ascontiguousarray(np.asarray(ltt, dtype=np.float64).reshape(-1, 6))
        n = x.shape[0]
        if ltt.shape[0] != n:
            raise ValueError("x and ltt have different lengths")
        nbytes = lib().lr_orbits_bytes(n)
        self.storage = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=device)
        self.c = lr_orbits()
        _check(lib().lr_orbits_init(float(t0), float(dt), n, x.ctypes.data, ltt.ctypes.data,
                                    ctypes.c_void_p(self.storage.data_ptr()), nbytes,
                                    ctypes.byref(self.c), _stream(stream)), "lr_orbits_init")

    @classmethod
    def from_samples(cls, s, **kw):
        return cls(s.t0, s.dt, s.x, s.ltt, **kw)

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def projection_padding(self, order, dt):
        f, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lr_projection_padding(self.ref, int(order), float(dt), ctypes.byref(f),
                                           ctypes.byref(b)), "lr_projection_padding")
        return f.value, b.value

    def tdi_padding(self, order, generation, dt):
        f, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lr_tdi_padding(self.ref, int(order), int(generation), float(dt),
                                    ctypes.byref(f), ctypes.byref(b)), "lr_tdi_padding")
        return f.value, b.value


class OrbitBounds:
    """Host-only orbit handle (lr_orbits_bounds): the spline fit's bounds of
    the light times and distances, enough for the padding rules, with no
    device involved (sizing buffers before anything is allocated)."""

    def __init__(self, t0, dt, x, ltt):
        import numpy as np
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3, 3))
        ltt = np.ascontiguousarray(np.asarray(ltt, dtype=np.float64).reshape(-1, 6))
        if ltt.shape[0] != x.shape[0]:
            raise ValueError("x and ltt have different lengths")
        self.c = lr_orbits()
        _check(lib().lr_orbits_bounds(float(t0), float(dt), x.shape[0], x.ctypes.data,
                                      ltt.ctypes.data, ctypes.byref(self.c)), "lr_orbits_bounds")

    @classmethod
    def from_samples(cls, s):
        return cls(s.t0, s.dt, s.x, s.ltt)

    ref = Orbits.ref
    projection_padding = Orbits.projection_padding
    tdi_padding = Orbits.tdi_padding


# ---------------------------------------------------------------------------
# Plain per-template calls
# ---------------------------------------------------------------------------

def _opt(t, name):
    return ctypes.c_void_p(0) if t is None else _dev(t, name)


def project_links(orb: Orbits, t0_h, dt, hp, hc, sky, order, y_start, n_y, y=None,
                  stream=None):
    """Link responses y[6][n_y] for the link samples at h-indices
    y_start .. y_start + n_y - 1 (lr_project_links).  ``sky`` is a device
    tensor [lam, beta]."""
    import torch
    if y is None:
        y = torch.empty((6, n_y), dtype=torch.float64, device=hp.device)
    _size(hc, "hc", numel=hp.numel())
    _size(sky, "sky", numel=2)
    _size(y, "y", shape=(6, n_y))
    _same_device(("hp", hp), ("hc", hc), ("sky", sky), ("y", y))
    _check(lib().lr_project_links(orb.ref, float(t0_h), float(dt), hp.numel(), _dev(hp, "hp"),
                                  _dev(hc, "hc"), _dev(sky, "sky"), int(order), int(y_start),
                                  int(n_y), _dev(y, "y"), _stream(stream)), "lr_project_links")
    return y


def tdi_combine(orb: Orbits, t0_y, dt, y, generation, order, channels, out_start, n_out,
                out=None, stream=None):
    """TDI channels out[3 or 6][n_out] at y-indices out_start .. out_start +
    n_out - 1 (lr_tdi_combine).  ``channels`` is "XYZ", "AET" or "XYZAET"."""
    import torch
    rows = 6 if channels == "XYZAET" else 3
    if out is None:
        out = torch.empty((rows, n_out), dtype=torch.float64, device=y.device)
    if y.dim() != 2 or y.shape[0] != 6:
        raise ValueError("y must be [6][n_y], got shape %s" % (tuple(y.shape),))
    _size(out, "out", shape=(rows, n_out))
    _same_device(("y", y), ("out", out))
    n_y = y.shape[-1]
    _check(lib().lr_tdi_combine(orb.ref, float(t0_y), float(dt), n_y, _dev(y, "y"),
                                int(generation), int(order), CHANNELS[channels], int(out_start),
                                int(n_out), _dev(out, "out"), _stream(stream)), "lr_tdi_combine")
    return out


# ---------------------------------------------------------------------------
# Adjoints and likelihood
# ---------------------------------------------------------------------------

def tdi_adjoint(orb: Orbits, t0_y, dt, n_y, generation, order, channels, out_start, g_out,
                g_y=None, stream=None):
    """g_y[6][n_y] = transpose of tdi_combine applied to g_out (lr_tdi_adjoint)."""
    import torch
    if g_y is None:
        g_y = torch.empty((6, n_y), dtype=torch.float64, device=g_out.device)
    rows = 6 if channels == "XYZAET" else 3
    if g_out.dim() != 2 or g_out.shape[0] != rows:
        raise ValueError("g_out must be [%d][n_out] for %s, got shape %s"
                         % (rows, channels, tuple(g_out.shape)))
    _size(g_y, "g_y", shape=(6, n_y))
    _same_device(("g_out", g_out), ("g_y", g_y))
    n_out = g_out.shape[-1]
    _check(lib().lr_tdi_adjoint(orb.ref, float(t0_y), float(dt), int(n_y), int(generation),
                                int(order), CHANNELS[channels], int(out_start), int(n_out),
                                _dev(g_out, "g_out"), _dev(g_y, "g_y"), _stream(stream)),
           "lr_tdi_adjoint")
    return g_y


def project_adjoint(orb: Orbits, t0_h, dt, n_h, hp, hc, sky, order, y_start, g_y, want_sky=True,
                    g_hp=None, g_hc=None, g_sky=None, work=None, stream=None):
    """(g_hp, g_hc, g_sky) = transpose of project_links applied to g_y
    (lr_project_adjoint); g_sky is None unless ``want_sky``."""
    import torch
    dev = g_y.device
    if g_y.dim() != 2 or g_y.shape[0] != 6:
        raise ValueError("g_y must be [6][n_y], got shape %s" % (tuple(g_y.shape),))
    n_y = g_y.shape[-1]
    _size(hp, "hp", numel=n_h)
    _size(hc, "hc", numel=n_h)
    _size(sky, "sky", numel=2)
    _size(g_hp, "g_hp", numel=n_h)
    _size(g_hc, "g_hc", numel=n_h)
    if g_hp is None:
        g_hp = torch.empty(n_h, dtype=torch.float64, device=dev)
    if g_hc is None:
        g_hc = torch.empty(n_h, dtype=torch.float64, device=dev)
    nbytes = 0
    if want_sky:
        if g_sky is None:
            g_sky = torch.empty(2, dtype=torch.float64, device=dev)
        nbytes = lib().lr_project_adjoint_workspace(n_y)
        if work is None:
            work = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=dev)
    else:
        g_sky = None
    _size(g_sky, "g_sky", numel=2)
    _same_device(("g_y", g_y), ("hp", hp), ("hc", hc), ("sky", sky), ("g_hp", g_hp),
                 ("g_hc", g_hc), ("g_sky", g_sky), ("work", work if want_sky else None))
    _check(lib().lr_project_adjoint(orb.ref, float(t0_h), float(dt), int(n_h), _opt(hp, "hp"),
                                    _opt(hc, "hc"), _dev(sky, "sky"), int(order), int(y_start),
                                    int(n_y), _dev(g_y, "g_y"), _dev(g_hp, "g_hp"),
                                    _dev(g_hc, "g_hc"), _opt(g_sky, "g_sky"),
                                    _opt(work if want_sky else None, "work"),
                                    work.numel() * 8 if want_sky else 0, _stream(stream)),
           "lr_project_adjoint")
    return g_hp, g_hc, g_sky


def project_adjoint_noalloc(orb: Orbits, t0_h, dt, n_h, hp, hc, sky, order, y_start, g_y,
                            g_hp, g_hc, g_sky=None, stream=None):
    """lr_project_adjoint_noalloc: project_adjoint with caller-provided outputs
    and the sky-gradient partial sums in the library's static device
    scratch (no allocation by the library).  g_sky is optional."""
    if g_y.dim() != 2 or g_y.shape[0] != 6:
        raise ValueError("g_y must be [6][n_y], got shape %s" % (tuple(g_y.shape),))
    n_y = g_y.shape[-1]
    _size(hp, "hp", numel=n_h)
    _size(hc, "hc", numel=n_h)
    _size(sky, "sky", numel=2)
    _size(g_hp, "g_hp", numel=n_h)
    _size(g_hc, "g_hc", numel=n_h)
    _size(g_sky, "g_sky", numel=2)
    _same_device(("g_y", g_y), ("hp", hp), ("hc", hc), ("sky", sky), ("g_hp", g_hp),
                 ("g_hc", g_hc), ("g_sky", g_sky))
    _check(lib().lr_project_adjoint_noalloc(orb.ref, float(t0_h), float(dt), int(n_h),
                                            _opt(hp, "hp"), _opt(hc, "hc"), _dev(sky, "sky"),
                                            int(order), int(y_start), int(n_y), _dev(g_y, "g_y"),
                                            _dev(g_hp, "g_hp"), _dev(g_hc, "g_hc"),
                                            _opt(g_sky, "g_sky"), _stream(stream)),
           "lr_project_adjoint_noalloc")
    return g_hp, g_hc, g_sky


def noalloc_scratch_bytes():
    """Bytes of the static device scratch behind the *_noalloc entry points."""
    return int(lib().lr_noalloc_scratch_bytes())


def loglike(h, data, sigma, want_grad=True, out=None, g_h=None, work=None, stream=None):
    """(loglike[1], g_h) of the white-noise likelihood (lr_loglike)."""
    import torch
    dev = h.device
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=dev)
    if want_grad and g_h is None:
        g_h = torch.empty_like(h)
    nbytes = lib().lr_loglike_workspace()
    if work is None:
        work = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    _size(data, "data", numel=h.numel())
    _size(out, "loglike", min_numel=1)
    if want_grad:
        _size(g_h, "g_h", numel=h.numel())
    _size(work, "work", min_numel=(nbytes + 7) // 8)
    _same_device(("h", h), ("data", data), ("loglike", out), ("g_h", g_h if want_grad else None),
                 ("work", work))
    _check(lib().lr_loglike(_dev(h, "h"), _dev(data, "data"), h.numel(), float(sigma),
                            _dev(out, "loglike"), _opt(g_h if want_grad else None, "g_h"),
                            _dev(work, "work"), work.numel() * 8, _stream(stream)), "lr_loglike")
    return out, (g_h if want_grad else None)


# ---------------------------------------------------------------------------
# Batches (lr_batch_*): many templates sharing one output time grid
# ---------------------------------------------------------------------------

class lr_template(ctypes.Structure):
    _fields_ = [("h_offset", ctypes.c_int64), ("n_h", ctypes.c_int64),
                ("out_start", ctypes.c_int64), ("n_out", ctypes.c_int64),
                ("out_offset", ctypes.c_int64)]


class lr_batch(ctypes.Structure):
    _fields_ = [("proj", lr_orbits), ("tdi", lr_orbits), ("t0", ctypes.c_double),
                ("dt", ctypes.c_double), ("order", ctypes.c_int), ("generation", ctypes.c_int),
                ("channels", ctypes.c_int), ("group", ctypes.c_int), ("front", ctypes.c_int),
                ("tile_out", ctypes.c_int), ("blocks", ctypes.c_int), ("adjoint", ctypes.c_int),
                ("tile", ctypes.c_int), ("segment", ctypes.c_int),
                ("n_templates", ctypes.c_int64), ("n_items", ctypes.c_int64),
                ("n_tdi_items", ctypes.c_int64), ("n_proj_items", ctypes.c_int64),
                ("n_like_items", ctypes.c_int64), ("n_tdi_citems", ctypes.c_int64),
                ("n_padj_citems", ctypes.c_int64), ("gy_doubles", ctypes.c_int64),
                ("h_extent", ctypes.c_int64), ("out_extent", ctypes.c_int64),
                ("ws", ctypes.c_void_p), ("off", ctypes.c_size_t * 24)]


def _batch_lib():
    L = lib()
    if getattr(L, "_batch_ready", False):
        return L
    d, i32, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    P = ctypes.POINTER
    pt, po, pb = P(lr_template), P(lr_orbits), P(lr_batch)
    L.lr_batch_workspace.restype = ctypes.c_size_t
    L.lr_batch_workspace.argtypes = [pt, i64, po, d, i32, i32, i32, i32, i32, i32, i32]
    L.lr_batch_prepare.argtypes = [pt, i64, po, po, d, d, i32, i32, i32, i32, i32, i32, i32, vp,
                                   ctypes.c_size_t, pb, vp]
    L.lr_response.argtypes = [pb, vp, vp, vp, vp, vp]
    L.lr_response_gb.argtypes = [pb, vp, vp, vp]
    L.lr_response_adjoint_gb.argtypes = [pb, vp, vp, vp, vp]
    L.lr_response_adjoint.argtypes = [pb, vp, vp, vp, vp, vp, vp, vp, vp]
    L.lr_batch_loglike.argtypes = [pb, vp, vp, d, vp, vp, vp]
    L.lr_batch_set_grid.argtypes = [pb, i32]
    for name in ("lr_batch_prepare", "lr_response", "lr_response_gb", "lr_response_adjoint",
                 "lr_response_adjoint_gb",
                 "lr_batch_loglike",
                 "lr_batch_set_grid"):
        getattr(L, name).restype = i32
    L._batch_ready = True
    return L


class Batch:
    """A prepared batch (lr_batch_prepare) and its device workspace.

    ``templates``: sequence of (h_offset, n_h, out_start, n_out, out_offset).
    ``group``: templates per forward work item; ``tile``: link samples per
    forward tile (256, 512, 1024; 0 = 512); ``segment``: tiles per forward
    work item, which pass the TDI halo on (1..64; 0 = automatic).
    The orbit objects must outlive the batch (it holds their device pointers).
    """

    def __init__(self, templates, orb_proj: Orbits, orb_tdi: Orbits, t0, dt, order=25,
                 generation=2, channels="XYZ", group=2, adjoint=False, device="cuda",
                 stream=None, tile=0, segment=0):
        import torch
        L = _batch_lib()
        n = len(templates)
        arr = (lr_template * max(n, 1))()
        for k, t in enumerate(templates):
            arr[k] = lr_template(*[int(v) for v in t])
        self.templates = [tuple(int(v) for v in t) for t in templates]
        self.orb_proj, self.orb_tdi = orb_proj, orb_tdi
        self.channels = channels
        self.rows = 6 if channels == "XYZAET" else 3
        nbytes = L.lr_batch_workspace(arr, n, orb_tdi.ref, float(dt), int(order), int(generation),
                                      CHANNELS[channels], int(group), int(tile), int(segment),
                                      int(bool(adjoint)))
        if nbytes == 0:
            raise LisaRespError(1, "lr_batch_workspace", L.lr_last_error().decode())
        self.ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
        self.c = lr_batch()
        _check(L.lr_batch_prepare(arr, n, orb_proj.ref, orb_tdi.ref, float(t0), float(dt),
                                  int(order), int(generation), CHANNELS[channels], int(group),
                                  int(tile), int(segment), int(bool(adjoint)),
                                  ctypes.c_void_p(self.ws.data_ptr()),
                                  self.ws.numel() * 8, ctypes.byref(self.c), _stream(stream)),
               "lr_batch_prepare")

    @property
    def n(self):
        return len(self.templates)

    def _check_inputs(self, hp, hc, sky):
        """h+ / hx cover every template's h range; sky holds n (lam, beta)."""
        _size(hp, "hp", min_numel=self.h_extent)
        _size(hc, "hc", min_numel=self.h_extent)
        _size(sky, "sky", min_numel=2 * self.n)

    @property
    def blocks(self):
        """Work-groups of the persistent forward launch."""
        return int(self.c.blocks)

    @property
    def tile(self):
        """Link samples per forward tile."""
        return int(self.c.tile)

    @property
    def segment(self):
        """Tiles per forward work item (the value the plan used)."""
        return int(self.c.segment)

    def set_grid(self, blocks):
        _check(_batch_lib().lr_batch_set_grid(ctypes.byref(self.c), int(blocks)),
               "lr_batch_set_grid")

    @property
    def h_extent(self):
        return int(self.c.h_extent)

    @property
    def out_extent(self):
        return int(self.c.out_extent)

    def response(self, hp, hc, sky, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(max(self.out_extent, 1), dtype=torch.float64, device=hp.device)
        self._check_inputs(hp, hc, sky)
        _size(out, "out", min_numel=self.out_extent)
        _same_device(("hp", hp), ("hc", hc), ("sky", sky), ("out", out))
        _check(_batch_lib().lr_response(ctypes.byref(self.c), _dev(hp, "hp"), _dev(hc, "hc"),
                                        _dev(sky, "sky"), _dev(out, "out"), _stream(stream)),
               "lr_response")
        return out

    def response_gb(self, params, out=None, stream=None):
        """lr_response_gb: the forward with h+ / hx synthesised in the kernel
        from Galactic-binary parameter rows params [n][8]."""
        import torch
        if params.dim() != 2 or params.shape[0] != self.n or params.shape[1] != 8:
            raise ValueError("params must be [%d][8], got shape %s" % (self.n,
                                                                     tuple(params.shape)))
        if out is None:
            out = torch.empty(max(self.out_extent, 1), dtype=torch.float64, device=params.device)
        _size(out, "out", min_numel=self.out_extent)
        _same_device(("params", params), ("out", out))
        _check(_batch_lib().lr_response_gb(ctypes.byref(self.c), _dev(params, "params"),
                                           _dev(out, "out"), _stream(stream)),
               "lr_response_gb")
        return out

    def adjoint_gb(self, params, g_out, g_params=None, stream=None):
        """lr_response_adjoint_gb: d<g_out, out>/d params [n][8] of the
        waveform-mode forward (``response_gb``)."""
        import torch
        if params.dim() != 2 or params.shape[0] != self.n or params.shape[1] != 8:
            raise ValueError("params must be [%d][8], got shape %s" % (self.n,
                                                                     tuple(params.shape)))
        if g_params is None:
            g_params = torch.empty_like(params)
        _size(g_params, "g_params", shape=(self.n, 8))
        _size(g_out, "g_out", min_numel=self.out_extent)
        _same_device(("params", params), ("g_out", g_out), ("g_params", g_params))
        _check(_batch_lib().lr_response_adjoint_gb(ctypes.byref(self.c), _dev(params, "params"),
                                                   _dev(g_out, "g_out"),
                                                   _dev(g_params, "g_params"), _stream(stream)),
               "lr_response_adjoint_gb")
        return g_params

    def adjoint(self, hp, hc, sky, g_out, want_sky=True, g_hp=None, g_hc=None, g_sky=None,
                stream=None):
        import torch
        dev = g_out.device
        if g_hp is None:
            g_hp = torch.empty(max(self.h_extent, 1), dtype=torch.float64, device=dev)
        if g_hc is None:
            g_hc = torch.empty(max(self.h_extent, 1), dtype=torch.float64, device=dev)
        if want_sky and g_sky is None:
            g_sky = torch.empty((max(self.n, 1), 2), dtype=torch.float64, device=dev)
        if want_sky and (hp is None or hc is None):
            raise ValueError("the sky gradient needs hp and hc")
        self._check_inputs(hp, hc, sky)
        _size(g_out, "g_out", min_numel=self.out_extent)
        _size(g_hp, "g_hp", min_numel=self.h_extent)
        _size(g_hc, "g_hc", min_numel=self.h_extent)
        if want_sky:
            _size(g_sky, "g_sky", min_numel=2 * self.n)
        _same_device(("hp", hp), ("hc", hc), ("sky", sky), ("g_out", g_out), ("g_hp", g_hp),
                     ("g_hc", g_hc), ("g_sky", g_sky if want_sky else None))
        _check(_batch_lib().lr_response_adjoint(
            ctypes.byref(self.c), _opt(hp, "hp"), _opt(hc, "hc"), _dev(sky, "sky"),
            _dev(g_out, "g_out"), _dev(g_hp, "g_hp"), _dev(g_hc, "g_hc"),
            _opt(g_sky if want_sky else None, "g_sky"), _stream(stream)), "lr_response_adjoint")
        return g_hp, g_hc, (g_sky if want_sky else None)

    def loglike(self, out, data, sigma, want_grad=True, ll=None, g_out=None, stream=None):
        import torch
        dev = out.device
        if ll is None:
            ll = torch.empty(max(self.n, 1), dtype=torch.float64, device=dev)
        if want_grad and g_out is None:
            g_out = torch.zeros_like(out)
        _size(out, "out", min_numel=self.out_extent)
        _size(data, "data", min_numel=self.out_extent)
        _size(ll, "loglike", min_numel=self.n)
        if want_grad:
            _size(g_out, "g_out", min_numel=self.out_extent)
        _same_device(("out", out), ("data", data), ("loglike", ll),
                     ("g_out", g_out if want_grad else None))
        _check(_batch_lib().lr_batch_loglike(
            ctypes.byref(self.c), _dev(out, "out"), _dev(data, "data"), float(sigma),
            _dev(ll, "loglike"), _opt(g_out if want_grad else None, "g_out"), _stream(stream)),
            "lr_batch_loglike")
        return ll, (g_out if want_grad else None)

    def output_block(self, out, k):
        """View of template k's [rows][n_out] output block."""
        _, _, _, n_out, off = self.templates[k]
        return out[off:off + self.rows * n_out].view(self.rows, n_out)


# ---------------------------------------------------------------------------
# Frequency-domain likelihood (lr_fd_*)
# ---------------------------------------------------------------------------

class lr_fd_plan(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_fft", ctypes.c_int64), ("max_batch", ctypes.c_int64),
                ("channels", ctypes.c_int), ("log2n", ctypes.c_int), ("passes", ctypes.c_int),
                ("q", ctypes.c_int * 3), ("dt", ctypes.c_double), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("off", ctypes.c_size_t * 6)]


def _fd_lib():
    L = lib()
    if getattr(L, "_fd_ready", False):
        return L
    d, i32, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    pp = ctypes.POINTER(lr_fd_plan)
    L.lr_fd_length.restype = i64
    L.lr_fd_length.argtypes = [i64]
    L.lr_fd_workspace.restype = ctypes.c_size_t
    L.lr_fd_workspace.argtypes = [i64, i32, i64]
    L.lr_fd_prepare.restype = i32
    L.lr_fd_prepare.argtypes = [i64, i32, d, vp, i64, vp, vp, i64, vp, ctypes.c_size_t, pp, vp]
    L.lr_fd_loglike.restype = i32
    L.lr_fd_loglike.argtypes = [pp, i64, vp, i64, i64, vp, vp, vp]
    L._fd_ready = True
    return L


def fd_length(n):
    """Transform length lr_fd_length(n) (power of two >= max(n, 4096))."""
    m = _fd_lib().lr_fd_length(int(n))
    if m < 0:
        raise ValueError("no transform length for n = %d" % n)
    return int(m)


class FdPlan:
    """Frequency-domain likelihood plan (lr_fd_prepare) and its workspace.

    ``data``: [C][n] device series (C = 2: A, E; C = 3: A, E, T); ``w_ae``,
    ``w_t``: device bin weights [fd_length(n) // 2 + 1] (w_t unused for C =
    2); ``max_batch``: templates per launch sequence (sets the workspace)."""

    def __init__(self, data, w_ae, w_t, dt, max_batch=1, stream=None):
        import torch
        if data.dim() != 2:
            raise ValueError("data must be [channels][n]")
        C, n = data.shape
        L = _fd_lib()
        if C not in (2, 3):
            raise ValueError("data must hold 2 (A, E) or 3 (A, E, T) channels")
        n_bins = fd_length(n) // 2 + 1
        _size(w_ae, "w_ae", numel=n_bins)
        if C == 3:
            if w_t is None:
                raise ValueError("w_t is needed for three channels")
            _size(w_t, "w_t", numel=n_bins)
        _same_device(("data", data), ("w_ae", w_ae), ("w_t", w_t if C == 3 else None))
        nbytes = L.lr_fd_workspace(n, C, max_batch)
        if nbytes == 0:
            raise ValueError("invalid plan arguments (n=%d, channels=%d, max_batch=%d)"
                             % (n, C, max_batch))
        self.ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=data.device)
        self.c = lr_fd_plan()
        _check(L.lr_fd_prepare(n, C, float(dt), _dev(data, "data"), data.stride(0),
                               _dev(w_ae, "w_ae"), _opt(w_t if C == 3 else None, "w_t"),
                               int(max_batch), _dev(self.ws, "ws"), nbytes, ctypes.byref(self.c),
                               _stream(stream)), "lr_fd_prepare")
        self.n, self.channels, self.dt = n, C, float(dt)
        self.n_fft, self.passes = int(self.c.n_fft), int(self.c.passes)
        self.max_batch = int(max_batch)

    def loglike(self, h, want_grad=True, stats=None, g_h=None, stream=None):
        """(stats [B][3] = rr, hh, dh; g_h = d logL/dh or None) for h of shape
        [B][C][n] (or [C][n], then B = 1)."""
        import torch
        hb = h.unsqueeze(0) if h.dim() == 2 else h
        if hb.shape[1:] != (self.channels, self.n):
            raise ValueError("h must be [B][%d][%d]" % (self.channels, self.n))
        B = hb.shape[0]
        if stats is None:
            stats = torch.empty((B, 3), dtype=torch.float64, device=h.device)
        if want_grad and g_h is None:
            g_h = torch.empty_like(hb)
        _size(stats, "stats", shape=(B, 3))
        if want_grad:
            if g_h.dim() == 2:
                g_h = g_h.unsqueeze(0)
            _size(g_h, "g_h", shape=tuple(hb.shape))
            if g_h.stride() != hb.stride():
                raise ValueError("g_h must be laid out like h")
        _same_device(("h", h), ("stats", stats), ("g_h", g_h if want_grad else None),
                     ("workspace", self.ws))
        _check(_fd_lib().lr_fd_loglike(ctypes.byref(self.c), B, _dev(hb, "h"), hb.stride(0),
                                       hb.stride(1), _dev(stats, "stats"),
                                       _opt(g_h if want_grad else None, "g_h"), _stream(stream)),
               "lr_fd_loglike")
        if want_grad and h.dim() == 2:
            g_h = g_h[0]
        return stats, (g_h if want_grad else None)


# ---------------------------------------------------------------------------
# Galactic-binary polarisations (lr_gb_*)
# ---------------------------------------------------------------------------

def _gb_lib():
    L = lib()
    if getattr(L, "_gb_ready", False):
        return L
    d, i64, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    L.lr_gb_polarizations.restype = ctypes.c_int
    L.lr_gb_polarizations.argtypes = [vp, i64, i64, i64, d, vp, vp, i64, vp]
    L.lr_gb_adjoint_workspace.restype = ctypes.c_size_t
    L.lr_gb_adjoint_workspace.argtypes = [i64, i64]
    L.lr_gb_polarizations_adjoint.restype = ctypes.c_int
    L.lr_gb_polarizations_adjoint.argtypes = [vp, i64, i64, i64, d, vp, vp, i64, vp, vp,
                                              ctypes.c_size_t, vp]
    L._gb_ready = True
    return L


def _dev_rows(t, name):
    """Pointer of a float64 CUDA tensor [n][m] whose rows are contiguous (any
    row stride)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError("%s must be [n][m] with contiguous rows" % name)
    return ctypes.c_void_p(t.data_ptr())


def gb_polarizations(params, k0, n_h, dt, hp=None, hc=None, stream=None):
    """(h+, hx) [n][n_h] for params [n][8] on t_j = (k0 + j) dt
    (lr_gb_polarizations)."""
    import torch
    if params.dim() != 2 or params.shape[1] != 8:
        raise ValueError("params must be [n][8], got shape %s" % (tuple(params.shape),))
    n = params.shape[0]
    if hp is None:
        hp = torch.empty((n, n_h), dtype=torch.float64, device=params.device)
    if hc is None:
        hc = torch.empty((n, n_h), dtype=torch.float64, device=params.device)
    if hp.stride(0) != hc.stride(0):
        raise ValueError("hp and hc must share one row stride")
    for name, t in (("hp", hp), ("hc", hc)):
        if t.dim() != 2 or t.shape[0] != n or t.shape[1] < n_h:
            raise ValueError("%s must be [%d][>= %d], got shape %s" % (name, n, n_h,
                                                                     tuple(t.shape)))
    _same_device(("params", params), ("hp", hp), ("hc", hc))
    _check(_gb_lib().lr_gb_polarizations(_dev(params, "params"), n, int(k0), int(n_h), float(dt),
                                         _dev_rows(hp, "hp"), _dev_rows(hc, "hc"),
                                         max(hp.stride(0), int(n_h)), _stream(stream)),
           "lr_gb_polarizations")
    return hp, hc


def gb_polarizations_adjoint(params, k0, dt, g_hp, g_hc, g_params=None, work=None, stream=None):
    """d/dparams of sum(g_hp h+ + g_hc hx), [n][8] (lr_gb_polarizations_adjoint)."""
    import torch
    if g_hp.dim() != 2 or g_hc.shape != g_hp.shape:
        raise ValueError("g_hp and g_hc must be [n][n_h] of one shape")
    n, n_h = g_hp.shape
    _size(params, "params", shape=(n, 8))
    L = _gb_lib()
    if g_params is None:
        g_params = torch.empty((n, 8), dtype=torch.float64, device=params.device)
    _size(g_params, "g_params", shape=(n, 8))
    nb = L.lr_gb_adjoint_workspace(n, n_h)
    if work is None:
        work = torch.empty((nb + 7) // 8, dtype=torch.float64, device=params.device)
    _size(work, "work", min_numel=(nb + 7) // 8)
    if g_hp.stride(0) != g_hc.stride(0):
        raise ValueError("g_hp and g_hc must share one row stride")
    _same_device(("params", params), ("g_hp", g_hp), ("g_hc", g_hc), ("g_params", g_params),
                 ("work", work))
    _check(L.lr_gb_polarizations_adjoint(_dev(params, "params"), n, int(k0), int(n_h), float(dt),
                                         _dev_rows(g_hp, "g_hp"), _dev_rows(g_hc, "g_hc"),
                                         max(g_hp.stride(0), int(n_h)),
                                         _dev(g_params, "g_params"), _dev(work, "work"),
                                         work.numel() * 8, _stream(stream)),
           "lr_gb_polarizations_adjoint")
    return g_params
