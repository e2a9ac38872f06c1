"""Plain CPU FP64 oracle of the generic LISA time-domain response.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may use it; the product path never does.  It
shares no code with the HIP library and never imports it.

Pieces and the passages of arXiv:2204.06633 they follow:
  * orbit interpolation (the coarse orbit data are interpolated once and
    evaluated at every sample time, Sec. IV.E): not-a-knot cubic splines from
    scipy, evaluated in C;
  * link projection y_ij (Sec. IV.B) and Michelson X1/X2 with Y, Z by cyclic
    relabelling (Sec. IV.C) in ``oracle.c``;
  * A, E, T (Sec. IV.C) and the white-noise log-likelihood -<d-h|d-h>/2 summed
    over channels (Sec. II.A and IV.C) in NumPy with exactly rounded sums;
  * the term lists of X1 / X2 in ``tdi_terms.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import tdi_terms

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
C_LIGHT = 299792458.0


def build(force=False):
    """Compile oracle.c with gcc (-O2, no fast-math, OpenMP)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        pd, pi64, pi32 = P(d), P(i64), P(i32)
        L.orc_lagrange_weights.argtypes = [i32, d, pd]
        L.orc_interp.argtypes = [pd, i64, i32, i64, d, pd]
        L.orc_interp.restype = i32
        L.orc_orbit_state.argtypes = [d, i64, pd, d, pd, pd]
        L.orc_project.argtypes = [d, i64, pd, d, d, pd, pd, i64, d, d, i32, pi64, i64, pd]
        L.orc_project.restype = i32
        L.orc_tdi.argtypes = [d, i64, pd, d, d, pd, i64, i32, i32, pi32, pi32, pi32, pi32, pi32,
                              pi64, i64, pd]
        L.orc_tdi.restype = i32
        L.orc_tdi_adjoint.argtypes = [d, i64, pd, d, d, i64, i32, i32, pi32, pi32, pi32, pi32,
                                      pi32, pi64, i64, pd, pd]
        L.orc_tdi_adjoint.restype = i32
        L.orc_project_adjoint.argtypes = [d, i64, pd, d, d, i64, d, d, i32, pi64, i64, pd, pd, pd]
        L.orc_project_adjoint.restype = i32
        L.orc_max_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_sky_basis.argtypes = [d, d, pd, pd, pd]
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def max_threads():
    return lib().orc_max_threads()


def set_threads(n):
    """Threads of the oracle's OpenMP loops (for timing at 1 thread and at
    all cores)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------------------
# Orbits: not-a-knot cubic splines of the 9 position and 6 light-time series.
# ---------------------------------------------------------------------------

class Orbits:
    """Spline representation of coarse orbit samples.

    ``t0`` is the absolute time of coarse sample 0; times given to the oracle
    functions are converted to "seconds since t0" once per call.
    """

    def __init__(self, t0, dt, x, ltt):
        from scipy.interpolate import CubicSpline
        x = np.asarray(x, dtype=np.float64).reshape(-1, 9)
        ltt = np.asarray(ltt, dtype=np.float64).reshape(-1, 6)
        n = x.shape[0]
        if n < 4:
            raise ValueError("need at least 4 coarse orbit samples")
        tk = dt * np.arange(n, dtype=np.float64)
        series = np.concatenate([x, ltt], axis=1)          # [n][15]
        coef = np.empty((15, n - 1, 4))
        for s in range(15):
            cs = CubicSpline(tk, series[:, s], bc_type="not-a-knot")
            coef[s] = cs.c[::-1].T                          # ascending powers
        self.t0, self.dt, self.nseg = float(t0), float(dt), n - 1
        self.coef = np.ascontiguousarray(coef)

    @classmethod
    def from_samples(cls, s):
        return cls(s.t0, s.dt, s.x, s.ltt)

    def state(self, t_abs):
        """Positions [3][3] and light times [6] at absolute time t_abs."""
        x9 = np.empty(9)
        L6 = np.empty(6)
        lib().orc_orbit_state(self.dt, self.nseg, _p(self.coef), float(t_abs - self.t0),
                              _p(x9), _p(L6))
        return x9.reshape(3, 3), L6


def sky_basis(lam, beta):
    """(k, u, v) of Sec. IV.A as three 3-vectors."""
    k, u, v = np.empty(3), np.empty(3), np.empty(3)
    lib().orc_sky_basis(float(lam), float(beta), _p(k), _p(u), _p(v))
    return k, u, v


def _idx(ix, n):
    if ix is None:
        ix = np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(np.asarray(ix, dtype=np.int64))


# ---------------------------------------------------------------------------
# Interpolation (Sec. IV.E)
# ---------------------------------------------------------------------------

def lagrange_weights(order, eps):
    w = np.empty(order + 1)
    lib().orc_lagrange_weights(int(order), float(eps), _p(w))
    return w


def interp(f, order, j0, eps):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = ctypes.c_double()
    st = lib().orc_interp(_p(f), f.size, int(order), int(j0), float(eps), ctypes.byref(out))
    if st:
        raise IndexError("stencil outside the series")
    return out.value


# ---------------------------------------------------------------------------
# Projection (Sec. IV.B) and TDI (Sec. IV.C)
# ---------------------------------------------------------------------------

def project_links(orb: Orbits, t0_h, dt, hp, hc, lam, beta, order, q=None):
    """y[6][len(q)] at h-indices q (default: every index of h).

    h[j] sits at absolute time t0_h + j*dt; orbit quantities at reception
    time t0_h + q*dt."""
    hp = np.ascontiguousarray(hp, dtype=np.float64)
    hc = np.ascontiguousarray(hc, dtype=np.float64)
    q = _idx(q, hp.size)
    y = np.empty((6, q.size))
    st = lib().orc_project(orb.dt, orb.nseg, _p(orb.coef), float(t0_h - orb.t0), float(dt),
                           _p(hp), _p(hc), hp.size, float(lam), float(beta), int(order),
                           _p(q, ctypes.c_int64), q.size, _p(y))
    if st:
        raise IndexError("projection stencil outside h (status %d)" % st)
    return y


def _term_arrays(generation):
    terms = tdi_terms.michelson_terms(generation)
    chan = np.array([t.channel for t in terms], dtype=np.int32)
    sign = np.array([t.sign for t in terms], dtype=np.int32)
    link = np.array([t.link for t in terms], dtype=np.int32)
    plen = np.array([len(t.path) for t in terms], dtype=np.int32)
    path = np.zeros((len(terms), 8), dtype=np.int32)
    for i, t in enumerate(terms):
        path[i, :len(t.path)] = t.path
    return len(terms), chan, sign, link, plen, np.ascontiguousarray(path)


def tdi_xyz(orb: Orbits, t0_y, dt, y, generation, order, p=None):
    """X, Y, Z [3][len(p)] at y-indices p; y[l][j] sits at t0_y + j*dt."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    n_y = y.shape[1]
    p = _idx(p, n_y)
    nt, chan, sign, link, plen, path = _term_arrays(generation)
    out = np.empty((3, p.size))
    i32 = ctypes.c_int32
    st = lib().orc_tdi(orb.dt, orb.nseg, _p(orb.coef), float(t0_y - orb.t0), float(dt), _p(y),
                       n_y, int(order), nt, _p(chan, i32), _p(sign, i32), _p(link, i32),
                       _p(plen, i32), _p(path, i32), _p(p, ctypes.c_int64), p.size, _p(out))
    if st:
        raise IndexError("TDI stencil outside y (status %d)" % st)
    return out


def aet(xyz):
    """A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3 (Sec. IV.C)."""
    X, Y, Z = xyz
    return np.stack([(Z - X) / math.sqrt(2.0), (X - 2.0 * Y + Z) / math.sqrt(6.0),
                     (X + Y + Z) / math.sqrt(3.0)])


def aet_transpose(g):
    """Transpose of ``aet``: gradient w.r.t. X, Y, Z from gradient w.r.t. A, E, T."""
    gA, gE, gT = g
    s2, s6, s3 = math.sqrt(2.0), math.sqrt(6.0), math.sqrt(3.0)
    return np.stack([-gA / s2 + gE / s6 + gT / s3,
                     -2.0 * gE / s6 + gT / s3,
                     gA / s2 + gE / s6 + gT / s3])


def response(orb_proj: Orbits, orb_tdi: Orbits, grid, hp, hc, lam, beta, order, generation,
             channels="XYZ", out_idx=None):
    """Full response of one template on a ``TemplateGrid``: projection on the
    whole y range, then TDI at the output samples (default: all of them).
    Returns [3][len(out_idx)]."""
    y = project_links(orb_proj, grid.t0_h, grid.dt, hp, hc, lam, beta, order,
                      np.arange(grid.y_start, grid.y_start + grid.n_y))
    if out_idx is None:
        out_idx = np.arange(grid.n_out)
    p = np.asarray(out_idx, dtype=np.int64) + grid.front_tdi
    t0_y = grid.t0_h + grid.y_start * grid.dt
    xyz = tdi_xyz(orb_tdi, t0_y, grid.dt, y, generation, order, p)
    return select_channels(xyz, channels)


def select_channels(xyz, channels):
    """X,Y,Z ("XYZ"), A,E,T ("AET") or both stacked ("XYZAET")."""
    if channels == "XYZ":
        return xyz
    if channels == "AET":
        return aet(xyz)
    if channels == "XYZAET":
        return np.concatenate([xyz, aet(xyz)])
    raise ValueError(channels)


# ---------------------------------------------------------------------------
# Adjoints
# ---------------------------------------------------------------------------

def tdi_adjoint(orb: Orbits, t0_y, dt, n_y, generation, order, p, g_xyz):
    p = _idx(p, n_y)
    nt, chan, sign, link, plen, path = _term_arrays(generation)
    g_xyz = np.ascontiguousarray(g_xyz, dtype=np.float64).reshape(3, p.size)
    g_y = np.zeros((6, n_y))
    i32 = ctypes.c_int32
    st = lib().orc_tdi_adjoint(orb.dt, orb.nseg, _p(orb.coef), float(t0_y - orb.t0), float(dt),
                               int(n_y), int(order), nt, _p(chan, i32), _p(sign, i32),
                               _p(link, i32), _p(plen, i32), _p(path, i32),
                               _p(p, ctypes.c_int64), p.size, _p(g_xyz), _p(g_y))
    if st:
        raise IndexError("TDI adjoint stencil outside y")
    return g_y


def project_adjoint(orb: Orbits, t0_h, dt, n_h, lam, beta, order, q, g_y):
    q = _idx(q, n_h)
    g_y = np.ascontiguousarray(g_y, dtype=np.float64).reshape(6, q.size)
    g_hp = np.zeros(n_h)
    g_hc = np.zeros(n_h)
    st = lib().orc_project_adjoint(orb.dt, orb.nseg, _p(orb.coef), float(t0_h - orb.t0),
                                   float(dt), int(n_h), float(lam), float(beta), int(order),
                                   _p(q, ctypes.c_int64), q.size, _p(g_y), _p(g_hp), _p(g_hc))
    if st:
        raise IndexError("projection adjoint stencil outside h")
    return g_hp, g_hc


def response_adjoint(orb_proj, orb_tdi, grid, lam, beta, order, generation, g_out,
                     channels="XYZ"):
    """Transpose of ``response`` w.r.t. (h+, hx) for a full-length output."""
    g = np.asarray(g_out, dtype=np.float64)
    if channels == "AET":
        g = aet_transpose(g)
    elif channels == "XYZAET":
        g = g[:3] + aet_transpose(g[3:])
    p = np.arange(grid.n_out) + grid.front_tdi
    t0_y = grid.t0_h + grid.y_start * grid.dt
    g_y = tdi_adjoint(orb_tdi, t0_y, grid.dt, grid.n_y, generation, order, p, g)
    q = np.arange(grid.y_start, grid.y_start + grid.n_y)
    return project_adjoint(orb_proj, grid.t0_h, grid.dt, grid.n_h, lam, beta, order, q, g_y)


# ---------------------------------------------------------------------------
# White-noise likelihood (Sec. II.A, eq. like; channel sum of Sec. IV.C)
# ---------------------------------------------------------------------------

def loglike(h, d, sigma):
    """-1/2 sum_ch sum_t (d - h)^2 / sigma^2, exactly rounded sum."""
    r = (np.asarray(d, dtype=np.float64) - np.asarray(h, dtype=np.float64)) / sigma
    return -0.5 * math.fsum((r * r).ravel().tolist())


def loglike_difference(h1, h0, d, sigma):
    """logL(h1) - logL(h0) = -1/2 sum (h0 - h1)(2d - h1 - h0) / sigma^2,
    avoiding the cancellation against <d|d>."""
    h1 = np.asarray(h1, dtype=np.float64)
    h0 = np.asarray(h0, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    terms = (h0 - h1) * (2.0 * d - h1 - h0) / (sigma * sigma)
    return -0.5 * math.fsum(terms.ravel().tolist())
