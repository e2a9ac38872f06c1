"""Galactic-binary polarisations (Sec. III) and their vector-Jacobian
product with respect to the eight source parameters (plain CPU oracle; test
infrastructure only, like the rest of ``oracle``).

  Phi(t) = 2 pi (f0 t + fdot t^2 / 2 + fddot t^3 / 6) + phi0,
  fddot = 11 fdot^2 / (3 f0),
  a+ = -(1 + cos^2 iota) A cos Phi,  ax = -2 cos(iota) A sin Phi,
  h+ = cos(2 psi) a+ - sin(2 psi) ax,  hx = sin(2 psi) a+ + cos(2 psi) ax.

The phase is accumulated in extended precision (NumPy longdouble, 64-bit
mantissa on x86-64) and reduced by whole cycles before the trigonometric
functions, so its rounding stays ~1e-13 rad over a year (plain FP64 would
leave ~1e-10 rad).  The vector-Jacobian product uses PyTorch's CPU autograd
on the same formulas, with the phase value replaced by the accurate one
(the derivatives of the phase are exact either way).
"""
from __future__ import annotations

import math

import numpy as np


def phase(params, t):
    """Phi(t) in radians, reduced by whole cycles (float64)."""
    A, f0, fdot, phi0 = (np.longdouble(params[k]) for k in (0, 1, 2, 3))
    t = np.asarray(t, dtype=np.longdouble)
    fddot = np.longdouble(11) / 3 * fdot * fdot / f0
    cyc = f0 * t + fdot * t * t / 2 + fddot * t * t * t / 6
    frac = cyc - np.rint(cyc)
    return (2 * np.longdouble(math.pi) * frac).astype(np.float64) + float(params[3])


def polarizations(params, t):
    """(h+, hx) at times t for params (A, f0, fdot, phi0, iota, psi, lam, beta)."""
    A, iota, psi = float(params[0]), float(params[4]), float(params[5])
    ph = phase(params, t)
    ci = math.cos(iota)
    ap = -(1.0 + ci * ci) * A * np.cos(ph)
    ac = -2.0 * ci * A * np.sin(ph)
    c2, s2 = math.cos(2 * psi), math.sin(2 * psi)
    return c2 * ap - s2 * ac, s2 * ap + c2 * ac


def polarizations_vjp(params, t, g_hp, g_hc):
    """d/dparams of sum_j (g_hp[j] h+(t_j) + g_hc[j] hx(t_j)), length 8."""
    import torch
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    tt = torch.tensor(np.asarray(t, dtype=np.float64))
    A, f0, fdot, phi0, iota, psi = (p[k] for k in range(6))
    fddot = 11.0 / 3.0 * fdot * fdot / f0
    ph64 = 2 * math.pi * (f0 * tt + fdot * tt * tt / 2 + fddot * tt * tt * tt / 6) + phi0
    acc = torch.tensor(phase(params, t))
    ph = acc + (ph64 - ph64.detach())          # accurate value, exact derivatives
    ci = torch.cos(iota)
    ap = -(1.0 + ci * ci) * A * torch.cos(ph)
    ac = -2.0 * ci * A * torch.sin(ph)
    c2, s2 = torch.cos(2 * psi), torch.sin(2 * psi)
    hp, hc = c2 * ap - s2 * ac, s2 * ap + c2 * ac
    L = (torch.tensor(np.asarray(g_hp, dtype=np.float64)) * hp).sum() + \
        (torch.tensor(np.asarray(g_hc, dtype=np.float64)) * hc).sum()
    L.backward()
    return p.grad.numpy().copy()
