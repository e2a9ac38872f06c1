"""Orbit-approximation tooling (Sec. IV.D and V).

* ``eq_positions``: the equal-armlength configuration, a function of its two
  free parameters (lam1, m1): the longitude of periastron and the initial
  mean anomaly of spacecraft 1 (spacecraft k's periastron at lam1 - 2 pi k
  / 3, all sharing one mean longitude).  It is the Keplerian motion to first
  order in the eccentricity e = L / (2 sqrt(3) a): about the guiding centre
  a (cos alpha, sin alpha, 0), alpha = Omega t + lam1 + m1, spacecraft k is
  displaced by a e (-cos M_k, 2 sin M_k, sqrt(3) cos M_k) in the (radial,
  along-track, ecliptic-normal) frame, M_k its mean anomaly.  At this order
  the triangle is rigid: armlength L exactly, plane at 60 degrees.
* ``fit_eq_orbits``: (lam1, m1) minimising the sum over spacecraft of the
  time-integrated distance |x_i^EQ(t) - x_i^true(t)| (trapezoidal rule on a
  uniform grid) by Nelder-Mead, as Sec. IV.D does against the accurate
  orbits.
* ``configurations``: the four orbit pairings of Sec. V for (projection,
  TDI): ESA, EQ, ESAEQ and EQESA, "ESA" standing for the accurate orbits.
* ``fitting_factor``: the Sec. II.A fitting factor, the overlap between the
  data and the template at the maximum of the likelihood, the maximum found
  by Nelder-Mead in the sampling coordinates from a starting point (the
  paper finds it with its sampler); ``TemplateScorer`` evaluates one
  template on the GPU (HIP polarisations, response with any orbit pairing,
  frequency-domain statistics against the data).

Host code: orbit fitting runs once per analysis, on coarse orbit samples.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs


def eq_positions(t, lam1, m1, L=inputs.L_ARM, a=inputs.AU):
    """Positions [len(t)][3][3] (m) of the equal-armlength configuration."""
    t = np.asarray(t, dtype=np.float64)
    e = L / (2.0 * math.sqrt(3.0) * a)
    alpha = 2.0 * math.pi / inputs.YEAR * t + lam1 + m1
    ca, sa = np.cos(alpha), np.sin(alpha)
    out = np.empty(t.shape + (3, 3))
    for k in range(3):
        M = alpha - (lam1 - 2.0 * math.pi * k / 3.0)
        dr, dt_, dz = -a * e * np.cos(M), 2.0 * a * e * np.sin(M), math.sqrt(3.0) * a * e * np.cos(M)
        out[..., k, 0] = (a + dr) * ca - dt_ * sa
        out[..., k, 1] = (a + dr) * sa + dt_ * ca
        out[..., k, 2] = dz
    return out


def eq_cost(params, t, x_true, L=inputs.L_ARM, a=inputs.AU):
    """Sum over spacecraft of the integral over t of |x_i^EQ - x_i^true|
    (metre seconds), trapezoidal on the grid ``t``."""
    lam1, m1 = params
    d = np.linalg.norm(eq_positions(t, lam1, m1, L, a) - x_true, axis=-1)   # [n][3]
    dt = np.diff(t)
    return float(np.sum(0.5 * (d[1:] + d[:-1]) * dt[:, None]))


def fit_eq_orbits(t, x_true, x0=(0.0, 0.0), L=inputs.L_ARM, a=inputs.AU, xatol=1e-10,
                  fatol=1e-3, maxiter=4000):
    """Nelder-Mead fit of (lam1, m1) to true positions x_true [len(t)][3][3].

    Returns (lam1, m1, cost)."""
    from scipy.optimize import minimize
    res = minimize(eq_cost, np.asarray(x0, dtype=np.float64), args=(t, x_true, L, a),
                   method="Nelder-Mead",
                   options={"xatol": xatol, "fatol": fatol, "maxiter": maxiter,
                            "initial_simplex": np.asarray(x0) + np.array([[0, 0], [1e-2, 0],
                                                                          [0, 1e-2]])})
    lam1, m1 = (float(v) for v in res.x)
    return lam1, m1, float(res.fun)


def eq_orbit_samples(t_begin, t_end, lam1, m1, **kw):
    """Coarse samples (positions and light times) of the equal-armlength
    configuration over [t_begin, t_end]."""
    return inputs.make_orbit_samples("function", t_begin, t_end,
                                     fn=lambda tt: eq_positions(tt, lam1, m1), **kw)


def configurations(accurate, equal_arm):
    """(projection orbits, TDI orbits) for the orbit models of Sec. V: the
    accurate orbits ("ESA"), the equal-armlength ones ("EQ"), and the two
    hybrids "ESAEQ" (accurate projection, equal-armlength TDI) and "EQESA"."""
    return {"ESA": (accurate, accurate), "EQ": (equal_arm, equal_arm),
            "ESAEQ": (accurate, equal_arm), "EQESA": (equal_arm, accurate)}


def overlap_statistics(stats, ss):
    """Sec. II.A diagnostics from the frequency-domain statistics of templates
    against noise-free data s: ``stats`` [..., 3] = (<s-h|s-h>, <h|h>, <s|h>)
    as lr_fd_loglike returns them, ``ss`` = <s|s>.  Returns a dict of arrays:
    optimal SNR sqrt(<h|h>), extraction SNR <s|h>/sqrt(<h|h>), overlap
    rho_ex / sqrt(<s|s>) and mismatch 1 - overlap."""
    st = np.asarray(stats, dtype=np.float64)
    hh, sh = st[..., 1], st[..., 2]
    rho_opt = np.sqrt(hh)
    rho_ex = sh / rho_opt
    overlap = rho_ex / math.sqrt(ss)
    return {"rho_opt": rho_opt, "rho_ex": rho_ex, "overlap": overlap, "mismatch": 1.0 - overlap,
            "loglike": -0.5 * st[..., 0]}


def fitting_factor(score, theta0, step, maxfev=4000, xatol=1e-12, fatol=1e-10):
    """Fitting factor (Sec. II.A): maximise the log-likelihood over the
    template parameters, then report the overlap there.

    ``score(theta) -> (loglike, overlap)`` for one parameter vector;
    ``theta0``: start (e.g. the injection); ``step``: the initial simplex
    edge per parameter.  Returns dict(theta, loglike, fitting_factor,
    loglike_start, overlap_start, nfev)."""
    from scipy.optimize import minimize
    theta0 = np.asarray(theta0, dtype=np.float64)
    step = np.asarray(step, dtype=np.float64)
    cache = {}

    def neg(th):
        key = tuple(np.asarray(th, dtype=np.float64))
        if key not in cache:
            cache[key] = score(np.asarray(th, dtype=np.float64))
        ll = cache[key][0]
        return -ll if np.isfinite(ll) else np.inf

    ll0, ov0 = score(theta0)
    simplex = np.vstack([theta0] + [theta0 + step[i] * np.eye(len(theta0))[i]
                                    for i in range(len(theta0))])
    res = minimize(neg, theta0, method="Nelder-Mead",
                   options={"maxfev": maxfev, "xatol": xatol, "fatol": fatol,
                            "initial_simplex": simplex, "adaptive": True})
    best = np.asarray(res.x, dtype=np.float64)
    if -res.fun < ll0:                     # the start is never worse than the result
        best = theta0
    ll, ov = score(best)
    return {"theta": best, "loglike": float(ll), "fitting_factor": float(ov),
            "loglike_start": float(ll0), "overlap_start": float(ov0), "nfev": int(res.nfev)}


class TemplateScorer:
    """(log L, overlap) of one Galactic-binary template against fixed data on
    the GPU: lr_gb_polarizations -> lr_project_links / lr_tdi_combine (any
    projection and TDI orbits) -> lr_fd_loglike statistics.  ``theta`` in the
    sampler's coordinates (sampler.to_source).  ``ss`` = <s|s> of the data."""

    def __init__(self, orb_proj, orb_tdi, grid, data, w_ae, w_t, order=25, generation=2,
                 device="cuda"):
        import torch

        from . import native, response
        self.torch = torch
        self.tpl = response.Template(orb_proj, orb_tdi, grid, order, generation, "AET")
        self.grid = grid
        self.plan = native.FdPlan(data, w_ae, w_t, grid.dt)
        self.out = torch.empty((3, grid.n_out), dtype=torch.float64, device=device)
        self.y = torch.empty((6, grid.n_y), dtype=torch.float64, device=device)
        self.stats = torch.empty((1, 3), dtype=torch.float64, device=device)
        self.hp = torch.empty((1, grid.n_h), dtype=torch.float64, device=device)
        self.hc = torch.empty_like(self.hp)
        self.device = device
        self.ss = None
        self.stats_of(None)   # <s|s> from a zero template: rr = <s|s>

    def stats_of(self, theta):
        from . import native, response, sampler
        torch = self.torch
        g = self.grid
        if theta is None:
            self.out.zero_()
        else:
            src = sampler.to_source(torch.as_tensor(theta, dtype=torch.float64,
                                                    device=self.device)[None]).contiguous()
            native.gb_polarizations(src, -g.out_start, g.n_h, g.dt, hp=self.hp, hc=self.hc)
            response.plain_forward(self.tpl, self.hp[0], self.hc[0], src[0, 6:8].contiguous(),
                                   y=self.y, out=self.out)
        self.plan.loglike(self.out, want_grad=False, stats=self.stats)
        st = self.stats[0].cpu().numpy()
        if theta is None:
            self.ss = float(st[0])
        return st

    def __call__(self, theta):
        rr, hh, sh = self.stats_of(theta)
        ov = sh / math.sqrt(hh * self.ss) if hh > 0 else 0.0
        return -0.5 * rr, ov
