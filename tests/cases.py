"""Test helpers: the seeded workloads (re-exported from the package), sampled
oracle evaluation and the parity error measure."""
from __future__ import annotations

import numpy as np

from paper_2204_06633_amd.workloads import Case, day_case, make_case, year_case  # noqa: F401


def sample_indices(n, k, seed, edge=8):
    """``k`` random indices of [0, n) plus the first and last ``edge``."""
    rng = np.random.default_rng(seed)
    mid = rng.choice(n, size=min(k, n), replace=False)
    idx = np.unique(np.concatenate([np.arange(min(edge, n)), np.arange(max(n - edge, 0), n), mid]))
    return idx.astype(np.int64)


def rel_err(got, ref):
    """Relative L2 error of a template's output, taken jointly over its
    channels: ||got - ref||_F / ||ref||_F.

    Per-channel normalisation is ill-posed for T (and for any channel that
    nearly cancels): its norm is ~(omega L)^2 below A and E, so a 1e-16
    perturbation of the orbits already moves it by ~1e-11 of its own norm."""
    got = np.atleast_2d(np.asarray(got, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def oracle_sampled_response(orb_p, orb_t, case, out_idx):
    """Oracle response at selected output samples: the link series is computed
    only where the TDI stencils of those samples read it (elsewhere NaN, so a
    stray read would show)."""
    import oracle
    g = case.grid
    half = (case.order + 1) // 2
    need = set()
    for p in np.asarray(out_idx) + g.front_tdi:
        need.update(range(max(p - g.front_tdi, 0), min(p + half + 2, g.n_y)))
    need = np.array(sorted(need), dtype=np.int64)
    y = np.full((6, g.n_y), np.nan)
    y[:, need] = oracle.project_links(orb_p, g.t0_h, g.dt, case.hp, case.hc, case.lam, case.beta,
                                      case.order, need + g.y_start)
    t0_y = g.t0_h + g.y_start * g.dt
    xyz = oracle.tdi_xyz(orb_t, t0_y, g.dt, y, case.generation, case.order,
                         np.asarray(out_idx) + g.front_tdi)
    return oracle.select_channels(xyz, case.channels)
