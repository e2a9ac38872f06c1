"""The oracle at selected output samples of a long template (test
infrastructure, like the rest of ``oracle``).

Full-size workloads (one year, millions of samples) are compared on sampled
outputs: each sampled output is computed by the oracle on its own, from the
link samples its TDI stencils read and nothing else.

  sampled_response  forward (Sec. IV.B then Sec. IV.C) at output indices;
  sampled_adjoint   the transpose of the response applied to a channel
                    gradient that is zero except at sampled outputs: the TDI
                    scatter of those outputs (transposes of eqs. tdi1/tdi2)
                    followed by the projection scatter of the link samples
                    it reaches (transpose of the Sec. IV.B interpolations).
"""
from __future__ import annotations

import numpy as np

from . import aet_transpose, project_adjoint, project_links, select_channels, tdi_adjoint, tdi_xyz


def _links_needed(case, out_idx):
    """y-indices that the TDI stencils of the outputs out_idx read (the
    grid's TDI padding bounds every delay chain and half stencil)."""
    g = case.grid
    half = (case.order + 1) // 2
    need = set()
    for p in np.asarray(out_idx) + g.front_tdi:
        need.update(range(max(p - g.front_tdi, 0), min(p + half + 2, g.n_y)))
    return np.array(sorted(need), dtype=np.int64)


def sampled_response(orb_p, orb_t, case, out_idx):
    """Channels [rows][len(out_idx)] of one template at the output indices
    out_idx.  The link series is evaluated only where those outputs' stencils
    read it; elsewhere it is NaN, so a stray read shows."""
    g = case.grid
    need = _links_needed(case, out_idx)
    y = np.full((6, g.n_y), np.nan)
    y[:, need] = project_links(orb_p, g.t0_h, g.dt, case.hp, case.hc, case.lam, case.beta,
                               case.order, need + g.y_start)
    t0_y = g.t0_h + g.y_start * g.dt
    xyz = tdi_xyz(orb_t, t0_y, g.dt, y, case.generation, case.order,
                  np.asarray(out_idx) + g.front_tdi)
    return select_channels(xyz, case.channels)


def sampled_adjoint(orb_p, orb_t, case, out_idx, g_sel):
    """(g_hp, g_hc), each [n_h], for the channel gradient g_out that equals
    g_sel [rows][len(out_idx)] at the outputs out_idx and zero elsewhere."""
    g = case.grid
    gs = np.asarray(g_sel, dtype=np.float64)
    if case.channels == "AET":
        gx = aet_transpose(gs)
    elif case.channels == "XYZAET":
        gx = gs[:3] + aet_transpose(gs[3:])
    else:
        gx = gs
    p = np.asarray(out_idx, dtype=np.int64) + g.front_tdi
    t0_y = g.t0_h + g.y_start * g.dt
    g_y = tdi_adjoint(orb_t, t0_y, g.dt, g.n_y, case.generation, case.order, p, gx)
    q = np.flatnonzero(np.any(g_y != 0.0, axis=0)).astype(np.int64)
    return project_adjoint(orb_p, g.t0_h, g.dt, g.n_h, case.lam, case.beta, case.order,
                           q + g.y_start, g_y[:, q])
