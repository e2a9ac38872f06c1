"""Per-template forward response on the GPU: projection then TDI.

Thin glue over the two C-ABI calls (lr_project_links, lr_tdi_combine); all
arithmetic runs in the HIP kernels.  The index bookkeeping follows
``inputs.TemplateGrid``: h on [0, n_h), links on [y_start, y_start + n_y),
output on [out_start, out_start + n_out) of the same uniform grid.
"""
from __future__ import annotations

from . import native


def plain_forward(orb_proj: native.Orbits, orb_tdi: native.Orbits, grid, hp, hc, lam, beta,
                  order, generation, channels="XYZ", y=None, out=None, stream=None):
    """Returns (out[3][n_out], y[6][n_y]) for one template."""
    y = native.project_links(orb_proj, grid.t0_h, grid.dt, hp, hc, lam, beta, order,
                             grid.y_start, grid.n_y, y=y, stream=stream)
    t0_y = grid.t0_h + grid.y_start * grid.dt
    out = native.tdi_combine(orb_tdi, t0_y, grid.dt, y, generation, order, channels,
                             grid.front_tdi, grid.n_out, out=out, stream=stream)
    return out, y
