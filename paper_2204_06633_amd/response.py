"""Per-template response on the GPU and its autograd wrappers.

Thin glue over the C-ABI calls: lr_project_links then lr_tdi_combine forward,
lr_tdi_adjoint then lr_project_adjoint backward, lr_loglike for the
white-noise likelihood and lr_fd_loglike for the noise-weighted
frequency-domain one.  All arithmetic runs in the HIP kernels.  The index
bookkeeping follows ``inputs.TemplateGrid``: h on [0, n_h), links on
[y_start, y_start + n_y), output on [out_start, out_start + n_out) of the same
uniform grid.
"""
from __future__ import annotations

import dataclasses

import torch

from . import native


@dataclasses.dataclass
class Template:
    """Everything a response call needs besides h+, hx and the sky angles."""
    orb_proj: native.Orbits
    orb_tdi: native.Orbits
    grid: object                 # inputs.TemplateGrid
    order: int = 25
    generation: int = 2
    channels: str = "XYZ"

    @property
    def t0_y(self):
        return self.grid.t0_h + self.grid.y_start * self.grid.dt


def plain_forward(tpl: Template, hp, hc, sky, y=None, out=None, stream=None):
    """Returns (out[3 or 6][n_out], y[6][n_y]) for one template."""
    g = tpl.grid
    y = native.project_links(tpl.orb_proj, g.t0_h, g.dt, hp, hc, sky, tpl.order, g.y_start,
                             g.n_y, y=y, stream=stream)
    out = native.tdi_combine(tpl.orb_tdi, tpl.t0_y, g.dt, y, tpl.generation, tpl.order,
                             tpl.channels, g.front_tdi, g.n_out, out=out, stream=stream)
    return out, y


def plain_adjoint(tpl: Template, hp, hc, sky, g_out, want_sky=True, stream=None):
    """Transpose of ``plain_forward``: (g_hp, g_hc, g_sky)."""
    g = tpl.grid
    g_y = native.tdi_adjoint(tpl.orb_tdi, tpl.t0_y, g.dt, g.n_y, tpl.generation, tpl.order,
                             tpl.channels, g.front_tdi, g_out, stream=stream)
    return native.project_adjoint(tpl.orb_proj, g.t0_h, g.dt, g.n_h, hp, hc, sky, tpl.order,
                                  g.y_start, g_y, want_sky=want_sky, stream=stream)


class ResponseFn(torch.autograd.Function):
    """out = R(h+, hx; lam, beta) with the hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx, hp, hc, sky, tpl):
        hp, hc, sky = hp.contiguous(), hc.contiguous(), sky.contiguous()
        out, _ = plain_forward(tpl, hp, hc, sky)
        ctx.save_for_backward(hp, hc, sky)
        ctx.tpl = tpl
        return out

    @staticmethod
    def backward(ctx, g_out):
        hp, hc, sky = ctx.saved_tensors
        g_hp, g_hc, g_sky = plain_adjoint(ctx.tpl, hp, hc, sky, g_out.contiguous(),
                                          want_sky=ctx.needs_input_grad[2])
        return g_hp, g_hc, g_sky, None


class LoglikeFn(torch.autograd.Function):
    """-1/2 sum (data - h)^2 / sigma^2 with gradient (data - h)/sigma^2."""

    @staticmethod
    def forward(ctx, h, data, sigma):
        ll, g = native.loglike(h.contiguous(), data.contiguous(), sigma,
                               want_grad=ctx.needs_input_grad[0])
        ctx.save_for_backward(g if g is not None else torch.empty(0, device=h.device))
        return ll[0]

    @staticmethod
    def backward(ctx, g_ll):
        (g,) = ctx.saved_tensors
        return g * g_ll, None, None


def response(tpl: Template, hp, hc, sky):
    return ResponseFn.apply(hp, hc, sky, tpl)


def loglike(h, data, sigma):
    return LoglikeFn.apply(h, data, sigma)


class FdLoglikeFn(torch.autograd.Function):
    """log L = -<d - h|d - h>/2 of the frequency-domain likelihood
    (lr_fd_loglike) for h [C][n] or [B][C][n]; backward returns
    g_ll * d log L / d h from the same call."""

    @staticmethod
    def forward(ctx, h, plan):
        h = h.contiguous()
        want = ctx.needs_input_grad[0]
        stats, g = plan.loglike(h, want_grad=want)
        ctx.save_for_backward(g if want else torch.empty(0, device=h.device))
        ll = -0.5 * stats[:, 0]
        return ll[0] if h.dim() == 2 else ll

    @staticmethod
    def backward(ctx, g_ll):
        (g,) = ctx.saved_tensors
        if g.dim() == 3:
            return g * g_ll.view(-1, 1, 1), None
        return g * g_ll, None


def fd_loglike(h, plan):
    return FdLoglikeFn.apply(h, plan)


class GbPolarizationsFn(torch.autograd.Function):
    """(h+, hx) [n][n_h] of Galactic binaries (lr_gb_polarizations) for
    params [n][8] on t_j = (k0 + j) dt; backward: lr_gb_polarizations_adjoint."""

    @staticmethod
    def forward(ctx, params, k0, n_h, dt):
        params = params.contiguous()
        hp, hc = native.gb_polarizations(params, k0, n_h, dt)
        ctx.save_for_backward(params)
        ctx.k0, ctx.dt = k0, dt
        return hp, hc

    @staticmethod
    def backward(ctx, g_hp, g_hc):
        (params,) = ctx.saved_tensors
        if g_hp is None:
            g_hp = torch.zeros_like(g_hc)
        if g_hc is None:
            g_hc = torch.zeros_like(g_hp)
        g = native.gb_polarizations_adjoint(params, ctx.k0, ctx.dt, g_hp.contiguous(),
                                            g_hc.contiguous())
        return g, None, None, None


def gb_polarizations(params, k0, n_h, dt):
    return GbPolarizationsFn.apply(params, k0, n_h, dt)
