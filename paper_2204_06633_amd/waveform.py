"""Galactic-binary polarisations in PyTorch (Sec. III), differentiable in the
eight source parameters (A, f0, fdot, phi0, iota, psi, lam, beta).

  Phi(t) = 2 pi (f0 t + fdot t^2 / 2 + fddot t^3 / 6) + phi0,
  fddot = 11 fdot^2 / (3 f0),
  h+S = A cos Phi,  hxS = A sin Phi,
  [h+; hx] = R(2 psi) [-(1 + cos^2 iota) h+S; -2 cos(iota) hxS].

This runs as ordinary torch elementwise ops on the GPU (the paper generates
it with CuPy); the response kernels take its output.
"""
from __future__ import annotations

import math

import torch


def gb_polarizations(params, t):
    """``params``: [..., 8] tensor; ``t``: [n] waveform times (s).
    Returns (h+, hx) of shape [..., n]."""
    A, f0, fdot, phi0, iota, psi = (params[..., k:k + 1] for k in range(6))
    fddot = 11.0 / 3.0 * fdot * fdot / f0
    phase = 2.0 * math.pi * (f0 * t + 0.5 * fdot * t * t + fddot * t * t * t / 6.0) + phi0
    hp_s = A * torch.cos(phase)
    hc_s = A * torch.sin(phase)
    ci = torch.cos(iota)
    a_p = -(1.0 + ci * ci) * hp_s
    a_c = -2.0 * ci * hc_s
    c2, s2 = torch.cos(2.0 * psi), torch.sin(2.0 * psi)
    return c2 * a_p - s2 * a_c, s2 * a_p + c2 * a_c
