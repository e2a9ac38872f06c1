"""Frequency-domain, noise-weighted likelihood (plain CPU FP64 oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the product path never
imports it, and it shares no code with the HIP library.

Follows Sec. II.A of arXiv:2204.06633: the inner product of two real time
series is four times the real part of the integral over positive frequencies
of conj(a~) b~ / S_n (Eq. for the noise-weighted inner product); the
log-likelihood is -1/2 <d - h|d - h> summed over the A, E, T channels; the
optimal SNR is sqrt(<h|h>), the extraction SNR <d|h> / sqrt(<h|h>), and
with noise-free data s the overlap is <s|h> / sqrt(<h|h><s|s>) and the
mismatch one minus it.

Discretisation (the paper states the continuous form only):
  * a~(f_k) = dt * sum_{n<N} a_n exp(-2 pi i k n / N), the series zero-padded
    to N = n_fft samples, f_k = k / (N dt), k = 0 .. N/2;
  * the integral becomes sum_{k=0}^{N/2} w_k Re(conj(a~_k) b~_k) with
    w_k = 4 df / S_n(f_k), df = 1 / (N dt); the caller supplies w (zero for
    excluded bins) so that the noise model stays outside the method;
  * d logL / d h_n = dt * sum_{k=0}^{N/2} w_k Re(r~_k exp(+2 pi i k n / N)),
    r = d - h: the derivative of the quadratic form above, term by term.

NumPy's FFT serves as the DFT; sums are exactly rounded (math.fsum).
"""
from __future__ import annotations

import math

import numpy as np


def spectrum(a, dt, n_fft):
    """a~_k = dt * DFT_N(a zero-padded to n_fft)_k for k = 0 .. n_fft/2."""
    a = np.asarray(a, dtype=np.float64)
    if a.shape[-1] > n_fft:
        raise ValueError("series longer than n_fft")
    return dt * np.fft.rfft(a, n=n_fft)


def inner(a, b, w, dt, n_fft):
    """<a|b> = sum_{k=0}^{N/2} w_k Re(conj(a~_k) b~_k)."""
    A = spectrum(a, dt, n_fft)
    B = spectrum(b, dt, n_fft)
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (n_fft // 2 + 1,)
    terms = w * (A.real * B.real + A.imag * B.imag)
    return math.fsum(terms.tolist())


def channel_weights(w_ae, w_t, n_channels):
    """Weights per channel: A and E share one noise curve, T has its own."""
    return [w_ae, w_ae, w_t][:n_channels]


def loglike(h, d, w_ae, w_t, dt, n_fft):
    """Statistics of template h against data d, both [C][n] with channels
    A, E (and T when C = 3).

    Returns a dict with rr = <d-h|d-h>, hh = <h|h>, dh = <d|h> summed over
    the channels, loglike = -rr/2, rho_opt = sqrt(hh), rho_ex = dh/sqrt(hh).
    """
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    ws = channel_weights(w_ae, w_t, h.shape[0])
    rr = math.fsum(inner(d[c] - h[c], d[c] - h[c], ws[c], dt, n_fft) for c in range(h.shape[0]))
    hh = math.fsum(inner(h[c], h[c], ws[c], dt, n_fft) for c in range(h.shape[0]))
    dh = math.fsum(inner(d[c], h[c], ws[c], dt, n_fft) for c in range(h.shape[0]))
    rho_opt = math.sqrt(hh)
    return {"rr": rr, "hh": hh, "dh": dh, "loglike": -0.5 * rr, "rho_opt": rho_opt,
            "rho_ex": dh / rho_opt if rho_opt > 0 else 0.0}


def overlap(h, s, w_ae, w_t, dt, n_fft):
    """Diagnostics of template h against noise-free data s (Sec. II.A):
    optimal SNR sqrt(<h|h>), extraction SNR <s|h>/sqrt(<h|h>), overlap
    <s|h>/sqrt(<h|h><s|s>) and mismatch 1 - overlap, inner products summed
    over the channels."""
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    ws = channel_weights(w_ae, w_t, h.shape[0])
    hh = math.fsum(inner(h[c], h[c], ws[c], dt, n_fft) for c in range(h.shape[0]))
    ss = math.fsum(inner(s[c], s[c], ws[c], dt, n_fft) for c in range(h.shape[0]))
    sh = math.fsum(inner(s[c], h[c], ws[c], dt, n_fft) for c in range(h.shape[0]))
    ov = sh / math.sqrt(hh * ss)
    return {"rho_opt": math.sqrt(hh), "rho_ex": sh / math.sqrt(hh), "overlap": ov,
            "mismatch": 1.0 - ov}


def loglike_grad(h, d, w_ae, w_t, dt, n_fft):
    """d logL / d h, same shape as h (see the module docstring)."""
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    n = h.shape[-1]
    ws = channel_weights(w_ae, w_t, h.shape[0])
    g = np.empty_like(h)
    for c in range(h.shape[0]):
        R = spectrum(d[c] - h[c], dt, n_fft) * np.asarray(ws[c], dtype=np.float64)
        full = np.zeros(n_fft, dtype=np.complex128)
        full[: n_fft // 2 + 1] = R
        # sum_{k=0}^{N/2} R_k exp(+2 pi i k n / N) = N * ifft(full)_n
        g[c] = dt * (n_fft * np.fft.ifft(full)).real[:n]
    return g


def inner_bruteforce(a, b, w, dt, n_fft):
    """<a|b> with the DFT written out as a double loop (tiny inputs only)."""
    a = [float(x) for x in a] + [0.0] * (n_fft - len(a))
    b = [float(x) for x in b] + [0.0] * (n_fft - len(b))
    total = []
    for k in range(n_fft // 2 + 1):
        ar = ai = br = bi = 0.0
        for n in range(n_fft):
            ang = -2.0 * math.pi * ((k * n) % n_fft) / n_fft
            c, s = math.cos(ang), math.sin(ang)
            ar += a[n] * c
            ai += a[n] * s
            br += b[n] * c
            bi += b[n] * s
        total.append(float(w[k]) * dt * dt * (ar * br + ai * bi))
    return math.fsum(total)


def loglike_grad_bruteforce(h, d, w, dt, n_fft):
    """d(-1/2 <d-h|d-h>)/dh_n for one channel by the explicit double sum."""
    h = [float(x) for x in h]
    d = [float(x) for x in d]
    n = len(h)
    r = [d[i] - h[i] for i in range(n)] + [0.0] * (n_fft - n)
    spec = []
    for k in range(n_fft // 2 + 1):
        re = im = 0.0
        for m in range(n_fft):
            ang = -2.0 * math.pi * ((k * m) % n_fft) / n_fft
            re += r[m] * math.cos(ang)
            im += r[m] * math.sin(ang)
        spec.append((dt * re, dt * im))
    g = []
    for i in range(n):
        acc = []
        for k in range(n_fft // 2 + 1):
            ang = 2.0 * math.pi * ((k * i) % n_fft) / n_fft
            acc.append(float(w[k]) * (spec[k][0] * math.cos(ang) - spec[k][1] * math.sin(ang)))
        g.append(dt * math.fsum(acc))
    return np.array(g)
