"""Pins of the frequency-domain likelihood oracle (Sec. II.A) against results
that do not come from the oracle itself: DFTs written out as loops, Parseval's
theorem, the spectrum of a sinusoid on a bin, and the exact Taylor expansion
of a quadratic form."""
import math

import numpy as np
import pytest

from oracle import fd


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("n,n_fft", [(8, 8), (5, 8), (11, 16), (16, 16)])
def test_inner_matches_written_out_dft(n, n_fft):
    rng = _rng(n * 100 + n_fft)
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    w = rng.uniform(0.5, 2.0, n_fft // 2 + 1)       # DC and Nyquist weighted too
    dt = 0.7
    ref = fd.inner_bruteforce(a, b, w, dt, n_fft)
    assert abs(fd.inner(a, b, w, dt, n_fft) - ref) <= 1e-13 * abs(ref) + 1e-14


def test_parseval_flat_weights():
    # w_0 = w_{N/2} = c and 2c elsewhere make the one-sided sum the full
    # two-sided one: <a|a> = c dt^2 N sum a^2 (Parseval).
    rng = _rng(1)
    n_fft, n, dt, c = 1024, 900, 3.0, 0.25
    a = rng.standard_normal(n)
    w = np.full(n_fft // 2 + 1, 2 * c)
    w[0] = w[-1] = c
    ref = c * dt * dt * n_fft * math.fsum((a * a).tolist())
    assert abs(fd.inner(a, a, w, dt, n_fft) - ref) <= 1e-12 * ref


def test_sinusoid_on_a_bin():
    # a_n = A cos(2 pi k0 n / N + phi): a~_{k0} = dt A N/2 e^{i phi} and zero
    # elsewhere; two different bins are orthogonal.
    n_fft, dt, amp, phi = 256, 2.0, 1.5, 0.3
    t = np.arange(n_fft)
    a = amp * np.cos(2 * np.pi * 17 * t / n_fft + phi)
    b = np.sin(2 * np.pi * 40 * t / n_fft)
    w = np.linspace(1.0, 3.0, n_fft // 2 + 1)
    ref = w[17] * (dt * amp * n_fft / 2) ** 2
    assert abs(fd.inner(a, a, w, dt, n_fft) - ref) <= 1e-12 * ref
    assert abs(fd.inner(a, b, w, dt, n_fft)) <= 1e-12 * ref


def test_loglike_statistics():
    rng = _rng(2)
    n_fft, n, dt = 64, 50, 5.0
    d = rng.standard_normal((3, n))
    w_ae = rng.uniform(0, 1, n_fft // 2 + 1)
    w_t = rng.uniform(0, 1, n_fft // 2 + 1)
    s = fd.loglike(d, d, w_ae, w_t, dt, n_fft)          # template equal to the data
    assert s["rr"] == 0.0 and s["loglike"] == 0.0
    assert abs(s["rho_ex"] - s["rho_opt"]) <= 1e-12 * s["rho_opt"]
    h = rng.standard_normal((3, n))
    s = fd.loglike(h, d, w_ae, w_t, dt, n_fft)
    dd = fd.loglike(np.zeros_like(d), d, w_ae, w_t, dt, n_fft)["rr"]
    # <d-h|d-h> = <d|d> + <h|h> - 2 <d|h>
    assert abs(s["rr"] - (dd + s["hh"] - 2 * s["dh"])) <= 1e-12 * (dd + s["hh"])
    # each channel carries its own weights: T with w_t, A and E with w_ae
    t_only = fd.inner(d[2] - h[2], d[2] - h[2], w_t, dt, n_fft)
    ae = sum(fd.inner(d[c] - h[c], d[c] - h[c], w_ae, dt, n_fft) for c in range(2))
    assert abs(s["rr"] - (ae + t_only)) <= 1e-12 * s["rr"]


@pytest.mark.parametrize("n,n_fft", [(7, 8), (12, 16)])
def test_gradient_matches_written_out_sum(n, n_fft):
    rng = _rng(3 + n)
    h, d = rng.standard_normal((1, n)), rng.standard_normal((1, n))
    w = rng.uniform(0.1, 1.0, n_fft // 2 + 1)
    dt = 1.3
    g = fd.loglike_grad(h, d, w, w, dt, n_fft)[0]
    ref = fd.loglike_grad_bruteforce(h[0], d[0], w, dt, n_fft)
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gradient_exact_for_the_quadratic():
    # logL is quadratic in h: the central difference along e equals g . e up
    # to rounding, and the second difference equals -<e|e>.
    rng = _rng(4)
    n_fft, n, dt = 128, 100, 4.0
    h, d = rng.standard_normal((3, n)), rng.standard_normal((3, n))
    e = rng.standard_normal((3, n))
    w_ae = rng.uniform(0, 1, n_fft // 2 + 1)
    w_t = rng.uniform(0, 2, n_fft // 2 + 1)
    g = fd.loglike_grad(h, d, w_ae, w_t, dt, n_fft)
    L = lambda x: fd.loglike(x, d, w_ae, w_t, dt, n_fft)["loglike"]
    t = 0.5
    lp, l0, lm = L(h + t * e), L(h), L(h - t * e)
    assert abs((lp - lm) / (2 * t) - np.sum(g * e)) <= 1e-10 * np.sum(np.abs(g * e))
    ee = fd.loglike(np.zeros_like(e), e, w_ae, w_t, dt, n_fft)["rr"]
    assert abs((lp - 2 * l0 + lm) / t ** 2 + ee) <= 1e-9 * ee


def test_gradient_ignores_padding_and_sign():
    # A plain mistake (exp(-i...) in place of exp(+i...), or r = h - d) flips
    # the directional derivative; the value at lag 0 pins the sign.
    n_fft, n, dt = 32, 32, 1.0
    h = np.zeros((1, n))
    d = np.zeros((1, n))
    d[0, 0] = 1.0
    w = np.ones(n_fft // 2 + 1)
    g = fd.loglike_grad(h, d, w, w, dt, n_fft)[0]
    # r = delta_0: r~_k = dt for every k, g_0 = dt^2 sum_k w_k > 0
    assert abs(g[0] - dt * dt * (n_fft // 2 + 1)) <= 1e-12 * (n_fft // 2 + 1)
