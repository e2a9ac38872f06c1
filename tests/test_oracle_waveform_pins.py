"""Pins of the Galactic-binary waveform oracle (Sec. III): the phase against
exact rational arithmetic, the polarisation invariants, and the
vector-Jacobian product against central differences."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import waveform as ow

SRC = (1.3e-22, 9.7e-3, 1.4e-14, 4.58, 1.11, 0.45, 5.23, 1.23)


def test_phase_against_exact_rationals():
    # the parameters and times are binary floats, so Fraction holds them exactly
    t = np.array([0.0, 10.0, 1234567.0, 31557600.0, -150.0])
    ph = ow.phase(SRC, t)
    f0, fdot, phi0 = (Fraction(v) for v in (SRC[1], SRC[2], SRC[3]))
    fddot = Fraction(11, 3) * fdot * fdot / f0
    for tk, got in zip(t, ph):
        T = Fraction(float(tk))
        cyc = f0 * T + fdot * T * T / 2 + fddot * T * T * T / 6
        frac = cyc - round(cyc)
        ref = 2 * math.pi * float(frac) + float(phi0)
        assert abs(got - ref) < 5e-12, (tk, got - ref)
    # plain FP64 at one year is off by ~1e-10 rad: the extended precision matters
    T = 31557600.0
    plain = (2 * math.pi * (SRC[1] * T + SRC[2] * T * T / 2 + 11 / 3 * SRC[2] ** 2 / SRC[1] * T ** 3 / 6)
             + SRC[3])
    assert abs(math.remainder(plain - ph[3], 2 * math.pi)) < 1e-8


def test_polarisation_invariants():
    t = np.linspace(-1e3, 3e7, 2001)
    hp, hc = ow.polarizations(SRC, t)
    A, ci = SRC[0], math.cos(SRC[4])
    ph = ow.phase(SRC, t)
    ref = A * A * ((1 + ci * ci) ** 2 * np.cos(ph) ** 2 + 4 * ci * ci * np.sin(ph) ** 2)
    assert np.allclose(hp * hp + hc * hc, ref, rtol=1e-13, atol=0)   # psi rotates
    src2 = list(SRC)
    src2[5] += math.pi / 2                                            # psi + pi/2 negates
    hp2, hc2 = ow.polarizations(src2, t)
    assert np.allclose(hp2, -hp, rtol=1e-12, atol=1e-12 * A) and np.allclose(hc2, -hc, rtol=1e-12, atol=1e-12 * A)
    # face-on (iota = 0): circular polarisation, h+ = -2 A cos(Phi + 2 psi)
    src3 = list(SRC)
    src3[4] = 0.0
    hp3, hc3 = ow.polarizations(src3, t)
    assert np.allclose(hp3, -2 * A * np.cos(ph + 2 * SRC[5]), rtol=0, atol=1e-12 * A)


def test_instantaneous_frequency():
    # dPhi/dt / 2 pi = f0 + fdot t + fddot t^2 / 2, fddot = 11 fdot^2 / (3 f0)
    t0, h = 2.0e7, 1.0
    ph = ow.phase(SRC, np.array([t0 - h, t0 + h]))
    f = math.remainder(ph[1] - ph[0], 2 * math.pi) / (2 * h) / (2 * math.pi)
    fddot = 11 / 3 * SRC[2] ** 2 / SRC[1]
    # remainder removes the whole cycles covered in 2 s (2 f0 h ~ 0.02 cycles: none)
    assert abs(f - (SRC[1] + SRC[2] * t0 + fddot * t0 * t0 / 2)) < 1e-12


@pytest.mark.parametrize("k", range(6))
def test_vjp_against_central_differences(k):
    rng = np.random.default_rng(k)
    t = np.arange(-50, 2000) * 15.0
    g_hp, g_hc = rng.standard_normal(t.size), rng.standard_normal(t.size)
    g = ow.polarizations_vjp(SRC, t, g_hp, g_hc)
    assert g[6] == 0.0 and g[7] == 0.0
    scale = [1e-24, 1e-9, 1e-16, 1e-4, 1e-4, 1e-4][k]

    def L(v):
        p = list(SRC)
        p[k] = v
        hp, hc = ow.polarizations(p, t)
        return float(np.dot(g_hp, hp) + np.dot(g_hc, hc))

    d1 = (L(SRC[k] + scale) - L(SRC[k] - scale)) / (2 * scale)
    d2 = (L(SRC[k] + 2 * scale) - L(SRC[k] - 2 * scale)) / (4 * scale)
    rich = (4 * d1 - d2) / 3
    assert abs(g[k] - rich) <= 1e-6 * abs(rich), (k, g[k], rich)
