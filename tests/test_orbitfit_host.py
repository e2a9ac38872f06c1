"""Host checks of the orbit-approximation tooling (Sec. IV.D and V): the
equal-armlength model, its Nelder-Mead fit and the overlap diagnostics."""
import math

import numpy as np

from oracle import fd as ofd
from paper_2204_06633_amd import inputs, orbitfit


def _grid(years=4.0, per_day=1):
    return np.linspace(0.0, years * inputs.YEAR, int(years * 365 * per_day) + 1)


def test_equal_arm_model_is_a_rigid_triangle():
    t = _grid(1.0, 4)
    x = orbitfit.eq_positions(t, 0.3, -1.1)
    for i, j in ((0, 1), (1, 2), (2, 0)):
        d = np.linalg.norm(x[:, i] - x[:, j], axis=-1)
        assert np.max(np.abs(d - inputs.L_ARM)) <= 1e-12 * inputs.L_ARM
    # plane at 60 degrees to the ecliptic, spacecraft clockwise seen from +z
    # (the convention of the synthetic orbits)
    n = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    nz = n[:, 2] / np.linalg.norm(n, axis=-1)
    xk = inputs.keplerian_orbits(t[:1])
    nk = np.cross(xk[0, 1] - xk[0, 0], xk[0, 2] - xk[0, 0])
    assert np.allclose(nz, -0.5, atol=1e-12) and nk[2] < 0
    # guiding centre at 1 AU
    c = x.mean(axis=1)
    assert np.allclose(np.linalg.norm(c[:, :2], axis=-1), inputs.AU, rtol=1e-4)


def test_equal_arm_model_is_the_keplerian_motion_to_first_order():
    # the exact Keplerian ellipses with the ideal tilt differ from it by
    # O(e^2 a), i.e. a fraction O(e) of the O(e a) displacements
    t = _grid(1.0, 4)
    e = inputs.L_ARM / (2 * math.sqrt(3) * inputs.AU)
    d = np.abs(inputs.keplerian_orbits(t, detune=0.0, phase=0.4, lam1=-0.2)
               - orbitfit.eq_positions(t, -0.2, 0.4))
    assert d.max() <= 5 * e * (e * inputs.AU)               # vs O(e a) = 7e8 m


def test_fit_recovers_equal_arm_parameters():
    t = _grid()
    x = orbitfit.eq_positions(t, 0.3, -1.1)
    lam1, m1, cost = orbitfit.fit_eq_orbits(t, x, x0=(0.25, -1.0))
    assert abs(lam1 - 0.3) < 1e-7 and abs(m1 + 1.1) < 1e-7
    assert cost / (3 * t[-1]) < 1.0                      # mean distance below a metre


def test_fit_to_flexing_orbits():
    t = _grid()
    x = inputs.keplerian_orbits(t, detune=0.01, phase=0.7, lam1=-0.4)
    c0 = orbitfit.eq_cost((0.0, 0.0), t, x)
    lam1, m1, cost = orbitfit.fit_eq_orbits(t, x, x0=(0.0, 0.0))
    assert abs(lam1 + 0.4) < 1e-6 and abs(m1 - 0.7) < 1e-6
    assert cost < 1e-2 * c0
    assert cost / (3 * t[-1]) < 1e-4 * inputs.AU         # mean distance


def test_configurations():
    c = orbitfit.configurations("acc", "eq")
    assert c == {"ESA": ("acc", "acc"), "EQ": ("eq", "eq"), "ESAEQ": ("acc", "eq"),
                 "EQESA": ("eq", "acc")}


def test_overlap_statistics_against_oracle():
    rng = np.random.default_rng(5)
    n_fft, n, dt = 256, 200, 10.0
    s = rng.standard_normal((3, n))
    h = s + 0.1 * rng.standard_normal((3, n))
    w_ae, w_t = rng.uniform(0, 1, n_fft // 2 + 1), rng.uniform(0, 2, n_fft // 2 + 1)
    st = ofd.loglike(h, s, w_ae, w_t, dt, n_fft)
    ss = ofd.loglike(np.zeros_like(s), s, w_ae, w_t, dt, n_fft)["rr"]
    got = orbitfit.overlap_statistics(np.array([st["rr"], st["hh"], st["dh"]]), ss)
    ref = ofd.overlap(h, s, w_ae, w_t, dt, n_fft)
    for k in ("rho_opt", "rho_ex", "overlap", "mismatch"):
        assert abs(float(got[k]) - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-3), k
    # Cauchy-Schwarz: overlap <= 1, equality for h = s (and any positive multiple)
    same = ofd.overlap(2.0 * s, s, w_ae, w_t, dt, n_fft)
    assert abs(same["mismatch"]) < 1e-14 and 0 < ref["mismatch"] < 1


def test_fitting_factor_finds_the_likelihood_maximum():
    """A closed-form score: log L = -1/2 (x - x*)^T Q (x - x*) with the maximum
    off the start, overlap = exp(-|x - x_o|^2) peaking elsewhere.  The fitting
    factor is the overlap at the likelihood maximum x* (Sec. II.A), not the
    largest overlap."""
    rng = np.random.default_rng(1)
    D = 8
    a = rng.standard_normal((D, D))
    Q = a @ a.T + D * np.eye(D)
    x_star = rng.standard_normal(D) * 0.3
    x_o = x_star + 0.2

    def score(x):
        d = x - x_star
        return -0.5 * float(d @ Q @ d), math.exp(-float(np.sum((x - x_o) ** 2)))

    r = orbitfit.fitting_factor(score, np.zeros(D), np.full(D, 0.1), maxfev=20000)
    assert np.max(np.abs(r["theta"] - x_star)) < 1e-6
    assert abs(r["fitting_factor"] - math.exp(-float(np.sum((x_star - x_o) ** 2)))) < 1e-9
    assert r["loglike"] >= r["loglike_start"]


def test_fitting_factor_at_the_start_when_it_is_the_maximum():
    """Data equal to the template at the start: the start is the likelihood
    maximum and the fitting factor is the overlap there (1)."""
    x0 = np.array([0.3, -1.0, 2.0])
    score = lambda x: (-float(np.sum((x - x0) ** 2)), 1.0 / (1.0 + float(np.sum((x - x0) ** 2))))
    r = orbitfit.fitting_factor(score, x0, np.full(3, 0.05))
    assert abs(r["fitting_factor"] - 1.0) < 1e-12 and np.max(np.abs(r["theta"] - x0)) < 1e-6
