"""Seeded synthetic inputs for the generic LISA time-domain response.

This module produces the *inputs* of the response and nothing else: spacecraft
orbits sampled on a coarse grid, the light travel times along the six links at
reception time, Galactic-binary source parameters drawn from the priors of the
paper's Table I, and the Galactic-binary polarisations h+ / hx sampled on the
data grid (Sec. III).  It holds none of the response's arithmetic (no
projection, no interpolation, no TDI), so both the CPU oracle and the HIP path
can be fed from it.

Conventions (Sec. IV, Fig. 1 and IV.A):
  * spacecraft 1..3 are ordered clockwise when looking down on +z;
  * link l = 0..5 is (receiver, emitter) = 12, 23, 31, 13, 32, 21;
  * positions are in metres in the SSB ecliptic frame, times in seconds,
    light travel times in seconds at reception time.

The paper's ESA orbit files and its second-order post-Minkowskian light times
are not available; the synthetic orbits below stand in for them with the same
scale (2.5e9 m arms, 1 AU heliocentric, annual period) and a flat-space
(zeroth-order) light-time solver.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299792458.0          # m/s
AU = 1.495978707e11            # m
YEAR = 31557600.0              # Julian year, s
L_ARM = 2.5e9                  # nominal armlength, m (Sec. IV.D)

# link l -> (receiver, emitter), spacecraft numbered 1..3
LINKS = ((1, 2), (2, 3), (3, 1), (1, 3), (3, 2), (2, 1))


# --------------------------------------------------------------------------
# Orbits
# --------------------------------------------------------------------------

def rigid_orbits(t, L=L_ARM, a=AU, phase=0.0):
    """Rigidly rotating equilateral constellation (exact armlength L).

    The centre moves on a circle of radius ``a`` in the ecliptic with an annual
    period; the constellation plane makes 60 degrees with the ecliptic
    (Sec. IV.D) and the triangle counter-rotates once per year ("cartwheel").
    Returns positions [len(t)][3][3] in metres.
    """
    t = np.asarray(t, dtype=np.float64)
    om = 2.0 * math.pi / YEAR
    ang = om * t + phase
    r_hat = np.stack([np.cos(ang), np.sin(ang), np.zeros_like(ang)], -1)
    t_hat = np.stack([-np.sin(ang), np.cos(ang), np.zeros_like(ang)], -1)
    z_hat = np.array([0.0, 0.0, 1.0])
    p_hat = 0.5 * (-r_hat + math.sqrt(3.0) * z_hat)   # in-plane, 60 deg tilt
    centre = a * r_hat
    rad = L / math.sqrt(3.0)
    out = np.empty(t.shape + (3, 3))
    for k in range(3):
        phi = ang + 2.0 * math.pi * k / 3.0
        out[..., k, :] = centre + rad * (np.cos(phi)[..., None] * p_hat
                                         + np.sin(phi)[..., None] * t_hat)
    return out


def keplerian_orbits(t, L=L_ARM, a=AU, detune=0.01, phase=0.0, lam1=0.0):
    """Three heliocentric Keplerian ellipses forming a flexing triangle.

    Eccentricity e = L / (2 sqrt(3) a); each orbit is tilted about its own
    rotated y-axis by arctan(sqrt(3) e (1 + detune)).  ``detune`` = 0.01 gives
    an armlength flex of about 1 % over a year (the ideal tilt gives about
    0.5 %).  Spacecraft k = 0, 1, 2 has longitude of periastron lam1 - 2 pi
    k / 3 and initial mean anomaly ``phase`` + 2 pi k / 3 (so ``lam1`` and
    ``phase`` are the two free parameters of an equal-armlength
    configuration, Sec. IV.D).  Kepler's equation is solved by Newton
    iteration in FP64.  Returns positions [len(t)][3][3] in metres.
    """
    t = np.asarray(t, dtype=np.float64)
    om = 2.0 * math.pi / YEAR
    e = L / (2.0 * math.sqrt(3.0) * a)
    tilt = math.atan(math.sqrt(3.0) * e * (1.0 + detune))
    out = np.empty(t.shape + (3, 3))
    for k in range(3):
        sig = lam1 - 2.0 * math.pi * k / 3.0
        mean = om * t + phase + 2.0 * math.pi * k / 3.0
        ecc = mean.copy()
        for _ in range(50):
            step = (ecc - e * np.sin(ecc) - mean) / (1.0 - e * np.cos(ecc))
            ecc = ecc - step
            if np.max(np.abs(step)) < 1e-16:
                break
        X = a * (np.cos(ecc) - e)
        Y = a * math.sqrt(1.0 - e * e) * np.sin(ecc)
        Xt = X * math.cos(tilt)
        Z = X * math.sin(tilt)
        cs, sn = math.cos(sig), math.sin(sig)
        out[..., k, 0] = cs * Xt - sn * Y
        out[..., k, 1] = sn * Xt + cs * Y
        out[..., k, 2] = Z
    return out


def static_orbits(t, positions):
    """Constant positions [3][3] broadcast over times ``t``."""
    t = np.asarray(t, dtype=np.float64)
    return np.broadcast_to(np.asarray(positions, dtype=np.float64),
                           t.shape + (3, 3)).copy()


def light_travel_times(pos_fn, t, tol=1e-15, max_iter=60):
    """Flat-space light travel time L_ij(t) = |x_i(t) - x_j(t - L_ij)| / c.

    Solved by fixed-point iteration (contraction ratio ~ v/c ~ 1e-4) at the
    reception times ``t``.  ``pos_fn(t) -> [len(t)][3][3]``.  Returns
    [len(t)][6] in seconds, links ordered as ``LINKS``.
    """
    t = np.asarray(t, dtype=np.float64)
    xr = pos_fn(t)
    out = np.empty(t.shape + (6,))
    for l, (r, e) in enumerate(LINKS):
        rx = xr[..., r - 1, :]
        lt = np.linalg.norm(rx - xr[..., e - 1, :], axis=-1) / C_LIGHT
        for _ in range(max_iter):
            xe = pos_fn(t - lt)[..., e - 1, :]
            new = np.linalg.norm(rx - xe, axis=-1) / C_LIGHT
            done = np.max(np.abs(new - lt)) <= tol * np.max(np.abs(new))
            lt = new
            if done:
                break
        out[..., l] = lt
    return out


@dataclasses.dataclass
class OrbitSamples:
    """Coarse orbit samples: t_k = t0 + k*dt, k = 0..n-1."""
    t0: float
    dt: float
    x: np.ndarray      # [n][3][3] m
    ltt: np.ndarray    # [n][6] s

    @property
    def n(self):
        return self.x.shape[0]


def make_orbit_samples(kind, t_begin, t_end, dt_orbit=1e4, margin=3, **kw):
    """Sample an orbit family on a coarse grid that covers [t_begin, t_end].

    ``kind`` is 'rigid', 'keplerian', 'static' (static needs ``positions``
    and optionally ``ltt`` = [6] constant light times; if ``ltt`` is omitted
    the geometric distances / c are used) or 'function' (``fn``: t ->
    positions [len(t)][3][3]).
    """
    k0 = math.floor(t_begin / dt_orbit) - margin
    k1 = math.ceil(t_end / dt_orbit) + margin
    t0 = k0 * dt_orbit
    t = t0 + dt_orbit * np.arange(k1 - k0 + 1, dtype=np.float64)
    if kind == "rigid":
        fn = lambda tt: rigid_orbits(tt, **kw)
    elif kind == "keplerian":
        fn = lambda tt: keplerian_orbits(tt, **kw)
    elif kind == "function":
        fn = kw["fn"]
    elif kind == "static":
        pos = np.asarray(kw["positions"], dtype=np.float64)
        x = static_orbits(t, pos)
        if kw.get("ltt") is not None:
            lt = np.broadcast_to(np.asarray(kw["ltt"], dtype=np.float64),
                                 t.shape + (6,)).copy()
        else:
            lt = np.stack([np.full(t.shape, np.linalg.norm(pos[r - 1] - pos[e - 1]) / C_LIGHT)
                           for r, e in LINKS], -1)
        return OrbitSamples(t0, dt_orbit, x, lt)
    else:
        raise ValueError(kind)
    return OrbitSamples(t0, dt_orbit, fn(t), light_travel_times(fn, t))


# --------------------------------------------------------------------------
# Galactic-binary source (Sec. III) and parameter draws (Table I)
# --------------------------------------------------------------------------

PARAM_NAMES = ("A", "f0", "fdot", "phi0", "iota", "psi", "lam", "beta")


def gb_polarizations(params, t):
    """SSB-frame h+, hx of a Galactic binary at times ``t`` (waveform time).

    Source frame: h+S = A cos(Phi), hxS = A sin(Phi),
    Phi = 2 pi (f0 t + fdot t^2 / 2 + fddot t^3 / 6) + phi0, fddot =
    11 fdot^2 / (3 f0); then the rotation by 2 psi of
    [-(1 + cos^2 iota) h+S, -2 cos(iota) hxS] (Sec. III).
    ``params`` = (A, f0, fdot, phi0, iota, psi, ...).
    """
    A, f0, fdot, phi0, iota, psi = [float(v) for v in params[:6]]
    t = np.asarray(t, dtype=np.float64)
    fddot = 11.0 / 3.0 * fdot * fdot / f0 if f0 != 0.0 else 0.0
    phase = 2.0 * math.pi * (f0 * t + 0.5 * fdot * t * t + fddot * t * t * t / 6.0) + phi0
    hp_s = A * np.cos(phase)
    hc_s = A * np.sin(phase)
    ci = math.cos(iota)
    a_p = -(1.0 + ci * ci) * hp_s
    a_c = -2.0 * ci * hc_s
    c2, s2 = math.cos(2.0 * psi), math.sin(2.0 * psi)
    return c2 * a_p - s2 * a_c, s2 * a_p + c2 * a_c


def draw_gb_params(rng, n=None, f_range=(1e-3, 1e-2), fdot_range=(1e-17, 1e-15),
                   amp_range=(1e-23, 1e-21)):
    """Seeded draws: f, fdot and A log-uniform on the given ranges; the angles
    follow Table I (phi0, psi, lambda uniform; cos iota, sin beta uniform)."""
    size = 1 if n is None else n
    lu = lambda lo, hi: np.exp(rng.uniform(math.log(lo), math.log(hi), size))
    A = lu(*amp_range)
    f0 = lu(*f_range)
    fdot = lu(*fdot_range)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, size)
    iota = np.arccos(rng.uniform(-1.0, 1.0, size))
    psi = rng.uniform(0.0, math.pi, size)
    lam = rng.uniform(0.0, 2.0 * math.pi, size)
    beta = np.arcsin(rng.uniform(-1.0, 1.0, size))
    out = np.stack([A, f0, fdot, phi0, iota, psi, lam, beta], -1)
    return out[0] if n is None else out


# Galactic binary of the paper's Fig. 3 caption, order (A, f0, fdot, phi0, iota, psi, lam, beta).
PAPER_FIG3_BINARY = (1e-22, 10e-3, 1.4e-14, 4.58, 1.11, 0.45, 5.23, 1.23)


# --------------------------------------------------------------------------
# Template layout on the data grid
# --------------------------------------------------------------------------

@dataclasses.dataclass
class TemplateGrid:
    """Index bookkeeping of one template on the uniform data grid.

    h[j] sits at absolute time t0_h + j*dt, j = 0..n_h-1.  The link series y
    covers h-indices [y_start, y_start + n_y); the TDI output covers
    h-indices [out_start, out_start + n_out).  The waveform time origin
    (t = 0) is the first output sample.
    """
    dt: float
    t_start: float       # absolute time of the first output sample
    n_out: int
    front_tdi: int
    back_tdi: int
    front_proj: int
    back_proj: int

    @property
    def n_y(self):
        return self.front_tdi + self.n_out + self.back_tdi

    @property
    def y_start(self):
        return self.front_proj

    @property
    def out_start(self):
        return self.front_proj + self.front_tdi

    @property
    def n_h(self):
        return self.front_proj + self.n_y + self.back_proj

    @property
    def t0_h(self):
        return self.t_start - self.out_start * self.dt

    def waveform_times(self):
        return (np.arange(self.n_h, dtype=np.float64) - self.out_start) * self.dt

    def h_times(self):
        return self.t0_h + np.arange(self.n_h, dtype=np.float64) * self.dt


def conservative_padding(orbits: OrbitSamples, order, dt, gen=2):
    """Generous stencil padding (samples) from the sampled orbit extent.

    Returns (front_tdi, back_tdi, front_proj, back_proj).  Libraries compute
    their own exact requirement; these values only need to be at least as
    large, so they use the sample maxima plus a safety margin.
    """
    half = (order + 1) // 2
    lmax = float(np.max(orbits.ltt)) * 1.01 + 1e-3
    rmax = float(np.max(np.linalg.norm(orbits.x, axis=-1))) * 1.01
    nlinks = 7 if gen == 2 else 3
    front_tdi = int(math.ceil(nlinks * lmax / dt)) + half + 2
    back_tdi = half + 2
    front_proj = int(math.ceil((lmax + rmax / C_LIGHT) / dt)) + half + 2
    back_proj = int(math.ceil(rmax / C_LIGHT / dt)) + half + 2
    return front_tdi, back_tdi, front_proj, back_proj


def make_template_grid(orbits, order, dt, t_start, n_out, gen=2):
    f_t, b_t, f_p, b_p = conservative_padding(orbits, order, dt, gen)
    return TemplateGrid(dt, t_start, n_out, f_t, b_t, f_p, b_p)


def orbit_span_for(grid: TemplateGrid):
    """Absolute time range the orbits must cover for a template grid."""
    return grid.t0_h, grid.t0_h + (grid.n_h - 1) * grid.dt


# --------------------------------------------------------------------------
# Noise curve for the frequency-domain likelihood (Sec. II.A)
# --------------------------------------------------------------------------
def noise_psd_aet(f, L=L_ARM, generation=2, acc=3e-15, oms=15e-12):
    """One-sided noise PSDs (S_AE, S_T) of the A/E and T channels, fractional
    frequency, for equal arms.

    A stand-in for the paper's tabulated design curve: test-mass acceleration
    noise ``acc`` m s^-2 / sqrt(Hz) reddened below 0.4 mHz and whitened above
    8 mHz, optical-metrology noise ``oms`` m / sqrt(Hz) reddened below 2 mHz,
    propagated through the equal-arm Michelson combinations (second
    generation: times 4 sin^2(2x)), x = 2 pi f L / c.
    """
    f = np.asarray(f, dtype=np.float64)
    s_acc = (acc ** 2 * (1.0 + (4e-4 / f) ** 2) * (1.0 + (f / 8e-3) ** 4)
             / (2.0 * math.pi * f * C_LIGHT) ** 2)
    s_oms = oms ** 2 * (1.0 + (2e-3 / f) ** 4) * (2.0 * math.pi * f / C_LIGHT) ** 2
    x = 2.0 * math.pi * f * L / C_LIGHT
    sx2 = np.sin(x) ** 2
    s_ae = 8.0 * sx2 * (2.0 * s_acc * (3.0 + 2.0 * np.cos(x) + np.cos(2.0 * x))
                        + s_oms * (2.0 + np.cos(x)))
    s_t = 16.0 * s_oms * (1.0 - np.cos(x)) * sx2 + 128.0 * s_acc * sx2 * np.sin(0.5 * x) ** 4
    if generation == 2:
        g2 = 4.0 * np.sin(2.0 * x) ** 2
        s_ae, s_t = s_ae * g2, s_t * g2
    return s_ae, s_t


def noise_weights(n_fft, dt, f_min=1e-4, f_max=2.5e-2, generation=2, L=L_ARM):
    """Bin weights w_k = 4 df / S_n(f_k), k = 0 .. n_fft/2, for the A/E and
    the T channel; zero outside [f_min, f_max] (the band stops below the
    first zero of the second-generation transfer function, c / (4 L))."""
    k = np.arange(n_fft // 2 + 1)
    f = k / (n_fft * dt)
    df = 1.0 / (n_fft * dt)
    band = (f >= f_min) & (f <= f_max)
    w_ae = np.zeros(k.shape)
    w_t = np.zeros(k.shape)
    s_ae, s_t = noise_psd_aet(f[band], L=L, generation=generation)
    w_ae[band] = 4.0 * df / s_ae
    w_t[band] = 4.0 * df / s_t
    return w_ae, w_t


def sample_indices(n, k, seed, edge=8):
    """``k`` seeded random indices of [0, n) plus the first and last ``edge``
    (sorted, unique): the output samples that a sampled comparison reads."""
    rng = np.random.default_rng(seed)
    mid = rng.choice(n, size=min(k, n), replace=False)
    idx = np.unique(np.concatenate([np.arange(min(edge, n)), np.arange(max(n - edge, 0), n), mid]))
    return idx.astype(np.int64)
