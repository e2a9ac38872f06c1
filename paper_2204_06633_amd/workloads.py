"""Seeded single-template workloads on the uniform data grid.

Built from ``inputs`` only (orbits, light times, source parameters,
polarisations); nothing here computes a response.  The named configurations
are the benchmark's: one day of a monochromatic source on rigid equal-arm
orbits with TDI-1, and one year at 10 s of a chirping source on flexing
Keplerian orbits with TDI-2.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import inputs


@dataclasses.dataclass
class Case:
    name: str
    orbits_proj: inputs.OrbitSamples
    orbits_tdi: inputs.OrbitSamples
    grid: inputs.TemplateGrid
    params: np.ndarray
    hp: np.ndarray
    hc: np.ndarray
    order: int
    generation: int
    channels: str

    @property
    def lam(self):
        return float(self.params[6])

    @property
    def beta(self):
        return float(self.params[7])


def make_case(name, orbit_kind, n_out, dt, order, generation, channels, seed, t_start=1.0e6,
              params=None, tdi_orbit_kind=None, monochromatic=False):
    rng = np.random.default_rng(seed)
    if params is None:
        params = inputs.draw_gb_params(rng)
        if monochromatic:
            params[0], params[1], params[2] = 1e-22, 3e-3, 0.0
    params = np.asarray(params, dtype=np.float64)
    t_end = t_start + n_out * dt
    orb_p = inputs.make_orbit_samples(orbit_kind, t_start, t_end)
    orb_t = orb_p if tdi_orbit_kind in (None, orbit_kind) else \
        inputs.make_orbit_samples(tdi_orbit_kind, t_start, t_end)
    grid = inputs.make_template_grid(orb_p, order, dt, t_start, n_out, generation)
    hp, hc = inputs.gb_polarizations(params, grid.waveform_times())
    return Case(name, orb_p, orb_t, grid, params, hp, hc, order, generation, channels)


# The benchmark configurations (single template): a day of a monochromatic
# source on rigid equal-arm orbits with TDI-1, and a year of a chirping
# source on flexing Keplerian orbits with TDI-2.
def day_case():
    return make_case("day8640_rigid_tdi1", "rigid", 8640, 10.0, 25, 1, "XYZ", seed=1,
                     monochromatic=True)


def year_case(channels="XYZAET"):
    return make_case("year_keplerian_tdi2", "keplerian", int(round(inputs.YEAR / 10.0)), 10.0,
                     25, 2, channels, seed=2)


@dataclasses.dataclass
class BatchLayout:
    """Templates laid out one after the other in shared h+ / hx / output
    arrays (offsets in elements)."""
    grids: list
    h_offsets: list
    out_offsets: list
    rows: int

    @property
    def n_h_total(self):
        return self.h_offsets[-1] + self.grids[-1].n_h if self.grids else 0

    @property
    def n_out_total(self):
        return self.out_offsets[-1] + self.rows * self.grids[-1].n_out if self.grids else 0

    def templates(self):
        return [(ho, g.n_h, g.out_start, g.n_out, oo)
                for g, ho, oo in zip(self.grids, self.h_offsets, self.out_offsets)]


def batch_layout(grids, rows):
    h_off, o_off, h, o = [], [], 0, 0
    for g in grids:
        h_off.append(h)
        o_off.append(o)
        h += g.n_h
        o += rows * g.n_out
    return BatchLayout(list(grids), h_off, o_off, rows)


def make_batch(n_templates, orbit_kind, n_out_list, dt, order, generation, seed, t_start=1.0e6,
               tdi_orbit_kind=None, params=None):
    """A batch of templates sharing the output start time t_start and the
    orbits, with per-template durations ``n_out_list`` and seeded source
    parameters (or ``params`` [n][8]).  Returns (layout, params, orbits_proj,
    orbits_tdi)."""
    rng = np.random.default_rng(seed)
    if params is None:
        params = inputs.draw_gb_params(rng, n_templates)
    n_max = int(max(n_out_list)) if len(n_out_list) else 0
    t_end = t_start + n_max * dt
    orb_p = inputs.make_orbit_samples(orbit_kind, t_start, t_end)
    orb_t = orb_p if tdi_orbit_kind in (None, orbit_kind) else \
        inputs.make_orbit_samples(tdi_orbit_kind, t_start, t_end)
    grids = []
    for n in n_out_list:
        g = inputs.make_template_grid(orb_p, order, dt, t_start, int(n), generation)
        g2 = inputs.make_template_grid(orb_t, order, dt, t_start, int(n), generation)
        # a few samples beyond the generous estimate, so the library's own
        # bound always fits inside
        g.front_tdi = max(g.front_tdi, g2.front_tdi) + 4
        g.back_tdi = max(g.back_tdi, g2.back_tdi) + 4
        grids.append(g)
    return grids, np.asarray(params, dtype=np.float64), orb_p, orb_t


@dataclasses.dataclass
class BatchCase:
    """A batch workload: per-template grids sharing the output start time,
    their layout in the shared arrays, source parameters [n][8] and orbits."""
    name: str
    grids: list
    layout: BatchLayout
    params: np.ndarray
    orbits_proj: inputs.OrbitSamples
    orbits_tdi: inputs.OrbitSamples
    dt: float
    order: int
    generation: int
    channels: str

    @property
    def t0(self):
        return self.grids[0].t_start

    @property
    def n_samples(self):
        return int(sum(g.n_out for g in self.grids))


def make_batch_case(name, n_out_list, dt, order, generation, channels, seed, params=None,
                    orbit_kind="keplerian", tdi_orbit_kind=None):
    grids, params, sp, st = make_batch(len(n_out_list), orbit_kind, n_out_list, dt, order,
                                       generation, seed, tdi_orbit_kind=tdi_orbit_kind,
                                       params=params)
    rows = 6 if channels == "XYZAET" else 3
    return BatchCase(name, grids, batch_layout(grids, rows), params, sp, st, dt, order,
                     generation, channels)


def uneven_batch_case(n_templates=512, seed=3):
    """512 Galactic binaries of uneven durations (uniform 0.25-1 yr at
    dt = 10 s), independent seeded parameters, flexing Keplerian orbits,
    TDI-2 A/E/T, order 25."""
    rng = np.random.default_rng(seed)
    full = int(round(inputs.YEAR / 10.0))
    n_out = np.round(rng.uniform(0.25, 1.0, n_templates) * full).astype(np.int64)
    return make_batch_case("batch%d_uneven_keplerian_tdi2" % n_templates, list(n_out), 10.0,
                           25, 2, "AET", seed)


def walker_batch_case(n_walkers=256, seed=5, spread=1e-6, tdi_orbit_kind="rigid"):
    """MCMC walkers around one Galactic binary: 1 yr at dt = 15 s each,
    Keplerian orbits for the projection and rigid equal-arm orbits for the
    TDI-2 delays (hybrid template; ``tdi_orbit_kind="keplerian"`` gives the
    full generic response), A/E/T, order 25.  Walker parameters are the
    source's scaled by (1 + spread * N(0,1)), angles shifted by
    spread * N(0,1)."""
    rng = np.random.default_rng(seed)
    base = inputs.draw_gb_params(rng)
    params = np.repeat(base[None, :], n_walkers, 0)
    params[:, :3] *= 1.0 + spread * rng.standard_normal((n_walkers, 3))
    params[:, 3:] += spread * rng.standard_normal((n_walkers, 5))
    n = int(round(inputs.YEAR / 15.0))
    name = "hybrid" if tdi_orbit_kind == "rigid" else tdi_orbit_kind
    return make_batch_case("walkers%d_%s_dt15" % (n_walkers, name), [n] * n_walkers, 15.0, 25, 2,
                           "AET", seed, params=params, tdi_orbit_kind=tdi_orbit_kind)


def device_polarizations(bc: BatchCase, device, params=None):
    """h+ and hx of every template of a batch, generated on the device with
    the torch waveform and laid out as bc.layout says.  Returns (hp, hc)."""
    import torch

    from . import waveform
    lay = bc.layout
    p = torch.as_tensor(bc.params if params is None else params, dtype=torch.float64,
                        device=device)
    hp = torch.empty(max(lay.n_h_total, 1), dtype=torch.float64, device=device)
    hc = torch.empty_like(hp)
    for k, (g, ho) in enumerate(zip(bc.grids, lay.h_offsets)):
        t = (torch.arange(g.n_h, dtype=torch.float64, device=device) - g.out_start) * g.dt
        a, b = waveform.gb_polarizations(p[k], t)
        hp[ho:ho + g.n_h] = a
        hc[ho:ho + g.n_h] = b
    return hp, hc


@dataclasses.dataclass
class FdCase:
    """Inputs of the frequency-domain likelihood: seeded A/E/T series of n
    samples at dt standing for the data and for n_templates templates, and
    the stand-in noise curve's bin weights."""
    name: str
    n: int
    dt: float
    n_templates: int
    seed: int
    f_min: float = 1e-4
    f_max: float = 2.5e-2

    def data(self, device):
        import torch
        g = torch.Generator(device=device).manual_seed(self.seed)
        return torch.randn((3, self.n), dtype=torch.float64, device=device, generator=g)

    def templates(self, device):
        import torch
        g = torch.Generator(device=device).manual_seed(self.seed + 1)
        return torch.randn((self.n_templates, 3, self.n), dtype=torch.float64, device=device,
                           generator=g)

    def weights(self, n_fft, device):
        import torch
        w_ae, w_t = inputs.noise_weights(n_fft, self.dt, self.f_min, self.f_max)
        return (torch.tensor(w_ae, dtype=torch.float64, device=device),
                torch.tensor(w_t, dtype=torch.float64, device=device))


def fd_case(n_templates=1, seed=11):
    """One year of A/E/T at dt = 10 s (3,155,760 samples) per template."""
    n = int(round(inputs.YEAR / 10.0))
    return FdCase("fd_1yr_dt10_aet", n, 10.0, n_templates, seed)


@dataclasses.dataclass
class OrbitConfigCase:
    """One source seen through the orbit models of Sec. V: accurate orbits
    (the flexing Keplerian stand-in for the ESA files) and the equal-armlength
    configuration fitted to them, on one template grid that suits both."""
    name: str
    accurate: inputs.OrbitSamples
    equal_arm: inputs.OrbitSamples
    eq_params: tuple
    grid: object
    params: np.ndarray
    hp: np.ndarray
    hc: np.ndarray
    order: int = 25
    generation: int = 2


def orbit_config_case(n_out, dt=10.0, t_start=1.0e6, params=inputs.PAPER_FIG3_BINARY, order=25,
                      fit_years=4.0):
    """The paper's Fig. 3 binary on n_out samples; the equal-armlength
    parameters come from the Nelder-Mead fit over ``fit_years`` (Sec. IV.D)."""
    from . import orbitfit
    t_end = t_start + n_out * dt
    acc = inputs.make_orbit_samples("keplerian", t_start, t_end)
    t_fit = np.linspace(0.0, fit_years * inputs.YEAR, int(fit_years * 365) + 1)
    lam1, m1, _ = orbitfit.fit_eq_orbits(t_fit, inputs.keplerian_orbits(t_fit), x0=(0.1, 0.1))
    eq = orbitfit.eq_orbit_samples(t_start, t_end, lam1, m1)
    pads = np.maximum(inputs.conservative_padding(acc, order, dt),
                      inputs.conservative_padding(eq, order, dt))
    grid = inputs.TemplateGrid(dt, t_start, n_out, *(int(v) for v in pads))
    params = np.asarray(params, dtype=np.float64)
    hp, hc = inputs.gb_polarizations(params, grid.waveform_times())
    return OrbitConfigCase("orbits_%d_dt%g" % (n_out, dt), acc, eq, (lam1, m1), grid, params,
                           hp, hc, order)


@dataclasses.dataclass
class SamplerCase:
    """A tempered-sampler run: ``T`` temperatures of ``W`` walkers on one
    output grid, noise-free data from the injected source (as in Sec. V)."""
    name: str
    T: int
    W: int
    orbits: inputs.OrbitSamples
    grid: object
    injection: np.ndarray
    order: int = 25
    generation: int = 2

    @property
    def m(self):
        return self.T * self.W // 2                     # proposals per half step

    def layout(self, m):
        g = self.grid
        return [(k * g.n_h, g.n_h, g.out_start, g.n_out, 3 * k * g.n_out) for k in range(m)]


def sampler_case(T=4, W=50, n_out=None, dt=15.0, t_start=1.0e6,
                 injection=inputs.PAPER_FIG3_BINARY, order=25):
    """The paper's sampler settings (4 temperatures of 50 walkers) on one
    year at dt = 15 s by default, flexing Keplerian orbits."""
    n_out = n_out or int(round(inputs.YEAR / dt))
    orb = inputs.make_orbit_samples("keplerian", t_start, t_start + n_out * dt)
    grid = inputs.make_template_grid(orb, order, dt, t_start, n_out, 2)
    return SamplerCase("sampler_T%d_W%d_n%d_dt%g" % (T, W, n_out, dt), T, W, orb, grid,
                       np.asarray(injection, dtype=np.float64), order)
