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
def config_c1():
    return make_case("c1_day_rigid_tdi1", "rigid", 8640, 10.0, 25, 1, "XYZ", seed=1,
                     monochromatic=True)


def config_c2(channels="XYZAET"):
    return make_case("c2_year_keplerian_tdi2", "keplerian", int(round(inputs.YEAR / 10.0)), 10.0,
                     25, 2, channels, seed=2)
