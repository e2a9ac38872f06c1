"""GPU parity of the forward response (projection, TDI) against the CPU oracle.

The HIP path is called through the C ABI; the oracle runs on the same seeded
inputs.  Bar: relative L2 error of the output, jointly over its channels,
<= 1e-11 (FP64 throughout).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2204_06633_amd import inputs
from tests import cases

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _gpu_orbits(s):
    from paper_2204_06633_amd import native
    return native.Orbits.from_samples(s)


def _t(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _padding_ok(case, gorb_p, gorb_t):
    g = case.grid
    fp, bp = gorb_p.projection_padding(case.order, g.dt)
    ft, bt = gorb_t.tdi_padding(case.order, case.generation, g.dt)
    assert g.front_proj >= fp and g.back_proj >= bp, (g.front_proj, fp, g.back_proj, bp)
    assert g.front_tdi >= ft and g.back_tdi >= bt, (g.front_tdi, ft, g.back_tdi, bt)


@pytest.mark.parametrize("order", [1, 3, 7, 25, 31])
@pytest.mark.parametrize("n_out", [1, 300, 1000])
def test_project_links_parity(torch_cuda, order, n_out):
    from paper_2204_06633_amd import native
    torch = torch_cuda
    case = cases.make_case("proj", "keplerian", n_out, 10.0, order, 2, "XYZ", seed=10 + order)
    g = case.grid
    gorb = _gpu_orbits(case.orbits_proj)
    _padding_ok(case, gorb, gorb)
    y = native.project_links(gorb, g.t0_h, g.dt, _t(torch, case.hp), _t(torch, case.hc),
                             _t(torch, [case.lam, case.beta]), order, g.y_start, g.n_y)
    torch.cuda.synchronize()
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    ref = oracle.project_links(orb, g.t0_h, g.dt, case.hp, case.hc, case.lam, case.beta, order,
                               np.arange(g.y_start, g.y_start + g.n_y))
    cases.check(y.cpu().numpy(), ref, TOL)


@pytest.mark.parametrize("gen", [1, 2])
@pytest.mark.parametrize("channels", ["XYZ", "AET", "XYZAET"])
@pytest.mark.parametrize("order", [1, 5, 25, 31])
def test_tdi_combine_parity(torch_cuda, gen, channels, order):
    from paper_2204_06633_amd import native
    torch = torch_cuda
    rng = np.random.default_rng(100 * gen + order)
    s = inputs.make_orbit_samples("keplerian", 2e6, 2e6 + 2e4)
    gorb = _gpu_orbits(s)
    dt = 10.0
    ft, bt = gorb.tdi_padding(order, gen, dt)
    n_out = 777
    n_y = ft + n_out + bt + 5
    y = rng.standard_normal((6, n_y))
    t0_y = 2e6 + 1000.0
    out = native.tdi_combine(gorb, t0_y, dt, _t(torch, y), gen, order, channels, ft + 2, n_out)
    torch.cuda.synchronize()
    orb = oracle.Orbits.from_samples(s)
    xyz = oracle.tdi_xyz(orb, t0_y, dt, y, gen, order, np.arange(ft + 2, ft + 2 + n_out))
    ref = oracle.select_channels(xyz, channels)
    cases.check(out.cpu().numpy(), ref, TOL)


def _gpu_response(torch, case):
    from paper_2204_06633_amd import response
    gp = _gpu_orbits(case.orbits_proj)
    gt = gp if case.orbits_tdi is case.orbits_proj else _gpu_orbits(case.orbits_tdi)
    _padding_ok(case, gp, gt)
    tpl = response.Template(gp, gt, case.grid, case.order, case.generation, case.channels)
    out, _ = response.plain_forward(tpl, _t(torch, case.hp), _t(torch, case.hc),
                                    _t(torch, [case.lam, case.beta]))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_response_day_full(torch_cuda):
    """One day of a monochromatic source, rigid equal-arm orbits, TDI-1 XYZ."""
    case = cases.day_case()
    got = _gpu_response(torch_cuda, case)
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    ref = oracle.response(orb, orb, case.grid, case.hp, case.hc, case.lam, case.beta,
                          case.order, case.generation, case.channels)
    cases.check(got, ref, TOL)


def test_response_year_sampled(torch_cuda):
    """One year at 10 s of a chirping source on flexing Keplerian orbits,
    TDI-2 X/Y/Z and A/E/T, compared on sampled outputs (the oracle computes
    each sampled output on its own)."""
    case = cases.year_case("XYZAET")
    got = _gpu_response(torch_cuda, case)
    idx = cases.sample_indices(case.grid.n_out, 400, seed=22)
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    ref = cases.oracle_sampled_response(orb, orb, case, idx)
    cases.check(got[:, idx], ref, TOL)


def test_response_hybrid_orbits(torch_cuda):
    """Keplerian orbits for the projection, rigid equal-arm for TDI (Sec. V)."""
    case = cases.make_case("hybrid", "keplerian", 5000, 15.0, 25, 2, "AET", seed=5,
                           tdi_orbit_kind="rigid")
    got = _gpu_response(torch_cuda, case)
    op = oracle.Orbits.from_samples(case.orbits_proj)
    ot = oracle.Orbits.from_samples(case.orbits_tdi)
    ref = oracle.response(op, ot, case.grid, case.hp, case.hc, case.lam, case.beta, case.order,
                          case.generation, case.channels)
    cases.check(got, ref, TOL)


def test_small_dt_uses_global_path(torch_cuda):
    """dt = 0.25 s: the stencil window of a tile exceeds the LDS tile, so the
    kernels read global memory; results must not change."""
    case = cases.make_case("small_dt", "keplerian", 700, 0.25, 9, 2, "XYZ", seed=6)
    got = _gpu_response(torch_cuda, case)
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    ref = oracle.response(orb, orb, case.grid, case.hp, case.hc, case.lam, case.beta, case.order,
                          case.generation, case.channels)
    cases.check(got, ref, TOL)


def test_empty_and_range_errors(torch_cuda):
    from paper_2204_06633_amd import native
    torch = torch_cuda
    case = cases.make_case("err", "keplerian", 100, 10.0, 25, 2, "XYZ", seed=7)
    g = case.grid
    gorb = _gpu_orbits(case.orbits_proj)
    hp, hc = _t(torch, case.hp), _t(torch, case.hc)
    sky = _t(torch, [0.1, 0.2])
    y = native.project_links(gorb, g.t0_h, g.dt, hp, hc, sky, 25, g.y_start, 0)
    assert y.shape == (6, 0)
    fp, _ = gorb.projection_padding(25, g.dt)
    with pytest.raises(native.LisaRespError) as e:
        native.project_links(gorb, g.t0_h, g.dt, hp, hc, sky, 25, fp - 1, 10)
    assert e.value.status == 2
    with pytest.raises(native.LisaRespError) as e:
        native.project_links(gorb, g.t0_h, g.dt, hp, hc, sky, 24, g.y_start, 10)
    assert e.value.status == 3
    with pytest.raises(native.LisaRespError) as e:     # orbit grid does not cover the times
        native.project_links(gorb, g.t0_h + 1e6, g.dt, hp, hc, sky, 25, g.y_start, 10)
    assert e.value.status == 2


def test_non_finite_sky_stays_in_bounds(torch_cuda):
    """NaN angles must give NaN link responses, never a stray access."""
    from paper_2204_06633_amd import native
    torch = torch_cuda
    case = cases.make_case("nan", "keplerian", 600, 10.0, 25, 2, "XYZ", seed=8)
    g = case.grid
    gorb = _gpu_orbits(case.orbits_proj)
    y = native.project_links(gorb, g.t0_h, g.dt, _t(torch, case.hp), _t(torch, case.hc),
                             _t(torch, [float("nan"), 0.3]), 25, g.y_start, g.n_y)
    torch.cuda.synchronize()
    assert torch.isnan(y).all()


def test_fast_varying_delays_exercise_misaligned_windows(torch_cuda):
    """Light times that change by ~1e-4 s per second make the two samples of
    a lane straddle integer positions in many waves, which takes the
    separate-window branch of both kernels; results must not change."""
    torch = torch_cuda
    from paper_2204_06633_amd import native, response
    t0, dto, n = 0.0, 1e4, 40
    tk = t0 + dto * np.arange(n)
    pos = inputs.keplerian_orbits(tk)
    base = np.array([8.21, 8.47, 8.05, 8.36, 8.12, 8.58])
    ltt = base[None, :] + 0.6 * np.sin(2 * math.pi * tk[:, None] / 7e4 + np.arange(6)[None, :])
    s = inputs.OrbitSamples(t0, dto, pos, ltt)
    case = cases.make_case("fast", "keplerian", 20000, 1.0, 25, 2, "XYZ", seed=17,
                           t_start=5e4)
    grid = inputs.make_template_grid(s, 25, 1.0, 5e4, 20000, 2)
    grid.front_tdi += 16                        # the spline bound of fast light times is loose
    case = cases.Case(case.name, s, s, grid, case.params, None, None, 25, 2, "XYZAET")
    case.hp, case.hc = inputs.gb_polarizations(case.params, case.grid.waveform_times())
    got = _gpu_response(torch, case)
    orb = oracle.Orbits.from_samples(s)
    ref = oracle.response(orb, orb, case.grid, case.hp, case.hc, case.lam, case.beta, 25, 2,
                          "XYZAET")
    cases.check(got, ref, TOL)


@pytest.mark.parametrize("n_out", [511, 512, 513, 1025])
def test_tile_boundaries(torch_cuda, n_out):
    case = cases.make_case("tiles", "keplerian", n_out, 10.0, 11, 2, "XYZAET", seed=n_out)
    got = _gpu_response(torch_cuda, case)
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    ref = oracle.response(orb, orb, case.grid, case.hp, case.hc, case.lam, case.beta, case.order,
                          case.generation, case.channels)
    cases.check(got, ref, TOL)


def _sky_of_direction(e_r):
    """(lam, beta) of the unit vector e_r pointing at the source."""
    e = np.asarray(e_r, dtype=np.float64) / np.linalg.norm(e_r)
    return math.atan2(e[1], e[0]) % (2.0 * math.pi), math.asin(max(-1.0, min(1.0, e[2])))


def _near_arm_sky(offset):
    """A sky position whose propagation direction k = -e_r lies within about
    `offset` rad of arm 1->2 at the first output time, so 1 - k.n is ~offset^2/2
    there (the response's 1/(2(1 - k.n)) factor is large but finite)."""
    case = cases.make_case("near_arm_probe", "keplerian", 100, 10.0, 25, 2, "AET", seed=41)
    s = case.orbits_proj
    k0 = int(round((case.grid.t_start - s.t0) / s.dt))
    n12 = s.x[k0, 0] - s.x[k0, 1]
    n12 /= np.linalg.norm(n12)
    perp = np.cross(n12, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp)
    k = n12 * math.cos(offset) + perp * math.sin(offset)
    return _sky_of_direction(-k)


@pytest.mark.parametrize("sky", ["north_pole", "south_pole", "lam_zero", "lam_2pi", "near_arm"])
def test_degenerate_sky_positions(torch_cuda, sky):
    """Sources at the ecliptic poles, at the wrap of lambda, and nearly along an
    arm (1 - k.n ~ 5e-3): one day of TDI-2 A/E/T on Keplerian orbits."""
    lam, beta = {"north_pole": (1.3, math.pi / 2), "south_pole": (4.0, -math.pi / 2),
                 "lam_zero": (0.0, 0.4), "lam_2pi": (2.0 * math.pi, 0.4),
                 "near_arm": None}[sky] or _near_arm_sky(0.1)
    params = np.array([1e-22, 4e-3, 1e-16, 0.7, 1.0, 0.3, lam, beta])
    case = cases.make_case("sky_" + sky, "keplerian", 8640, 10.0, 25, 2, "AET", seed=42,
                           params=params)
    got = _gpu_response(torch_cuda, case)
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    ref = oracle.response(orb, orb, case.grid, case.hp, case.hc, case.lam, case.beta,
                          case.order, case.generation, case.channels)
    assert np.all(np.isfinite(got))
    cases.check(got, ref, TOL)
