"""Pins of the oracle's sampled evaluation (oracle/sampled.py, CPU only).

The full-size GPU parity tests compare millions-of-sample outputs with the
oracle at sampled outputs only.  Those helpers must give exactly what the
whole-template oracle gives there: the forward at the sampled indices, and
the transpose applied to a channel gradient that vanishes elsewhere.  A
too-narrow window of link samples would read a NaN (sampled_response fills
the rest with NaN), a wrong index offset would move every value.
"""
import numpy as np
import pytest

import oracle
from oracle import sampled
from paper_2204_06633_amd import inputs, workloads


def _case(channels, gen, orbit="keplerian"):
    return workloads.make_case("sampled_pin", orbit, 1200, 10.0, 25, gen, channels, seed=61,
                               tdi_orbit_kind="rigid" if orbit == "keplerian" else None)


@pytest.mark.parametrize("channels,gen", [("AET", 2), ("XYZ", 1), ("XYZAET", 2)])
def test_sampled_response_equals_the_whole_template(channels, gen):
    case = _case(channels, gen)
    op = oracle.Orbits.from_samples(case.orbits_proj)
    ot = oracle.Orbits.from_samples(case.orbits_tdi)
    full = oracle.response(op, ot, case.grid, case.hp, case.hc, case.lam, case.beta, case.order,
                           case.generation, case.channels)
    idx = inputs.sample_indices(case.grid.n_out, 40, seed=3, edge=3)
    assert idx.min() == 0 and idx.max() == case.grid.n_out - 1
    got = sampled.sampled_response(op, ot, case, idx)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, full[:, idx])


@pytest.mark.parametrize("channels,gen", [("AET", 2), ("XYZ", 1)])
def test_sampled_adjoint_equals_the_whole_template(channels, gen):
    case = _case(channels, gen)
    op = oracle.Orbits.from_samples(case.orbits_proj)
    ot = oracle.Orbits.from_samples(case.orbits_tdi)
    idx = inputs.sample_indices(case.grid.n_out, 25, seed=4, edge=2)
    rows = 3
    gs = np.random.default_rng(5).standard_normal((rows, idx.size))
    g_full = np.zeros((rows, case.grid.n_out))
    g_full[:, idx] = gs
    rhp, rhc = oracle.response_adjoint(op, ot, case.grid, case.lam, case.beta, case.order,
                                       case.generation, g_full, case.channels)
    shp, shc = sampled.sampled_adjoint(op, ot, case, idx, gs)
    scale = max(np.abs(rhp).max(), np.abs(rhc).max())
    # the whole-template transpose adds exact zeros for the other outputs;
    # the sums agree to rounding
    assert np.abs(shp - rhp).max() <= 1e-14 * scale
    assert np.abs(shc - rhc).max() <= 1e-14 * scale
    assert np.count_nonzero(shp) > 0 and np.count_nonzero(shp) < shp.size


def test_compare_measures():
    """rel_err is the joint L2 measure, max_err the element-wise one; a
    single wrong element shows in max_err at full size."""
    from oracle import compare
    ref = np.ones((3, 10000))
    got = ref.copy()
    got[1, 77] += 1e-9
    e2, em = compare.errors(got, ref)
    assert np.isclose(em, 1e-9, rtol=1e-6)
    assert np.isclose(e2, 1e-9 / np.sqrt(30000), rtol=1e-6)
    with pytest.raises(AssertionError):
        compare.check(got, ref, 1e-10)
    assert compare.check(ref, ref, 0.0) == (0.0, 0.0)
    bad = ref.copy()
    bad[0, 0] = np.nan
    assert np.isnan(compare.max_err(bad, ref))
