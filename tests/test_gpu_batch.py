"""GPU parity of the batched response (fused persistent forward, batched
adjoint and likelihood, graph capture) against the oracle and the
per-template GPU path."""
import numpy as np
import pytest

import oracle
from paper_2204_06633_amd import inputs, workloads
from tests import cases

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _t(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _build(torch, n_out_list, order=25, gen=2, channels="AET", group=2, adjoint=False, seed=3,
           dt=10.0, tdi_orbit_kind=None, segment=0):
    from paper_2204_06633_amd import native
    grids, params, sp, st = workloads.make_batch(len(n_out_list), "keplerian", n_out_list, dt,
                                                 order, gen, seed, tdi_orbit_kind=tdi_orbit_kind)
    rows = 6 if channels == "XYZAET" else 3
    lay = workloads.batch_layout(grids, rows)
    hp = np.zeros(max(lay.n_h_total, 1))
    hc = np.zeros(max(lay.n_h_total, 1))
    for g, ho, p in zip(grids, lay.h_offsets, params):
        a, b = inputs.gb_polarizations(p, g.waveform_times())
        hp[ho:ho + g.n_h] = a
        hc[ho:ho + g.n_h] = b
    gp = native.Orbits.from_samples(sp)
    gt = gp if st is sp else native.Orbits.from_samples(st)
    batch = native.Batch(lay.templates(), gp, gt, grids[0].t_start, dt, order, gen, channels,
                         group=group, adjoint=adjoint, segment=segment)
    sky = np.ascontiguousarray(params[:, 6:8])
    return dict(batch=batch, lay=lay, grids=grids, params=params, sp=sp, st=st, hp=hp, hc=hc,
                sky=sky, orbs=(gp, gt), order=order, gen=gen, channels=channels)


def _halo_cap(group, tile):
    """TDI halo the fused kernel's rows carry from tile to tile for a group
    and tile length: two values per lane over 6 * group rows, 0 below 32,
    at most 64."""
    c = (tile // (6 * group)) & ~1
    return 0 if c < 32 else min(c, 64)


def _oracle_out(B, k):
    g = B["grids"][k]
    ho = B["lay"].h_offsets[k]
    p = B["params"][k]
    op = oracle.Orbits.from_samples(B["sp"])
    ot = op if B["st"] is B["sp"] else oracle.Orbits.from_samples(B["st"])
    return oracle.response(op, ot, g, B["hp"][ho:ho + g.n_h], B["hc"][ho:ho + g.n_h], p[6], p[7],
                           B["order"], B["gen"], B["channels"])


@pytest.mark.parametrize("group", [1, 2, 4])
@pytest.mark.parametrize("gen,channels", [(2, "AET"), (1, "XYZ"), (2, "XYZAET")])
def test_fused_forward_matches_oracle(torch_cuda, group, gen, channels):
    torch = torch_cuda
    n_out_list = [1500, 0, 977, 1, 2100, 480, 481, 1200, 33]
    B = _build(torch, n_out_list, gen=gen, channels=channels, group=group, seed=group + 10 * gen)
    out = B["batch"].response(_t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"]))
    torch.cuda.synchronize()
    for k, n in enumerate(n_out_list):
        if n == 0:
            continue
        got = B["batch"].output_block(out, k).cpu().numpy()
        cases.check(got, _oracle_out(B, k), TOL, "template %d (%d samples)" % (k, n))


def test_fused_forward_hybrid_orbits_and_order(torch_cuda):
    """Keplerian projection with rigid equal-arm TDI (the paper's hybrid
    template, Sec. V), order 9, dt = 15 s."""
    torch = torch_cuda
    n_out_list = [900, 1300, 640]
    B = _build(torch, n_out_list, order=9, group=2, dt=15.0, tdi_orbit_kind="rigid", seed=21)
    out = B["batch"].response(_t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"]))
    torch.cuda.synchronize()
    for k in range(len(n_out_list)):
        got = B["batch"].output_block(out, k).cpu().numpy()
        cases.check(got, _oracle_out(B, k), TOL, "template %d" % k)


def test_batch_adjoint_and_loglike(torch_cuda):
    """Batched adjoint against the per-template GPU adjoint and the oracle;
    batched likelihood against the oracle."""
    torch = torch_cuda
    from paper_2204_06633_amd import native, response
    n_out_list = [1100, 700, 0, 1500]
    B = _build(torch, n_out_list, group=2, adjoint=True, seed=5)
    batch = B["batch"]
    hp, hc, sky = _t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"])
    out = batch.response(hp, hc, sky)
    rng = np.random.default_rng(1)
    data = out.cpu().numpy() + 1e-24 * rng.standard_normal(out.shape)
    ll, g_out = batch.loglike(out, _t(torch, data), 1e-24)
    ghp, ghc, gsky = batch.adjoint(hp, hc, sky, g_out)
    torch.cuda.synchronize()
    gp, gt = B["orbs"]
    for k, n in enumerate(n_out_list):
        g = B["grids"][k]
        ho, oo = B["lay"].h_offsets[k], B["lay"].out_offsets[k]
        blk = slice(oo, oo + 3 * n)
        ref_ll = oracle.loglike(out.cpu().numpy()[blk], data[blk], 1e-24)
        assert abs(float(ll[k]) - ref_ll) <= 1e-12 * max(abs(ref_ll), 1.0)
        if n == 0:
            assert float(ll[k]) == 0.0 and float(gsky[k, 0]) == 0.0
            continue
        tpl = response.Template(gp, gt, g, 25, 2, "AET")
        hk, ck = hp[ho:ho + g.n_h].contiguous(), hc[ho:ho + g.n_h].contiguous()
        gk = g_out[blk].view(3, n).contiguous()
        rhp, rhc, rsky = response.plain_adjoint(tpl, hk, ck, sky[k].contiguous(), gk)
        got = np.stack([ghp[ho:ho + g.n_h].cpu().numpy(), ghc[ho:ho + g.n_h].cpu().numpy()])
        ref = np.stack([rhp.cpu().numpy(), rhc.cpu().numpy()])
        cases.check(got, ref, 1e-12, "likelihood gradient")
        assert np.allclose(gsky[k].cpu().numpy(), rsky.cpu().numpy(), rtol=1e-12, atol=0)
    # one template against the oracle transpose
    k = 0
    g = B["grids"][k]
    ho, oo, n = B["lay"].h_offsets[k], B["lay"].out_offsets[k], n_out_list[k]
    op = oracle.Orbits.from_samples(B["sp"])
    rhp, rhc = oracle.response_adjoint(op, op, g, B["params"][k][6], B["params"][k][7], 25, 2,
                                       g_out[oo:oo + 3 * n].view(3, n).cpu().numpy(), "AET")
    got = np.stack([ghp[ho:ho + g.n_h].cpu().numpy(), ghc[ho:ho + g.n_h].cpu().numpy()])
    cases.check(got, np.stack([rhp, rhc]), 1e-10, "batch adjoint")


@pytest.mark.parametrize("segment", [0, 3])
def test_graph_capture_replays_match_eager(torch_cuda, segment):
    """Forward, likelihood and adjoint captured in one HIP graph; replays with
    new sky angles and new polarisations match eager calls each time (work
    items of one tile, and of three passing the TDI halo on)."""
    torch = torch_cuda
    n_out_list = [1300, 800, 1000]
    B = _build(torch, n_out_list, group=2, adjoint=True, seed=9, segment=segment)
    batch = B["batch"]
    assert batch.segment == (segment or 1)
    hp, hc, sky = _t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"])
    out = torch.empty(batch.out_extent, dtype=torch.float64, device="cuda")
    data = torch.zeros_like(out)
    ll = torch.empty(batch.n, dtype=torch.float64, device="cuda")
    g_out = torch.zeros_like(out)
    ghp = torch.empty(batch.h_extent, dtype=torch.float64, device="cuda")
    ghc = torch.empty_like(ghp)
    gsky = torch.empty((batch.n, 2), dtype=torch.float64, device="cuda")

    def step():
        batch.response(hp, hc, sky, out=out)
        batch.loglike(out, data, 1e-21, ll=ll, g_out=g_out)
        batch.adjoint(hp, hc, sky, g_out, g_hp=ghp, g_hc=ghc, g_sky=gsky)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                                    # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    rng = np.random.default_rng(4)
    for r in range(4):
        sky.copy_(_t(torch, B["sky"] + 1e-3 * rng.standard_normal(B["sky"].shape)))
        hp.mul_(1.0 + 0.1 * r)
        data.copy_(out * 0.5)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        snap = [x.clone() for x in (out, ll, ghp, ghc, gsky)]
        step()                                    # eager on the same inputs
        torch.cuda.synchronize()
        # every stage sums in a fixed order (the adjoint's carries, tile folds
        # and at most two global additions onto zero per entry): bit for bit
        for k, (a, b) in enumerate(zip(snap, (out, ll, ghp, ghc, gsky))):
            assert torch.equal(a, b), (r, k)


def test_group_tile_and_grid_do_not_change_results(torch_cuda, tmp_path):
    """Each template's arithmetic is the same whatever the group size, the
    persistent grid, the tile length (256, 512, 1024 link samples) and the
    segment length (tiles per work item passing the TDI halo on in LDS;
    templates ending inside a segment, segments cut short by the longest
    template's end): the outputs agree bit for bit; the autotuner returns
    one of the candidates and caches it."""
    torch = torch_cuda
    from paper_2204_06633_amd import autotune, native
    n_out_list = [1200, 300, 2500, 777, 1, 1600]
    B = _build(torch, n_out_list, group=1, seed=17)
    hp, hc, sky = _t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"])
    ref = B["batch"].response(hp, hc, sky).clone()
    gp, gt = B["orbs"]
    tpl = B["lay"].templates()
    t0 = B["grids"][0].t_start
    for g in (1, 2, 4):
        for tile in autotune.TILES:
            if not autotune.variant_exists(g, tile):
                continue
            for seg in (1, 2, 3, 64):
                b = native.Batch(tpl, gp, gt, t0, 10.0, 25, 2, "AET", group=g, tile=tile,
                                 segment=seg)
                assert b.tile == tile
                carries = tile - b.c.tile_out <= _halo_cap(g, tile)
                assert b.segment == (seg if carries else 1), (g, tile, seg, b.segment)
                for blocks in (1, 3, b.blocks, 2 * b.blocks):
                    b.set_grid(blocks)
                    out = b.response(hp, hc, sky)
                    torch.cuda.synchronize()
                    assert torch.equal(out, ref), (g, tile, seg, blocks)
    cache = str(tmp_path / "tune.json")
    r = autotune.tune(tpl, gp, gt, t0, 10.0, 25, 2, "AET", hp, hc, sky, reps=2, cache_path=cache)
    assert r["group"] in autotune.GROUPS and r["grid_scale"] in autotune.GRID_SCALES
    assert autotune.variant_exists(r["group"], r["tile"])
    n_variants = sum(autotune.variant_exists(g, t) for g in autotune.GROUPS for t in autotune.TILES)
    assert len(r["trials"]) == n_variants * len(autotune.GRID_SCALES)
    assert autotune.tune(tpl, gp, gt, t0, 10.0, 25, 2, "AET", hp, hc, sky,
                         cache_path=cache)["tuned_at"] == r["tuned_at"]
    b, _ = autotune.tuned_batch(tpl, gp, gt, t0, 10.0, 25, 2, "AET", hp, hc, sky, cache_path=cache)
    out = b.response(hp, hc, sky)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


@pytest.mark.parametrize("order,dt", [(1, 10.0), (31, 10.0), (25, 0.25)])
def test_fused_forward_orders_and_small_dt(torch_cuda, order, dt):
    """Extreme orders, and dt = 0.25 s, where the projection window of a tile
    no longer fits the LDS window and the fused kernel reads h from global
    memory (TDI still fits)."""
    torch = torch_cuda
    n_out_list = [700, 1500, 1]
    B = _build(torch, n_out_list, order=order, group=2, dt=dt, seed=31 + order)
    out = B["batch"].response(_t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"]))
    torch.cuda.synchronize()
    for k in range(len(n_out_list)):
        got = B["batch"].output_block(out, k).cpu().numpy()
        cases.check(got, _oracle_out(B, k), TOL, "template %d" % k)


def test_batch_adjoint_small_dt_against_oracle(torch_cuda):
    """dt = 0.25 s: the adjoint footprints exceed the LDS tiles, so the paired
    TDI adjoint and the projection adjoint scatter to global memory."""
    torch = torch_cuda
    n_out_list = [900, 400]
    B = _build(torch, n_out_list, group=2, adjoint=True, seed=77, dt=0.25)
    batch = B["batch"]
    hp, hc, sky = _t(torch, B["hp"]), _t(torch, B["hc"]), _t(torch, B["sky"])
    rng = np.random.default_rng(3)
    g_out = _t(torch, rng.standard_normal(batch.out_extent))
    ghp, ghc, _ = batch.adjoint(hp, hc, sky, g_out, want_sky=False)
    torch.cuda.synchronize()
    op = oracle.Orbits.from_samples(B["sp"])
    for k, n in enumerate(n_out_list):
        g = B["grids"][k]
        ho, oo = B["lay"].h_offsets[k], B["lay"].out_offsets[k]
        rhp, rhc = oracle.response_adjoint(op, op, g, B["params"][k][6], B["params"][k][7], 25,
                                           2, g_out[oo:oo + 3 * n].view(3, n).cpu().numpy(),
                                           "AET")
        got = np.stack([ghp[ho:ho + g.n_h].cpu().numpy(), ghc[ho:ho + g.n_h].cpu().numpy()])
        cases.check(got, np.stack([rhp, rhc]), 1e-10, "template %d adjoint" % k)


def test_waveform_mode_forward_and_parameter_adjoint(torch_cuda):
    """lr_response_gb (h+ / hx synthesised in the fused kernel's windows from
    the 8 source parameters) equals lr_gb_polarizations + lr_response bit
    for bit, and the oracle (its own waveform, response) to 1e-11;
    lr_response_adjoint_gb (straight to d/d params) equals the two-step
    chain (lr_response_adjoint to g_h and the sky, lr_gb_polarizations_
    adjoint) to 1e-9 per component and the oracle's chain (transposed
    response, waveform vector-Jacobian product) for the six waveform
    parameters to 1e-9; two runs agree bit for bit.  Uneven templates,
    one empty."""
    torch = torch_cuda
    from oracle import waveform as owf
    from paper_2204_06633_amd import native
    n_out_list = [1300, 0, 777, 2048]
    B = _build(torch, n_out_list, group=2, adjoint=True, seed=23)
    batch = B["batch"]
    params = _t(torch, B["params"])
    gp_, gt_ = B["orbs"]
    # the GPU waveform into the batch's h arrays (waveform time 0 at output 0)
    hp = torch.zeros(max(batch.h_extent, 1), dtype=torch.float64, device="cuda")
    hc = torch.zeros_like(hp)
    for k, g in enumerate(B["grids"]):
        if g.n_out == 0:
            continue
        ho = B["lay"].h_offsets[k]
        a, b = native.gb_polarizations(params[k:k + 1].contiguous(), -g.out_start, g.n_h, g.dt)
        hp[ho:ho + g.n_h] = a[0]
        hc[ho:ho + g.n_h] = b[0]
    sky = params[:, 6:8].contiguous()
    out_ref = batch.response(hp, hc, sky)
    out_gb = batch.response_gb(params)
    torch.cuda.synchronize()
    assert torch.equal(out_gb[:batch.out_extent], out_ref[:batch.out_extent])
    op = oracle.Orbits.from_samples(B["sp"])
    ot = op if B["st"] is B["sp"] else oracle.Orbits.from_samples(B["st"])
    rng = np.random.default_rng(4)
    g_out = torch.zeros_like(out_ref)
    g_out[:batch.out_extent] = _t(torch, rng.standard_normal(batch.out_extent))
    g_par = batch.adjoint_gb(params, g_out)
    g_par2 = batch.adjoint_gb(params, g_out)
    ghp, ghc, gsky = batch.adjoint(hp, hc, sky, g_out)
    torch.cuda.synchronize()
    assert torch.equal(g_par, g_par2)
    for k, g in enumerate(B["grids"]):
        if g.n_out == 0:
            assert torch.all(g_par[k] == 0)
            continue
        ho, oo = B["lay"].h_offsets[k], B["lay"].out_offsets[k]
        two = native.gb_polarizations_adjoint(params[k:k + 1].contiguous(), -g.out_start, g.dt,
                                              ghp[ho:ho + g.n_h][None].contiguous(),
                                              ghc[ho:ho + g.n_h][None].contiguous())[0]
        two[6:8] = gsky[k]
        got = g_par[k].cpu().numpy()
        ref = two.cpu().numpy()
        assert np.all(np.abs(got - ref) <= 1e-9 * np.abs(ref)), (k, got, ref)
        # the oracle: waveform, transposed response, waveform VJP
        p = B["params"][k]
        h_p, h_c = owf.polarizations(p, g.waveform_times())
        out_o = oracle.response(op, ot, g, h_p, h_c, p[6], p[7], 25, 2, "AET")
        cases.check(out_gb[oo:oo + 3 * g.n_out].view(3, g.n_out).cpu().numpy(), out_o, TOL,
                    "template %d waveform-mode forward" % k)
        go = g_out[oo:oo + 3 * g.n_out].view(3, g.n_out).cpu().numpy()
        rhp, rhc = oracle.response_adjoint(op, ot, g, p[6], p[7], 25, 2, go, "AET")
        vjp = owf.polarizations_vjp(p, g.waveform_times(), rhp, rhc)
        assert np.all(np.abs(got[:6] - vjp[:6]) <= 1e-9 * np.abs(vjp[:6])), (k, got, vjp)


def test_waveform_mode_every_compiled_shape_and_the_rest_refused(torch_cuda):
    """Waveform mode is its own kernel variant, compiled for groups of 1 and
    2 at 512 link samples and of 2 at 1024: each of those equals the array
    mode fed with lr_gb_polarizations bit for bit; a batch prepared with
    another shape gets LR_E_UNSUPPORTED from lr_response_gb, before any
    launch."""
    torch = torch_cuda
    from paper_2204_06633_amd import autotune, native
    n_out_list = [900, 1500, 333]
    B = _build(torch, n_out_list, group=1, seed=31)
    params = _t(torch, B["params"])
    gp, gt = B["orbs"]
    tpl = B["lay"].templates()
    hp = torch.zeros(max(B["lay"].n_h_total, 1), dtype=torch.float64, device="cuda")
    hc = torch.zeros_like(hp)
    for k, g in enumerate(B["grids"]):
        ho = B["lay"].h_offsets[k]
        a, b = native.gb_polarizations(params[k:k + 1].contiguous(), -g.out_start, g.n_h, g.dt)
        hp[ho:ho + g.n_h] = a[0]
        hc[ho:ho + g.n_h] = b[0]
    sky = params[:, 6:8].contiguous()
    t0 = B["grids"][0].t_start
    ref = None
    for g in autotune.GROUPS:
        for tile in autotune.TILES:
            if not autotune.variant_exists(g, tile):
                continue
            b = native.Batch(tpl, gp, gt, t0, 10.0, 25, 2, "AET", group=g, tile=tile)
            out = b.response(hp, hc, sky)
            if ref is None:
                ref = out.clone()
            if autotune.variant_exists(g, tile, wave=True):
                out_gb = b.response_gb(params)
                torch.cuda.synchronize()
                assert torch.equal(out_gb[:b.out_extent], ref[:b.out_extent]), (g, tile)
                # segments of several tiles carrying the TDI halo
                b3 = native.Batch(tpl, gp, gt, t0, 10.0, 25, 2, "AET", group=g, tile=tile,
                                  segment=3)
                assert b3.segment == 3
                out_gb = b3.response_gb(params)
                torch.cuda.synchronize()
                assert torch.equal(out_gb[:b.out_extent], ref[:b.out_extent]), (g, tile, 3)
            else:
                with pytest.raises(native.LisaRespError) as e:
                    b.response_gb(params)
                assert e.value.status == native.LR_E_UNSUPPORTED, (g, tile)


@pytest.mark.parametrize("order,gen,group", [(1, 1, 1), (7, 2, 2), (31, 2, 2), (13, 1, 2)])
def test_waveform_mode_other_orders_and_generations(torch_cuda, order, gen, group):
    """The waveform-mode kernel variants of other tap counts and of TDI-1:
    lr_response_gb equals lr_gb_polarizations + lr_response bit for bit,
    and one template against the oracle fed with the oracle's waveform."""
    torch = torch_cuda
    from oracle import waveform as owf
    from paper_2204_06633_amd import native
    channels = "XYZ" if gen == 1 else "AET"
    B = _build(torch, [700, 1234], order=order, gen=gen, channels=channels, group=group,
               seed=40 + order)
    batch = B["batch"]
    params = _t(torch, B["params"])
    hp = torch.zeros(max(batch.h_extent, 1), dtype=torch.float64, device="cuda")
    hc = torch.zeros_like(hp)
    for k, g in enumerate(B["grids"]):
        ho = B["lay"].h_offsets[k]
        a, b = native.gb_polarizations(params[k:k + 1].contiguous(), -g.out_start, g.n_h, g.dt)
        hp[ho:ho + g.n_h] = a[0]
        hc[ho:ho + g.n_h] = b[0]
    out_ref = batch.response(hp, hc, params[:, 6:8].contiguous())
    out_gb = batch.response_gb(params)
    torch.cuda.synchronize()
    assert torch.equal(out_gb[:batch.out_extent], out_ref[:batch.out_extent])
    k = 1
    g = B["grids"][k]
    oo = B["lay"].out_offsets[k]
    p = B["params"][k]
    op = oracle.Orbits.from_samples(B["sp"])
    h_p, h_c = owf.polarizations(p, g.waveform_times())
    ref = oracle.response(op, op, g, h_p, h_c, p[6], p[7], order, gen, channels)
    cases.check(out_gb[oo:oo + 3 * g.n_out].view(3, g.n_out).cpu().numpy(), ref, TOL,
                "waveform mode, order %d, TDI-%d" % (order, gen))


@pytest.mark.parametrize("order,gen,dt,carries", [
    (25, 1, 10.0, True),      # TDI-1: F + B odd, the halo rounded up to even
    (25, 2, 4.3, True),       # halo of 42 samples: exactly what the rows of a 2 x 256 item hold
    (25, 2, 4.0, False),      # halo of 44: one-tile work items
    (31, 2, 10.0, True),
    (1, 2, 10.0, True),
])
def test_segments_at_the_halo_limits(torch_cuda, order, gen, dt, carries):
    """Work items of several tiles (the TDI halo passed on in LDS) equal
    one-tile items bit for bit at other orders, TDI-1 (odd padding) and
    halos at and beyond the kernel's capacity (where the plan falls back to
    one tile), with templates ending inside segments; one template against
    the oracle."""
    torch = torch_cuda
    channels = "XYZ" if gen == 1 else "AET"
    n_out_list = [2600, 1900, 777, 1]
    B1 = _build(torch, n_out_list, order=order, gen=gen, channels=channels, dt=dt, seed=60 + order,
                segment=1)
    B3 = _build(torch, n_out_list, order=order, gen=gen, channels=channels, dt=dt, seed=60 + order,
                segment=3)
    assert B1["batch"].segment == 1
    assert B3["batch"].segment == (3 if carries else 1)
    args = (_t(torch, B1["hp"]), _t(torch, B1["hc"]), _t(torch, B1["sky"]))
    out1 = B1["batch"].response(*args)
    out3 = B3["batch"].response(*args)
    torch.cuda.synchronize()
    n = B1["batch"].out_extent
    assert torch.equal(out1[:n], out3[:n])
    k = 0
    got = B3["batch"].output_block(out3, k).cpu().numpy()
    cases.check(got, _oracle_out(B3, k), TOL, "order %d TDI-%d dt %g" % (order, gen, dt))
