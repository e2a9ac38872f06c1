"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: the 512-template uneven batch (1.0e9 output samples) checked on
sampled outputs of several templates against the oracle (the samples include
the outputs at the fused forward's tile edges, where a tile takes over the
TDI halo of the one before), the 256-walker forward + adjoint against the
oracle on sampled outputs, and checked by the dot-product identity, which
holds at any size."""
import numpy as np
import pytest

import oracle
from paper_2204_06633_amd import workloads
from tests import cases

pytestmark = pytest.mark.gpu


def _with_segment_edges(idx, batch, n_out):
    """The sampled outputs plus those at the fused forward's tile edges in a
    few segments (first, second, middle, last): a segment's first tile has
    T_out outputs, each later tile `tile`, after the halo carried over."""
    T_out, tile, K = int(batch.c.tile_out), batch.tile, batch.segment
    seg_out = T_out + (K - 1) * tile
    n_seg = -(-n_out // seg_out)
    edges = []
    for sg in sorted({0, 1, n_seg // 2, n_seg - 1}):
        base = sg * seg_out
        for t in range(K):
            start = base + (0 if t == 0 else T_out + (t - 1) * tile)
            edges += [start - 1, start, start + 1]
        edges += [base + seg_out - 1]
    edges = [e for e in edges if 0 <= e < n_out]
    return np.unique(np.concatenate([idx, np.array(edges, dtype=idx.dtype)]))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_uneven_batch_512_sampled(torch_cuda):
    torch = torch_cuda
    from paper_2204_06633_amd import autotune, native
    dev = torch.device("cuda:0")
    bc = workloads.uneven_batch_case()
    orb = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    hp, hc = workloads.device_polarizations(bc, dev)
    sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    batch, _ = autotune.tuned_batch(bc.layout.templates(), orb, orb, bc.t0, bc.dt, bc.order,
                                    bc.generation, bc.channels, hp, hc, sky, use_cache=False,
                                    reps=1, max_templates=16)
    assert batch.segment > 1                  # work items carrying the TDI halo
    out = batch.response(hp, hc, sky)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    op = oracle.Orbits.from_samples(bc.orbits_proj)
    durations = [g.n_out for g in bc.grids]
    picks = sorted({0, len(durations) - 1, int(np.argmin(durations)), int(np.argmax(durations)),
                    137, 301})
    for k in picks:
        g = bc.grids[k]
        ho = bc.layout.h_offsets[k]
        case = workloads.Case("uneven_%d" % k, bc.orbits_proj, bc.orbits_tdi, g, bc.params[k],
                              hp[ho:ho + g.n_h].cpu().numpy(), hc[ho:ho + g.n_h].cpu().numpy(),
                              bc.order, bc.generation, bc.channels)
        idx = _with_segment_edges(cases.sample_indices(g.n_out, 40, seed=k, edge=3), batch,
                                  g.n_out)
        ref = cases.oracle_sampled_response(op, op, case, idx)
        got = batch.output_block(out, k)[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
        cases.check(got, ref, 1e-11, str(k))


def test_walkers_256_dot_product(torch_cuda):
    """<g, R v> = <R^T g, v> for random polarisations v and random channel
    gradients g over all 256 one-year walkers (hybrid orbits, dt = 15 s)."""
    torch = torch_cuda
    from paper_2204_06633_amd import native
    dev = torch.device("cuda:0")
    bc = workloads.walker_batch_case()
    orb_p = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    orb_t = native.Orbits.from_samples(bc.orbits_tdi, device=dev)
    sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    batch = native.Batch(bc.layout.templates(), orb_p, orb_t, bc.t0, bc.dt, bc.order,
                         bc.generation, bc.channels, group=2, adjoint=True, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    vp = torch.randn(batch.h_extent, dtype=torch.float64, device=dev, generator=gen)
    vc = torch.randn(batch.h_extent, dtype=torch.float64, device=dev, generator=gen)
    out = batch.response(vp, vc, sky)
    g = torch.randn(batch.out_extent, dtype=torch.float64, device=dev, generator=gen)
    ghp, ghc, _ = batch.adjoint(None, None, sky, g, want_sky=False)
    torch.cuda.synchronize()
    for k in (0, 100, 255):
        _, _, _, n, off = batch.templates[k]
        ho, nh = batch.templates[k][0], batch.templates[k][1]
        lhs = float(torch.dot(g[off:off + 3 * n], out[off:off + 3 * n]))
        rhs = float(torch.dot(ghp[ho:ho + nh], vp[ho:ho + nh]) +
                    torch.dot(ghc[ho:ho + nh], vc[ho:ho + nh]))
        scale = float(torch.linalg.norm(g[off:off + 3 * n]) * torch.linalg.norm(out[off:off + 3 * n]))
        assert abs(lhs - rhs) <= 1e-12 * scale, (k, lhs, rhs)


def _fd_richardson(f, x0, step):
    d1 = (f(x0 + step) - f(x0 - step)) / (2 * step)
    d2 = (f(x0 + step / 2) - f(x0 - step / 2)) / step
    return (4 * d2 - d1) / 3


def test_walkers_256_against_oracle(torch_cuda):
    """The 256-walker forward + adjoint workload at its own shape (1 yr at
    dt = 15 s, order 25, Keplerian projection with rigid equal-arm TDI
    orbits, TDI-2 A/E/T), all walkers in one autotuned fused launch:
      * forward: sampled outputs of four walkers against the oracle;
      * adjoint: a channel gradient that is zero except at those sampled
        outputs, against the oracle's TDI scatter at exactly those outputs
        followed by its projection scatter; every other walker's gradient
        must be exactly zero;
      * sky gradient of the same walkers against central differences of
        the oracle's <g, response(lam, beta)> at the sampled outputs."""
    torch = torch_cuda
    from paper_2204_06633_amd import autotune, native
    dev = torch.device("cuda:0")
    bc = workloads.walker_batch_case()
    orb_p = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    orb_t = native.Orbits.from_samples(bc.orbits_tdi, device=dev)
    hp, hc = workloads.device_polarizations(bc, dev)
    sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    tpl = bc.layout.templates()
    tuned = autotune.tune(tpl, orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                          hp, hc, sky, use_cache=False, reps=1, max_templates=16)
    batch = native.Batch(tpl, orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                         group=tuned["group"], adjoint=True, device=dev)
    batch.set_grid(max(1, int(round(batch.blocks * tuned["grid_scale"]))))
    assert batch.segment > 1
    out = batch.response(hp, hc, sky)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    op = oracle.Orbits.from_samples(bc.orbits_proj)
    ot = oracle.Orbits.from_samples(bc.orbits_tdi)
    picks = (0, 1, 127, 255)
    rng = np.random.default_rng(55)
    g_out = torch.zeros_like(out)
    sel = {}
    for k in picks:
        g = bc.grids[k]
        ho, off = bc.layout.h_offsets[k], bc.layout.out_offsets[k]
        case = workloads.Case("walker_%d" % k, bc.orbits_proj, bc.orbits_tdi, g, bc.params[k],
                              hp[ho:ho + g.n_h].cpu().numpy(), hc[ho:ho + g.n_h].cpu().numpy(),
                              bc.order, bc.generation, bc.channels)
        idx = _with_segment_edges(cases.sample_indices(g.n_out, 150, seed=500 + k, edge=3),
                                  batch, g.n_out)
        ref = cases.sampled_response(op, ot, case, idx)
        got = batch.output_block(out, k)[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
        cases.check(got, ref, 1e-11, "forward walker %d" % k)
        gs = rng.standard_normal((3, idx.size))
        blk = g_out[off:off + 3 * g.n_out].view(3, g.n_out)
        blk[:, torch.from_numpy(idx).to(dev)] = torch.tensor(gs, dtype=torch.float64, device=dev)
        sel[k] = (case, idx, gs)
    ghp, ghc, gsky = batch.adjoint(hp, hc, sky, g_out)
    torch.cuda.synchronize()
    mask = torch.ones(batch.h_extent, dtype=torch.bool, device=dev)
    gsky_np = gsky.cpu().numpy()
    for k, (case, idx, gs) in sel.items():
        g = case.grid
        ho = bc.layout.h_offsets[k]
        mask[ho:ho + g.n_h] = False
        rhp, rhc = cases.sampled_adjoint(op, ot, case, idx, gs)
        got = np.stack([ghp[ho:ho + g.n_h].cpu().numpy(), ghc[ho:ho + g.n_h].cpu().numpy()])
        cases.check(got, np.stack([rhp, rhc]), 1e-10, "adjoint walker %d" % k)

        def J(lam, beta, case=case, idx=idx, gs=gs):
            c = workloads.Case(case.name, case.orbits_proj, case.orbits_tdi, case.grid,
                               np.concatenate([case.params[:6], [lam, beta]]), case.hp, case.hc,
                               case.order, case.generation, case.channels)
            return float(np.sum(cases.sampled_response(op, ot, c, idx) * gs))

        fd_lam = _fd_richardson(lambda x: J(x, case.beta), case.lam, 1e-4)
        fd_beta = _fd_richardson(lambda x: J(case.lam, x), case.beta, 1e-4)
        assert abs(gsky_np[k, 0] - fd_lam) <= 1e-6 * abs(fd_lam), (k, gsky_np[k, 0], fd_lam)
        assert abs(gsky_np[k, 1] - fd_beta) <= 1e-6 * abs(fd_beta), (k, gsky_np[k, 1], fd_beta)
    rest = [k for k in range(batch.n) if k not in sel]
    assert float(ghp[mask].abs().max()) == 0.0 and float(ghc[mask].abs().max()) == 0.0
    assert np.all(gsky_np[rest] == 0.0)


def test_walkers_256_keplerian_waveform_mode_against_oracle(torch_cuda):
    """The walker workload with the full generic response (Keplerian orbits
    for the projection and the TDI delays) in waveform mode, all 256 walkers
    in one launch at the tuned waveform-mode shape:
      * forward (h+ / hx synthesised in the fused kernel): sampled outputs of
        two walkers against the oracle fed with the oracle's own waveform;
      * gradient to the 8 parameters (lr_response_adjoint_gb) of a channel
        gradient that is zero except at those outputs: the six waveform
        parameters against the oracle's transposed response at exactly those
        outputs followed by the waveform's vector-Jacobian product, the sky
        angles against central differences of the oracle's <g, response>;
        every other walker's gradient exactly zero."""
    torch = torch_cuda
    from oracle import waveform as owf
    from paper_2204_06633_amd import autotune, native
    dev = torch.device("cuda:0")
    bc = workloads.walker_batch_case(tdi_orbit_kind="keplerian")
    assert bc.orbits_tdi is bc.orbits_proj
    orb = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    params = torch.tensor(bc.params, dtype=torch.float64, device=dev).contiguous()
    tpl = bc.layout.templates()
    tuned = autotune.tune(tpl, orb, orb, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                          None, None, None, params=params, use_cache=False, reps=1,
                          max_templates=16)
    assert autotune.variant_exists(tuned["group"], tuned["tile"], wave=True)
    batch = native.Batch(tpl, orb, orb, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                         group=tuned["group"], tile=tuned["tile"], adjoint=True, device=dev)
    batch.set_grid(max(1, int(round(batch.blocks * tuned["grid_scale"]))))
    assert batch.segment > 1
    out = batch.response_gb(params)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    op = oracle.Orbits.from_samples(bc.orbits_proj)
    rng = np.random.default_rng(77)
    g_out = torch.zeros_like(out)
    sel = {}
    for k in (3, 200):
        g = bc.grids[k]
        off = bc.layout.out_offsets[k]
        hp_o, hc_o = owf.polarizations(bc.params[k], g.waveform_times())
        case = workloads.Case("walker_%d" % k, bc.orbits_proj, bc.orbits_tdi, g, bc.params[k],
                              hp_o, hc_o, bc.order, bc.generation, bc.channels)
        idx = _with_segment_edges(cases.sample_indices(g.n_out, 120, seed=700 + k, edge=3),
                                  batch, g.n_out)
        ref = cases.sampled_response(op, op, case, idx)
        got = batch.output_block(out, k)[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
        cases.check(got, ref, 1e-11, "waveform-mode forward walker %d" % k)
        gs = rng.standard_normal((3, idx.size))
        blk = g_out[off:off + 3 * g.n_out].view(3, g.n_out)
        blk[:, torch.from_numpy(idx).to(dev)] = torch.tensor(gs, dtype=torch.float64, device=dev)
        sel[k] = (case, idx, gs)
    g_par = batch.adjoint_gb(params, g_out).cpu().numpy()
    for k, (case, idx, gs) in sel.items():
        g = case.grid
        rhp, rhc = cases.sampled_adjoint(op, op, case, idx, gs)
        vjp = owf.polarizations_vjp(case.params, g.waveform_times(), rhp, rhc)
        assert np.all(np.abs(g_par[k, :6] - vjp[:6]) <= 1e-9 * np.abs(vjp[:6])), \
            (k, g_par[k], vjp)

        def J(lam, beta, case=case, idx=idx, gs=gs):
            c = workloads.Case(case.name, case.orbits_proj, case.orbits_tdi, case.grid,
                               np.concatenate([case.params[:6], [lam, beta]]), case.hp, case.hc,
                               case.order, case.generation, case.channels)
            return float(np.sum(cases.sampled_response(op, op, c, idx) * gs))

        fd_lam = _fd_richardson(lambda x: J(x, case.beta), case.lam, 1e-4)
        fd_beta = _fd_richardson(lambda x: J(case.lam, x), case.beta, 1e-4)
        assert abs(g_par[k, 6] - fd_lam) <= 1e-6 * abs(fd_lam), (k, g_par[k, 6], fd_lam)
        assert abs(g_par[k, 7] - fd_beta) <= 1e-6 * abs(fd_beta), (k, g_par[k, 7], fd_beta)
    rest = [k for k in range(batch.n) if k not in sel]
    assert np.all(g_par[rest] == 0.0)
