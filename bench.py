#!/usr/bin/env python
"""Benchmark of the generic LISA time-domain response on one MI355X.

Headline workload (the largest single-GPU configuration): 512 Galactic-binary
templates of uneven durations (uniform 0.25-1 yr at dt = 10 s, 1.01e9 output
samples in all), independent seeded sky positions and source parameters,
flexing Keplerian orbits shared by all, Lagrange order 25, TDI-2 A/E/T, FP64.
One step = one batched forward (lr_response: the persistent fused projection
+ TDI kernel over the whole batch), replayed from a captured HIP graph with
the autotuned group and grid; inputs resident in HBM.  Throughput counts
templates x 6 links x time samples per second.

The JSON line carries, beside the headline:
  roofline            the fused kernel against the FP64 vector issue peak
                      (algorithmic lane-ops per launch / its mean event time)
  plain_per_template  the per-template forward (lr_project_links then
                      lr_tdi_combine) on 8 templates of the same batch
  walkers             256 MCMC walkers, 1 yr at dt = 15 s, Keplerian
                      projection with rigid equal-arm TDI orbits: forward +
                      likelihood + adjoint (gradients to h+, hx and the sky
                      angles) in one captured graph, with its roofline
  single_template     one 1-yr template: plain forward, forward + adjoint,
                      the TDI adjoint kernel's roofline, the Lagrange order
                      sweep 1..25 (Sec. IV.E), the batch-of-one fused path
  fd_likelihood, orbit_models, gradient_step, sampler
                      the widened rows (frequency-domain likelihood, orbit
                      models of Sec. V, the 8-parameter gradient, the
                      tempered sampler)
  cpu_baseline        the CPU oracle on bounded samples of the headline and
                      walker workloads, at all host cores and at one thread,
                      with the parity of the timed GPU outputs on the same
                      samples

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--headline-only]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("response samples/s (templates×links×time) fwd & fwd+adjoint at 1e-11 rel "
          "err; % HBM peak")
UNIT = "samples/s (templates×links×time)"


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_source_hash(names):
    """Hash of the kernel sources a recorded counter summary belongs to."""
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_2204_06633_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


FUSED_SOURCES = ("device_common.hpp", "forward_kernels.hpp", "batch_kernels.hpp",
                 "batch_types.hpp", "gb_device.hpp")


def recorded_traffic(name, sources):
    """HBM bytes per launch from a committed rocprofv3 counter record
    (profiles/traffic_<name>.json), or None if there is none for the current
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash(sources):
        return None
    return rec.get("bytes_per_launch")


def _timed(fn, steps, warmup):
    """Mean milliseconds of fn() over `steps` calls after `warmup`, from HIP
    events recorded on the current stream (the stream the library launches
    on), bracketed by device synchronisations."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[steps]) / steps


def _capture(fn):
    """fn() captured in a HIP graph (after one eager run on a side stream)."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    return graph


def _roofline(lane_ops, ms, kernel, traffic=None, algorithmic_bytes=None):
    from paper_2204_06633_amd import costs
    achieved = lane_ops / (ms * 1e-3)
    r = {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e12,
         "peak": costs.LANE_OPS_PEAK / 1e12, "unit": "T FP64 lane-op/s",
         "frac": achieved / costs.LANE_OPS_PEAK, "traffic": traffic,
         "lane_ops_per_launch": lane_ops, "ms_per_launch": ms}
    if algorithmic_bytes is not None:
        r["algorithmic_bytes"] = algorithmic_bytes
        r["hbm_GBps"] = algorithmic_bytes / (ms * 1e-3) / 1e9
        r["hbm_frac"] = algorithmic_bytes / (ms * 1e-3) / costs.HBM_PEAK
        if traffic:
            r["traffic_over_algorithmic"] = traffic / algorithmic_bytes
    return r


# ---------------------------------------------------------------------------
# Headline: the 512-template uneven batch, fused forward from a captured graph
# ---------------------------------------------------------------------------

def bench_headline(steps, warmup, keep):
    import numpy as np
    import torch

    from paper_2204_06633_amd import autotune, costs, native, response, workloads
    dev = torch.device("cuda:0")
    bc = workloads.uneven_batch_case()
    log("headline: %s, %d templates, %d output samples" % (bc.name, len(bc.grids),
                                                           bc.n_samples))
    orb = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    hp, hc = workloads.device_polarizations(bc, dev)
    sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    tpl = bc.layout.templates()
    batch, tuned = autotune.tuned_batch(tpl, orb, orb, bc.t0, bc.dt, bc.order, bc.generation,
                                        bc.channels, hp, hc, sky)
    log("autotuned: group %d, tile %d, grid x%.1f (%d work-groups)"
        % (tuned["group"], batch.tile, tuned["grid_scale"], batch.blocks))
    out = torch.empty(batch.out_extent, dtype=torch.float64, device=dev)
    graph = _capture(lambda: batch.response(hp, hc, sky, out=out))
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        graph.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_launch = ev[0].elapsed_time(ev[steps]) / steps
    ms_step = wall / steps * 1e3
    n = bc.n_samples

    # plain per-template forward (project_links then tdi_combine) on 8
    # templates of the same batch
    pick = list(range(0, len(bc.grids), len(bc.grids) // 8))[:8]
    n_plain, ms_plain = 0, 0.0
    for k in pick:
        g = bc.grids[k]
        ho = bc.layout.h_offsets[k]
        t = response.Template(orb, orb, g, bc.order, bc.generation, bc.channels)
        hk, ck = hp[ho:ho + g.n_h], hc[ho:ho + g.n_h]
        y = torch.empty((6, g.n_y), dtype=torch.float64, device=dev)
        o = torch.empty((3, g.n_out), dtype=torch.float64, device=dev)
        ms_plain += _timed(lambda: response.plain_forward(t, hk, ck, sky[k], y=y, out=o),
                           max(2, steps // 2), 1)
        n_plain += g.n_out
    plain_rate = 6.0 * n_plain / (ms_plain * 1e-3)
    rate = 6.0 * n / (ms_step * 1e-3)

    group = tuned["group"]
    ops = costs.lane_ops_fused_forward(bc.grids, bc.order, bc.generation, group)
    nbytes = costs.batch_bytes(bc.grids, 3)
    traffic = recorded_traffic("fused_forward_batch512", FUSED_SOURCES)
    kernel = "fused_forward_kernel<26,2,%d,%d>" % (group, batch.tile // 2)
    roof = _roofline(ops, ms_launch, kernel, traffic, nbytes)
    roof["note"] = ("mean HIP-event time of the graph replay on the launch stream (the "
                    "preparation kernel (work counter, sky trigonometry; a few us) and the fused "
                    "kernel)")

    # keep what the CPU baseline compares: the sampled templates' inputs and
    # outputs, on the host
    for k in keep:
        g = bc.grids[k]
        ho = bc.layout.h_offsets[k]
        keep[k] = dict(hp=hp[ho:ho + g.n_h].cpu().numpy(), hc=hc[ho:ho + g.n_h].cpu().numpy(),
                       out=batch.output_block(out, k).cpu().numpy())
    del graph, out, hp, hc
    res = {"workload": bc.name, "templates": len(bc.grids), "time_samples": n,
           "value": rate, "ms_per_step": ms_step, "ms_per_launch_events": ms_launch,
           "group": group, "tile": batch.tile, "segment": batch.segment,
           "grid_scale": tuned["grid_scale"],
           "blocks": batch.blocks,
           "roofline": roof,
           "plain_per_template": {"value": plain_rate, "unit": UNIT, "templates_timed": len(pick),
                                  "time_samples": n_plain, "ms": ms_plain,
                                  "fused_speedup": rate / plain_rate}}
    return res, bc


# ---------------------------------------------------------------------------
# Walkers: forward + likelihood + adjoint of 256 one-year walkers
# ---------------------------------------------------------------------------

def bench_walkers(steps, warmup, keep, tdi_orbit_kind="rigid"):
    """256 one-year walkers at dt = 15 s in waveform mode: each walker's h+ /
    hx synthesised inside the fused kernel from its 8 source parameters
    (lr_response_gb), the A/E/T likelihood, and the adjoint down to the 8
    parameters (lr_response_adjoint_gb): no h or h-gradient arrays.  TDI
    delays from rigid equal-arm orbits (hybrid template) or, with
    tdi_orbit_kind="keplerian", from the same flexing orbits as the
    projection (the full generic response)."""
    import torch

    from paper_2204_06633_amd import autotune, costs, native, workloads
    dev = torch.device("cuda:0")
    bc = workloads.walker_batch_case(tdi_orbit_kind=tdi_orbit_kind)
    log("walkers: %s, %d walkers, %d samples" % (bc.name, len(bc.grids), bc.n_samples))
    orb_p = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    orb_t = native.Orbits.from_samples(bc.orbits_tdi, device=dev)
    params = torch.tensor(bc.params, dtype=torch.float64, device=dev).contiguous()
    tpl = bc.layout.templates()
    tuned = autotune.tune(tpl, orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                          None, None, None, params=params)
    batch = native.Batch(tpl, orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                         group=tuned["group"], tile=tuned.get("tile", 0), adjoint=True,
                         device=dev)
    batch.set_grid(max(1, int(round(batch.blocks * tuned["grid_scale"]))))
    out = torch.empty(batch.out_extent, dtype=torch.float64, device=dev)
    # data: walker 0's response plus white noise (sigma = 1e-21), one copy per
    # walker block
    batch.response_gb(params, out=out)
    sigma = 1e-21
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    blk = batch.output_block(out, 0).reshape(-1)
    one = blk + sigma * torch.randn(blk.shape, dtype=torch.float64, device=dev, generator=gen)
    data = one.repeat(len(bc.grids))
    del one
    ll = torch.empty(batch.n, dtype=torch.float64, device=dev)
    g_out = torch.empty_like(out)
    g_par = torch.empty_like(params)

    def step():
        batch.response_gb(params, out=out)
        batch.loglike(out, data, sigma, ll=ll, g_out=g_out)
        batch.adjoint_gb(params, g_out, g_params=g_par)

    graph = _capture(step)
    ms = _timed(graph.replay, steps, warmup)
    ms_fwd = _timed(lambda: batch.response_gb(params, out=out), steps, 1)
    ms_like = _timed(lambda: batch.loglike(out, data, sigma, ll=ll, g_out=g_out), steps, 1)
    ms_adj = _timed(lambda: batch.adjoint_gb(params, g_out, g_params=g_par), steps, 1)
    n = bc.n_samples
    finite = bool(torch.isfinite(ll).all()) and bool(torch.isfinite(g_par).all())
    ops = costs.lane_ops_fwd_adjoint(bc.grids, bc.order, bc.generation, tuned["group"], 2)
    ops_adj = ops - costs.lane_ops_fused_forward(bc.grids, bc.order, bc.generation,
                                                 tuned["group"])
    nbytes = costs.fwd_adjoint_step_bytes_gb(bc.grids, 3)
    for k in keep:
        g = bc.grids[k]
        keep[k] = dict(params=bc.params[k], out=batch.output_block(out, k).cpu().numpy())
    del graph, out, data, g_out
    return {"workload": bc.name, "templates": len(bc.grids), "time_samples": n,
            "value": 6.0 * n / (ms * 1e-3), "unit": UNIT, "ms_per_step": ms,
            "steps": steps, "graph": True, "group": tuned["group"], "tile": batch.tile,
            "segment": batch.segment,
            "stage_ms": {"forward": ms_fwd, "likelihood": ms_like, "adjoint": ms_adj},
            "step_over_forward": ms / ms_fwd, "gradients_finite": finite,
            "roofline": _roofline(ops, ms, "whole step (fused forward with in-kernel waveform, "
                                           "likelihood, TDI adjoint, projection adjoint to the "
                                           "parameter sums, sky gradient)", None, nbytes),
            "roofline_adjoint": _roofline(ops_adj, ms_adj, "lr_response_adjoint_gb (all its "
                                                           "kernels)"),
            "step": "lr_response_gb -> lr_batch_loglike (A/E/T, sigma 1e-21) -> "
                    "lr_response_adjoint_gb (d log L / d 8 source parameters per walker) in "
                    "one HIP graph; no h+/hx or h-gradient arrays"}, bc


# ---------------------------------------------------------------------------
# One 1-yr template: plain forward, adjoint, TDI adjoint roofline, order sweep
# ---------------------------------------------------------------------------

def bench_single_template(steps):
    import numpy as np
    import torch

    from paper_2204_06633_amd import costs, native, response, workloads
    dev = torch.device("cuda:0")
    case = workloads.year_case("XYZAET")
    g = case.grid
    log("single template: %s, %d samples" % (case.name, g.n_out))
    orb = native.Orbits.from_samples(case.orbits_proj, device=dev)
    hp = torch.tensor(case.hp, dtype=torch.float64, device=dev)
    hc = torch.tensor(case.hc, dtype=torch.float64, device=dev)
    y = torch.empty((6, g.n_y), dtype=torch.float64, device=dev)
    out = torch.empty((6, g.n_out), dtype=torch.float64, device=dev)
    t0_y = g.t0_h + g.y_start * g.dt
    sky = torch.tensor([case.lam, case.beta], dtype=torch.float64, device=dev)

    def proj(order=case.order):
        native.project_links(orb, g.t0_h, g.dt, hp, hc, sky, order, g.y_start, g.n_y, y=y)

    def tdi(order=case.order):
        native.tdi_combine(orb, t0_y, g.dt, y, case.generation, order, case.channels,
                           g.front_tdi, g.n_out, out=out)

    ms_proj = _timed(proj, steps, 2)
    ms_tdi = _timed(tdi, steps, 2)
    ms_fwd = _timed(lambda: (proj(), tdi()), steps, 2)
    n = g.n_out
    ops_tdi = costs.lane_ops_tdi(case.order, case.generation) * n
    ops_proj = costs.lane_ops_projection(case.order) * g.n_y
    res = {"workload": case.name, "time_samples": n,
           "forward": {"value": 6.0 * n / (ms_fwd * 1e-3), "unit": UNIT, "ms": ms_fwd,
                       "step": "lr_project_links then lr_tdi_combine (TDI-2 XYZ+AET)"},
           "roofline_tdi": _roofline(ops_tdi, ms_tdi, "tdi_kernel<26,2>",
                                     recorded_traffic("tdi_1yr", ("device_common.hpp",
                                                                  "forward_kernels.hpp")),
                                     costs.tdi_bytes_per_sample(case.channels) * n),
           "roofline_projection": _roofline(ops_proj, ms_proj, "project_links_kernel<26>", None,
                                            costs.projection_bytes_per_sample() * g.n_y)}

    # the TDI adjoint alone (zero fill of g_y, then the scatter kernel)
    g_out = torch.randn(out.shape, dtype=torch.float64, device=dev,
                        generator=torch.Generator(device=dev).manual_seed(3))
    g_y = torch.empty_like(y)
    ms_tadj = _timed(lambda: native.tdi_adjoint(orb, t0_y, g.dt, g.n_y, case.generation,
                                                case.order, case.channels, g.front_tdi, g_out,
                                                g_y=g_y), steps, 2)
    res["roofline_tdi_adjoint"] = _roofline(ops_tdi, ms_tadj, "tdi_adjoint_carry_kernel<26,2> "
                                            "(with the zero fill of g_y)")
    res["roofline_tdi_adjoint"]["over_forward_tdi"] = ms_tadj / ms_tdi

    # forward + likelihood + adjoint of the template (A/E/T rows)
    tpl = response.Template(orb, orb, g, case.order, case.generation, case.channels)
    data = out[3:].clone()
    ll_buf = torch.empty(1, dtype=torch.float64, device=dev)
    g_buf = torch.zeros_like(out)
    work = torch.empty(native.lib().lr_loglike_workspace() // 8, dtype=torch.float64, device=dev)

    def fwd_adj():
        response.plain_forward(tpl, hp, hc, sky, y=y, out=out)
        native.loglike(out[3:], data, 1e-21, out=ll_buf, g_h=g_buf[3:], work=work)
        response.plain_adjoint(tpl, hp, hc, sky, g_buf)

    ms_fa = _timed(fwd_adj, max(3, steps // 2), 1)
    res["fwd_adjoint"] = {"value": 6.0 * n / (ms_fa * 1e-3), "unit": UNIT, "ms": ms_fa,
                          "step": "forward, white-noise likelihood over A/E/T with gradient, "
                                  "adjoint to h+, hx and (lam, beta)"}

    # Lagrange order sweep (Sec. IV.E: the order changes the time by a factor
    # of order unity on the paper's GPU); the padding of order 25 serves all
    sweep = []
    for order in range(1, 26, 2):
        mp = _timed(lambda: proj(order), max(3, steps // 2), 1)
        mt = _timed(lambda: tdi(order), max(3, steps // 2), 1)
        sweep.append({"order": order, "projection_ms": mp, "tdi_ms": mt, "forward_ms": mp + mt,
                      "value": 6.0 * n / ((mp + mt) * 1e-3)})
    base = sweep[0]["forward_ms"]
    for s in sweep:
        s["over_order1"] = s["forward_ms"] / base
    res["order_sweep"] = sweep

    # the same template as a batch of one (fused kernel)
    one = native.Batch([(0, g.n_h, g.out_start, g.n_out, 0)], orb, orb, g.t_start, g.dt,
                       case.order, case.generation, case.channels, group=1, device=dev)
    out1 = torch.empty(one.out_extent, dtype=torch.float64, device=dev)
    ms_one = _timed(lambda: one.response(hp, hc, sky.view(1, 2), out=out1), steps, 2)
    res["fused_single"] = {"value": 6.0 * n / (ms_one * 1e-3), "unit": UNIT, "ms": ms_one,
                           "step": "lr_response on a batch of one (group 1)"}
    del out1, g_y, g_out
    return res, dict(case=case, orb=orb, hp=hp, hc=hc, out=out, y=y, g_buf=g_buf, data=data)


# ---------------------------------------------------------------------------
# Widened rows: frequency-domain likelihood, orbit models, parameter gradient,
# tempered sampler
# ---------------------------------------------------------------------------

def bench_widened(steps, st):
    import numpy as np
    import torch

    from paper_2204_06633_amd import costs, inputs, native, orbitfit, response, waveform, \
        workloads
    dev = torch.device("cuda:0")
    case, orb, hp, hc, out, y, g_buf, data = (st[k] for k in ("case", "orb", "hp", "hc", "out",
                                                              "y", "g_buf", "data"))
    g = case.grid
    n = g.n_out
    sky = torch.tensor([case.lam, case.beta], dtype=torch.float64, device=dev)
    tpl = response.Template(orb, orb, g, case.order, case.generation, case.channels)
    res = {}

    log("frequency-domain likelihood")
    n_fft = native.fd_length(n)
    w_ae, w_t = inputs.noise_weights(n_fft, g.dt)
    w_ae_d = torch.tensor(w_ae, dtype=torch.float64, device=dev)
    w_t_d = torch.tensor(w_t, dtype=torch.float64, device=dev)
    plan = native.FdPlan(data, w_ae_d, w_t_d, g.dt)
    fd_stats = torch.empty((1, 3), dtype=torch.float64, device=dev)

    def fd_fwd_adj():
        response.plain_forward(tpl, hp, hc, sky, y=y, out=out)
        plan.loglike(out[3:], stats=fd_stats, g_h=g_buf[3:])
        response.plain_adjoint(tpl, hp, hc, sky, g_buf)

    ms_fd_fa = _timed(fd_fwd_adj, max(3, steps // 2), 1)
    ms_fd = _timed(lambda: plan.loglike(out[3:], stats=fd_stats, g_h=g_buf[3:]), steps, 2)
    ms_fd_stats = _timed(lambda: plan.loglike(out[3:], want_grad=False, stats=fd_stats),
                         steps, 2)
    fd_b = costs.fd_bytes(n, n_fft, 3, plan.passes, True)
    fd_b_stats = costs.fd_bytes(n, n_fft, 3, plan.passes, False)
    res["fd_likelihood"] = {"ms": ms_fd, "ms_stats_only": ms_fd_stats, "n_fft": n_fft,
                            "bytes": fd_b, "hbm_GBps": fd_b / (ms_fd * 1e-3) / 1e9,
                            "hbm_frac": fd_b / (ms_fd * 1e-3) / costs.HBM_PEAK,
                            "hbm_frac_stats_only": fd_b_stats / (ms_fd_stats * 1e-3) /
                            costs.HBM_PEAK,
                            "fwd_adjoint_ms": ms_fd_fa,
                            "step": "lr_fd_loglike on the 1-yr template's A/E/T: <d-h|d-h>, "
                                    "<h|h>, <d|h> with the stand-in noise curve and d logL/dh"}
    del plan

    log("orbit configurations ESA / EQ / ESAEQ / EQESA")
    oc = workloads.orbit_config_case(n, g.dt)
    oc_orb = {"acc": native.Orbits.from_samples(oc.accurate, device=dev),
              "eq": native.Orbits.from_samples(oc.equal_arm, device=dev)}
    oc_cfg = orbitfit.configurations("acc", "eq")
    oc_names = list(oc_cfg)
    oc_tpl = [response.Template(oc_orb[oc_cfg[k][0]], oc_orb[oc_cfg[k][1]], oc.grid, oc.order,
                                oc.generation, "AET") for k in oc_names]
    oc_hp = torch.tensor(oc.hp, dtype=torch.float64, device=dev)
    oc_hc = torch.tensor(oc.hc, dtype=torch.float64, device=dev)
    oc_sky = torch.tensor(oc.params[6:8], dtype=torch.float64, device=dev)
    oc_h = torch.empty((4, 3, oc.grid.n_out), dtype=torch.float64, device=dev)
    oc_y = torch.empty((6, oc.grid.n_y), dtype=torch.float64, device=dev)
    oc_stats = torch.empty((4, 3), dtype=torch.float64, device=dev)
    for k, tp in enumerate(oc_tpl):
        response.plain_forward(tp, oc_hp, oc_hc, oc_sky, y=oc_y, out=oc_h[k])
    oc_plan = native.FdPlan(oc_h[0].clone(), w_ae_d, w_t_d, g.dt, max_batch=4)

    def orbit_step():
        for k, tp in enumerate(oc_tpl):
            response.plain_forward(tp, oc_hp, oc_hc, oc_sky, y=oc_y, out=oc_h[k])
        oc_plan.loglike(oc_h, want_grad=False, stats=oc_stats)

    ms_orb = _timed(orbit_step, max(3, steps // 4), 1)
    oc_st = oc_stats.cpu().numpy()
    oc_diag = orbitfit.overlap_statistics(oc_st, ss=oc_st[0, 1])
    # fitting factor (Sec. II.A): Nelder-Mead on the GPU likelihood from the
    # injection, per approximate orbit model, against the accurate-orbit data
    from paper_2204_06633_amd import sampler as smp
    th0 = smp.to_theta(torch.tensor(oc.params)).numpy()
    step = np.array([1e-3, 1e-6, 1e-18, 1e-3, 1e-3, 1e-3, 1e-4, 1e-4])
    ff = {}
    t_ff = time.perf_counter()
    for name in ("EQ", "ESAEQ", "EQESA"):
        p, t = oc_cfg[name]
        sc = orbitfit.TemplateScorer(oc_orb[p], oc_orb[t], oc.grid, oc_h[0].clone(), w_ae_d,
                                     w_t_d, order=oc.order)
        r = orbitfit.fitting_factor(sc, th0, step, maxfev=1500)
        ff[name] = {"fitting_factor": r["fitting_factor"], "overlap_at_injection":
                    r["overlap_start"], "loglike_at_injection": r["loglike_start"],
                    "loglike_at_maximum": r["loglike"], "evaluations": r["nfev"]}
        del sc
    res["orbit_models"] = {
        "ms_per_step": ms_orb, "eq_fit_lam1_m1": list(oc.eq_params),
        "step": "4 templates (orbit models) forward + frequency-domain statistics against the "
                "accurate-orbit data, 1 yr",
        "mismatch": {k: float(oc_diag["mismatch"][i]) for i, k in enumerate(oc_names)},
        "rho_opt": {k: float(oc_diag["rho_opt"][i]) for i, k in enumerate(oc_names)},
        "fitting_factor": ff, "fitting_factor_seconds": time.perf_counter() - t_ff}
    del oc_plan, oc_h, oc_y, oc_orb

    # the differentiation step: the paper's Fig. 3 binary, data = injection +
    # white noise sigma = 1e-21; 8 source parameters -> polarisations (HIP
    # kernel) -> response -> A/E/T likelihood -> adjoints -> parameters
    log("likelihood gradient with respect to the source parameters")
    tpl_aet = response.Template(orb, orb, g, case.order, case.generation, "AET")
    theta = torch.tensor(inputs.PAPER_FIG3_BINARY, dtype=torch.float64, device=dev)
    with torch.no_grad():
        hp0, hc0 = response.gb_polarizations(theta[None], -g.out_start, g.n_h, g.dt)
        inj, _ = response.plain_forward(tpl_aet, hp0[0].contiguous(), hc0[0].contiguous(),
                                        theta[6:8].contiguous())
        gen = torch.Generator(device=dev)
        gen.manual_seed(4)
        data_aet = inj + 1e-21 * torch.randn(inj.shape, dtype=torch.float64, device=dev,
                                             generator=gen)
        del hp0, hc0, inj

    def grad_step_hip():
        p = theta.clone().requires_grad_(True)
        hp_, hc_ = response.gb_polarizations(p[None], -g.out_start, g.n_h, g.dt)
        ll = response.loglike(response.response(tpl_aet, hp_[0], hc_[0], p[6:8]), data_aet,
                              1e-21)
        ll.backward()
        return p.grad

    t_w = torch.tensor(g.waveform_times(), dtype=torch.float64, device=dev)

    def grad_step_torch():
        p = theta.clone().requires_grad_(True)
        hp_, hc_ = waveform.gb_polarizations(p, t_w)
        ll = response.loglike(response.response(tpl_aet, hp_, hc_, p[6:8]), data_aet, 1e-21)
        ll.backward()
        return p.grad

    ms_grad = _timed(grad_step_hip, max(3, steps // 2), 1)
    ms_grad_torch = _timed(grad_step_torch, max(3, steps // 2), 1)
    g_h, g_t = grad_step_hip(), grad_step_torch()
    res["gradient_step"] = {"value": 6.0 * n / (ms_grad * 1e-3), "unit": UNIT, "ms": ms_grad,
                            "step": "8 source parameters -> h+, hx (lr_gb_polarizations) -> "
                                    "response (A/E/T) -> likelihood -> adjoints -> parameters",
                            "gradient_finite": bool(torch.isfinite(g_h).all()),
                            "ms_torch_waveform": ms_grad_torch,
                            "hip_vs_torch_waveform_rel_diff":
                                float(((g_h - g_t).abs() / g_t.abs().clamp_min(1e-300)).max())}
    del data_aet, t_w
    torch.cuda.empty_cache()

    log("tempered sampler")
    from paper_2204_06633_amd import sampler
    sc = workloads.sampler_case()
    run = sampler.setup_run(sc, device="cuda:0", log=log)
    run.step()                                                         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc_tot = torch.zeros(sc.T, dtype=torch.int64, device="cuda:0")
    sampler_steps = 3
    for _ in range(sampler_steps):
        acc, _ = run.step()
        acc_tot += acc
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / sampler_steps * 1e3
    evals = 2 * sc.m
    res["sampler"] = {"workload": sc.name, "temperatures": sc.T, "walkers_per_temperature": sc.W,
                      "group": run.tuned["group"], "time_samples": sc.grid.n_out,
                      "ms_per_step": ms, "steps": sampler_steps,
                      "likelihood_evals_per_s": evals / (ms * 1e-3),
                      "value": evals * 6.0 * sc.grid.n_out / (ms * 1e-3), "unit": UNIT,
                      "acceptance_per_temperature":
                          (acc_tot.float() / (sampler_steps * sc.W)).tolist(),
                      "step": "tempered stretch move over 4 x 50 walkers: per half step one "
                              "captured graph of lr_response_gb (waveform synthesised in the "
                              "fused kernel) -> lr_fd_loglike (statistics), then tempering "
                              "swaps"}
    return res


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on bounded samples of the same workloads
# ---------------------------------------------------------------------------

def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_block(op, ot, case, p0, m):
    """Oracle forward of m contiguous outputs from p0: the link samples those
    outputs' TDI stencils read, then TDI.  Returns the channels [3][m]."""
    import numpy as np

    import oracle
    g = case.grid
    ys = np.arange(p0, p0 + m + g.front_tdi + g.back_tdi)          # y-indices needed
    y = oracle.project_links(op, g.t0_h, g.dt, case.hp, case.hc, case.lam, case.beta, case.order,
                             ys + g.y_start)
    t0_y = g.t0_h + (g.y_start + p0) * g.dt
    xyz = oracle.tdi_xyz(ot, t0_y, g.dt, y, case.generation, case.order,
                         np.arange(g.front_tdi, g.front_tdi + m))
    return oracle.select_channels(xyz, case.channels), y


def _oracle_block_adjoint(op, ot, case, p0, m, g_sel, y):
    """Oracle adjoint of the same block for the channel gradient g_sel."""
    import numpy as np

    import oracle
    g = case.grid
    gx = oracle.aet_transpose(g_sel) if case.channels == "AET" else g_sel
    t0_y = g.t0_h + (g.y_start + p0) * g.dt
    n_y = y.shape[1]
    g_y = oracle.tdi_adjoint(ot, t0_y, g.dt, n_y, case.generation, case.order,
                             np.arange(g.front_tdi, g.front_tdi + m), gx)
    oracle.project_adjoint(op, g.t0_h, g.dt, g.n_h, case.lam, case.beta, case.order,
                           np.arange(p0, p0 + n_y) + g.y_start, g_y)


def cpu_baseline(c3, c3_keep, c5, c5_keep, target_s):
    """The oracle (plain loops, OpenMP over samples) timed on bounded samples:
    a contiguous block of outputs of each of 8 templates of the headline
    batch (forward), and of 4 walkers (forward + adjoint); all host cores,
    then one thread.  The GPU outputs of the timed runs are compared with
    the oracle's on the same blocks."""
    import numpy as np

    import oracle
    from oracle import compare
    from oracle import waveform as owf
    from paper_2204_06633_amd import workloads
    cores = oracle.max_threads()
    res = {"kind": "oracle", "cores": cores, "cpu_model": _cpu_model(), "unit": UNIT,
           "note": "plain FP64 oracle (textbook O(n^2) Lagrange weights, OpenMP over samples), "
                   "not a tuned CPU code; full-workload times are linear extrapolations"}

    def cases_of(bc, keep):
        op = oracle.Orbits.from_samples(bc.orbits_proj)
        ot = op if bc.orbits_tdi is bc.orbits_proj else oracle.Orbits.from_samples(bc.orbits_tdi)
        cs = []
        for k, v in keep.items():
            g = bc.grids[k]
            if "hp" in v:
                hp, hc = v["hp"], v["hc"]
            else:                                   # waveform mode: the oracle's own waveform
                hp, hc = owf.polarizations(np.asarray(v["params"]), g.waveform_times())
            cs.append((k, workloads.Case("t%d" % k, bc.orbits_proj, bc.orbits_tdi, g,
                                         bc.params[k], hp, hc, bc.order,
                                         bc.generation, bc.channels), v["out"]))
        return op, ot, cs

    def leg(bc, keep, adjoint, threads, seconds, parity):
        oracle.set_threads(threads)
        op, ot, cs = cases_of(bc, keep)
        # calibrate on 256 outputs per template, then size the block
        t0 = time.perf_counter()
        for _, c, _ in cs:
            blk, y = _oracle_block(op, ot, c, c.grid.n_out // 3, 256)
            if adjoint:
                _oracle_block_adjoint(op, ot, c, c.grid.n_out // 3, 256, np.ones_like(blk), y)
        cal = time.perf_counter() - t0
        m = int(max(256, min(min(c.grid.n_out for _, c, _ in cs) // 3,
                             256 * seconds / max(cal, 1e-6))))
        worst = (0.0, 0.0)
        t0 = time.perf_counter()
        for k, c, out in cs:
            p0 = c.grid.n_out // 3
            blk, y = _oracle_block(op, ot, c, p0, m)
            if adjoint:
                _oracle_block_adjoint(op, ot, c, p0, m, np.ones_like(blk), y)
            if parity:
                e = compare.errors(out[:, p0:p0 + m], blk)
                worst = (max(worst[0], e[0]), max(worst[1], e[1]))
        el = time.perf_counter() - t0
        n_s = m * len(cs)
        rate = 6.0 * n_s / el
        r = {"value": rate, "threads": threads, "seconds": el,
             "sample": "%d contiguous outputs (from a third of the way in) of each of %d "
                       "templates (%s)%s" % (m, len(cs), ", ".join(str(k) for k, _, _ in cs),
                                             " forward + adjoint" if adjoint else " forward"),
             "extrapolated_full_workload_s": 6.0 * bc.n_samples / rate}
        if parity:
            r["parity_gpu_vs_oracle"] = {"rel_err": worst[0], "max_err": worst[1],
                                         "outputs_compared": n_s, "tolerance": 1e-11}
        return r

    log("CPU oracle: headline batch, all %d threads" % cores)
    res["headline_all_cores"] = leg(c3, c3_keep, False, cores, target_s, True)
    log("CPU oracle: headline batch, one thread")
    res["headline_one_thread"] = leg(c3, c3_keep, False, 1, target_s, False)
    if c5 is not None:
        log("CPU oracle: walkers (forward + adjoint), all threads")
        res["walkers_all_cores"] = leg(c5, c5_keep, True, cores, target_s, True)
        log("CPU oracle: walkers (forward + adjoint), one thread")
        res["walkers_one_thread"] = leg(c5, c5_keep, True, 1, target_s / 2, False)
    oracle.set_threads(cores)
    res["value"] = res["headline_all_cores"]["value"]
    res["sample"] = res["headline_all_cores"]["sample"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--headline-only", action="store_true",
                    help="the headline workload only (no other legs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the response runs on one MI355X and no "
              "multi-GPU path is built; got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2204_06633_amd import native
    c3_keep = {0: None, 137: None, 255: None, 301: None, 384: None, 450: None, 500: None,
               511: None}
    c5_keep = {0: None, 85: None, 170: None, 255: None}
    head, c3 = bench_headline(args.steps, args.warmup, c3_keep)
    torch.cuda.empty_cache()
    result = {
        "metric": METRIC, "value": head["value"], "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "512 Galactic-binary templates of uneven durations (uniform "
                               "0.25-1 yr at dt = 10 s, %d output samples), Keplerian flexing "
                               "orbits, Lagrange order 25, TDI-2 A/E/T, one fused batched "
                               "forward per step (captured graph, autotuned)" % head["time_samples"],
                   "templates": head["templates"], "time_samples": head["time_samples"],
                   "order": 25, "generation": 2, "channels": "AET", "dt": 10.0,
                   "group": head["group"], "blocks": head["blocks"]},
        "roofline": head["roofline"],
        "headline": head,
        "build_config": native.build_config(),
    }
    c5 = None
    if not args.headline_only:
        result["walkers"], c5 = bench_walkers(3, 1, c5_keep)
        torch.cuda.empty_cache()
        result["walkers_keplerian"], _ = bench_walkers(3, 1, {}, tdi_orbit_kind="keplerian")
        torch.cuda.empty_cache()
        # the batched forward + adjoint against the plain per-template forward
        plain = head["plain_per_template"]["value"]
        for leg in ("walkers", "walkers_keplerian"):
            result[leg]["vs_plain_per_template_forward"] = result[leg]["value"] / plain
        single, st = bench_single_template(args.steps)
        result["single_template"] = single
        result.update(bench_widened(args.steps, st))
        del st
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(c3, c3_keep, c5, c5_keep, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
