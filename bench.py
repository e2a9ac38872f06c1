#!/usr/bin/env python
"""Benchmark of the generic LISA time-domain response on one MI355X.

Workload: one Galactic-binary template, one year at dt = 10 s (3,155,760
output samples), flexing Keplerian orbits, Lagrange order 25, TDI-2 X/Y/Z plus
A/E/T, FP64.  One step = the whole per-template forward path: projection onto
the six links (lr_project_links) then TDI-2 (lr_tdi_combine), inputs resident
in HBM.  Throughput counts templates x 6 links x time samples per second.

Printed: one JSON line with the throughput, per-kernel times from HIP events
on the launch stream, the roofline of the dominant kernel (FP64 vector ALU),
algorithmic HBM bandwidth, a sampled parity check against the CPU oracle and
the oracle's own throughput on a bounded sample on the host cores.

Beside the headline it reports, in the same line:
  fwd_adjoint          the same template, forward + likelihood + adjoint
                       (gradients to h+, hx and the sky angles) per step;
  fd_likelihood,       the noise-weighted frequency-domain likelihood of its
  fd_fwd_adjoint       A/E/T (2^22-point transforms) alone, and in the
                       forward + likelihood + adjoint step;
  orbit_models         the paper's Fig. 3 binary through the accurate, the
                       fitted equal-armlength and the two hybrid orbit
                       models, scored by mismatch against the accurate data;
  batched_forward      512 templates of uneven durations (0.25-1 yr at
                       dt = 10 s) in one persistent fused launch, replayed
                       from a HIP graph, autotuned, against the plain
                       per-template forward on templates of the same batch;
  batched_fwd_adjoint  256 walkers, 1 yr at dt = 15 s, hybrid orbits:
                       forward + likelihood + adjoint in one HIP graph;
  sampler              the tempered ensemble sampler (4 x 50 walkers, stretch
                       move) on 1 yr at dt = 15 s, proposals scored by the
                       batched response and frequency-domain likelihood.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-batch]
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


def kernel_source_hash():
    """Hash of the sources that define the per-template forward kernels
    (tdi_kernel, project_links_kernel): a recorded counter summary is used
    only while they are unchanged."""
    h = hashlib.sha256()
    for name in ("device_common.hpp", "forward_kernels.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2204_06633_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, workload):
    """HBM traffic of a kernel from a committed rocprofv3 counter summary, or
    None if there is none for the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(case, target_s=10.0):
    """The CPU oracle (plain loops, OpenMP over samples) on a contiguous block
    of output samples of the same workload, sized for ~target_s seconds."""
    import numpy as np

    import oracle
    orb = oracle.Orbits.from_samples(case.orbits_proj)
    g = case.grid

    def run(m):
        p0 = g.n_out // 2
        ys = np.arange(p0, p0 + m + g.front_tdi + g.back_tdi)        # y-indices needed
        y = oracle.project_links(orb, g.t0_h, g.dt, case.hp, case.hc, case.lam, case.beta,
                                 case.order, ys + g.y_start)
        t0_y = g.t0_h + (g.y_start + p0) * g.dt
        xyz = oracle.tdi_xyz(orb, t0_y, g.dt, y, case.generation, case.order,
                             np.arange(g.front_tdi, g.front_tdi + m))
        oracle.select_channels(xyz, case.channels)

    m = 2048
    t0 = time.perf_counter()
    run(m)
    dt_cal = time.perf_counter() - t0
    # the second half of the template at most; repeated if that is shorter
    # than the target time
    m = int(min(g.n_out // 2 - g.back_tdi - 1, max(m, m * target_s / max(dt_cal, 1e-6))))
    reps, el = 0, 0.0
    while reps < 4 and (reps == 0 or el < target_s):
        t0 = time.perf_counter()
        run(m)
        el += time.perf_counter() - t0
        reps += 1
    return {"value": 6.0 * m * reps / el, "unit": "samples/s (templates×links×time)",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d contiguous output samples of the same 1-yr template, run %d time(s) "
                      "(%.1f s in total)" % (m, reps, el)}


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _timed(fn, steps, warmup):
    """Mean milliseconds of fn() over `steps` calls after `warmup`, from HIP
    events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = _events(steps + 1)
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[steps]) / steps


def _batch_parity(bc, k_list, hp, hc, out, batch, n_samples=48):
    """Joint relative error of sampled outputs of templates k_list against the
    oracle fed with the same (device-generated) polarisations."""
    import torch

    import oracle
    from paper_2204_06633_amd import workloads
    from tests import cases
    op = oracle.Orbits.from_samples(bc.orbits_proj)
    ot = op if bc.orbits_tdi is bc.orbits_proj else oracle.Orbits.from_samples(bc.orbits_tdi)
    worst = 0.0
    for k in k_list:
        g = bc.grids[k]
        ho = bc.layout.h_offsets[k]
        case = workloads.Case("batch%d" % k, bc.orbits_proj, bc.orbits_tdi, g, bc.params[k],
                              hp[ho:ho + g.n_h].cpu().numpy(), hc[ho:ho + g.n_h].cpu().numpy(),
                              bc.order, bc.generation, bc.channels)
        idx = cases.sample_indices(g.n_out, n_samples, seed=1000 + k, edge=2)
        ref = cases.oracle_sampled_response(op, ot, case, idx)
        got = batch.output_block(out, k)[:, torch.from_numpy(idx).to(out.device)].cpu().numpy()
        worst = max(worst, cases.rel_err(got, ref))
    return worst


def bench_batched_forward(steps, warmup, log):
    """512 uneven templates, fused forward from a captured graph; the plain
    per-template forward timed on 8 of the same templates."""
    import numpy as np
    import torch

    from paper_2204_06633_amd import autotune, costs, native, response, workloads
    dev = torch.device("cuda:0")
    bc = workloads.uneven_batch_case()
    log("batched forward: %s, %d templates, %d samples" % (bc.name, len(bc.grids), bc.n_samples))
    orb = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    hp, hc = workloads.device_polarizations(bc, dev)
    sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    tpl = bc.layout.templates()
    batch, tuned = autotune.tuned_batch(tpl, orb, orb, bc.t0, bc.dt, bc.order, bc.generation,
                                        bc.channels, hp, hc, sky)
    log("autotuned: group %d, grid x%.1f (%d work-groups)" % (tuned["group"],
                                                             tuned["grid_scale"], batch.blocks))
    out = torch.empty(batch.out_extent, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.response(hp, hc, sky, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.response(hp, hc, sky, out=out)
    ms = _timed(graph.replay, steps, warmup)
    n = bc.n_samples
    err = _batch_parity(bc, [0, len(bc.grids) // 2, len(bc.grids) - 1], hp, hc, out, batch)

    # plain per-template forward (project_links then tdi_combine) on 8 templates
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
    rate = 6.0 * n / (ms * 1e-3)
    f = sum(costs.tdi_flops_per_sample(bc.order, bc.generation, bc.channels) * g.n_out +
            costs.projection_flops_per_sample(bc.order) * g.n_y for g in bc.grids)
    b = sum(costs.tdi_bytes_per_sample(bc.channels) * g.n_out for g in bc.grids) + \
        sum(16.0 * g.n_y for g in bc.grids)
    del graph, out, hp, hc
    return {"workload": bc.name, "templates": len(bc.grids), "time_samples": n,
            "value": rate, "unit": "samples/s (templates×links×time)", "ms_per_step": ms,
            "steps": steps, "graph": True, "group": tuned["group"],
            "grid_scale": tuned["grid_scale"], "blocks": batch.blocks,
            "alu_frac": f / (ms * 1e-3) / costs.FP64_VECTOR_PEAK,
            "hbm_frac": b / (ms * 1e-3) / costs.HBM_PEAK,
            "plain_per_template": {"value": plain_rate, "templates_timed": len(pick),
                                   "speedup": rate / plain_rate},
            "parity": {"rel_err": err, "templates": 3, "tolerance": 1e-11}}


def bench_batched_fwd_adjoint(steps, warmup, log):
    """256 walkers: forward + likelihood + adjoint (with sky gradient) in one
    captured graph."""
    import torch

    from paper_2204_06633_amd import autotune, costs, native, workloads
    dev = torch.device("cuda:0")
    bc = workloads.walker_batch_case()
    log("batched fwd+adjoint: %s, %d walkers, %d samples" % (bc.name, len(bc.grids),
                                                            bc.n_samples))
    orb_p = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    orb_t = native.Orbits.from_samples(bc.orbits_tdi, device=dev)
    hp, hc = workloads.device_polarizations(bc, dev)
    sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    tpl = bc.layout.templates()
    tuned = autotune.tune(tpl, orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                          hp, hc, sky)
    batch = native.Batch(tpl, orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation, bc.channels,
                         group=tuned["group"], adjoint=True, device=dev)
    batch.set_grid(max(1, int(round(batch.blocks * tuned["grid_scale"]))))
    out = torch.empty(batch.out_extent, dtype=torch.float64, device=dev)
    # data: walker 0's response plus white noise (sigma = 1e-21), one copy per walker block
    batch.response(hp, hc, sky, out=out)
    sigma = 1e-21
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    blk = batch.output_block(out, 0).reshape(-1)
    one = blk + sigma * torch.randn(blk.shape, dtype=torch.float64, device=dev, generator=gen)
    data = one.repeat(len(bc.grids))
    del one
    ll = torch.empty(batch.n, dtype=torch.float64, device=dev)
    g_out = torch.empty_like(out)
    ghp = torch.empty(batch.h_extent, dtype=torch.float64, device=dev)
    ghc = torch.empty_like(ghp)
    gsky = torch.empty((batch.n, 2), dtype=torch.float64, device=dev)

    def step():
        batch.response(hp, hc, sky, out=out)
        batch.loglike(out, data, sigma, ll=ll, g_out=g_out)
        batch.adjoint(hp, hc, sky, g_out, g_hp=ghp, g_hc=ghc, g_sky=gsky)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    ms = _timed(graph.replay, steps, warmup)
    ms_fwd = _timed(lambda: batch.response(hp, hc, sky, out=out), steps, 1)
    err = _batch_parity(bc, [0, len(bc.grids) - 1], hp, hc, out, batch)
    n = bc.n_samples
    finite = bool(torch.isfinite(ll).all()) and bool(torch.isfinite(gsky).all())
    del graph, out, data, g_out, ghp, ghc, hp, hc
    return {"workload": bc.name, "templates": len(bc.grids), "time_samples": n,
            "value": 6.0 * n / (ms * 1e-3), "unit": "samples/s (templates×links×time)",
            "ms_per_step": ms, "forward_only_ms": ms_fwd, "steps": steps, "graph": True,
            "group": tuned["group"], "gradients_finite": finite,
            "parity_forward": {"rel_err": err, "templates": 2, "tolerance": 1e-11}}


def bench_sampler(steps, log):
    """Four temperatures of 50 walkers (Sec. II.B) on one year at dt = 15 s:
    tempered stretch-move steps whose proposals are scored by
    lr_gb_polarizations, lr_response and lr_fd_loglike, 100 walkers per
    call."""
    import torch

    from paper_2204_06633_amd import sampler, workloads
    sc = workloads.sampler_case()
    run = sampler.setup_run(sc, device="cuda:0", log=log)
    run.step()                                                         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc_tot = torch.zeros(sc.T, dtype=torch.int64, device="cuda:0")
    for _ in range(steps):
        acc, _ = run.step()
        acc_tot += acc
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    evals = 2 * sc.m
    g = sc.grid
    return {"workload": sc.name, "temperatures": sc.T, "walkers_per_temperature": sc.W,
            "group": run.tuned["group"], "grid_scale": run.tuned["grid_scale"],
            "time_samples": g.n_out, "ms_per_step": ms, "steps": steps,
            "likelihood_evals_per_s": evals / (ms * 1e-3),
            "value": evals * 6.0 * g.n_out / (ms * 1e-3),
            "unit": "samples/s (templates×links×time)",
            "acceptance_per_temperature": (acc_tot.float() / (steps * sc.W)).tolist(),
            "step": "tempered stretch move over 4 x 50 walkers: lr_gb_polarizations -> lr_response "
                    "-> lr_fd_loglike (statistics) per half step, then tempering swaps"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batch", action="store_true", help="headline workload only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the response runs on one MI355X; "
              "multi-GPU sharding is not built); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_06633_amd import costs, native, response, workloads
    from tests import cases

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    case = workloads.year_case("XYZAET")
    g = case.grid
    print("bench: workload %s, n_out=%d, n_h=%d" % (case.name, g.n_out, g.n_h), file=sys.stderr,
          flush=True)
    orb = native.Orbits.from_samples(case.orbits_proj, device=dev)
    hp = torch.tensor(case.hp, dtype=torch.float64, device=dev)
    hc = torch.tensor(case.hc, dtype=torch.float64, device=dev)
    y = torch.empty((6, g.n_y), dtype=torch.float64, device=dev)
    out = torch.empty((6, g.n_out), dtype=torch.float64, device=dev)
    t0_y = g.t0_h + g.y_start * g.dt
    sky = torch.tensor([case.lam, case.beta], dtype=torch.float64, device=dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        native.project_links(orb, g.t0_h, g.dt, hp, hc, sky, case.order, g.y_start, g.n_y, y=y)
        if ev is not None:
            ev[1].record()
        native.tdi_combine(orb, t0_y, g.dt, y, case.generation, case.order, case.channels,
                           g.front_tdi, g.n_out, out=out)
        if ev is not None:
            ev[2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el / args.steps * 1e3
    t_proj = float(np.mean([e[0].elapsed_time(e[1]) for e in events])) * 1e-3
    t_tdi = float(np.mean([e[1].elapsed_time(e[2]) for e in events])) * 1e-3

    # parity of the timed output on sampled samples (outside the timed region)
    import oracle
    idx = cases.sample_indices(g.n_out, 200, seed=99)
    o = oracle.Orbits.from_samples(case.orbits_proj)
    ref = cases.oracle_sampled_response(o, o, case, idx)
    err = cases.rel_err(out[:, torch.from_numpy(idx).to(dev)].cpu().numpy(), ref)

    def log(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    # forward + likelihood + adjoint of the same template
    tpl = response.Template(orb, orb, g, case.order, case.generation, case.channels)
    # likelihood over A, E, T (rows 3..5); X, Y, Z get no gradient
    data = out[3:].clone()
    ll_buf = torch.empty(1, dtype=torch.float64, device=dev)
    g_buf = torch.zeros_like(out)
    work = torch.empty(native.lib().lr_loglike_workspace() // 8, dtype=torch.float64, device=dev)

    def fwd_adj():
        response.plain_forward(tpl, hp, hc, sky, y=y, out=out)
        native.loglike(out[3:], data, 1e-21, out=ll_buf, g_h=g_buf[3:], work=work)
        response.plain_adjoint(tpl, hp, hc, sky, g_buf)

    log("forward + adjoint of the same template")
    ms_fa = _timed(fwd_adj, max(3, args.steps // 2), 1)

    # the same step with the noise-weighted frequency-domain likelihood (the
    # stand-in noise curve; data = the template itself, no noise, as in the
    # paper's runs)
    from paper_2204_06633_amd import inputs
    log("forward + frequency-domain likelihood + adjoint of the same template")
    n_fft = native.fd_length(g.n_out)
    w_ae, w_t = inputs.noise_weights(n_fft, g.dt)
    plan = native.FdPlan(data, torch.tensor(w_ae, dtype=torch.float64, device=dev),
                         torch.tensor(w_t, dtype=torch.float64, device=dev), g.dt)
    fd_stats = torch.empty((1, 3), dtype=torch.float64, device=dev)

    def fd_fwd_adj():
        response.plain_forward(tpl, hp, hc, sky, y=y, out=out)
        plan.loglike(out[3:], stats=fd_stats, g_h=g_buf[3:])
        response.plain_adjoint(tpl, hp, hc, sky, g_buf)

    ms_fd_fa = _timed(fd_fwd_adj, max(3, args.steps // 2), 1)
    ms_fd = _timed(lambda: plan.loglike(out[3:], stats=fd_stats, g_h=g_buf[3:]), args.steps, 2)
    ms_fd_stats = _timed(lambda: plan.loglike(out[3:], want_grad=False, stats=fd_stats),
                         args.steps, 2)
    fd_b = costs.fd_bytes(g.n_out, n_fft, 3, plan.passes, True)
    fd_b_stats = costs.fd_bytes(g.n_out, n_fft, 3, plan.passes, False)
    del plan

    # orbit models (Sec. V): the paper's Fig. 3 binary for a year through the
    # accurate orbits, the fitted equal-armlength ones and the two hybrids,
    # scored against noise-free data with the frequency-domain statistics
    from paper_2204_06633_amd import orbitfit
    log("orbit configurations ESA / EQ / ESAEQ / EQESA")
    oc = workloads.orbit_config_case(g.n_out, g.dt)
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
    oc_plan = native.FdPlan(oc_h[0].clone(), torch.tensor(w_ae, dtype=torch.float64, device=dev),
                            torch.tensor(w_t, dtype=torch.float64, device=dev), g.dt, max_batch=4)

    def orbit_step():
        for k, tp in enumerate(oc_tpl):
            response.plain_forward(tp, oc_hp, oc_hc, oc_sky, y=oc_y, out=oc_h[k])
        oc_plan.loglike(oc_h, want_grad=False, stats=oc_stats)

    ms_orb = _timed(orbit_step, max(3, args.steps // 4), 1)
    oc_st = oc_stats.cpu().numpy()
    oc_diag = orbitfit.overlap_statistics(oc_st, ss=oc_st[0, 1])
    orbit_result = {"ms_per_step": ms_orb, "eq_fit_lam1_m1": list(oc.eq_params),
                    "step": "4 templates (orbit models) forward + frequency-domain statistics "
                            "against the accurate-orbit data, 1 yr",
                    "mismatch": {k: float(oc_diag["mismatch"][i]) for i, k in enumerate(oc_names)},
                    "rho_opt": {k: float(oc_diag["rho_opt"][i]) for i, k in enumerate(oc_names)}}
    del oc_plan, oc_h, oc_y, oc_orb

    # the differentiation step: source parameters -> polarisations (torch)
    # -> response -> A/E/T likelihood -> hand-written adjoint -> autograd to
    # the eight parameters (the paper's Fig. 3 binary, data = injection +
    # white noise sigma = 1e-21)
    from paper_2204_06633_amd import inputs, waveform
    log("likelihood gradient with respect to the source parameters")
    tpl_aet = response.Template(orb, orb, g, case.order, case.generation, "AET")
    t_w = torch.tensor(g.waveform_times(), dtype=torch.float64, device=dev)
    theta = torch.tensor(inputs.PAPER_FIG3_BINARY, dtype=torch.float64, device=dev)
    with torch.no_grad():
        hp0, hc0 = waveform.gb_polarizations(theta, t_w)
        inj, _ = response.plain_forward(tpl_aet, hp0.contiguous(), hc0.contiguous(),
                                        theta[6:8].contiguous())
        gen = torch.Generator(device=dev)
        gen.manual_seed(4)
        data_aet = inj + 1e-21 * torch.randn(inj.shape, dtype=torch.float64, device=dev,
                                             generator=gen)
        del hp0, hc0, inj

    def grad_step():
        p = theta.clone().requires_grad_(True)
        hp_, hc_ = waveform.gb_polarizations(p, t_w)
        ll = response.loglike(response.response(tpl_aet, hp_, hc_, p[6:8]), data_aet, 1e-21)
        ll.backward()
        return p.grad

    ms_grad = _timed(grad_step, max(3, args.steps // 2), 1)
    grad_ok = bool(torch.isfinite(grad_step()).all())

    def grad_step_hip():
        # the same with the polarisations and their adjoint in the HIP library
        p = theta.clone().requires_grad_(True)
        hp_, hc_ = response.gb_polarizations(p[None], -g.out_start, g.n_h, g.dt)
        ll = response.loglike(response.response(tpl_aet, hp_[0], hc_[0], p[6:8]), data_aet, 1e-21)
        ll.backward()
        return p.grad

    ms_grad_hip = _timed(grad_step_hip, max(3, args.steps // 2), 1)
    g_t, g_h = grad_step(), grad_step_hip()
    grad_agree = float(((g_h - g_t).abs() / g_t.abs().clamp_min(1e-300)).max())
    del data_aet

    # the same template through the fused batch kernel (a batch of one)
    log("the same template as a batch of one (fused kernel)")
    one = native.Batch([(0, g.n_h, g.out_start, g.n_out, 0)], orb, orb, g.t_start, g.dt,
                       case.order, case.generation, case.channels, group=1, device=dev)
    out1 = torch.empty(one.out_extent, dtype=torch.float64, device=dev)
    sky1 = sky.view(1, 2)
    ms_one = _timed(lambda: one.response(hp, hc, sky1, out=out1), args.steps, 2)
    err_one = cases.rel_err(one.output_block(out1, 0)[:, torch.from_numpy(idx).to(dev)].cpu().numpy(),
                            ref)
    del out1

    n = g.n_out
    value = 6.0 * n / (ms_step * 1e-3)
    f_tdi = costs.tdi_flops_per_sample(case.order, case.generation, case.channels) * n
    f_proj = costs.projection_flops_per_sample(case.order) * g.n_y
    b_tdi = costs.tdi_bytes_per_sample(case.channels) * n
    b_proj = costs.projection_bytes_per_sample() * g.n_y
    traffic = recorded_traffic("tdi", "1yr")
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s (templates×links×time)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single Galactic-binary template, 1 yr at dt=10 s (%d samples), "
                               "Keplerian flexing orbits, Lagrange order 25, TDI-2 XYZ+AET, "
                               "plain per-template forward" % n,
                   "templates": 1, "time_samples": n, "order": case.order,
                   "generation": case.generation, "channels": "XYZ+AET", "dt": g.dt},
        "roofline": {"bound": "alu", "kernel": "tdi_kernel<26,2>",
                     "achieved": f_tdi / t_tdi / 1e12, "peak": costs.FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": f_tdi / t_tdi / costs.FP64_VECTOR_PEAK,
                     "traffic": traffic},
        "kernels": {
            "project_links": {"ms": t_proj * 1e3, "tflops": f_proj / t_proj / 1e12,
                              "alu_frac": f_proj / t_proj / costs.FP64_VECTOR_PEAK,
                              "hbm_GBps": b_proj / t_proj / 1e9,
                              "hbm_frac": b_proj / t_proj / costs.HBM_PEAK},
            "tdi_combine": {"ms": t_tdi * 1e3, "tflops": f_tdi / t_tdi / 1e12,
                            "alu_frac": f_tdi / t_tdi / costs.FP64_VECTOR_PEAK,
                            "hbm_GBps": b_tdi / t_tdi / 1e9,
                            "hbm_frac": b_tdi / t_tdi / costs.HBM_PEAK},
        },
        "hbm_frac_step": (b_tdi + b_proj) / (ms_step * 1e-3) / costs.HBM_PEAK,
        "parity": {"rel_err": err, "samples": int(idx.size), "tolerance": 1e-11},
        "fwd_adjoint": {"value": 6.0 * n / (ms_fa * 1e-3), "unit": "samples/s (templates×links×time)",
                        "ms_per_step": ms_fa,
                        "step": "forward, white-noise likelihood over A/E/T with gradient, "
                                "adjoint to h+, hx and (lam, beta)"},
        "fd_likelihood": {"ms": ms_fd, "ms_stats_only": ms_fd_stats, "n_fft": n_fft,
                          "hbm_GBps": fd_b / (ms_fd * 1e-3) / 1e9,
                          "hbm_frac": fd_b / (ms_fd * 1e-3) / costs.HBM_PEAK,
                          "bytes": fd_b,
                          "hbm_frac_stats_only": fd_b_stats / (ms_fd_stats * 1e-3) / costs.HBM_PEAK,
                          "step": "lr_fd_loglike on the template's A/E/T: <d-h|d-h>, <h|h>, "
                                  "<d|h> with the stand-in noise curve and d logL/dh"},
        "fd_fwd_adjoint": {"value": 6.0 * n / (ms_fd_fa * 1e-3),
                           "unit": "samples/s (templates×links×time)", "ms_per_step": ms_fd_fa,
                           "step": "forward, frequency-domain likelihood over A/E/T with "
                                   "gradient, adjoint to h+, hx and (lam, beta)"},
        "orbit_models": orbit_result,
        "gradient_step": {"value": 6.0 * n / (ms_grad * 1e-3),
                          "unit": "samples/s (templates×links×time)", "ms_per_step": ms_grad,
                          "step": "8 source parameters -> h+, hx (torch) -> response (A/E/T) -> "
                                  "likelihood -> adjoint -> autograd to the parameters",
                          "gradient_finite": grad_ok,
                          "ms_per_step_hip_waveform": ms_grad_hip,
                          "hip_vs_torch_waveform_rel_diff": grad_agree},
        "fused_single": {"value": 6.0 * n / (ms_one * 1e-3),
                         "unit": "samples/s (templates×links×time)", "ms_per_step": ms_one,
                         "step": "the headline template through lr_response (fused projection "
                                 "+ TDI, link series kept in LDS), group 1",
                         "parity_rel_err": err_one},
    }
    if not args.no_batch:
        del y, data, g_buf
        torch.cuda.empty_cache()
        result["batched_forward"] = bench_batched_forward(max(3, args.steps // 4), 1, log)
        torch.cuda.empty_cache()
        result["batched_fwd_adjoint"] = bench_batched_fwd_adjoint(3, 1, log)
        torch.cuda.empty_cache()
        result["sampler"] = bench_sampler(3, log)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
