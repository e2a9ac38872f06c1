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

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import glob
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
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2204_06633_amd", "csrc", "*.h*"))):
        h.update(open(p, "rb").read())
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
    m = int(min(g.n_out // 2 - g.back_tdi - 1, max(m, m * target_s / max(dt_cal, 1e-6))))
    t0 = time.perf_counter()
    run(m)
    el = time.perf_counter() - t0
    return {"value": 6.0 * m / el, "unit": "samples/s (templates×links×time)",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d contiguous output samples of the same 1-yr template (%.1f s)" % (m, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
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
    case = workloads.config_c2("XYZAET")
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

    n = g.n_out
    value = 6.0 * n / (ms_step * 1e-3)
    f_tdi = costs.tdi_flops_per_sample(case.order, case.generation, case.channels) * n
    f_proj = costs.projection_flops_per_sample(case.order) * g.n_y
    b_tdi = costs.tdi_bytes_per_sample(case.channels) * n
    b_proj = costs.projection_bytes_per_sample() * g.n_y
    traffic = recorded_traffic("tdi", "c2")
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
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
