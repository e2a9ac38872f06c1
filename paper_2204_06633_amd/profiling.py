"""Kernel driver for rocprofv3 runs (kernel traces and hardware counters).

    python -m paper_2204_06633_amd.profiling --what forward --reps 5
    python -m paper_2204_06633_amd.profiling --what adjoint --reps 5
    python -m paper_2204_06633_amd.profiling --what copy --copy-mib 1024
    python -m paper_2204_06633_amd.profiling --what batch --templates 64
    python -m paper_2204_06633_amd.profiling --what batch-adjoint --templates 32 --waveform
    python -m paper_2204_06633_amd.profiling --what fd --templates 4
    python -m paper_2204_06633_amd.profiling --what sampler --reps 2

``forward`` runs the per-template forward (projection + TDI-2 XYZ+AET) on the
1-yr, dt = 10 s, order-25 Keplerian workload; ``adjoint`` adds the adjoint
pair; ``copy`` runs one device-to-device copy of known size (the reference
for scaling the HBM byte counters); ``batch`` runs the fused batched forward
on the first ``--templates`` templates of the 512-template uneven batch
(``--group``, ``--tile``, ``--grid-scale``: the autotuner's knobs);
``batch-adjoint`` runs forward, likelihood and adjoint of that many 1-yr,
dt = 15 s walkers with hybrid orbits; ``--waveform`` runs either batch in
waveform mode (h+ / hx synthesised in the kernels from each template's
parameter row, the adjoint down to the 8 parameters); ``fd`` runs the
frequency-domain likelihood with its gradient on ``--templates`` one-year
A/E/T series at dt = 10 s (2^22-point transforms); ``sampler`` runs
tempered stretch-move steps of 4 x 50 walkers on one year at dt = 15 s.
Each step prints a line so a profiler run shows progress.
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", choices=["forward", "adjoint", "copy", "batch", "batch-adjoint", "fd",
                             "sampler"],
                    default="forward")
    ap.add_argument("--templates", type=int, default=64)
    ap.add_argument("--group", type=int, default=2)
    ap.add_argument("--tile", type=int, default=0, help="link samples per fused tile")
    ap.add_argument("--segment", type=int, default=0,
                    help="fused tiles per work item (0: the plan's automatic choice)")
    ap.add_argument("--grid-scale", type=float, default=1.0)
    ap.add_argument("--waveform", action="store_true",
                    help="waveform mode (lr_response_gb / lr_response_adjoint_gb)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args(argv)

    import torch

    dev = torch.device("cuda:0")
    if args.what == "copy":
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for r in range(args.reps):
            dst.copy_(src)
            torch.cuda.synchronize()
            print("copy %d: %d bytes read, %d written" % (r, 8 * n, 8 * n), flush=True)
        return

    from . import native, response, workloads
    if args.what in ("batch", "batch-adjoint"):
        return run_batch(args, dev)
    if args.what == "fd":
        return run_fd(args, dev)
    if args.what == "sampler":
        import time as _time

        from . import sampler
        # group 2 and the resident grid, the tuner's choice for this batch
        # (its trial launches would crowd the trace)
        run = sampler.setup_run(workloads.sampler_case(), device=dev, tune=False,
                                log=lambda msg: print(msg, flush=True))
        for r in range(args.reps + 1):
            t0 = _time.perf_counter()
            run.step()
            torch.cuda.synchronize()
            print("sampler step %d: %.1f ms per step" % (r, (_time.perf_counter() - t0) * 1e3),
                  flush=True)
        return
    case = workloads.year_case("XYZAET")
    g = case.grid
    orb = native.Orbits.from_samples(case.orbits_proj, device=dev)
    tpl = response.Template(orb, orb, g, case.order, case.generation, case.channels)
    hp = torch.tensor(case.hp, dtype=torch.float64, device=dev)
    hc = torch.tensor(case.hc, dtype=torch.float64, device=dev)
    sky = torch.tensor([case.lam, case.beta], dtype=torch.float64, device=dev)
    y = torch.empty((6, g.n_y), dtype=torch.float64, device=dev)
    out = torch.empty((6, g.n_out), dtype=torch.float64, device=dev)
    g_out = torch.ones_like(out)
    for r in range(args.reps):
        response.plain_forward(tpl, hp, hc, sky, y=y, out=out)
        if args.what == "adjoint":
            response.plain_adjoint(tpl, hp, hc, sky, g_out)
        torch.cuda.synchronize()
        print("%s step %d done (%d samples)" % (args.what, r, g.n_out), flush=True)


def run_batch(args, dev):
    import torch

    from . import native, workloads
    adj = args.what == "batch-adjoint"
    full = workloads.walker_batch_case(args.templates) if adj else workloads.uneven_batch_case()
    bc = full
    if not adj:
        k = args.templates
        bc = workloads.make_batch_case(full.name, [g.n_out for g in full.grids[:k]], full.dt,
                                       full.order, full.generation, full.channels, 3,
                                       params=full.params[:k])
    orb_p = native.Orbits.from_samples(bc.orbits_proj, device=dev)
    orb_t = orb_p if bc.orbits_tdi is bc.orbits_proj else \
        native.Orbits.from_samples(bc.orbits_tdi, device=dev)
    if args.waveform:
        params = torch.tensor(bc.params, dtype=torch.float64, device=dev).contiguous()
        g_par = torch.empty_like(params)
    else:
        hp, hc = workloads.device_polarizations(bc, dev)
        sky = torch.tensor(bc.params[:, 6:8], dtype=torch.float64, device=dev).contiguous()
    b = native.Batch(bc.layout.templates(), orb_p, orb_t, bc.t0, bc.dt, bc.order, bc.generation,
                     bc.channels, group=args.group, tile=args.tile, segment=args.segment,
                     adjoint=adj, device=dev)
    b.set_grid(max(1, int(round(b.blocks * args.grid_scale))))
    out = torch.empty(b.out_extent, dtype=torch.float64, device=dev)
    data = torch.zeros_like(out) if adj else None
    for r in range(args.reps):
        if args.waveform:
            b.response_gb(params, out=out)
        else:
            b.response(hp, hc, sky, out=out)
        if adj:
            _, g_out = b.loglike(out, data, 1e-21)
            if args.waveform:
                b.adjoint_gb(params, g_out, g_params=g_par)
            else:
                b.adjoint(hp, hc, sky, g_out)
        torch.cuda.synchronize()
        print("%s step %d done (%d templates, %d samples)" % (args.what, r, len(bc.grids),
                                                            bc.n_samples), flush=True)


def run_fd(args, dev):
    import torch

    from . import native, workloads
    fc = workloads.fd_case(args.templates)
    w_ae, w_t = fc.weights(native.fd_length(fc.n), dev)
    plan = native.FdPlan(fc.data(dev), w_ae, w_t, fc.dt, max_batch=args.templates)
    h = fc.templates(dev)
    stats = torch.empty((args.templates, 3), dtype=torch.float64, device=dev)
    g = torch.empty_like(h)
    for r in range(args.reps):
        plan.loglike(h, stats=stats, g_h=g)
        torch.cuda.synchronize()
        print("fd step %d done (%d templates, %d-point transforms)" % (r, args.templates,
                                                                       plan.n_fft), flush=True)


if __name__ == "__main__":
    sys.exit(main())
