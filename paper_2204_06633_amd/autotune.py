"""Autotuner of the batched forward (persistent fused projection + TDI).

Knobs, timed on the caller's own batch (or an evenly spread subset of it):

* ``group``: templates per work item (1, 2 or 4).  Larger groups share each
  TDI Lagrange coefficient sequence among more templates but hold more link
  series in LDS, so fewer work-groups fit on a CU.
* ``tile``: link samples per tile (256, 512 or 1024; workgroups of 128,
  256 or 512 lanes, two samples per lane).  Longer tiles hold more LDS per
  work-group; a work item is a segment of consecutive tiles, of which only
  the first computes the TDI halo (about 34 link samples at dt = 10 s), the
  others take it from the tile before.  The segment length is the plan's
  automatic choice (up to 8 tiles, enough work items for the grid), not a
  tuned knob.
* ``grid``: work-groups of the persistent launch, as a multiple of the
  resident count that ``lr_batch_prepare`` picks.

Every knob value gives bit-identical outputs (each sample's arithmetic does
not depend on how samples are grouped into items).  The samples per lane
(two: the pair recurrence) and the tap layout (parity-split LDS windows, so
a wave reads consecutive addresses per tap) are fixed: both were measured
against the alternatives on the single-template kernels.

Results are cached in a JSON file keyed by device name, order, generation,
channels, dt and buckets of the batch shape (template count and mean
duration, powers of two), so a tuned configuration is reused by later
batches of the same kind.  The cache path comes from the argument, else the
environment variable LISARESP_TUNE_CACHE, else ~/.cache/lisaresp/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import native

GROUPS = (1, 2, 4)
TILES = (256, 512, 1024)
GRID_SCALES = (0.5, 1.0, 2.0)


def variant_exists(group, tile, wave=False):
    """Compiled fused-kernel variants (groups of 4 at 1024 would need 196 KB
    of LDS); the waveform-mode kernel (``wave``) is compiled for groups of 1
    and 2 at 512 link samples and of 2 at 1024."""
    if wave:
        return (group, tile) in ((1, 512), (2, 512), (2, 1024))
    return group in GROUPS and tile in TILES and not (group == 4 and tile == 1024)


def _cache_path(path=None):
    if path:
        return path
    env = os.environ.get("LISARESP_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "lisaresp", "tune.json")


def _bucket(x):
    return 0 if x <= 0 else int(round(math.log2(x)))


def tune_key(device_name, order, generation, channels, dt, templates):
    n = len(templates)
    mean = sum(t[3] for t in templates) / max(n, 1)
    return "%s|o%d|g%d|%s|dt%.6g|n2^%d|len2^%d|tiles" % (device_name, order, generation,
                                                         channels, dt, _bucket(n), _bucket(mean))


def load_cache(path=None):
    p = _cache_path(path)
    try:
        with open(p) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=None):
    p = _cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def subset(templates, max_templates):
    """Evenly spread subset (by duration rank) of at most max_templates,
    re-laid out contiguously; returns (templates, source indices)."""
    n = len(templates)
    if n <= max_templates:
        return list(templates), list(range(n))
    order = sorted(range(n), key=lambda k: templates[k][3])
    pick = [order[int(i * (n - 1) / (max_templates - 1))] for i in range(max_templates)]
    return [templates[k] for k in pick], pick


def _time_ms(fn, reps):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    fn()                                    # warm-up
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        start.record()
        fn()
        stop.record()
        stop.synchronize()
        best = min(best, start.elapsed_time(stop))
    return best


def tune(templates, orb_proj, orb_tdi, t0, dt, order, generation, channels, hp, hc, sky,
         reps=3, max_templates=64, cache_path=None, use_cache=True, verbose=False, params=None):
    """Pick (group, tile, grid scale) for a batch.  hp, hc, sky: the batch's
    device inputs (sky [n][2]); or ``params`` [n][8] for the waveform-mode
    forward (lr_response_gb; hp, hc, sky then unused).  The timing runs
    write into scratch outputs only.  Returns a dict {"group", "tile",
    "grid_scale", "ms", "trials"}."""
    import torch
    dev = params.device if params is not None else hp.device
    key = tune_key(torch.cuda.get_device_name(dev), order, generation, channels, dt, templates)
    if params is not None:
        key += "|wave"
    cache = load_cache(cache_path) if use_cache else {}
    if key in cache:
        return cache[key]

    sub, pick = subset(templates, max_templates)
    rows = 6 if channels == "XYZAET" else 3
    # contiguous re-layout of the subset's outputs (inputs stay where they are)
    lay, off = [], 0
    for (ho, nh, os_, no, _) in sub:
        lay.append((ho, nh, os_, no, off))
        off += rows * no
    sel = torch.tensor(pick, device=dev)
    out = torch.empty(max(off, 1), dtype=torch.float64, device=dev)
    if params is not None:
        par_sub = params[sel].contiguous()
        run = lambda b: b.response_gb(par_sub, out=out)
    else:
        sky_sub = sky[sel].contiguous()
        run = lambda b: b.response(hp, hc, sky_sub, out=out)
    trials = []
    for g in GROUPS:
        for tile in TILES:
            if not variant_exists(g, tile, wave=params is not None):
                continue
            try:
                b = native.Batch(lay, orb_proj, orb_tdi, t0, dt, order, generation, channels,
                                 group=g, tile=tile, device=dev)
            except native.LisaRespError:          # e.g. dt too small for a short tile
                continue
            base = b.blocks
            for s in GRID_SCALES:
                blocks = max(1, int(round(base * s)))
                b.set_grid(blocks)
                ms = _time_ms(lambda: run(b), reps)
                trials.append({"group": g, "tile": tile, "grid_scale": s, "blocks": blocks,
                               "ms": ms})
                if verbose:
                    print("tune group=%d tile=%d grid=%d (x%.1f): %.3f ms"
                          % (g, tile, blocks, s, ms), flush=True)
    best = min(trials, key=lambda r: r["ms"])
    res = {"group": best["group"], "tile": best["tile"], "grid_scale": best["grid_scale"],
           "ms": best["ms"], "trials": trials, "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")}
    if use_cache:
        cache = load_cache(cache_path)
        cache[key] = res
        save_cache(cache, cache_path)
    return res


def tuned_batch(templates, orb_proj, orb_tdi, t0, dt, order, generation, channels, hp, hc, sky,
                adjoint=False, **kw):
    """A native.Batch prepared with the tuned group, tile and grid."""
    r = tune(templates, orb_proj, orb_tdi, t0, dt, order, generation, channels, hp, hc, sky, **kw)
    dev = kw["params"].device if kw.get("params") is not None else hp.device
    b = native.Batch(templates, orb_proj, orb_tdi, t0, dt, order, generation, channels,
                     group=r["group"], tile=r.get("tile", 0), adjoint=adjoint, device=dev)
    b.set_grid(max(1, int(round(b.blocks * r["grid_scale"]))))
    return b, r
