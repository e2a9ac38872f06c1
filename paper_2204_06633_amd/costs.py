"""Algorithmic FLOP and HBM-byte counts per output sample of each kernel.

These are properties of the algorithm as the kernels implement it, not
measurements: they turn measured kernel times into roofline fractions.
FLOPs count an FMA as 2.  N = order + 1 interpolation taps.

Lagrange weights by prefix / suffix products cost 5N FLOPs per retarded
position (N differences eps - x_m, N prefix products, N suffix products, 2N
products w_m = pre_m * suf_m * c_m); applying them to one series costs N FMAs
(2N FLOPs).  Orbit splines cost one cubic (3 FMAs, 6 FLOPs) per series.
"""
from __future__ import annotations

# Second-generation X, Y, Z: 48 terms, 6 undelayed, 42 delayed, whose delays
# take 36 distinct values (delay groups); first generation: 24 terms, 6
# undelayed, 18 delayed, 15 distinct delays.
TDI_SHAPE = {1: dict(groups=15, delayed=18, direct=6, mean_links=2.0),
             2: dict(groups=36, delayed=42, direct=6, mean_links=150.0 / 36.0)}


def weights_flops(taps):
    return 5 * taps


def tdi_flops_per_sample(order, generation, channels="XYZ"):
    n = order + 1
    s = TDI_SHAPE[generation]
    orbit = 6 * 6                                             # 6 light-time splines
    delays = s["groups"] * (s["mean_links"] - 1 + 3)          # sums + split (mul, floor, sub)
    weights = s["groups"] * weights_flops(n)
    taps = s["delayed"] * 2 * n
    direct = s["direct"]
    aet = 0 if channels == "XYZ" else 12
    return orbit + delays + weights + taps + direct + aet


def projection_flops_per_sample(order):
    n = order + 1
    orbit = 15 * 6                                           # 9 positions + 6 light times
    geometry = 3 * 6 + 3 * (3 + 6 + 2 + 3 + 3 * 5 + 4) + 6 * 5   # k.x, arms (n, xi, k.n), 1/(2(1-k.n))
    positions = 9 * 4
    weights = 9 * weights_flops(n)
    taps = 9 * 2 * 2 * n                                     # h+ and hx per position
    assemble = 6 * 7
    return orbit + geometry + positions + weights + taps + assemble


def tdi_bytes_per_sample(channels="XYZ"):
    rows = 6 if channels == "XYZAET" else 3
    return 6 * 8 + rows * 8                                  # read y, write channels


def projection_bytes_per_sample():
    return 2 * 8 + 6 * 8                                     # read h+, hx; write y


# MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 FLOPs (FMA) x 2.4 GHz.
FP64_VECTOR_PEAK = 256 * 4 * 16 * 2 * 2.4e9                  # 78.6 TFLOP/s
HBM_PEAK = 8.0e12                                            # bytes/s


def fd_bytes(n, n_fft, channels=3, passes=3, grad=True):
    """HBM bytes per template of the frequency-domain likelihood as the
    passes move them: the first forward pass reads the channel series and
    writes the complex signals (A + iE, and T + i0 with T), middle passes
    read and write them, the last forward pass also reads the data spectrum
    and the weights, and with the gradient every inverse pass reads and
    writes again, the last one writing the channel series.  The minimum any
    method must move (series in, gradient out, data spectrum and weights in)
    is ``fd_io_bytes``."""
    sig = 2 if channels == 3 else 1
    cplx = 16 * sig * n_fft
    series = 8 * channels * n
    spec = 24 * sig * n_fft                                   # data spectrum + weights
    fwd = series + cplx + 2 * cplx * (passes - 1) + spec
    if passes == 1:
        fwd = series + spec
    if not grad:
        return fwd - (cplx if passes > 1 else 0)              # last pass writes nothing
    if passes == 1:
        return fwd + series
    return fwd + 2 * cplx * (passes - 2) + cplx + series


def fd_io_bytes(n, n_fft, channels=3, grad=True):
    sig = 2 if channels == 3 else 1
    return 8 * channels * n * (2 if grad else 1) + 24 * sig * n_fft


# ---------------------------------------------------------------------------
# FP64 lane-operation model (every FP64 operation one lane-op, an FMA too)
# against the vector issue peak: 256 CUs x 64 lanes x 2.4 GHz.  Per (template,
# sample), N = order + 1 taps:
#   Lagrange weights of one retarded position   5N (prefix and suffix products)
#   one interpolated series                     N  (one multiply-add per tap)
#   projection geometry and orbit evaluation    200 + 120
# so the projection costs 9 * 5N + 9 * 2N + 320 per link sample (nine
# positions, h+ and hx share the weights), TDI 5N per delay group (shared by
# the templates of a work item, which share the orbits) plus N per delayed
# term, and the sky gradient 9 * 15N (weights and their derivatives) + 9 * 4N
# (value and derivative of h+ and hx) + 420 per link sample.  The adjoints
# scatter with the same weights as their forwards and cost the same.
# ---------------------------------------------------------------------------
LANE_OPS_PEAK = 256 * 64 * 2.4e9                              # 3.93e13 FP64 lane-ops/s


def lane_ops_projection(order):
    n = order + 1
    return 9 * 5 * n + 9 * 2 * n + 200 + 120


def lane_ops_tdi(order, generation, share=1):
    n = order + 1
    s = TDI_SHAPE[generation]
    return s["groups"] * 5 * n / share + s["delayed"] * n


def lane_ops_sky(order):
    n = order + 1
    return 9 * 15 * n + 9 * 4 * n + 420


def lane_ops_fused_forward(grids, order, generation, share):
    """Algorithmic lane-ops of one fused batched forward: the projection of
    every link sample a template's outputs need (n_y = n_out + TDI padding)
    and TDI with each weight set shared by ``share`` templates."""
    return sum(lane_ops_projection(order) * g.n_y +
               lane_ops_tdi(order, generation, share) * g.n_out for g in grids if g.n_out > 0)


def lane_ops_fwd_adjoint(grids, order, generation, share_fwd, share_adj, sky=True):
    """Forward (as above) plus the TDI adjoint (weights shared by
    ``share_adj`` templates), the projection adjoint and the sky gradient."""
    f = lane_ops_fused_forward(grids, order, generation, share_fwd)
    a = sum(lane_ops_tdi(order, generation, share_adj) * g.n_out +
            (lane_ops_projection(order) + (lane_ops_sky(order) if sky else 0)) * g.n_y
            for g in grids if g.n_out > 0)
    return f + a


def batch_bytes(grids, rows=3):
    """Algorithmic HBM bytes of a batched forward: read h+ and hx over each
    template's h range, write its channels."""
    return sum(16.0 * g.n_h + 8.0 * rows * g.n_out for g in grids if g.n_out > 0)


def fwd_adjoint_step_bytes(grids, rows=3):
    """Algorithmic HBM bytes of forward + likelihood + adjoint: the forward
    reads h+, hx and writes the channels; the likelihood reads them and the
    data and writes their gradient; the adjoint reads that gradient and
    h+, hx (for the sky gradient) and writes the gradients of h+ and hx."""
    return sum(48.0 * g.n_h + 8.0 * rows * 5 * g.n_out for g in grids if g.n_out > 0)


def fwd_adjoint_step_bytes_gb(grids, rows=3):
    """The same step in waveform mode (h synthesised in the kernels from the
    parameters): the forward writes the channels; the likelihood reads them
    and the data and writes their gradient; the adjoint reads that gradient.
    No h+, hx or h-gradient traffic."""
    return sum(8.0 * rows * 4 * g.n_out for g in grids if g.n_out > 0)
