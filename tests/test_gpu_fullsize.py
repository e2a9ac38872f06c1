"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: the 512-template uneven batch (1.0e9 output samples) checked on
sampled outputs of several templates against the oracle, and the
256-walker forward + adjoint checked by the dot-product identity, which
holds at any size."""
import numpy as np
import pytest

import oracle
from paper_2204_06633_amd import workloads
from tests import cases

pytestmark = pytest.mark.gpu


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
        idx = cases.sample_indices(g.n_out, 40, seed=k, edge=3)
        ref = cases.oracle_sampled_response(op, op, case, idx)
        got = batch.output_block(out, k)[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
        assert cases.rel_err(got, ref) <= 1e-11, k


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
