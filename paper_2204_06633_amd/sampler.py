"""Parallel-tempered ensemble sampler with the stretch move (Sec. II.B),
driving the batched response and the frequency-domain likelihood.

Per step and temperature the walkers are split into two halves; each walker
of the active half moves along the line through a random walker of the
other half (the affine-invariant stretch move of Goodman and Weare, 2010):
y = x_k + z (x_j - x_k) with z drawn from g(z) ~ 1/sqrt(z) on [1/a, a], and
is accepted with probability min(1, z^(D-1) pi(y) L(y)^beta / (pi(x_j)
L(x_j)^beta)).  All proposals of a half step, over every temperature, are
scored in one batched likelihood call (polarisations, response and
likelihood all in the HIP library).  Then adjacent temperatures exchange
walkers, hottest pair first (the parallel-tempering swaps of ptemcee,
Vousden et al. 2016): walkers of the two chains are paired by two random
permutations and a pair swaps with probability min(1, exp((beta_i -
beta_{i+1}) (log L_{i+1} - log L_i))).

The random numbers are drawn up front (``draw``) and passed to ``step``, so
a step is a deterministic function of its inputs.  The parameter vector is
theta = (ln A, f0 [mHz], fdot [Hz/s], cos iota, phi0, psi, lambda, sin beta)
with the uniform box prior of Table I.
"""
from __future__ import annotations

import dataclasses
import math

import torch

G_MSUN_C3 = 4.925490947641267e-06        # G M_sun / c^3 in seconds
NDIM = 8


def fdot_gw(f0, mc_solar):
    """Eq. (fdot): fdot = 96/5 pi^(8/3) (G Mc / c^3)^(5/3) f^(11/3)."""
    return 96.0 / 5.0 * math.pi ** (8.0 / 3.0) * (mc_solar * G_MSUN_C3) ** (5.0 / 3.0) * \
        f0 ** (11.0 / 3.0)


def prior_box(A_star, f0_star):
    """Lower and upper bounds of theta (Table I)."""
    lo = [math.log(A_star * 1e-2), 0.5, fdot_gw(f0_star, 1e-3), -1.0, 0.0, 0.0, 0.0, -1.0]
    hi = [math.log(A_star * 1e2), 12.0, fdot_gw(f0_star, 1.0), 1.0, 2 * math.pi, math.pi,
          2 * math.pi, 1.0]
    return lo, hi


def to_theta(source):
    """Waveform parameters (A, f0, fdot, phi0, iota, psi, lam, beta) -> theta."""
    s = torch.as_tensor(source, dtype=torch.float64)
    return torch.stack([torch.log(s[..., 0]), s[..., 1] * 1e3, s[..., 2], torch.cos(s[..., 4]),
                        s[..., 3], s[..., 5], s[..., 6], torch.sin(s[..., 7])], -1)


def to_source(theta):
    """theta -> waveform parameters (A, f0, fdot, phi0, iota, psi, lam, beta)."""
    th = theta
    return torch.stack([torch.exp(th[..., 0]), th[..., 1] * 1e-3, th[..., 2],
                        th[..., 4], torch.acos(th[..., 3].clamp(-1.0, 1.0)), th[..., 5],
                        th[..., 6], torch.asin(th[..., 7].clamp(-1.0, 1.0))], -1)


@dataclasses.dataclass
class StepDraws:
    """Random numbers of one step: T temperatures, W walkers (even)."""
    z: torch.Tensor            # [2][T][W/2] stretch factors
    partner: torch.Tensor      # [2][T][W/2] index into the other half
    log_u: torch.Tensor        # [2][T][W/2] log of uniform(0, 1) for acceptance
    perm_hi: torch.Tensor      # [T-1][W] walker order of the hotter chain of pair i
    perm_lo: torch.Tensor      # [T-1][W] walker order of the colder chain
    log_u_swap: torch.Tensor   # [T-1][W]


def draw(gen, T, W, a=2.0, device="cuda"):
    """StepDraws from a torch generator (on ``device``)."""
    h = W // 2
    u = torch.rand((2, T, h), dtype=torch.float64, device=device, generator=gen)
    z = ((a - 1.0) * u + 1.0) ** 2 / a
    partner = torch.randint(0, h, (2, T, h), device=device, generator=gen)
    log_u = torch.log(torch.rand((2, T, h), dtype=torch.float64, device=device, generator=gen))
    perm_hi = torch.stack([torch.randperm(W, device=device, generator=gen) for _ in range(T - 1)]) \
        if T > 1 else torch.empty((0, W), dtype=torch.int64, device=device)
    perm_lo = torch.stack([torch.randperm(W, device=device, generator=gen) for _ in range(T - 1)]) \
        if T > 1 else torch.empty((0, W), dtype=torch.int64, device=device)
    log_u_swap = torch.log(torch.rand((max(T - 1, 0), W), dtype=torch.float64, device=device,
                                      generator=gen))
    return StepDraws(z, partner, log_u, perm_hi, perm_lo, log_u_swap)


def log_prior(theta, lo, hi):
    """0 inside the box, -inf outside (a uniform density up to a constant)."""
    lo = torch.as_tensor(lo, dtype=theta.dtype, device=theta.device)
    hi = torch.as_tensor(hi, dtype=theta.dtype, device=theta.device)
    inside = ((theta >= lo) & (theta <= hi)).all(-1)
    return torch.where(inside, torch.zeros_like(theta[..., 0]),
                       torch.full_like(theta[..., 0], -math.inf))


class PTSampler:
    """State x [T][W][D], log L [T][W], log prior [T][W] on the device.

    ``loglike(theta [M][D]) -> [M]`` scores a batch of proposals; entries
    outside the prior are never used (they are clamped into the box before
    the call so every template stays finite)."""

    def __init__(self, loglike, betas, lo, hi, a=2.0):
        self.loglike = loglike
        self.betas = torch.as_tensor(betas, dtype=torch.float64)
        if self.betas.dim() != 1 or len(self.betas) < 1:
            raise ValueError("betas must be a non-empty list")
        if not bool((self.betas[:-1] >= self.betas[1:]).all()) or float(self.betas[0]) > 1.0 \
                or float(self.betas[-1]) < 0.0:
            raise ValueError("betas must fall from at most 1 to at least 0")
        if len(lo) != len(hi) or any(l >= h for l, h in zip(lo, hi)):
            raise ValueError("prior box: lo < hi in every dimension")
        self.lo, self.hi, self.a = lo, hi, a

    def _check(self, x):
        T, W, D = x.shape
        if T != len(self.betas):
            raise ValueError("%d temperatures in the state, %d betas" % (T, len(self.betas)))
        if W < 4 or W % 2:
            raise ValueError("walkers per temperature must be even and at least 4, got %d" % W)
        if D != len(self.lo):
            raise ValueError("%d parameters in the state, %d in the prior box" % (D, len(self.lo)))

    def initial(self, x):
        self._check(x)
        T, W, D = x.shape
        lp = log_prior(x, self.lo, self.hi)
        ll = self.loglike(x.reshape(T * W, D)).reshape(T, W)
        return x.clone(), ll, lp

    def step(self, x, ll, lp, d: StepDraws):
        self._check(x)
        T, W, D = x.shape
        h = W // 2
        betas = self.betas.to(x.device)
        lo = torch.as_tensor(self.lo, dtype=x.dtype, device=x.device)
        hi = torch.as_tensor(self.hi, dtype=x.dtype, device=x.device)
        x, ll, lp = x.clone(), ll.clone(), lp.clone()
        n_acc = torch.zeros((T,), dtype=torch.int64, device=x.device)
        tix = torch.arange(T, device=x.device)[:, None]
        for half in range(2):
            act = slice(half * h, (half + 1) * h)
            oth = slice((1 - half) * h, (2 - half) * h)
            xa, xo = x[:, act], x[:, oth]
            xk = xo[tix, d.partner[half]]                       # [T][h][D]
            z = d.z[half]
            y = xk + z[..., None] * (xa - xk)
            lp_y = log_prior(y, self.lo, self.hi)
            ll_y = self.loglike(torch.minimum(torch.maximum(y, lo), hi).reshape(T * h, D))
            ll_y = ll_y.reshape(T, h)
            log_r = (D - 1) * torch.log(z) + betas[:, None] * (ll_y - ll[:, act]) + lp_y - \
                lp[:, act]
            acc = torch.isfinite(lp_y) & (d.log_u[half] < log_r)
            x[:, act] = torch.where(acc[..., None], y, xa)
            ll[:, act] = torch.where(acc, ll_y, ll[:, act])
            lp[:, act] = torch.where(acc, lp_y, lp[:, act])
            n_acc += acc.sum(-1)
        n_swap = torch.zeros((max(T - 1, 0),), dtype=torch.int64, device=x.device)
        for i in range(T - 1, 0, -1):                           # hottest pair first
            hi_i, lo_i = d.perm_hi[i - 1], d.perm_lo[i - 1]
            p_acc = (betas[i - 1] - betas[i]) * (ll[i, hi_i] - ll[i - 1, lo_i])
            sel = d.log_u_swap[i - 1] < p_acc
            a_hi, a_lo = hi_i[sel], lo_i[sel]
            for arr in (x, ll, lp):
                tmp = arr[i, a_hi].clone()
                arr[i, a_hi] = arr[i - 1, a_lo]
                arr[i - 1, a_lo] = tmp
            n_swap[i - 1] = sel.sum()
        return x, ll, lp, n_acc, n_swap


class BatchLoglike:
    """log L(theta) for walkers sharing one output grid: lr_response_gb (the
    fused batch kernel synthesising each walker's h+ / hx in its LDS windows
    from the parameter rows) -> lr_fd_loglike statistics, ``m`` walkers per
    call.  ``batch``: a native.Batch of ``m`` equal templates (their h
    offsets unused), each with n_h h-samples at waveform times (k0 + j) dt,
    k0 = -out_start; ``plan``: an FdPlan on the data; theta [M][8] with M a
    multiple of m.

    With ``graph`` (the default) the sequence of one chunk of m walkers
    (sampling coordinates -> source parameters, response, statistics,
    log L) is captured once in a HIP graph with static input and output
    buffers and replayed for every chunk.  Replays give the same numbers as
    the eager sequence, bit for bit."""

    def __init__(self, batch, plan, k0, n_h, dt, m, device="cuda", graph=True):
        self.batch, self.plan, self.m = batch, plan, m
        self.k0, self.n_h, self.dt = int(k0), int(n_h), float(dt)
        self.n_out = plan.n
        self.out = torch.empty(batch.out_extent, dtype=torch.float64, device=device)
        self.stats = torch.empty((m, 3), dtype=torch.float64, device=device)
        self.theta_in = torch.zeros((m, NDIM), dtype=torch.float64, device=device)
        self.src = torch.empty((m, NDIM), dtype=torch.float64, device=device)
        self.ll_out = torch.empty(m, dtype=torch.float64, device=device)
        self.use_graph = bool(graph)
        self.graph = None

    def _chunk(self):
        """One chunk on the current stream, from theta_in to ll_out."""
        m = self.m
        self.src.copy_(to_source(self.theta_in))
        self.batch.response_gb(self.src, out=self.out)
        h = self.out[:m * 3 * self.n_out].view(m, 3, self.n_out)
        self.plan.loglike(h, want_grad=False, stats=self.stats)
        torch.mul(self.stats[:, 0], -0.5, out=self.ll_out)

    def _capture(self):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._chunk()                               # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._chunk()
        self.graph = g

    def __call__(self, theta):
        M, m = theta.shape[0], self.m
        if M % m:
            raise ValueError("%d proposals for a batch of %d walkers" % (M, m))
        out = []
        for c in range(0, M, m):
            self.theta_in.copy_(theta[c:c + m])
            if self.use_graph:
                if self.graph is None:
                    self._capture()
                self.graph.replay()
            else:
                self._chunk()
            out.append(self.ll_out.clone())
        return torch.cat(out)


@dataclasses.dataclass
class PTRun:
    """A ready tempered run on the device: sampler, state and random source."""
    case: object
    sampler: PTSampler
    x: torch.Tensor
    ll: torch.Tensor
    lp: torch.Tensor
    gen: torch.Generator
    tuned: dict

    def step(self):
        d = draw(self.gen, self.case.T, self.case.W, device=self.x.device)
        self.x, self.ll, self.lp, acc, sw = self.sampler.step(self.x, self.ll, self.lp, d)
        return acc, sw


def setup_run(sc, device="cuda", betas=(1.0, 0.25, 0.0625, 0.0), seed=9, tune=True, log=None):
    """Everything a tempered run on a ``workloads.SamplerCase`` needs: the
    orbits on the device, a batch of T W / 2 walkers (group and grid tuned on
    the batch when ``tune``), noise-free data from the injection, the
    frequency-domain plan with the stand-in noise curve, the Table I prior
    box around the injection, and walkers started in a small ball around it
    (the initial likelihoods evaluated)."""
    import numpy as np

    from . import autotune, inputs, native
    dev = torch.device(device)
    g = sc.grid
    orb = native.Orbits.from_samples(sc.orbits, device=dev)
    src_all = torch.tensor(sc.injection, dtype=torch.float64, device=dev).repeat(sc.m, 1)
    if tune:
        batch, tuned = autotune.tuned_batch(sc.layout(sc.m), orb, orb, g.t_start, g.dt,
                                            sc.order, sc.generation, "AET", None, None, None,
                                            params=src_all)
    else:
        batch = native.Batch(sc.layout(sc.m), orb, orb, g.t_start, g.dt, sc.order,
                             sc.generation, "AET", group=2, device=dev)
        tuned = {"group": 2, "grid_scale": 1.0}
    if log:
        log("sampler: %s, %d proposals per half step, group %d, tile %d, grid x%.1f"
            % (sc.name, sc.m, tuned["group"], batch.tile, tuned["grid_scale"]))
    # noise-free data: the injection through the same batch machinery
    one = native.Batch(sc.layout(1), orb, orb, g.t_start, g.dt, sc.order, sc.generation, "AET",
                       group=1, device=dev)
    data = torch.empty(one.out_extent, dtype=torch.float64, device=dev)
    one.response_gb(src_all[:1].contiguous(), out=data)
    del one
    n_fft = native.fd_length(g.n_out)
    w_ae, w_t = inputs.noise_weights(n_fft, g.dt)
    plan = native.FdPlan(data.view(3, g.n_out), torch.tensor(w_ae, device=dev),
                         torch.tensor(w_t, device=dev), g.dt, max_batch=sc.m)
    lo, hi = prior_box(sc.injection[0], sc.injection[1])
    ps = PTSampler(BatchLoglike(batch, plan, -g.out_start, g.n_h, g.dt, sc.m, device=dev),
                   list(betas), lo, hi)
    rng = np.random.default_rng(seed)
    th0 = to_theta(torch.tensor(sc.injection)).numpy()
    scale = np.array([1e-2, 1e-7, 1e-17, 1e-2, 1e-2, 1e-2, 1e-3, 1e-3])
    x, ll, lp = ps.initial(torch.tensor(th0 + scale * rng.standard_normal((sc.T, sc.W, 8)),
                                        device=dev))
    gen = torch.Generator(device=dev).manual_seed(seed + 1)
    return PTRun(sc, ps, x, ll, lp, gen, tuned)
