"""One step of the parallel-tempered stretch-move ensemble sampler (plain
NumPy loops; test infrastructure only, like the rest of ``oracle``).

Follows Sec. II.B of arXiv:2204.06633 (emcee's ensemble architecture with
ptemcee's parallel tempering, stretch proposal only), written from the
published definitions:
  * stretch move (Goodman and Weare 2010): for walker j of the active half
    of the ensemble at inverse temperature beta and a walker k of the other
    half, y = x_k + z (x_j - x_k), z ~ g(z) = 1/sqrt(z) on [1/a, a]; accept
    if log u < (D - 1) log z + beta (log L(y) - log L(x_j)) + log pi(y) -
    log pi(x_j).  The first half of the walkers moves first, then the
    second half against the updated first half;
  * tempering swaps (Vousden et al. 2016): for each pair of adjacent
    temperatures, hottest pair first, walker perm_hi[w] of the hotter chain
    and perm_lo[w] of the colder chain exchange places if log u <
    (beta_cold - beta_hot) (log L_hot - log L_cold).
The random numbers (z, partner indices, log u, permutations) are inputs.
"""
from __future__ import annotations

import math



def log_prior_box(theta, lo, hi):
    return 0.0 if all(lo[i] <= theta[i] <= hi[i] for i in range(len(theta))) else -math.inf


def step(x, ll, lp, betas, draws, loglike, lo, hi, margins=None):
    """x [T][W][D], ll, lp [T][W] (NumPy, not modified); draws: dict of
    NumPy arrays z, partner, log_u [2][T][W/2], perm_hi, perm_lo,
    log_u_swap [T-1][W]; loglike(list of theta) -> list of log L.
    Returns (x, ll, lp, accepted per temperature, swaps per pair).  If
    ``margins`` is a list, |log u - log r| of every finite decision is
    appended to it."""
    x, ll, lp = x.copy(), ll.copy(), lp.copy()
    T, W, D = x.shape
    h = W // 2
    n_acc = [0] * T
    for half in range(2):
        act = range(half * h, (half + 1) * h)
        oth = range((1 - half) * h, (2 - half) * h)
        props = []
        for t in range(T):
            for i, j in enumerate(act):
                k = oth[int(draws["partner"][half][t][i])]
                z = float(draws["z"][half][t][i])
                props.append([x[t, k, m] + z * (x[t, j, m] - x[t, k, m]) for m in range(D)])
        # proposals outside the prior are scored at their nearest in-box point
        # (the value never matters: such proposals are rejected)
        clamped = [[min(max(v, lo[m]), hi[m]) for m, v in enumerate(p)] for p in props]
        lls = loglike(clamped)
        for t in range(T):
            for i, j in enumerate(act):
                idx = t * h + i
                y = props[idx]
                lp_y = log_prior_box(y, lo, hi)
                z = float(draws["z"][half][t][i])
                log_r = (D - 1) * math.log(z) + betas[t] * (lls[idx] - ll[t, j]) + lp_y - lp[t, j]
                if margins is not None and math.isfinite(log_r):
                    margins.append(abs(float(draws["log_u"][half][t][i]) - log_r))
                if math.isfinite(lp_y) and float(draws["log_u"][half][t][i]) < log_r:
                    x[t, j] = y
                    ll[t, j] = lls[idx]
                    lp[t, j] = lp_y
                    n_acc[t] += 1
    n_swap = [0] * max(T - 1, 0)
    for i in range(T - 1, 0, -1):
        for w in range(W):
            a = int(draws["perm_hi"][i - 1][w])
            b = int(draws["perm_lo"][i - 1][w])
            p_acc = (betas[i - 1] - betas[i]) * (ll[i, a] - ll[i - 1, b])
            if margins is not None:
                margins.append(abs(float(draws["log_u_swap"][i - 1][w]) - p_acc))
            if float(draws["log_u_swap"][i - 1][w]) < p_acc:
                for arr in (x, ll, lp):
                    arr[i, a], arr[i - 1, b] = arr[i - 1, b].copy(), arr[i, a].copy()
                n_swap[i - 1] += 1
    return x, ll, lp, n_acc, n_swap


def theta_to_source(theta):
    """(ln A, f0 [mHz], fdot, cos iota, phi0, psi, lambda, sin beta) ->
    (A, f0 [Hz], fdot, phi0, iota, psi, lambda, beta), the sampling
    coordinates of Table I."""
    t = [float(v) for v in theta]
    return [math.exp(t[0]), t[1] * 1e-3, t[2], t[4], math.acos(max(-1.0, min(1.0, t[3]))), t[5],
            t[6], math.asin(max(-1.0, min(1.0, t[7])))]
