"""Sampler diagnostics and posterior summaries (Sec. 3.4, Sec. 3.6, Sec. 5;
the calibration of the synthetic test in Sec. 4).

Test infrastructure: the plain FP64 reference the GPU path is checked
against.  Only the tests, the smoke entry point and the benchmark's CPU
baseline use it.

* credibility bounds: per parameter, the percentile of probability p over
  the samples, interpolated linearly between the order statistics around
  (S - 1) p (numpy's default percentile);
* calibration: where a reference value (the synthetic truth) falls among
  a parameter's samples, (#below + #equal / 2) / S;
* effective sample size over draws x[K][C][P] (C chains of K draws): chain
  means and variances (divisor K - 1), W = mean within-chain variance,
  B/K = variance of the chain means (divisor C - 1), var+ = (K-1)/K W + B/K;
  rho_t = 1 - (W - mean_c acov_c(t)) / var+ with the chain autocovariance
  acov_c(t) = (1/K) sum_{i<K-t} (x_i - mu_c)(x_{i+t} - mu_c), rho_0 = 1;
  Geyer's initial positive sequence of pair sums rho_2k + rho_2k+1, made
  non-increasing; tau = -1 + 2 sum, ESS = C K / tau (NaN if var+ = 0);
* step-size ratio: at a chain's state, the likelihood gradients of its next
  K sampler minibatches, their per-coordinate variance Var(g) (divisor
  K - 1), and step V Var(g) / (2 a^2): the variance of the drift term
  step V g of the update over that of the injected noise a sqrt(2 step V)
  eta, with V the pSGLD preconditioner 1/(sqrt(v) + eps_p) (or 1).
"""
from __future__ import annotations

import numpy as np

from . import batch as batch_mod
from . import likelihood as lk


def quantiles(samples, probs):
    """[len(probs), ...] percentiles over the first axis of samples."""
    return np.percentile(np.asarray(samples, np.float64), 100.0 * np.asarray(probs), axis=0)


def sample_ranks(samples, values):
    """Position of values [...] among samples [S, ...] as a fraction."""
    s = np.asarray(samples, np.float64)
    below = (s < values).sum(0)
    ties = (s == values).sum(0)
    return (below + 0.5 * ties) / s.shape[0]


def ess(draws):
    """Effective sample size of each parameter of draws [K, C, P]."""
    x = np.asarray(draws, np.float64)
    K, C = x.shape[0], x.shape[1]
    mu = x.mean(0)                                  # [C, P]
    W = x.var(0, ddof=1).mean(0)                    # [P]
    BK = mu.var(0, ddof=1) if C > 1 else np.zeros_like(W)
    var_plus = (K - 1) / K * W + BK
    d = x - mu[None]
    out = np.full(W.shape, np.nan)
    for p in range(W.shape[0]):
        if not var_plus[p] > 0.0:
            continue

        def rho(t):
            if t == 0:
                return 1.0
            acov = (d[:K - t, :, p] * d[t:, :, p]).sum(0) / K   # [C]
            return 1.0 - (W[p] - acov.mean()) / var_plus[p]

        total, prev, k = 0.0, np.inf, 0
        while 2 * k + 1 < K:
            pk = rho(2 * k) + rho(2 * k + 1)
            if not pk > 0.0:
                break
            pk = min(pk, prev)
            prev = pk
            total += pk
            k += 1
        out[p] = C * K / (-1.0 + 2.0 * total)
    return out


def gradient_variance(prob, net, theta, seed, stream, chain, t0, n, K, mode=lk.WHITEN_EXACT):
    """Per-coordinate variance (divisor K - 1) of the likelihood gradients
    (scale N/n) of the minibatches of steps t0 .. t0+K-1 of a chain."""
    Gs = []
    for k in range(K):
        idx = batch_mod.batch_indices(seed, stream, chain, t0 + k, prob.N, n)
        bt = lk.batch_terms(prob, net, theta, idx, mode)
        Gs.append(lk.likelihood_gradient(prob, bt, prob.N / n)[0])
    return np.var(np.stack(Gs), axis=0, ddof=1)


def noise_ratio(var_g, v, step, eps_p=1e-5, noise_scale=1.0, precond=True):
    """step V Var(g) / (2 a^2) per coordinate."""
    V = 1.0 / (np.sqrt(v) + eps_p) if precond else np.ones_like(var_g)
    return step * V * var_g / (2.0 * noise_scale ** 2)
