"""SGLD / pSGLD sampler and posterior moments (Sec. 3.2, Sec. 3.4).

Step t of chain c (theta_t -> theta_{t+1}):
  1. minibatch of n observations (batch.batch_indices)
  2. g_t = grad log p(theta_t) + (N/n) sum_batch grad log p(y | theta_t)  (eq:sgd)
  3. SGLD:   theta += eps g_t + a sqrt(2 eps) eta                  (as printed)
     pSGLD:  v_t = beta2 v_{t-1} + (1 - beta2) g_t * g_t
             V_t = 1 / (sqrt(v_t) + eps_p)
             theta += eps V_t * g_t + a sqrt(2 eps V_t) * eta      (eq:pSGLD)
     V is diagonal and used elementwise, v starts at 0, no bias correction.
     a is the noise scale (1 while sampling; 0 turns the noise off).
Stages after the initial solution (Sec. 3.2): a warm-up with the injected
noise off, a linear ramp of the noise from zero to full amplitude, then
sampling at full amplitude; stage_noise_scales gives a per step.
  4. after the update of step t, if t >= burn and (t - burn) % thin == 0,
     theta_{t+1} enters the per-event running mean and covariance (Welford).
No Metropolis-Hastings correction (Sec. 3.2).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import batch as batch_mod
from . import likelihood as lk
from . import philox


@dataclasses.dataclass
class SamplerConfig:
    step: float = 1e-4
    beta2: float = 0.99
    eps_p: float = 1e-5
    noise_scale: float = 1.0
    precond: int = 1          # 0 plain SGLD, 1 pSGLD
    burn_in: int = 0
    thin: int = 1
    seed: int = 0
    whiten: int = lk.WHITEN_EXACT
    with_prior: bool = True
    with_centroid: bool = True


@dataclasses.dataclass
class Moments:
    count: int
    mean: np.ndarray   # [M,4]
    m2: np.ndarray     # [M,10]: xx,xy,xz,xt,yy,yz,yt,zz,zt,tt


UPPER = [(a, b) for a in range(4) for b in range(a, 4)]


def moments_empty(M):
    return Moments(0, np.zeros((M, 4)), np.zeros((M, 10)))


def welford(mom: Moments, x):
    """One sample x [M,4] into the running mean and co-moment sums."""
    mom.count += 1
    delta = x - mom.mean
    mom.mean = mom.mean + delta / mom.count
    after = x - mom.mean
    for k, (a, b) in enumerate(UPPER):
        mom.m2[:, k] += delta[:, a] * after[:, b]
    return mom


def pooled(moms):
    """Combine per-chain moments (Chan, Golub and LeVeque's pairwise update)."""
    out = Moments(0, np.zeros_like(moms[0].mean), np.zeros_like(moms[0].m2))
    for m in moms:
        if m.count == 0:
            continue
        n = out.count + m.count
        delta = m.mean - out.mean
        out.m2 = out.m2 + m.m2
        f = out.count * m.count / n
        for k, (a, b) in enumerate(UPPER):
            out.m2[:, k] += delta[:, a] * delta[:, b] * f
        out.mean = out.mean + delta * (m.count / n)
        out.count = n
    return out


def covariance(mom: Moments):
    """Upper-triangle sample covariance, divisor count - 1."""
    return mom.m2 / max(mom.count - 1, 1)


def update(theta, v, g, cfg: SamplerConfig, eta):
    """One Langevin update given the stochastic gradient g and noise eta."""
    if cfg.precond == 0:
        return theta + cfg.step * g + cfg.noise_scale * np.sqrt(2.0 * cfg.step) * eta, v
    v = cfg.beta2 * v + (1.0 - cfg.beta2) * g * g
    V = 1.0 / (np.sqrt(v) + cfg.eps_p)
    theta = theta + cfg.step * V * g + cfg.noise_scale * np.sqrt(2.0 * cfg.step * V) * eta
    return theta, v


@dataclasses.dataclass
class Chain:
    theta: np.ndarray
    v: np.ndarray
    step: int
    mom: Moments


def new_chain(prob: lk.Problem) -> Chain:
    return Chain(prob.hypo0.copy(), np.zeros_like(prob.hypo0), 0, moments_empty(prob.M))


def stochastic_gradient(prob, net, chain: Chain, cfg: SamplerConfig, stream: int,
                        chain_id: int, n: int):
    idx = batch_mod.batch_indices(cfg.seed, stream, chain_id, chain.step, prob.N, n)
    g, lp, bt = lk.grad_log_post(prob, net, chain.theta, idx, cfg.whiten,
                                 cfg.with_prior, cfg.with_centroid)
    return g, lp, idx


def step(prob, net, chain: Chain, cfg: SamplerConfig, stream: int, chain_id: int, n: int):
    """Advance `chain` by one step; returns the log posterior estimate at theta_t."""
    g, lp, _ = stochastic_gradient(prob, net, chain, cfg, stream, chain_id, n)
    eta = philox.noise(cfg.seed, stream, chain_id, chain.step, np.arange(prob.M))
    chain.theta, chain.v = update(chain.theta, chain.v, g, cfg, eta)
    t = chain.step
    if t >= cfg.burn_in and (t - cfg.burn_in) % cfg.thin == 0:
        welford(chain.mom, chain.theta)
    chain.step += 1
    return lp


def stage_noise_scales(warmup: int, ramp: int, sample: int) -> np.ndarray:
    """Noise amplitude a of each step of the staged schedule: 0 during the
    warm-up, k / ramp at step k = 0 .. ramp-1 of the ramp (rising from zero
    toward full amplitude), 1 while sampling."""
    return np.concatenate([np.zeros(warmup), np.arange(ramp) / max(ramp, 1), np.ones(sample)])


def run(prob, net, cfg: SamplerConfig, n: int, steps: int, stream: int = 0, chain_id: int = 0,
        chain: Chain | None = None, keep_states=False, noise_scales=None):
    """`steps` steps of one chain; noise_scales (one per step) overrides
    cfg.noise_scale step by step."""
    chain = new_chain(prob) if chain is None else chain
    states = []
    for k in range(steps):
        c = cfg if noise_scales is None else dataclasses.replace(cfg, noise_scale=float(noise_scales[k]))
        step(prob, net, chain, c, stream, chain_id, n)
        if keep_states:
            states.append(chain.theta.copy())
    return chain, states
