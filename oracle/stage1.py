"""Stage 1: a robust initial solution (Sec. 3.2, eq:stage1loss).

Test infrastructure: the plain FP64 reference the GPU path is checked
against.  Only the tests, the smoke entry point and the benchmark's CPU
baseline use it.

The loss is the L1 norm of the dd residuals over a minibatch,
  L(theta) = (1/n) sum_{k<n} |r_k(theta)|,   r = tau - tau^(theta)  (Eq. 1),
minimised with Adam (eta from Table 1) and no priors.  Its gradient is
  dL/dtheta = -(1/n) sum_k sign(r_k) dtau^_k/dtheta,
i.e. the likelihood gradient's assembly with z = sign(r) and scale 1/n.
After Stage 1, observations whose residual lies more than 4 median absolute
deviations from the median residual are discarded (outlier_mask).
Minibatch t of chain c is the sampler's (batch.batch_indices), and Adam's
bias correction uses step k = t + 1:
  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
  theta -= eta (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import batch as batch_mod
from . import likelihood as lk


@dataclasses.dataclass
class AdamConfig:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    seed: int = 0


@dataclasses.dataclass
class AdamState:
    theta: np.ndarray
    m: np.ndarray
    v: np.ndarray
    step: int


def new_state(prob: lk.Problem) -> AdamState:
    z = np.zeros_like(prob.hypo0)
    return AdamState(prob.hypo0.copy(), z, z.copy(), 0)


def l1_loss_gradient(prob: lk.Problem, net, theta, idx):
    """L and -dL/dtheta ([M,4]) of the minibatch idx, with its batch terms."""
    idx = np.asarray(idx, np.int64)
    n = idx.shape[0]
    bt = lk.batch_terms(prob, net, theta, idx, lk.L1)
    G, _ = lk.likelihood_gradient(prob, bt, 1.0 / n)
    return float(np.abs(bt.r).sum()) / n, G, bt


def adam_update(theta, m, v, g, k: int, cfg: AdamConfig):
    """One Adam step on gradient g at step k (1-based)."""
    m = cfg.beta1 * m + (1.0 - cfg.beta1) * g
    v = cfg.beta2 * v + (1.0 - cfg.beta2) * g * g
    mh = m / (1.0 - cfg.beta1 ** k)
    vh = v / (1.0 - cfg.beta2 ** k)
    return theta - cfg.lr * mh / (np.sqrt(vh) + cfg.eps), m, v


def step(prob, net, st: AdamState, cfg: AdamConfig, stream: int, chain_id: int, n: int):
    """Advance st by one Adam step on the minibatch L1 loss; returns L."""
    idx = batch_mod.batch_indices(cfg.seed, stream, chain_id, st.step, prob.N, n)
    loss, G, _ = l1_loss_gradient(prob, net, st.theta, idx)
    st.theta, st.m, st.v = adam_update(st.theta, st.m, st.v, -G, st.step + 1, cfg)
    st.step += 1
    return loss


def run(prob, net, cfg: AdamConfig, n: int, steps: int, stream: int = 0, chain_id: int = 0,
        st: AdamState | None = None):
    st = new_state(prob) if st is None else st
    losses = [step(prob, net, st, cfg, stream, chain_id, n) for _ in range(steps)]
    return st, losses


def outlier_mask(prob: lk.Problem, net, theta, k_mad: float = 4.0):
    """Residuals of all observations at theta, their median and median
    absolute deviation MAD = median |r - median(r)|, and the mask of the
    observations with |r - median(r)| <= k_mad MAD."""
    r = lk.batch_terms(prob, net, theta, np.arange(prob.N), lk.L1).r
    med = float(np.median(r))
    mad = float(np.median(np.abs(r - med)))
    return np.abs(r - med) <= k_mad * mad, med, mad, r
