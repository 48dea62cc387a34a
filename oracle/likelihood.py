"""Correlated-Gaussian double-difference likelihood of Sec. 3.1.

Observation n links events i = xi^1_n and j = xi^2_n at station eta_n in
phase phi_n (0 = P, 1 = S); its station-phase group is g = eta_n + L phi_n.
Each phase has its own travel-time network T_phi and its own sigma_phi,
kappa_phi (Sec. 3.1); a catalog without S observations has groups = stations.

  residual   r_n = tau_n - [T_phi(x_i; s) - T_phi(x_j; s) + t_i - t_j]
             (Eq. 1 and eq:forwardmodel; the latent term Delta b is
             marginalised, so r_g = W_g^{1/2} A_g b_g + eps_g)
  weights    w~_e = (d_e / ell)^p + eps,  d_e = |x_i - x_j|   (eq:correlation_decay)
             normalised to mean 1 over each group's observations in the
             catalog; d_e is taken at the initial locations theta_0.
  covariance Sigma_g = sigma_phi^2 I + kappa_phi^2 W^{1/2} A A^T W^{1/2}   (eq:marginal_sigma)
             A has +1 at event i and -1 at event j of each row.
  likelihood log p = sum_g -1/2 r_g^T Sigma_g^{-1} r_g + const.

A minibatch uses the Gaussian marginal of its own observations, whose
covariance is the sub-block Sigma_B of Sigma_g on them; z = Sigma_B^{-1} r is
found by a sparse direct solve of Sigma_B itself (U U^T is sparse: two rows
couple only when they share an event in the same group).

Gradient (ascent, d/dtheta of log p):  dtau^/dx_i = grad T(x_i), dtau^/dt_i = 1,
dtau^/dx_j = -grad T(x_j), dtau^/dt_j = -1, and d(-1/2 r^T Sigma^-1 r)/dtheta
= (dtau^/dtheta)^T z.  The minibatch term is scaled by N/n (eq:sgd).

Priors (Sec. 3.1):  theta_m ~ N(mu_e = theta0_m, diag sigma_e^2), and the
centroid thetabar = mean_m theta_m ~ N(mu_c = mean_m theta0_m, diag sigma_c^2).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .travel_time import travel_time

WHITEN_NONE, WHITEN_DIAG, WHITEN_EXACT = 0, 1, 2
L1 = 3  # not a whitening: z = sign(r), the derivative of |r| (Stage 1 loss)


@dataclasses.dataclass
class Problem:
    """A catalog as the oracle sees it after its own load step."""
    hypo0: np.ndarray       # [M,4]
    stations: np.ndarray    # [L,3]
    pair_i: np.ndarray
    pair_j: np.ndarray
    obs_pair: np.ndarray
    obs_sta: np.ndarray     # [N] station
    obs_dt: np.ndarray      # float64 copy of the float32 observations
    w_pair: np.ndarray      # [P] unnormalised edge weights
    inv_mean: np.ndarray    # [G] 1 / group mean of w over the catalog
    sigma: float            # P phase
    kappa: float
    prior_sigma: np.ndarray  # [4]
    centroid_sigma: np.ndarray  # [4]
    mu_c: np.ndarray        # [4]
    obs_phase: np.ndarray = None  # [N] 0 = P, 1 = S
    obs_group: np.ndarray = None  # [N] station + L phase
    sigma_s: float = None   # S phase
    kappa_s: float = None

    @property
    def M(self):
        return self.hypo0.shape[0]

    @property
    def N(self):
        return self.obs_pair.shape[0]

    @property
    def G(self):
        return self.inv_mean.shape[0]

    @property
    def two_phase(self):
        return bool(np.any(self.obs_phase))

    def row_sigma_kappa(self, phase):
        """sigma_phi and kappa_phi of observations of the given phases."""
        return (np.where(phase == 1, self.sigma_s, self.sigma),
                np.where(phase == 1, self.kappa_s, self.kappa))


def edge_weights(hypo0, pair_i, pair_j, ell, p, eps_w):
    """w~_e = (d_e/ell)^p + eps with d_e from the initial locations."""
    d = np.sqrt(((hypo0[pair_i, 0:3] - hypo0[pair_j, 0:3]) ** 2).sum(1))
    return (d / ell) ** p + eps_w


def group_inverse_mean(w_pair, obs_pair, group, G):
    """1 / mean over each group's catalog observations of w~."""
    cnt = np.bincount(group, minlength=G).astype(np.float64)
    tot = np.bincount(group, weights=w_pair[obs_pair], minlength=G)
    inv = np.zeros(G)
    nz = cnt > 0
    inv[nz] = cnt[nz] / tot[nz]
    return inv


def load(cat, sigma=None, kappa=None, p=None, ell=None, eps_w=None,
         prior_sigma=None, centroid_sigma=None, sigma_s=None, kappa_s=None) -> Problem:
    wl = cat.wl
    sigma = wl.sigma if sigma is None else sigma
    kappa = wl.kappa if kappa is None else kappa
    sigma_s = wl.sigma_s if sigma_s is None else sigma_s
    kappa_s = wl.kappa_s if kappa_s is None else kappa_s
    p = wl.p if p is None else p
    ell = wl.ell if ell is None else ell
    eps_w = wl.eps_w if eps_w is None else eps_w
    w_pair = edge_weights(cat.hypo0, cat.pair_i, cat.pair_j, ell, p, eps_w)
    sta = cat.obs_sta.astype(np.int64)
    phase = (np.zeros(cat.N, np.int64) if cat.obs_phase is None
             else cat.obs_phase.astype(np.int64))
    n_phases = 2 if np.any(phase) else 1
    group = sta + cat.L * phase
    inv_mean = group_inverse_mean(w_pair, cat.obs_pair, group, n_phases * cat.L)
    return Problem(
        hypo0=np.asarray(cat.hypo0, np.float64), stations=np.asarray(cat.stations, np.float64),
        pair_i=cat.pair_i.astype(np.int64), pair_j=cat.pair_j.astype(np.int64),
        obs_pair=cat.obs_pair.astype(np.int64), obs_sta=sta,
        obs_phase=phase, obs_group=group, sigma_s=float(sigma_s), kappa_s=float(kappa_s),
        obs_dt=cat.obs_dt.astype(np.float64), w_pair=w_pair, inv_mean=inv_mean,
        sigma=float(sigma), kappa=float(kappa),
        prior_sigma=np.asarray(wl.prior_sigma if prior_sigma is None else prior_sigma, np.float64),
        centroid_sigma=np.asarray(wl.centroid_sigma if centroid_sigma is None else centroid_sigma,
                                  np.float64),
        mu_c=np.asarray(cat.hypo0, np.float64).mean(0))


@dataclasses.dataclass
class BatchTerms:
    ev_i: np.ndarray
    ev_j: np.ndarray
    group: np.ndarray
    phase: np.ndarray
    tau: np.ndarray
    w: np.ndarray
    T_i: np.ndarray
    T_j: np.ndarray
    gT_i: np.ndarray
    gT_j: np.ndarray
    r: np.ndarray
    z: np.ndarray


def gather(prob: Problem, idx):
    idx = np.asarray(idx, np.int64)
    pr = prob.obs_pair[idx]
    ev_i, ev_j = prob.pair_i[pr], prob.pair_j[pr]
    g = prob.obs_group[idx]
    w = prob.w_pair[pr] * prob.inv_mean[g]
    return ev_i, ev_j, g, prob.obs_dt[idx], w


def phase_nets(net):
    """(P network, S network) from one network or a pair of them."""
    return tuple(net) if isinstance(net, (tuple, list)) else (net, net)


def travel_times(nets, phase, x, s):
    """T and dT/dx of rows with sources x and receivers s, each row through
    the network of its phase."""
    T = np.empty(x.shape[0])
    g = np.empty((x.shape[0], 3))
    for ph, net in enumerate(phase_nets(nets)):
        sel = phase == ph
        if np.any(sel):
            T[sel], g[sel] = travel_time(net, x[sel], s[sel])
    return T, g


def residuals(T_i, T_j, t_i, t_j, tau):
    """r_n = tau_n - [(T_i - T_j) + (t_i - t_j)]."""
    return tau - ((T_i - T_j) + (t_i - t_j))


def whiten(r, w, group, ev_i, ev_j, M, sigma, kappa, mode):
    """z = Sigma_B^{-1} r for the minibatch's observations; sigma and kappa
    are scalars or per-observation values (those of its group's phase)."""
    s2 = np.asarray(sigma, np.float64) ** 2
    k = np.asarray(kappa, np.float64)
    if mode == L1:
        return np.sign(r)
    if mode == WHITEN_NONE or np.all(k == 0.0):
        return r / s2
    if mode == WHITEN_DIAG:
        return r / (s2 + 2.0 * k * k * w)
    # columns of A_B: the (group, event) pairs the batch touches; A is block
    # diagonal over groups, +1 at event i and -1 at event j of each row
    key_i = group * M + ev_i
    key_j = group * M + ev_j
    nodes, inv = np.unique(np.concatenate([key_i, key_j]), return_inverse=True)
    n = r.shape[0]
    # row n of U is kappa_n sqrt(w_n) A_n: rows of different groups never
    # share a node, so U U^T holds each group's kappa_phi^2 W^1/2 A A^T W^1/2
    kw = np.broadcast_to(k, (n,)) * np.sqrt(w)
    rows = np.concatenate([np.arange(n), np.arange(n)])
    U = sp.csr_matrix((np.concatenate([kw, -kw]), (rows, inv)), shape=(n, nodes.shape[0]))
    Sigma = sp.diags(np.broadcast_to(s2, (n,))) + U @ U.T
    return np.atleast_1d(spla.spsolve(Sigma.tocsc(), r))


def batch_terms(prob: Problem, net, theta, idx, mode=WHITEN_EXACT) -> BatchTerms:
    """Per-observation terms of minibatch idx; net is the network, or the
    (P, S) pair of a two-phase catalog."""
    ev_i, ev_j, g, tau, w = gather(prob, idx)
    idx = np.asarray(idx, np.int64)
    ph = prob.obs_phase[idx]
    s = prob.stations[prob.obs_sta[idx]]
    T_i, gT_i = travel_times(net, ph, theta[ev_i, 0:3], s)
    T_j, gT_j = travel_times(net, ph, theta[ev_j, 0:3], s)
    r = residuals(T_i, T_j, theta[ev_i, 3], theta[ev_j, 3], tau)
    sig, kap = prob.row_sigma_kappa(ph)
    z = whiten(r, w, g, ev_i, ev_j, prob.M, sig, kap, mode)
    return BatchTerms(ev_i, ev_j, g, ph, tau, w, T_i, T_j, gT_i, gT_j, r, z)


def likelihood_gradient(prob: Problem, bt: BatchTerms, scale: float):
    """scale * sum_n (dtau^_n/dtheta)^T z_n as an [M,4] array, and the batch
    log-likelihood -1/2 scale * r^T z (up to an additive constant)."""
    G = np.zeros((prob.M, 4))
    cz = scale * bt.z
    np.add.at(G[:, 0:3], bt.ev_i, cz[:, None] * bt.gT_i)
    np.add.at(G[:, 3], bt.ev_i, cz)
    np.add.at(G[:, 0:3], bt.ev_j, -cz[:, None] * bt.gT_j)
    np.add.at(G[:, 3], bt.ev_j, -cz)
    return G, -0.5 * scale * float(np.dot(bt.r, bt.z))


def event_prior_gradient(prob: Problem, theta):
    return -(theta - prob.hypo0) / prob.prior_sigma ** 2


def centroid(theta):
    return theta.mean(0)


def centroid_gradient(prob: Problem, theta):
    """d/dtheta_m of -1/2 (thetabar - mu_c)^T Sigma_c^{-1} (thetabar - mu_c),
    the same 4-vector for every event."""
    g = -(centroid(theta) - prob.mu_c) / prob.centroid_sigma ** 2 / prob.M
    return np.broadcast_to(g, theta.shape)


def log_prior(prob: Problem, theta):
    e = -0.5 * float((((theta - prob.hypo0) / prob.prior_sigma) ** 2).sum())
    c = -0.5 * float((((centroid(theta) - prob.mu_c) / prob.centroid_sigma) ** 2).sum())
    return e + c


def grad_log_post(prob: Problem, net, theta, idx, mode=WHITEN_EXACT,
                  with_prior=True, with_centroid=True):
    """Stochastic gradient of eq:sgd: grad log p(theta) + (N/n) sum grad log p(y|theta)."""
    idx = np.asarray(idx, np.int64)
    scale = prob.N / idx.shape[0]
    bt = batch_terms(prob, net, theta, idx, mode)
    G, ll = likelihood_gradient(prob, bt, scale)
    lp = ll
    if with_prior:
        G = G + event_prior_gradient(prob, theta)
        lp += -0.5 * float((((theta - prob.hypo0) / prob.prior_sigma) ** 2).sum())
    if with_centroid:
        G = G + centroid_gradient(prob, theta)
        lp += -0.5 * float((((centroid(theta) - prob.mu_c) / prob.centroid_sigma) ** 2).sum())
    return G, lp, bt
