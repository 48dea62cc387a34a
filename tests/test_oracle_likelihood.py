"""Pins for the oracle's likelihood: residual assembly, edge weights, the
marginal covariance Sigma_g and its whitening, the gradient and the priors."""
import math

import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import travel_time as tt
from paper_2508_12117_amd import synth


@pytest.fixture(scope="module")
def prob_tiny(tiny):
    return lk.load(tiny)


def test_residuals_brute_force_homogeneous(tiny, prob_tiny):
    """r_n by explicit loops over (pair, station) with T = |x - s|/v0 (Eq. 1)."""
    net = synth.net_for(tiny, zero_output=True)
    theta = synth.random_theta(tiny, 1)
    idx = synth.random_batch(tiny.N, 300, 2)
    bt = lk.batch_terms(prob_tiny, net, theta, idx, lk.WHITEN_NONE)
    for k, n in enumerate(idx):
        p = tiny.obs_pair[n]
        i, j, s = tiny.pair_i[p], tiny.pair_j[p], tiny.obs_sta[n]
        Ti = math.dist(theta[i, 0:3], tiny.stations[s]) / 6.0
        Tj = math.dist(theta[j, 0:3], tiny.stations[s]) / 6.0
        r = float(tiny.obs_dt[n]) - (Ti - Tj + theta[i, 3] - theta[j, 3])
        assert abs(bt.r[k] - r) < 1e-13
        assert bt.group[k] == s


def test_batch_travel_times_use_the_right_points(tiny, prob_tiny):
    net = synth.net_for(tiny)
    theta = synth.random_theta(tiny, 3)
    idx = synth.random_batch(tiny.N, 50, 4)
    bt = lk.batch_terms(prob_tiny, net, theta, idx, lk.WHITEN_DIAG)
    for k, n in enumerate(idx):
        p = tiny.obs_pair[n]
        i, j, s = tiny.pair_i[p], tiny.pair_j[p], tiny.obs_sta[n]
        Ti, gi = tt.travel_time(net, theta[i:i + 1, 0:3], tiny.stations[s:s + 1])
        Tj, gj = tt.travel_time(net, theta[j:j + 1, 0:3], tiny.stations[s:s + 1])
        # BLAS blocking may differ with the row count: equal to a few ulps
        np.testing.assert_allclose([bt.T_i[k], bt.T_j[k]], [Ti[0], Tj[0]], rtol=1e-14)
        np.testing.assert_allclose(np.r_[bt.gT_i[k], bt.gT_j[k]], np.r_[gi[0], gj[0]],
                                   rtol=1e-12, atol=1e-15)


def test_edge_weights_mean_one_per_group(tiny, prob_tiny):
    w = prob_tiny.w_pair[prob_tiny.obs_pair] * prob_tiny.inv_mean[prob_tiny.obs_sta]
    for g in range(tiny.L):
        np.testing.assert_allclose(w[prob_tiny.obs_sta == g].mean(), 1.0, rtol=1e-14)


def test_edge_weights_length_scale_cancels_and_monotone(tiny):
    a = lk.load(tiny, ell=5.0)
    b = lk.load(tiny, ell=40.0)
    wa = a.w_pair * a.inv_mean[0]
    wb = b.w_pair * b.inv_mean[0]
    # after normalisation ell only enters through eps (eq:correlation_decay)
    np.testing.assert_allclose(wa, wb, rtol=1e-4)
    d = np.linalg.norm(tiny.hypo0[tiny.pair_i, 0:3] - tiny.hypo0[tiny.pair_j, 0:3], axis=1)
    o = np.argsort(d)
    assert np.all(np.diff(a.w_pair[o]) >= 0)
    np.testing.assert_allclose(a.w_pair, (d / 5.0) ** 0.25 + 1e-5, rtol=1e-15)


def _whiten(r, w, g, ei, ej, M, s, k, mode=lk.WHITEN_EXACT):
    return lk.whiten(np.asarray(r, float), np.asarray(w, float), np.asarray(g), np.asarray(ei),
                     np.asarray(ej), M, s, k, mode)


def test_whitening_isolated_edges():
    """No shared events: Sigma is diagonal with sigma^2 + 2 kappa^2 w."""
    rng = np.random.default_rng(0)
    n = 40
    ei = np.arange(0, 2 * n, 2)
    ej = ei + 1
    g = rng.integers(0, 3, n)
    w = rng.uniform(0.2, 3.0, n)
    r = rng.normal(0, 0.05, n)
    z = _whiten(r, w, g, ei, ej, 2 * n, 0.01, 0.03)
    np.testing.assert_allclose(z, r / (1e-4 + 2 * 9e-4 * w), rtol=1e-12)
    np.testing.assert_allclose(_whiten(r, w, g, ei, ej, 2 * n, 0.01, 0.03, lk.WHITEN_DIAG), z,
                               rtol=1e-12)
    np.testing.assert_allclose(_whiten(r, w, g, ei, ej, 2 * n, 0.01, 0.03, lk.WHITEN_NONE),
                               r / 1e-4, rtol=1e-15)


@pytest.mark.parametrize("second,sign", [((0, 2), +1.0), ((2, 0), -1.0), ((1, 2), -1.0),
                                         ((2, 1), +1.0)])
def test_whitening_two_edges_sharing_an_event(second, sign):
    """2x2 Sigma in closed form; the sign follows the +1 (event i) / -1 (event j)
    convention of A_g, and the correlation tends to 1/2 for long legs."""
    s, k = 0.01, 0.03
    w1, w2 = 0.7, 1.9
    ei = np.array([0, second[0]])
    ej = np.array([1, second[1]])
    r = np.array([0.013, -0.021])
    c12 = sign * k * k * math.sqrt(w1 * w2)
    S = np.array([[s * s + 2 * k * k * w1, c12], [c12, s * s + 2 * k * k * w2]])
    det = S[0, 0] * S[1, 1] - c12 * c12
    zc = np.array([S[1, 1] * r[0] - c12 * r[1], -c12 * r[0] + S[0, 0] * r[1]]) / det
    z = _whiten(r, [w1, w2], [0, 0], ei, ej, 3, s, k)
    np.testing.assert_allclose(z, zc, rtol=1e-12)
    # different groups do not couple
    z2 = _whiten(r, [w1, w2], [0, 1], ei, ej, 3, s, k)
    np.testing.assert_allclose(z2, r / np.diag(S), rtol=1e-12)
    # correlation -> 1/2 as the legs grow (Sec. 4.5 reports a maximum of about 0.5)
    for w in [1e2, 1e4, 1e6]:
        rho = k * k * w / (s * s + 2 * k * k * w)
        assert 0.5 - rho < 0.5 * s * s / (k * k * w)


def _dense_sigma(w, g, ei, ej, M, s, k):
    """Sigma_B from eq:marginal_sigma with explicit incidence matrices per group."""
    n = len(w)
    S = np.zeros((n, n))
    for grp in np.unique(g):
        rows = np.flatnonzero(g == grp)
        A = np.zeros((rows.size, M))
        A[np.arange(rows.size), ei[rows]] += 1.0
        A[np.arange(rows.size), ej[rows]] -= 1.0
        Wh = np.diag(np.sqrt(w[rows]))
        S[np.ix_(rows, rows)] = s * s * np.eye(rows.size) + k * k * Wh @ A @ A.T @ Wh
    return S


def test_whitening_general_matches_dense_solve():
    rng = np.random.default_rng(1)
    M, n = 12, 60
    ei = rng.integers(0, M, n)
    ej = (ei + rng.integers(1, M, n)) % M
    g = rng.integers(0, 3, n)
    w = rng.uniform(0.1, 2.0, n)
    r = rng.normal(0, 0.05, n)
    S = _dense_sigma(w, g, ei, ej, M, 0.01, 0.03)
    z = _whiten(r, w, g, ei, ej, M, 0.01, 0.03)
    np.testing.assert_allclose(z, np.linalg.solve(S, r), rtol=1e-10, atol=1e-10)
    # duplicated rows are allowed (sigma^2 I keeps Sigma positive definite)
    ei2, ej2, g2 = np.r_[ei, ei[:5]], np.r_[ej, ej[:5]], np.r_[g, g[:5]]
    w2, r2 = np.r_[w, w[:5]], np.r_[r, r[:5]]
    S2 = _dense_sigma(w2, g2, ei2, ej2, M, 0.01, 0.03)
    np.testing.assert_allclose(_whiten(r2, w2, g2, ei2, ej2, M, 0.01, 0.03),
                               np.linalg.solve(S2, r2), rtol=1e-9, atol=1e-9)


def test_sigma_is_the_covariance_of_the_latent_model():
    """Monte Carlo of r_g = W^{1/2} A b + eps with b ~ N(0, kappa^2), eps ~ N(0, sigma^2):
    the covariance the whitening inverts is the sample covariance (eq:marginal_sigma)."""
    rng = np.random.default_rng(2)
    M = 5
    ei = np.array([0, 0, 1, 3, 2])
    ej = np.array([1, 2, 2, 4, 4])
    w = np.array([0.5, 1.5, 1.0, 0.8, 1.2])
    s, k = 0.01, 0.03
    n = len(w)
    g = np.zeros(n, int)
    Sinv = np.column_stack([_whiten(np.eye(n)[c], w, g, ei, ej, M, s, k) for c in range(n)])
    S = np.linalg.inv(Sinv)
    S_draws = 400_000
    b = rng.normal(0, k, (S_draws, M))
    eps = rng.normal(0, s, (S_draws, n))
    r = np.sqrt(w) * (b[:, ei] - b[:, ej]) + eps
    C = np.cov(r.T)
    se = np.sqrt((C ** 2 + np.outer(np.diag(C), np.diag(C))) / S_draws)
    assert np.all(np.abs(C - S) < 5 * se)
    # sign structure of the differencing (Sec. 3.3: cov(V t) = sigma^2 V V^T)
    # (0,1)&(0,2) share i: +; (0,1)&(1,2): event 1 is j then i: -; (1,2)&(2,4): -
    assert S[0, 1] > 0 and S[0, 2] < 0 and S[3, 4] > 0 and S[2, 4] < 0
    assert abs(S[0, 3]) < 1e-12 * S[0, 0]


def _jacobian_dense(prob, bt, M):
    n = bt.r.shape[0]
    J = np.zeros((n, 4 * M))
    for k in range(n):
        J[k, 4 * bt.ev_i[k]:4 * bt.ev_i[k] + 3] += bt.gT_i[k]
        J[k, 4 * bt.ev_i[k] + 3] += 1.0
        J[k, 4 * bt.ev_j[k]:4 * bt.ev_j[k] + 3] -= bt.gT_j[k]
        J[k, 4 * bt.ev_j[k] + 3] -= 1.0
    return J


def test_kappa_zero_is_weighted_least_squares(tiny):
    """kappa = 0: G = (N/n) J^T r / sigma^2, J the dense Jacobian of tau^."""
    prob = lk.load(tiny, kappa=0.0)
    net = synth.net_for(tiny)
    theta = synth.random_theta(tiny, 5)
    idx = synth.random_batch(tiny.N, 256, 6)
    G, lp, bt = lk.grad_log_post(prob, net, theta, idx, with_prior=False, with_centroid=False)
    J = _jacobian_dense(prob, bt, prob.M)
    c = prob.N / 256
    np.testing.assert_allclose(G.reshape(-1), c * J.T @ bt.r / 1e-4, rtol=1e-10, atol=1e-6)
    assert abs(lp + 0.5 * c * (bt.r ** 2).sum() / 1e-4) < 1e-9 * abs(lp)


def test_gradient_invariants(tiny, prob_tiny):
    net = synth.net_for(tiny)
    theta = synth.random_theta(tiny, 7)
    idx = synth.random_batch(tiny.N, 512, 8)
    G, lp, bt = lk.grad_log_post(prob_tiny, net, theta, idx, with_prior=False,
                                 with_centroid=False)
    # every observation adds +c z to t_i and -c z to t_j
    assert abs(G[:, 3].sum()) < 1e-9 * np.abs(G[:, 3]).sum()
    # events outside the batch get nothing
    touched = np.zeros(prob_tiny.M, bool)
    touched[bt.ev_i] = True
    touched[bt.ev_j] = True
    assert np.all(G[~touched] == 0)
    # (i, j, tau) -> (j, i, -tau) leaves the problem unchanged
    sw = synth.Catalog(tiny.wl, tiny.hypo_true, tiny.hypo0, tiny.stations, tiny.pair_j,
                       tiny.pair_i, tiny.obs_pair, tiny.obs_sta, -tiny.obs_dt)
    G2, lp2, _ = lk.grad_log_post(lk.load(sw), net, theta, idx, with_prior=False,
                                  with_centroid=False)
    np.testing.assert_allclose(G2, G, rtol=1e-9, atol=1e-9 * np.abs(G).max())
    assert abs(lp2 - lp) < 1e-10 * abs(lp)


def test_centroid_gradient(tiny, prob_tiny):
    theta = synth.random_theta(tiny, 9)
    g = lk.centroid_gradient(prob_tiny, theta)
    total = -(theta.mean(0) - tiny.hypo0.mean(0)) / np.array(tiny.wl.centroid_sigma) ** 2
    np.testing.assert_allclose(g.sum(0), total, rtol=1e-12)
    assert np.all(g == g[0])


@pytest.mark.parametrize("mode", [lk.WHITEN_EXACT, lk.WHITEN_DIAG])
def test_whole_gradient_central_differences(tiny, prob_tiny, mode):
    """grad log p^ (fixed batch, priors and centroid on) vs central differences."""
    net = synth.net_for(tiny)
    theta = synth.random_theta(tiny, 11)
    idx = synth.random_batch(tiny.N, 512, 12)
    G, lp, bt = lk.grad_log_post(prob_tiny, net, theta, idx, mode)
    rng = np.random.default_rng(3)
    ev = np.concatenate([bt.ev_i[:10], rng.integers(0, tiny.M, 4)])
    h = 1e-5
    for m in ev:
        for a in range(4):
            tp = theta.copy()
            tm = theta.copy()
            tp[m, a] += h
            tm[m, a] -= h
            fd = (lk.grad_log_post(prob_tiny, net, tp, idx, mode)[1]
                  - lk.grad_log_post(prob_tiny, net, tm, idx, mode)[1]) / (2 * h)
            assert abs(fd - G[m, a]) < 1e-5 * abs(G[m, a]) + 1e-4 * (1 + abs(lp) * 1e-10 / h)


@pytest.mark.parametrize("mode", [lk.WHITEN_NONE, lk.WHITEN_DIAG, lk.WHITEN_EXACT])
def test_whitening_solves_the_batch_system(mode):
    """The oracle's z (sparse direct solve) satisfies Sigma_B z = r under the
    matrix-free application of Sigma_B the GPU tests use, on random batches
    whose event graphs have shared events and cycles."""
    from gpu_common import sigma_apply
    rng = np.random.default_rng(5)
    M, n = 30, 400
    ei = rng.integers(0, M, n)
    ej = (ei + rng.integers(1, M, n)) % M
    g = rng.integers(0, 4, n)
    w = rng.uniform(0.2, 3.0, n)
    r = rng.normal(0, 0.05, n)
    z = _whiten(r, w, g, ei, ej, M, 0.01, 0.03, mode)
    Sz = sigma_apply(z, w, g, ei, ej, M, 0.01, 0.03, mode)
    np.testing.assert_allclose(Sz, r, rtol=0, atol=1e-13)
    # a wrong sign convention or a dropped coupling would not solve it
    if mode == lk.WHITEN_EXACT:
        assert np.max(np.abs(sigma_apply(z, w, g, ej, ej, M, 0.01, 0.03, mode) - r)) > 1e-3


# ------------------------------------------------------------------ two phases

@pytest.fixture(scope="module")
def two_phase():
    cat = synth.make_catalog("tiny2ph")
    return cat, (synth.net_for(cat), synth.net_for(cat, phase=1)), lk.load(cat)


def _subset(cat, keep):
    import dataclasses
    return dataclasses.replace(cat, obs_pair=cat.obs_pair[keep], obs_sta=cat.obs_sta[keep],
                               obs_dt=cat.obs_dt[keep], obs_phase=None)


def test_two_phase_groups_and_weights(two_phase):
    """Groups are (station, phase) pairs; the edge weights are normalised to
    mean 1 over each of them (Sec. 3.1)."""
    cat, _, prob = two_phase
    assert prob.two_phase and prob.G == 2 * cat.L
    np.testing.assert_array_equal(prob.obs_group, cat.obs_sta + cat.L * cat.obs_phase)
    w = prob.w_pair[prob.obs_pair] * prob.inv_mean[prob.obs_group]
    for g in range(prob.G):
        np.testing.assert_allclose(w[prob.obs_group == g].mean(), 1.0, rtol=1e-13)


def test_two_phase_batch_splits_by_phase(two_phase):
    """Groups of different phases share no covariance, so a mixed minibatch's
    z and gradient are those of its P rows in the P-only catalog (P network,
    sigma_P, kappa_P) plus those of its S rows in the S-only catalog (S
    network, sigma_S, kappa_S) with the same weight normalisation."""
    cat, nets, prob = two_phase
    ph = cat.obs_phase.astype(bool)
    pos_p, pos_s = np.flatnonzero(~ph), np.flatnonzero(ph)
    prob_p = lk.load(_subset(cat, ~ph))
    prob_s = lk.load(_subset(cat, ph), sigma=cat.wl.sigma_s, kappa=cat.wl.kappa_s)
    theta = synth.random_theta(cat, 5)
    idx = np.sort(synth.random_batch(cat.N, 2048, 6))
    bt = lk.batch_terms(prob, nets, theta, idx)
    in_s = ph[idx]
    assert 0 < in_s.sum() < len(idx)
    bp = lk.batch_terms(prob_p, nets[0], theta, np.searchsorted(pos_p, idx[~in_s]))
    bs = lk.batch_terms(prob_s, nets[1], theta, np.searchsorted(pos_s, idx[in_s]))
    np.testing.assert_allclose(bt.r[~in_s], bp.r, rtol=0, atol=1e-14)
    np.testing.assert_allclose(bt.r[in_s], bs.r, rtol=0, atol=1e-14)
    np.testing.assert_allclose(bt.w[~in_s], bp.w, rtol=1e-14)
    np.testing.assert_allclose(bt.w[in_s], bs.w, rtol=1e-14)
    np.testing.assert_allclose(bt.z[~in_s], bp.z, rtol=1e-9, atol=1e-9 * np.abs(bp.z).max())
    np.testing.assert_allclose(bt.z[in_s], bs.z, rtol=1e-9, atol=1e-9 * np.abs(bs.z).max())
    G, _ = lk.likelihood_gradient(prob, bt, 3.0)
    Gp, _ = lk.likelihood_gradient(prob_p, bp, 3.0)
    Gs, _ = lk.likelihood_gradient(prob_s, bs, 3.0)
    np.testing.assert_allclose(G, Gp + Gs, rtol=1e-8, atol=1e-8 * np.abs(G).max())


def test_two_phase_whitening_dense():
    """z against a dense Sigma_B built entry by entry from eq:marginal_sigma
    with each group's own sigma_phi, kappa_phi: Sigma[n, m] = [n = m]
    sigma_n^2 + [g_n = g_m] kappa_n^2 sqrt(w_n w_m) (A_n . A_m)."""
    rng = np.random.default_rng(9)
    M, n = 6, 14
    ei = rng.integers(0, M, n)
    ej = (ei + rng.integers(1, M, n)) % M
    g = rng.integers(0, 4, n)           # groups 0, 1: P; 2, 3: S
    w = rng.uniform(0.3, 2.0, n)
    sig = np.where(g >= 2, 0.02, 0.01)
    kap = np.where(g >= 2, 0.05, 0.03)
    S = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            dot = (int(ei[a] == ei[b]) - int(ei[a] == ej[b]) - int(ej[a] == ei[b])
                   + int(ej[a] == ej[b]))
            S[a, b] = (a == b) * sig[a] ** 2 + (g[a] == g[b]) * kap[a] ** 2 * \
                math.sqrt(w[a] * w[b]) * dot
    r = rng.normal(0.0, 0.05, n)
    z = lk.whiten(r, w, g, ei, ej, M, sig, kap, lk.WHITEN_EXACT)
    np.testing.assert_allclose(z, np.linalg.solve(S, r), rtol=1e-10)
    zd = lk.whiten(r, w, g, ei, ej, M, sig, kap, lk.WHITEN_DIAG)
    np.testing.assert_allclose(zd, r / (sig ** 2 + 2 * kap ** 2 * w), rtol=1e-14)
