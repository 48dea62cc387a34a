"""Pins for the oracle's sampler diagnostics (Sec. 3.4 credibility bounds,
Sec. 4 calibration, Sec. 3.6 and Sec. 5: effective sample size and the
gradient-noise to injected-noise variance ratio)."""
import numpy as np

from oracle import diagnostics as dg
from oracle import likelihood as lk
from paper_2508_12117_amd import synth


def test_quantiles_closed_forms():
    rng = np.random.default_rng(0)
    s = rng.permutation(101).astype(float)[:, None] * np.ones((1, 3))
    q = dg.quantiles(s, [0.0, 0.005, 0.25, 0.5, 0.995, 1.0])
    np.testing.assert_allclose(q[:, 0], [0.0, 0.5, 25.0, 50.0, 99.5, 100.0], atol=1e-12)
    # interpolation between order statistics: h = 3 * 0.9 = 2.7 -> 2 + 0.7 * (4 - 2)
    np.testing.assert_allclose(dg.quantiles(np.array([[4.0], [0.0], [2.0], [1.0]]), [0.9]),
                               [[3.4]], rtol=1e-15)
    assert dg.quantiles(np.array([[7.0, -1.0]]), [0.3])[0].tolist() == [7.0, -1.0]


def test_sample_ranks_closed_forms_and_calibration():
    s = np.arange(1.0, 11.0)[:, None]
    np.testing.assert_allclose(dg.sample_ranks(s, np.array([5.0])), [0.45])
    np.testing.assert_allclose(dg.sample_ranks(s, np.array([0.0])), [0.0])
    np.testing.assert_allclose(dg.sample_ranks(s, np.array([11.0])), [1.0])
    np.testing.assert_allclose(dg.sample_ranks(s, np.array([5.5])), [0.5])
    # a calibrated posterior: truth and samples from the same law -> uniform ranks
    rng = np.random.default_rng(1)
    truth = rng.normal(0.0, 1.0, 4000)
    u = np.sort(dg.sample_ranks(rng.normal(0.0, 1.0, (500, 4000)), truth))
    ks = np.max(np.abs(u - (np.arange(4000) + 0.5) / 4000))
    assert ks < 1.63 / np.sqrt(4000)   # KS at the 1% level


def _ar1(K, C, P, phi, seed, shift=None):
    rng = np.random.default_rng(seed)
    x = np.empty((K, C, P))
    x[0] = rng.normal(0.0, 1.0, (C, P)) / np.sqrt(1 - phi ** 2)
    for i in range(1, K):
        x[i] = phi * x[i - 1] + rng.normal(0.0, 1.0, (C, P))
    if shift is not None:
        x += shift[None, :, None]
    return x


def test_ess_of_iid_and_ar1_draws():
    """iid draws: ESS = C K; AR(1) with coefficient phi: the integrated
    autocorrelation time is (1 + phi)/(1 - phi)."""
    K, C, P = 2000, 4, 60
    e0 = dg.ess(_ar1(K, C, P, 0.0, 2))
    assert abs(np.mean(e0) / (C * K) - 1.0) < 0.05
    for phi in (0.5, 0.9):
        e = dg.ess(_ar1(K, C, P, phi, 3))
        tau = (1 + phi) / (1 - phi)
        assert abs(np.mean(e) * tau / (C * K) - 1.0) < 0.1, phi


def test_ess_sees_chains_that_disagree():
    """Chains stuck 5 s.d. apart: the between-chain variance drives every
    rho_t towards 1 and the ESS far below C K; constant draws give NaN."""
    x = _ar1(1000, 4, 20, 0.0, 4, shift=np.array([0.0, 5.0, -5.0, 10.0]))
    assert np.all(dg.ess(x) < 0.05 * 4000)
    assert np.all(np.isnan(dg.ess(np.ones((50, 2, 3)))))


def test_gradient_variance_of_disjoint_batches():
    """Without whitening the likelihood gradient is (N/n) sum over the batch
    of per-observation contributions c_i; for the disjoint batches of one
    epoch of a random permutation the expected sample variance across batches
    is exactly N^2 S^2 / n, S^2 the variance of c_i over all N (divisor N - 1).
    Summed over coordinates, the oracle's estimate from 31 batches of 1,024
    (one epoch of the tiny catalog) matches within sampling error."""
    cat = synth.make_catalog("tiny")
    net = synth.net_for(cat)
    prob = lk.load(cat)
    theta = synth.random_theta(cat, 7)
    n, K = 1024, 31
    var = dg.gradient_variance(prob, net, theta, 5, 2, 1, 0, n, K, lk.WHITEN_NONE)
    bt = lk.batch_terms(prob, net, theta, np.arange(cat.N), lk.WHITEN_NONE)
    N = cat.N
    c = np.zeros((N, prob.M, 4))    # per-observation contribution to each coordinate
    rows = np.arange(N)
    c[rows, bt.ev_i, 0:3] += bt.z[:, None] * bt.gT_i
    c[rows, bt.ev_i, 3] += bt.z
    c[rows, bt.ev_j, 0:3] -= bt.z[:, None] * bt.gT_j
    c[rows, bt.ev_j, 3] -= bt.z
    want = N ** 2 * c.var(0, ddof=1) / n
    assert abs(var.sum() / want.sum() - 1.0) < 0.05
    # and per coordinate the estimate scatters around it (chi^2 with 30 d.o.f.)
    ratio = var / want
    assert 0.9 < np.median(ratio) < 1.1


def test_noise_ratio_scales():
    """Linear in the step (Sec. 3.6), inverse in the squared noise amplitude,
    and the pSGLD preconditioner enters as V = 1/(sqrt(v) + eps_p)."""
    rng = np.random.default_rng(6)
    var = rng.uniform(1e2, 1e4, (50, 4))
    v = rng.uniform(1e6, 1e8, (50, 4))
    r = dg.noise_ratio(var, v, 1e-4)
    np.testing.assert_allclose(dg.noise_ratio(var, v, 2e-4), 2 * r, rtol=1e-15)
    np.testing.assert_allclose(dg.noise_ratio(var, v, 1e-4, noise_scale=2.0), r / 4, rtol=1e-15)
    np.testing.assert_allclose(dg.noise_ratio(var, v, 1e-4, precond=False) / r,
                               np.sqrt(v) + 1e-5, rtol=1e-12)
    # a full batch (n = N) has no gradient noise: every batch is the catalog
    cat = synth.make_catalog("tiny")
    prob = lk.load(cat)
    g = dg.gradient_variance(prob, synth.net_for(cat), cat.hypo0, 1, 0, 0, 0, cat.N, 3,
                             lk.WHITEN_DIAG)
    G = lk.likelihood_gradient(prob, lk.batch_terms(prob, synth.net_for(cat), cat.hypo0,
                                                    np.arange(cat.N), lk.WHITEN_DIAG), 1.0)[0]
    assert np.all(np.sqrt(g) <= 1e-10 * np.abs(G).max())
