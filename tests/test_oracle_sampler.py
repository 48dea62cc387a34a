"""Pins for the oracle's Langevin updates and posterior moments."""
import numpy as np
import pytest

from oracle import likelihood as lk
from oracle import sampler
from paper_2508_12117_amd import synth


def _gaussian_run(P, mu, cfg, steps, v0=None, seed=0):
    d = P.shape[0]
    theta = mu.copy()
    v = np.zeros(d) if v0 is None else v0.copy()
    out = np.empty((steps, d))
    etas = np.random.default_rng(seed).normal(size=(steps, d))
    for t in range(steps):
        g = -P @ (theta - mu)
        theta, v = sampler.update(theta, v, g, cfg, etas[t])
        out[t] = theta
    return out


def _batch_means_se(x, nb=50):
    """Standard error of the mean of x [T, ...] by batch means (autocorrelation-robust)."""
    T = x.shape[0] // nb * nb
    bm = x[:T].reshape(nb, T // nb, *x.shape[1:]).mean(1)
    return bm.std(0, ddof=1) / np.sqrt(nb)


def test_sgld_gaussian_stationary_covariance():
    """Plain SGLD (theta += eps g + sqrt(2 eps) eta) on N(mu, P^-1) with the full gradient:
    the discrete chain's stationary covariance solves S = A S A^T + 2 eps I, A = I - eps P,
    i.e. S = (P (I - eps P / 2))^{-1}."""
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    lam = np.array([1.0, 4.0, 20.0])
    P = Q @ np.diag(lam) @ Q.T
    mu = np.array([1.0, -2.0, 0.5])
    eps = 0.02
    cfg = sampler.SamplerConfig(step=eps, precond=0)
    x = _gaussian_run(P, mu, cfg, 200_000)[1000:]
    S = np.linalg.inv(P @ (np.eye(3) - eps * P / 2))
    # the discrete-chain correction is ~ eps*lam/2 = 20% on the stiff direction: resolved
    assert not np.allclose(S, np.linalg.inv(P), rtol=0.05)
    C = np.cov(x.T)
    se = _batch_means_se(np.einsum("ti,tj->tij", x - mu, x - mu))
    assert np.all(np.abs(C - S) < 5 * se + 1e-4)
    assert np.all(np.abs(x.mean(0) - mu) < 5 * _batch_means_se(x))


def test_psgld_frozen_preconditioner_gaussian():
    """pSGLD with beta2 = 1 keeps v fixed: V = 1/(sqrt(v) + eps_p) is a constant diagonal
    preconditioner and the stationary variance of an axis-aligned Gaussian is
    1/(lambda (1 - eps V lambda / 2)) per coordinate (eq:pSGLD)."""
    lam = np.array([2.0, 10.0, 50.0, 5.0])
    P = np.diag(lam)
    mu = np.zeros(4)
    v0 = np.array([4.0, 1.0, 0.25, 9.0])
    eps = 0.01
    cfg = sampler.SamplerConfig(step=eps, precond=1, beta2=1.0, eps_p=1e-5)
    x = _gaussian_run(P, mu, cfg, 200_000, v0=v0, seed=3)[1000:]
    V = 1.0 / (np.sqrt(v0) + 1e-5)
    want = 1.0 / (lam * (1.0 - eps * V * lam / 2))
    se = _batch_means_se((x - mu) ** 2)
    assert np.all(np.abs(x.var(0) - want) < 5 * se + 1e-5)


def test_psgld_update_formula():
    """One pSGLD step checked component by component against eq:pSGLD."""
    rng = np.random.default_rng(4)
    th, v, g, eta = (rng.normal(size=(7, 4)) for _ in range(4))
    v = np.abs(v)
    cfg = sampler.SamplerConfig(step=3e-3, beta2=0.9, eps_p=1e-3, noise_scale=0.5, precond=1)
    t2, v2 = sampler.update(th, v, g, cfg, eta)
    for a in range(7):
        for b in range(4):
            vv = 0.9 * v[a, b] + 0.1 * g[a, b] ** 2
            VV = 1 / (vv ** 0.5 + 1e-3)
            want = th[a, b] + 3e-3 * VV * g[a, b] + 0.5 * (2 * 3e-3 * VV) ** 0.5 * eta[a, b]
            assert abs(v2[a, b] - vv) < 1e-15 and abs(t2[a, b] - want) < 1e-14


def test_welford_matches_two_pass_and_pooling():
    rng = np.random.default_rng(5)
    xs = rng.normal(size=(3, 57, 6, 4)) * np.array([1.0, 2.0, 0.1, 5.0]) + 100.0
    moms = []
    for c in range(3):
        m = sampler.moments_empty(6)
        for x in xs[c]:
            sampler.welford(m, x)
        moms.append(m)
        np.testing.assert_allclose(m.mean, xs[c].mean(0), rtol=1e-13)
        for k, (a, b) in enumerate(sampler.UPPER):
            two = np.array([np.cov(xs[c][:, e, a], xs[c][:, e, b])[0, 1] for e in range(6)])
            np.testing.assert_allclose(sampler.covariance(m)[:, k], two, rtol=1e-10)
    pool = sampler.pooled(moms)
    allx = xs.reshape(-1, 6, 4)
    assert pool.count == allx.shape[0]
    np.testing.assert_allclose(pool.mean, allx.mean(0), rtol=1e-13)
    for k, (a, b) in enumerate(sampler.UPPER):
        two = np.array([np.cov(allx[:, e, a], allx[:, e, b])[0, 1] for e in range(6)])
        np.testing.assert_allclose(sampler.covariance(pool)[:, k], two, rtol=1e-10)


def test_sampler_is_deterministic_and_thins(tiny):
    prob = lk.load(tiny)
    net = synth.net_for(tiny)
    cfg = sampler.SamplerConfig(step=1e-4, seed=77, burn_in=4, thin=3)
    a, sa = sampler.run(prob, net, cfg, 1024, 12, keep_states=True)
    b, _ = sampler.run(prob, net, cfg, 1024, 12)
    assert np.array_equal(a.theta, b.theta) and np.array_equal(a.v, b.v)
    # samples after steps 4, 7, 10
    assert a.mom.count == 3
    kept = np.stack([sa[4], sa[7], sa[10]])
    np.testing.assert_allclose(a.mom.mean, kept.mean(0), rtol=1e-14)
    # the chain moves, and stays finite
    assert np.all(np.isfinite(a.theta)) and np.abs(a.theta - prob.hypo0).max() > 0


def test_resume_is_exact(tiny):
    """Counter-based streams: stopping after k steps and resuming from the state equals
    an uninterrupted run bit for bit."""
    prob = lk.load(tiny)
    net = synth.net_for(tiny)
    cfg = sampler.SamplerConfig(step=1e-4, seed=5)
    full, _ = sampler.run(prob, net, cfg, 1024, 8)
    half, _ = sampler.run(prob, net, cfg, 1024, 5)
    rest, _ = sampler.run(prob, net, cfg, 1024, 3, chain=half)
    assert np.array_equal(full.theta, rest.theta)


def test_psgld_update_tolerance_bounds_gradient_errors():
    """The GPU tests' bound on how far a gradient error of up to dG moves one
    pSGLD update holds for sampled errors, including gradients near zero."""
    from gpu_common import psgld_update_tolerance
    rng = np.random.default_rng(3)
    n = 2000
    theta = rng.normal(0, 5, (n, 4))
    v = np.where(rng.random((n, 4)) < 0.5, 0.0, rng.uniform(0, 1e4, (n, 4)))
    G = rng.normal(0, 1, (n, 4)) * 10.0 ** rng.uniform(-6, 4, (n, 4))
    dG = np.abs(G) * 10.0 ** rng.uniform(-6, 1, (n, 4))
    eta = rng.normal(0, 1, (n, 4))
    cfg = sampler.SamplerConfig(step=1e-4)
    tol_th, tol_v = psgld_update_tolerance(theta, v, G, dG, cfg, eta)
    th0, v0 = sampler.update(theta, v, G, cfg, eta)
    for _ in range(20):
        th1, v1 = sampler.update(theta, v, G + dG * rng.uniform(-1, 1, G.shape), cfg, eta)
        assert np.all(np.abs(th1 - th0) <= tol_th)
        assert np.all(np.abs(v1 - v0) <= tol_v)


def test_stage_noise_scales():
    """Warm-up with the noise off, a linear ramp from zero, then full amplitude (Sec. 3.2)."""
    a = sampler.stage_noise_scales(3, 4, 2)
    np.testing.assert_array_equal(a, [0, 0, 0, 0, 0.25, 0.5, 0.75, 1, 1])
    assert sampler.stage_noise_scales(0, 0, 5).tolist() == [1.0] * 5


def test_noise_off_finds_the_mode():
    """With the injected noise off (the warm-up stage) pSGLD is preconditioned
    gradient ascent: on a Gaussian target it converges to the mean."""
    lam = np.array([2.0, 10.0, 50.0])
    P = np.diag(lam)
    mu = np.array([1.0, -2.0, 0.5])
    cfg = sampler.SamplerConfig(step=1e-3, precond=1, noise_scale=0.0)
    theta, v = mu + np.array([3.0, -1.0, 2.0]), np.zeros(3)
    for _ in range(20000):
        theta, v = sampler.update(theta, v, -P @ (theta - mu), cfg, np.ones(3))
    np.testing.assert_allclose(theta, mu, atol=1e-8)


def test_noise_scale_scales_the_stationary_covariance():
    """SGLD with noise amplitude a on N(mu, P^-1): the discrete chain's
    stationary covariance is a^2 (P (I - eps P / 2))^{-1}."""
    lam = np.array([1.0, 4.0, 20.0])
    P = np.diag(lam)
    mu = np.zeros(3)
    eps = 0.02
    cfg = sampler.SamplerConfig(step=eps, precond=0, noise_scale=0.5)
    x = _gaussian_run(P, mu, cfg, 200_000, seed=7)[1000:]
    want = 0.25 / (lam * (1 - eps * lam / 2))
    se = _batch_means_se((x - mu) ** 2)
    assert np.all(np.abs(x.var(0) - want) < 5 * se + 1e-5)
    # and not the a = 1 covariance
    assert np.all(np.abs(x.var(0) - 4 * want) > 10 * se)
