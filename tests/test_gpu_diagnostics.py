"""GPU parity of the sample buffer and the sampler diagnostics, through the
C ABI, against the oracle (oracle/diagnostics.py) on seeded inputs.

Tolerances: stored samples are the chain states bit for bit and their mean
is the moment accumulator's within FP64 rounding; percentiles within 1e-15
of the samples' range (the interpolation's rounding); ranks exact; ESS
within 1e-10 relative (FP64 sums in another order); the variance ratio
within what the FP32 gradient tolerance (1e-5 of S_m per gradient) can move
a sample variance.
"""
import numpy as np
import pytest

from gpu_common import dev, grad_scale, host, lk, make_ctx, spider, synth, torch
from oracle import batch as obatch
from oracle import diagnostics as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny(ctx):
    cat = synth.make_catalog("tiny")
    net = synth.net_for(cat)
    return cat, net, ctx.load_catalog(cat, stream_id=3), ctx.load_net(net)


def test_sample_buffer_holds_the_recorded_states(ctx, tiny):
    cat, _, cid, nid = tiny
    C, K = 3, 6
    buf = torch.full((K, C, cat.M, 4), np.nan, dtype=torch.float64, device="cuda")
    ctx.reset_chains(cid, C)
    ctx.set_sample_buffer(cid, buf)
    th = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    states = []
    for t in range(9):  # burn 2, thin 2: steps 2, 4, 6, 8 are recorded
        ctx.sgld_steps([(cid, nid, C, 1024, spider.FP32)], 1, seed=3, burn_in=2, thin=2)
        if t >= 2 and (t - 2) % 2 == 0:
            row = []
            for c in range(C):
                ctx.get_state(cid, c, th)
                row.append(host(th))
            states.append(row)
    ctx.set_sample_buffer(cid, None)
    b = host(buf)
    for k, st in enumerate(states):
        for c in range(C):
            assert np.array_equal(b[k, c], st[c])
    assert np.all(np.isnan(b[len(states):]))
    mean = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    assert ctx.moments(cid, 1, mean, None) == len(states)
    np.testing.assert_allclose(host(mean), b[:len(states), 1].mean(0), rtol=0, atol=1e-12)


@pytest.mark.parametrize("S,P", [(1, 5), (7, 300), (1000, 257), (8192, 40)])
def test_quantiles_match_oracle(ctx, S, P):
    rng = np.random.default_rng(S + P)
    s = rng.normal(0.0, 1.0, (S, P)) * rng.uniform(0.1, 10.0, P)
    s[:, 0] = 1.0  # a constant parameter
    probs = [0.0, 0.005, 0.025, 0.5, 0.975, 0.995, 1.0]
    got = host(ctx.quantiles(dev(s), probs))
    want = dg.quantiles(s, probs)
    span = s.max(0) - s.min(0) + 1e-300
    assert np.all(np.abs(got - want) <= 1e-15 * span + 1e-300 + 4e-16 * np.abs(want))


def test_quantiles_reject_too_many_samples(ctx):
    s = torch.zeros(8193, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(spider.SpiderError):
        ctx.quantiles(s, [0.5])
    with pytest.raises(spider.SpiderError):
        ctx.quantiles(s[:10], [1.5])


def test_sample_ranks_match_oracle(ctx):
    rng = np.random.default_rng(9)
    s = np.round(rng.normal(0.0, 1.0, (777, 1000)), 2)   # ties
    v = np.round(rng.normal(0.0, 1.0, 1000), 2)
    got = host(ctx.sample_ranks(dev(s), dev(v)))
    assert np.array_equal(got, dg.sample_ranks(s, v))


@pytest.mark.parametrize("K,C,phi", [(400, 1, 0.0), (500, 4, 0.7), (64, 8, 0.95)])
def test_ess_matches_oracle(ctx, K, C, phi):
    rng = np.random.default_rng(K + C)
    P = 300
    x = np.empty((K, C, P))
    x[0] = rng.normal(0.0, 1.0, (C, P))
    for i in range(1, K):
        x[i] = phi * x[i - 1] + rng.normal(0.0, 1.0, (C, P))
    x[:, :, 0] = 2.5   # constant: NaN on both sides
    got = host(ctx.ess(dev(x)))
    want = dg.ess(x)
    assert np.isnan(got[0]) and np.isnan(want[0])
    np.testing.assert_allclose(got[1:], want[1:], rtol=1e-10)


def test_noise_ratio_matches_oracle(ctx, tiny):
    cat, net, cid, nid = tiny
    prob = lk.load(cat)
    rng = np.random.default_rng(12)
    theta = synth.random_theta(cat, 41)
    v = rng.uniform(1e6, 1e8, (cat.M, 4))
    ctx.reset_chains(cid, 2)
    ctx.set_state(cid, 1, dev(theta), dev(v), step=5)
    K, n, seed, step = 8, 1024, 21, 3e-4
    ratio, mean = ctx.noise_ratio(cid, nid, 1, n, K, step=step, seed=seed)
    var_o = dg.gradient_variance(prob, net, theta, seed, 3, 1, 5, n, K)
    want = dg.noise_ratio(var_o, v, step)
    # each GPU gradient is within d = 1e-5 max(S_m, 1) of the oracle's; a
    # sample variance then moves by at most (4 d sum_k |g_k - mean|)/(K-1) + 4 d^2 K/(K-1)
    Gs, d = [], np.zeros((cat.M, 4))
    for k in range(K):
        idx = obatch.batch_indices(seed, 3, 1, 5 + k, cat.N, n)
        bt = lk.batch_terms(prob, net, theta, idx)
        Gs.append(lk.likelihood_gradient(prob, bt, cat.N / n)[0])
        S = grad_scale(prob, bt, cat.N / n, theta)
        d = np.maximum(d, 1e-5 * np.maximum(S, 1.0)[:, None])
    Gs = np.stack(Gs)
    dev_sum = np.abs(Gs - Gs.mean(0)).sum(0)
    dvar = (4 * d * dev_sum + 4 * d * d * K) / (K - 1)
    tol = step * (1.0 / (np.sqrt(v) + 1e-5)) * dvar / 2.0 + 1e-15 * np.abs(want)
    got = host(ratio)
    assert np.all(np.abs(got - want) <= tol)
    assert abs(mean - got.mean()) <= 1e-12 * abs(got.mean())
    th = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    assert ctx.get_state(cid, 1, th) == 5 and np.array_equal(host(th), theta)


def test_calibration_on_synthetic_truth(ctx):
    """Sec. 4's calibration check, end to end: with the true forward model
    (zero-output network, T = |x - s| / 6) and the true noise model (sigma =
    0.01 s, kappa = 0) the sampler's posterior over the event locations
    relative to their centroid (what double differences constrain; the
    centroid itself is held by the prior centred on the initial locations) is
    calibrated: the rank of the truth among 4,000 samples is uniform over the
    200 events (KS below the 1% critical value) and the standardised errors
    have mean ~0 and s.d. ~1.  The step size 1e-3 puts the gradient-noise to
    injected-noise ratio at 1, the top of the paper's range."""
    cat = synth.make_catalog("tiny")
    net = synth.make_net(32, 3, *synth.net_box(cat), zero_output=True)
    cid = ctx.load_catalog(cat, whiten=spider.WHITEN_EXACT, stream_id=1, kappa=0.0)
    nid = ctx.load_net(net)
    C, n, steps, thin = 4, 4096, 400_000, 200
    K = steps // 2 // thin
    ctx.reset_chains(cid, C)
    ctx.sgld_steps([(cid, nid, C, n, spider.FP32)], 2000, step=1e-3, seed=11)
    _, ratio = ctx.noise_ratio(cid, nid, 0, n, 16, step=1e-3, seed=99)
    assert 0.5 < ratio < 2.0
    ctx.reset_chains(cid, C)
    buf = torch.empty(K, C, cat.M, 4, dtype=torch.float64, device="cuda")
    ctx.set_sample_buffer(cid, buf)
    ctx.sgld_steps([(cid, nid, C, n, spider.FP32)], steps, step=1e-3, seed=11,
                   burn_in=steps // 2, thin=thin)
    ctx.set_sample_buffer(cid, None)
    ess = host(ctx.ess(buf.reshape(K, C, cat.M * 4))).reshape(cat.M, 4)
    assert np.all(np.median(ess, axis=0) > 10)
    cen = (buf - buf.mean(dim=2, keepdim=True)).reshape(K * C, cat.M * 4).contiguous()
    truth = cat.hypo_true - cat.hypo_true.mean(0)
    u = host(ctx.sample_ranks(cen, dev(truth.reshape(-1)))).reshape(cat.M, 4)
    x = host(cen).reshape(K * C, cat.M, 4)
    z = (truth - x.mean(0)) / x.std(0)
    for k in range(4):
        us = np.sort(u[:, k])
        ks = np.max(np.abs(us - (np.arange(cat.M) + 0.5) / cat.M))
        assert ks < 1.63 / np.sqrt(cat.M), k
        assert abs(z[:, k].mean()) < 0.2 and 0.7 < z[:, k].std() < 1.3, k


def test_four_stage_pipeline(ctx):
    """The paper's workflow through the C ABI (Sec. 3.2): linear-regime
    filter and Stage 1 (L1 + Adam) on the full catalog, the 4-MAD screen, the
    kept observations reloaded as a catalog that starts from the Stage-1
    states, then warm-up, ramp and sampling.  With the true forward model the
    Stage-1 solution and the posterior mean both place the events relative
    to each other far closer to the truth than the initial locations (the
    posterior mean also carries the event prior around the initial
    locations, so it need not beat the prior-free Stage-1 solution)."""
    import dataclasses
    cat = synth.make_catalog("tiny")
    net = synth.make_net(32, 3, *synth.net_box(cat), zero_output=True)
    nid = ctx.load_net(net)
    cid = ctx.load_catalog(cat, stream_id=2, kappa=0.0)
    C, n = 2, 4096
    ctx.reset_chains(cid, C)
    lin, n_lin = ctx.linearity(cid, nid)
    ctx.map_steps([(cid, nid, C, n, spider.FP32)], 3000, lr=1e-3, seed=5)
    keep, n_keep, _, mad = ctx.outliers(cid, nid)
    keep = host(keep).astype(bool) & host(lin).astype(bool)
    assert 0 < keep.sum() < cat.N and mad > 0
    sub = dataclasses.replace(cat, obs_pair=cat.obs_pair[keep], obs_sta=cat.obs_sta[keep],
                              obs_dt=cat.obs_dt[keep])
    fid = ctx.load_catalog(sub, stream_id=2, kappa=0.0)
    ctx.reset_chains(fid, C)
    th = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    s1 = []
    for c in range(C):
        ctx.get_state(cid, c, th)
        s1.append(host(th))
        ctx.set_state(fid, c, th.clone(), step=0)
    ctx.sgld_stages([(fid, nid, C, 2048, spider.FP32)], 2000, 2000, 20000, thin=20, step=3e-4,
                    seed=6)
    mean = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    assert ctx.moments(fid, -1, mean, None) == C * 1000
    truth = cat.hypo_true[:, 0:3] - cat.hypo_true[:, 0:3].mean(0)

    def rel_err(th):
        return np.sqrt(np.mean(((th[:, 0:3] - th[:, 0:3].mean(0)) - truth) ** 2))
    e0, e1, e2 = rel_err(cat.hypo0), np.mean([rel_err(s) for s in s1]), rel_err(host(mean))
    assert e1 < 0.3 * e0 and e2 < 0.3 * e0, (e0, e1, e2)


def test_sample_buffer_detaches_on_reset(ctx):
    """A buffer sized for C chains is detached when the chains are reset (to
    another count), so later steps never write past it; attaching needs
    chains."""
    cat = synth.make_catalog("tiny")
    net = synth.net_for(cat)
    cid, nid = ctx.load_catalog(cat, stream_id=4), ctx.load_net(net)
    buf = torch.full((4, 1, cat.M, 4), np.nan, dtype=torch.float64, device="cuda")
    with pytest.raises(spider.SpiderError):
        ctx.set_sample_buffer(cid, buf)
    ctx.reset_chains(cid, 1)
    ctx.set_sample_buffer(cid, buf)
    ctx.reset_chains(cid, 3)
    ctx.sgld_steps([(cid, nid, 3, 1024, spider.FP32)], 5, seed=1)
    assert np.all(np.isnan(host(buf)))
