"""GPU parity of two-phase (P and S) catalogs against the oracle, through the
C ABI (Sec. 3.1: station-phase groups, one forward model and one sigma,
kappa per phase).  Workload tiny2ph: the tiny catalog plus S observations
for about half of its (pair, station) P observations.

Tolerances as for one phase (FP32 network): travel time and gradient 1e-5
relative, residual 1e-5 of the magnitudes it is the difference of, z
solving Sigma_B z = r with each group's own sigma_phi, kappa_phi to 1e-10,
per-event gradients 1e-5 of S_m; the state after one pSGLD step within
what that gradient tolerance can move it.
"""
import numpy as np
import pytest

from gpu_common import (dev, grad_scale, host, lk, make_ctx, psgld_update_tolerance,
                        scaled_grad_error, spider, synth, torch, whitening_residual)
from oracle import linearity, philox, sampler, stage1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


@pytest.fixture(scope="module")
def two(ctx):
    cat = synth.make_catalog("tiny2ph")
    nets = (synth.net_for(cat), synth.net_for(cat, phase=1))
    nid_p, nid_s = ctx.load_net(nets[0]), ctx.load_net(nets[1])
    return cat, nets, nid_p, nid_s


def _load(ctx, two, whiten=spider.WHITEN_EXACT):
    cat, _, nid_p, nid_s = two
    cid = ctx.load_catalog(cat, whiten=whiten, stream_id=3)
    ctx.set_phase_net(cid, nid_s)
    return cid


@pytest.mark.parametrize("whiten", [spider.WHITEN_NONE, spider.WHITEN_DIAG, spider.WHITEN_EXACT])
def test_batch_terms_two_phase(ctx, two, whiten):
    cat, nets, nid_p, _ = two
    cid = _load(ctx, two, whiten)
    prob = lk.load(cat)
    theta = synth.random_theta(cat, 31)
    idx = synth.random_batch(cat.N, 1024, 32)
    out = ctx.batch_terms(cid, nid_p, dev(theta), dev(idx))
    bt = lk.batch_terms(prob, nets, theta, idx, whiten)
    assert 0 < bt.phase.sum() < len(idx)
    Ti, Tj, r, z = (host(out[k]) for k in ("T_i", "T_j", "r", "z"))
    assert np.max(np.abs(Ti - bt.T_i) / bt.T_i) < 1e-5
    assert np.max(np.abs(Tj - bt.T_j) / bt.T_j) < 1e-5
    gi, gj = host(out["gT_i"]), host(out["gT_j"])
    assert np.max(np.linalg.norm(gi - bt.gT_i, axis=1) / np.linalg.norm(bt.gT_i, axis=1)) < 1e-5
    assert np.max(np.linalg.norm(gj - bt.gT_j, axis=1) / np.linalg.norm(bt.gT_j, axis=1)) < 1e-5
    mag = np.abs(bt.T_i) + np.abs(bt.T_j) + np.abs(bt.tau) + np.abs(theta[bt.ev_i, 3] - theta[bt.ev_j, 3])
    assert np.max(np.abs(r - bt.r) / mag) < 1e-5
    assert whitening_residual(r, z, bt, prob, whiten) < 1e-10


@pytest.mark.parametrize("n", [1024, 4096])
def test_grad_two_phase(ctx, two, n):
    cat, nets, nid_p, _ = two
    cid = _load(ctx, two)
    prob = lk.load(cat)
    theta = synth.random_theta(cat, 33)
    idx = synth.random_batch(cat.N, n, 34)
    G = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    lp = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.grad(cid, nid_p, dev(theta), G, batch_idx=dev(idx), logpost=lp)
    Go, lpo, bt = lk.grad_log_post(prob, nets, theta, idx)
    S = grad_scale(prob, bt, prob.N / n, theta)
    assert scaled_grad_error(host(G), Go, S, floor=1.0) < 1e-5
    assert abs(float(host(lp)[0]) - lpo) < 1e-5 * (abs(lpo) + 1)


def test_travel_times_bf16_by_phase(ctx, two):
    cat, nets, nid_p, _ = two
    cid = _load(ctx, two)
    prob = lk.load(cat)
    theta = synth.random_theta(cat, 35)
    idx = synth.random_batch(cat.N, 4096, 36)
    out = ctx.batch_terms(cid, nid_p, dev(theta), dev(idx), precision=spider.BF16)
    bt = lk.batch_terms(prob, nets, theta, idx)
    for k, ref in (("T_i", bt.T_i), ("T_j", bt.T_j)):
        assert np.max(np.abs(host(out[k]) - ref) / ref) < 1e-2


def test_missing_s_network_is_an_error(ctx, two):
    cat, _, nid_p, _ = two
    cid = ctx.load_catalog(cat, stream_id=3)
    G = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(spider.SpiderError):
        ctx.grad(cid, nid_p, dev(cat.hypo0), G, n=1024)
    with pytest.raises(spider.SpiderError):
        ctx.set_phase_net(cid, 99)
    bad = synth.make_catalog("tiny2ph")
    bad.obs_phase = bad.obs_phase.copy()
    bad.obs_phase[3] = 2
    with pytest.raises(spider.SpiderError):
        ctx.load_catalog(bad)


@pytest.mark.parametrize("t", [0, 40])
def test_sgld_one_step_two_phase(ctx, two, t):
    """Step t -> t + 1 from the oracle's own state at step t: the sampler
    minibatch's gradient and the pSGLD state after the GPU's step."""
    cat, nets, nid_p, _ = two
    prob = lk.load(cat)
    seed = 17
    cfg = sampler.SamplerConfig(step=1e-4, seed=seed)
    ch, _ = sampler.run(prob, nets, cfg, 1024, t, stream=3, chain_id=1)
    th_t, v_t = ch.theta.copy(), ch.v.copy()
    G_o, _, idx = sampler.stochastic_gradient(prob, nets, ch, cfg, 3, 1, 1024)
    cid = _load(ctx, two)
    ctx.reset_chains(cid, 2)
    for c in range(2):
        ctx.set_state(cid, c, dev(th_t), dev(v_t), step=t)
    G = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    ctx.grad(cid, nid_p, dev(th_t), G, n=1024, seed=seed, chain=1, step=t)
    bt = lk.batch_terms(prob, nets, th_t, idx)
    S = grad_scale(prob, bt, prob.N / 1024, th_t)
    assert scaled_grad_error(host(G), G_o, S, floor=1.0) < 1e-5
    ctx.sgld_steps([(cid, nid_p, 2, 1024, spider.FP32)], 1, seed=seed)
    th = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    v = torch.empty_like(th)
    assert ctx.get_state(cid, 1, th, v) == t + 1
    eta = philox.noise(seed, 3, 1, t, np.arange(cat.M))
    th_o, v_o = sampler.update(th_t, v_t, G_o, cfg, eta)
    dG = 1e-5 * np.maximum(S, 1.0)[:, None] * np.ones((1, 4))
    tol_th, tol_v = psgld_update_tolerance(th_t, v_t, G_o, dG, cfg, eta)
    assert np.all(np.abs(host(v) - v_o) <= tol_v)
    assert np.all(np.abs(host(th) - th_o) <= tol_th)


def test_two_phase_sets_step_as_alone(ctx, two):
    """Chain sets that include a two-phase catalog are never fused: stepping
    two of them together equals stepping each alone, bit for bit."""
    cat, _, nid_p, _ = two
    a, b = _load(ctx, two), _load(ctx, two)
    sets = [(a, nid_p, 2, 1024, spider.BF16), (b, nid_p, 1, 2048, spider.BF16)]

    def states():
        out = []
        for cid, C in ((a, 2), (b, 1)):
            for c in range(C):
                th = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
                ctx.get_state(cid, c, th)
                out.append(host(th))
        return out

    ctx.reset_chains(a, 2)
    ctx.reset_chains(b, 1)
    ctx.sgld_steps(sets, 3, seed=5)
    together = states()
    ctx.reset_chains(a, 2)
    ctx.reset_chains(b, 1)
    for s in sets:
        ctx.sgld_steps([s], 3, seed=5)
    alone = states()
    assert all(np.all(np.isfinite(x)) for x in together)
    assert all(np.array_equal(x, y) for x, y in zip(together, alone))


def test_screens_two_phase(ctx, two):
    """Outlier and linear-regime screens of a two-phase catalog: each
    observation's residual and travel times come from its own phase's
    network, so the masks match the oracle's away from the thresholds."""
    cat, nets, nid_p, _ = two
    cid = _load(ctx, two)
    ctx.reset_chains(cid, 1)
    prob = lk.load(cat)
    keep, n_keep, med, mad = ctx.outliers(cid, nid_p)
    keep_o, med_o, mad_o, r_o = stage1.outlier_mask(prob, nets, cat.hypo0)
    bt = lk.batch_terms(prob, nets, cat.hypo0, np.arange(cat.N), lk.L1)
    mag = np.abs(bt.T_i) + np.abs(bt.T_j) + np.abs(bt.tau)
    delta = 1e-5 * mag.max()
    assert abs(med - med_o) <= delta and abs(mad - mad_o) <= 2 * delta
    clear = np.abs(np.abs(r_o - med_o) - 4 * mad_o) > 10 * delta
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(host(keep).astype(bool)[clear], keep_o[clear])
    lk_keep, _ = ctx.linearity(cid, nid_p)
    lin_o, _ = linearity.linearity_mask(prob, nets, cat.hypo0)
    dT, lin = linearity.linearisation_terms(prob, nets, cat.hypo0)
    err = 1.05e-5 * (bt.T_i + bt.T_j) + 1e-5 * np.linalg.norm(bt.gT_i, axis=1) * \
        np.linalg.norm(cat.hypo0[prob.pair_j[prob.obs_pair], 0:3]
                       - cat.hypo0[prob.pair_i[prob.obs_pair], 0:3], axis=1)
    clear = np.abs(np.abs(dT - lin) - 0.05 * np.abs(dT)) > 2 * err
    assert clear.mean() > 0.95
    np.testing.assert_array_equal(host(lk_keep).astype(bool)[clear], lin_o[clear])
