"""Pins for the oracle's Stage 1 (L1 loss, Adam; Sec. 3.2, eq:stage1loss)."""
import dataclasses

import numpy as np

from oracle import batch as obatch
from oracle import likelihood as lk
from oracle import stage1
from paper_2508_12117_amd import synth


def test_l1_gradient_matches_central_differences():
    """-G is dL/dtheta of L = mean |r| wherever no residual of the event
    crosses zero within the step."""
    cat = synth.make_catalog("tiny")
    net = synth.net_for(cat)
    prob = lk.load(cat)
    theta = synth.random_theta(cat, 3)
    idx = synth.random_batch(cat.N, 1024, 4)
    loss, G, bt = stage1.l1_loss_gradient(prob, net, theta, idx)
    assert abs(loss - np.abs(bt.r).mean()) < 1e-15
    rng = np.random.default_rng(5)
    h = 1e-7
    checked = 0
    for m in rng.permutation(np.unique(np.concatenate([bt.ev_i, bt.ev_j])))[:40]:
        touch = (bt.ev_i == m) | (bt.ev_j == m)
        if np.abs(bt.r[touch]).min() < 1e-5:
            continue
        for a in range(4):
            tp, tm = theta.copy(), theta.copy()
            tp[m, a] += h
            tm[m, a] -= h
            fd = (stage1.l1_loss_gradient(prob, net, tp, idx)[0]
                  - stage1.l1_loss_gradient(prob, net, tm, idx)[0]) / (2 * h)
            assert abs(fd - (-G[m, a])) < 1e-6 * abs(G[m, a]) + 1e-9
            checked += 1
    assert checked >= 40
    # a sign error in z would reverse it: the derivative of the loss is not +G
    assert np.abs(G).max() > 1e-5


def test_adam_first_step_has_length_lr():
    """After one step the bias-corrected moments are g and g^2, so every
    coordinate moves by lr |g| / (|g| + eps) against the gradient."""
    rng = np.random.default_rng(1)
    g = rng.normal(size=(9, 4)) * 10.0 ** rng.uniform(-6, 3, (9, 4))
    th0 = rng.normal(size=(9, 4))
    cfg = stage1.AdamConfig(lr=3e-3, eps=1e-8)
    th1, m, v = stage1.adam_update(th0, np.zeros_like(g), np.zeros_like(g), g, 1, cfg)
    np.testing.assert_allclose(th1 - th0, -3e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_minimises_a_quadratic():
    lam = np.array([0.5, 3.0, 40.0])
    mu = np.array([1.0, -2.0, 0.25])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    cfg = stage1.AdamConfig(lr=1e-3)
    for k in range(1, 20001):
        th, m, v = stage1.adam_update(th, m, v, lam * (th - mu), k, cfg)
    np.testing.assert_allclose(th, mu, atol=2e-3)


def test_stage1_reduces_the_l1_loss():
    """Adam on the minibatch L1 loss moves the tiny catalog to a lower loss on
    a fixed evaluation batch, following the sampler's minibatch stream."""
    cat = synth.make_catalog("tiny")
    net = synth.net_for(cat)
    prob = lk.load(cat)
    cfg = stage1.AdamConfig(lr=1e-3, seed=9)
    st, losses = stage1.run(prob, net, cfg, 1024, 60, stream=3)
    assert st.step == 60
    ev = np.arange(cat.N)
    before = stage1.l1_loss_gradient(prob, net, prob.hypo0, ev)[0]
    after = stage1.l1_loss_gradient(prob, net, st.theta, ev)[0]
    assert after < 0.9 * before
    # the first minibatch is the sampler's
    idx0 = obatch.batch_indices(9, 3, 0, 0, cat.N, 1024)
    assert abs(losses[0] - stage1.l1_loss_gradient(prob, net, prob.hypo0, idx0)[0]) < 1e-15


def _screen(cat, shift=None):
    cat = dataclasses.replace(cat, obs_dt=cat.obs_dt.copy())
    if shift is not None:
        cat.obs_dt += shift.astype(cat.obs_dt.dtype)
    prob = lk.load(cat)
    return stage1.outlier_mask(prob, synth.net_for(cat), prob.hypo0)


def test_outlier_mask_removes_planted_outliers():
    """Observed times shifted by 5 s (beyond every genuine residual, which
    stay within 0.9 s at the start) are all screened out; the median and MAD
    hardly move with 0.6% of the data corrupted."""
    cat = synth.make_catalog("tiny")
    keep0, med0, mad0, r0 = _screen(cat)
    rng = np.random.default_rng(8)
    bad = rng.choice(cat.N, 200, replace=False)
    shift = np.zeros(cat.N)
    shift[bad] = np.where(rng.random(200) < 0.5, 5.0, -5.0)
    keep, med, mad, r = _screen(cat, shift)
    assert not keep[bad].any()
    np.testing.assert_allclose(r[bad], r0[bad] + shift[bad], atol=1e-5)  # r = observed - predicted
    assert abs(med - med0) < 0.02 * mad0 and abs(mad - mad0) < 0.02 * mad0
    good = np.setdiff1d(np.arange(cat.N), bad)
    # genuine observations well inside (or outside) the threshold keep their fate
    clear = np.abs(np.abs(r0[good] - med0) - 4 * mad0) > 0.05 * mad0
    np.testing.assert_array_equal(keep[good][clear], keep0[good][clear])


def test_median_and_mad_by_counting():
    """The median splits the residuals in halves and the MAD is the median
    distance from it (counted, for the even N of this catalog)."""
    cat = synth.make_catalog("tiny")
    assert cat.N % 2 == 0
    keep, med, mad, r = _screen(cat)
    n = cat.N
    assert np.sum(r < med) == n // 2 and np.sum(r > med) == n // 2
    d = np.abs(r - med)
    assert np.sum(d < mad) <= n // 2 <= np.sum(d <= mad)
    assert 0 < keep.sum() < n


def test_outlier_mask_is_shift_invariant():
    """A constant added to every observed time moves the median by it and
    leaves the MAD and the mask unchanged (centering at the median)."""
    cat = synth.make_catalog("tiny")
    keep0, med0, mad0, _ = _screen(cat)
    keep1, med1, mad1, _ = _screen(cat, np.full(cat.N, 0.25))
    assert abs(med1 - med0 - 0.25) < 1e-5 and abs(mad1 - mad0) < 1e-5
    d = np.abs(_screen(cat)[3] - med0)
    near = np.abs(d - 4 * mad0) < 1e-4
    np.testing.assert_array_equal(keep0[~near], keep1[~near])
