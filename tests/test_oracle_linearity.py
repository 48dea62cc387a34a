"""Pins for the oracle's linearisation filter (Sec. 2.1,
eq:dd_linearization and eq:dd_criterion; 5% in Sec. 4)."""
import types

import numpy as np

from oracle import likelihood as lk
from oracle import linearity
from oracle import travel_time as ott
from paper_2508_12117_amd import synth

V = 6.0  # speed of the homogeneous medium a zero-output network gives


def _homogeneous():
    return synth.make_net(64, 3, center=[0.0, 0.0, 5.0], half_extent=[30.0, 30.0, 10.0],
                          zero_output=True)


def _problem(xi, xj, s):
    """One observation per row: pair k = (event 2k, event 2k+1) at station k."""
    R = xi.shape[0]
    theta = np.zeros((2 * R, 4))
    theta[0::2, 0:3], theta[1::2, 0:3] = xi, xj
    prob = types.SimpleNamespace(obs_pair=np.arange(R), pair_i=np.arange(0, 2 * R, 2),
                                 pair_j=np.arange(1, 2 * R, 2), obs_sta=np.arange(R),
                                 stations=s)
    return prob, theta


def _geometry(R, seed, sep=2.0):
    rng = np.random.default_rng(seed)
    xi = np.column_stack([rng.uniform(-10, 10, R), rng.uniform(-10, 10, R), rng.uniform(1, 12, R)])
    xj = xi + rng.normal(0.0, sep, (R, 3))
    s = np.column_stack([rng.uniform(-25, 25, R), rng.uniform(-25, 25, R), np.zeros(R)])
    return xi, xj, s


def test_homogeneous_medium_closed_form():
    """T = |x - s| / c and grad T = (x - s) / (c |x - s|) (Sec. 2.1)."""
    xi, xj, s = _geometry(500, 1)
    prob, theta = _problem(xi, xj, s)
    dT, lin = linearity.linearisation_terms(prob, _homogeneous(), theta)
    ri, rj = np.linalg.norm(xi - s, axis=1), np.linalg.norm(xj - s, axis=1)
    np.testing.assert_allclose(dT, (rj - ri) / V, rtol=0, atol=1e-13)
    unit = (xi - s) / ri[:, None]
    np.testing.assert_allclose(lin, np.sum(unit * (xj - xi), axis=1) / V, rtol=0, atol=1e-13)


def test_taylor_remainder_bounds():
    """For T = r/c (convex) the remainder dT - lin is >= 0 and at most
    |dx|^2 / (2 c d_min), d_min the distance from s to the segment x_i x_j
    (the Hessian norm is 1/(c r), eq:dd_criterion)."""
    xi, xj, s = _geometry(2000, 2, sep=3.0)
    prob, theta = _problem(xi, xj, s)
    dT, lin = linearity.linearisation_terms(prob, _homogeneous(), theta)
    dx = xj - xi
    t = np.clip(np.sum((s - xi) * dx, axis=1) / np.sum(dx * dx, axis=1), 0.0, 1.0)
    dmin = np.linalg.norm(xi + t[:, None] * dx - s, axis=1)
    rem = dT - lin
    assert np.all(rem >= -1e-13)
    assert np.all(rem <= np.sum(dx * dx, axis=1) / (2 * V * dmin) + 1e-13)


def test_ray_and_perpendicular_displacements():
    """Along the ray from the station the expansion is exact (kept); a move
    perpendicular to it has lin = 0, so e = 1 (dropped at 5%); coincident
    events have dT = lin = 0 (kept)."""
    xi, _, s = _geometry(300, 3)
    u = (xi - s) / np.linalg.norm(xi - s, axis=1)[:, None]
    perp = np.cross(u, np.array([0.0, 0.0, 1.0]))
    perp /= np.linalg.norm(perp, axis=1)[:, None]
    net = _homogeneous()
    for xj, want_keep, want_e in [(xi + 1.5 * u, True, 0.0), (xi + 1.5 * perp, False, 1.0),
                                  (xi.copy(), True, 0.0)]:
        prob, theta = _problem(xi, xj, s)
        keep, e = linearity.linearity_mask(prob, net, theta)
        assert np.all(keep == want_keep)
        np.testing.assert_allclose(e, want_e, atol=1e-9)


def test_remainder_is_the_second_order_term():
    """For the catalog's (non-homogeneous) network the remainder dT - lin of
    a small separation h d is (h^2 / 2) d^T H(x_i) d, with H d taken by central
    differences of the network's gradient (eq:dd_criterion's expansion about
    x_i): an expansion about x_j flips its sign, a sign error in lin or a
    gradient that is not the network's leaves an O(h) remainder."""
    cat = synth.make_catalog("tiny")
    net = synth.net_for(cat)
    rng = np.random.default_rng(4)
    R = 400
    xi = cat.hypo0[rng.choice(cat.M, R), 0:3]
    s = cat.stations[rng.integers(0, cat.L, R)]
    d = rng.normal(0.0, 1.0, (R, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    eps = 1e-4
    gp = ott.travel_time(net, xi + eps * d, s)[1]
    gm = ott.travel_time(net, xi - eps * d, s)[1]
    dHd = np.sum(d * (gp - gm), axis=1) / (2 * eps)
    h = 0.005
    prob, theta = _problem(xi, xi + h * d, s)
    dT, lin = linearity.linearisation_terms(prob, net, theta)
    want = 0.5 * h * h * dHd
    big = np.abs(dHd) > 1e-3 * np.abs(dHd).max()
    assert big.mean() > 0.9
    np.testing.assert_allclose((dT - lin)[big], want[big], rtol=0.1)


def test_catalog_filter_keeps_a_subset():
    cat = synth.make_catalog("tiny")
    prob = lk.load(cat)
    keep, e = linearity.linearity_mask(prob, synth.net_for(cat), prob.hypo0)
    assert keep.shape == (cat.N,) and 0 < keep.sum() < cat.N
    np.testing.assert_array_equal(keep, e <= 0.05)
