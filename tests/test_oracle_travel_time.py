"""Pins for the oracle's travel-time network and its hand-written source gradient."""
import numpy as np
import pytest
import torch

from oracle import travel_time as tt
from paper_2508_12117_amd import synth


def _points(n, seed):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.uniform(0, 10, n), rng.uniform(0, 10, n), rng.uniform(0.5, 10, n)])
    s = np.column_stack([rng.uniform(-5, 15, n), rng.uniform(-5, 15, n), np.zeros(n)])
    return x, s


def _net(H, D, zero_output=False, seed=3):
    return synth.make_net(H, D, center=[5.0, 5.0, 3.0], half_extent=[10.0, 10.0, 5.0],
                          seed=seed, zero_output=zero_output)


@pytest.mark.parametrize("H,D", [(32, 3), (128, 4)])
def test_zero_output_layer_is_homogeneous_medium(H, D):
    """o = 0 gives f = 1: T = |x - s|/v0 and grad T = (x - s)/(v0 |x - s|) (Sec. 2.1)."""
    x, s = _points(500, 1)
    T, g = tt.travel_time(_net(H, D, zero_output=True), x, s)
    r = np.linalg.norm(x - s, axis=1)
    np.testing.assert_allclose(T, r / 6.0, rtol=1e-15, atol=0)
    np.testing.assert_allclose(g, (x - s) / (6.0 * r[:, None]), rtol=1e-14, atol=1e-16)
    # eikonal: |grad T| = 1/c
    np.testing.assert_allclose(np.linalg.norm(g, axis=1), 1 / 6.0, rtol=1e-14)


def test_homogeneous_hessian_by_finite_differences():
    """H_T = (I - r^ r^T)/(c r), operator norm 1/(c r) (Sec. 2.1)."""
    net = _net(32, 3, zero_output=True)
    x, s = _points(20, 2)
    h = 1e-4
    for k in range(x.shape[0]):
        Hfd = np.zeros((3, 3))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            gp = tt.travel_time(net, (x[k] + e)[None], s[k][None])[1][0]
            gm = tt.travel_time(net, (x[k] - e)[None], s[k][None])[1][0]
            Hfd[:, a] = (gp - gm) / (2 * h)
        d = x[k] - s[k]
        r = np.linalg.norm(d)
        rh = d / r
        Hx = (np.eye(3) - np.outer(rh, rh)) / (6.0 * r)
        np.testing.assert_allclose(Hfd, Hx, atol=1e-8)
        assert abs(np.linalg.norm(Hfd, 2) - 1 / (6.0 * r)) < 1e-7


@pytest.mark.parametrize("H,D", [(32, 3), (128, 4), (64, 1)])
def test_gradient_central_differences(H, D):
    """Hand-written reverse sweep vs central differences, h = 1e-3 km."""
    net = _net(H, D)
    x, s = _points(200, 4)
    T, g = tt.travel_time(net, x, s)
    h = 1e-3
    fd = np.zeros_like(g)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd[:, a] = (tt.travel_time(net, x + e, s)[0] - tt.travel_time(net, x - e, s)[0]) / (2 * h)
    # truncation error h^2/6 T''' is ~1e-8 s/km here
    np.testing.assert_allclose(g, fd, atol=2e-7, rtol=0)


def test_gradient_matches_torch_autograd_float64():
    """Same network written in torch, differentiated by torch.autograd (float64, CPU)."""
    net = _net(128, 4, seed=9)
    x, s = _points(300, 5)
    T, g = tt.travel_time(net, x, s)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(s, dtype=torch.float64)
    c = torch.tensor(net.center)
    h = torch.tensor(net.half_extent)
    a = torch.cat([(xt - c) / h, (st - c) / h], dim=1)
    for l in range(net.D):
        a = torch.tanh(a @ torch.tensor(net.W[l], dtype=torch.float64).T
                       + torch.tensor(net.b[l], dtype=torch.float64))
    o = a @ torch.tensor(net.W[net.D][0], dtype=torch.float64) + float(net.b[net.D][0])
    Tt = torch.linalg.norm(xt - st, dim=1) / net.v0 * torch.nn.functional.softplus(o) / np.log(2.0)
    Tt.sum().backward()
    np.testing.assert_allclose(T, Tt.detach().numpy(), rtol=1e-14)
    np.testing.assert_allclose(g, xt.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_softplus_scale_is_stable_for_large_outputs():
    """f = softplus(o)/ln 2 stays finite and ~o/ln2 for large o, ~e^o/ln 2 for very negative o."""
    o = np.array([-800.0, -30.0, 0.0, 30.0, 800.0])
    f = np.logaddexp(0.0, o) / tt.LN2
    assert np.all(np.isfinite(f))
    np.testing.assert_allclose(f[3:], o[3:] / tt.LN2, rtol=1e-12)
    assert f[2] == 1.0
