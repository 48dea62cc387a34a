"""BF16 error budget of the network kernel, on the CPU: the kernel's
arithmetic emulated in numpy (hidden-layer weights and the activations or
backward vectors entering each product rounded to BF16 with round to nearest
even, FP32 results, FP16 derivative factors 1 - a^2) against the FP64
oracle.  Pins the stated BF16 bound from the arithmetic alone and the
split-BF16 variants discussed with it: one layer's activations split into
BF16 hi + lo leaves the error where it was; weights and activations both
split bring the travel time to FP32-like accuracy."""
import numpy as np
import pytest

from oracle import travel_time as ott
from paper_2508_12117_amd import synth


def _bf16(a):
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _f16(a):
    return np.asarray(a, np.float16).astype(np.float64)


def _split(a, on):
    hi = _bf16(a)
    return hi + _bf16(a - hi) if on else hi


def _emulate(net, x, s, split_act=(), split_w=False):
    """Network output o and do/dx with BF16 products; layer l in split_act
    has its forward input and backward vector split into hi + lo."""
    W = [np.asarray(w, np.float64) for w in net.W]
    b = [np.asarray(v, np.float64) for v in net.b]
    D = len(W) - 1
    c, h = np.asarray(net.center), np.asarray(net.half_extent)
    u = np.concatenate([(x - c) / h, (s - c) / h], axis=1)
    Wq = [None] + [_split(W[l], split_w) for l in range(1, D)]
    a = _f32(np.tanh(_f32(u @ W[0].T + b[0])))
    acts = [a]
    for l in range(1, D):
        a = _f32(np.tanh(_f32(_split(a, l in split_act) @ Wq[l].T + b[l])))
        acts.append(a)
    o = _f32(a @ W[D][0] + b[D][0])
    delta = _f32(W[D][0][None, :] * _f16(1.0 - acts[D - 1] ** 2))
    for l in range(D - 1, 0, -1):
        delta = _f32(_f32(_split(delta, l in split_act) @ Wq[l]) * _f16(1.0 - acts[l - 1] ** 2))
    return o, _f32(delta @ W[0])[:, :3] / h


def _errors(net, x, s, Tw, gw, **kw):
    o, dodx = _emulate(net, x, s, **kw)
    diff = x - s
    dist = np.sqrt((diff ** 2).sum(1))
    T0 = dist / net.v0
    f = np.logaddexp(0.0, o) / np.log(2.0)
    T = T0 * f
    g = (f / (net.v0 * dist))[:, None] * diff + \
        (T0 / (1.0 + np.exp(-o)) / np.log(2.0))[:, None] * dodx
    eT = np.abs(T - Tw) / np.abs(Tw)
    eg = np.linalg.norm(g - gw, axis=1) / np.linalg.norm(gw, axis=1)
    return eT.max(), eg.max()


@pytest.fixture(scope="module")
def case():
    net = synth.make_net(256, 6, center=[100.0, 100.0, 15.0], half_extent=[100.0, 100.0, 15.0],
                         seed=5)
    rng = np.random.default_rng(3)
    n = 1024
    x = np.column_stack([rng.uniform(0, 200, n), rng.uniform(0, 200, n), rng.uniform(0.5, 30, n)])
    s = np.column_stack([rng.uniform(0, 200, n), rng.uniform(0, 200, n), np.zeros(n)])
    Tw, gw = ott.travel_time(net, x, s)
    return net, x, s, Tw, gw


def test_emulated_bf16_within_stated_bound(case):
    eT, eg = _errors(*case)
    # the BF16 path's stated bound (the tests of the device path hold the same)
    assert 5e-4 < eT < 1e-2 and 5e-3 < eg < 5e-2


def test_one_split_layer_does_not_tighten_the_bound(case):
    eT, eg = _errors(*case)
    for l in range(1, 6):
        eT1, eg1 = _errors(*case, split_act=(l,))
        assert eT1 > 0.5 * eT and eg1 > 0.5 * eg


def test_full_split_reaches_fp32_like_travel_times(case):
    eT, eg = _errors(*case, split_act=tuple(range(1, 6)), split_w=True)
    assert eT < 2e-5
    # the gradient is then bounded by the FP16 derivative factors (2^-11)
    assert 1e-4 < eg < 5e-3
