"""Independent pins of the oracle's travel-time network (Sec. 2.1, Sec. 3.2).

The network definition, written out here with Python scalars and the math
module only (no matrix code, no call into the oracle's arithmetic):

    u_k   = (x_k - c_k)/h_k,  u_{3+k} = (s_k - c_k)/h_k           k = 0, 1, 2
    a1_n  = tanh(b0_n + sum_k W0[n][k] u_k)                       (6 inputs)
    a2_n  = tanh(b1_n + sum_m W1[n][m] a1_m)                      (hidden layer)
    o     = b2 + sum_n W2[0][n] a_D,n                             (no activation)
    f     = log(1 + e^o)/ln 2,  T = (|x - s|/v0) f

and the source gradient by the chain rule summed over paths (forward mode,
unlike the oracle's reverse sweep):

    do/dx_k = (1/h_k) sum_n W2[0][n] (1 - a2_n^2) sum_m W1[n][m] (1 - a1_m^2) W0[m][k]
    dT/dx_k = f (x_k - s_k)/(v0 |x - s|) + (|x - s|/v0) sigmoid(o)/ln 2 do/dx_k

The hand-picked weights are asymmetric and the biases non-zero, so a dropped
bias, a transposed hidden matrix, an extra or missing tanh layer, or a tanh on
the output each move T by far more than the tolerance (checked below by
planting each mistake in a scalar copy of the definition).
"""
import math

import numpy as np
import pytest

from oracle import travel_time as tt
from paper_2508_12117_amd import synth

# H = 2 hidden units, D = 2 tanh layers: 6 -> 2 -> 2 -> 1
W0 = [[0.30, -0.20, 0.50, 0.10, -0.40, 0.25],
      [-0.60, 0.45, 0.20, -0.35, 0.15, 0.05]]
B0 = [0.10, -0.20]
W1 = [[0.90, -0.70],
      [0.40, 1.10]]          # not symmetric: a transpose changes the result
B1 = [0.05, 0.30]
W2 = [[1.20, -0.80]]
B2 = [0.35]
V0 = 6.0
CENTER = [5.0, 5.0, 3.0]
HALF = [10.0, 10.0, 5.0]


def _net(w0=W0, b0=B0, w1=W1, b1=B1, w2=W2, b2=B2):
    f32 = lambda a: np.asarray(a, np.float32)
    W = [f32(w0), f32(w1), f32(w2)]
    b = [f32(b0), f32(b1), f32(b2)]
    return synth.Net(2, 2, W, b, V0, np.asarray(CENTER), np.asarray(HALF))


def _f32(v):
    """The weights as the network stores them (float32), widened exactly."""
    return float(np.float32(v))


def _by_hand(x, s, *, drop_bias=False, transpose_w1=False, extra_layer=False,
             skip_layer=False, tanh_output=False):
    """T and dT/dx from the definition, Python scalars only."""
    w0 = [[_f32(v) for v in row] for row in W0]
    w1 = [[_f32(v) for v in row] for row in W1]
    if transpose_w1:
        w1 = [[w1[m][n] for m in range(2)] for n in range(2)]
    w2 = [_f32(v) for v in W2[0]]
    b0 = [0.0 if drop_bias else _f32(v) for v in B0]
    b1 = [_f32(v) for v in B1]
    b2 = _f32(B2[0])
    u = [(x[k] - CENTER[k]) / HALF[k] for k in range(3)] + \
        [(s[k] - CENTER[k]) / HALF[k] for k in range(3)]
    a1 = [math.tanh(b0[n] + sum(w0[n][k] * u[k] for k in range(6))) for n in range(2)]
    if skip_layer:
        a2 = a1
    else:
        a2 = [math.tanh(b1[n] + sum(w1[n][m] * a1[m] for m in range(2))) for n in range(2)]
    if extra_layer:
        a2 = [math.tanh(b1[n] + sum(w1[n][m] * a2[m] for m in range(2))) for n in range(2)]
    o = b2 + sum(w2[n] * a2[n] for n in range(2))
    if tanh_output:
        o = math.tanh(o)
    f = math.log1p(math.exp(o)) / math.log(2.0)
    d = [x[k] - s[k] for k in range(3)]
    r = math.sqrt(sum(v * v for v in d))
    T = r / V0 * f
    sig = 1.0 / (1.0 + math.exp(-o))
    grad = []
    for k in range(3):
        dodx = 0.0
        for n in range(2):
            inner = 0.0
            for m in range(2):
                inner += w1[n][m] * (1.0 - a1[m] ** 2) * w0[m][k]
            dodx += w2[n] * (1.0 - a2[n] ** 2) * inner
        dodx /= HALF[k]
        grad.append(f * d[k] / (V0 * r) + r / V0 * sig / math.log(2.0) * dodx)
    return T, grad


POINTS = [((1.0, 2.0, 3.0), (-4.0, 7.5, 0.0)),
          ((8.5, 0.5, 9.0), (12.0, -3.0, 0.0)),
          ((5.0, 5.0, 0.6), (5.3, 4.1, 0.0))]


@pytest.mark.parametrize("x,s", POINTS)
def test_network_matches_definition_by_hand(x, s):
    T, g = tt.travel_time(_net(), np.array([x]), np.array([s]))
    Th, gh = _by_hand(x, s)
    assert abs(T[0] - Th) <= 1e-14 * Th
    np.testing.assert_allclose(g[0], gh, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("mistake", ["drop_bias", "transpose_w1", "extra_layer", "skip_layer",
                                     "tanh_output"])
def test_each_planted_mistake_is_caught(mistake):
    """Every plausible slip in the forward pass moves T by far more than the
    1e-14 tolerance of the pin above, at every point."""
    for x, s in POINTS:
        Th, _ = _by_hand(x, s)
        Tm, _ = _by_hand(x, s, **{mistake: True})
        assert abs(Tm - Th) > 1e-6 * Th, (mistake, x, s)


def test_network_shape_notation_counts_tanh_layers():
    """6 -> 256x6 -> 1 has exactly six tanh layers: with W0 copying input 0
    into neuron 0, identity hidden matrices, zero biases and the output reading
    neuron 0, the network output is tanh applied six times to u_0."""
    H, D = 256, 6
    net = synth.make_net(H, D, center=[0.0, 0.0, 0.0], half_extent=[1.0, 1.0, 1.0])
    assert len(net.W) == D + 1 and len(net.b) == D + 1
    assert net.W[0].shape == (H, 6) and net.W[D].shape == (1, H)
    assert all(net.W[l].shape == (H, H) for l in range(1, D))
    W = [np.zeros((H, 6), np.float32)] + [np.eye(H, dtype=np.float32) for _ in range(1, D)]
    W[0][0, 0] = 1.0
    wout = np.zeros((1, H), np.float32)
    wout[0, 0] = 1.0
    W.append(wout)
    b = [np.zeros(H, np.float32) for _ in range(D)] + [np.zeros(1, np.float32)]
    probe = synth.Net(H, D, W, b, 6.0, np.zeros(3), np.ones(3))
    x = np.array([[0.7, 0.1, 0.2]])
    s = np.array([[0.0, 0.0, 0.0]])
    o, _ = tt.network(probe, x, s)
    want = 0.7
    for _ in range(D):
        want = math.tanh(want)
    assert abs(o[0] - want) < 1e-15
    # one layer more or fewer is far away
    assert abs(math.tanh(want) - want) > 1e-3 and abs(math.atanh(want) - want) > 1e-3
