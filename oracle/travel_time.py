"""Travel-time network T(x; s) and its gradient with respect to the source.

The paper uses a pretrained physics-informed Eikonal network (EikoNet,
Sec. 3.2) and notes any differentiable T will do (Sec. 5).  Here T is the
homogeneous-medium time of Sec. 2.1 scaled by a network correction:

    u = ((x - c0)/h, (s - c0)/h)                         inputs in [-1, 1]
    a_1 = tanh(W_0 u + b_0),  a_{l+1} = tanh(W_l a_l + b_l)   (D layers)
    o = W_D a_D + b_D
    f = softplus(o) / ln 2        (o = 0 gives f = 1: the homogeneous medium)
    T = (|x - s| / v0) * f

Gradients are reverse-mode (Sec. 3.2), written out by hand:
    delta_D = w_out * (1 - a_D^2),  delta_l = (delta_{l+1} W_l) * (1 - a_l^2)
    do/du = delta_1 W_0,  do/dx = (do/du)[:3] / h
    dT/dx = f (x - s)/(v0 |x - s|) + (|x - s|/v0) * sigmoid(o)/ln 2 * do/dx
All arithmetic in float64 (the float32 weights are widened exactly).
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

LN2 = np.log(2.0)
CHUNK = 1 << 16


def _layers(net):
    W = [np.asarray(w, np.float64) for w in net.W]
    b = [np.asarray(v, np.float64) for v in net.b]
    return W, b


def network(net, x, s):
    """Network output o and do/dx for sources x [R,3] and receivers s [R,3]."""
    W, b = _layers(net)
    D = len(W) - 1
    c = np.asarray(net.center, np.float64)
    h = np.asarray(net.half_extent, np.float64)
    R = x.shape[0]
    o = np.empty(R)
    dodx = np.empty((R, 3))
    for lo in range(0, R, CHUNK):
        hi = min(R, lo + CHUNK)
        u = np.concatenate([(x[lo:hi] - c) / h, (s[lo:hi] - c) / h], axis=1)
        acts = []
        a = u
        for l in range(D):
            a = np.tanh(a @ W[l].T + b[l])
            acts.append(a)
        o[lo:hi] = a @ W[D][0] + b[D][0]
        delta = W[D][0][None, :] * (1.0 - acts[D - 1] ** 2)
        for l in range(D - 1, 0, -1):
            delta = (delta @ W[l]) * (1.0 - acts[l - 1] ** 2)
        dodu = delta @ W[0]
        dodx[lo:hi] = dodu[:, 0:3] / h
    return o, dodx


def travel_time(net, x, s):
    """T(x; s) [R] and dT/dx [R,3] in float64."""
    x = np.asarray(x, np.float64)
    s = np.asarray(s, np.float64)
    o, dodx = network(net, x, s)
    diff = x - s
    dist = np.sqrt((diff ** 2).sum(1))
    T0 = dist / net.v0
    f = np.logaddexp(0.0, o) / LN2
    T = T0 * f
    grad = (f / (net.v0 * dist))[:, None] * diff + (T0 * expit(o) / LN2)[:, None] * dodx
    return T, grad
