"""The linearisation filter on the data (Sec. 2.1, eq:dd_linearization;
the 5% threshold of Sec. 4).

Test infrastructure: the plain FP64 reference the GPU path is checked
against.  Only the tests, the smoke entry point and the benchmark's CPU
baseline use it.

An observation of pair (i, j) at station s is in the linear regime when the
difference of travel times is close to its first-order Taylor expansion about
the first event:
  dT   = T(x_j; s) - T(x_i; s)                  (non-linear forward model)
  lin  = grad_x T(x_i; s) . (x_j - x_i)         (linearised forward model)
  e    = |dT - lin| / |dT|                      (linearisation error)
and it is kept iff |dT - lin| <= e_max |dT|, e_max = 0.05 (which keeps an
observation with dT = lin = 0 and drops one with dT = 0 != lin).
"""
from __future__ import annotations

import numpy as np

from . import likelihood as lk


def linearisation_terms(prob, net, theta):
    """dT and lin of every observation at the state theta [M,4] (net: the
    network, or the (P, S) pair of a two-phase catalog)."""
    pr = prob.obs_pair
    xi = theta[prob.pair_i[pr], 0:3]
    xj = theta[prob.pair_j[pr], 0:3]
    s = prob.stations[prob.obs_sta]
    ph = getattr(prob, "obs_phase", None)
    ph = np.zeros(len(pr), np.int64) if ph is None else ph
    Ti, gi = lk.travel_times(net, ph, xi, s)
    Tj, _ = lk.travel_times(net, ph, xj, s)
    dT = Tj - Ti
    lin = np.sum(gi * (xj - xi), axis=1)
    return dT, lin


def linearity_mask(prob, net, theta, max_rel_err: float = 0.05):
    """(keep mask, linearisation error e) of every observation."""
    dT, lin = linearisation_terms(prob, net, theta)
    dev = np.abs(dT - lin)
    keep = dev <= max_rel_err * np.abs(dT)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(dev == 0.0, 0.0, dev / np.abs(dT))
    return keep, e
