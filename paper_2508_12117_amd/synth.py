"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds the input recipe only: event geometry, station layout,
event-pair graph, observed differential times, network weights and the
hyperparameters of each workload.  It holds none of the method's
arithmetic (no travel-time network, no weights W_g, no likelihood, no
sampler): both sides compute those on their own from what is generated here.

Synthetic truth.  The paper's data sets are not available, so observed
differential times come from a homogeneous "true earth" (speed 6 km/s,
the closed-form medium of the paper's Sec. 2.1): tau_obs = (|x_i - s| -
|x_j - s|)/6 + (t_i - t_j) + N(0, 0.01^2), with true origin-time offsets 0.
Initial locations (the prior means) are the true ones plus
N(0, diag(0.2^2, 0.2^2, 0.2^2, 0.1^2)) (Sec. 4, event prior).  The network
that the method inverts with is a seeded random MLP (weights N(0, 1/fan_in),
biases 0), so the inverting forward model is deliberately not the truth, as
in the paper's synthetic test where a 1D model inverts 3D synthetics.

Two-phase workloads add S observations for a random subset of the P ones:
the same truth at speed 6/1.73 km/s with noise N(0, 0.02^2), inverted with
their own seeded network (scale speed v0/1.73) and their own sigma, kappa.

Units: km and s, z is depth (positive down), stations at z = 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

MASTER_SEED = 20250817
V_TRUE = 6.0          # km/s, homogeneous truth and network scale speed
NOISE_SIGMA = 0.01    # s, observation noise on differential times
THETA0_SIGMA = (0.2, 0.2, 0.2, 0.1)
VP_VS = 1.73          # P to S speed ratio of the S-phase observations


@dataclasses.dataclass
class Workload:
    """Sizes and hyperparameters of one synthetic workload."""
    name: str
    M: int
    L: int
    knn: int
    keep: float            # probability that a (pair, station) observation exists
    H: int                 # hidden width of the travel-time MLP
    D: int                 # number of hidden tanh layers
    batch: int             # minibatch size n per chain
    chains: int
    steps: int
    step_size: float = 1e-4
    beta2: float = 0.99
    eps_p: float = 1e-5
    sigma: float = 0.01    # s, IID term of Sigma_g (Table 1)
    kappa: float = 0.03    # s, shared-event term of Sigma_g (Table 1)
    p: float = 0.25        # decay exponent of the edge weights (Table 1)
    ell: float = 40.0      # km, length scale of the edge weights (Table 1)
    eps_w: float = 1e-5
    prior_sigma: tuple = (0.2, 0.2, 0.2, 0.1)        # Sec. 4, real catalogs
    centroid_sigma: tuple = (0.01, 0.01, 0.01, 0.01)  # Sec. 4
    v0: float = V_TRUE
    index: int = 0
    side: float = 200.0    # km, horizontal box side of the clustered generator
    s_frac: float = 0.0    # probability that a P observation also has an S observation
    sigma_s: float = 0.02  # s, IID term of the S-phase groups
    kappa_s: float = 0.05  # s, shared-event term of the S-phase groups


WORKLOADS = {
    # 200 events in a 10 km box, 20 stations, 8-NN pairs x all stations (32k obs)
    "tiny": Workload("tiny", M=200, L=20, knn=8, keep=1.0, H=32, D=3,
                     batch=1024, chains=1, steps=200, index=0),
    # tiny plus S observations for about half of the (pair, station) P ones
    "tiny2ph": Workload("tiny2ph", M=200, L=20, knn=8, keep=1.0, H=32, D=3,
                        batch=1024, chains=1, steps=200, index=5, s_frac=0.5),
    # 10k events (three planar faults + 20% background), 50 stations, 10-NN (5M obs)
    "faults10k": Workload("faults10k", M=10_000, L=50, knn=10, keep=1.0,
                          H=128, D=4, batch=65_536, chains=1, steps=5000, index=1),
    # 200k clustered events, 100 stations, 12-NN, 5/6 of (pair, station) kept (~200M obs)
    "clustered200k": Workload("clustered200k", M=200_000, L=100, knn=12,
                              keep=5.0 / 6.0, H=256, D=6, batch=1 << 20,
                              chains=8, steps=2000, index=3),
}


@dataclasses.dataclass
class Catalog:
    """One synthetic catalog in the layout the C-ABI loader takes."""
    wl: Workload
    hypo_true: np.ndarray   # [M,4] f64
    hypo0: np.ndarray       # [M,4] f64 (initial state and prior mean)
    stations: np.ndarray    # [L,3] f64
    pair_i: np.ndarray      # [P] i32
    pair_j: np.ndarray      # [P] i32
    obs_pair: np.ndarray    # [N] i32
    obs_sta: np.ndarray     # [N] i16
    obs_dt: np.ndarray      # [N] f32
    obs_phase: np.ndarray = None  # [N] i8, 0 = P, 1 = S (None: all P)

    @property
    def M(self):
        return self.hypo0.shape[0]

    @property
    def L(self):
        return self.stations.shape[0]

    @property
    def P(self):
        return self.pair_i.shape[0]

    @property
    def N(self):
        return self.obs_pair.shape[0]


def _rng(wl: Workload, seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([seed, wl.index, stream])))


def _planar_patch(rng, n, center, length, width, scatter):
    """Points on a randomly oriented planar patch plus normal scatter."""
    strike = rng.uniform(0.0, math.pi)
    dip = rng.uniform(math.pi / 4, math.pi / 2)
    s_hat = np.array([math.cos(strike), math.sin(strike), 0.0])
    d_hat = np.array([-math.sin(strike) * math.cos(dip),
                      math.cos(strike) * math.cos(dip), math.sin(dip)])
    n_hat = np.cross(s_hat, d_hat)
    a = rng.uniform(-length / 2, length / 2, n)
    b = rng.uniform(-width / 2, width / 2, n)
    c = rng.normal(0.0, scatter, n)
    return center + a[:, None] * s_hat + b[:, None] * d_hat + c[:, None] * n_hat


def _events_tiny(rng, wl):
    xyz = np.empty((wl.M, 3))
    xyz[:, 0:2] = rng.uniform(0.0, 10.0, (wl.M, 2))
    xyz[:, 2] = rng.uniform(0.5, 10.0, wl.M)
    sta = np.zeros((wl.L, 3))
    sta[:, 0:2] = rng.uniform(-5.0, 15.0, (wl.L, 2))
    return xyz, sta


def _events_faults(rng, wl):
    n_bg = wl.M // 5
    n_f = wl.M - n_bg
    sizes = [n_f // 3, n_f // 3, n_f - 2 * (n_f // 3)]
    parts = []
    for n in sizes:
        center = np.array([rng.uniform(10, 40), rng.uniform(10, 40), rng.uniform(6, 14)])
        parts.append(_planar_patch(rng, n, center, rng.uniform(10, 20),
                                   rng.uniform(5, 10), 0.05))
    bg = np.column_stack([rng.uniform(0, 50, n_bg), rng.uniform(0, 50, n_bg),
                          rng.uniform(0.5, 20, n_bg)])
    xyz = np.concatenate(parts + [bg])
    xyz[:, 2] = np.clip(xyz[:, 2], 0.5, 20.0)
    sta = np.zeros((wl.L, 3))
    sta[:, 0:2] = rng.uniform(0.0, 50.0, (wl.L, 2))
    return xyz, sta


def _events_clustered(rng, wl, side=200.0, depth=30.0):
    parts = []
    total = 0
    while total < wl.M:
        size = int(round(math.exp(rng.uniform(math.log(10), math.log(5000)))))
        size = min(size, wl.M - total)
        center = np.array([rng.uniform(0, side), rng.uniform(0, side),
                           rng.uniform(2.0, depth - 2.0)])
        patch = 0.1 * math.sqrt(size)
        parts.append(_planar_patch(rng, size, center, patch, patch, 0.05))
        total += size
    xyz = np.concatenate(parts)
    xyz[:, 2] = np.clip(xyz[:, 2], 0.5, depth)
    sta = np.zeros((wl.L, 3))
    sta[:, 0:2] = rng.uniform(0.0, side, (wl.L, 2))
    return xyz, sta


def make_catalog(name, seed: int = MASTER_SEED) -> Catalog:
    """Build workload `name` (or a Workload) from `seed`; identical arrays on every machine."""
    wl = name if isinstance(name, Workload) else WORKLOADS[name]
    geo = _rng(wl, seed, 0)
    if wl.name in ("tiny", "tiny2ph"):
        xyz, sta = _events_tiny(geo, wl)
    elif wl.name == "faults10k":
        xyz, sta = _events_faults(geo, wl)
    else:
        xyz, sta = _events_clustered(geo, wl, side=wl.side)
    M, L = wl.M, wl.L
    hypo_true = np.zeros((M, 4))
    hypo_true[:, 0:3] = xyz
    hypo0 = hypo_true + _rng(wl, seed, 1).normal(0.0, 1.0, (M, 4)) * np.array(THETA0_SIGMA)
    hypo0[:, 2] = np.maximum(hypo0[:, 2], 0.05)

    # directed k-nearest-neighbour event pairs (i, j in kNN(i)), in 3D
    _, nn = cKDTree(hypo_true[:, 0:3]).query(hypo_true[:, 0:3], k=wl.knn + 1)
    pair_i = np.repeat(np.arange(M, dtype=np.int32), wl.knn)
    pair_j = nn[:, 1:].reshape(-1).astype(np.int32)
    P = pair_i.shape[0]

    # true travel times of the homogeneous truth, [M, L]
    t_true = np.sqrt(((hypo_true[:, None, 0:3] - sta[None, :, :]) ** 2).sum(-1)) / V_TRUE

    obs = _rng(wl, seed, 2)
    noise = _rng(wl, seed, 3)
    pairs_per_sta = []
    for s in range(L):
        if wl.keep >= 1.0:
            idx = np.arange(P, dtype=np.int32)
        else:
            idx = np.flatnonzero(obs.random(P) < wl.keep).astype(np.int32)
        pairs_per_sta.append(idx)
    N = sum(len(x) for x in pairs_per_sta)
    obs_pair = np.empty(N, np.int32)
    obs_sta = np.empty(N, np.int16)
    obs_dt = np.empty(N, np.float32)
    o = 0
    for s, idx in enumerate(pairs_per_sta):
        k = len(idx)
        pi, pj = pair_i[idx], pair_j[idx]
        dt = (t_true[pi, s] - t_true[pj, s]) + (hypo_true[pi, 3] - hypo_true[pj, 3])
        dt += noise.normal(0.0, NOISE_SIGMA, k)
        obs_pair[o:o + k] = idx
        obs_sta[o:o + k] = s
        obs_dt[o:o + k] = dt
        o += k
    if wl.s_frac <= 0.0:
        return Catalog(wl, hypo_true, hypo0, sta, pair_i, pair_j, obs_pair, obs_sta, obs_dt)
    # S observations: a random subset of the P ones, times of the same
    # homogeneous truth at the S speed V_TRUE / VP_VS
    pick = _rng(wl, seed, 4).random(N) < wl.s_frac
    ns = int(pick.sum())
    sp, ss = obs_pair[pick], obs_sta[pick].astype(np.int64)
    pi, pj = pair_i[sp], pair_j[sp]
    dt_s = VP_VS * (t_true[pi, ss] - t_true[pj, ss]) + (hypo_true[pi, 3] - hypo_true[pj, 3])
    dt_s += _rng(wl, seed, 5).normal(0.0, 2 * NOISE_SIGMA, ns)
    return Catalog(wl, hypo_true, hypo0, sta, pair_i, pair_j,
                   np.concatenate([obs_pair, sp]), np.concatenate([obs_sta, obs_sta[pick]]),
                   np.concatenate([obs_dt, dt_s.astype(np.float32)]),
                   np.concatenate([np.zeros(N, np.int8), np.ones(ns, np.int8)]))


@dataclasses.dataclass
class Net:
    """Seeded random travel-time MLP 6 -> H x D (tanh) -> 1 in float32.

    W[0]: [H,6]; W[1..D-1]: [H,H]; W[D]: [1,H]; b[0..D-1]: [H]; b[D]: [1].
    center/half_extent map source and receiver coordinates to [-1, 1].
    """
    H: int
    D: int
    W: list
    b: list
    v0: float
    center: np.ndarray
    half_extent: np.ndarray


def make_net(H: int, D: int, center, half_extent, seed: int = MASTER_SEED,
             v0: float = V_TRUE, zero_output: bool = False) -> Net:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7, H, D])))
    W, b = [], []
    fan_in = 6
    for _ in range(D):
        W.append((rng.normal(0.0, 1.0, (H, fan_in)) / math.sqrt(fan_in)).astype(np.float32))
        b.append(np.zeros(H, np.float32))
        fan_in = H
    w_out = (rng.normal(0.0, 1.0, (1, H)) / math.sqrt(H)).astype(np.float32)
    if zero_output:
        w_out[:] = 0.0
    W.append(w_out)
    b.append(np.zeros(1, np.float32))
    return Net(H, D, W, b, float(v0), np.asarray(center, np.float64),
               np.asarray(half_extent, np.float64))


def net_box(cat: Catalog):
    """Center and half-extent of the box holding the initial events and the stations."""
    pts = np.concatenate([cat.hypo0[:, 0:3], cat.stations])
    lo, hi = pts.min(0), pts.max(0)
    return (lo + hi) / 2, np.maximum((hi - lo) / 2, 1e-3)


def net_for(cat: Catalog, seed: int = MASTER_SEED, phase: int = 0, **kw) -> Net:
    """The catalog's network for phase 0 (P) or 1 (S: scale speed v0 / VP_VS,
    its own weights)."""
    c, h = net_box(cat)
    if phase == 1:
        return make_net(cat.wl.H, cat.wl.D, c, h, seed=seed + 1, v0=cat.wl.v0 / VP_VS, **kw)
    return make_net(cat.wl.H, cat.wl.D, c, h, seed=seed, v0=cat.wl.v0, **kw)


# Several catalogs of uneven size advanced together: one catalog of 10^6
# events (200 stations, 1/6 of the (pair, station) observations kept,
# ~400M) and 16 catalogs of M_c events, log-uniform in [1k, 200k] (100
# stations, 5/6 kept, ~1,000 M_c observations each).  All come from the
# clustered generator with the box side scaled as 200 sqrt(M_c / 200k) km, so
# the areal density matches the 200k workload; 4 chains each; the minibatch
# is clamp(2^ceil(log2(0.01 N_c)), 2^14, 2^20); all share one network
# 6 -> 256 x 8 -> 1.
MULTI = {"multi17": dict(big=1_000_000, big_L=200, big_keep=1.0 / 6.0, n_small=16,
                         small_lo=1_000, small_hi=200_000, small_L=100, small_keep=5.0 / 6.0,
                         chains=4, H=256, D=8, index=20)}


def multi_workloads(name: str, seed: int = MASTER_SEED):
    """The per-catalog workloads of multi-catalog workload `name` (batch not yet set)."""
    m = MULTI[name]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, m["index"], 99])))
    sizes = [m["big"]] + [int(round(math.exp(rng.uniform(math.log(m["small_lo"]),
                                                          math.log(m["small_hi"])))))
                          for _ in range(m["n_small"])]
    out = []
    for k, M in enumerate(sizes):
        big = k == 0
        out.append(Workload(f"{name}.{k}", M=M, L=m["big_L"] if big else m["small_L"], knn=12,
                            keep=m["big_keep"] if big else m["small_keep"], H=m["H"], D=m["D"],
                            batch=0, chains=m["chains"], steps=2000, index=m["index"] + 1 + k,
                            side=200.0 * math.sqrt(M / 200_000)))
    return out


def multi_batch(N: int) -> int:
    """Minibatch of a catalog of N observations in a multi-catalog workload."""
    return int(min(max(1 << math.ceil(math.log2(0.01 * N)), 1 << 14), 1 << 20))


def make_multi(name: str, seed: int = MASTER_SEED, progress=None):
    """The catalogs of multi-catalog workload `name` and their shared network;
    `progress(k, cat)` is called after each catalog is made."""
    cats = []
    for k, wl in enumerate(multi_workloads(name, seed)):
        cat = make_catalog(wl, seed)
        cat.wl = dataclasses.replace(wl, batch=min(multi_batch(cat.N), cat.N))
        cats.append(cat)
        if progress is not None:
            progress(k, cat)
    return cats, net_for(cats[0], seed)


def random_theta(cat: Catalog, seed: int, scale=(0.05, 0.05, 0.05, 0.02)) -> np.ndarray:
    """A state near hypo0 (for gradient parity at a point other than the start)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    return cat.hypo0 + rng.normal(0.0, 1.0, cat.hypo0.shape) * np.asarray(scale)


def random_batch(N: int, n: int, seed: int) -> np.ndarray:
    """n distinct observation indices in [0, N), int64 (explicit-batch inputs)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 13])))
    return np.sort(rng.choice(N, size=n, replace=False)).astype(np.int64)
