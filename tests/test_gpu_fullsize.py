"""GPU parity at the full sizes the benchmark runs, through the C ABI.

clustered200k: 200,000 events, 200,002,156 observations, 6-256x6-1 network,
minibatch 2^20 per chain, 8 chains per launch, exact whitening, pSGLD, the
benchmark's seed and catalog stream.  The oracle evaluates one whole 2^20
minibatch of chain 0 at step 0 (about 20 s on the host), so every stage is
compared element by element at full size:

* batch indices: bit-exact (several chains and steps);
* FP32 path: per-event gradient within 1e-5 of S_m (the tolerance of the
  small-size tests), log posterior within 1e-5 relative, and the state after
  one 8-chain pSGLD step within what that gradient tolerance can move one
  update;
* BF16 path: travel times and source gradients of all 2^21 rows within the
  stated BF16 bound (1e-2 / 5e-2 relative), residuals within the bound those
  imply, and z solving Sigma_B z = r (matrix-free check of the definition);
* chain independence: chain 0 of the 8-chain launch equals a 1-chain launch
  bit for bit, in both precisions.

multi17: the 17 uneven catalogs (1,630,412 events, 1,030,414,821
observations, 6-256x8-1 network, 4 chains each).  One fused BF16 step over
all of them equals each catalog stepped alone, bit for bit, and sampled
network rows of the largest and a small catalog's minibatch are within the
BF16 bound of the oracle.
"""
import sys

import numpy as np
import pytest

from gpu_common import (dev, grad_scale, host, lk, make_ctx, psgld_update_tolerance,
                        scaled_grad_error, spider, synth, torch, whitening_residual)
from oracle import batch as obatch
from oracle import philox, sampler
from oracle import travel_time as ott

pytestmark = pytest.mark.gpu

SEED = 20250817          # the benchmark's seed
BF16_T_REL = 1e-2        # as in the small-size BF16 bound test
BF16_G_REL = 5e-2


def say(msg):
    print(f"[fullsize] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


@pytest.fixture(scope="module")
def c4(ctx):
    say("clustered200k: generating")
    cat = synth.make_catalog("clustered200k")
    net = synth.net_for(cat)
    wl = cat.wl
    cid = ctx.load_catalog(cat, whiten=spider.WHITEN_EXACT, stream_id=0)
    nid = ctx.load_net(net)
    say("clustered200k: oracle minibatch of chain 0, step 0")
    prob = lk.load(cat)
    idx = obatch.batch_indices(SEED, 0, 0, 0, cat.N, wl.batch)
    G, lp, bt = lk.grad_log_post(prob, net, prob.hypo0, idx, lk.WHITEN_EXACT)
    say("clustered200k: oracle done")
    return dict(cat=cat, net=net, wl=wl, cid=cid, nid=nid, prob=prob, idx=idx, G=G, lp=lp, bt=bt)


@pytest.mark.parametrize("chain,step", [(0, 0), (7, 0), (3, 190), (5, 191)])
def test_full_batch_indices(ctx, c4, chain, step):
    cat, wl = c4["cat"], c4["wl"]
    out = torch.empty(wl.batch, dtype=torch.int64, device="cuda")
    ctx.batch_indices(c4["cid"], SEED, chain, step, wl.batch, out)
    ref = c4["idx"] if (chain, step) == (0, 0) else obatch.batch_indices(SEED, 0, chain, step,
                                                                          cat.N, wl.batch)
    assert np.array_equal(host(out), ref)


def test_full_grad_fp32(ctx, c4):
    cat, prob, bt = c4["cat"], c4["prob"], c4["bt"]
    n = c4["wl"].batch
    G = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
    lp = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.grad(c4["cid"], c4["nid"], dev(prob.hypo0), G, n=n, seed=SEED, chain=0, step=0,
             logpost=lp, precision=spider.FP32)
    S = grad_scale(prob, bt, prob.N / n, prob.hypo0)
    # at theta_0 the prior terms vanish; events outside the batch carry only
    # the rounding of the GPU's centroid, so S_m is floored at 1
    err = scaled_grad_error(host(G), c4["G"], S, floor=1.0)
    say(f"FP32 gradient, 2^20 minibatch: max error / S_m = {err:.3e}")
    assert err < 1e-5
    assert abs(float(host(lp)[0]) - c4["lp"]) < 1e-5 * (abs(c4["lp"]) + 1)


def test_full_batch_terms_bf16(ctx, c4):
    prob, bt = c4["prob"], c4["bt"]
    out = ctx.batch_terms(c4["cid"], c4["nid"], dev(prob.hypo0), None, n=c4["wl"].batch,
                          seed=SEED, chain=0, step=0, precision=spider.BF16)
    Ti, Tj, r, z = (host(out[k]) for k in ("T_i", "T_j", "r", "z"))
    gi, gj = host(out["gT_i"]), host(out["gT_j"])
    eT = max(np.max(np.abs(Ti - bt.T_i) / bt.T_i), np.max(np.abs(Tj - bt.T_j) / bt.T_j))
    eg = max(np.max(np.linalg.norm(gi - bt.gT_i, axis=1) / np.linalg.norm(bt.gT_i, axis=1)),
             np.max(np.linalg.norm(gj - bt.gT_j, axis=1) / np.linalg.norm(bt.gT_j, axis=1)))
    say(f"BF16 rows of a 2^20 minibatch: T rel max {eT:.3e}, dT/dx rel max {eg:.3e}")
    assert eT < BF16_T_REL and eg < BF16_G_REL
    # r differs from the oracle's only through T: |dr| <= eT (T_i + T_j) + FP64 rounding
    assert np.all(np.abs(r - bt.r) <= eT * (bt.T_i + bt.T_j) + 1e-9)
    assert whitening_residual(r, z, bt, prob, lk.WHITEN_EXACT) < 1e-10


def _one_step_states(ctx, cid, nid, M, chains, n, prec, step_size):
    ctx.reset_chains(cid, chains)
    ctx.sgld_steps([(cid, nid, chains, n, prec)], 1, step=step_size, seed=SEED)
    out = []
    for c in range(chains):
        th = torch.empty(M, 4, dtype=torch.float64, device="cuda")
        ctx.get_state(cid, c, th)
        out.append(host(th))
    return out


@pytest.mark.parametrize("prec", [spider.FP32, spider.BF16])
def test_full_sgld_step_bench_launch(ctx, c4, prec):
    """One pSGLD step of all 8 chains in one launch, as the benchmark times it."""
    cat, wl, prob = c4["cat"], c4["wl"], c4["prob"]
    eight = _one_step_states(ctx, c4["cid"], c4["nid"], cat.M, wl.chains, wl.batch, prec,
                             wl.step_size)
    one = _one_step_states(ctx, c4["cid"], c4["nid"], cat.M, 1, wl.batch, prec, wl.step_size)
    assert all(np.all(np.isfinite(t)) for t in eight)
    assert np.array_equal(eight[0], one[0])
    assert not np.array_equal(eight[0], eight[7])
    if prec != spider.FP32:
        return
    # the oracle's state after the step, and how far a gradient error of
    # 1e-5 S_m can move it
    cfg = sampler.SamplerConfig(step=wl.step_size, seed=SEED)
    G = c4["G"]
    eta = philox.noise(SEED, 0, 0, 0, np.arange(cat.M))
    v0 = np.zeros_like(prob.hypo0)
    th_ref, _ = sampler.update(prob.hypo0, v0, G, cfg, eta)
    S = grad_scale(prob, c4["bt"], prob.N / wl.batch, prob.hypo0)
    dG = 1e-5 * np.maximum(S, 1.0)[:, None] * np.ones((1, 4))
    tol, _ = psgld_update_tolerance(prob.hypo0, v0, G, dG, cfg, eta)
    excess = np.abs(eight[0] - th_ref) / tol
    say(f"FP32 state after one step: max |error| / propagated tolerance = {excess.max():.3e}")
    assert np.all(excess <= 1.0)


# ------------------------------------------------------------------ multi17

@pytest.fixture(scope="module")
def c5(ctx):
    say("multi17: generating 17 catalogs")
    cats, net = synth.make_multi("multi17")
    ids = [ctx.load_catalog(c, whiten=spider.WHITEN_EXACT, stream_id=k) for k, c in enumerate(cats)]
    nid = ctx.load_net(net)
    say("multi17: loaded")
    return cats, net, ids, nid


def test_multi17_fused_step_equals_separate(ctx, c5):
    cats, _, ids, nid = c5
    sets = [(cid, nid, c.wl.chains, c.wl.batch, spider.BF16) for cid, c in zip(ids, cats)]

    def states():
        out = []
        for cid, c in zip(ids, cats):
            for ch in range(c.wl.chains):
                th = torch.empty(c.M, 4, dtype=torch.float64, device="cuda")
                ctx.get_state(cid, ch, th)
                out.append(host(th))
        return out

    for cid, c in zip(ids, cats):
        ctx.reset_chains(cid, c.wl.chains)
    ctx.sgld_steps(sets, 1, seed=SEED)
    fused = states()
    for cid, c in zip(ids, cats):
        ctx.reset_chains(cid, c.wl.chains)
    for s in sets:
        ctx.sgld_steps([s], 1, seed=SEED)
    alone = states()
    assert len(fused) == 68
    assert all(np.all(np.isfinite(a)) for a in fused)
    assert all(np.array_equal(a, b) for a, b in zip(fused, alone))


@pytest.mark.parametrize("which", [0, 1])
def test_multi17_network_rows_bf16(ctx, c5, which):
    """Sampled rows of chain 0's first minibatch (the 1M-event catalog and the
    smallest one) against the oracle's travel times."""
    cats, net, ids, nid = c5
    k = 0 if which == 0 else int(np.argmin([c.M for c in cats]))
    cat, cid = cats[k], ids[k]
    n = cat.wl.batch
    out = ctx.batch_terms(cid, nid, dev(cat.hypo0), None, n=n, seed=SEED, chain=0, step=0,
                          precision=spider.BF16)
    rng = np.random.default_rng(11 + k)
    slots = np.sort(rng.choice(n, size=min(n, 4096), replace=False))
    obs = obatch.permute(slots.astype(np.uint64), cat.N, SEED, k, 0, 0)
    pr = cat.obs_pair[obs]
    s = cat.stations[cat.obs_sta[obs]]
    Ti_w, gi_w = ott.travel_time(net, cat.hypo0[cat.pair_i[pr], 0:3], s)
    Tj_w, gj_w = ott.travel_time(net, cat.hypo0[cat.pair_j[pr], 0:3], s)
    Ti, Tj = host(out["T_i"])[slots], host(out["T_j"])[slots]
    gi, gj = host(out["gT_i"])[slots], host(out["gT_j"])[slots]
    eT = max(np.max(np.abs(Ti - Ti_w) / Ti_w), np.max(np.abs(Tj - Tj_w) / Tj_w))
    eg = max(np.max(np.linalg.norm(gi - gi_w, axis=1) / np.linalg.norm(gi_w, axis=1)),
             np.max(np.linalg.norm(gj - gj_w, axis=1) / np.linalg.norm(gj_w, axis=1)))
    say(f"multi17 catalog {k} (M={cat.M}): T rel max {eT:.3e}, dT/dx rel max {eg:.3e}")
    assert eT < BF16_T_REL and eg < BF16_G_REL
