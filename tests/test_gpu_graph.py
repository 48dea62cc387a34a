"""HIP-graph replay of sampler steps against launching every step on the
stream: the same states, step counters and moments bit for bit, checked after
every call (each call captures a graph of one step and replays it), with
eager work and synchronisations between the calls; one catalog with several
chains and two catalogs fused into one step."""
import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, spider, synth, torch

pytestmark = pytest.mark.gpu


def _state(ctx, cid, C, M):
    out = []
    for c in range(C):
        th = torch.empty(M, 4, dtype=torch.float64, device="cuda")
        v = torch.empty_like(th)
        step = ctx.get_state(cid, c, th, v)
        out.append((host(th), host(v), step))
    mean = torch.empty(M, 4, dtype=torch.float64, device="cuda")
    cov = torch.empty(M, 10, dtype=torch.float64, device="cuda")
    cnt = ctx.moments(cid, -1, mean, cov)
    return out, host(mean), host(cov), cnt


def _run(graphs, cats, calls, steps, chains, batch, prec):
    ctx = make_ctx()
    try:
        ctx.set_graphs(graphs)
        net = synth.net_for(cats[0])
        nid = ctx.load_net(net)
        cids = [ctx.load_catalog(c, whiten=spider.WHITEN_EXACT, stream_id=10 + k)
                for k, c in enumerate(cats)]
        for cid in cids:
            ctx.reset_chains(cid, chains)
        sets = [(cid, nid, chains, batch, prec) for cid in cids]
        snaps = []
        for k in range(calls):
            ctx.sgld_steps(sets, steps, seed=41, burn_in=steps, thin=2)
            ctx.sync()
            # eager work between the replays of consecutive calls
            scratch = torch.randn(4096, device="cuda").sum()
            torch.cuda.synchronize()
            assert torch.isfinite(scratch)
            snaps.append([_state(ctx, cid, chains, c.M) for cid, c in zip(cids, cats)])
        return snaps
    finally:
        ctx.close()


def _equal(a, b):
    for sa, sb in zip(a, b):
        for (thetas_a, mean_a, cov_a, cnt_a), (thetas_b, mean_b, cov_b, cnt_b) in zip(sa, sb):
            assert cnt_a == cnt_b
            assert np.array_equal(mean_a, mean_b) and np.array_equal(cov_a, cov_b)
            for (ta, va, sta), (tb, vb, stb) in zip(thetas_a, thetas_b):
                assert sta == stb
                assert np.array_equal(ta, tb) and np.array_equal(va, vb)


@pytest.mark.parametrize("prec", [spider.FP32, spider.BF16])
def test_graph_steps_equal_stream_steps(prec):
    cat = synth.make_catalog("tiny")
    a = _run(True, [cat], calls=4, steps=25, chains=3, batch=1024, prec=prec)
    b = _run(False, [cat], calls=4, steps=25, chains=3, batch=1024, prec=prec)
    _equal(a, b)
    # the chains moved, and the moments were recorded
    assert a[-1][0][0][0][2] == 100 and a[-1][0][3] > 0


def test_graph_steps_fused_catalogs():
    tiny = synth.make_catalog("tiny")
    two = synth.make_catalog("tiny", seed=synth.MASTER_SEED + 1)
    a = _run(True, [tiny, two], calls=3, steps=10, chains=2, batch=512, prec=spider.FP32)
    b = _run(False, [tiny, two], calls=3, steps=10, chains=2, batch=512, prec=spider.FP32)
    _equal(a, b)
