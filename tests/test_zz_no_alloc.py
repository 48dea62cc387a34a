"""The allocation-free travel-time entry point against spider_travel_time,
through the C ABI: the same network kernel and assembly, so the results
must agree bit for bit; two calls in a row (the second smaller, so it reads
the scratch the first one left), both precisions, the size limit, and zero
rows."""
import ctypes as ct

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, spider, synth, torch
from oracle import travel_time as ott

pytestmark = pytest.mark.gpu


def _points(n, seed, box=10.0):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.uniform(0, box, n), rng.uniform(0, box, n), rng.uniform(0.5, box, n)])
    s = np.column_stack([rng.uniform(-box / 2, 1.5 * box, n), rng.uniform(-box / 2, 1.5 * box, n),
                         np.zeros(n)])
    return x, s


def _call(ctx, fn, nid, prec, x, s, with_grad=True):
    rows = x.shape[0]
    T = torch.full((rows,), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.full((rows, 3), float("nan"), dtype=torch.float64, device="cuda") if with_grad else None
    rc = fn(ctx._h, nid, prec, ct.c_void_p(x.data_ptr()), ct.c_void_p(s.data_ptr()), rows,
            ct.c_void_p(T.data_ptr()), ct.c_void_p(g.data_ptr()) if with_grad else None)
    assert rc == spider.OK, spider.lib().spider_last_error(ctx._h)
    return host(T), (host(g) if with_grad else None)


@pytest.mark.parametrize("H,D,prec", [(256, 6, spider.BF16), (256, 6, spider.FP32),
                                      (32, 3, spider.FP32), (48, 5, spider.FP32)])
def test_noalloc_matches_travel_time(H, D, prec):
    ctx = make_ctx()
    try:
        net = synth.make_net(H, D, center=[5.0, 5.0, 4.0], half_extent=[10.0, 10.0, 6.0],
                             seed=H * 3 + D)
        nid = ctx.load_net(net)
        L = spider.lib()
        # first call: several tiles and a ragged tail; second: fewer rows, so
        # any read of stale scratch rows would show
        for rows, seed in ((70_001, 1), (1_037, 2)):
            x, s = _points(rows, seed)
            xd, sd = dev(x), dev(s)
            T0, g0 = _call(ctx, L.spider_travel_time, nid, prec, xd, sd)
            T1, g1 = _call(ctx, L.spider_travel_time_noalloc, nid, prec, xd, sd)
            assert np.array_equal(T1, T0)
            assert np.array_equal(g1, g0)
            # and the oracle's bound for the precision (FP32: 1e-5 relative)
            if prec == spider.FP32:
                Tw, gw = ott.travel_time(net, x[:2000], s[:2000])
                assert np.max(np.abs(T1[:2000] - Tw) / Tw) < 1e-5
                err = np.linalg.norm(g1[:2000] - gw, axis=1) / np.linalg.norm(gw, axis=1)
                assert err.max() < 1e-5
        # T only
        x, s = _points(513, 3)
        T2, _ = _call(ctx, L.spider_travel_time_noalloc, nid, prec, dev(x), dev(s),
                      with_grad=False)
        T3, _ = _call(ctx, L.spider_travel_time, nid, prec, dev(x), dev(s), with_grad=False)
        assert np.array_equal(T2, T3)
    finally:
        ctx.close()


def test_noalloc_limits():
    ctx = make_ctx()
    try:
        net = synth.make_net(32, 3, center=[5.0, 5.0, 4.0], half_extent=[10.0, 10.0, 6.0])
        nid = ctx.load_net(net)
        L = spider.lib()
        e = torch.empty(0, 3, dtype=torch.float64, device="cuda")
        T = torch.empty(0, dtype=torch.float64, device="cuda")
        assert L.spider_travel_time_noalloc(ctx._h, nid, spider.FP32, ct.c_void_p(e.data_ptr()),
                                            ct.c_void_p(e.data_ptr()), 0,
                                            ct.c_void_p(T.data_ptr()), None) == spider.OK
        # one row more than the scratch holds: rejected before any launch
        big = spider.lib().spider_travel_time_noalloc(ctx._h, nid, spider.FP32, None, None,
                                                      1048576 + 1, None, None)
        assert big == spider.E_INVALID
        assert b"SPIDER_NOALLOC_MAX_ROWS" in L.spider_last_error(ctx._h)
        assert L.spider_travel_time_noalloc(ctx._h, 99, spider.FP32, None, None, 5, None,
                                            None) == spider.E_INVALID
    finally:
        ctx.close()
