"""SPIDER hot path on MI355X (gfx950): per-step double-difference likelihood
gradient and (preconditioned) Langevin update over a whole catalog.

The compute runs in the HIP library ``libspider.so`` (C-ABI declared in
``include/spider.h``); ``paper_2508_12117_amd.spider`` is its thin ctypes
binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.

A whole inversion in the paper's four stages (Sec. 3.2), with torch tensors
for device memory::

    ctx = spider.Context(0)
    cid = ctx.load_catalog(cat)                  # events, stations, dd observations
    nid = ctx.load_net(net)                      # travel-time network (per phase)
    ctx.reset_chains(cid, 8)
    keep, _ = ctx.linearity(cid, nid)            # optional: linear-regime filter
    ctx.map_steps([(cid, nid, 8, n, spider.BF16)], k1)          # Stage 1: L1 + Adam
    keep, n_keep, med, mad = ctx.outliers(cid, nid)              # 4-MAD screen
    # reload the kept observations as a catalog, copy the Stage-1 states
    # over with set_state, then stages 2-4:
    ctx.sgld_stages([(cid, nid, 8, n, spider.BF16)], warmup, ramp, sample, thin=10)
    ctx.moments(cid, -1, mean, cov)              # pooled posterior moments

Sampler health: ``noise_ratio`` (the gradient-noise to injected-noise
ratio the paper targets at 0.1-1.0), ``set_sample_buffer`` + ``ess``,
``quantiles`` (credibility bounds) and ``sample_ranks`` (calibration).
"""
__all__ = ["synth", "spider"]
