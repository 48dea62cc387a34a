"""SPIDER hot path on MI355X (gfx950): per-step double-difference likelihood
gradient and (preconditioned) Langevin update over a whole catalog.

The compute runs in the HIP library ``libspider.so`` (C-ABI declared in
``include/spider.h``); ``paper_2508_12117_amd.spider`` is its thin ctypes
binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
__all__ = ["synth", "spider"]
