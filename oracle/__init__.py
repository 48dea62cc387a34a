"""FP64 CPU oracle for the SPIDER hot path (arXiv 2508.12117).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
numpy/scipy implementation of what the GPU path computes, written from the
paper.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code
with the HIP library: its only common input is the seeded generator
``paper_2508_12117_amd.synth``, which holds none of the method's arithmetic.

Modules
  philox      Philox4x32-10 counter-based generator, 53-bit uniforms,
              Box-Muller normals (the Langevin noise stream).
  batch       keyed Feistel bijection of [0, N) that picks each minibatch
              without replacement within an epoch.
  travel_time travel-time network T(x; s) and its source gradient.
  likelihood  dd residuals (Eq. 1 / eq:forwardmodel), edge weights
              (eq:correlation_decay), whitening with Sigma_g
              (eq:marginal_sigma), per-event gradient, priors (Sec. 3.1).
  sampler     stochastic gradient (eq:sgd), SGLD and pSGLD updates
              (Sec. 3.2, eq:pSGLD), posterior moments (Sec. 3.4).

Every function is pinned by a test in ``tests/test_oracle_*.py`` against a
closed form, an invariant, brute force or an independent library routine.
"""
