"""CPU oracle for parallel brute-force Bayesian cross-validation (PCV).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, fp64 restatement of
what the method computes, written from the paper (Cooper, Vehtari, Forbes,
Simpson, Kennedy: "Bayesian cross-validation by parallel Markov chain Monte
Carlo").  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it.  The product path (the HIP library and its Python binding)
never imports, calls or links anything here, and this package shares no code
with it: not kernels, not helpers, not constants.

Modules
  philox       counter-based random numbers (Philox4x32-10, Salmon et al. 2011)
  folds        per-fold row roles: excluded / train / test   (Appendix B, Sec. 2.2)
  model        masked log density, its gradient, log predictive (Appendix B)
  hmc          one HMC transition with fixed trajectory        (Section 3.3)
  sampler      online single-model LogS sampler                (Algorithm A2)
  diagnostics  elpd, MCSE, ESS, Rhat, Rhat_max                  (Sections 2.4, 4; App. A)
  closed_form  conjugate Gaussian posteriors and predictives (pins for the above)
  c_oracle     ctypes wrapper of c/pcv_oracle.c: the hot path (masked log density,
               HMC, Algorithm A2's accumulators, diagnostics) restated in plain C
               fp64 loops, independently of the numpy modules above

Parity status of every function is stated in its module header.
"""
