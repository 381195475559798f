"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 CPU implementation of everything the GPU library
computes, written from the paper ("Preconditioned BFGS-based Uncertainty
Quantification in Elastic Full Waveform Inversion", Liu, Beller, Lei, Peter &
Tromp, 2020).  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the GPU library neither imports nor links it, and the two
share no code (the seeded input generators in ``workloads`` aside, which hold
none of the method's arithmetic).

Modules
  dense    eq. (3) inverse BFGS update applied recursively to a dense matrix
           (float64 and exact rationals), eq. (2) Hessian update.
  recursion eq. (3) applied to a block as a recursion on the pair index (C, OpenMP).
  bfgs     Alg. 1 driven full-history BFGS with exact line search on a
           quadratic (used to pin the input generator, never to feed the GPU).
  rsvd     Alg. 3 single-pass randomized SVD and eq. (10)/(14) posterior
           variance, step by step with LAPACK QR / LU / symmetric eigensolver.
  probes   Philox4x64-10 + Box-Muller probe vectors.
  mlp      float64 forward/backward/Adam of the learned-preconditioner network.

Parity status of every function is stated in its docstring; all are pinned by
``tests/test_oracle_*.py`` unless marked "parity unpinned".
"""
