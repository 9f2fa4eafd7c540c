"""CPU float64 oracle for sketched flexible LSQR / LSMR.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP implementation: it is
a plain, slow restatement of the paper's definitions and algorithms (numpy /
scipy, float64), used to decide what the GPU must compute.

Modules
  philox     Philox4x64-10 counter-based generator (Salmon et al., SC'11)
  sketches   sparse-sign / CountSketch, SRHT, Gaussian and identity sketches
  fgk        partially orthogonalised flexible Golub-Kahan; sFLSQR (Alg. 1),
             sFLSMR (Alg. 2), and full-orthogonalisation FLSQR / FLSMR
             (Sec. 2.2) for comparison
  lowrank    rank-r truncation tau_r of eq. (def:lowr-trc) (full SVD) and its
             randomized-SVD variant (Halko-Martinsson-Tropp), as flexible
             operators
  derivative forward-mode derivative of x_k in b and eps
  dense      definitional dense forms x_k = Z_k (S A Z_k)^+ S b, bounds of
             Theorem 1 and the expectation of Corollary 1
"""
