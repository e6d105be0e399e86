"""Plain FP64 CPU oracle for the stochastic multiscale flux basis method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the GPU library never
does.  Every function follows a passage of the paper (arXiv:1802.06263) and
cites it by section / equation label; where the paper is silent the reading
taken is named in the docstring.

Modules
  geometry     subdomains, interfaces, mortar spaces and index maps (Sec. 3)
  kl           separable-exponential KL expansion per region (Sec. 2.1, 6)
  collocation  Gauss-Hermite, tensor and Smolyak grids, local sets (Sec. 4)
  darcy        RT0-Q0 Darcy subdomain problems (Sec. 5.1, eqs. starD/barD)
  stokes       Q2-Q1 Stokes subdomain problems (Sec. 5.1, eqs. starS/barS)
  interface    interface operator, CG and FETI projection (Sec. 5.1)
  methods      Methods S1, S2, S3 and the moments (Sec. 5.2-5.4, Sec. 2)
  monolithic   the fully discrete coupled system solved directly (Sec. 4)
"""
