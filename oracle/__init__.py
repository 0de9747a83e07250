"""FP64 CPU oracle for GCP-CROWN bound propagation (arXiv 2208.05740).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
(the HIP library and its binding) never does.  It shares no code with the
HIP path: its only common dependency is the seeded input generator in
``workloads``, which holds none of the bound arithmetic.

Modules
  gcp_oracle  Theorem 3.1 bound, its gradient (torch float64 autograd),
              the projected Adam loop.
  lp          The LP with cuts (eq. lp_with_cuts) and the MIP
              (eqs. mip_output..mip_inactive) through SciPy/HiGHS, the
              sampled minimum, and a plain forward pass.
  crown       Textbook CROWN / alpha-CROWN in primal form (an independent
              derivation used to pin the beta = gamma = 0 special case).
  root_bounds Layer-by-layer CROWN root bounds of the benchmark workloads
              (the Theorem 3.1 bound at beta = gamma = 0 on each prefix
              network); as a script it writes the stored bounds that the
              input generator reads.
"""
