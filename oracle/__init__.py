"""Plain, slow, obviously-correct FP64 CPU oracle for the mu-mode exponential
integrator path.

TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, imports or
links this package; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg do. It shares no code with the HIP path: the only module both
sides read is ``synth`` (seeded problem data, no method arithmetic).

Modules
  adr       extraction (eq:linop, eq:nonlin, eq:amaxbeta), 1D operators and the
            finite-difference remainder g(u) and full right-hand side F(u)
  expo      1D exponential factors (closed form through the sine transform),
            mu-mode products (Sec. 1 and Sec. 5.2), phi-functions, quadrature phi1
  schemes   the Lawson and exponential Runge-Kutta steps of the Appendix
  stability the scalar stability functions of Sec. 2 (Theorems thm:expeuler ..
            thm:stablawson2), used as pins
  fourier1d the periodic 1D pseudo-spectral setting of Sec. 4.1 (used only to
            reproduce the printed errors of Figure fig:ad1dex0_diffdeltaa)
  brute     brute-force checks: full Kronecker-sum matrix and its expm

Parity status per function is recorded in each module's header.
"""
