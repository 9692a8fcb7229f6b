"""Plain FP64 CPU oracle for the GA-NGMRES transport-registration hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library (no kernels,
headers, helpers, tables or constants); the two meet only at the seeded input
generators in `synth`.

It follows He & Mang, "A generalized alternating NGMRES method for
PDE-constrained optimization problems governed by transport equations":

  spectral.py   Fourier pseudo-spectral calculus on [0,2pi)^d (Sec. 2.2,
                "Numerical Discretization"); regularisation operator and its
                inverse with the zero-mode rule; Leray projection (Sec. 3.5).
  interp.py     periodic tensor-product cubic Lagrange interpolation used by
                the semi-Lagrangian scheme (Sec. 2.2).
  transport.py  RK2 characteristics, state / adjoint semi-Lagrangian solves,
                objective (eq. e:varopt, e:varopt-optimal-transport) and the
                reduced gradient (eq. e:reduced-gradient, e:adjoint).
  ngmres.py     preconditioned fixed-point map with Armijo backtracking
                (eqs. e:linesearch, e:armijo, e:rpgd, e:fixedpoint), the
                least-squares mixing step, GA-NGMRES (Alg. 1 and Alg. 3) and
                GA-AA (Alg. 2 with the alternation of Alg. 3).
  deformation.py  the transport map y and det grad y reported with the
                results (Sec. 3, Sec. 3.5).

Every function is written for clarity: full complex FFTs, explicit loops over
the interpolation stencil, no fusion.  Readings of passages the paper leaves
open are listed in the module docstrings and in the design notes.

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, textbook routines or brute force; none is
"parity unpinned".
"""
