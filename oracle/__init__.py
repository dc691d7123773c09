"""Plain, slow CPU oracle of the mQO hot path (arXiv 2605.06921).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the library never
does, and it imports nothing of the library.  It is written from the
paper: each function names the passage it follows.  Floating point is
float64 except the float32 replay used wherever a float decides an integer
(rounding at 0.5 / 0, clip masks), because those decisions must be taken in
the precision the GPU computes in.

Modules:
  philox      Philox4x64-10 counter-based generator (random draws)
  objectives  h, f_L, f_P, f_A, f_B and gradients (Sec. 3, Eq. (3)-(7))
  pga         PGA step (float64 / float32 replay), initialisation, adjoint
  discrete    rounding, evaluation, checker (8), gains, local search, reset
  solver      the round schedule with reset and acceptance (Sec. 4)
  brute       exhaustive answers for n <= 20
"""
from . import philox, objectives, pga, discrete, solver, brute  # noqa: F401
