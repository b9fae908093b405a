"""CPU oracle for the shifted SPAI-preconditioned CG solves of
Singh, Ahuja and Fassbender, "Preconditioned Iterative Solves in Model
Reduction of Second Order Linear Dynamical Systems" (arXiv 1606.01216).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written from the paper (binary64 unless stated; the reference solve
also runs in double-double).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call, link or execute anything in it.
It shares no code with the HIP library and never imports it; the two meet only
through the seeded inputs of the ``synthetic`` package.

Modules
  pencil     -- the shifted operator K(s) = s^2 M + s D + K, D = alpha M + beta K,
                for real and complex expansion points
  direct     -- banded Cholesky reference solve (binary64 and double-double);
                complex symmetric band L D L^T for complex expansion points
  spai       -- SPAI build (eq. (3.1), real or complex), SPAI update (Section
                3.2) and the preconditioner chain of the update algorithm
  pcg        -- preconditioned conjugate gradients; conjugate orthogonal CG
                for the complex symmetric K(s) of complex expansion points
  moments    -- Galerkin projection (eq. (1.4)) and the interpolation property
                of the reduced transfer function at the expansion points
  airga_loop -- AIRGA's outer iteration (Algorithm 1) with its readings
"""
from . import pencil, direct, spai, pcg, moments  # noqa: F401
