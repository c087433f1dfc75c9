"""Plain FP64 CPU oracle for the all-at-once Radau IIA heat solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU path: the only module both sides use is
``heat_inputs`` (seeded synthetic inputs, no method arithmetic).

Every routine is the plain definition of what the paper computes, written for
a reader to check against the paper by eye (references are to the sections and
equations of "Mixed precision solvers for the all-at-once Runge--Kutta
discretization of the heat equation"):

* ``tableau``    -- Radau IIA Butcher tableau by collocation; Crout factor of
                    A_RK used by Rana's stage preconditioner (Sec. 3).
* ``grid``       -- finite-difference stiffness K (M = I) on the unit
                    square/cube, constant or variable diffusivity.
* ``allatonce``  -- the all-at-once operator of eq. (2.4) and its blocks
                    Phi, Psi1, Psi2, Theta, dense (tiny) and block-wise.
* ``stepping``   -- sequential Radau IIA stepping, eqs. (2.2)-(2.3): the
                    unique solution of eq. (2.4).  LU or exact DST solve.
* ``adjoint``    -- reverse stepping for A^T lambda = g, and gradients.
* ``multigrid``  -- geometric V-cycle for I + aK (the inexact inverse of the
                    shifted blocks, Sec. 4 / Sec. 5).
* ``precond``    -- the ideal block preconditioner P of eq. (3.1), the
                    practical P-tilde of eqs. (3.2)-(3.3) with inner GMRES
                    preconditioned by Rana's block-lower-triangular stage
                    preconditioner, and FGMRES (Algorithm 1, P_L = I).
* ``mms``        -- closed-form discrete solution for the sin-sin-exp
                    manufactured problem.

Parity status of each function is stated in its module header.
"""
