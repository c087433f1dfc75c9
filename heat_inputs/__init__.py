"""Seeded synthetic inputs for the all-at-once heat solve.

This module only draws and samples input data (sources, initial conditions,
diffusivity fields, workload sizes).  It holds none of the method's
arithmetic, so both the GPU path's tests/benchmark and the CPU oracle use it.

The paper's own workloads are manufactured finite-element problems (Sec. 5);
no public dataset is involved.  These synthetic inputs stand in for them:

* ``mms``      -- u = sin(pi x) sin(pi y) e^{-t} (2D): u0 and f in closed form.
* ``bumps``    -- f(x, t) = sum_k a_k exp(-|x - x_k|^2 / (2 w_k^2))
                  sin(2 pi om_k t + ph_k), k = 1..8, a_k ~ N(0,1),
                  x_k ~ U[0.15, 0.85]^d, w_k ~ U[0.03, 0.12],
                  om_k ~ U[0.5, 3], ph_k ~ U[0, 2 pi].
* ``smooth``   -- u0 = sum over modes k_a <= 8 of c_k prod_a sin(k_a pi x_a)
                  / |k|^2, c_k ~ N(0, 1).
* ``paper_case_inputs`` -- the manufactured solution of the paper's
                  parallel test cases (Sec. 5.2, Table 4) at the nodes.
* ``kappa``    -- log kappa ~ N(0, 1) per cell of an 8^d patch partition of
                  the unit domain, kappa = clip(exp(.), 0.1, 10), sampled at
                  the interior nodes (the value of the patch holding the node).

Fields are flat FP64 arrays with x fastest (index i + n j + n^2 k), node
coordinates ((i+1) h, ...), h = 1/(n+1).
"""
from .generators import (  # noqa: F401
    WORKLOADS, Workload, nodes, sin_product, mms_source, bump_source,
    smooth_initial, lognormal_kappa, workload_inputs, batch_problem_specs,
    gradient_problem_specs, spec_inputs, spec_target_inputs, PaperCase, PAPER_CASES, paper_case_inputs,
)
