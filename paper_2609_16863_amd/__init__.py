"""MI355X-native all-at-once Radau IIA solver for the heat equation.

Hot path: right-preconditioned FP64 FGMRES on the all-at-once system of the
paper's eq. (2.4), with the block-triangular preconditioner of eqs.
(3.2)-(3.3) applied in FP64, FP32, BF16 or FP16 (inner GMRES with Rana's
stage preconditioner, geometric-multigrid V-cycles on the shifted blocks),
plus the transposed (adjoint) solve.  All arithmetic runs in hand-written HIP
kernels for gfx950 behind the C ABI of include/aao_heat.h.
"""
from .autograd import heat_solve  # noqa: F401
from .binding import AAOError, HeatBatch, HeatProblem  # noqa: F401
