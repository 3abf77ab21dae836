"""MI355X (gfx950) hot path of a monolithic ALE Newton-Krylov FSI solver.

FGMRES preconditioned by a geometric multigrid V-cycle with a
Richardson / restricted-additive-Schwarz smoother on interface-split patches
(Aulisa, Bna, Bornia 2017), as hand-written HIP kernels behind a C ABI
(include/fsi_mg.h); the host-side problem builder (include/fsi_problem.h)
generates the linear systems; the device assembly and Newton loop
(include/fsi_assembly.h) run the nonlinear iteration on the GPU.
"""

from ._lib import FsiError, lib  # noqa: F401
from .solver import MG, Assembly, Problem, Server, fmg, krylov_opts, mg_opts, stream_read_gbps  # noqa: F401
