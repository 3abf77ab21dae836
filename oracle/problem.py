"""Checker: the multigrid hierarchy of one seeded steady FSI system (CPU, FP64).

Test infrastructure only.

Level l mesh = finest mesh coarsened l times by two in every direction
(midpoint refinement in reverse, section "Geometric Multigrid
preconditioner"); the finest operator is the exact Jacobian at the seeded
state, coarser ones are Galerkin products; patches on every level above the
coarsest.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fem, patches, solver, transfer


@dataclass
class Hierarchy:
    spec: object
    meshes: list          # coarsest first
    flags: list
    levels: list          # solver.Level, coarsest first
    b: np.ndarray
    y: np.ndarray
    r: np.ndarray


def mesh_sizes(spec):
    n = (spec.nx, spec.ny, spec.nz)[: spec.dim]
    L = spec.levels
    return [tuple(m // 2 ** (L - 1 - l) for m in n) for l in range(L)]


def build(spec, coeffs, factor=True):
    sizes = mesh_sizes(spec)
    meshes = [fem.Mesh(spec, s) for s in sizes]
    flags = [m.dirichlet(spec.u_peak)[0] for m in meshes]
    fine = meshes[-1]
    if getattr(spec, "transient", False):
        y_prev, y = fem.transient_states(fine, spec, coeffs)
        r, J = fem.assemble(fine, spec, y, y_prev=y_prev)
    else:
        y = fem.seeded_state(fine, spec, coeffs)
        r, J = fem.assemble(fine, spec, y)
    b = -r
    b[flags[-1]] = 0.0
    levels = [None] * spec.levels
    levels[-1] = solver.Level(J=J)
    for l in range(spec.levels - 1, 0, -1):
        P = transfer.prolongation(meshes[l], meshes[l - 1], flags[l], flags[l - 1])
        R = transfer.restriction(meshes[l], meshes[l - 1], flags[l], flags[l - 1])
        levels[l].P = P
        levels[l].R = R
        levels[l - 1] = solver.Level(J=transfer.galerkin(R, levels[l].J, P, flags[l - 1]))
    for l in range(1, spec.levels):
        ptr, dof, owned, kind = patches.build_patches(meshes[l], spec.patch, flags[l])
        lv = levels[l]
        lv.ptr, lv.dof, lv.owned, lv.kind = ptr, dof, owned, kind
    h = Hierarchy(spec, meshes, flags, levels, b, y, r)
    if factor:
        solver.setup_factors(levels, fluid_ilu=getattr(spec, "fluid_ilu", False))
    return h


def preconditioner(h):
    s = h.spec
    return lambda v: solver.vcycle(h.levels, len(h.levels) - 1, v, s.nu_pre, s.nu_post, s.omega)


def solve(h, **kw):
    s = h.spec
    kw.setdefault("restart", s.restart)
    kw.setdefault("rtol", s.rtol)
    kw.setdefault("maxit", s.maxit)
    return solver.fgmres(h.levels[-1].J, h.b, preconditioner(h), **kw)


def solve_paper(h, **kw):
    """The paper's Krylov setting (section "Details on the iterative solver"):
    left-preconditioned GMRES(10), one classical Gram-Schmidt pass, rtol 1e-4
    on the left-preconditioned residual; the V-cycle sweeps are the spec's."""
    kw.setdefault("restart", 10)
    kw.setdefault("rtol", 1e-4)
    kw.setdefault("maxit", h.spec.maxit)
    kw.setdefault("orth", "cgs")
    return solver.gmres_left(h.levels[-1].J, h.b, preconditioner(h), **kw)
