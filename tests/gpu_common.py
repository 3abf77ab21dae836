"""Shared helpers of the GPU parity tests (inputs from the native builder,
expected values from the checker)."""

import functools

import numpy as np
import scipy.sparse as sp

from oracle import problem as oprob
from oracle import solver as osolver
from synth import config, fourier_coefficients


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def csr_of(p, level, which="J"):
    rp, ci, v, sh = p.csr(level, which)
    return sp.csr_matrix((v, ci, rp), shape=sh)


@functools.lru_cache(maxsize=None)
def product_problem(name, **kw):
    from paper_1709_05660_amd import Problem
    s = config(name).with_(**kw) if kw else config(name)
    return Problem(s, fourier_coefficients(s.dim, s.seed))


@functools.lru_cache(maxsize=None)
def oracle_hierarchy(name, fluid_ilu=False):
    """The checker's own, independently assembled hierarchy (with ILU(0)
    local solves on the fluid blocks when fluid_ilu)."""
    s = config(name).with_(fluid_ilu=fluid_ilu)
    return oprob.build(s, fourier_coefficients(s.dim, s.seed))


@functools.lru_cache(maxsize=None)
def oracle_on_product(name, fluid_ilu=False, **kw):
    """The checker's algorithm (LU local solves, or ILU(0) on the fluid
    blocks, V-cycle, FGMRES) run on the product builder's matrices and
    patches (of the named workload, or of it with the fields kw changed)."""
    p = product_problem(name, **kw)
    levels = []
    for l in range(p.nlevels):
        lv = osolver.Level(J=csr_of(p, l, "J"))
        if l > 0:
            lv.P = csr_of(p, l, "P")
            lv.R = csr_of(p, l, "R")
            lv.ptr, lv.dof, lv.owned, lv.kind = p.patches(l)
        levels.append(lv)
    osolver.setup_factors(levels, fluid_ilu=fluid_ilu)
    s = config(name).with_(fluid_ilu=fluid_ilu, **kw)
    h = oprob.Hierarchy(s, None, None, levels, p.b.copy(), p.y.copy(), None)
    return h
