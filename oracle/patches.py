"""Checker: Schwarz patches split along the fluid/solid interface (CPU).

Test infrastructure only.

Section "Richardson-Schwarz smoother": the domain is first split into its
solid and fluid parts and each part into non-overlapping blocks made of whole
elements; the block matrix B_k is J restricted to the dofs of the block
(Vanka-type closure: every d, u, p dof of the block's elements), the overlap
comes from shared d/u nodes, and the restricted variant writes back only the
non-overlapping part R^0_k.

Readings: blocks are element boxes of patch^dim aligned to multiples of
`patch`, each split by material; order: all solid blocks (box order, x
fastest), then all fluid blocks; Dirichlet dofs are left out of every block;
a dof is owned (kept by R^0) by the first block in this order that contains
it, so interface d/u dofs belong to solid blocks.
"""

from __future__ import annotations

import itertools

import numpy as np


def build_patches(mesh, patch, dirichlet_flag):
    """Returns (ptr, dof, owned, kind): CSR-like patch lists.

    ptr (npatch+1,) int64; dof (ptr[-1],) int32 strictly increasing per patch;
    owned (ptr[-1],) uint8; kind (npatch,) uint8 (1 solid, 0 fluid).
    """
    dim = mesh.dim
    if any(m % patch for m in mesh.n):
        raise ValueError("mesh not divisible by the patch size")
    nb = [m // patch for m in mesh.n]
    boxes = sorted(itertools.product(*[range(b) for b in nb]), key=lambda b: tuple(reversed(b)))
    l2g = mesh.loc2glob()
    lists = {True: [], False: []}
    for b in boxes:
        ranges = [range(b[d] * patch, (b[d] + 1) * patch) for d in range(dim)]
        els = []
        for eix in itertools.product(*ranges):
            e = 0
            for d in reversed(range(dim)):
                e = e * mesh.n[d] + eix[d]
            els.append(e)
        els = np.array(els)
        for solid in (True, False):
            sel = els[mesh.solid[els] == solid]
            if sel.size == 0:
                continue
            dofs = np.unique(l2g[sel].ravel())
            dofs = dofs[~dirichlet_flag[dofs]]
            lists[solid].append(dofs)
    ordered = [(1, d) for d in lists[True]] + [(0, d) for d in lists[False]]
    seen = np.zeros(mesh.ndof, bool)
    ptr = [0]
    dof, owned, kind = [], [], []
    for k, d in ordered:
        own = ~seen[d]
        seen[d] = True
        dof.append(d)
        owned.append(own)
        kind.append(k)
        ptr.append(ptr[-1] + d.size)
    return (np.array(ptr, np.int64), np.concatenate(dof).astype(np.int32),
            np.concatenate(owned).astype(np.uint8), np.array(kind, np.uint8))


def closure_size(dim, patch, pressure="Q1dup"):
    """Number of dofs of the closure of one patch^dim element block (Dirichlet dofs included).

    pressure="P1disc" counts the paper's discontinuous linear pressure
    (dim+1 dofs per element); "Q1dup" counts Q1 vertices of one material.
    """
    nodes = (2 * patch + 1) ** dim
    if pressure == "P1disc":
        return 2 * dim * nodes + (dim + 1) * patch ** dim
    return 2 * dim * nodes + (patch + 1) ** dim


def p1disc_unknowns(dim, n):
    """Unknown count of the Q2-P1disc discretisation on an n-element box mesh."""
    nodes = int(np.prod([2 * m + 1 for m in n]))
    return 2 * dim * nodes + (dim + 1) * int(np.prod(n))
