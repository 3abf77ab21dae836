"""Checker: intergrid transfers and Galerkin coarse operators (FP64, CPU).

Test infrastructure only.

Prolongation (section "Geometric Multigrid preconditioner"): the natural
injection of the coarse finite element space into the fine one, i.e. the
coarse basis functions evaluated at the fine nodes, per field (Q2 for d and u,
Q1 for p, per material copy).  Restriction: the transpose of those weights
applied to *equations*, respecting the shuffled row layout (equations
restr_blocks / prol_blocks and the remark that both change when rows are
shuffled): a coarse momentum row (solid, interface or fluid momentum) gathers
the fine momentum rows of the same component wherever they are stored; a
coarse mesh-motion row gathers fine mesh-motion rows; a coarse solid
kinematic row gathers fine solid kinematic rows only; pressure rows gather
pressure rows of the same material.  Coarse operator: J_{l-1} = R J_l P
(Galerkin), with identity rows at coarse Dirichlet dofs.
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .fem import FLUID, SOLID, IFACE

# equation types of a row
ALE, SM, IM, FM, KS, PF, PS = range(7)
_MOMENTUM = (SM, IM, FM)


def _q2_weights_1d(I, nc):
    """Coarse Q2 nodes and basis values at fine Q2 grid index I (half-spacing of the fine mesh)."""
    ec = min(I // 4, nc - 1)
    t = (I - 4 * ec) / 4.0
    vals = [(2 * t - 1) * (t - 1), 4 * t * (1 - t), t * (2 * t - 1)]
    return [(2 * ec + a, v) for a, v in enumerate(vals) if v != 0.0]


def _q1_weights_1d(i):
    if i % 2 == 0:
        return [(i // 2, 1.0)]
    return [((i - 1) // 2, 0.5), ((i + 1) // 2, 0.5)]


def q2_injection(fine, coarse):
    """Scalar Q2 injection weights W (N2_fine x N2_coarse): W[j, i] = phi_i^coarse(x_j)."""
    dim = fine.dim
    rows, cols, vals = [], [], []
    for j, g in enumerate(fine.node_grid):
        per_dim = [_q2_weights_1d(int(g[d]), coarse.n[d]) for d in range(dim)]
        for combo in itertools.product(*per_dim):
            idx = 0
            v = 1.0
            for d in reversed(range(dim)):
                idx = idx * coarse.g2[d] + combo[d][0]
            for d in range(dim):
                v *= combo[d][1]
            rows.append(j)
            cols.append(idx)
            vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.N2, coarse.N2))


def p1disc_injection(fine, coarse):
    """P1disc injection: the coarse element's linear pressure restricted to each child.

    With the basis (1, 2(x_d - c_d)/h_d) the child coefficients are
    b_0 = a_0 + sum_d a_d s_d / 2 (s_d = -1 / +1 for the lower / upper child)
    and b_d = a_d / 2.
    """
    dim = fine.dim
    fe = fine.epdofs()
    ce = coarse.epdofs()
    rows, cols, vals = [], [], []
    for e in range(fine.ne):
        ix = fine.eidx[e]
        E = 0
        for d in reversed(range(dim)):
            E = E * coarse.n[d] + ix[d] // 2
        rows.append(fe[e, 0]); cols.append(ce[E, 0]); vals.append(1.0)
        for d in range(dim):
            s = -1.0 if ix[d] % 2 == 0 else 1.0
            rows.append(fe[e, 0]); cols.append(ce[E, 1 + d]); vals.append(0.5 * s)
            rows.append(fe[e, 1 + d]); cols.append(ce[E, 1 + d]); vals.append(0.5)
    return rows, cols, vals


def pressure_injection(fine, coarse):
    return q1_injection(fine, coarse) if fine.pspace == "q1" else p1disc_injection(fine, coarse)


def q1_injection(fine, coarse):
    """Pressure injection per material copy (ndof_p_fine x ndof_p_coarse in global p numbering)."""
    dim = fine.dim
    vgrid = np.array(list(itertools.product(*[range(m) for m in reversed(fine.g1)])))[:, ::-1]
    rows, cols, vals = [], [], []
    for v, g in enumerate(vgrid):
        per_dim = [_q1_weights_1d(int(g[d])) for d in range(dim)]
        for copy_f, copy_c in ((fine.pf, coarse.pf), (fine.ps, coarse.ps)):
            if copy_f[v] < 0:
                continue
            for combo in itertools.product(*per_dim):
                idx = 0
                w = 1.0
                for d in reversed(range(dim)):
                    idx = idx * coarse.g1[d] + combo[d][0]
                for d in range(dim):
                    w *= combo[d][1]
                assert copy_c[idx] >= 0, "coarse vertex lacks the material copy"
                rows.append(copy_f[v])
                cols.append(copy_c[idx])
                vals.append(w)
    return rows, cols, vals


def prolongation(fine, coarse, flag_f, flag_c):
    """P (n_fine x n_coarse): natural injection per field, zero rows at fine and
    zero columns at coarse Dirichlet dofs."""
    W = q2_injection(fine, coarse).tocoo()
    rows, cols, vals = [], [], []
    for f in range(2 * fine.dim):
        rows.append(f * fine.N2 + W.row)
        cols.append(f * coarse.N2 + W.col)
        vals.append(W.data)
    pr, pc, pv = pressure_injection(fine, coarse)
    rows.append(np.array(pr, np.int64))
    cols.append(np.array(pc, np.int64))
    vals.append(np.array(pv))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    keep = ~flag_f[r] & ~flag_c[c]
    P = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(fine.ndof, coarse.ndof))
    P.sort_indices()
    return P


def row_types(mesh):
    """Equation type of every row in the shuffled layout."""
    t = np.empty(mesh.ndof, np.int64)
    cls = mesh.nclass
    dtype = np.where(cls == FLUID, ALE, np.where(cls == SOLID, SM, IM))
    utype = np.where(cls == FLUID, FM, KS)
    for c in range(mesh.dim):
        t[mesh.d_dof(c, np.arange(mesh.N2))] = dtype
        t[mesh.u_dof(c, np.arange(mesh.N2))] = utype
    if mesh.pspace == "q1":
        t[mesh.pf[mesh.pf >= 0]] = PF
        t[mesh.ps[mesh.ps >= 0]] = PS
    else:
        ep = mesh.epdofs()
        t[ep[~mesh.solid].ravel()] = PF
        t[ep[mesh.solid].ravel()] = PS
    return t


def restriction(fine, coarse, flag_f, flag_c):
    """Equation-aware restriction R (n_coarse x n_fine).

    R[(coarse row of node i, component c), (fine row of node j, component c)]
    = phi_i(x_j) when the two rows hold compatible equations (any momentum
    with any momentum; mesh motion with mesh motion; solid kinematics with
    solid kinematics), whichever slot (d or u) each is stored in.  Pressure
    rows use the Q1 weights of their material.  Zero rows at coarse and zero
    columns at fine Dirichlet dofs.
    """
    W = q2_injection(fine, coarse).tocoo()
    tf = row_types(fine)
    tc = row_types(coarse)
    rows, cols, vals = [], [], []
    for c in range(fine.dim):
        for sf in (0, 1):              # fine slot: d or u
            for sc in (0, 1):          # coarse slot
                fr = (sf * fine.dim + c) * fine.N2 + W.row
                cr = (sc * coarse.dim + c) * coarse.N2 + W.col
                a, b = tc[cr], tf[fr]
                mom = np.isin(a, _MOMENTUM) & np.isin(b, _MOMENTUM)
                same = ((a == ALE) & (b == ALE)) | ((a == KS) & (b == KS))
                ok = mom | same
                rows.append(cr[ok])
                cols.append(fr[ok])
                vals.append(W.data[ok])
    pr, pc, pv = pressure_injection(fine, coarse)
    rows.append(np.array(pc, np.int64))
    cols.append(np.array(pr, np.int64))
    vals.append(np.array(pv))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    keep = ~flag_c[r] & ~flag_f[c]
    R = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(coarse.ndof, fine.ndof))
    R.sort_indices()
    return R


def galerkin(R, J, P, flag_c):
    """J_c = R J P with identity rows at the coarse Dirichlet dofs."""
    Jc = (R @ J @ P).tocsr()
    dn = np.nonzero(flag_c)[0]
    Jc = Jc + sp.csr_matrix((np.ones(dn.size), (dn, dn)), shape=Jc.shape)
    Jc = Jc.tocsr()
    Jc.sort_indices()
    return Jc
