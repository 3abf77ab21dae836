"""Checker: structured Q2-P1disc monolithic ALE discretisation (FP64, CPU).

Test infrastructure only (see the package docstring).

Follows the paper's monolithic weak form (section "Weak FSI problem":
equations weakmom, cntsld, cntfld, kinsld, kinfld) in the steady case, on a
structured box mesh, with the readings used throughout this repository:

* velocity/displacement in Q2 and pressure in P1disc, the paper's pair
  (section "Discretization of the operator formulation"): dim+1 pressure
  dofs per element (its value at the element centre and its slopes), so the
  pressure is discontinuous between elements and across the interface.  A
  continuous Q1 pressure per material (duplicated at interface vertices) is
  kept as an option (spec.pressure = "q1"); the box-patch Richardson-Schwarz
  smoother diverges with it (a slow CPU test shows this);
* rows in the shuffled layout (equation jac_blocks_shuf): the displacement
  slot of a node carries the mesh-motion equation (fluid-only nodes), the
  solid momentum (solid-only nodes) or the interface momentum (interface
  nodes); the velocity slot carries the fluid momentum (fluid-only nodes) or
  the solid kinematic equation (solid-only and interface nodes);
* mesh motion in its harmonic form k grad(d):grad(phi) with k = 1/V_el
  (equation ale_eqn gives the symmetric form with the same k);
* neo-Hookean solid sigma = -p I + mu_s F F^T (2 C1 = mu_s);
* Dirichlet dofs are identity rows; their columns are dropped.

The Jacobian is the exact derivative of the residual, computed element by
element by complex-step differentiation, which is exact to rounding for the
analytic integrands used here (the paper uses automatic differentiation).
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

# node classes
FLUID, SOLID, IFACE = 0, 1, 2

_GP = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GW = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def q2_1d(t):
    """Quadratic Lagrange basis on [0,1] with nodes 0, 1/2, 1, and derivatives."""
    t = np.asarray(t, dtype=float)
    v = np.stack([(2 * t - 1) * (t - 1), 4 * t * (1 - t), t * (2 * t - 1)], axis=-1)
    dv = np.stack([4 * t - 3, 4 - 8 * t, 4 * t - 1], axis=-1)
    return v, dv


def q1_1d(t):
    t = np.asarray(t, dtype=float)
    return np.stack([1 - t, t], axis=-1)


@dataclass
class Tables:
    """Basis values at the 3^dim Gauss points of one (uniform) element."""

    N: np.ndarray      # (nq, na) Q2 values
    dN: np.ndarray     # (nq, na, dim) physical gradients
    psi: np.ndarray    # (nq, nv) Q1 values
    w: np.ndarray      # (nq,) physical weights
    vol: float


def element_tables(dim, h, pspace="p1disc"):
    t = (_GP + 1.0) / 2.0
    w1 = _GW / 2.0
    v, dv = q2_1d(t)            # (3 qp, 3 basis)
    p = q1_1d(t)                # (3 qp, 2 basis)
    qs = sorted(itertools.product(range(3), repeat=dim), key=lambda q: tuple(reversed(q)))
    As = sorted(itertools.product(range(3), repeat=dim), key=lambda a: tuple(reversed(a)))
    Vs = sorted(itertools.product(range(2), repeat=dim), key=lambda a: tuple(reversed(a)))
    nq, na = len(qs), len(As)
    nv = len(Vs) if pspace == "q1" else dim + 1
    N = np.ones((nq, na))
    dN = np.ones((nq, na, dim))
    psi = np.ones((nq, nv))
    w = np.ones(nq)
    for iq, q in enumerate(qs):
        for d in range(dim):
            w[iq] *= w1[q[d]] * h[d]
        for ia, a in enumerate(As):
            for d in range(dim):
                N[iq, ia] *= v[q[d], a[d]]
                for k in range(dim):
                    dN[iq, ia, k] *= (dv[q[d], a[d]] / h[d]) if k == d else v[q[d], a[d]]
        if pspace == "q1":
            for iv, a in enumerate(Vs):
                for d in range(dim):
                    psi[iq, iv] *= p[q[d], a[d]]
        else:
            # P1disc: 1 and the scaled centred coordinates 2 (x_d - x_c,d) / h_d
            for d in range(dim):
                psi[iq, 1 + d] = 2.0 * t[q[d]] - 1.0
    return Tables(N, dN, psi, w, float(np.prod(h)))


class Mesh:
    """Structured box mesh with a box-shaped solid, Q2 nodes and Q1 vertices.

    Element index e = ex + nx*(ey + ny*ez); Q2 node (I,J,K) on the half-spacing
    grid has index I + (2nx+1)*(J + (2ny+1)*K); Q1 vertex (i,j,k) has index
    i + (nx+1)*(j + (ny+1)*k).  An element is solid iff its centre lies
    strictly inside the solid box.
    """

    def __init__(self, spec, n):
        self.dim = spec.dim
        self.n = tuple(n[: self.dim])
        self.L = (spec.lx, spec.ly, spec.lz)[: self.dim]
        self.h = tuple(self.L[d] / self.n[d] for d in range(self.dim))
        dim = self.dim
        self.ne = int(np.prod(self.n))
        self.g2 = tuple(2 * m + 1 for m in self.n)
        self.g1 = tuple(m + 1 for m in self.n)
        self.N2 = int(np.prod(self.g2))
        self.N1 = int(np.prod(self.g1))
        eidx = np.array(list(itertools.product(*[range(m) for m in reversed(self.n)])))[:, ::-1]
        self.eidx = eidx                                      # (ne, dim) element multi-index
        lo, hi = spec.solid_lo[:dim], spec.solid_hi[:dim]
        centre = (eidx + 0.5) * np.array(self.h)
        self.solid = np.all((centre > np.array(lo)) & (centre < np.array(hi)), axis=1)
        As = sorted(itertools.product(range(3), repeat=dim), key=lambda a: tuple(reversed(a)))
        Vs = sorted(itertools.product(range(2), repeat=dim), key=lambda a: tuple(reversed(a)))
        self.enodes = np.zeros((self.ne, len(As)), dtype=np.int64)
        self.everts = np.zeros((self.ne, len(Vs)), dtype=np.int64)
        for ia, a in enumerate(As):
            idx = np.zeros(self.ne, dtype=np.int64)
            for d in reversed(range(dim)):
                idx = idx * self.g2[d] + (2 * eidx[:, d] + a[d])
            self.enodes[:, ia] = idx
        for iv, a in enumerate(Vs):
            idx = np.zeros(self.ne, dtype=np.int64)
            for d in reversed(range(dim)):
                idx = idx * self.g1[d] + (eidx[:, d] + a[d])
            self.everts[:, iv] = idx
        # node classes
        has_s = np.zeros(self.N2, bool)
        has_f = np.zeros(self.N2, bool)
        for e in range(self.ne):
            if self.solid[e]:
                has_s[self.enodes[e]] = True
            else:
                has_f[self.enodes[e]] = True
        self.nclass = np.where(has_s & has_f, IFACE, np.where(has_s, SOLID, FLUID))
        vs = np.zeros(self.N1, bool)
        vf = np.zeros(self.N1, bool)
        for e in range(self.ne):
            if self.solid[e]:
                vs[self.everts[e]] = True
            else:
                vf[self.everts[e]] = True
        # dof numbering: d_c, u_c over Q2 nodes (field-major), then pressure:
        # P1disc: dim+1 dofs per element, element-major; Q1: vertex copies,
        # fluid copy before solid copy.
        self.pspace = getattr(spec, "pressure", "p1disc")
        self.p_off = 2 * dim * self.N2
        self.pf = -np.ones(self.N1, dtype=np.int64)
        self.ps = -np.ones(self.N1, dtype=np.int64)
        k = self.p_off
        if self.pspace == "q1":
            for v in range(self.N1):
                if vf[v]:
                    self.pf[v] = k
                    k += 1
                if vs[v]:
                    self.ps[v] = k
                    k += 1
        else:
            k += (dim + 1) * self.ne
        self.ndof = k
        # node coordinates
        grid = np.array(list(itertools.product(*[range(m) for m in reversed(self.g2)])))[:, ::-1]
        self.xnode = grid * (np.array(self.h) / 2.0)
        vgrid = np.array(list(itertools.product(*[range(m) for m in reversed(self.g1)])))[:, ::-1]
        self.xvert = vgrid * np.array(self.h)
        self.node_grid = grid
        self.tab = element_tables(dim, self.h, self.pspace)

    def d_dof(self, c, node):
        return c * self.N2 + node

    def u_dof(self, c, node):
        return (self.dim + c) * self.N2 + node

    def p_dof(self, vert, solid):
        return self.ps[vert] if solid else self.pf[vert]

    def epdofs(self):
        """(ne, nv) pressure dofs of every element (its own P1disc dofs, or its material's Q1 copies)."""
        if self.pspace == "q1":
            return np.where(self.solid[:, None], self.ps[self.everts], self.pf[self.everts])
        nv = self.dim + 1
        return self.p_off + nv * np.arange(self.ne)[:, None] + np.arange(nv)[None, :]

    def solid_pressure_dofs(self):
        """Dofs holding the solid pressure level (Q1 solid copies, or P1disc constants of solid elements)."""
        if self.pspace == "q1":
            return self.ps[self.ps >= 0]
        return self.epdofs()[self.solid, 0]

    def loc2glob(self):
        """(ne, nloc) global dof of each element-local dof [d_c(a)..., u_c(a)..., p(v)]."""
        cols = []
        for c in range(self.dim):
            cols.append(self.d_dof(c, self.enodes))
        for c in range(self.dim):
            cols.append(self.u_dof(c, self.enodes))
        cols.append(self.epdofs())
        return np.concatenate(cols, axis=1)

    # ---------------------------------------------------------------- boundary
    def boundary_masks(self):
        g = self.node_grid
        on_bnd = np.zeros(self.N2, bool)
        wall = np.zeros(self.N2, bool)
        for d in range(self.dim):
            lo = g[:, d] == 0
            hi = g[:, d] == self.g2[d] - 1
            on_bnd |= lo | hi
            if d >= 1:
                wall |= lo | hi
        inflow = g[:, 0] == 0
        return on_bnd, inflow, wall

    def dirichlet(self, u_peak):
        """Dirichlet flags and values for every dof (reading of the boundary set-up).

        d = 0 on the whole outer boundary; u prescribed on the inflow (x = 0,
        parabolic profile of peak u_peak) and on the walls (no slip); the
        outflow x = Lx is stress free.  Pressure has no Dirichlet dofs.
        """
        on_bnd, inflow, wall = self.boundary_masks()
        flag = np.zeros(self.ndof, bool)
        val = np.zeros(self.ndof)
        prof = self.inflow_profile(u_peak)
        for c in range(self.dim):
            flag[self.d_dof(c, np.arange(self.N2))] = on_bnd
            uset = inflow | wall
            flag[self.u_dof(c, np.arange(self.N2))] = uset
            if c == 0:
                val[self.u_dof(0, np.arange(self.N2))] = np.where(uset, np.where(inflow, prof, 0.0), 0.0)
        return flag, val

    def inflow_profile(self, u_peak):
        x = self.xnode
        Ly = self.L[1]
        prof = u_peak * 4.0 * x[:, 1] * (Ly - x[:, 1]) / Ly ** 2
        if self.dim == 3:
            Lz = self.L[2]
            prof = prof * 4.0 * x[:, 2] * (Lz - x[:, 2]) / Lz ** 2
        return prof


# -------------------------------------------------------------------- state
def seeded_state(mesh, spec, coeffs):
    """Seeded linearisation state y = (d, u, p).

    d = 0; Dirichlet dofs take their boundary values; fluid-only free
    velocity nodes carry the inflow profile plus the smooth Fourier
    perturbation amp * S_c / max|S_c| with
    S_c = sum_{k,l(,m)=1..4} a_{c,k,l(,m)} / (k^2+l^2(+m^2)) prod sin(k pi x / L);
    solid and interface velocities are 0 (steady kinematics); fluid pressure
    dofs are 0 and the solid pressure level is mu_s (stress-free solid at d = 0).
    """
    dim = mesh.dim
    flag, val = mesh.dirichlet(spec.u_peak)
    y = np.zeros(mesh.ndof)
    prof = mesh.inflow_profile(spec.u_peak)
    free_f = mesh.nclass == FLUID
    shapes = fourier_shapes(mesh, coeffs)
    for c in range(dim):
        du = spec.amp * shapes[c]
        base = prof if c == 0 else 0.0
        uc = np.where(free_f, base + du, 0.0)
        y[mesh.u_dof(c, np.arange(mesh.N2))] = uc
    y[mesh.solid_pressure_dofs()] = spec.mu_s
    y[flag] = val[flag]
    return y


def fourier_shapes(mesh, coeffs):
    """S_c / max|S_c| at the Q2 nodes, c = 0..dim-1, with
    S_c = sum_{k,l(,m)=1..K} a_{c,k,l(,m)} / (k^2+l^2(+m^2)) prod sin(k pi x / L)."""
    dim = mesh.dim
    x = mesh.xnode
    K = coeffs.shape[1]
    out = []
    for c in range(dim):
        S = np.zeros(mesh.N2)
        for ks in itertools.product(range(1, K + 1), repeat=dim):
            term = np.full(mesh.N2, coeffs[(c,) + tuple(k - 1 for k in ks)] / float(sum(k * k for k in ks)))
            for d in range(dim):
                term = term * np.sin(ks[d] * np.pi * x[:, d] / mesh.L[d])
            S += term
        out.append(S / np.max(np.abs(S)))
    return out


def transient_states(mesh, spec, coeffs):
    """States of one Crank-Nicolson time step: y_n = the seeded state, and the
    Newton iterate y_{n+1} at which the Jacobian is taken: y_n with every free
    displacement dof moved by amp_d * S_c / max|S_c| (the shape of the
    velocity perturbation); Dirichlet dofs keep their boundary values."""
    y0 = seeded_state(mesh, spec, coeffs)
    y1 = y0.copy()
    flag, _ = mesh.dirichlet(spec.u_peak)
    shapes = fourier_shapes(mesh, coeffs)
    nodes = np.arange(mesh.N2)
    for c in range(mesh.dim):
        dd = mesh.d_dof(c, nodes)
        y1[dd] += np.where(flag[dd], 0.0, spec.amp_d * shapes[c])
    return y0, y1


# ------------------------------------------------------------- integrands
def _det_inv(F):
    """Determinant and inverse of (..., dim, dim) complex matrices (adjugate formulas)."""
    dim = F.shape[-1]
    if dim == 2:
        a, b, c, d = F[..., 0, 0], F[..., 0, 1], F[..., 1, 0], F[..., 1, 1]
        det = a * d - b * c
        inv = np.empty_like(F)
        inv[..., 0, 0] = d / det
        inv[..., 0, 1] = -b / det
        inv[..., 1, 0] = -c / det
        inv[..., 1, 1] = a / det
        return det, inv
    cof = np.empty_like(F)
    for i in range(3):
        for j in range(3):
            i1, i2 = (i + 1) % 3, (i + 2) % 3
            j1, j2 = (j + 1) % 3, (j + 2) % 3
            cof[..., i, j] = F[..., i1, j1] * F[..., i2, j2] - F[..., i1, j2] * F[..., i2, j1]
    det = F[..., 0, 0] * cof[..., 0, 0] + F[..., 0, 1] * cof[..., 0, 1] + F[..., 0, 2] * cof[..., 0, 2]
    inv = np.swapaxes(cof, -1, -2) / det[..., None, None]
    return det, inv


def _kinematics(T, dim, Ue):
    """Displacement/velocity/pressure fields of a batch of elements at the
    quadrature points: d, u, p (nodal), grad_hat d, F, J, F^{-1}, p_q, u_q."""
    na = T.N.shape[1]
    E = Ue.shape[0]
    d = Ue[:, : dim * na].reshape(E, dim, na)
    u = Ue[:, dim * na: 2 * dim * na].reshape(E, dim, na)
    p = Ue[:, 2 * dim * na:]
    Gd = np.einsum("eca,qak->eqck", d, T.dN)
    F = Gd + np.eye(dim)
    Jd, Finv = _det_inv(F)
    pq = np.einsum("ev,qv->eq", p, T.psi)
    uq = np.einsum("eca,qa->eqc", u, T.N)
    return d, u, p, Gd, F, Jd, Finv, pq, uq


def element_residual_cn(mesh, spec, Ue, Ue0, solid, k_scale=1.0):
    """Local residuals of one Crank-Nicolson step (section "Discretization of
    the operator formulation", the time-discretized operators F_n, S_n):
    the state at t_{n+1} is Ue (real or complex), the state at t_n is Ue0.
    Fluid momentum: (rho/dt)(u1 J1 - u0 J0) phi, then half of each of
    -rho div(w) u phi + rho ((u - w).grad) u phi + sigma : grad phi on the
    configuration of t_{n+1} (from Ue) and of t_n (from Ue0), with the mesh
    velocity w = (d1 - d0)/dt; continuity at t_{n+1}; mesh motion as in the
    steady form, at t_{n+1}.  Solid momentum: (rho_s/dt)(J1 u1 - J0 u0) phi
    plus half of each Piola stress term; incompressibility (J1 - 1) psi;
    kinematics -(d1 - d0)/dt + (u1 + u0)/2 against phi.  Returns (mom, aux, pres)
    as element_residual."""
    dim = mesh.dim
    T = mesh.tab
    dt = spec.dt
    w = T.w
    eye = np.eye(dim)
    d1, u1, p1, Gd1, F1, J1, Fi1, pq1, uq1 = _kinematics(T, dim, Ue)
    d0, u0, p0, Gd0, F0, J0, Fi0, pq0, uq0 = _kinematics(T, dim, Ue0)
    if not solid:
        wq = np.einsum("eca,qa->eqc", (d1 - d0) / dt, T.N)          # mesh velocity
        Gw = (Gd1 - Gd0) / dt                                        # grad_hat w
        gu1 = np.einsum("eqck,eqkb->eqcb", np.einsum("eca,qak->eqck", u1, T.dN), Fi1)
        gu0 = np.einsum("eqck,eqkb->eqcb", np.einsum("eca,qak->eqck", u0, T.dN), Fi0)
        divw1 = np.einsum("eqck,eqkc->eq", Gw, Fi1)
        divw0 = np.einsum("eqck,eqkc->eq", Gw, Fi0)
        sig1 = -pq1[..., None, None] * eye + spec.mu * (gu1 + np.swapaxes(gu1, -1, -2))
        sig0 = -pq0[..., None, None] * eye + spec.mu * (gu0 + np.swapaxes(gu0, -1, -2))
        rho = spec.rho
        v1 = (rho / dt) * uq1 - 0.5 * rho * divw1[..., None] * uq1 \
            + 0.5 * rho * np.einsum("eqcb,eqb->eqc", gu1, uq1 - wq)
        v0 = -(rho / dt) * uq0 - 0.5 * rho * divw0[..., None] * uq0 \
            + 0.5 * rho * np.einsum("eqcb,eqb->eqc", gu0, uq0 - wq)
        gphi1 = np.einsum("qak,eqkb->eqab", T.dN, Fi1)
        gphi0 = np.einsum("qak,eqkb->eqab", T.dN, Fi0)
        wJ1, wJ0 = w * J1, w * J0
        mom = (np.einsum("eq,eqc,qa->eca", wJ1, v1, T.N) + np.einsum("eq,eqc,qa->eca", wJ0, v0, T.N)
               + 0.5 * np.einsum("eq,eqcb,eqab->eca", wJ1, sig1, gphi1)
               + 0.5 * np.einsum("eq,eqcb,eqab->eca", wJ0, sig0, gphi0))
        pres = np.einsum("eq,qv->ev", wJ1 * np.einsum("eqcc->eq", gu1), T.psi)
        k = k_scale / T.vol
        aux = k * np.einsum("q,eqcb,qab->eca", w, Gd1, T.dN)
    else:
        def piola(F, J, Fi, pq):
            sig = -pq[..., None, None] * eye + spec.mu_s * np.einsum("eqik,eqjk->eqij", F, F)
            return J[..., None, None] * np.einsum("eqck,eqbk->eqcb", sig, Fi)
        P1, P0 = piola(F1, J1, Fi1, pq1), piola(F0, J0, Fi0, pq0)
        mass = (spec.rho_s / dt) * (J1[..., None] * uq1 - J0[..., None] * uq0)
        mom = np.einsum("q,eqc,qa->eca", w, mass, T.N) + 0.5 * np.einsum("q,eqcb,qab->eca", w, P1 + P0, T.dN)
        pres = np.einsum("q,eq,qv->ev", w, J1 - 1.0, T.psi)
        dq1 = np.einsum("eca,qa->eqc", d1, T.N)
        dq0 = np.einsum("eca,qa->eqc", d0, T.N)
        kin = -(dq1 - dq0) / dt + 0.5 * (uq1 + uq0)
        aux = np.einsum("q,eqc,qa->eca", w, kin, T.N)
    return mom, aux, pres


def element_residual(mesh, spec, Ue, solid, k_scale=1.0):
    """Local residual vectors of a batch of elements of one material.

    Ue: (E, nloc) local dof values [d_c(a), u_c(a), p(v)] (real or complex).
    Returns (mom, aux, pres): mom (E, dim, na) is the fluid momentum
    (weakmom, fluid part, steady) or the solid momentum (weakmom, solid part);
    aux (E, dim, na) is the mesh-motion equation (kinfld, harmonic) for fluid
    elements or the solid kinematic equation (kinsld, steady: (u, phi)) for
    solid ones; pres (E, nv) is the fluid continuity (cntfld) or the solid
    incompressibility (cntsld).  Integrals are on the reference (ALE)
    configuration: dx = J dx_hat, grad(phi) = F^{-T} grad_hat(phi).
    """
    dim = mesh.dim
    T = mesh.tab
    na = T.N.shape[1]
    E = Ue.shape[0]
    d = Ue[:, : dim * na].reshape(E, dim, na)
    u = Ue[:, dim * na: 2 * dim * na].reshape(E, dim, na)
    p = Ue[:, 2 * dim * na:]
    Gd = np.einsum("eca,qak->eqck", d, T.dN)
    F = Gd + np.eye(dim)
    Jd, Finv = _det_inv(F)
    pq = np.einsum("ev,qv->eq", p, T.psi)
    uq = np.einsum("eca,qa->eqc", u, T.N)
    w = T.w
    eye = np.eye(dim)
    if not solid:
        Guh = np.einsum("eca,qak->eqck", u, T.dN)
        gu = np.einsum("eqck,eqkb->eqcb", Guh, Finv)           # Eulerian grad u
        sig = -pq[..., None, None] * eye + spec.mu * (gu + np.swapaxes(gu, -1, -2))
        conv = spec.rho * np.einsum("eqcb,eqb->eqc", gu, uq)
        gphi = np.einsum("qak,eqkb->eqab", T.dN, Finv)          # Eulerian grad phi
        wJ = w * Jd
        mom = np.einsum("eq,eqc,qa->eca", wJ, conv, T.N) + np.einsum("eq,eqcb,eqab->eca", wJ, sig, gphi)
        div = np.einsum("eqcc->eq", gu)
        pres = np.einsum("eq,qv->ev", wJ * div, T.psi)
        k = k_scale / T.vol
        aux = k * np.einsum("q,eqcb,qab->eca", w, Gd, T.dN)
    else:
        B = np.einsum("eqik,eqjk->eqij", F, F)
        sig = -pq[..., None, None] * eye + spec.mu_s * B
        Piola = Jd[..., None, None] * np.einsum("eqck,eqbk->eqcb", sig, Finv)
        mom = np.einsum("q,eqcb,qab->eca", w, Piola, T.dN)
        pres = np.einsum("q,eq,qv->ev", w, Jd - 1.0, T.psi)
        aux = np.einsum("q,eqc,qa->eca", w, uq, T.N)
    return mom, aux, pres


def local_rows(mesh, solid_mat, transient=False):
    """Structural dependency mask (nloc_rows x nloc_cols) of one element type.

    Local rows are [mom(c,a), aux(c,a), pres(v)], local columns [d(c,a), u(c,a), p(v)].
    Fluid: momentum depends on d, u, p; mesh motion (harmonic) on the same
    displacement component; continuity on d and u.  Solid (steady): momentum
    on d and p; kinematics on the same velocity component; incompressibility on d.
    A Crank-Nicolson step adds the solid momentum's dependence on the same
    velocity component (mass) and the kinematics' on the same displacement
    component (section "Structure of the Jacobian": the blocks that vanish
    only in the steady case).
    """
    dim = mesh.dim
    na = mesh.tab.N.shape[1]
    nv = mesh.tab.psi.shape[1]
    nd = dim * na
    nl = 2 * nd + nv
    M = np.zeros((nl, nl), bool)
    sl_d = slice(0, nd)
    sl_u = slice(nd, 2 * nd)
    sl_p = slice(2 * nd, nl)
    comp = np.repeat(np.arange(dim), na)
    same = comp[:, None] == comp[None, :]
    if not solid_mat:
        M[0:nd, :] = True
        M[nd:2 * nd, sl_d] = same
        M[2 * nd:, sl_d] = True
        M[2 * nd:, sl_u] = True
    else:
        M[0:nd, sl_d] = True
        M[0:nd, sl_p] = True
        M[nd:2 * nd, sl_u] = same
        M[2 * nd:, sl_d] = True
        if transient:
            M[0:nd, sl_u] = same
            M[nd:2 * nd, sl_d] = same
    return M


def row_targets(mesh):
    """Global row of every element-local residual row, or -1 where discarded.

    Routing of the shuffled layout: in a fluid element, at a fluid-only node
    the momentum goes to the velocity slot and the mesh motion to the
    displacement slot; at an interface node the fluid momentum goes to the
    displacement slot (interface momentum) and the mesh-motion row is
    dropped.  In a solid element the momentum goes to the displacement slot
    and the kinematics to the velocity slot.  Pressure rows go to the copy of
    the element's material.
    """
    dim = mesh.dim
    ne = mesh.ne
    na = mesh.enodes.shape[1]
    cls = mesh.nclass[mesh.enodes]                            # (ne, na)
    tgt_mom = np.zeros((ne, dim, na), np.int64)
    tgt_aux = np.zeros((ne, dim, na), np.int64)
    for c in range(dim):
        dslot = mesh.d_dof(c, mesh.enodes)
        uslot = mesh.u_dof(c, mesh.enodes)
        fl = ~mesh.solid[:, None]
        tgt_mom[:, c, :] = np.where(fl, np.where(cls == FLUID, uslot, dslot), dslot)
        tgt_aux[:, c, :] = np.where(fl, np.where(cls == FLUID, dslot, -1), uslot)
    return np.concatenate([tgt_mom.reshape(ne, -1), tgt_aux.reshape(ne, -1), mesh.epdofs()], axis=1)


def assemble(mesh, spec, y, jacobian=True, h=1e-30, k_scale=1.0, y_prev=None):
    """Residual r(y) (Dirichlet rows y_j - g_j) and the exact Jacobian (CSR, FP64).

    The Jacobian of every element is obtained column by column by the complex
    step d r / d y_j = Im r(y + i h e_j) / h.  Only the structural couplings
    of `local_rows` are stored (values may be zero); Dirichlet rows become
    identity rows and Dirichlet columns are dropped.  `k_scale` multiplies
    the mesh-motion coefficient k = 1/V_el (used to evaluate k on another level).
    With y_prev (the state at t_n) the residual is that of one Crank-Nicolson
    step taken at the state y at t_{n+1} (element_residual_cn).
    """
    def local(Ue, solid):
        if y_prev is None:
            return element_residual(mesh, spec, Ue, solid, k_scale)
        return element_residual_cn(mesh, spec, Ue, y_prev[l2g[els]], solid, k_scale)

    flag, val = mesh.dirichlet(spec.u_peak)
    l2g = mesh.loc2glob()
    tgt = row_targets(mesh)
    nl = l2g.shape[1]
    r = np.zeros(mesh.ndof)
    rows, cols, vals = [], [], []
    for solid in (False, True):
        els = np.nonzero(mesh.solid == solid)[0]
        if els.size == 0:
            continue
        Ue = y[l2g[els]]
        mom, aux, pres = local(Ue, solid)
        Rl = np.concatenate([mom.reshape(len(els), -1), aux.reshape(len(els), -1), pres], axis=1)
        T = tgt[els]
        ok = T >= 0
        np.add.at(r, T[ok], Rl[ok])
        if not jacobian:
            continue
        Jl = np.zeros((len(els), nl, nl))
        Uc = Ue.astype(complex)
        for j in range(nl):
            Up = Uc.copy()
            Up[:, j] += 1j * h
            m2, a2, p2 = local(Up, solid)
            Jl[:, :, j] = np.concatenate([m2.reshape(len(els), -1), a2.reshape(len(els), -1), p2], axis=1).imag / h
        M = local_rows(mesh, solid, y_prev is not None)
        C = l2g[els]
        RR = np.broadcast_to(T[:, :, None], Jl.shape)
        CC = np.broadcast_to(C[:, None, :], Jl.shape)
        keep = M[None] & (RR >= 0)
        keep &= ~flag[np.maximum(RR, 0)] & ~flag[CC]
        rows.append(RR[keep])
        cols.append(CC[keep])
        vals.append(Jl[keep])
    r[flag] = y[flag] - val[flag]
    if not jacobian:
        return r, None
    dn = np.nonzero(flag)[0]
    rows.append(dn)
    cols.append(dn)
    vals.append(np.ones(dn.size))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.ndof, mesh.ndof)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return r, A
