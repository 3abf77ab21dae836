"""Newton's method and full multigrid for the steady system (checker; test
infrastructure, never called by the GPU solver path).

Section "Monolithic Newton-Krylov solver with Multigrid-Richardson-Schwarz
preconditioner": every nonlinear step linearises the monolithic residual
exactly (here the complex-step Jacobian of `fem.assemble`) and solves for the
correction; for steady problems the paper places the Newton iteration inside
full multigrid: Newton runs on a sequence of nested meshes, coarsest first,
each mesh started from the previous mesh's iterate carried over by the
prolongation.  Section "Details on the iterative solver": convergence at step
k when ||y^k - y^{k-1}||_2 < eps ||y^k||_2 with eps = 1e-8.

The linear solve of each step is a sparse direct solve: the Newton iterates
are those of an exact linear solve, against which the device's Krylov solves
(to a tight tolerance) are compared.
"""

import numpy as np
import scipy.sparse.linalg as sla

from . import fem, transfer


def newton(mesh, spec, y, tol=1e-8, max_steps=20, y_prev=None):
    """Exact Newton from y (not modified).  Returns (y, steps, converged,
    history of (||r||, ||e|| / ||y||) per step)."""
    y = np.array(y, dtype=np.float64, copy=True)
    hist = []
    for k in range(max_steps):
        r, J = fem.assemble(mesh, spec, y, y_prev=y_prev)
        e = sla.spsolve(J.tocsc(), -r)
        y += e
        en, yn = np.linalg.norm(e), np.linalg.norm(y)
        hist.append((float(np.linalg.norm(r)), float(en / yn)))
        if en <= tol * yn:
            return y, k + 1, True, hist
    return y, max_steps, False, hist


def cn_steps(mesh, spec, y0, nsteps, tol=1e-8, max_steps=20):
    """nsteps Crank-Nicolson steps from the state y0 (section "Discretization
    of the operator formulation"): each step's residual takes the current
    state as the state at t_n, and Newton from that state gives the state at
    t_{n+1}.  Returns (final state, per-step list of (steps, converged,
    history))."""
    y = np.array(y0, dtype=np.float64, copy=True)
    out = []
    for _ in range(nsteps):
        y_prev = y.copy()
        y, steps, conv, hist = newton(mesh, spec, y, tol=tol, max_steps=max_steps, y_prev=y_prev)
        out.append((steps, conv, hist))
    return y, out


def fmg(spec, coeffs, sizes, tol=1e-8, max_steps=20, seeded_base=True):
    """Full multigrid over the nested meshes `sizes` (coarsest first, each
    twice as fine per direction as the one before).  The coarsest mesh starts
    from its seeded state.  Every finer mesh starts from the previous mesh's
    iterate carried over by the prolongation P (zero columns at coarse
    Dirichlet dofs): with seeded_base, as s_j + P (y_{j-1} - s_{j-1}) with s
    the seeded states, whose difference vanishes on the coarse Dirichlet dofs,
    so no boundary data is lost; else as P y_{j-1}.  The fine Dirichlet dofs
    are then set to their values.  max_steps: one Newton step limit, or one
    per mesh; a mesh below the finest need not converge (its iterate only
    starts the next mesh).  Returns (finest y, per-mesh list of (steps,
    converged, history))."""
    meshes = [fem.Mesh(spec, tuple(s)) for s in sizes]
    caps = list(max_steps) if isinstance(max_steps, (list, tuple)) else [int(max_steps)] * len(meshes)
    out = []
    seeds = [fem.seeded_state(m, spec, coeffs) for m in meshes]
    y = seeds[0].copy()
    for j, mesh in enumerate(meshes):
        flag, val = mesh.dirichlet(spec.u_peak)
        if j > 0:
            cflag = meshes[j - 1].dirichlet(spec.u_peak)[0]
            P = transfer.prolongation(mesh, meshes[j - 1], flag, cflag)
            y = seeds[j] + P @ (y - seeds[j - 1]) if seeded_base else P @ y
            y[flag] = val[flag]
        y, steps, conv, hist = newton(mesh, spec, y, tol=tol, max_steps=caps[j])
        out.append((steps, conv, hist))
    return y, out
