"""Pins of the checker's Crank-Nicolson step (section "Discretization of the
operator formulation": the time-discretized operators F_n and S_n).

* The Jacobian is the derivative of the CN residual in the state at t_{n+1}
  (central differences, 2D and 3D, at a state that moves the mesh).
* At rest (the state at t_{n+1} equal to the one at t_n) the mesh velocity
  and every time difference vanish and the averaged terms add up: the CN
  residual is the steady residual, row by row.
* Closed forms of the time-difference terms: a uniform velocity increment c
  of a fluid at rest gives momentum rows summing to (rho / dt) c |Omega|; a
  uniform solid velocity gives (rho_s / dt) c |Omega_s| (stress-free solid);
  a uniform displacement increment delta gives kinematic rows summing to
  -(delta / dt) |Omega_s|.
* The blocks that vanish in the steady case (solid momentum on the velocity,
  solid kinematics on the displacement, section "Structure of the
  Jacobian") are present in the CN Jacobian.
"""

import numpy as np
import pytest

from oracle import fem, problem, transfer
from synth import ProblemSpec, config, fourier_coefficients


def _mesh_states(dim):
    if dim == 2:
        s = config("c5_2d_16x4_cn")
        n = (16, 4, 1)
    else:
        s = ProblemSpec(dim=3, nx=8, ny=2, nz=2, patch=2, transient=True)
        n = (8, 2, 2)
    mesh = fem.Mesh(s, n)
    y0, y1 = fem.transient_states(mesh, s, fourier_coefficients(dim, s.seed))
    return s, mesh, y0, y1


@pytest.mark.parametrize("dim", [2, 3])
def test_cn_jacobian_matches_finite_differences(dim):
    s, mesh, y0, y1 = _mesh_states(dim)
    assert np.abs(y1 - y0).max() > 0                       # the mesh moves in the step
    flag, _ = mesh.dirichlet(s.u_peak)
    r, J = fem.assemble(mesh, s, y1, y_prev=y0)
    rng = np.random.default_rng(12)
    for _ in range(2):
        v = rng.standard_normal(mesh.ndof)
        v[flag] = 0
        v[mesh.p_off:] *= s.mu_s * 1e-3
        eps = 1e-6
        rp, _ = fem.assemble(mesh, s, y1 + eps * v, jacobian=False, y_prev=y0)
        rm, _ = fem.assemble(mesh, s, y1 - eps * v, jacobian=False, y_prev=y0)
        fd = (rp - rm) / (2 * eps)
        Jv = J @ v
        assert np.linalg.norm(fd - Jv) <= 1e-6 * np.linalg.norm(Jv)


@pytest.mark.parametrize("dim", [2, 3])
def test_cn_at_rest_is_the_steady_residual(dim):
    s, mesh, y0, y1 = _mesh_states(dim)
    for y in (y0, y1):
        rs, _ = fem.assemble(mesh, s, y, jacobian=False)
        rc, _ = fem.assemble(mesh, s, y, jacobian=False, y_prev=y)
        # rounding of the stress-free solid's cancelling terms (mu_s = 5e5) is
        # about 1e-13; a wrong factor or sign would show at O(0.1)
        assert np.max(np.abs(rc - rs)) <= 1e-12 * max(1.0, np.max(np.abs(rs)))


def _sum_rows(mesh, s, y, y_prev, solid, part, c):
    els = np.nonzero(mesh.solid == solid)[0]
    l2g = mesh.loc2glob()[els]
    mom, aux, pres = fem.element_residual_cn(mesh, s, y[l2g], y_prev[l2g], solid)
    return (mom if part == "mom" else aux)[:, c, :].sum()


def test_cn_time_difference_closed_forms():
    dt = 0.02
    fl = ProblemSpec(dim=2, nx=8, ny=4, solid_lo=(9, 9, 9), solid_hi=(9.5, 9.5, 9.5), transient=True, dt=dt)
    mesh = fem.Mesh(fl, (8, 4, 1))
    nodes = np.arange(mesh.N2)
    y0 = np.zeros(mesh.ndof)
    y1 = np.zeros(mesh.ndof)
    c = (0.3, -0.7)
    for k in range(2):
        y1[mesh.u_dof(k, nodes)] = c[k]
    area = float(np.prod(mesh.L))
    for k in range(2):
        assert _sum_rows(mesh, fl, y1, y0, False, "mom", k) == pytest.approx(fl.rho / dt * c[k] * area, rel=1e-12)
    so = ProblemSpec(dim=2, nx=4, ny=4, lx=1.0, ly=1.0, solid_lo=(-1, -1, -1), solid_hi=(2, 2, 2),
                     transient=True, dt=dt, rho_s=1700.0, mu_s=2.0e4)
    mesh = fem.Mesh(so, (4, 4, 1))
    nodes = np.arange(mesh.N2)
    y0 = np.zeros(mesh.ndof)
    y0[mesh.solid_pressure_dofs()] = so.mu_s          # stress-free at d = 0
    y1 = y0.copy()
    for k in range(2):
        y1[mesh.u_dof(k, nodes)] = c[k]
    for k in range(2):
        assert _sum_rows(mesh, so, y1, y0, True, "mom", k) == pytest.approx(so.rho_s / dt * c[k], rel=1e-12)
        # kinematics at a uniform velocity and no displacement increment: (u1 + u0)/2 = c / 2
        assert _sum_rows(mesh, so, y1, y0, True, "aux", k) == pytest.approx(0.5 * c[k], rel=1e-12)
    y2 = y0.copy()
    delta = (2e-3, -1e-3)
    for k in range(2):
        y2[mesh.d_dof(k, nodes)] = delta[k]
    for k in range(2):
        assert _sum_rows(mesh, so, y2, y0, True, "aux", k) == pytest.approx(-delta[k] / dt, rel=1e-12)


def test_cn_transient_blocks_are_present():
    s, mesh, y0, y1 = _mesh_states(2)
    _, Jc = fem.assemble(mesh, s, y1, y_prev=y0)
    _, Js = fem.assemble(mesh, s, y1)
    t = transfer.row_types(mesh)
    ucols = lambda A: (A.col >= 2 * mesh.N2) & (A.col < 4 * mesh.N2)   # noqa: E731
    dcols = lambda A: A.col < 2 * mesh.N2                              # noqa: E731
    for J, present in ((Jc.tocoo(), True), (Js.tocoo(), False)):
        su = np.any((t[J.row] == transfer.SM) & ucols(J) & (J.data != 0))
        kd = np.any((t[J.row] == transfer.KS) & dcols(J) & (J.data != 0))
        assert su == present and kd == present


def test_cn_multigrid_solve():
    """MG-FGMRES on the CN step of the 16x4 system reaches the dense solution."""
    s = config("c5_2d_16x4_cn")
    h = problem.build(s, fourier_coefficients(2, s.seed))
    x, info = problem.solve(h)
    assert info.converged and info.true_relres <= s.rtol
    xd = np.linalg.solve(h.levels[-1].J.toarray(), h.b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
