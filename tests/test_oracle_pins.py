"""Pins of the FP64 checker against facts fixed by the paper and by mathematics.

Each test ties one part of the checker to something other than itself:
values printed in the paper (golden files with citations), closed-form
integrals, polynomial reproduction, finite differences, algebraic identities
and dense direct solves on small systems.
"""

import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fem, patches, problem, solver, transfer
from synth import ProblemSpec, config, fourier_coefficients

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    return rows


# ---------------------------------------------------------------- counts
def test_paper_unknown_table_3d():
    """Table number_of_unknowns, 3D: 6 N_Q2 + 4 E on the 8x2x2*2^(l-1) meshes."""
    for level, nx, ny, nz, n in _golden("paper_unknowns.txt"):
        assert patches.p1disc_unknowns(3, (nx, ny, nz)) == n
        if level <= 2:      # the checker's own numbering gives the same count
            s = ProblemSpec(dim=3, nx=nx, ny=ny, nz=nz)
            assert fem.Mesh(s, (nx, ny, nz)).ndof == n


def test_paper_block_sizes():
    """372 (2D, 16 elements) and 4630 (3D, 64 elements) dofs per Schwarz block."""
    for dim, p, m in _golden("paper_block_sizes.txt"):
        assert patches.closure_size(dim, p, "P1disc") == m
        n = (4 * p, 2 * p, 2 * p)[:dim]
        s = ProblemSpec(dim=dim, nx=n[0], ny=n[1], nz=n[2] if dim == 3 else 1, patch=p,
                        solid_lo=(9, 9, 9), solid_hi=(9.5, 9.5, 9.5))
        mesh = fem.Mesh(s, n)
        ptr, dof, owned, kind = patches.build_patches(mesh, p, np.zeros(mesh.ndof, bool))
        assert set(np.diff(ptr).tolist()) == {m}


def test_config_sizes():
    assert fem.Mesh(config("c0_2d_16x4"), (16, 4, 1)).ndof == 1380
    assert fem.Mesh(config("c1_2d_128x32"), (128, 32, 1)).ndof == 79108


# ------------------------------------------------------------ jacobian
@pytest.mark.parametrize("dim", [2, 3])
def test_jacobian_matches_finite_differences(dim):
    """Exact Jacobian = derivative of the residual (central differences), also
    at a state with a random displacement (shape-derivative blocks)."""
    if dim == 2:
        s = config("c0_2d_16x4")
        n = (16, 4, 1)
    else:
        s = ProblemSpec(dim=3, nx=8, ny=2, nz=2, patch=2)
        n = (8, 2, 2)
    mesh = fem.Mesh(s, n)
    y = fem.seeded_state(mesh, s, fourier_coefficients(dim, s.seed))
    flag, _ = mesh.dirichlet(s.u_peak)
    rng = np.random.default_rng(7)
    for with_d in (False, True):
        yy = y.copy()
        if with_d:
            dd = rng.standard_normal(mesh.ndof) * 1e-2
            dd[mesh.p_off:] = 0
            dd[2 * dim * mesh.N2 // 2:mesh.p_off] = 0   # displacement only
            dd[flag] = 0
            yy = yy + dd
        r, J = fem.assemble(mesh, s, yy)
        for _ in range(2):
            v = rng.standard_normal(mesh.ndof)
            v[flag] = 0
            v[mesh.p_off:] *= s.mu_s * 1e-3
            eps = 1e-6
            rp, _ = fem.assemble(mesh, s, yy + eps * v, jacobian=False)
            rm, _ = fem.assemble(mesh, s, yy - eps * v, jacobian=False)
            fd = (rp - rm) / (2 * eps)
            Jv = J @ v
            assert np.linalg.norm(fd - Jv) <= 1e-6 * np.linalg.norm(Jv)


def test_steady_zero_blocks():
    """Steady case (section "Structure of the Jacobian"): solid momentum does not
    depend on velocity, the solid kinematic rows do not depend on displacement."""
    s = config("c0_2d_16x4")
    mesh = fem.Mesh(s, (16, 4, 1))
    y = fem.seeded_state(mesh, s, fourier_coefficients(2, s.seed))
    _, J = fem.assemble(mesh, s, y)
    t = transfer.row_types(mesh)
    J = J.tocoo()
    ncol_u = (J.col >= 2 * mesh.N2) & (J.col < 4 * mesh.N2)
    ncol_d = J.col < 2 * mesh.N2
    assert not np.any((t[J.row] == transfer.SM) & ncol_u & (J.data != 0))
    assert not np.any((t[J.row] == transfer.KS) & ncol_d & (J.data != 0))
    # interface velocity rows receive no fluid contribution: no fluid pressure columns
    pcols = J.col >= mesh.p_off
    assert not np.any((t[J.row] == transfer.KS) & pcols)


# ------------------------------------------------ residual closed forms
def _raw_element_sums(mesh, s, y, solid):
    els = np.nonzero(mesh.solid == solid)[0]
    Ue = y[mesh.loc2glob()[els]]
    return els, fem.element_residual(mesh, s, Ue, solid)


def _node_sum(mesh, els, vec, nodes_mask, c):
    """Sum of element contributions vec[:, c, a] over local nodes a lying in nodes_mask."""
    tot = 0.0
    for i, e in enumerate(els):
        sel = nodes_mask[mesh.enodes[e]]
        tot += vec[i, c, sel].sum()
    return tot


def test_fluid_stress_and_ale_transform_closed_form():
    """Uniform shear u = (g y_hat, 0), pressure p0, on a mesh stretched by
    d = (a x_hat, 0): the Eulerian field is the same shear on the stretched
    channel.  Summing the momentum of the nodes of one face gives the face
    traction: right face -p0 * Ly, top face mu g (1 + a) Lx."""
    s = ProblemSpec(dim=2, nx=8, ny=4, solid_lo=(9, 9, 9), solid_hi=(9.5, 9.5, 9.5), rho=1000.0, mu=1.7)
    mesh = fem.Mesh(s, (8, 4, 1))
    g, p0, a = 0.3, 2.5, 0.2
    y = np.zeros(mesh.ndof)
    X = mesh.xnode
    y[mesh.d_dof(0, np.arange(mesh.N2))] = a * X[:, 0]
    y[mesh.u_dof(0, np.arange(mesh.N2))] = g * X[:, 1]
    y[mesh.epdofs()[:, 0]] = p0
    els, (mom, aux, pres) = _raw_element_sums(mesh, s, y, False)
    right = mesh.node_grid[:, 0] == mesh.g2[0] - 1
    top = mesh.node_grid[:, 1] == mesh.g2[1] - 1
    Lx, Ly = mesh.L
    # x momentum of the right-face nodes: traction sigma_xx * Ly = -p0 Ly
    fx_right = _node_sum(mesh, els, mom, right, 0)
    assert fx_right == pytest.approx(-p0 * Ly + 0.0, rel=1e-12)
    fx_top = _node_sum(mesh, els, mom, top, 0)
    assert fx_top == pytest.approx(s.mu * g * (1 + a) * Lx, rel=1e-12)
    # continuity: div u = 0 for a shear
    assert np.abs(pres).max() < 1e-12


def test_fluid_convection_closed_form():
    """u = (x, -y) (divergence free, (u.grad)u = (x, y)), no pressure, d = 0:
    the momentum summed over all test functions (partition of unity) equals
    rho * int (x, y) = rho * (Lx^2 Ly / 2, Lx Ly^2 / 2)."""
    s = ProblemSpec(dim=2, nx=8, ny=4, solid_lo=(9, 9, 9), solid_hi=(9.5, 9.5, 9.5))
    mesh = fem.Mesh(s, (8, 4, 1))
    y = np.zeros(mesh.ndof)
    X = mesh.xnode
    y[mesh.u_dof(0, np.arange(mesh.N2))] = X[:, 0]
    y[mesh.u_dof(1, np.arange(mesh.N2))] = -X[:, 1]
    els, (mom, aux, pres) = _raw_element_sums(mesh, s, y, False)
    Lx, Ly = mesh.L
    assert mom[:, 0, :].sum() == pytest.approx(s.rho * Lx ** 2 * Ly / 2, rel=1e-12)
    assert mom[:, 1, :].sum() == pytest.approx(s.rho * Lx * Ly ** 2 / 2, rel=1e-12)
    assert abs(pres[:, 0].sum()) < 1e-10


def test_fluid_continuity_and_ale_closed_form():
    """u = (x, 0): sum over elements of the constant-pressure continuity rows
    = int div u = |Omega|.  d linear: harmonic mesh-motion residual vanishes
    at nodes whose test functions vanish on the boundary."""
    s = ProblemSpec(dim=2, nx=8, ny=4, solid_lo=(9, 9, 9), solid_hi=(9.5, 9.5, 9.5))
    mesh = fem.Mesh(s, (8, 4, 1))
    y = np.zeros(mesh.ndof)
    X = mesh.xnode
    y[mesh.u_dof(0, np.arange(mesh.N2))] = X[:, 0]
    els, (mom, aux, pres) = _raw_element_sums(mesh, s, y, False)
    assert pres[:, 0].sum() == pytest.approx(np.prod(mesh.L), rel=1e-12)
    y2 = np.zeros(mesh.ndof)
    y2[mesh.d_dof(0, np.arange(mesh.N2))] = 0.01 * X[:, 0] + 0.02 * X[:, 1]
    y2[mesh.d_dof(1, np.arange(mesh.N2))] = -0.03 * X[:, 0]
    r, _ = fem.assemble(mesh, s, y2, jacobian=False)
    on_bnd, _, _ = mesh.boundary_masks()
    interior = np.nonzero(~on_bnd)[0]
    for c in range(2):
        assert np.abs(r[mesh.d_dof(c, interior)]).max() < 1e-12


def test_solid_piola_closed_form():
    """Solid-only mesh, homogeneous isochoric stretch F = diag(l, 1/l), pressure p:
    incompressibility residual is 0 and the momentum summed over the right-face
    nodes is the traction P_xx Ly with P = J sigma F^{-T},
    sigma = -p I + mu_s F F^T: P_xx = (-p + mu_s l^2) / l."""
    s = ProblemSpec(dim=2, nx=4, ny=4, lx=1.0, ly=1.0, solid_lo=(-1, -1, -1), solid_hi=(2, 2, 2), mu_s=3.0e4)
    mesh = fem.Mesh(s, (4, 4, 1))
    lam, p = 1.1, 123.0
    X = mesh.xnode
    y = np.zeros(mesh.ndof)
    y[mesh.d_dof(0, np.arange(mesh.N2))] = (lam - 1.0) * X[:, 0]
    y[mesh.d_dof(1, np.arange(mesh.N2))] = (1.0 / lam - 1.0) * X[:, 1]
    y[mesh.epdofs()[:, 0]] = p
    els, (mom, aux, pres) = _raw_element_sums(mesh, s, y, True)
    assert np.abs(pres).max() < 1e-12
    right = mesh.node_grid[:, 0] == mesh.g2[0] - 1
    Pxx = (-p + s.mu_s * lam ** 2) / lam
    assert _node_sum(mesh, els, mom, right, 0) == pytest.approx(Pxx * mesh.L[1], rel=1e-12)
    top = mesh.node_grid[:, 1] == mesh.g2[1] - 1
    Pyy = (-p + s.mu_s / lam ** 2) * lam
    assert _node_sum(mesh, els, mom, top, 1) == pytest.approx(Pyy * mesh.L[0], rel=1e-12)
    # kinematics: sum over test functions of (u, phi) = |Omega_s| * u
    y[mesh.u_dof(1, np.arange(mesh.N2))] = 0.7
    els, (mom, aux, pres) = _raw_element_sums(mesh, s, y, True)
    assert aux[:, 1, :].sum() == pytest.approx(0.7 * 1.0, rel=1e-12)


def test_poiseuille_is_discrete_solution():
    """Poiseuille flow u = U 4 y (1 - y), p = -8 U mu x is exact in Q2/P1disc and
    solves steady Navier-Stokes: the residual vanishes at interior nodes."""
    s = ProblemSpec(dim=2, nx=8, ny=4, solid_lo=(9, 9, 9), solid_hi=(9.5, 9.5, 9.5), mu=1.3)
    mesh = fem.Mesh(s, (8, 4, 1))
    U = 0.4
    X = mesh.xnode
    y = np.zeros(mesh.ndof)
    y[mesh.u_dof(0, np.arange(mesh.N2))] = U * 4 * X[:, 1] * (1 - X[:, 1])
    ep = mesh.epdofs()
    xc = (mesh.eidx[:, 0] + 0.5) * mesh.h[0]
    y[ep[:, 0]] = -8 * U * s.mu * xc
    y[ep[:, 1]] = -8 * U * s.mu * mesh.h[0] / 2
    r, _ = fem.assemble(mesh, s, y, jacobian=False)
    on_bnd, _, _ = mesh.boundary_masks()
    interior = np.nonzero(~on_bnd)[0]
    for c in range(2):
        assert np.abs(r[mesh.u_dof(c, interior)]).max() < 1e-11
    assert np.abs(r[mesh.p_off:]).max() < 1e-12


# ------------------------------------------------------------ transfers
@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_reproduces_polynomials(dim):
    """Natural injection: Q2 (d, u) and P1disc (p) polynomials are reproduced exactly."""
    if dim == 2:
        s = ProblemSpec(dim=2, nx=8, ny=4)
        nf, nc = (8, 4, 1), (4, 2, 1)
    else:
        s = ProblemSpec(dim=3, nx=8, ny=4, nz=4)
        nf, nc = (8, 4, 4), (4, 2, 2)
    F, C = fem.Mesh(s, nf), fem.Mesh(s, nc)
    P = transfer.prolongation(F, C, np.zeros(F.ndof, bool), np.zeros(C.ndof, bool))
    rng = np.random.default_rng(3)
    for _ in range(3):
        co = rng.standard_normal(8)

        def q2(X):
            x, y = X[:, 0], X[:, 1]
            z = X[:, 2] if dim == 3 else 0 * x
            return co[0] + co[1] * x + co[2] * y * x + co[3] * x * x * y * y + co[4] * z * x * x + co[5] * y * y

        vc = np.zeros(C.ndof)
        vf_exact = np.zeros(F.ndof)
        for f in range(2 * dim):
            vc[f * C.N2:(f + 1) * C.N2] = (f + 1) * q2(C.xnode)
            vf_exact[f * F.N2:(f + 1) * F.N2] = (f + 1) * q2(F.xnode)

        def lin(M):
            xc = (M.eidx + 0.5) * np.array(M.h)
            out = np.zeros((M.ne, dim + 1))
            out[:, 0] = co[6] + xc @ co[1:1 + dim]
            for d in range(dim):
                out[:, 1 + d] = co[1 + d] * M.h[d] / 2
            return out.ravel()

        vc[C.p_off:] = lin(C)
        vf_exact[F.p_off:] = lin(F)
        vf = P @ vc
        assert np.max(np.abs(vf - vf_exact)) <= 1e-13 * np.max(np.abs(vf_exact))


def _linear_state(mesh, s):
    y = np.zeros(mesh.ndof)
    y[mesh.solid_pressure_dofs()] = s.mu_s
    return y


@pytest.mark.parametrize("dim", [2, 3])
def test_galerkin_equals_coarse_assembly(dim):
    """R J_fine P equals the coarse Jacobian assembled directly at the linear
    state (u = 0, d = 0, stress-free solid), with the mesh-motion coefficient
    evaluated on the fine level: the restriction respects the shuffled rows."""
    if dim == 2:
        s = config("c0_2d_16x4")
        nf, nc = (16, 4, 1), (8, 2, 1)
    else:
        s = ProblemSpec(dim=3, nx=16, ny=4, nz=4, patch=2)
        nf, nc = (16, 4, 4), (8, 2, 2)      # solid box element-aligned on both
    F, C = fem.Mesh(s, nf), fem.Mesh(s, nc)
    assert F.solid.any() and C.solid.any()
    ff, fc = F.dirichlet(s.u_peak)[0], C.dirichlet(s.u_peak)[0]
    _, Jf = fem.assemble(F, s, _linear_state(F, s))
    _, Jc = fem.assemble(C, s, _linear_state(C, s), k_scale=2.0 ** dim)
    P = transfer.prolongation(F, C, ff, fc)
    R = transfer.restriction(F, C, ff, fc)
    G = transfer.galerkin(R, Jf, P, fc)
    D = (G - Jc).tocsr()
    scale = np.abs(Jc).max(axis=1).toarray().ravel()
    rowmax = np.abs(D).max(axis=1).toarray().ravel()
    assert np.all(rowmax <= 1e-12 * np.maximum(scale, 1e-300))


def test_restriction_is_not_plain_transpose_at_interface():
    """Coarse interface rows restrict solid kinematics only and gather the
    fine fluid momentum stored in velocity slots (shuffled layout)."""
    s = config("c0_2d_16x4")
    F, C = fem.Mesh(s, (16, 4, 1)), fem.Mesh(s, (8, 2, 1))
    ff, fc = F.dirichlet(s.u_peak)[0], C.dirichlet(s.u_peak)[0]
    P = transfer.prolongation(F, C, ff, fc)
    R = transfer.restriction(F, C, ff, fc)
    D = (R - P.T).tocoo()
    D.eliminate_zeros()
    tc = transfer.row_types(C)
    assert D.nnz > 0
    assert set(np.unique(tc[D.row]).tolist()) <= {transfer.IM, transfer.KS}


# ------------------------------------------------------------ patches
def test_patches_partition_and_order():
    s = config("c1_2d_128x32").with_(nx=32, ny=8)
    mesh = fem.Mesh(s, (32, 8, 1))
    flag = mesh.dirichlet(s.u_peak)[0]
    ptr, dof, owned, kind = patches.build_patches(mesh, 4, flag)
    cnt = np.zeros(mesh.ndof, int)
    np.add.at(cnt, dof[owned.astype(bool)], 1)
    assert np.all(cnt[~flag] == 1) and np.all(cnt[flag] == 0)
    assert np.all(np.diff(kind.astype(int)) <= 0)          # solid blocks first
    for k in range(len(ptr) - 1):
        d = dof[ptr[k]:ptr[k + 1]]
        assert np.all(np.diff(d) > 0)
    # interface displacement/velocity dofs are owned by solid blocks
    iface = np.nonzero(mesh.nclass == fem.IFACE)[0]
    sel = owned.astype(bool) & np.isin(dof, mesh.u_dof(0, iface))
    owner = np.searchsorted(ptr, np.nonzero(sel)[0], side="right") - 1
    assert np.all(kind[owner] == 1)


# ------------------------------------------------------------ solvers
def test_lu_properties():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((60, 60))
    lu, piv = sla.lu_factor(A)
    L = np.tril(lu, -1) + np.eye(60)
    U = np.triu(lu)
    PA = A.copy()
    for i, p in enumerate(piv):
        PA[[i, p]] = PA[[p, i]]
    assert np.abs(L).max() <= 1.0
    assert np.linalg.norm(PA - L @ U) <= 60 * 2.2e-16 * np.linalg.norm(A) * 10
    x = rng.standard_normal(60)
    assert np.allclose(sla.lu_solve((lu, piv), A @ x), x, rtol=1e-10)


def _small_hierarchy(**kw):
    s = config("c0_2d_16x4").with_(**kw)
    return problem.build(s, fourier_coefficients(2, s.seed))


def test_single_subdomain_smoother_is_exact():
    """One block holding every free dof, omega = 1: one Richardson-RAS sweep
    from e = 0 gives e = J^{-1} r (the block is the whole free operator)."""
    h = _small_hierarchy()
    lv = h.levels[-1]
    flag = h.flags[-1]
    free = np.nonzero(~flag)[0].astype(np.int32)
    one = solver.Level(J=lv.J, ptr=np.array([0, free.size]), dof=free,
                       owned=np.ones(free.size, np.uint8), kind=np.zeros(1, np.uint8))
    one.lu = [sla.lu_factor(solver.extract_block(lv.J, free))]
    rng = np.random.default_rng(2)
    r = rng.standard_normal(lv.J.shape[0])
    r[flag] = 0
    e = solver.smooth(one, r, np.zeros_like(r), 1, 1.0, first_zero=True)
    x = np.linalg.solve(lv.J.toarray(), r)
    assert np.linalg.norm(e - x) <= 1e-8 * np.linalg.norm(x)


def test_vcycle_is_linear():
    h = _small_hierarchy()
    M = problem.preconditioner(h)
    rng = np.random.default_rng(4)
    n = h.b.size
    r1, r2 = rng.standard_normal(n), rng.standard_normal(n)
    z = M(2.0 * r1 - 3.0 * r2)
    zz = 2.0 * M(r1) - 3.0 * M(r2)
    assert np.linalg.norm(z - zz) <= 1e-12 * np.linalg.norm(zz)


def test_fgmres_identity_preconditioner_matches_dense_solve():
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, info = solver.fgmres(sp.csr_matrix(A), b, lambda v: v.copy(), restart=n + 5, rtol=1e-13)
    assert info.converged
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)
    assert abs(info.true_relres - info.est_relres) <= 1e-12 + 1e-3 * info.true_relres
    h = np.array(info.history)
    assert np.all(np.diff(h[1:]) <= 1e-12 * h[0])


def test_fgmres_exact_preconditioner_one_iteration():
    rng = np.random.default_rng(6)
    n = 30
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.2
    b = rng.standard_normal(n)
    Ainv = np.linalg.inv(A)
    x, info = solver.fgmres(sp.csr_matrix(A), b, lambda v: Ainv @ v, restart=10, rtol=1e-10)
    assert info.iters == 1 and info.converged


def test_mg_fgmres_solves_config0():
    h = _small_hierarchy()
    x, info = problem.solve(h)
    assert info.converged and info.true_relres <= 1e-10
    xd = np.linalg.solve(h.levels[-1].J.toarray(), h.b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_more_sweeps_fewer_iterations():
    """Trend of Table FSI_results_pre_post: more smoothing, fewer Krylov steps."""
    a = problem.solve(_small_hierarchy(nu_pre=1, nu_post=1))[1].iters
    b = problem.solve(_small_hierarchy(nu_pre=4, nu_post=4))[1].iters
    assert b < a
