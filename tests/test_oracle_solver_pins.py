"""Pins of the checker's smoother, V-cycle and restarted FGMRES.

Each test reduces a solver function to a case whose answer follows from the
algebra of the method alone, computed here with dense direct solves:

* Richardson with the exact inverse of J on the free dofs (one Schwarz block
  holding every free dof) contracts the error by (1 - omega) per sweep
  (section "Richardson-Schwarz smoother"), so nu sweeps from e = 0 give
  e = (1 - (1 - omega)^nu) J^{-1} r;
* with such exact smoothers on every smoothing level, the V-cycle (section
  "Geometric Multigrid preconditioner") obeys the recursion
  V_l(r) = x_l + q (P_l V_{l-1}(R_l r) - x_l), x_l = J_l^{-1} r,
  q = (1 - omega)^(nu_pre + nu_post), V_0 = J_0^{-1};
* the two-grid coarse correction I - P J_c^{-1} R J is a projection when
  J_c = R J P (Galerkin operators);
* restarted FGMRES with M = I reaches the dense solution, and its first cycle
  is the first cycle of an unrestarted run.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import problem, solver
from synth import config, fourier_coefficients


def _hier(name="c0_2d_16x4", **kw):
    s = config(name).with_(**kw)
    return problem.build(s, fourier_coefficients(s.dim, s.seed))


def _exact_block_level(lv, flag):
    """The level with one Schwarz block over all free dofs, every one owned."""
    free = np.nonzero(~flag)[0].astype(np.int32)
    one = solver.Level(J=lv.J, P=lv.P, R=lv.R, ptr=np.array([0, free.size]), dof=free,
                       owned=np.ones(free.size, np.uint8), kind=np.zeros(1, np.uint8))
    one.lu = [sla.lu_factor(solver.extract_block(lv.J, free))]
    return one


def _rhs(h, l, seed):
    r = np.random.default_rng(seed).standard_normal(h.levels[l].J.shape[0])
    r[h.flags[l]] = 0.0
    return r


@pytest.mark.parametrize("nu", [1, 2, 3])
def test_richardson_exact_block_contracts_by_one_minus_omega(nu):
    h = _hier()
    one = _exact_block_level(h.levels[-1], h.flags[-1])
    r = _rhs(h, len(h.levels) - 1, 11 + nu)
    x = np.linalg.solve(h.levels[-1].J.toarray(), r)
    omega = 0.7
    e = solver.smooth(one, r, np.zeros_like(r), nu, omega, first_zero=True)
    ref = (1.0 - (1.0 - omega) ** nu) * x
    assert np.linalg.norm(e - ref) <= 1e-9 * np.linalg.norm(ref)
    # the same sweeps started from a nonzero e: the error e - x contracts
    e0 = np.random.default_rng(3).standard_normal(r.size)
    e0[h.flags[-1]] = 0.0
    e = solver.smooth(one, r, e0, nu, omega, first_zero=False)
    ref = x + (1.0 - omega) ** nu * (e0 - x)
    assert np.linalg.norm(e - ref) <= 1e-9 * np.linalg.norm(ref)


def _recursive_reference(h, l, r, q):
    """V_l(r) of the recursion in the module docstring, by dense solves."""
    J = h.levels[l].J.toarray()
    if l == 0:
        return np.linalg.solve(J, r)
    x = np.linalg.solve(J, r)
    lv = h.levels[l]
    c = lv.P @ _recursive_reference(h, l - 1, lv.R @ r, q)
    return x + q * (c - x)


@pytest.mark.parametrize("name,levels,nu_pre,nu_post,omega", [
    ("c0_2d_16x4", 2, 1, 0, 1.0),      # exact pre-smoothing: the coarse residual is zero
    ("c0_2d_16x4", 2, 0, 1, 1.0),      # exact post-smoothing after the coarse correction
    ("c0_2d_16x4", 2, 2, 2, 0.7),
    ("c0_2d_16x4", 2, 1, 3, 0.7),
    ("c1_2d_128x32", 3, 2, 1, 0.7),    # 32x8, three levels: the recursion through a smoothed level
])
def test_vcycle_with_exact_smoothers_follows_recursion(name, levels, nu_pre, nu_post, omega):
    kw = {"levels": levels}
    if name == "c1_2d_128x32":
        kw.update(nx=32, ny=8, patch=2)
    h = _hier(name, **kw)
    for l in range(1, len(h.levels)):
        h.levels[l] = _exact_block_level(h.levels[l], h.flags[l])
    L = len(h.levels) - 1
    r = _rhs(h, L, 5)
    z = solver.vcycle(h.levels, L, r, nu_pre, nu_post, omega)
    q = (1.0 - omega) ** (nu_pre + nu_post)
    ref = _recursive_reference(h, L, r, q)
    assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)
    if q == 0.0:            # an exact smoothing sweep makes the cycle an exact solve
        x = np.linalg.solve(h.levels[L].J.toarray(), r)
        assert np.linalg.norm(z - x) <= 1e-9 * np.linalg.norm(x)


def test_two_grid_coarse_correction_is_a_projection():
    """E = I - P J_c^{-1} R J (the V-cycle without smoothing) satisfies E E = E
    and E P = 0: the coarse operator is the Galerkin product."""
    h = _hier()
    L = len(h.levels) - 1
    J = h.levels[L].J

    def E(v):
        return v - solver.vcycle(h.levels, L, J @ v, 0, 0, 0.7)

    rng = np.random.default_rng(8)
    v = rng.standard_normal(J.shape[0])
    v[h.flags[L]] = 0.0
    ev = E(v)
    assert np.linalg.norm(ev) > 1e-3 * np.linalg.norm(v)        # not trivially zero
    assert np.linalg.norm(E(ev) - ev) <= 1e-9 * np.linalg.norm(ev)
    vc = rng.standard_normal(h.levels[L - 1].J.shape[0])
    pv = h.levels[L].P @ vc
    assert np.linalg.norm(E(pv)) <= 1e-9 * np.linalg.norm(pv)


def _dense_system(n=40, seed=5):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.6
    b = rng.standard_normal(n)
    return A, b


def test_restarted_fgmres_reaches_dense_solution():
    A, b = _dense_system()
    xd = np.linalg.solve(A, b)
    x, info = solver.fgmres(sp.csr_matrix(A), b, lambda v: v.copy(), restart=5, rtol=1e-12, maxit=500)
    assert info.converged and info.restarts >= 3
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001
    # the first cycle is the first cycle of an unrestarted run
    _, full = solver.fgmres(sp.csr_matrix(A), b, lambda v: v.copy(), restart=60, rtol=1e-12, maxit=500)
    assert np.allclose(info.history[:6], full.history[:6], rtol=1e-12, atol=0)
    # each cycle starts from the true residual, which the previous cycle's last
    # estimate equals in exact arithmetic: the estimates never increase
    hist = np.array(info.history)
    assert np.all(np.diff(hist) <= 1e-10 * hist[0])


def test_fgmres_from_nonzero_start():
    """x0 = the exact solution: no iteration; x0 = a perturbed solution: the
    iterate solves the system and the initial residual is |b - A x0|."""
    A, b = _dense_system(seed=9)
    xd = np.linalg.solve(A, b)
    M = lambda v: v.copy()  # noqa: E731
    x, info = solver.fgmres(sp.csr_matrix(A), b, M, restart=5, rtol=1e-10, x0=xd)
    assert info.iters == 0 and info.converged
    x0 = xd + 0.1 * np.random.default_rng(1).standard_normal(xd.size)
    x, info = solver.fgmres(sp.csr_matrix(A), b, M, restart=5, rtol=1e-12, maxit=500, x0=x0)
    assert info.history[0] == pytest.approx(np.linalg.norm(b - A @ x0), rel=1e-13)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_fixed_iterations_run_exactly_that_many():
    A, b = _dense_system(seed=4)
    x, info = solver.fgmres(sp.csr_matrix(A), b, lambda v: v.copy(), restart=5, rtol=1e-12, fixed_iters=13)
    assert info.iters == 13 and info.restarts == 3


@pytest.mark.slow
def test_q1_pressure_box_smoother_fails_where_p1disc_converges():
    """Why the pressure space is the paper's P1disc: with a continuous Q1
    pressure per material the box-patch Richardson-Schwarz V-cycle does not
    precondition the system (FGMRES stalls), while with P1disc, whose pressure
    dofs belong to single elements, the same hierarchy converges quickly
    (section "Richardson-Schwarz smoother": with element-local pressure the
    blocks exchange only momentum and kinematic information).  64x16 mesh,
    three levels, 4x4-element blocks, nu = (2, 2), omega = 0.7."""
    res = {}
    for pres in ("q1", "p1disc"):
        h = _hier("c1_2d_128x32", nx=64, ny=16, levels=3, patch=4, pressure=pres)
        x, info = problem.solve(h, maxit=60)
        res[pres] = info
    assert not res["q1"].converged and res["q1"].true_relres > 0.5
    assert res["p1disc"].converged and res["p1disc"].iters <= 20


# ------------------------------------------------------------ paper mode: left GMRES
def _left_system(n=30, seed=12, pert=0.4):
    """A dense system and a dense preconditioner M^{-1} = (A + E)^{-1}."""
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.5
    E = rng.standard_normal((n, n)) * pert
    Minv = np.linalg.inv(A + E)
    b = rng.standard_normal(n)
    return A, Minv, b


def test_left_gmres_residuals_are_krylov_minima():
    """GMRES minimises |M^{-1}(b - A x)| over x0 + K_j(M^{-1} A, r0): each
    estimate equals the least-squares minimum over an orthonormal basis of
    the power basis [r0, B r0, ..., B^{j-1} r0], B = M^{-1} A, computed densely."""
    A, Minv, b = _left_system()
    B = Minv @ A
    r0 = Minv @ b
    for orth in ("cgs", "cgs2"):
        x, info = solver.gmres_left(sp.csr_matrix(A), b, lambda v: Minv @ v, restart=30, rtol=1e-12,
                                    fixed_iters=8, orth=orth)
        K = np.empty((b.size, 8))
        v = r0.copy()
        for j in range(8):
            K[:, j] = v
            v = B @ v
        for j in range(1, 9):
            Q, _ = np.linalg.qr(K[:, :j])
            y, *_ = np.linalg.lstsq(B @ Q, r0, rcond=None)
            rmin = np.linalg.norm(r0 - B @ Q @ y)
            assert info.history[j] == pytest.approx(rmin, rel=1e-8, abs=1e-13 * np.linalg.norm(r0))
        # the returned iterate attains the last minimum
        assert np.linalg.norm(Minv @ (b - A @ x)) == pytest.approx(info.history[8], rel=1e-8)


def test_left_gmres_stopping_rule_and_rate():
    """Exit when |M^{-1}(b - A x)| <= rtol |M^{-1} b| (x0 = 0), not one
    iteration earlier; rho = (r_N / r_0)^(1/N) of those norms; an exact
    preconditioner needs one iteration."""
    A, Minv, b = _left_system(seed=3)
    rtol = 1e-6
    x, info = solver.gmres_left(sp.csr_matrix(A), b, lambda v: Minv @ v, restart=10, rtol=rtol)
    r0 = np.linalg.norm(Minv @ b)
    rN = np.linalg.norm(Minv @ (b - A @ x))
    assert info.converged and rN <= rtol * r0 * 1.0001
    x1, i1 = solver.gmres_left(sp.csr_matrix(A), b, lambda v: Minv @ v, restart=10, rtol=rtol,
                               fixed_iters=info.iters - 1)
    assert np.linalg.norm(Minv @ (b - A @ x1)) > rtol * r0
    assert info.rho == pytest.approx((rN / r0) ** (1.0 / info.iters), rel=1e-6)
    assert info.true_relres == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b), rel=1e-10)
    Ainv = np.linalg.inv(A)
    _, ie = solver.gmres_left(sp.csr_matrix(A), b, lambda v: Ainv @ v, restart=10, rtol=1e-10)
    assert ie.iters == 1 and ie.converged


def test_left_gmres_restarts_reach_the_solution():
    A, Minv, b = _left_system(n=40, seed=8, pert=0.05)
    x, info = solver.gmres_left(sp.csr_matrix(A), b, lambda v: Minv @ v, restart=3, rtol=1e-12, maxit=400)
    xd = np.linalg.solve(A, b)
    assert info.converged and info.restarts >= 2
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("passes", ["cgs", "cgs2"])
def test_fgmres_one_and_two_gram_schmidt_passes_agree(passes):
    """In exact arithmetic one and two classical Gram-Schmidt passes give the
    same basis: on a well-conditioned system the histories agree."""
    A, b = _dense_system(seed=7)
    _, i1 = solver.fgmres(sp.csr_matrix(A), b, lambda v: v.copy(), restart=40, rtol=1e-12, orth=passes)
    _, i2 = solver.fgmres(sp.csr_matrix(A), b, lambda v: v.copy(), restart=40, rtol=1e-12, orth="cgs2")
    h1, h2 = np.array(i1.history), np.array(i2.history)
    assert h1.size == h2.size
    assert np.all(np.abs(h1 - h2) <= 1e-9 * h2[0])


def test_paper_mode_rate_trends():
    """Trends of Tables FSI_results_mg and FSI_results_pre_post in the paper's
    Krylov setting (left GMRES(10), one CGS pass, rtol 1e-4): the average
    convergence rate does not grow when the mesh is refined by one level
    (32x8 on two levels, 64x16 on three), and (4, 4) sweeps converge faster
    than (2, 2)."""
    rho = {}
    for (nx, ny, L) in ((32, 8, 2), (64, 16, 3)):
        for sw in ((2, 2), (4, 4)):
            h = _hier("c1_2d_128x32", nx=nx, ny=ny, levels=L, nu_pre=sw[0], nu_post=sw[1])
            x, info = problem.solve_paper(h)
            assert info.converged and info.est_relres <= 1e-4
            rho[(nx, sw)] = info.rho
    for sw in ((2, 2), (4, 4)):
        assert rho[(64, sw)] <= 1.1 * rho[(32, sw)]
    for nx in (32, 64):
        assert rho[(nx, (4, 4))] < rho[(nx, (2, 2))]
