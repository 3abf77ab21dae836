"""The Galerkin coarse operators on the device (fsi_mg_galerkin; section
"Geometric Multigrid preconditioner"): recomputed from the finest values they
equal the builder's R J P, and a new Newton Jacobian of the same sparsity
needs only its finest values (set, Galerkin, refactor) to solve as the
system built for it on the host does."""

import sys

import numpy as np
import pytest

from gpu_common import csr_of, dev, host

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(**kw):
    from paper_1709_05660_amd import Problem
    from synth import config, fourier_coefficients
    s = config("c1_2d_128x32").with_(**kw)
    return Problem(s, fourier_coefficients(2, s.seed))


def _coarse_products_match(mg, p, tol=1e-12):
    """Every level's J x on the device against the host CSR of p, per entry
    within tol (|J| |x|)."""
    rng = np.random.default_rng(31)
    for l in range(p.nlevels - 1):
        A = csr_of(p, l)
        x = rng.standard_normal(A.shape[1])
        y = host(mg.apply(l, 0, dev(x)))
        bound = tol * (abs(A) @ abs(x)) + 1e-300
        err = np.abs(y - A @ x)
        _say(f"  level {l}: max err / bound {float(np.max(err / bound)):.3f}")
        assert np.all(err <= bound)


def _scipy_galerkin(p, finest):
    """The plain definition, independent of both builders' SpGEMM: per level
    A_{l-1} = R_l A_l P_l by scipy's sparse products, then unit diagonals on
    the coarse Dirichlet rows (zero rows and columns there otherwise); with
    |R| |A| |P| alongside, the scale of each product's rounding."""
    import scipy.sparse as sp
    ops, absops = {p.nlevels - 1: finest}, {p.nlevels - 1: abs(finest)}
    for l in range(p.nlevels - 1, 0, -1):
        R, P = csr_of(p, l, "R"), csr_of(p, l, "P")
        A = (R @ ops[l] @ P).tocsr()
        flags = p.dirichlet(l - 1).astype(bool)
        keep = sp.diags((~flags).astype(float))
        ops[l - 1] = (keep @ A + sp.diags(flags.astype(float))).tocsr()
        absops[l - 1] = (abs(R) @ absops[l] @ abs(P) + sp.diags(flags.astype(float))).tocsr()
    return ops, absops


def test_galerkin_of_a_new_jacobian_equals_the_sparse_products():
    """A different Jacobian of the same sparsity (another material, inflow and
    seed) set as the finest values of a handle built for the first system's
    time step: every coarse operator the device computes equals R J P by plain
    sparse products within 1e-13 of |R| |J| |P| |x|."""
    from paper_1709_05660_amd import MG
    p0 = _problem(nx=64, ny=16, levels=3, transient=True)
    p1 = _problem(nx=64, ny=16, levels=3, transient=True, mu_s=2.0e5, u_peak=0.3, seed=5)
    f0, f1 = csr_of(p0, p0.nlevels - 1), csr_of(p1, p1.nlevels - 1)
    assert np.array_equal(f0.indptr, f1.indptr) and np.array_equal(f0.indices, f1.indices)
    mg = MG(p0, precision="fp64")
    mg.set_jvalues(p0.nlevels - 1, dev(f1.data))
    mg.galerkin()
    ops, absops = _scipy_galerkin(p0, f1)
    rng = np.random.default_rng(17)
    for l in range(p0.nlevels - 1):
        x = rng.standard_normal(ops[l].shape[1])
        y = host(mg.apply(l, 0, dev(x)))
        bound = 1e-13 * (absops[l] @ np.abs(x)) + 1e-300
        err = np.abs(y - ops[l] @ x)
        _say(f"  level {l}: max err / bound {float(np.max(err / bound)):.3f}")
        assert np.all(err <= bound)
    mg.close()


def test_galerkin_reproduces_the_builders_coarse_operators():
    from paper_1709_05660_amd import MG
    p = _problem(nx=64, ny=16, levels=3)
    mg = MG(p, precision="fp64")
    mg.galerkin()
    _coarse_products_match(mg, p)
    mg.galerkin()                     # again: the patterns are prepared once
    _coarse_products_match(mg, p)
    mg.close()


@pytest.mark.parametrize("transient", [False, True])
def test_new_newton_jacobian_from_its_finest_values(transient):
    from paper_1709_05660_amd import MG
    p0 = _problem(transient=transient)
    p1 = _problem(transient=transient, mu_s=2.0e5, u_peak=0.3, seed=99)
    f0, f1 = csr_of(p0, p0.nlevels - 1), csr_of(p1, p1.nlevels - 1)
    assert np.array_equal(f0.indptr, f1.indptr) and np.array_equal(f0.indices, f1.indices)
    mg = MG(p0, precision="fp64", use_graph=True)
    b = dev(p1.b)
    mg.fgmres(b, rtol=1e-10)           # a solve of the old system first (graphs captured)
    mg.set_jvalues(p0.nlevels - 1, dev(f1.data))
    mg.galerkin()
    mg.refactor()
    _coarse_products_match(mg, p1)
    x, info = mg.fgmres(b, rtol=1e-10)
    ref = MG(p1, precision="fp64", use_graph=True)
    xr, ir = ref.fgmres(b, rtol=1e-10)
    x, xr = host(x), host(xr)
    rel = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
    _say(f"transient {transient}: iters {info['iters']} vs {ir['iters']}, rel diff {rel:.2e}")
    assert info["converged"] == 1 and abs(info["iters"] - ir["iters"]) <= 1
    assert rel <= 1e-10
    mg.close()
    ref.close()


def test_new_newton_jacobian_mixed_form():
    from paper_1709_05660_amd import MG
    p0 = _problem(nx=64, ny=16, levels=3)
    p1 = _problem(nx=64, ny=16, levels=3, mu_s=3.0e4, u_peak=0.15, seed=7)
    mg = MG(p0, precision="bf16")
    mg.set_jvalues(p0.nlevels - 1, dev(csr_of(p1, p1.nlevels - 1).data))
    mg.galerkin()
    mg.refactor()
    x, info = mg.fgmres(dev(p1.b), rtol=1e-8)
    x = host(x)
    J = csr_of(p1, p1.nlevels - 1)
    relres = float(np.linalg.norm(p1.b - J @ x) / np.linalg.norm(p1.b))
    _say(f"mixed: iters {info['iters']} host relres {relres:.2e}")
    assert info["converged"] == 1 and relres <= 1e-8 * 1.001
    mg.close()
