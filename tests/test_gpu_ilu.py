"""GPU parity of the ILU(0) local solves of the fluid blocks (fluid_ilu;
section "Richardson-Schwarz smoother"): one Schwarz application against the
checker's ILU(0) solves on the same matrices, the V-cycle, and FGMRES on the
time step and on the steady system against the checker's own hierarchy
(fixed-iteration protocol, 1e-10), FP64 and the mixed forms."""

import sys

import numpy as np
import pytest

from gpu_common import csr_of, dev, host, oracle_hierarchy, oracle_on_product, product_problem
from oracle import problem as oprob
from oracle import solver as osolver

pytestmark = pytest.mark.gpu

MIXED_ERR_BOUND = 1e-7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["c5_2d_16x4_cn", "c0_2d_16x4"])
def test_ilu_schwarz_and_vcycle_match_checker(name):
    from paper_1709_05660_amd import MG
    p = product_problem(name)
    oh = oracle_on_product(name, fluid_ilu=True)
    s = oh.spec
    mg = MG(p, precision="fp64", fluid_ilu=True)
    rng = np.random.default_rng(21)
    for l in range(1, p.nlevels):
        assert any(isinstance(f[0], str) for f in oh.levels[l].lu)
        r = rng.standard_normal(csr_of(p, l).shape[0])
        y = host(mg.apply(l, 4, dev(r)))
        ref = osolver.ras(oh.levels[l], r)
        _say(f"{name} level {l} Schwarz (ILU fluid) rel diff {_rel(y, ref):.2e}")
        assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    r = rng.standard_normal(p.n)
    z = host(mg.vcycle(dev(r)))
    ref = osolver.vcycle(oh.levels, len(oh.levels) - 1, r, s.nu_pre, s.nu_post, s.omega)
    _say(f"{name} V-cycle (ILU fluid) rel diff {_rel(z, ref):.2e}")
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)   # the V-cycle parity bound
    mg.close()


@pytest.mark.parametrize("name,fixed", [("c5_2d_16x4_cn", None), ("c4_2d_128x32_cn", None),
                                        ("c0_2d_16x4", 60)])
def test_ilu_fgmres_parity(name, fixed):
    """FP64 with ILU(0) fluid blocks: the iterate after the checker's
    iteration count (or a fixed 60 for the slow steady case, over two
    restarts) equals the checker's to 1e-10; converged counts within one."""
    from paper_1709_05660_amd import MG
    p = product_problem(name)
    oh = oracle_hierarchy(name, fluid_ilu=True)
    s = oh.spec
    if fixed is None:
        x_o, io = oprob.solve(oh)
        k = io.iters
    else:
        k = fixed
    x_fix, _ = oprob.solve(oh, fixed_iters=k)
    mg = MG(p, precision="fp64", fluid_ilu=True, use_graph=True)
    b = dev(p.b)
    xg, ig = mg.fgmres(b, rtol=s.rtol, fixed_iters=k)
    rel = _rel(host(xg), x_fix)
    _say(f"{name} ILU fluid: iters {k} fixed rel diff {rel:.2e}")
    assert rel <= 1e-10
    if fixed is None:
        x2, i2 = mg.fgmres(b, rtol=s.rtol)
        x2 = host(x2)
        assert i2["converged"] == 1 and abs(i2["iters"] - k) <= 1
        assert _rel(x2, x_o) <= 1e-8
    mg.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_ilu_mixed_time_step_against_checker(prec):
    from paper_1709_05660_amd import MG
    name = "c4_2d_128x32_cn"
    p = product_problem(name)
    oh = oracle_hierarchy(name)
    x_o, _ = oprob.solve(oh)
    mg = MG(p, precision=prec, fluid_ilu=True)
    x, info = mg.fgmres(dev(p.b), rtol=1e-8)
    x = host(x)
    J = csr_of(p, p.nlevels - 1)
    relres = float(np.linalg.norm(p.b - J @ x) / np.linalg.norm(p.b))
    err = _rel(x, x_o)
    _say(f"{name} {prec} ILU fluid: iters {info['iters']} host relres {relres:.2e} err {err:.2e}")
    assert info["converged"] == 1 and relres <= 1e-8 * 1.001
    assert err <= MIXED_ERR_BOUND
    mg.close()


def test_ilu_3d_blocks_from_memory():
    """3D 2x2x2-element blocks (up to ~780 dofs): their factors exceed the LDS
    staging, so the substitutions read them from memory; one Schwarz
    application and a V-cycle of a 16x4x4 time step against the checker's
    ILU(0) solves on the same matrices."""
    import scipy.sparse as sp

    from paper_1709_05660_amd import MG, Problem
    from synth import config, fourier_coefficients
    s = config("c3_3d_32x8x8").with_(nx=16, ny=4, nz=4, levels=2, patch=2, transient=True, rtol=1e-10)
    p = Problem(s, fourier_coefficients(3, s.seed))
    levels = []
    for l in range(p.nlevels):
        lv = osolver.Level(J=csr_of(p, l, "J"))
        if l > 0:
            lv.P, lv.R = csr_of(p, l, "P"), csr_of(p, l, "R")
            lv.ptr, lv.dof, lv.owned, lv.kind = p.patches(l)
        levels.append(lv)
    osolver.setup_factors(levels, fluid_ilu=True)
    mg = MG(p, precision="fp64", fluid_ilu=True)
    li = mg.level_info(1)
    _say(f"3D ILU blocks {li['nilu']}, factor entries {li['ilu_entries']}, largest m {np.diff(levels[1].ptr).max()}")
    assert li["nilu"] > 0 and li["ilu_entries"] * 10 // li["nilu"] > 150 * 1024   # beyond the LDS staging
    rng = np.random.default_rng(23)
    r = rng.standard_normal(p.n)
    y = host(mg.apply(1, 4, dev(r)))
    ref = osolver.ras(levels[1], r)
    _say(f"3D Schwarz (ILU fluid) rel diff {_rel(y, ref):.2e}")
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    z = host(mg.vcycle(dev(r)))
    zref = osolver.vcycle(levels, 1, r, s.nu_pre, s.nu_post, s.omega)
    mg.close()
    # the same comparison with exact local solves everywhere: on this stiff 3D
    # step the V-cycle's output carries the rounding of its residual updates
    # (the checker itself moves by ~2e-12 under a 1e-15 change of r), so the
    # ILU path is held to the exact path's agreement with the checker
    lu = [osolver.Level(J=lv.J, P=lv.P, R=lv.R, ptr=lv.ptr, dof=lv.dof, owned=lv.owned, kind=lv.kind)
          for lv in levels]
    osolver.setup_factors(lu)
    mg_lu = MG(p, precision="fp64")
    z_lu = host(mg_lu.vcycle(dev(r)))
    mg_lu.close()
    d_lu = _rel(z_lu, osolver.vcycle(lu, 1, r, s.nu_pre, s.nu_post, s.omega))
    d_ilu = _rel(z, zref)
    _say(f"3D V-cycle rel diff: ILU fluid {d_ilu:.2e}, exact {d_lu:.2e}")
    assert d_ilu <= max(1e-10, 10 * d_lu)
