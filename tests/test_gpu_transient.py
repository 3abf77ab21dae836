"""GPU parity of the solve of one Crank-Nicolson time step (section
"Discretization of the operator formulation"): the native builder's time-step
hierarchy solved on the GPU against the checker's own, independently
assembled one.  The time step adds the solid momentum's mass block and the
kinematics' displacement block, which the steady systems do not have."""

import sys

import numpy as np
import pytest

from gpu_common import csr_of, dev, host, oracle_hierarchy, product_problem
from oracle import problem as oprob

pytestmark = pytest.mark.gpu

# Error bound of a mixed-precision solution against the checker's FP64 one,
# as for the steady systems: ten times the relative residual target 1e-8.
MIXED_ERR_BOUND = 1e-7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,graph", [("c5_2d_16x4_cn", False), ("c5_2d_16x4_cn", True),
                                        ("c4_2d_128x32_cn", True)])
def test_time_step_fgmres_parity(name, graph):
    """FGMRES(30) in FP64: the iterate after the checker's iteration count
    equals the checker's to 1e-10, the converged count is the checker's
    within one, and the true residual meets the target."""
    from paper_1709_05660_amd import MG
    p = product_problem(name)
    oh = oracle_hierarchy(name)
    s = oh.spec
    assert np.max(np.abs(p.b - oh.b)) <= 1e-13 * np.max(np.abs(oh.b))
    x_o, io = oprob.solve(oh)
    k = io.iters
    x_fix, _ = oprob.solve(oh, fixed_iters=k)
    mg = MG(p, precision="fp64", use_graph=graph)
    b = dev(p.b)
    xg, ig = mg.fgmres(b, rtol=s.rtol, fixed_iters=k)
    rel = _rel(host(xg), x_fix)
    _say(f"{name} graph {graph}: checker iters {k} rho {io.rho:.4f}; gpu fixed rel diff {rel:.2e}")
    assert ig["history"][0] == pytest.approx(io.history[0], rel=1e-10)
    assert rel <= 1e-10
    x2, i2 = mg.fgmres(b, rtol=s.rtol)
    x2 = host(x2)
    _say(f"  converged: iters {i2['iters']} true {i2['true_relres']:.2e} rel diff {_rel(x2, x_o):.2e}")
    assert i2["converged"] == 1 and abs(i2["iters"] - k) <= 1
    J = csr_of(p, p.nlevels - 1)
    assert np.linalg.norm(p.b - J @ x2) <= s.rtol * np.linalg.norm(p.b) * 1.001
    assert _rel(x2, x_o) <= 1e-8
    mg.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_time_step_mixed_against_checker(prec):
    """The mixed-precision V-cycle on the 128x32 time step: FP64 true residual
    at 1e-8 and the solution within MIXED_ERR_BOUND of the checker's."""
    from paper_1709_05660_amd import MG
    name = "c4_2d_128x32_cn"
    p = product_problem(name)
    oh = oracle_hierarchy(name)
    x_o, _ = oprob.solve(oh)
    mg = MG(p, precision=prec)
    x, info = mg.fgmres(dev(p.b), rtol=1e-8)
    x = host(x)
    err = _rel(x, x_o)
    _say(f"{name} {prec}: iters {info['iters']} true {info['true_relres']:.2e} err vs checker {err:.2e}")
    assert info["converged"] == 1 and info["true_relres"] <= 1e-8
    assert err <= MIXED_ERR_BOUND
    mg.close()
