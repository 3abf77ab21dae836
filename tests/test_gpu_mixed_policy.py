"""GPU tests of the per-kind precision policy of the mixed forms (section
"Richardson-Schwarz smoother": exact local solves are required on the solid
blocks, fluid blocks may be solved inexactly): solid blocks stored in FP32
(solid_precision) or solved with FP32 refinement sweeps of their 16-bit
inverses (refine_sweeps), against the FP64 checker."""

import sys

import numpy as np
import pytest

from gpu_common import csr_of, dev, host, oracle_hierarchy, oracle_on_product, product_problem
from oracle import problem as oprob
from oracle import solver as osolver

pytestmark = pytest.mark.gpu

MIXED_ERR_BOUND = 1e-7     # as in test_gpu_oracle_parity


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _owned_by_kind(p, level):
    """Dofs owned by solid and by fluid blocks on a level."""
    ptr, dof, owned, kind = p.patches(level)
    solid, fluid = [], []
    for k in range(len(ptr) - 1):
        d = dof[ptr[k]:ptr[k + 1]][owned[ptr[k]:ptr[k + 1]].astype(bool)]
        (solid if kind[k] == 1 else fluid).append(d)
    return np.concatenate(solid), np.concatenate(fluid)


def test_solid_policies_sharpen_the_solid_local_solves():
    """One Schwarz application on the 128x32 finest level (fsi_mg_apply op 6)
    against the checker's exact LU solves: on the solid-owned dofs one
    refinement sweep of the bf16 inverses cuts the error by at least 10x, a
    second one further, and FP32 solid storage likewise; the fluid-owned dofs
    are computed by the same kernel on the same data in every policy."""
    from paper_1709_05660_amd import MG
    name = "c1_2d_128x32"
    p = product_problem(name)
    oh = oracle_on_product(name)
    L = p.nlevels - 1
    rng = np.random.default_rng(17)
    x = rng.standard_normal(p.n)
    ref = osolver.ras(oh.levels[L], x)
    sdofs, fdofs = _owned_by_kind(p, L)
    err = {}
    fluid = {}
    for tag, kw in (("bf16", {}), ("bf16+1", dict(refine_sweeps=1)), ("bf16+2", dict(refine_sweeps=2)),
                    ("bf16/fp32", dict(solid_precision="fp32"))):
        mg = MG(p, precision="bf16", **kw)
        y = host(mg.apply(L, 6, dev(x)))
        mg.close()
        err[tag] = np.linalg.norm(y[sdofs] - ref[sdofs]) / np.linalg.norm(ref[sdofs])
        fluid[tag] = y[fdofs]
        _say(f"{tag}: solid rel err {err[tag]:.3e}, fluid rel err "
             f"{np.linalg.norm(y[fdofs] - ref[fdofs]) / np.linalg.norm(ref[fdofs]):.3e}")
    assert err["bf16+1"] <= 0.1 * err["bf16"]
    assert err["bf16+2"] <= err["bf16+1"]
    assert err["bf16/fp32"] <= 0.1 * err["bf16"]
    for tag in ("bf16+1", "bf16+2", "bf16/fp32"):
        assert np.array_equal(fluid[tag], fluid["bf16"])


@pytest.mark.parametrize("name,prec,kw", [("c1_2d_128x32", "bf16", dict(refine_sweeps=1)),
                                          ("c1_2d_128x32", "fp16", dict(refine_sweeps=1)),
                                          ("c1_2d_128x32", "bf16", dict(solid_precision="fp32")),
                                          ("c3_3d_32x8x8", "bf16", dict(refine_sweeps=1))])
def test_policy_solves_against_checker(name, prec, kw):
    """FGMRES with each policy converges to 1e-8: the residual on the host
    (with the checker's own Jacobian in 2D, the builder's in 3D, equal to the
    checker's at full size) and the error against the checker's FP64 solution."""
    from paper_1709_05660_amd import MG
    p = product_problem(name)
    if name.startswith("c1"):
        oh = oracle_hierarchy(name)
        J, b = oh.levels[-1].J, oh.b
    else:
        oh = oracle_on_product(name)
        J, b = csr_of(p, p.nlevels - 1), p.b
    x_o, io = oprob.solve(oh, rtol=1e-10)
    mg = MG(p, precision=prec, use_graph=True, **kw)
    x, info = mg.fgmres(dev(p.b), restart=30, rtol=1e-8)
    x = host(x)
    relres = float(np.linalg.norm(b - J @ x) / np.linalg.norm(b))
    e = float(np.linalg.norm(x - x_o) / np.linalg.norm(x_o))
    _say(f"{name} {prec} {kw}: iters {info['iters']}, host relres {relres:.3e}, err {e:.3e}")
    assert info["converged"] == 1 and relres <= 1e-8 * 1.01 and e <= MIXED_ERR_BOUND
    mg.close()


def test_refined_graph_equals_eager():
    from paper_1709_05660_amd import MG
    p = product_problem("c1_2d_128x32")
    out = []
    for graph in (False, True):
        mg = MG(p, precision="bf16", refine_sweeps=1, use_graph=graph)
        x, info = mg.fgmres(dev(p.b), restart=30, rtol=1e-8)
        out.append((host(x), info["iters"]))
        mg.close()
    assert out[0][1] == out[1][1] and np.array_equal(out[0][0], out[1][0])
