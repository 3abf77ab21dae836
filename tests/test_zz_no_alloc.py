"""GPU test of fsi_fgmres_solve_noalloc (through the C ABI): the same results
as fsi_fgmres_solve on two calls in a row, the second with a smaller system,
no device memory taken by the call, and the workspace limit reported."""

import ctypes as C
import sys

import numpy as np
import pytest

from gpu_common import dev, host, oracle_hierarchy, product_problem
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solve(mg, entry, b, x, **kw):
    """Calls one of the two solve entry points; returns (status, info, history)."""
    import torch

    from paper_1709_05660_amd import _lib as L
    from paper_1709_05660_amd.solver import krylov_opts
    hist = np.zeros(kw.get("maxit", 1000) + 2)
    ko = krylov_opts(history=hist, **kw)
    info = L.SolveInfo()
    st = getattr(L.lib(), entry)(mg.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(ko),
                                 C.byref(info), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, info.as_dict(), hist


def test_noalloc_solve_equals_the_allocating_solve():
    import torch

    from paper_1709_05660_amd import MG
    for name, kw in (("c1_2d_128x32", dict(restart=30, rtol=1e-10)),
                     ("c0_2d_16x4", dict(restart=5, rtol=1e-10)),            # smaller, restarted
                     ("c0_2d_16x4", dict(restart=10, rtol=1e-4, side="left", orth="cgs"))):
        _say("no-alloc solve", name, kw)
        p = product_problem(name)
        mg = MG(p, precision="fp64")
        b = dev(p.b)
        xa = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        xb = torch.full((p.n,), 7.0, dtype=torch.float64, device="cuda")   # overwritten (x0 = 0)
        sa, ia, ha = _solve(mg, "fsi_fgmres_solve", b, xa, **kw)
        free0 = torch.cuda.mem_get_info()[0]
        sb, ib, hb = _solve(mg, "fsi_fgmres_solve_noalloc", b, xb, **kw)
        free1 = torch.cuda.mem_get_info()[0]
        assert sa == sb == 0
        assert free1 == free0                       # the call took no device memory
        assert ia["iters"] == ib["iters"] and ia["restarts"] == ib["restarts"]
        assert np.array_equal(host(xa), host(xb))   # same kernels, same arithmetic
        assert np.array_equal(ha[: ia["iters"] + 1], hb[: ib["iters"] + 1])
        assert ia["true_relres"] == ib["true_relres"] and ia["rho"] == ib["rho"]
        if kw.get("side") != "left":                # and both equal the checker's solution
            x_o, io = oprob.solve(oracle_hierarchy(name), restart=kw["restart"])
            rel = np.linalg.norm(host(xb) - x_o) / np.linalg.norm(x_o)
            _say("  iters", ib["iters"], "checker", io.iters, "rel diff", rel)
            assert abs(ib["iters"] - io.iters) <= 1 and rel <= 1e-10
        mg.close()


def test_noalloc_warm_start_and_limit():
    import torch

    from paper_1709_05660_amd import MG
    p = product_problem("c0_2d_16x4")
    mg = MG(p, precision="fp64")
    b = dev(p.b)
    x0 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    _solve(mg, "fsi_fgmres_solve", b, x0, restart=30, rtol=1e-10, fixed_iters=10)
    xa, xb = x0.clone(), x0.clone()
    sa, ia, _ = _solve(mg, "fsi_fgmres_solve", b, xa, restart=30, rtol=1e-10, x0=True)
    sb, ib, _ = _solve(mg, "fsi_fgmres_solve_noalloc", b, xb, restart=30, rtol=1e-10, x0=True)
    assert sa == sb == 0 and ia["iters"] == ib["iters"]
    assert np.array_equal(host(xa), host(xb))
    mg.close()
    # a workspace larger than the static one is refused with the sizes named
    from paper_1709_05660_amd import _lib as L
    p1 = product_problem("c1_2d_128x32")
    mg = MG(p1, precision="fp64")
    x = torch.zeros(p1.n, dtype=torch.float64, device="cuda")
    st, _, _ = _solve(mg, "fsi_fgmres_solve_noalloc", dev(p1.b), x, restart=60, rtol=1e-10)
    msg = L.lib().fsi_last_error().decode()
    _say("limit:", msg)
    assert st == -6 and "static workspace" in msg
    mg.close()
