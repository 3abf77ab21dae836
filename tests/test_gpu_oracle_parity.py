"""GPU results against the FP64 checker for restarted FGMRES, a nonzero start,
the mixed-precision forms, the full-size patch lists and served requests.

Expected values come from the checker only: its own independently assembled
hierarchy where that is affordable (2D), or its algorithm (LU local solves,
V-cycle, FGMRES) on the builder's matrices (3D; the builder's full-size 3D
hierarchy equals the checker's, J to 1e-12 per row and P, R and the patch
lists bit for bit, in tests/test_abi_cpu.py).
"""

import functools
import sys

import numpy as np
import pytest

from gpu_common import csr_of, dev, host, oracle_hierarchy, oracle_on_product, product_problem
from oracle import problem as oprob
from synth import config, fourier_coefficients, serving_stream

pytestmark = pytest.mark.gpu

# Error bound of a mixed-precision solution against the checker's FP64 one:
# ten times the workload's relative residual target (1e-8).  The relative
# error is at most cond(J) times the relative residual; the measured errors
# are near 1e-9, the bound leaves a decade for other right-hand sides.
MIXED_ERR_BOUND = 1e-7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@functools.lru_cache(maxsize=None)
def _oracle_solution(name, on_product=False, **kw):
    h = oracle_on_product(name) if on_product else oracle_hierarchy(name)
    return oprob.solve(h, **kw)


# ------------------------------------------------------------ restarts, x0
@pytest.mark.parametrize("graph", [False, True])
def test_restarted_fgmres_parity_c0(graph):
    """FGMRES(5) on the 16x4 system: 54 iterations in 11 cycles.  The GPU run
    for the checker's iteration count equals the checker's to 1e-10; the
    converged run takes the same number of iterations."""
    from paper_1709_05660_amd import MG
    p = product_problem("c0_2d_16x4")
    oh = oracle_hierarchy("c0_2d_16x4")
    s = oh.spec
    x_o, io = _oracle_solution("c0_2d_16x4", restart=5)
    k = io.iters
    assert io.restarts >= 3
    x_fix, i_fix = oprob.solve(oh, restart=5, fixed_iters=k)
    _say("c0 restart 5: checker iters", k, "cycles", io.restarts, "graph", graph)
    mg = MG(p, precision="fp64", use_graph=graph)
    xg, ig = mg.fgmres(dev(p.b), restart=5, rtol=s.rtol, fixed_iters=k)
    xg = host(xg)
    assert ig["iters"] == k and ig["restarts"] == i_fix.restarts
    rel = _rel(xg, x_fix)
    _say("  fixed-iteration rel diff", rel)
    assert rel <= 1e-10
    x2, i2 = mg.fgmres(dev(p.b), restart=5, rtol=s.rtol)
    x2 = host(x2)
    _say("  converged: iters", i2["iters"], "cycles", i2["restarts"], "rel diff", _rel(x2, x_o))
    assert i2["converged"] == 1 and abs(i2["iters"] - k) <= 1
    assert _rel(x2, x_o) <= 1e-10
    J = oh.levels[-1].J
    assert np.linalg.norm(oh.b - J @ x2) <= s.rtol * np.linalg.norm(oh.b) * 1.001
    mg.close()


@pytest.mark.parametrize("restart,graph", [(5, False), (30, True)])
def test_fgmres_nonzero_start_parity_c0(restart, graph):
    """A warm start (the checker's iterate after 10 steps, as a later Newton
    step would pass the previous solution): fixed-iteration parity at 1e-10
    and equal converged iteration counts."""
    from paper_1709_05660_amd import MG
    p = product_problem("c0_2d_16x4")
    oh = oracle_hierarchy("c0_2d_16x4")
    s = oh.spec
    x0, _ = oprob.solve(oh, fixed_iters=10)
    x_o, io = oprob.solve(oh, restart=restart, x0=x0)
    k = io.iters
    x_fix, _ = oprob.solve(oh, restart=restart, x0=x0, fixed_iters=k)
    mg = MG(p, precision="fp64", use_graph=graph)
    xg = dev(x0)
    xg, ig = mg.fgmres(dev(p.b), xg, restart=restart, rtol=s.rtol, fixed_iters=k, x0=True)
    rel = _rel(host(xg), x_fix)
    _say("c0 x0 restart", restart, "checker iters", k, "fixed rel diff", rel, "hist0", ig["history"][0],
         "checker hist0", io.history[0])
    assert ig["history"][0] == pytest.approx(io.history[0], rel=1e-9)
    assert rel <= 1e-10
    xg = dev(x0)
    xg, ig = mg.fgmres(dev(p.b), xg, restart=restart, rtol=s.rtol, x0=True)
    assert ig["converged"] == 1 and abs(ig["iters"] - k) <= 1
    assert _rel(host(xg), x_o) <= 1e-10
    mg.close()


# ------------------------------------------------------------ mixed forms
@pytest.fixture(scope="module")
def c1_oracle():
    _say("checker hierarchy and solution of c1_2d_128x32")
    oh = oracle_hierarchy("c1_2d_128x32")
    x_o, io = _oracle_solution("c1_2d_128x32")
    return oh, x_o, io


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_mixed_against_checker_c1(c1_oracle, prec):
    """Mixed V-cycle with FP64 Krylov on the 128x32 system: the residual of
    the GPU solution, computed on the host with the checker's own Jacobian,
    is <= 1e-8 relative, and the solution is within MIXED_ERR_BOUND of the
    checker's FP64 solution."""
    from paper_1709_05660_amd import MG
    oh, x_o, io = c1_oracle
    p = product_problem("c1_2d_128x32")
    mg = MG(p, precision=prec)
    x, info = mg.fgmres(dev(p.b), restart=30, rtol=1e-8)
    x = host(x)
    J = oh.levels[-1].J
    relres = float(np.linalg.norm(oh.b - J @ x) / np.linalg.norm(oh.b))
    err = _rel(x, x_o)
    _say(f"c1 {prec}: iters {info['iters']} (FP64 checker {io.iters} to 1e-10), host relres {relres:.3e}, "
         f"err vs checker {err:.3e}")
    assert info["converged"] == 1
    assert relres <= 1e-8 * 1.01
    assert err <= MIXED_ERR_BOUND
    mg.close()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mixed_against_checker_3d(prec):
    from paper_1709_05660_amd import MG
    name = "c3_3d_32x8x8"
    p = product_problem(name)
    x_o, io = _oracle_solution(name, on_product=True, rtol=1e-10)
    mg = MG(p, precision=prec)
    x, info = mg.fgmres(dev(p.b), restart=30, rtol=1e-8)
    x = host(x)
    J = csr_of(p, p.nlevels - 1)
    relres = float(np.linalg.norm(p.b - J @ x) / np.linalg.norm(p.b))
    err = _rel(x, x_o)
    _say(f"3d {prec}: iters {info['iters']}, host relres {relres:.3e}, err vs checker {err:.3e}")
    assert info["converged"] == 1
    assert relres <= 1e-8 * 1.01
    assert err <= MIXED_ERR_BOUND
    mg.close()


# ------------------------------------------------------------ full-size patch lists
def test_patch_lists_bit_exact_c1(c1_oracle):
    """Device patch lists of every smoothing level of the 128x32 system equal
    the checker's independently built lists; every device-extracted block
    equals J[I_k, I_k] of the operator the device holds, bit for bit."""
    from oracle import solver as osolver
    from paper_1709_05660_amd import MG
    oh, _, _ = c1_oracle
    p = product_problem("c1_2d_128x32")
    mg = MG(p, precision="fp64")
    for l in range(1, p.nlevels):
        ptr, dof, owned, B = mg.export_patches(l, blocks=True)
        lv = oh.levels[l]
        assert np.array_equal(ptr, lv.ptr)
        assert np.array_equal(dof, lv.dof)
        assert np.array_equal(owned, lv.owned)
        J = csr_of(p, l)
        off = 0
        for k in range(len(ptr) - 1):
            I = dof[ptr[k]:ptr[k + 1]]
            m = I.size
            assert np.array_equal(B[off:off + m * m].reshape(m, m), osolver.extract_block(J, I)), (l, k)
            off += m * m
        _say("c1 level", l, "patches", len(ptr) - 1, "bit-exact")
    mg.close()


# ------------------------------------------------------------ served requests
def _one_per_mesh_class():
    """One request of each mesh size in the serving stream, alternately a
    sweep point and a time step (32x8 steady, 64x16 a time step, 128x32
    steady): the first of that kind and size."""
    stream = serving_stream(256)
    sizes = sorted({(r.nx, r.ny) for r in stream})
    out = []
    for i, sz in enumerate(sizes):
        out.append(next(r for r in stream if (r.nx, r.ny) == sz and r.transient == bool(i % 2)))
    return out


def _wait(server, ticket, timeout=120.0):
    import time
    t0 = time.time()
    while True:
        st, x, info = server.poll(ticket)
        if st != 2:
            return st, x, info
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} not finished")
        time.sleep(0.001)


@pytest.mark.parametrize("batched", [False, True])
def test_served_results_match_checker(batched):
    """One request of each mesh class of the serving stream (sweep points and
    a time step), served in FP64 for the checker's iteration count (1e-10
    against the checker's iterate) and in the mixed bf16 form to 1e-8 (host
    residual with the checker's Jacobian <= 1e-8, error <= MIXED_ERR_BOUND),
    with each system's V-cycles on its own stream or batched."""
    from paper_1709_05660_amd import Problem, Server
    base = config("c2_2d_128x32_mixed")
    srv = Server(hbm_budget_bytes=8 << 30, max_slots=4, batch_vcycles=batched)
    try:
        for r in _one_per_mesh_class():
            s = base.with_(nx=r.nx, ny=r.ny, levels=r.levels, mu_s=r.mu_s, u_peak=r.u_peak, seed=r.seed,
                           rtol=1e-10, transient=r.transient)
            a = fourier_coefficients(2, r.seed)
            _say(f"served {r.nx}x{r.ny} {'time step' if r.transient else 'steady'} mu_s {r.mu_s:.3g} "
                 f"u_peak {r.u_peak:.3f} batched {batched}: checker hierarchy")
            oh = oprob.build(s, a)
            x_o, io = oprob.solve(oh)
            k = io.iters
            x_fix, _ = oprob.solve(oh, fixed_iters=k)
            p = Problem(s, a)
            t64 = srv.submit(p, precision="fp64", rtol=1e-10, fixed_iters=k)
            t16 = srv.submit(p, precision="bf16", rtol=1e-8)
            st, x64, i64 = _wait(srv, t64)
            assert st in (0, 1), i64
            assert i64["iters"] == k
            rel64 = _rel(x64, x_fix)
            st, x16, i16 = _wait(srv, t16)
            assert st == 0, i16
            J = oh.levels[-1].J
            relres = float(np.linalg.norm(oh.b - J @ x16) / np.linalg.norm(oh.b))
            err = _rel(x16, x_o)
            _say(f"  fp64 fixed {k}: rel diff {rel64:.3e}; bf16: iters {i16['iters']}, host relres "
                 f"{relres:.3e}, err {err:.3e}")
            assert rel64 <= 1e-10
            assert relres <= 1e-8 * 1.01
            assert err <= MIXED_ERR_BOUND
    finally:
        srv.close()
