"""Device assembly of the residual and exact Jacobian, and Newton's method
on the device (include/fsi_assembly.h; section "Monolithic Newton-Krylov
solver with Multigrid-Richardson-Schwarz preconditioner").

* The device assembly at the seeded state equals the host builder's finest
  Jacobian and residual (steady and Crank-Nicolson, 2D and 3D, small and at
  the bench's full sizes); at a state
  away from it, the checker's own assembly (complex-step Jacobian) is the
  reference.
* Newton on the device (assembly, Galerkin products, refactor, FGMRES, update)
  drives the checker's residual of the time step down to rounding.
"""

import sys

import numpy as np
import pytest

from gpu_common import csr_of, dev, host
from oracle import fem
from synth import config, fourier_coefficients

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [("c0_2d_16x4", {}), ("c5_2d_16x4_cn", {}),
         ("c3_3d_32x8x8", dict(nx=16, ny=4, nz=4, levels=2, patch=2)),
         ("c3_3d_32x8x8", dict(nx=16, ny=4, nz=4, levels=2, patch=2, transient=True))]


def _setup(name, kw):
    from paper_1709_05660_amd import Assembly, Problem
    s = config(name).with_(**kw)
    a = fourier_coefficients(s.dim, s.seed)
    p = Problem(s, a)
    return s, a, p, Assembly(p)


# the full-size systems of the bench's 2D, time-step and 3D legs (4,096 and
# 2,048 elements), in the launch configuration the bench times
FULL = [("c1_2d_128x32", {}), ("c4_2d_128x32_cn", {}), ("c3_3d_32x8x8", {})]


@pytest.mark.parametrize("name,kw", CASES + FULL)
def test_device_assembly_equals_the_builders(name, kw):
    s, coeffs, p, asm = _setup(name, kw)
    r, jv = asm.run(dev(p.y))
    J = csr_of(p, p.nlevels - 1)
    jv = host(jv)
    rowmax = np.maximum(np.abs(J).max(axis=1).toarray().ravel(), 1e-300)
    rows = np.repeat(np.arange(J.shape[0]), np.diff(J.indptr))
    err = np.abs(jv - J.data) / rowmax[rows]
    r_host = p.residual(p.y)
    rerr = float(np.max(np.abs(host(r) - r_host)) / max(np.max(np.abs(r_host)), 1e-300))
    _say(f"{name} {kw}: J max row-relative err {err.max():.2e}, r err {rerr:.2e}")
    assert err.max() <= 1e-12
    assert rerr <= 1e-12
    asm.close()


@pytest.mark.parametrize("name,kw", CASES[:2] + CASES[3:])
def test_device_assembly_off_state_against_checker(name, kw):
    s, coeffs, p, asm = _setup(name, kw)
    rng = np.random.default_rng(41)
    y = p.y + 1e-3 * rng.standard_normal(p.n) * (np.abs(p.y) + 1e-2)
    flags = p.dirichlet(p.nlevels - 1).astype(bool)
    y[flags] = p.y[flags]
    r, jv = asm.run(dev(y))
    n = (s.nx, s.ny, s.nz if s.dim == 3 else 1)
    mesh = fem.Mesh(s, n)
    y_prev = fem.transient_states(mesh, s, coeffs)[0] if getattr(s, "transient", False) else None
    r_o, J_o = fem.assemble(mesh, s, y, y_prev=y_prev)
    J_o = J_o.tocsr()
    J_o.sort_indices()
    J = csr_of(p, p.nlevels - 1)
    Jd = J.copy()
    Jd.data = host(jv)
    diff = abs(Jd - J_o)
    rowmax = np.maximum(abs(J_o).max(axis=1).toarray().ravel(), 1e-300)
    jerr = float((diff.max(axis=1).toarray().ravel() / rowmax).max())
    rerr = float(np.max(np.abs(host(r) - r_o)) / np.max(np.abs(r_o)))
    _say(f"{name} {kw} off state: J err {jerr:.2e}, r err {rerr:.2e}")
    assert jerr <= 1e-10 and rerr <= 1e-11
    asm.close()


@pytest.mark.parametrize("name", ["c5_2d_16x4_cn", "c4_2d_128x32_cn"])
def test_newton_on_the_device_solves_the_time_step(name):
    """From the Newton iterate y_{n+1} of the time step, Newton on the device
    reaches the paper's stopping test |e| <= 1e-8 |y|, and the checker's
    residual at the result is down by many orders."""
    from paper_1709_05660_amd import MG
    s, coeffs, p, asm = _setup(name, {})
    mg = MG(p, precision="fp64", use_graph=True)
    y = dev(p.y)
    info = asm.newton(mg, y, max_newton=12, tol=1e-8, rtol=1e-10)
    y = host(y)
    mesh = fem.Mesh(s, (s.nx, s.ny, 1))
    y0, y1 = fem.transient_states(mesh, s, coeffs)
    r1, _ = fem.assemble(mesh, s, y1, jacobian=False, y_prev=y0)
    rN, _ = fem.assemble(mesh, s, y, jacobian=False, y_prev=y0)
    flags = p.dirichlet(p.nlevels - 1).astype(bool)
    drop = float(np.linalg.norm(rN[~flags]) / np.linalg.norm(r1[~flags]))
    _say(f"{name}: Newton {info}, checker residual drop {drop:.2e}")
    assert info["converged"] == 1
    assert drop <= 1e-9
    assert np.all(y[flags] == p.y[flags])           # Dirichlet values kept
    mg.close()
    asm.close()


def test_failed_creation_frees_its_memory():
    """A creation that fails after uploading the element data (here: a
    Dirichlet row of the pattern without its diagonal) returns FSI_E_INVALID
    and frees what it allocated: ten such failures hold no more device memory
    than one (the runtime may keep freed blocks for reuse), where each would
    otherwise keep about 14 MB; a valid assembler beside them still equals
    the builder."""
    import ctypes as C

    import torch

    from paper_1709_05660_amd import _lib as L
    from paper_1709_05660_amd.solver import _stream
    s, coeffs, p, asm = _setup("c1_2d_128x32", {})
    ed, J = asm.ed, p.levels[p.nlevels - 1].J
    rp = np.ctypeslib.as_array(J.rowptr, shape=(J.nrows + 1,))
    col = np.ctypeslib.as_array(J.colind, shape=(J.nnz,)).copy()
    dirf = np.ctypeslib.as_array(ed.dirichlet, shape=(ed.ndof,))
    i = int(np.flatnonzero(dirf)[0])
    pos = int(rp[i] + np.flatnonzero(col[rp[i]:rp[i + 1]] == i)[0])
    col[pos] = i + 1 if i + 1 < J.ncols else i - 1
    bad = L.Csr(J.nrows, J.ncols, J.nnz, J.rowptr, col.ctypes.data_as(C.POINTER(C.c_int32)), J.val)

    def fail_once():
        h = C.c_void_p()
        st = L.lib().fsi_assembly_create(C.byref(ed), C.byref(bad), _stream(), C.byref(h))
        assert st == L.FSI_E_INVALID and not h.value
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    free1 = fail_once()
    for _ in range(9):
        free10 = fail_once()
    _say(f"device memory held by nine more failed creations: {(free1 - free10) / 2**20:.1f} MiB")
    assert free1 - free10 < 4 << 20
    r, jv = asm.run(dev(p.y))
    Jh = csr_of(p, p.nlevels - 1)
    assert np.abs(host(jv) - Jh.data).max() <= 1e-12 * np.abs(Jh.data).max()
    asm.close()
