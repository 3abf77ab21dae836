"""Time integration by Crank-Nicolson steps on the device (fsi_cn_steps;
section "Discretization of the operator formulation"): each step's state at
t_n is the previous step's result, and Newton on the device gives the next.

* 16x4: three steps equal the checker's (its own assembly, exact Newton with
  direct solves): Newton counts per step and the final state.
* 128x32: three steps converge, the Dirichlet values stay, and the checker's
  Crank-Nicolson residual of the last step at the result is down by many
  orders from its value at the step's start.
"""

import sys

import numpy as np
import pytest

from gpu_common import dev, host
from oracle import fem
from oracle import newton as onewton
from synth import config, fourier_coefficients

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(name):
    from paper_1709_05660_amd import MG, Assembly, Problem
    s = config(name)
    p = Problem(s, fourier_coefficients(s.dim, s.seed))
    return s, p, Assembly(p), MG(p, precision="fp64", use_graph=True)


def test_time_steps_equal_the_checkers():
    s, p, asm, mg = _setup("c5_2d_16x4_cn")
    y = dev(p.y)
    infos, st = asm.time_steps(mg, y, 3, tol=1e-8, rtol=1e-12)
    y = host(y)
    mesh = fem.Mesh(s, (s.nx, s.ny, 1))
    y_o, out = onewton.cn_steps(mesh, s, p.y, 3, tol=1e-8)
    rel = float(np.linalg.norm(y - y_o) / np.linalg.norm(y_o))
    _say("device Newton steps", [i["steps"] for i in infos], "checker", [o[0] for o in out], "rel diff", rel)
    assert st == 0 and all(i["converged"] == 1 for i in infos) and all(o[1] for o in out)
    assert all(abs(i["steps"] - o[0]) <= 1 for i, o in zip(infos, out))
    assert rel <= 1e-9
    mg.close()
    asm.close()


def test_time_steps_full_size():
    s, p, asm, mg = _setup("c4_2d_128x32_cn")
    y = dev(p.y)
    infos, st = asm.time_steps(mg, y, 2, tol=1e-8, rtol=1e-10)
    y2 = host(y).copy()
    infos3, st3 = asm.time_steps(mg, y, 1, tol=1e-8, rtol=1e-10)
    y3 = host(y)
    _say("Newton steps per time step", [i["steps"] for i in infos + infos3],
         "Krylov", [i["krylov_iters"] for i in infos + infos3])
    assert st == 0 and st3 == 0
    flags = p.dirichlet(p.nlevels - 1).astype(bool)
    assert np.all(y3[flags] == p.y[flags])
    mesh = fem.Mesh(s, (s.nx, s.ny, 1))
    r_start, _ = fem.assemble(mesh, s, y2, jacobian=False, y_prev=y2)
    r_end, _ = fem.assemble(mesh, s, y3, jacobian=False, y_prev=y2)
    drop = float(np.linalg.norm(r_end[~flags]) / np.linalg.norm(r_start[~flags]))
    _say(f"checker residual of the last step: drop {drop:.2e}")
    assert drop <= 1e-6
    mg.close()
    asm.close()
