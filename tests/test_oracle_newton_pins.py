"""Pins of the checker's Newton iteration and full multigrid (section
"Monolithic Newton-Krylov solver with Multigrid-Richardson-Schwarz
preconditioner"; stopping rule of section "Details on the iterative
solver").

* Newton on the 16x4 mesh converges, and quadratically: an exact Jacobian
  gives |e_{k+1}| <= C |e_k|^2 near the root, which a dropped or wrong
  Jacobian term (linear convergence) breaks.
* At the converged state the residual is zero up to rounding.
* The full-multigrid transfer of a coarse iterate that equals the coarse
  seeded state is the fine seeded state (the base transfer loses nothing),
  and its Dirichlet dofs hold their values.
"""

import numpy as np

from oracle import fem, transfer
from oracle import newton as onewton
from synth import config, fourier_coefficients


def _spec():
    s = config("c1_2d_128x32")
    return s, fourier_coefficients(2, s.seed)


def test_newton_converges_quadratically_on_16x4():
    s, a = _spec()
    mesh = fem.Mesh(s, (16, 4))
    y0 = fem.seeded_state(mesh, s, a)
    y, steps, conv, hist = onewton.newton(mesh, s, y0, tol=1e-8, max_steps=15)
    assert conv and steps <= 12
    r, _ = fem.assemble(mesh, s, y, jacobian=False)
    flag = mesh.dirichlet(s.u_peak)[0]
    assert np.linalg.norm(r[~flag]) <= 1e-6 * hist[0][0]
    assert np.all(r[flag] == 0.0)
    # past the stopping test, down to rounding: every step that starts with
    # 1e-7 <= |e_k| <= 1e-2 contracts quadratically, |e_{k+1}| <= 2 |e_k|^2
    # (a Jacobian off by 0.1 % contracts linearly and fails this)
    y, steps, conv, hist = onewton.newton(mesh, s, y0, tol=1e-15, max_steps=14)
    e = [q * np.linalg.norm(y) for _, q in hist]
    checked = 0
    for k in range(len(e) - 1):
        if 1e-7 <= e[k] <= 1e-2 and e[k + 1] > 1e-9:
            assert e[k + 1] <= 2.0 * e[k] ** 2, (k, e)
            checked += 1
    assert checked >= 1, e


def test_fmg_base_transfer_reproduces_the_seeded_state():
    s, a = _spec()
    mc, mf = fem.Mesh(s, (16, 4)), fem.Mesh(s, (32, 8))
    fc, _ = mc.dirichlet(s.u_peak)
    ff, vf = mf.dirichlet(s.u_peak)
    sc, sf = fem.seeded_state(mc, s, a), fem.seeded_state(mf, s, a)
    P = transfer.prolongation(mf, mc, ff, fc)
    y = sf + P @ (sc - sc)
    y[ff] = vf[ff]
    assert np.array_equal(y, sf)


def test_time_steps_keep_a_steady_solution():
    """A steady solution is a fixed point of the Crank-Nicolson step (at rest
    the step's residual is the steady residual): the checker's time steps
    from the converged 16x4 steady state stop after one Newton step with a
    negligible update and leave the state where it was."""
    s, a = _spec()
    mesh = fem.Mesh(s, (16, 4))
    y, _, conv, _ = onewton.newton(mesh, s, fem.seeded_state(mesh, s, a), tol=1e-12, max_steps=15)
    assert conv
    y2, out = onewton.cn_steps(mesh, s, y, 2, tol=1e-8)
    for steps, conv, hist in out:
        assert conv and steps == 1 and hist[0][1] <= 1e-9
    assert np.linalg.norm(y2 - y) <= 1e-9 * np.linalg.norm(y)
