"""Pins of the checker's ILU(0) local solver for fluid blocks (section
"Richardson-Schwarz smoother": an incomplete factorization suffices on
fluid subdomains, the exact one is kept on solid ones).

* The defining property of ILU(0): L unit lower and U upper triangular,
  zero off the pattern, with (L U)_ij = B_ij at every pattern position,
  checked by multiplying the factors out (random sparse blocks and a real
  fluid block of the saddle-point system, whose pressure rows have no
  stored diagonal).
* Where elimination creates no fill outside the pattern (a full pattern; a
  tridiagonal block) ILU(0) is the exact LU: its solve equals a dense solve.
* The Richardson-Schwarz V-cycle with ILU(0) on the fluid blocks
  preconditions FGMRES on a Crank-Nicolson step to the dense solution.
"""

import numpy as np
import pytest

from oracle import problem as oprob
from oracle import solver as osolver
from synth import config, fourier_coefficients


def _factors(F):
    L = np.tril(F, -1) + np.eye(F.shape[0])
    U = np.triu(F)
    return L, U


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilu0_defining_property_random(seed):
    rng = np.random.default_rng(seed)
    m = 40
    pat = rng.random((m, m)) < 0.15
    np.fill_diagonal(pat, True)
    B = np.where(pat, rng.standard_normal((m, m)), 0.0)
    B += np.diag(np.abs(B).sum(axis=1) + 1.0)          # no zero pivot
    F = osolver.ilu0_factor(B, pat)
    L, U = _factors(F)
    assert np.all(F[~pat] == 0.0)
    LU = L @ U
    assert np.max(np.abs(LU[pat] - B[pat])) <= 1e-12 * np.max(np.abs(B))
    # fill is dropped: off the pattern the product differs from B (= 0) somewhere
    assert np.max(np.abs(LU[~pat])) > 1e-6


def test_ilu0_full_pattern_is_the_lu():
    rng = np.random.default_rng(3)
    m = 30
    B = rng.standard_normal((m, m)) + m * np.eye(m)
    pat = np.ones((m, m), dtype=bool)
    F = osolver.ilu0_factor(B, pat)
    L, U = _factors(F)
    assert np.max(np.abs(L @ U - B)) <= 1e-12 * np.max(np.abs(B))
    g = rng.standard_normal(m)
    assert np.allclose(osolver.ilu0_solve(F, g), np.linalg.solve(B, g), rtol=1e-12, atol=1e-14)


def test_ilu0_tridiagonal_is_exact():
    m = 50
    rng = np.random.default_rng(4)
    B = np.diag(4.0 + rng.random(m)) + np.diag(rng.standard_normal(m - 1), 1) + \
        np.diag(rng.standard_normal(m - 1), -1)
    pat = B != 0.0
    g = rng.standard_normal(m)
    x = osolver.ilu0_solve(osolver.ilu0_factor(B, pat), g)
    assert np.allclose(x, np.linalg.solve(B, g), rtol=1e-12, atol=1e-14)


def test_ilu0_on_a_fluid_block_of_the_saddle_point_system():
    s = config("c5_2d_16x4_cn")
    h = oprob.build(s, fourier_coefficients(2, s.seed), factor=False)
    lv = h.levels[1]
    k = int(np.nonzero(lv.kind == 0)[0][0])
    I = lv.dof[lv.ptr[k]:lv.ptr[k + 1]]
    B = lv.J[I][:, I].toarray()
    pat = osolver.block_pattern(lv.J, I)
    zero_diag = np.nonzero(np.diag(B) == 0.0)[0]
    assert zero_diag.size > 0                    # the continuity rows store no diagonal
    F = osolver.ilu0_factor(B, pat)
    L, U = _factors(F)
    assert np.max(np.abs((L @ U)[pat] - B[pat])) <= 1e-10 * np.max(np.abs(B))
    assert np.all(np.abs(np.diag(U)[zero_diag]) > 0)   # filled by the elimination


def test_fluid_ilu_vcycle_preconditions_the_time_step():
    s = config("c5_2d_16x4_cn").with_(fluid_ilu=True)
    h = oprob.build(s, fourier_coefficients(2, s.seed))
    assert any(isinstance(f[0], str) for f in h.levels[1].lu)
    x, info = oprob.solve(h)
    assert info.converged and info.true_relres <= s.rtol
    xd = np.linalg.solve(h.levels[-1].J.toarray(), h.b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    h_lu = oprob.build(config("c5_2d_16x4_cn"), fourier_coefficients(2, s.seed))
    _, info_lu = oprob.solve(h_lu)
    assert info.iters >= info_lu.iters           # the incomplete local solves are weaker
