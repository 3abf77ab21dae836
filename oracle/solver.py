"""Checker: dense LU, Richardson-RAS smoother, V-cycle and FGMRES (FP64, CPU).

Test infrastructure only.

* Local solves: LU with partial pivoting of B_k = J[I_k, I_k] (the paper's
  exact local direct solve, mandatory on solid blocks), via LAPACK getrf.
* Smoother (section "Richardson-Schwarz smoother"): Richardson iteration
  e <- e - omega B^{-1}(J e + r) for J e = -r, i.e. e <- e + omega B^{-1}(r - J e)
  for J e = r, with the restricted additive Schwarz operator
  B^{-1} = sum_k (R^0_k)^T B_k^{-1} R^delta_k.
* V-cycle (section "Geometric Multigrid preconditioner"): pre-smoothing,
  restriction of the residual, recursive coarse correction, prolongation,
  post-smoothing; a direct solve on the coarsest level.
* Krylov: right-preconditioned flexible GMRES(m) (Saad) with classical
  Gram-Schmidt applied twice; the paper's PETSc GMRES is left-preconditioned
  with a single classical Gram-Schmidt pass.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla


@dataclass
class Level:
    J: object                       # scipy CSR
    P: object = None                # n_l x n_{l-1}
    R: object = None                # n_{l-1} x n_l
    ptr: np.ndarray = None
    dof: np.ndarray = None
    owned: np.ndarray = None
    kind: np.ndarray = None
    lu: list = field(default_factory=list)


def setup_factors(levels):
    """LU factors of every patch block (levels >= 1) and of the coarsest operator."""
    levels[0].lu = [sla.lu_factor(levels[0].J.toarray(), check_finite=True)]
    for lv in levels[1:]:
        A = lv.J
        lv.lu = []
        for k in range(len(lv.ptr) - 1):
            I = lv.dof[lv.ptr[k]:lv.ptr[k + 1]]
            Bk = A[I][:, I].toarray()
            lv.lu.append(sla.lu_factor(Bk, check_finite=True))


def extract_block(J, I):
    """B_k = J[I_k, I_k] as a dense FP64 array."""
    return J[I][:, I].toarray()


def ras(lv, s):
    """delta = sum_k (R^0_k)^T B_k^{-1} R^delta_k s."""
    out = np.zeros_like(s)
    for k in range(len(lv.ptr) - 1):
        a, b = lv.ptr[k], lv.ptr[k + 1]
        I = lv.dof[a:b]
        y = sla.lu_solve(lv.lu[k], s[I])
        own = lv.owned[a:b].astype(bool)
        out[I[own]] += y[own]
    return out


def smooth(lv, r, e, sweeps, omega, first_zero):
    for it in range(sweeps):
        s = r if (first_zero and it == 0) else r - lv.J @ e
        e = e + omega * ras(lv, s)
    return e


def vcycle(levels, l, r, nu_pre, nu_post, omega):
    """z = M_l^{-1} r on level l (0 = coarsest, direct solve)."""
    if l == 0:
        return sla.lu_solve(levels[0].lu[0], r)
    lv = levels[l]
    e = np.zeros_like(r)
    e = smooth(lv, r, e, nu_pre, omega, first_zero=True)
    rc = lv.R @ (r - lv.J @ e)
    e = e + lv.P @ vcycle(levels, l - 1, rc, nu_pre, nu_post, omega)
    e = smooth(lv, r, e, nu_post, omega, first_zero=False)
    return e


@dataclass
class SolveInfo:
    iters: int
    restarts: int
    converged: bool
    true_relres: float
    est_relres: float
    history: list


def fgmres(A, b, M, restart=30, rtol=1e-10, maxit=1000, x0=None, fixed_iters=None):
    """Right-preconditioned FGMRES(restart) with CGS2.

    Per step j: z_j = M(v_j); w = A z_j; h = V^T w, w -= V h; h' = V^T w,
    w -= V h'; h += h'; h_{j+1,j} = |w|; v_{j+1} = w / h_{j+1,j}; the stored
    Givens rotations are applied to the new column, a new rotation
    (c, s) = (h_jj, h_{j+1,j}) / hypot(h_jj, h_{j+1,j}) annihilates h_{j+1,j}
    and g_{j+1} = -s g_j, g_j = c g_j.  The cycle stops when |g_{j+1}| <=
    rtol |b|, on a happy breakdown (h_{j+1,j} <= 1e-14 |h_{:,j}|), when the
    restart length is reached or at the iteration limit; then y = H^{-1} g,
    x += Z y and the true residual b - A x decides exit or restart.
    `fixed_iters` runs exactly that many preconditioner applications
    (ignoring the tolerance) for fixed-iteration comparisons.
    """
    n = b.size
    x = np.zeros(n) if x0 is None else x0.astype(float).copy()
    bnorm = float(np.linalg.norm(b))
    tol = rtol * bnorm
    limit = maxit if fixed_iters is None else fixed_iters
    iters = 0
    restarts = 0
    hist = []
    est = float("nan")
    while True:
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        if not hist:
            hist.append(beta)
        if fixed_iters is None and beta <= tol:
            return x, SolveInfo(iters, restarts, True, beta / bnorm, beta / bnorm, hist)
        if iters >= limit or beta == 0.0:
            return x, SolveInfo(iters, restarts, beta <= tol, beta / bnorm, est, hist)
        m = restart
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            Z[:, j] = M(V[:, j])
            iters += 1
            w = A @ Z[:, j]
            h = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h
            h2 = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            breakdown = hn <= 1e-14 * float(np.linalg.norm(h))
            if not breakdown:
                V[:, j + 1] = w / hn
            for i in range(j):
                t1 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                t2 = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j], H[i + 1, j] = t1, t2
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / bnorm
            hist.append(abs(g[j + 1]))
            k = j + 1
            if (fixed_iters is None and abs(g[j + 1]) <= tol) or breakdown or iters >= limit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:, :k] @ y
        restarts += 1
