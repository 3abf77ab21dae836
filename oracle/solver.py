"""Checker: dense LU, Richardson-RAS smoother, V-cycle and FGMRES (FP64, CPU).

Test infrastructure only.

* Local solves: LU with partial pivoting of B_k = J[I_k, I_k] (the paper's
  exact local direct solve, mandatory on solid blocks), via LAPACK getrf; or,
  on fluid blocks, ILU(0) (section "Richardson-Schwarz smoother": an
  incomplete factorization suffices there): no pivoting, no fill beyond the
  block's stored entries and its diagonal.
* Smoother (section "Richardson-Schwarz smoother"): Richardson iteration
  e <- e - omega B^{-1}(J e + r) for J e = -r, i.e. e <- e + omega B^{-1}(r - J e)
  for J e = r, with the restricted additive Schwarz operator
  B^{-1} = sum_k (R^0_k)^T B_k^{-1} R^delta_k.
* V-cycle (section "Geometric Multigrid preconditioner"): pre-smoothing,
  restriction of the residual, recursive coarse correction, prolongation,
  post-smoothing; a direct solve on the coarsest level.
* Krylov: right-preconditioned flexible GMRES(m) (Saad) with classical
  Gram-Schmidt applied twice (or once), and the paper's setting (section
  "Details on the iterative solver"): GMRES on M^{-1} J (left
  preconditioning) with one classical Gram-Schmidt pass, restart 10, stopped
  when the left-preconditioned residual |M^{-1}(b - J x_j)| falls below rtol
  times its initial value.
* The average convergence rate rho = (r_N / r_0)^(1/N) of the monitored
  residual over the N iterations (defined with the tables of section
  "Condition number estimates").
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


def block_pattern(J, I):
    """Positions of B_k = J[I_k, I_k] that hold a stored entry of J, and the
    diagonal (a boolean m x m array)."""
    B = J[I][:, I].tocoo()
    pat = np.zeros((len(I), len(I)), dtype=bool)
    pat[B.row, B.col] = True
    np.fill_diagonal(pat, True)
    return pat


def ilu0_factor(B, pattern):
    """ILU(0) of the dense block B on `pattern` (boolean, diagonal included):
    L unit lower and U upper triangular, both zero off the pattern, with
    (L U)_ij = B_ij on the pattern.  Row by row (i ascending): for each pattern
    column k < i in ascending order, l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj
    at the pattern columns j > k of row i.  Returns L (below the diagonal)
    and U (on and above it) in one array."""
    A = np.where(pattern, B, 0.0).astype(np.float64)
    m = A.shape[0]
    for i in range(1, m):
        for k in np.nonzero(pattern[i, :i])[0]:
            A[i, k] = A[i, k] / A[k, k]
            A[i, k + 1:] -= np.where(pattern[i, k + 1:], A[i, k] * A[k, k + 1:], 0.0)
    return A


def ilu0_solve(F, g):
    """(L U)^{-1} g for the combined factors F of ilu0_factor: L y = g by
    forward substitution (unit diagonal), then U z = y by back substitution
    (LAPACK's triangular solves)."""
    y = sla.solve_triangular(F, np.asarray(g, dtype=np.float64), lower=True, unit_diagonal=True)
    return sla.solve_triangular(F, y, lower=False)


def setup_factors(levels, fluid_ilu=False):
    """LU factors of every patch block (levels >= 1) and of the coarsest
    operator; with fluid_ilu, ILU(0) factors (tagged "ilu0") of the fluid
    blocks (kind 0) instead."""
    levels[0].lu = [sla.lu_factor(levels[0].J.toarray(), check_finite=True)]
    for lv in levels[1:]:
        A = lv.J
        lv.lu = []
        for k in range(len(lv.ptr) - 1):
            I = lv.dof[lv.ptr[k]:lv.ptr[k + 1]]
            Bk = A[I][:, I].toarray()
            if fluid_ilu and lv.kind is not None and lv.kind[k] == 0:
                lv.lu.append(("ilu0", ilu0_factor(Bk, block_pattern(A, I))))
            else:
                lv.lu.append(sla.lu_factor(Bk, check_finite=True))


def local_solve(f, g):
    """B_k^{-1} g with the block's factors (LU, or tagged ILU(0))."""
    if isinstance(f[0], str):
        return ilu0_solve(f[1], g)
    return sla.lu_solve(f, g)


def extract_block(J, I):
    """B_k = J[I_k, I_k] as a dense FP64 array."""
    return J[I][:, I].toarray()


def ras(lv, s):
    """delta = sum_k (R^0_k)^T B_k^{-1} R^delta_k s."""
    out = np.zeros_like(s)
    for k in range(len(lv.ptr) - 1):
        a, b = lv.ptr[k], lv.ptr[k + 1]
        I = lv.dof[a:b]
        y = local_solve(lv.lu[k], s[I])
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
    rho: float = 0.0          # (r_N / r_0)^(1/N) of the monitored residual


def convergence_rate(r0, rN, iters):
    """rho = (r_N / r_0)^(1/N): the geometric mean of the ratios of consecutive residuals."""
    return (rN / r0) ** (1.0 / iters) if iters > 0 and r0 > 0 else 0.0


def _orthogonalize(V, w, j, passes):
    """Classical Gram-Schmidt of w against V[:, :j+1], applied `passes` times;
    returns (h, w)."""
    h = np.zeros(j + 1)
    for _ in range(passes):
        hp = V[:, : j + 1].T @ w
        w = w - V[:, : j + 1] @ hp
        h = h + hp
    return h, w


def _givens_step(H, cs, sn, g, j):
    """Applies the stored rotations to column j of H, then a new rotation that
    annihilates H[j+1, j]; updates g."""
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


def _back_solve(H, g, k):
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return y


def gmres_left(A, b, M, restart=10, rtol=1e-4, maxit=1000, x0=None, fixed_iters=None, orth="cgs"):
    """GMRES(restart) on M^{-1} A x = M^{-1} b (left preconditioning).

    Per step j: w = M(A v_j); w is orthogonalised against V by classical
    Gram-Schmidt (one pass for "cgs", two for "cgs2"); h_{j+1,j} = |w|;
    v_{j+1} = w / h_{j+1,j}; Givens rotations as in `fgmres`.  |g_{j+1}| is
    the preconditioned residual norm |M^{-1}(b - A x_j)|.  The solve stops
    when it is <= rtol times the initial |M^{-1}(b - A x_0)| (or at a happy
    breakdown, at the restart length, at maxit); then x += V y and the
    preconditioned residual of the new x decides exit or restart.
    true_relres is |b - A x| / |b| of the returned x; est_relres the last
    preconditioned residual over the initial one.
    """
    passes = {"cgs": 1, "cgs2": 2}[orth]
    n = b.size
    x = np.zeros(n) if x0 is None else x0.astype(float).copy()
    bnorm = float(np.linalg.norm(b))
    limit = maxit if fixed_iters is None else fixed_iters
    iters = restarts = 0
    hist = []
    r = M(b - A @ x)
    beta = beta0 = float(np.linalg.norm(r))
    hist.append(beta)
    tol = rtol * beta0

    def done(conv):
        tr = float(np.linalg.norm(b - A @ x)) / bnorm if bnorm > 0 else 0.0
        return x, SolveInfo(iters, restarts, conv, tr, beta / beta0 if beta0 > 0 else 0.0, hist,
                            convergence_rate(beta0, beta, iters))

    while True:
        if (fixed_iters is None and beta <= tol) or iters >= limit or beta == 0.0:
            return done(beta <= tol)
        m = restart
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs, sn, g = np.zeros(m), np.zeros(m), np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            w = M(A @ V[:, j])
            iters += 1
            h, w = _orthogonalize(V, w, j, passes)
            hn = float(np.linalg.norm(w))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            breakdown = hn <= 1e-14 * float(np.linalg.norm(h))
            if not breakdown:
                V[:, j + 1] = w / hn
            _givens_step(H, cs, sn, g, j)
            hist.append(abs(g[j + 1]))
            k = j + 1
            if (fixed_iters is None and abs(g[j + 1]) <= tol) or breakdown or iters >= limit:
                break
        x = x + V[:, :k] @ _back_solve(H, g, k)
        restarts += 1
        r = M(b - A @ x)
        beta = float(np.linalg.norm(r))


def fgmres(A, b, M, restart=30, rtol=1e-10, maxit=1000, x0=None, fixed_iters=None, orth="cgs2"):
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
    (ignoring the tolerance) for fixed-iteration comparisons.  orth="cgs"
    orthogonalises with one classical Gram-Schmidt pass instead of two.
    """
    passes = {"cgs": 1, "cgs2": 2}[orth]
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
            return x, SolveInfo(iters, restarts, True, beta / bnorm, beta / bnorm, hist,
                                convergence_rate(hist[0], beta, iters))
        if iters >= limit or beta == 0.0:
            return x, SolveInfo(iters, restarts, beta <= tol, beta / bnorm, est, hist,
                                convergence_rate(hist[0], beta, iters))
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
            h, w = _orthogonalize(V, w, j, passes)
            hn = float(np.linalg.norm(w))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            breakdown = hn <= 1e-14 * float(np.linalg.norm(h))
            if not breakdown:
                V[:, j + 1] = w / hn
            _givens_step(H, cs, sn, g, j)
            est = abs(g[j + 1]) / bnorm
            hist.append(abs(g[j + 1]))
            k = j + 1
            if (fixed_iters is None and abs(g[j + 1]) <= tol) or breakdown or iters >= limit:
                break
        x = x + Z[:, :k] @ _back_solve(H, g, k)
        restarts += 1
