"""GPU tests of the coarsest-level direct solve at every size class of its
Gauss-Jordan kernels (through the C ABI, a one-level hierarchy).

The matrices are seeded saddle-point systems [[K, B^T], [B, 0]]: the zero
block forces row pivoting.  The reference is numpy's dense FP64 solve."""

import ctypes as C
import sys

import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def saddle(n, seed):
    """n x n saddle-point matrix: K (SPD, 4/5 of the rows) and a full-rank B."""
    rng = np.random.default_rng(seed)
    nk = n - n // 5
    nb = n - nk
    K = sp.random(nk, nk, density=min(1.0, 12.0 / nk), random_state=rng, format="csr")
    K = K + K.T + sp.diags(np.full(nk, 30.0))
    B = sp.random(nb, nk, density=min(1.0, 8.0 / nk), random_state=rng, format="csr")
    B = B + sp.hstack([sp.identity(nb), sp.csr_matrix((nb, nk - nb))])   # full row rank
    A = sp.bmat([[K, B.T], [B, None]], format="csr")
    A.sort_indices()
    return A


class OneLevel:
    """A hierarchy made of the coarsest level only (for fsi_mg_setup)."""

    def __init__(self, A):
        from paper_1709_05660_amd import _lib as L
        A = sp.csr_matrix(A)
        A.sort_indices()
        self.rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.col = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(A.data, dtype=np.float64)
        self.levels = (L.LevelC * 1)()
        J = self.levels[0].J
        J.nrows = J.ncols = A.shape[0]
        J.nnz = A.nnz
        J.rowptr = self.rowptr.ctypes.data_as(C.POINTER(C.c_int64))
        J.colind = self.col.ctypes.data_as(C.POINTER(C.c_int32))
        J.val = self.val.ctypes.data_as(C.POINTER(C.c_double))
        self.nlevels = 1
        self.n = A.shape[0]


# sizes covering (panel width, rows per thread): 16/1, 16/2, 16/3, 8/6, 4/12, and the largest
# coarsest size accepted (6144); none but the last a multiple of 16
@pytest.mark.parametrize("n", [37, 301, 703, 1381, 2003, 3501, 6144])
def test_coarsest_solve_matches_dense(n):
    import torch

    from paper_1709_05660_amd import MG
    A = saddle(n, 100 + n)
    _say("coarse n", n, "nnz", A.nnz)
    mg = MG(OneLevel(A), precision="fp64")
    rng = np.random.default_rng(n)
    b = rng.standard_normal(n)
    y = mg.apply(0, 5, torch.as_tensor(b, device="cuda")).cpu().numpy()
    mg.close()
    ref = np.linalg.solve(A.toarray(), b)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    _say("  rel err", err)
    assert err <= 1e-11


def test_coarsest_singular_is_reported():
    from paper_1709_05660_amd import MG, FsiError
    A = saddle(301, 7).tolil()
    A[150, :] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    with pytest.raises(FsiError) as e:
        MG(OneLevel(A), precision="fp64")
    assert "coarsest" in str(e.value)


# FGMRES on a one-level hierarchy (the preconditioner is the exact inverse):
# n = 37 leaves most of the 256 row chunks of the Krylov reductions empty
@pytest.mark.parametrize("n,graph", [(37, False), (37, True), (301, True)])
def test_fgmres_one_level_small(n, graph):
    import torch

    from paper_1709_05660_amd import MG
    A = saddle(n, 500 + n)
    mg = MG(OneLevel(A), precision="fp64", use_graph=graph)
    rng = np.random.default_rng(n + 1)
    b = rng.standard_normal(n)
    x, info = mg.fgmres(torch.as_tensor(b, device="cuda"), rtol=1e-12)
    x = x.cpu().numpy()
    mg.close()
    ref = np.linalg.solve(A.toarray(), b)
    _say("one level", n, graph, info["iters"], info["true_relres"])
    assert info["status"] == 0 and info["converged"] == 1
    assert info["iters"] <= 2
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def with_diagonal_dofs(nf, nd, ndecoy, seed):
    """A saddle-point block on nf dofs, plus nd dofs whose row and column hold
    only a (nonzero, random) diagonal, plus ndecoy rows with a single
    diagonal entry whose column another row also uses (these belong to the
    dense part), all interleaved by a random permutation."""
    rng = np.random.default_rng(seed)
    parts = [saddle(nf, seed)] if nf else []
    if ndecoy:
        # decoy rows: [[a I, 0], [C, A_F]] stays nonsingular
        A_F = parts[0]
        Cc = sp.random(nf, ndecoy, density=min(1.0, 4.0 / nf), random_state=rng, format="csr")
        Cc = Cc + sp.csr_matrix((np.ones(ndecoy), (np.arange(ndecoy) % nf, np.arange(ndecoy))),
                                shape=(nf, ndecoy))
        top = sp.hstack([sp.diags(rng.uniform(1.0, 3.0, ndecoy)), sp.csr_matrix((ndecoy, nf))])
        parts = [sp.vstack([top, sp.hstack([Cc, A_F])]).tocsr()]
    dvals = rng.uniform(0.5, 2.0, nd) * rng.choice([-1.0, 1.0], nd)
    if nd:
        parts.append(sp.diags(dvals).tocsr())
    A = sp.block_diag(parts, format="csr")
    perm = rng.permutation(A.shape[0])
    A = A[perm][:, perm].tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("nf,nd,ndecoy", [(300, 100, 0), (700, 990, 37), (1100, 306, 0), (0, 64, 0)])
def test_coarsest_with_diagonal_only_dofs(nf, nd, ndecoy):
    """Dofs whose row and column hold only the diagonal are inverted by a
    reciprocal and the rest densely; decoy single-entry rows whose column
    is used elsewhere stay in the dense part."""
    import torch

    from paper_1709_05660_amd import MG
    A = with_diagonal_dofs(nf, nd, ndecoy, 900 + nf + nd)
    n = A.shape[0]
    _say("coarse with diagonal dofs", nf, nd, ndecoy, "n", n)
    mg = MG(OneLevel(A), precision="fp64")
    rng = np.random.default_rng(n)
    b = rng.standard_normal(n)
    y = mg.apply(0, 5, torch.as_tensor(b, device="cuda")).cpu().numpy()
    mg.close()
    ref = np.linalg.solve(A.toarray(), b)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    _say("  rel err", err)
    assert err <= 1e-11


def test_coarsest_zero_diagonal_only_dof_is_reported():
    from paper_1709_05660_amd import MG, FsiError
    A = with_diagonal_dofs(200, 40, 0, 77)
    colcnt = np.bincount(A.indices, minlength=A.shape[0])
    rows = [i for i in range(A.shape[0]) if A.indptr[i + 1] - A.indptr[i] == 1
            and A.indices[A.indptr[i]] == i and colcnt[i] == 1]
    assert len(rows) == 40
    A.data[A.indptr[rows[5]]] = 0.0     # a stored zero: still a diagonal-only dof
    with pytest.raises(FsiError) as e:
        MG(OneLevel(A), precision="fp64")
    assert "coarsest" in str(e.value)
