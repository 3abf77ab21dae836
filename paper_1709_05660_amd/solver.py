"""Python front end of the native FSI multigrid/FGMRES library.

PyTorch supplies device memory (tensors on cuda) and the HIP stream; every
step of the solve runs in the library's kernels.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _vec(t, n, name):
    """Device pointer of an FP64 vector of n entries, after checking that the
    tensor is what the library will read or write through it (the library
    sees only the pointer: a short, strided, host or FP32 tensor would be
    accessed out of bounds on the device)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: dtype must be float64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: expected {n} entries, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def stream_read_gbps(nbytes, reps=20, cold=False):
    """Best rate (GB/s) of the library's plain streaming-read kernel over
    nbytes of device memory, timed with events on the current stream: the
    read rate the HBM-bound kernels are compared with.  cold: each read
    follows a 512 MiB read of another buffer (outside the events), which
    evicts the data from the last-level cache."""
    import torch
    n = (nbytes // 16) * 2
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty(L.lib().fsi_stream_read_blocks(), dtype=torch.float64, device="cuda")
    flush = torch.ones(64 << 20, dtype=torch.float64, device="cuda") if cold else None
    st = torch.cuda.current_stream()
    best = None
    for r in range(reps + 3):
        if cold:
            flush.sum()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        L.check(L.lib().fsi_stream_read(_dptr(x), n, _dptr(out), C.c_void_p(st.cuda_stream)),
                "stream read")
        e1.record(st)
        e1.synchronize()
        if r >= 3:
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
    if abs(float(out.sum()) - n) > 1e-6 * n:
        raise RuntimeError("stream read returned a wrong sum")
    return n * 8 / (best * 1e-3) / 1e9


class Problem:
    """A generated multigrid hierarchy (host arrays owned by the native builder)."""

    def __init__(self, spec, coeffs):
        lib = L.lib()
        coeffs = np.asarray(coeffs, dtype=np.float64)
        kmax = coeffs.shape[1] if coeffs.ndim > 1 else int(round((coeffs.size / spec.dim) ** (1.0 / spec.dim)))
        if coeffs.size != spec.dim * kmax ** spec.dim:
            raise ValueError("coefficient array must hold dim * kmax^dim values")
        c = np.ascontiguousarray(coeffs).ravel()
        self._coeffs = c
        ps = L.ProblemSpecC()
        ps.dim, ps.nx, ps.ny, ps.nz = spec.dim, spec.nx, spec.ny, spec.nz
        ps.levels, ps.patch = spec.levels, spec.patch
        ps.lx, ps.ly, ps.lz = spec.lx, spec.ly, spec.lz
        for d in range(3):
            ps.solid_lo[d] = spec.solid_lo[d]
            ps.solid_hi[d] = spec.solid_hi[d]
        ps.rho, ps.mu, ps.mu_s, ps.u_peak, ps.amp = spec.rho, spec.mu, spec.mu_s, spec.u_peak, spec.amp
        ps.kmax = kmax
        ps.coeffs = L._ptr(c, C.c_double)
        ps.transient = 1 if getattr(spec, "transient", False) else 0
        ps.dt = getattr(spec, "dt", 0.0)
        ps.rho_s = getattr(spec, "rho_s", 0.0)
        ps.amp_d = getattr(spec, "amp_d", 0.0)
        h = C.c_void_p()
        st = lib.fsi_problem_build(C.byref(ps), C.byref(h))
        if st != 0:
            raise L.FsiError(st, "problem build failed: " + lib.fsi_problem_last_error().decode())
        self.h = h
        self.spec = spec
        self.nlevels = lib.fsi_problem_nlevels(h)
        self.levels = (L.LevelC * self.nlevels)()
        L.check(lib.fsi_problem_levels(h, self.levels), "levels")
        bp = C.POINTER(C.c_double)()
        yp = C.POINTER(C.c_double)()
        n = C.c_int64()
        L.check(lib.fsi_problem_vectors(h, C.byref(bp), C.byref(yp), C.byref(n)))
        self.n = n.value
        self.b = np.ctypeslib.as_array(bp, shape=(self.n,)).copy()
        self.y = np.ctypeslib.as_array(yp, shape=(self.n,)).copy()

    def dirichlet(self, level):
        fp = C.POINTER(C.c_uint8)()
        L.check(L.lib().fsi_problem_dirichlet(self.h, level, C.byref(fp)))
        n = self.levels[level].J.nrows
        return np.ctypeslib.as_array(fp, shape=(n,)).astype(bool)

    def csr(self, level, which="J"):
        """(rowptr, colind, val, shape) copies of J, P or R of a level."""
        A = getattr(self.levels[level], which)
        nnz = A.nnz
        rp = np.ctypeslib.as_array(A.rowptr, shape=(A.nrows + 1,)).copy()
        ci = np.ctypeslib.as_array(A.colind, shape=(max(nnz, 1),))[:nnz].copy()
        v = np.ctypeslib.as_array(A.val, shape=(max(nnz, 1),))[:nnz].copy()
        return rp, ci, v, (A.nrows, A.ncols)

    def patches(self, level):
        P = self.levels[level].patches
        ptr = np.ctypeslib.as_array(P.ptr, shape=(P.npatch + 1,)).copy()
        tot = int(ptr[-1])
        dof = np.ctypeslib.as_array(P.dof, shape=(tot,)).copy()
        owned = np.ctypeslib.as_array(P.owned, shape=(tot,)).copy()
        kind = np.ctypeslib.as_array(P.kind, shape=(P.npatch,)).copy()
        return ptr, dof, owned, kind

    def residual(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        r = np.empty(self.n)
        L.check(L.lib().fsi_problem_residual(self.h, y.ctypes.data_as(C.c_void_p),
                                             r.ctypes.data_as(C.c_void_p)))
        return r

    def close(self):
        if getattr(self, "h", None):
            L.lib().fsi_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mg_opts(nu_pre=2, nu_post=2, omega=0.7, precision="fp64", solid_precision=None,
            refine_sweeps=0, use_graph=False, tuning_db=None, fluid_ilu=False):
    o = L.MgOpts()
    o.fluid_ilu = 1 if fluid_ilu else 0
    o.nu_pre, o.nu_post, o.omega = nu_pre, nu_post, omega
    o.precision = L.PREC[precision]
    o.solid_precision = -1 if solid_precision is None else L.PREC[solid_precision]
    o.refine_sweeps = refine_sweeps
    o.use_graph = 1 if use_graph else 0
    o.tuning_db = tuning_db.encode() if tuning_db else None
    return o


def krylov_opts(restart=30, rtol=1e-10, maxit=1000, orth="cgs2", x0=False, history=None, fixed_iters=0,
                side="right"):
    ko = L.KrylovOpts()
    ko.restart, ko.rtol, ko.maxit = restart, rtol, maxit
    ko.orth = L.ORTH[orth]
    ko.x0_nonzero = 1 if x0 else 0
    ko.history = L._ptr(history, C.c_double) if history is not None else None
    ko.fixed_iters = fixed_iters
    ko.side = L.SIDE[side]
    return ko


class MG:
    """Device-resident multigrid hierarchy: V-cycle and FGMRES on the GPU."""

    def __init__(self, problem, **opts):
        import torch
        self.problem = problem       # keeps the host arrays alive during setup
        self.opts = mg_opts(**opts)
        h = C.c_void_p()
        st = L.lib().fsi_mg_setup(problem.levels, problem.nlevels, C.byref(self.opts), _stream(), C.byref(h))
        L.check(st, "fsi_mg_setup")
        self.h = h
        self.n = problem.n
        self.nlevels = problem.nlevels
        self.device = torch.device("cuda")

    def level_info(self, level):
        out = (C.c_int64 * 8)()
        L.check(L.lib().fsi_mg_level_info(self.h, level, out))
        return dict(zip(["n", "nnz", "npatch", "sum_m", "sum_m2", "sum_om", "nilu", "ilu_entries"], list(out)))

    def vcycle(self, r, z=None):
        import torch
        if z is None:
            z = torch.empty(self.n, dtype=torch.float64, device="cuda")
        L.check(L.lib().fsi_mg_vcycle(self.h, _vec(r, self.n, "r"), _vec(z, self.n, "z"), _stream()),
                "vcycle")
        return z

    @staticmethod
    def vcycle_batch(mgs, rs, zs=None):
        """z_i = M_i^{-1} r_i for several systems in batched launches
        (fsi_mg_vcycle_batch); each z_i equals mgs[i].vcycle(rs[i])."""
        import torch
        if not mgs or len(rs) != len(mgs) or (zs is not None and len(zs) != len(mgs)):
            raise ValueError("vcycle_batch: one r (and z) per handle")
        if zs is None:
            zs = [torch.empty(m.n, dtype=torch.float64, device="cuda") for m in mgs]
        hs = (C.c_void_p * len(mgs))(*[m.h.value for m in mgs])
        rp = (C.c_void_p * len(mgs))(*[_vec(r, m.n, "r").value for m, r in zip(mgs, rs)])
        zp = (C.c_void_p * len(mgs))(*[_vec(z, m.n, "z").value for m, z in zip(mgs, zs)])
        L.check(L.lib().fsi_mg_vcycle_batch(hs, len(mgs), rp, zp, _stream()), "vcycle_batch")
        return zs

    def apply(self, level, op, x, r=None, y=None):
        """One operator of a level (fsi_mg_apply): op 0 J x, 1 r - J x, 2 P x,
        3 R x, 4 one Schwarz application, 5 the coarsest direct solve."""
        import torch
        if not 0 <= level < self.nlevels:
            raise ValueError(f"level {level} out of range")
        n = self.level_info(level)["n"]
        nc = self.level_info(level - 1)["n"] if level > 0 else 0
        nin, nout = {2: (nc, n), 3: (n, nc)}.get(op, (n, n))
        if y is None:
            y = torch.empty(nout, dtype=torch.float64, device="cuda")
        rp = _vec(r, n, "r") if r is not None else None
        L.check(L.lib().fsi_mg_apply(self.h, level, op, _vec(x, nin, "x"), rp, _vec(y, nout, "y"),
                                     _stream()), "apply")
        return y

    def fgmres(self, b, x=None, restart=30, rtol=1e-10, maxit=1000, fixed_iters=0, x0=False,
               orth="cgs2", side="right"):
        """GMRES preconditioned by the V-cycle (fsi_fgmres_solve): side "right"
        is flexible GMRES stopping on |b - J x| <= rtol |b|; side "left" is the
        paper's left-preconditioned GMRES stopping on the preconditioned
        residual relative to its initial value.  Returns (x, info dict)."""
        import torch
        if x is None:
            if x0:
                raise ValueError("x0=True needs the starting vector x")
            x = torch.zeros(self.n, dtype=torch.float64, device="cuda")
        hist = np.zeros(maxit + 2)
        ko = krylov_opts(restart, rtol, maxit, orth, x0, hist, fixed_iters, side)
        info = L.SolveInfo()
        st = L.lib().fsi_fgmres_solve(self.h, _vec(b, self.n, "b"), _vec(x, self.n, "x"), C.byref(ko),
                                      C.byref(info), _stream())
        L.check(st, "fgmres")
        d = info.as_dict()
        d["status"] = st
        d["history"] = hist[: d["iters"] + 1].copy()
        return x, d

    def refactor(self):
        """Re-run extraction, block inversion and coarse inversion on the device."""
        L.check(L.lib().fsi_mg_refactor(self.h, _stream()), "refactor")

    def set_jvalues(self, level, values):
        """Copy a device FP64 tensor of nnz(J_level) values into the operator."""
        nnz = self.level_info(level)["nnz"]
        L.check(L.lib().fsi_mg_set_jvalues(self.h, level, _vec(values, nnz, "values"), _stream()), "set_jvalues")

    def galerkin(self):
        """Recompute the coarse operators R J P on the device from the finest values."""
        L.check(L.lib().fsi_mg_galerkin(self.h, _stream()), "galerkin")

    def autotune(self, db_path=None):
        """Pick SpMV lanes-per-row and the block-inversion panel width by timing;
        returns the number of new measurements (0 when db_path had them all)."""
        m = C.c_int32()
        L.check(L.lib().fsi_mg_autotune(self.h, db_path.encode() if db_path else None, _stream(),
                                        C.byref(m)), "autotune")
        return m.value

    def profile_start(self):
        L.check(L.lib().fsi_mg_profile(self.h, 1, None))

    def profile_stop(self):
        """(Schwarz ms, Schwarz launches, inversion ms, inversion launches) since profile_start."""
        out = (C.c_double * 4)()
        L.check(L.lib().fsi_mg_profile(self.h, 0, out))
        return out[0], int(out[1]), out[2], int(out[3])

    def export_patches(self, level, blocks=False):
        info = self.level_info(level)
        ptr = np.zeros(info["npatch"] + 1, np.int64)
        dof = np.zeros(info["sum_m"], np.int32)
        owned = np.zeros(info["sum_m"], np.uint8)
        B = np.zeros(info["sum_m2"]) if blocks else None
        L.check(L.lib().fsi_mg_export_patches(
            self.h, level, ptr.ctypes.data_as(C.c_void_p), dof.ctypes.data_as(C.c_void_p),
            owned.ctypes.data_as(C.c_void_p), B.ctypes.data_as(C.c_void_p) if blocks else None))
        return ptr, dof, owned, B

    def close(self):
        if getattr(self, "h", None):
            L.lib().fsi_mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (fsi_server_* of the C ABI).

    Requests are copied at submit; the server keeps admitted hierarchies on
    the device, admits in arrival order while the memory budget and a slot
    allow, and advances all active systems one FGMRES step per tick.  With
    batch_vcycles the V-cycles of the systems stepping in a tick run as
    batched launches (one per phase of the cycle) over all of them.
    """

    def __init__(self, hbm_budget_bytes=4 << 30, max_slots=16, device=0, batch_vcycles=False):
        so = L.ServerOpts(int(hbm_budget_bytes), int(max_slots), int(device), 1 if batch_vcycles else 0, 0)
        h = C.c_void_p()
        L.check(L.lib().fsi_server_create(C.byref(so), C.byref(h)), "server create")
        self.h = h
        self.sizes = {}

    def submit(self, problem, b=None, precision="bf16", rtol=1e-8, restart=30, maxit=1000, fixed_iters=0,
               **mg):
        b = problem.b if b is None else np.ascontiguousarray(b, dtype=np.float64)
        if b.shape != (problem.n,):
            raise ValueError(f"b: expected {problem.n} entries, got {b.shape}")
        mo = mg_opts(precision=precision, **mg)
        ko = krylov_opts(restart, rtol, maxit, fixed_iters=fixed_iters)
        t = C.c_uint64()
        L.check(L.lib().fsi_serve_submit(self.h, problem.levels, problem.nlevels,
                                         b.ctypes.data_as(C.c_void_p), C.byref(mo), C.byref(ko),
                                         C.byref(t)), "submit")
        self.sizes[t.value] = problem.n
        return t.value

    def poll(self, ticket):
        """(status, x, info); status 2 (pending) gives x = info = None."""
        n = self.sizes.get(ticket, 0)
        x = np.empty(max(n, 1))
        info = L.SolveInfo()
        st = L.lib().fsi_serve_poll(self.h, C.c_uint64(ticket), x.ctypes.data_as(C.c_void_p),
                                    C.byref(info))
        if st == L.FSI_PENDING:
            return st, None, None
        self.sizes.pop(ticket, None)
        if st < 0:
            return st, None, {"error": L.lib().fsi_last_error().decode()}
        return st, x[:n], info.as_dict()

    def stats(self):
        out = (C.c_int64 * 12)()
        L.check(L.lib().fsi_server_stats(self.h, out))
        keys = ["submitted", "finished", "active", "queued", "bytes_in_use", "peak_bytes", "ticks",
                "max_coresident", "pool_allocated_bytes", "pool_peak_in_use_bytes", "batched_groups",
                "batched_systems"]
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "h", None):
            L.lib().fsi_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Assembly:
    """Device assembly of a problem's finest residual and exact Jacobian
    (fsi_assembly_*), and Newton's method on the device (fsi_newton_solve)."""

    def __init__(self, problem):
        self.problem = problem
        ed = L.ElementData()
        L.check(L.lib().fsi_problem_element_data(problem.h, C.byref(ed)), "element data")
        self.ed = ed
        self.n = int(ed.ndof)
        J = problem.levels[problem.nlevels - 1].J
        self.nnz = int(J.nnz)
        h = C.c_void_p()
        L.check(L.lib().fsi_assembly_create(C.byref(ed), C.byref(J), _stream(), C.byref(h)), "assembly create")
        self.h = h

    def run(self, y, r=None, jval=None):
        """r = R(y) and the Jacobian's values at y (device float64 tensors)."""
        import torch
        if r is None:
            r = torch.empty(self.n, dtype=torch.float64, device="cuda")
        if jval is None:
            jval = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        L.check(L.lib().fsi_assembly_run(self.h, _vec(y, self.n, "y"), _vec(r, self.n, "r"),
                                         _vec(jval, self.nnz, "jval"), _stream()), "assembly run")
        return r, jval

    def newton(self, mg, y, max_newton=20, tol=1e-8, rtol=1e-8, restart=30, maxit=1000):
        """Newton's method on the device from y (updated in place); returns the info."""
        no = L.NewtonOpts(int(max_newton), float(tol))
        ko = krylov_opts(restart, rtol, maxit)
        info = L.NewtonInfo()
        st = L.lib().fsi_newton_solve(self.h, mg.h, _vec(y, self.n, "y"), C.byref(no), C.byref(ko),
                                      C.byref(info), _stream())
        L.check(st, "newton")
        return info.as_dict()

    def time_steps(self, mg, y, nsteps, max_newton=20, tol=1e-8, rtol=1e-8, restart=30, maxit=1000):
        """nsteps Crank-Nicolson steps from the state y (updated in place;
        fsi_cn_steps); returns (one Newton record per step, status: 0 when
        every step converged, 1 otherwise)."""
        no = L.NewtonOpts(int(max_newton), float(tol))
        ko = krylov_opts(restart, rtol, maxit)
        infos = (L.NewtonInfo * int(nsteps))()
        st = L.lib().fsi_cn_steps(self.h, mg.h, _vec(y, self.n, "y"), int(nsteps), C.byref(no), C.byref(ko), infos,
                                  _stream())
        L.check(st, "time steps")
        return [i.as_dict() for i in infos], st

    def close(self):
        if getattr(self, "h", None):
            L.lib().fsi_assembly_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fmg(assemblies, mgs, y0, bases=None, max_newton=20, tol=1e-8, rtol=1e-8, restart=30, maxit=1000):
    """Full multigrid on the device (fsi_fmg_solve): Newton on each nested
    mesh, coarsest first, each started from the prolongation of the mesh
    below.  assemblies, mgs: one per mesh; y0: the coarsest mesh's initial
    iterate (updated in place); bases: None or one state per mesh holding
    its Dirichlet values (the transfer is then base_j + P (y_{j-1} -
    base_{j-1})); max_newton: one limit for every mesh or a list per mesh.
    Returns (iterates per mesh, infos per mesh, status: 0 when the finest
    mesh converged, 1 otherwise)."""
    import torch
    n = len(assemblies)
    if n < 1 or len(mgs) != n:
        raise ValueError("one multigrid handle per assembly, at least one mesh")
    if bases is not None and len(bases) != n:
        raise ValueError("one base state per mesh")
    caps = list(max_newton) if isinstance(max_newton, (list, tuple)) else [int(max_newton)] * n
    if len(caps) != n:
        raise ValueError("one Newton step limit per mesh")
    ys = [y0] + [torch.empty(a.n, dtype=torch.float64, device="cuda") for a in assemblies[1:]]
    ah = (C.c_void_p * n)(*[a.h for a in assemblies])
    mh = (C.c_void_p * n)(*[m.h for m in mgs])
    yh = (C.c_void_p * n)(*[_vec(y, a.n, "y") for y, a in zip(ys, assemblies)])
    bh = None
    if bases is not None:
        bh = C.cast((C.c_void_p * n)(*[_vec(b, a.n, "base") for b, a in zip(bases, assemblies)]),
                    C.POINTER(C.c_void_p))
    ch = (C.c_int32 * n)(*caps)
    no = L.NewtonOpts(int(max(caps)), float(tol))
    ko = krylov_opts(restart, rtol, maxit)
    infos = (L.NewtonInfo * n)()
    st = L.lib().fsi_fmg_solve(n, C.cast(ah, C.POINTER(C.c_void_p)), C.cast(mh, C.POINTER(C.c_void_p)),
                               C.cast(yh, C.POINTER(C.c_void_p)), bh, ch, C.byref(no), C.byref(ko), infos,
                               _stream())
    L.check(st, "fmg")
    return ys, [i.as_dict() for i in infos], st
