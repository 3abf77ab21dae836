/*
 * fsi_mg.h -- C ABI of the MI355X (gfx950) linear-solve hot path of a
 * monolithic ALE Newton-Krylov FSI solver (Aulisa, Bna, Bornia, 2017).
 *
 * Solves J x = b, the linear system of one Newton step (section "Structure of
 * the Jacobian": J e = -r), with right-preconditioned flexible GMRES whose
 * preconditioner is one geometric multigrid V-cycle (section "Geometric
 * Multigrid preconditioner") with Galerkin coarse operators supplied by the
 * caller, a Richardson smoother preconditioned by restricted additive Schwarz
 * on element patches split along the fluid/solid interface (section
 * "Richardson-Schwarz smoother", B^{-1} = sum_k (R^0_k)^T B_k^{-1} R^delta_k)
 * and a direct solve on the coarsest level.
 *
 * Conventions
 *   - Every call returns fsi_status (0 = OK, > 0 informational, < 0 error).
 *     No C++ exception crosses the ABI.  fsi_last_error() gives a
 *     thread-local message for the last failure of the calling thread.
 *   - Host pointers are borrowed for the duration of the call only (copied).
 *   - Device pointers (suffix _dev) are borrowed and stream-ordered on the
 *     HIP stream passed in (NULL = the library's own stream of the handle).
 *   - Handles own all device memory they allocate; the library never frees
 *     caller memory.  One fsi_mg handle is used by one thread at a time.
 *   - Levels are indexed 0 = coarsest ... nlevels-1 = finest.
 *   - CSR: 0-based, int64 row offsets, int32 column indices strictly
 *     increasing within each row, FP64 values.
 */
#ifndef FSI_MG_H
#define FSI_MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSI_ABI_VERSION 4

typedef int32_t fsi_status;
enum {
  FSI_OK = 0,
  FSI_NOT_CONVERGED = 1,   /* iteration limit reached; x holds the last iterate */
  FSI_PENDING = 2,         /* serving: request not finished yet */
  FSI_E_INVALID = -1,      /* malformed input (message says which) */
  FSI_E_OOM = -2,          /* device allocation failed */
  FSI_E_SINGULAR = -3,     /* zero or non-finite pivot in a block or the coarse operator */
  FSI_E_DEVICE = -4,       /* HIP runtime error */
  FSI_E_NONFINITE = -5,    /* NaN/Inf in the right-hand side */
  FSI_E_CAPACITY = -6,     /* serving: request larger than the memory budget */
  FSI_E_UNKNOWN_TICKET = -7
};

/* Precision of the V-cycle (the Krylov method, the true residual and the
 * coarsest solve are always FP64).  FP64: blocks inverted and applied in
 * FP64.  MIXED_*: V-cycle vectors, operators and transfers in FP32; the
 * blocks are inverted in FP32 (Gauss-Jordan on the FP32 matrix cores) and
 * the owned rows of each inverse stored in the named 16-bit type with
 * two-sided FP32 scaling (B^{-1} = diag(rs) W diag(cs)) and applied with FP32
 * accumulation; MIXED_FP32: owned rows stored in FP32. */
enum { FSI_PREC_FP64 = 0, FSI_PREC_MIXED_BF16 = 1, FSI_PREC_MIXED_FP16 = 2, FSI_PREC_MIXED_FP32 = 3 };

/* Orthogonalisation of the Krylov basis: classical Gram-Schmidt applied
 * twice (the default) or once (the paper's PETSc setting, section "Details
 * on the iterative solver"). */
enum { FSI_ORTH_CGS2 = 0, FSI_ORTH_CGS = 1 };

/* Side of the preconditioner.  RIGHT: flexible GMRES (Saad) on J M^{-1},
 * the basis of preconditioned vectors z_j = M^{-1} v_j kept, stop when the
 * true residual |b - J x| <= rtol |b|.  LEFT: GMRES on M^{-1} J with the
 * paper's stopping rule |M^{-1}(b - J x_j)| < rtol |M^{-1}(b - J x_0)| on the
 * left-preconditioned residual (section "Details on the iterative solver";
 * the paper runs restart 10, FSI_ORTH_CGS, rtol 1e-4). */
enum { FSI_SIDE_RIGHT = 0, FSI_SIDE_LEFT = 1 };

typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;
  const int64_t *rowptr;   /* nrows+1 */
  const int32_t *colind;   /* nnz, strictly increasing per row, in [0, ncols) */
  const double *val;       /* nnz */
} fsi_csr;

/* Schwarz patches of one level (section "Richardson-Schwarz smoother"). */
typedef struct {
  int32_t npatch;
  const int64_t *ptr;      /* npatch+1 offsets into dof/owned */
  const int32_t *dof;      /* R^delta_k: dofs of patch k, strictly increasing */
  const uint8_t *owned;    /* 1 where patch k writes its result back (R^0_k); every
                              free dof owned by exactly one patch */
  const uint8_t *kind;     /* per patch: 0 fluid, 1 solid (precision policy) */
} fsi_patches;

typedef struct {
  fsi_csr J;               /* level operator (finest: exact Jacobian, coarser: R J P) */
  fsi_csr P;               /* n_l x n_{l-1} prolongation; ignored on level 0 */
  fsi_csr R;               /* n_{l-1} x n_l restriction; ignored on level 0 */
  fsi_patches patches;     /* ignored on level 0 (direct solve) */
  const uint8_t *dirichlet; /* optional (NULL: unchecked): n_l flags, 1 at a Dirichlet dof.
                              Checked at setup: a flagged row of J is the identity row
                              (its only entry is the diagonal, 1.0) and no patch holds
                              a flagged dof (the Newton correction is zero there) */
} fsi_level;

typedef struct {
  int32_t nu_pre, nu_post; /* Richardson sweeps before / after the coarse correction */
  double omega;            /* Richardson damping (the paper uses 0.7) */
  int32_t precision;       /* FSI_PREC_* */
  int32_t solid_precision; /* storage of the solid blocks' inverses (patch kind 1): -1 or
                              `precision` (every block alike), or FSI_PREC_MIXED_FP32 in a
                              mixed hierarchy (solid blocks in FP32, fluid blocks in
                              `precision`).  The paper requires exact local solves on the
                              solid blocks (section "Richardson-Schwarz smoother") */
  int32_t refine_sweeps;   /* 0..4, mixed hierarchies only: refinement sweeps of each solid
                              block's local solve, y <- y + B~^{-1}(g - B_k y) with the
                              FP32 inverse B~^{-1} (all its rows kept) and the block B_k
                              taken from J in FP32; fluid blocks are solved once */
  int32_t use_graph;       /* replay the V-cycle and each Arnoldi step from hipGraphs */
  const char *tuning_db;   /* NULL, or a text database path: setup then runs the
                              autotuner (fsi_mg_autotune) with it */
  int32_t fluid_ilu;       /* 0, or 1: the fluid blocks (patch kind 0) are solved with
                              ILU(0) factors (no pivoting, no fill beyond the block's
                              stored entries and its diagonal) instead of their exact
                              inverse; solid blocks stay exact.  Section "Richardson-
                              Schwarz smoother": an incomplete factorization suffices on
                              fluid subdomains.  Factored at every refactor (a zero pivot
                              fails it with FSI_E_SINGULAR); applied by forward and
                              backward substitution in the V-cycle's precision */
} fsi_mg_opts;

typedef struct {
  int32_t restart;         /* GMRES(m) restart length, 1..60 */
  double rtol;             /* relative tolerance (see FSI_SIDE_*) */
  int32_t maxit;           /* total preconditioner applications */
  int32_t orth;            /* FSI_ORTH_* */
  int32_t x0_nonzero;      /* 1: x_dev holds the initial guess; 0: x0 = 0 */
  double *history;         /* optional host buffer of maxit+1 residual norms: the initial
                              one, then each step's estimate (RIGHT: of |b - J x|,
                              LEFT: of |M^{-1}(b - J x)|) */
  int32_t fixed_iters;     /* > 0: run exactly this many iterations, ignore rtol */
  int32_t side;            /* FSI_SIDE_* */
} fsi_krylov_opts;

typedef struct {
  int32_t iters, restarts, converged;
  double true_relres;      /* |b - J x| / |b| of the returned x */
  double est_relres;       /* last monitored norm over the stopping rule's reference
                              (RIGHT: |b|, LEFT: |M^{-1}(b - J x_0)|) */
  double setup_ms, solve_ms;
  double rho;              /* average convergence rate (r_N / r_0)^(1/N) of the monitored
                              residual over the N iterations (defined with the tables of
                              section "Condition number estimates": the geometric mean
                              of the ratios of consecutive residuals); 0 when N = 0 */
} fsi_solve_info;

struct fsi_mg;

int32_t fsi_abi_version(void);
const char *fsi_status_string(fsi_status s);
const char *fsi_last_error(void);

/* Sections "Geometric Multigrid preconditioner" (levels, Galerkin coarse
 * operators, transfers) and "Richardson-Schwarz smoother" (blocks B_k =
 * R^delta_k J R^delta_k^T solved exactly, restricted write-back R^0_k).
 * Uploads the hierarchy, extracts B_k = J_l[I_k, I_k] for every patch, inverts
 * it (Gauss-Jordan, partial pivoting; the paper's local direct solve) keeping
 * the rows selected by R^0_k, and inverts the coarsest operator (its dofs
 * whose row and column hold only the diagonal, the eliminated Dirichlet dofs,
 * by a reciprocal, the others by Gauss-Jordan; the sparsity pattern decides,
 * so a refactor keeps the split).  Blocks of up to 800 dofs are inverted
 * together in one batched launch; larger ones (up to 6144 dofs, such as the
 * 3D 64-element patches) one after another, each by a chain of launches over
 * the whole device; ILU(0) blocks and blocks with refinement sweeps are
 * limited to 800 dofs.  levels: host array of nlevels views, coarsest first,
 * borrowed for the call; *out receives the handle (NULL on error).  Errors:
 * FSI_E_INVALID (malformed CSR/patch lists, a patch above its size limit,
 * dimension mismatch, owned sets not a partition of the covered dofs, a
 * Dirichlet flag on a non-identity row or inside a patch), FSI_E_SINGULAR
 * (message names level and patch), FSI_E_OOM, FSI_E_DEVICE. */
fsi_status fsi_mg_setup(const fsi_level *levels, int32_t nlevels, const fsi_mg_opts *opts,
                        void *hip_stream, struct fsi_mg **out);

/* Section "Geometric Multigrid preconditioner" (V-cycle, direct solve on the
 * coarsest level) with the smoother of section "Richardson-Schwarz
 * smoother": nu_pre sweeps e <- e + omega B^{-1}(r - J e) from e = 0, the
 * coarse correction e <- e + P V(R (r - J e)), nu_post sweeps.
 * z = M^{-1} r: r_dev, z_dev distinct or equal device arrays of n_finest
 * doubles, stream-ordered on hip_stream.  Errors: FSI_E_INVALID (null
 * argument), FSI_E_DEVICE (launch failure). */
fsi_status fsi_mg_vcycle(struct fsi_mg *mg, const double *r_dev, double *z_dev, void *hip_stream);

/* The V-cycles of count independent systems (the same section), each phase
 * of the cycle (Schwarz step, residual, transfer, coarsest solve of one
 * depth) as one batched launch over the systems that have it; each
 * z_dev[i] = M_i^{-1} r_dev[i] equals what fsi_mg_vcycle gives for system i
 * (the same arithmetic).  The handles must share nu_pre, nu_post, omega and
 * the V-cycle's precision class (FP64, or mixed with more than one level),
 * and r_dev[i] != z_dev[i]; a handle appears once (its level vectors are
 * the cycle's workspace); all on hip_stream (NULL: the first handle's
 * stream).  Errors: FSI_E_INVALID (null argument, count < 1, incompatible
 * or repeated handles, aliased vectors), FSI_E_DEVICE. */
fsi_status fsi_mg_vcycle_batch(struct fsi_mg *const *mgs, int32_t count, const double *const *r_dev,
                               double *const *z_dev, void *hip_stream);

/* Section "Details on the iterative solver" (GMRES preconditioned by one
 * V-cycle per step) for J_finest x = b, the linear system of a Newton step
 * (section "Structure of the Jacobian").  kopts->side picks flexible GMRES
 * with right preconditioning (default) or the paper's left-preconditioned
 * GMRES; kopts->orth the Gram-Schmidt variant.  b_dev, x_dev: device arrays
 * of n_finest doubles; x_dev holds x0 on entry when kopts->x0_nonzero, else
 * it is overwritten.  The call returns when the solve is over (the host
 * waits for each step's few result bytes).  Returns FSI_OK,
 * FSI_NOT_CONVERGED (maxit reached; x holds the last iterate) or an error:
 * FSI_E_INVALID (options), FSI_E_NONFINITE (NaN/Inf in b or a residual),
 * FSI_E_DEVICE.  info (may be NULL) is filled whenever the solve ran. */
fsi_status fsi_fgmres_solve(struct fsi_mg *mg, const double *b_dev, double *x_dev,
                            const fsi_krylov_opts *kopts, fsi_solve_info *info, void *hip_stream);

/* For callers that cannot allocate device memory while they solve (tight
 * serving loops, code that must not call hipMalloc): the same solve as
 * fsi_fgmres_solve (same kernels, same results, launched one by one, never
 * from graphs) whose Krylov buffers live in a static device workspace of
 * 64 MiB that the library holds on each device it runs on until the process
 * ends; the call itself allocates nothing (the handle took its pinned
 * result slot and event at setup).  The workspace takes
 * 8 (n (2 restart + 2) + O(restart^2) + 33,000) bytes, rounded per buffer:
 * up to about 130,000 unknowns at restart 30.  Larger requests return
 * FSI_E_CAPACITY with the sizes in the message.  Every call on a device
 * shares that device's workspace and leaves its contents behind (no buffer
 * needs to start at zero: every value is written before it is read in the
 * same call); calls that overlap on one device, from several threads or on
 * several streams, race and must be serialised by the caller.  The handle's
 * device must be current (else FSI_E_INVALID).  Other errors as
 * fsi_fgmres_solve. */
fsi_status fsi_fgmres_solve_noalloc(struct fsi_mg *mg, const double *b_dev, double *x_dev,
                                    const fsi_krylov_opts *kopts, fsi_solve_info *info,
                                    void *hip_stream);

/* Debug/parity: applies one operator of level `level` to x_dev (device, FP64):
 * op 0: y = J x;  1: y = r - J x (r_dev given);  2: y = P x;  3: y = R x;
 * 4: y = sum_k R^0_k^T B_k^{-1} R^delta_k x (one Schwarz application, FP64
 *    hierarchies); 5: y = coarsest direct solve of x (level 0);
 * 6: the Schwarz application as the V-cycle performs it in the hierarchy's
 *    precision (mixed: x rounded to FP32, the stored inverses, refined solid
 *    blocks, the result widened to FP64). */
fsi_status fsi_mg_apply(struct fsi_mg *mg, int32_t level, int32_t op, const double *x_dev,
                        const double *r_dev, double *y_dev, void *hip_stream);

/* Debug/parity: the patch lists as stored on the device (canonical order of
 * the input) and, when blocks != NULL, the dense FP64 blocks B_k extracted
 * on the device (row-major, concatenated, sum of m_k^2 doubles).  Host
 * buffers sized by the caller from fsi_mg_level_info. */
fsi_status fsi_mg_export_patches(struct fsi_mg *mg, int32_t level, int64_t *ptr, int32_t *dof,
                                 uint8_t *owned, double *blocks);

/* Section "Monolithic Newton-Krylov solver with Multigrid-Richardson-Schwarz
 * preconditioner": every Newton step brings a new Jacobian with the same
 * sparsity.  Recomputes the block inverses and the coarsest inverse from the
 * operator values resident on the device (written through fsi_mg_jvalues),
 * on hip_stream; returns when done.  Same errors as setup. */
fsi_status fsi_mg_refactor(struct fsi_mg *mg, void *hip_stream);

/* Device pointer to the FP64 values of J on `level` (the input CSR order),
 * owned by the handle; callers may overwrite them before fsi_mg_refactor. */
fsi_status fsi_mg_jvalues(struct fsi_mg *mg, int32_t level, double **val_dev);

/* Copies nnz(J_level) FP64 values (the input CSR order) from the device
 * array val_dev into the handle's operator of `level`, on hip_stream (the
 * caller keeps val_dev alive until the stream passes the copy).  Errors:
 * FSI_E_INVALID (bad argument), FSI_E_DEVICE. */
fsi_status fsi_mg_set_jvalues(struct fsi_mg *mg, int32_t level, const double *val_dev, void *hip_stream);

/* Section "Geometric Multigrid preconditioner" (Galerkin coarse operators,
 * section "Monolithic Newton-Krylov solver with Multigrid-Richardson-Schwarz
 * preconditioner": a new Jacobian every Newton step): recomputes every coarse
 * operator J_{l-1} = R_l J_l P_l on the device from the current finest values
 * (finest level first), on the coarse operators' given patterns, with a unit
 * diagonal on their Dirichlet rows (the input flags, else the rows whose only
 * entry is a unit diagonal).  A new Newton step then needs only the finest
 * values: fsi_mg_set_jvalues, fsi_mg_galerkin, fsi_mg_refactor.  The first
 * call builds, on the host from read-back patterns and the constant P and R
 * values, the intermediate pattern of J_l P_l and the list of every entry's
 * terms (device memory of about 12 bytes per term); every call is
 * stream-ordered on hip_stream and gives a row-by-column product's sums bit
 * for bit.
 * Errors: FSI_E_INVALID (R J P has an entry outside a given coarse pattern, or
 * a Dirichlet row holds no diagonal), FSI_E_OOM, FSI_E_DEVICE. */
fsi_status fsi_mg_galerkin(struct fsi_mg *mg, void *hip_stream);

/* Measurement hook: HIP events recorded at the own start and end of the
 * finest-level Schwarz kernel and of the batched block inversion, on the
 * streams they run on.  enable = 1 starts (V-cycles and Arnoldi steps then
 * run without graphs), enable = 0 stops and writes out[0] = total Schwarz
 * kernel milliseconds, out[1] = its launches, out[2] = total batched
 * inversion milliseconds, out[3] = its launches (out may be NULL). */
fsi_status fsi_mg_profile(struct fsi_mg *mg, int32_t enable, double out[4]);

/* Autotuner: times the lanes-per-row of every level's SpMV (J, P, R, in the
 * V-cycle's precision) and the panel width of the batched block inversion
 * with events on the stream, keeps the fastest, and persists the choices in
 * the text database db_path (may be NULL; entries found there are applied
 * without measuring).  *measured (may be NULL) = number of new measurements.
 * Captured graphs are rebuilt afterwards. */
fsi_status fsi_mg_autotune(struct fsi_mg *mg, const char *db_path, void *hip_stream,
                           int32_t *measured);

/* Sizes of level `level`: n, nnz(J), npatch, sum m_k, sum m_k^2, sum owned_k * m_k over the
 * blocks kept as explicit inverses, number of ILU blocks, their factor entries (L, U and the
 * diagonal; fluid_ilu). */
fsi_status fsi_mg_level_info(struct fsi_mg *mg, int32_t level, int64_t out[8]);

fsi_status fsi_mg_destroy(struct fsi_mg *mg);

/* Measurement helper, not part of the method: a plain streaming read of the
 * n doubles at x_dev (device memory, 16-byte aligned, n even and >= 2) on the
 * given stream, 16-byte loads, fsi_stream_read_blocks() workgroups of 256
 * threads each reading one contiguous chunk (the fastest read pattern
 * measured on this device); out_dev (device, fsi_stream_read_blocks() doubles, owned by the
 * caller) receives one partial sum per workgroup.  Timing it gives the read
 * rate the HBM-bound kernels are compared with.  FSI_E_INVALID on a bad size
 * or alignment; launch errors as FSI_E_DEVICE. */
fsi_status fsi_stream_read(const double *x_dev, int64_t n, double *out_dev, void *hip_stream);
int32_t fsi_stream_read_blocks(void);

/* ---------------------------------------------------------------- serving
 * A server keeps the hierarchies of admitted systems resident on the device,
 * admits queued requests in arrival order while their estimated device
 * footprint fits the budget and a slot is free, and advances every active
 * system by one FGMRES iteration as soon as its previous one has finished,
 * the systems' kernels overlapping on the device; a converged system is
 * retired (result copied to host, device memory returned to the server's
 * cache, released when the server is destroyed) and the next request
 * admitted.  With batch_vcycles the iterations advance in lockstep ticks:
 * the V-cycles of the systems at an Arnoldi step in a tick run together,
 * each phase of the cycle (Schwarz step, residual, transfer, coarsest solve
 * of one depth) as one batched launch over up to 16 systems with the same
 * smoothing options and V-cycle precision; each system's arithmetic is that
 * of its own V-cycle. */
typedef struct {
  int64_t hbm_budget_bytes; /* admission budget of device memory */
  int32_t max_slots;        /* maximum co-resident systems */
  int32_t device;           /* HIP device ordinal */
  int32_t batch_vcycles;    /* 0: each system's V-cycles on its own stream; 1: batched (lockstep ticks) */
  int32_t reserved;         /* must be 0 */
} fsi_server_opts;

struct fsi_server;

fsi_status fsi_server_create(const fsi_server_opts *o, struct fsi_server **out);
/* Section "Details on the iterative solver" applied to independent systems
 * (the paper solves one system at a time; serving them together is this
 * library's).  Copies the request (levels, b; mo->tuning_db is ignored) and
 * queues it; returns a ticket.  Errors at submit: FSI_E_INVALID (options,
 * level dimensions, row or patch offsets, patch dofs out of range;
 * ko->x0_nonzero must be 0), FSI_E_CAPACITY (the request's estimated
 * footprint exceeds the budget).  The entries themselves (column order and
 * range, patch partition, Dirichlet flags) are checked by the setup thread:
 * such a request fails alone and its poll returns FSI_E_INVALID. */
fsi_status fsi_serve_submit(struct fsi_server *s, const fsi_level *levels, int32_t nlevels,
                            const double *b_host, const fsi_mg_opts *mo, const fsi_krylov_opts *ko,
                            uint64_t *ticket);
/* FSI_PENDING until the request finished; then copies x (n_finest doubles) to
 * x_host and fills info; timing fields: setup_ms = queue + setup, solve_ms =
 * solve; returns the solve's status.  A finished ticket is released. */
fsi_status fsi_serve_poll(struct fsi_server *s, uint64_t ticket, double *x_host, fsi_solve_info *info);
/* Server counters: [0] submitted, [1] finished, [2] active, [3] queued,
 * [4] admitted footprint bytes, [5] peak admitted footprint bytes, [6] ticks,
 * [7] max co-resident, [8] device bytes the server's pool allocated (kept
 * until fsi_server_destroy), [9] peak device bytes handed out by the pool.
 * [10] batched V-cycle groups, [11] systems in them (batch_vcycles; the
 * mean batch is [11] / [10]).  The admitted footprint is an estimate that
 * includes the pool's rounding slack; [9] is what the systems actually held. */
fsi_status fsi_server_stats(struct fsi_server *s, int64_t out[12]);
fsi_status fsi_server_destroy(struct fsi_server *s);

#ifdef __cplusplus
}
#endif
#endif /* FSI_MG_H */
