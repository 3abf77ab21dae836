/* Device assembly and the Newton loop on the GPU (gfx950).
 *
 * Section "Monolithic Newton-Krylov solver with Multigrid-Richardson-Schwarz
 * preconditioner": every Newton step assembles the residual and the exact
 * Jacobian of the monolithic ALE system at the current iterate and solves
 * J e = -r with the multigrid-preconditioned Krylov method; the iteration
 * stops when |y^k - y^{k-1}| < tol |y^k|.  The residual is the one of section
 * "Discretization of the operator formulation" (steady, or one Crank-Nicolson
 * step), its Jacobian by forward-mode differentiation, element by element.
 *
 * The assembler takes the finest level's element data of include/fsi_problem.h
 * (any producer of that layout) and the finest Jacobian's CSR pattern; the
 * Newton loop drives an fsi_mg handle built for that pattern (its coarse
 * operators recomputed on the device by fsi_mg_galerkin at every step). */
#ifndef FSI_ASSEMBLY_H
#define FSI_ASSEMBLY_H

#include <stdint.h>

#include "fsi_mg.h"
#include "fsi_problem.h"

#ifdef __cplusplus
extern "C" {
#endif

struct fsi_assembly;

/* Uploads the element data and the pattern (host arrays, copied) on the
 * current HIP device.  J: the finest Jacobian's CSR (only rowptr, colind
 * and the sizes are read), holding every coupled entry of the element
 * residuals and the unit diagonal of every Dirichlet row.  Besides copies of
 * the inputs the assembler holds the CSR position of every element Jacobian
 * entry (4 * ne * nl^2 bytes: 25 MB for 4,096 2D elements, 226 MB for 2,048
 * 3D ones), found once here; the call returns after that work is done on
 * hip_stream.  Errors: FSI_E_INVALID (null or inconsistent sizes, dim not 2
 * or 3), FSI_E_OOM, FSI_E_DEVICE. */
fsi_status fsi_assembly_create(const fsi_element_data *ed, const fsi_csr *J, void *hip_stream,
                               struct fsi_assembly **out);

/* r = R(y) (ndof doubles) and the values of J = dR/dy in the pattern's order
 * (nnz doubles), all device arrays, stream-ordered on hip_stream.  Dirichlet
 * rows: r_i = y_i - g_i and a unit diagonal.  One launch per element colour:
 * the element residual's per-point coefficients differentiated along each
 * local dof (forward mode), then contracted with the test functions; every
 * entry is written by one thread per colour (no atomics, the same result
 * every run).
 * Errors: FSI_E_INVALID (null), FSI_E_DEVICE. */
fsi_status fsi_assembly_run(struct fsi_assembly *a, const double *y_dev, double *r_dev, double *jval_dev,
                            void *hip_stream);

typedef struct {
  int32_t max_newton;      /* Newton steps at most */
  double tol;              /* stop when |e| <= tol |y| (the paper: 1e-8) */
} fsi_newton_opts;

typedef struct {
  int32_t steps;           /* Newton steps taken */
  int32_t converged;       /* 1 when |e| <= tol |y| */
  int32_t krylov_iters;    /* Krylov iterations over all steps */
  double last_update;      /* |e| / |y| of the last step */
  double res0, res_last;   /* |r| at the start and before the last step */
} fsi_newton_info;

/* Newton's method for R(y) = 0 on the device, y_dev updated in place: per
 * step the device assembly at y, b = -r, the finest values into mg
 * (fsi_mg_set_jvalues), fsi_mg_galerkin, fsi_mg_refactor, the Krylov solve
 * of J e = b with kopts (x0 = 0), y += e.  The host reads norms only.  mg
 * must have been set up for the assembly's pattern.  Errors: those of the
 * calls it makes; FSI_NOT_CONVERGED when max_newton steps end above tol. */
fsi_status fsi_newton_solve(struct fsi_assembly *a, struct fsi_mg *mg, double *y_dev,
                            const fsi_newton_opts *nopts, const fsi_krylov_opts *kopts,
                            fsi_newton_info *info, void *hip_stream);

/* Time integration by Crank-Nicolson steps (section "Discretization of the
 * operator formulation": the time-discrete system of one step; section
 * "Details on the iterative solver": Newton's method in every step): nsteps
 * steps from the state in y_dev (device, ndof doubles, updated in place).
 * Each step makes the current state the assembly's state at t_n and runs
 * fsi_newton_solve (nopts, kopts) from it for the state at t_{n+1}.  The
 * assembly must have been created from a time step's element data (its
 * y_prev).  info (may be NULL) receives one record per step.  Returns FSI_OK
 * when every step converged, else FSI_NOT_CONVERGED after the first step that
 * did not (the records up to it filled).  Errors: FSI_E_INVALID (null
 * argument, nsteps < 1, a steady assembly), and those of the calls it makes. */
fsi_status fsi_cn_steps(struct fsi_assembly *a, struct fsi_mg *mg, double *y_dev, int32_t nsteps,
                        const fsi_newton_opts *nopts, const fsi_krylov_opts *kopts, fsi_newton_info *info,
                        void *hip_stream);

/* Full multigrid for the steady case (section "Monolithic Newton-Krylov
 * solver with Multigrid-Richardson-Schwarz preconditioner": Newton wrapped
 * in a full multigrid algorithm; section "Details on the iterative solver":
 * the Newton count reported is the finest mesh's).  nlev nested meshes,
 * coarsest first, each refining the one before; a[j] and mg[j] are mesh j's
 * assembly and multigrid handle, and for j > 0 mesh j-1 is the level below
 * the finest of mg[j] (the same dof numbering), so mg[j]'s finest
 * prolongation P maps mesh j-1's dofs to mesh j's.
 *   y_dev[0]   device, n_0 doubles: the coarsest mesh's initial iterate, on
 *              return its last iterate; y_dev[j], j > 0 (n_j doubles each):
 *              receive mesh j's iterates.
 *   base_dev   NULL, or nlev device vectors: a state of each mesh that holds
 *              its Dirichlet values (the seeded state, say).  The iterate of
 *              mesh j > 0 starts as base_j + P (y_{j-1} - base_{j-1}): P has
 *              zero columns at coarse Dirichlet dofs, and the difference is
 *              zero there, so no boundary data is lost (y_{j-1} is restored).
 *              NULL: P y_{j-1}.  In both cases the Dirichlet dofs are then
 *              set to their values.
 *   max_newton NULL, or nlev step limits (each >= 1); NULL: nopts->max_newton
 *              on every mesh.
 * Then Newton (fsi_newton_solve) from that iterate.  A mesh below the finest
 * that ends above tol is not an error: its iterate only starts the next mesh.
 * info (may be NULL) receives one record per mesh.  Stream-ordered on
 * hip_stream; the host reads norms only.  Returns FSI_OK when the finest mesh
 * converged, FSI_NOT_CONVERGED otherwise.  Errors: FSI_E_INVALID (nlev < 1, a
 * null handle or vector, a step limit below 1, handles whose sizes do not
 * chain as above), and those of the calls it makes. */
fsi_status fsi_fmg_solve(int32_t nlev, struct fsi_assembly *const *a, struct fsi_mg *const *mg,
                         double *const *y_dev, const double *const *base_dev, const int32_t *max_newton,
                         const fsi_newton_opts *nopts, const fsi_krylov_opts *kopts, fsi_newton_info *info,
                         void *hip_stream);

fsi_status fsi_assembly_destroy(struct fsi_assembly *a);

#ifdef __cplusplus
}
#endif
#endif /* FSI_ASSEMBLY_H */
