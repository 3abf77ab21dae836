/*
 * fsi_problem.h -- host-side builder of the linear systems solved by fsi_mg.
 *
 * Generates, for a structured channel with a box-shaped solid clamped to the
 * bottom wall, the multigrid hierarchy of one Newton step of the steady
 * monolithic ALE FSI problem of Aulisa, Bna, Bornia (2017): the exact
 * Jacobian at a seeded state (section "Monolithic Newton-Krylov solver",
 * "Structure of the Jacobian", shuffled rows of equation jac_blocks_shuf),
 * natural-injection prolongations and equation-aware restrictions
 * (equations restr_blocks / prol_blocks), Galerkin coarse operators
 * J_{l-1} = R J_l P, Schwarz patches split along the fluid/solid interface
 * (section "Richardson-Schwarz smoother") and b = -r with zero Dirichlet rows.
 *
 * Discretisation: Q2 displacement/velocity, P1disc pressure (the paper's
 * Q2-P1disc pair), harmonic mesh motion with k = 1/V_el, incompressible
 * neo-Hookean solid sigma = -p I + mu_s F F^T, Newtonian fluid; steady, or
 * one Crank-Nicolson time step (spec.transient).
 * Dof order: d_c then u_c over the Q2 nodes (x fastest), then dim+1 pressure
 * dofs per element.  Dirichlet dofs are identity rows with dropped columns.
 *
 * The arrays are owned by the fsi_problem handle; the fsi_level views stay
 * valid until fsi_problem_destroy.  Errors: FSI_E_INVALID for an
 * inconsistent spec (mesh not divisible by 2^(levels-1) * patch, solid not
 * element-aligned on a level, ...).
 */
#ifndef FSI_PROBLEM_H
#define FSI_PROBLEM_H

#include <stdint.h>

#include "fsi_mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim;             /* 2 or 3 */
  int32_t nx, ny, nz;      /* finest-level elements (nz ignored in 2D) */
  int32_t levels;          /* multigrid levels */
  int32_t patch;           /* Schwarz block = patch^dim elements */
  double lx, ly, lz;       /* channel [0,lx] x [0,ly] (x [0,lz]) */
  double solid_lo[3], solid_hi[3];
  double rho, mu;          /* fluid density and viscosity */
  double mu_s;             /* solid shear modulus */
  double u_peak;           /* inflow peak velocity */
  double amp;              /* velocity perturbation amplitude */
  int32_t kmax;            /* Fourier modes per direction of the perturbation */
  const double *coeffs;    /* dim * kmax^dim coefficients in [-1,1], order (c, k, l[, m]) */
  /* One Crank-Nicolson time step (section "Discretization of the operator
   * formulation") instead of the steady problem when transient != 0: the
   * state at t_n is the seeded state, the Jacobian is taken at the Newton
   * iterate at t_{n+1} whose free displacements are moved by amp_d times the
   * normalised Fourier shape of the velocity perturbation. */
  int32_t transient;
  double dt;               /* time step */
  double rho_s;            /* solid density */
  double amp_d;            /* displacement increment of the iterate */
} fsi_problem_spec;

struct fsi_problem;

fsi_status fsi_problem_build(const fsi_problem_spec *spec, struct fsi_problem **out);
int32_t fsi_problem_nlevels(const struct fsi_problem *p);
/* levels[0] coarsest ... levels[nlevels-1] finest (views into the handle) */
fsi_status fsi_problem_levels(const struct fsi_problem *p, fsi_level *levels);
/* right-hand side b = -r(y) (finest size), the state y, the Dirichlet flags of level l */
fsi_status fsi_problem_vectors(const struct fsi_problem *p, const double **b, const double **y,
                               int64_t *n);
fsi_status fsi_problem_dirichlet(const struct fsi_problem *p, int32_t level, const uint8_t **flags);
/* residual of the finest level at state y (for tests): r (n doubles); for a
 * transient problem the state at t_n is the seeded one */
fsi_status fsi_problem_residual(const struct fsi_problem *p, const double *y, double *r);
fsi_status fsi_problem_destroy(struct fsi_problem *p);
/* thread-local message of the last failed fsi_problem_build of the calling thread */
const char *fsi_problem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSI_PROBLEM_H */
