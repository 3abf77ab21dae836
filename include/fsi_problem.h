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
/* The finest level's element data, for an assembler of the same residual
 * elsewhere (the device assembly of include/fsi_assembly.h); arrays owned by
 * the problem, valid until fsi_problem_destroy.  Local dofs of an element:
 * [d_c(a)] component-major, [u_c(a)], [p_j] (nl = 2 dim na + dim + 1); local
 * residual rows in the same order: [momentum_c(a)], [mesh motion (fluid) or
 * kinematics (solid)_c(a)], [continuity / incompressibility_j]. */
typedef struct {
  int32_t dim, ne, nl, na, np, nq, ncolor;
  int64_t ndof;
  const int32_t *l2g;         /* ne * nl: global dof of each local dof */
  const int32_t *tgt;         /* ne * nl: global row of each local residual row, -1 when dropped
                                 (mesh motion at an interface node of a fluid element) */
  const uint8_t *solid;       /* ne: 1 for a solid element */
  const int32_t *color_ptr;   /* ncolor + 1 offsets into color_elems */
  const int32_t *color_elems; /* ne element ids by colour; two elements of a colour share no node */
  const double *N, *dN, *psi, *w; /* quadrature: N[q na + a], dN[(q na + a) dim + k] (physical
                                     gradients on the structured mesh), psi[q np + j], w[q] */
  double vol;                 /* element volume (mesh-motion stiffness 1 / vol) */
  const uint8_t *dirichlet;   /* ndof flags */
  const double *dval;         /* ndof Dirichlet values */
  const double *y_prev;       /* ndof: the state at t_n of a time step, or NULL (steady) */
  double mu, rho, mu_s, dt, rho_s;
} fsi_element_data;
fsi_status fsi_problem_element_data(const struct fsi_problem *p, fsi_element_data *out);

fsi_status fsi_problem_destroy(struct fsi_problem *p);
/* thread-local message of the last failed fsi_problem_build of the calling thread */
const char *fsi_problem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSI_PROBLEM_H */
