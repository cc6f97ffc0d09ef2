/*
 * lbm_ref.h -- FP64 CPU oracle of the axisymmetric double-population
 * (D2Q9 flow + D2Q4 temperature) lattice Boltzmann LES step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker for the HIP
 * implementation; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no header, table or helper
 * with the GPU library.
 *
 * What it computes (Djebali, Calve, Pateyron, El Ganaoui, Sammouda):
 *   - section 2.1, eq. (1): the two LBGK updates, with the axisymmetric
 *     source terms F1, F2 and S;
 *   - section 2.1, eq. (2): the macroscopic moments rho, u, T;
 *   - section 2.1, text after eq. (1): nu = (tau_nu - 1/2)/3,
 *     alpha = (tau_alpha - 1/2)/2 in lattice units;
 *   - section 2.2, eqs. (3)-(5): Smagorinsky closure, closed-form local
 *     relaxation time, turbulent diffusivity nu_t / Pr_t;
 *   - section 2.3, eq. (6): temperature-dependent nu(T), alpha(T), supplied
 *     here as multiplier tables on a uniform T grid;
 *   - section 2.4, eq. (7): inlet profiles, supplied as per-node inlet rows.
 * The source terms are not printed in the paper; the forms used are derived
 * from the axisymmetric incompressible Navier-Stokes and energy equations
 * (see the header of lbm_ref.c).
 *
 * Errors: every call returns 0 or a negative LBM_REF_E* code and never
 * prints or aborts.
 */
#ifndef LBM_REF_H
#define LBM_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_REF_OK = 0,
  LBM_REF_EINVAL = -1,
  LBM_REF_ENOMEM = -2,
  LBM_REF_EUNSTABLE = -3,
  LBM_REF_ESTATE = -5
};

/* Edge rules.  Sides are indexed 0 = x0 (i = -1), 1 = x1 (i = nx),
 * 2 = r0 (j = -1), 3 = r1 (j = nr). */
enum {
  LBM_REF_BC_INLET = 0,    /* x0 only: equilibrium ghost from the inlet row    */
  LBM_REF_BC_OUTFLOW = 1,  /* x1 only: zero-gradient copy of column nx-1       */
  LBM_REF_BC_PERIODIC = 2, /* x0 and x1 together                               */
  LBM_REF_BC_AXIS = 3,     /* r0 only, r0 == 0: half-way specular mirror       */
  LBM_REF_BC_FREESLIP = 4, /* r sides: half-way specular mirror                */
  LBM_REF_BC_WALL = 5,     /* any side: half-way bounce-back; thermal Dirichlet
                              (anti-bounce-back) unless wall_T is NaN          */
  LBM_REF_BC_EQ = 6        /* any side: equilibrium of eq_state[side]          */
};

typedef struct {
  int32_t nx, nr;             /* fluid nodes along x (axial) and r (radial)   */
  double r0;                  /* r_j = r0 + j + 1/2                            */
  double tau_nu, tau_alpha;   /* base relaxation times (table multiplier 1)    */
  double cs, delta, pr_t;     /* Smagorinsky constant, filter width, Pr_t      */
  int32_t table_n;            /* 0: constant properties, else >= 2 entries     */
  const double *nu_mult;      /* table_n multipliers of nu, copied             */
  const double *alpha_mult;   /* table_n multipliers of alpha, copied          */
  double t_lo, t_hi;          /* the tables span T in [t_lo, t_hi]             */
  int32_t bc[4];              /* LBM_REF_BC_* for x0, x1, r0, r1               */
  double wall_T[4];           /* Dirichlet T of a WALL side; NaN = adiabatic   */
  double eq_state[4][4];      /* EQ side state: rho, ux, ur, T                 */
  double body_force_x;        /* G: rho*G added to F_x                         */
  double rho0, ux0, ur0, T0;  /* uniform initial state                         */
  int32_t hoop;               /* 0: explicit -2 rho nu u_r / r^2;
                                 1: -2 rho nu u_r / (r^2 + 2 nu)               */
  int32_t threads;            /* OpenMP threads over radial rows; <= 0: default */
} lbm_ref_config;

typedef struct lbm_ref_handle lbm_ref_handle;

int lbm_ref_create(const lbm_ref_config *cfg, lbm_ref_handle **out);
void lbm_ref_destroy(lbm_ref_handle *h);
/* n_t rows of nr values each (row-major); step s uses row s mod n_t. */
int lbm_ref_set_inlet(lbm_ref_handle *h, int32_t n_t, const double *ux,
                      const double *ur, const double *T);
int lbm_ref_step(lbm_ref_handle *h, int64_t n_steps);
int64_t lbm_ref_step_count(const lbm_ref_handle *h);
/* Pre-collision moments at the current step: each nr*nx, i fastest.  NULL skips. */
int lbm_ref_moments(lbm_ref_handle *h, double *rho, double *ux, double *ur, double *T);
/* Sum_ij r_j rho_ij and Sum_ij r_j T_ij of the same moments. */
int lbm_ref_conservation(lbm_ref_handle *h, double *mass3d, double *energy3d);
/* Centreline (j = 0) u_x and T (nx each); exit column (i = nx-1) u_x, T (nr each). */
int lbm_ref_profiles(lbm_ref_handle *h, double *ux_axis, double *T_axis,
                     double *ux_exit, double *T_exit);
/* Equilibrium fill from fields (each nr*nx); clears the unstable flag. */
int lbm_ref_set_state(lbm_ref_handle *h, const double *rho, const double *ux,
                      const double *ur, const double *T);
/* Stored post-collision populations: f is 9*nr*nx, g is 4*nr*nx, k slowest. */
int lbm_ref_get_populations(const lbm_ref_handle *h, double *f, double *g);
int lbm_ref_set_populations(lbm_ref_handle *h, const double *f, const double *g,
                            int64_t step);

/* Node-level pieces, exported for unit checks. */
void lbm_ref_feq(double rho, double ux, double ur, double out[9]);
void lbm_ref_geq(double T, double ux, double ur, double out[4]);
double lbm_ref_table_lookup(const double *tab, int32_t n, double t_lo,
                            double t_hi, double T);
/* One collision of the pre-collision populations f, g of a node at radius r.
 * diag (may be NULL) receives, in order: rho, ux, ur, T, nu, alpha, tau_nu(T),
 * Qxx, Qxr, Qrr, |Q|, tau_tot, nu_tot, nu_t, alpha_tot, tau_alpha_tot, theta,
 * F_x, F_r, S (20 values). */
int lbm_ref_collide_node(const lbm_ref_handle *h, const double f[9],
                         const double g[4], double r, double fout[9],
                         double gout[4], double diag[20]);

#ifdef __cplusplus
}
#endif
#endif
