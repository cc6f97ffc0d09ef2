/*
 * lbm_ref_abi.c -- the solver C-ABI exported by the FP64 oracle library:
 * argument-translating adapters over the lbm_ref_* calls of lbm_ref.c.
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_ref_abi.h).  No arithmetic of the method
 * lives here: each call checks the ABI fields the oracle cannot honour,
 * copies the configuration field by field into the oracle's own structure
 * and forwards.
 */
#include "lbm_ref_abi.h"

#include <stdlib.h>

#include "lbm_ref.h"

struct lbm_handle {
  lbm_ref_handle *ref;
};

int lbm_create(const lbm_config *cfg, lbm_handle **out) {
  if (!out) return LBM_EINVAL;
  *out = NULL;
  if (!cfg || cfg->abi_version != LBM_ABI_VERSION || cfg->precision != LBM_PREC_FP64 ||
      (cfg->layout != 0 && cfg->layout != 1))
    return LBM_EINVAL;
  lbm_ref_config c;
  c.nx = cfg->nx;
  c.nr = cfg->nr;
  c.r0 = cfg->r0;
  c.tau_nu = cfg->tau_nu;
  c.tau_alpha = cfg->tau_alpha;
  c.cs = cfg->cs;
  c.delta = cfg->delta;
  c.pr_t = cfg->pr_t;
  c.table_n = cfg->table_n;
  c.nu_mult = cfg->nu_mult;
  c.alpha_mult = cfg->alpha_mult;
  c.t_lo = cfg->t_lo;
  c.t_hi = cfg->t_hi;
  for (int s = 0; s < 4; ++s) {
    c.bc[s] = cfg->bc[s];
    c.wall_T[s] = cfg->wall_T[s];
    for (int q = 0; q < 4; ++q) c.eq_state[s][q] = cfg->eq_state[s][q];
  }
  c.body_force_x = cfg->body_force_x;
  c.rho0 = cfg->rho0;
  c.ux0 = cfg->ux0;
  c.ur0 = cfg->ur0;
  c.T0 = cfg->T0;
  c.hoop = cfg->hoop;
  c.threads = 0;
  lbm_handle *h = (lbm_handle *)calloc(1, sizeof *h);
  if (!h) return LBM_ENOMEM;
  const int rc = lbm_ref_create(&c, &h->ref);
  if (rc != LBM_REF_OK) {
    free(h);
    return rc;
  }
  *out = h;
  return LBM_OK;
}

void lbm_destroy(lbm_handle *h) {
  if (!h) return;
  lbm_ref_destroy(h->ref);
  free(h);
}

int lbm_set_inlet(lbm_handle *h, int32_t n_t, const double *ux, const double *ur,
                  const double *T) {
  return h ? lbm_ref_set_inlet(h->ref, n_t, ux, ur, T) : LBM_EINVAL;
}

int lbm_step(lbm_handle *h, int64_t n_steps) {
  return h ? lbm_ref_step(h->ref, n_steps) : LBM_EINVAL;
}

int lbm_moments(lbm_handle *h, double *rho, double *ux, double *ur, double *T) {
  return h ? lbm_ref_moments(h->ref, rho, ux, ur, T) : LBM_EINVAL;
}

int64_t lbm_step_count(const lbm_handle *h) { return h ? lbm_ref_step_count(h->ref) : -1; }

int lbm_sync(lbm_handle *h) { return h ? LBM_OK : LBM_EINVAL; }

int lbm_set_state(lbm_handle *h, const double *rho, const double *ux, const double *ur,
                  const double *T) {
  return h ? lbm_ref_set_state(h->ref, rho, ux, ur, T) : LBM_EINVAL;
}

int lbm_get_populations(lbm_handle *h, double *f, double *g) {
  return h ? lbm_ref_get_populations(h->ref, f, g) : LBM_EINVAL;
}

int lbm_set_populations(lbm_handle *h, const double *f, const double *g, int64_t step) {
  return h ? lbm_ref_set_populations(h->ref, f, g, step) : LBM_EINVAL;
}

int lbm_conservation(lbm_handle *h, double *mass3d, double *energy3d) {
  return h ? lbm_ref_conservation(h->ref, mass3d, energy3d) : LBM_EINVAL;
}

int lbm_profiles(lbm_handle *h, double *ux_axis, double *T_axis, double *ux_exit,
                 double *T_exit) {
  return h ? lbm_ref_profiles(h->ref, ux_axis, T_axis, ux_exit, T_exit) : LBM_EINVAL;
}

const char *lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument or configuration";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EUNSTABLE: return "unstable: non-finite value or non-positive density";
    case LBM_ESTATE: return "call not valid in the current state";
    default: return "unknown error";
  }
}
