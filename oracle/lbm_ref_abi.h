/*
 * lbm_ref_abi.h -- the solver C-ABI (lbm_create, lbm_set_inlet, lbm_step,
 * lbm_moments, lbm_destroy and the state extras) as exported by the FP64
 * oracle library, liblbm_ref.so.
 *
 * TEST INFRASTRUCTURE ONLY: the checker of the HIP implementation.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * this library.
 *
 * The GPU library exports the same names with the same argument lists, so one
 * test body can drive either library.  This header is written on its own (it
 * includes nothing of the GPU library); its struct and enum values match the
 * GPU library's by contract, and a CPU test checks the match by driving the
 * oracle through both this ABI and its own lbm_ref_* calls.
 *
 * Differences from the GPU library: precision must be LBM_PREC_FP64 (the
 * oracle computes in FP64 only); rho_ref and g_ref are ignored; layout is
 * accepted (0 or 1) and ignored (the oracle keeps two FP64 buffers); the
 * calls are synchronous.
 */
#ifndef LBM_REF_ABI_H
#define LBM_REF_ABI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2u

enum { LBM_OK = 0, LBM_EINVAL = -1, LBM_ENOMEM = -2, LBM_EUNSTABLE = -3,
       LBM_EDEVICE = -4, LBM_ESTATE = -5 };
enum { LBM_PREC_FP64 = 0 };

typedef struct lbm_handle lbm_handle;

typedef struct {
  uint32_t abi_version;
  int32_t nx, nr;
  double r0;
  double tau_nu, tau_alpha;
  double cs, delta, pr_t;
  int32_t table_n;
  const double *nu_mult;
  const double *alpha_mult;
  double t_lo, t_hi;
  int32_t bc[4];
  double wall_T[4];
  double eq_state[4][4];
  double body_force_x;
  double rho0, ux0, ur0, T0;
  int32_t hoop;
  int32_t precision;
  double rho_ref, g_ref;
  int32_t layout;
} lbm_config;

int lbm_create(const lbm_config *cfg, lbm_handle **out);
int lbm_set_inlet(lbm_handle *h, int32_t n_t, const double *ux, const double *ur,
                  const double *T);
int lbm_step(lbm_handle *h, int64_t n_steps);
int lbm_moments(lbm_handle *h, double *rho, double *ux, double *ur, double *T);
void lbm_destroy(lbm_handle *h);

int64_t lbm_step_count(const lbm_handle *h);
int lbm_sync(lbm_handle *h);
int lbm_set_state(lbm_handle *h, const double *rho, const double *ux, const double *ur,
                  const double *T);
int lbm_get_populations(lbm_handle *h, double *f, double *g);
int lbm_set_populations(lbm_handle *h, const double *f, const double *g, int64_t step);
int lbm_conservation(lbm_handle *h, double *mass3d, double *energy3d);
int lbm_profiles(lbm_handle *h, double *ux_axis, double *T_axis, double *ux_exit,
                 double *T_exit);
const char *lbm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
