/*
 * lbm_ref.c -- FP64 CPU oracle of the axisymmetric D2Q9 + D2Q4 LBGK-LES step.
 *
 * TEST INFRASTRUCTURE ONLY: the checker of the HIP path.  Plain, slow and
 * written to be read against the paper: one function per step of the method,
 * in the order the paper states it.  Build: -O2 -ffp-contract=off, optional
 * OpenMP over radial rows (a step has no reductions except the stability
 * flag, so results do not depend on the thread count).
 *
 * Paper: Djebali, Calve, Pateyron, El Ganaoui, Sammouda, "Les methodes de
 * resolution de type lattice Boltzmann sont-elles utilisables pour simuler
 * les jets plasmas souffles atmospheriques utilises en projection ?".
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *  - Equilibria (named in the nomenclature, not printed): standard
 *    second-order D2Q9 form, c_s^2 = 1/3, and first-order D2Q4 form,
 *    c_s^2 = 1/2, which are the lattice speeds implied by the relations
 *    nu = (tau-1/2)/3 and alpha = (tau-1/2)/2 given after eq. (1).
 *  - F1 (eq. 1, added to all nine links): read as w_k * theta with
 *    theta = -rho u_r / r, so that the links sum to the axisymmetric mass
 *    source of the continuity equation written in (x, r).
 *  - F2 (eq. 1, weighted by e_ki / 6; sum_k e_kx^2 = 6 on D2Q9 so the links
 *    sum to F): the axisymmetric momentum source
 *      F_i = -rho u_i u_r / r + (rho nu / r)(d_r u_i + d_i u_r)
 *            - 2 rho nu u_r / r^2 delta_ir
 *    with the strain taken from the node's non-equilibrium stress,
 *    rho nu (d_a u_b + d_b u_a) = -(1 - 1/(2 tau)) Q_ab, and nu = nu_tot.
 *  - S (eq. 1, added to all four links): read as S/4 per link with
 *      S = -T u_r / r + (alpha / r) d_r T,
 *    alpha d_r T = -(1 - 1/(2 tau_alpha)) sum_k e_kr (g_k - g_k^eq),
 *    alpha = alpha_tot.
 *  - |Q_ij| in eq. (4): sqrt(2 Q:Q) over xx, xr (twice), rr.
 *  - tau_nu in eq. (4) is the node's tau_nu(T) = 1/2 + 3 nu(T) (section 2.3).
 *  - Node centres at r_j = r0 + j + 1/2, so a symmetry axis at r = 0 is a
 *    half-way specular mirror and 1/r <= 2.
 *  - Hoop term near the axis: explicit (hoop = 0) or, as a stabilised
 *    variant, -2 rho nu u_r / (r^2 + 2 nu) (hoop = 1).
 *  - Edges (Fig. 1 is missing): equilibrium inlet ghost (rho = 1), zero-
 *    gradient outflow, half-way specular axis and free-slip, half-way bounce-
 *    back walls with anti-bounce-back for a Dirichlet temperature.  Corners:
 *    the r-side rule is applied first; a mirrored pull then goes through the
 *    x-side rule at the edge row.
 */
#include "lbm_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattices ------------------------------------------------------------
 * D2Q9, links k = 0..8 of eq. (1) line 1, as (e_x, e_r). */
static const int EX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int ER9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};  /* -e_k        */
static const int MIR9[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};  /* e_r -> -e_r */
/* D2Q4, the paper's k = 1..4 of eq. (1) line 2, stored as 0..3. */
static const int EX4[4] = {1, 0, -1, 0};
static const int ER4[4] = {0, 1, 0, -1};
static const int OPP4[4] = {2, 3, 0, 1};
static const int MIR4[4] = {0, 3, 2, 1};

enum { FLOW = 0, HEAT = 1 };
enum { SX0 = 0, SX1 = 1, SR0 = 2, SR1 = 3 };

struct lbm_ref_handle {
  lbm_ref_config c;
  double nu0, alpha0; /* base nu and alpha, relations after eq. (1) */
  double *tab_nu, *tab_alpha;
  double *f[2], *g[2];
  int cur;
  int64_t step;
  int32_t n_t;
  double *in_ux, *in_ur, *in_T;
  int unstable;
};

/* ---- equilibria (nomenclature; moments fixed by eq. 2) ------------------- */
void lbm_ref_feq(double rho, double ux, double ur, double out[9]) {
  double uu = ux * ux + ur * ur;
  for (int k = 0; k < 9; ++k) {
    double eu = EX9[k] * ux + ER9[k] * ur;
    out[k] = W9[k] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

void lbm_ref_geq(double T, double ux, double ur, double out[4]) {
  for (int k = 0; k < 4; ++k) {
    double eu = EX4[k] * ux + ER4[k] * ur;
    out[k] = 0.25 * T * (1.0 + 2.0 * eu);
  }
}

/* ---- eq. (6): property multiplier, linear on a uniform grid, clamped ---- */
double lbm_ref_table_lookup(const double *tab, int32_t n, double t_lo,
                            double t_hi, double T) {
  if (n <= 0 || tab == NULL) return 1.0;
  double x = (T - t_lo) / (t_hi - t_lo);
  if (!(x > 0.0)) x = 0.0; /* also maps NaN to the first entry */
  if (x > 1.0) x = 1.0;
  double sigma = x * (double)(n - 1);
  int i0 = (int)floor(sigma);
  if (i0 > n - 2) i0 = n - 2;
  double w = sigma - (double)i0;
  return (1.0 - w) * tab[i0] + w * tab[i0 + 1];
}

/* ---- one collision: eqs. (2), (4), (5), (6), then the right side of (1) -- */
int lbm_ref_collide_node(const lbm_ref_handle *h, const double f[9],
                         const double g[4], double r, double fout[9],
                         double gout[4], double diag[20]) {
  const lbm_ref_config *c = &h->c;

  /* eq. (2): rho, u, T */
  double rho = 0.0, mx = 0.0, mr = 0.0, T = 0.0;
  for (int k = 0; k < 9; ++k) {
    rho += f[k];
    mx += EX9[k] * f[k];
    mr += ER9[k] * f[k];
  }
  for (int k = 0; k < 4; ++k) T += g[k];
  double ux = mx / rho, ur = mr / rho;

  double feq[9], geq[4];
  lbm_ref_feq(rho, ux, ur, feq);
  lbm_ref_geq(T, ux, ur, geq);

  /* eq. (6) and the relations after eq. (1): nu(T), alpha(T), tau_nu(T) */
  double nu = h->nu0 * lbm_ref_table_lookup(h->tab_nu, c->table_n, c->t_lo,
                                            c->t_hi, T);
  double alpha = h->alpha0 * lbm_ref_table_lookup(h->tab_alpha, c->table_n,
                                                  c->t_lo, c->t_hi, T);
  double tau_nu = 0.5 + 3.0 * nu;

  /* eq. (4): Q_ij from the pre-collision populations */
  double qxx = 0.0, qxr = 0.0, qrr = 0.0;
  for (int k = 0; k < 9; ++k) {
    double fn = f[k] - feq[k];
    qxx += EX9[k] * EX9[k] * fn;
    qxr += EX9[k] * ER9[k] * fn;
    qrr += ER9[k] * ER9[k] * fn;
  }
  double qnorm = sqrt(2.0 * (qxx * qxx + 2.0 * qxr * qxr + qrr * qrr));
  double csd = c->cs * c->delta;
  double tau = 0.5 * (tau_nu + sqrt(tau_nu * tau_nu + 18.0 * csd * csd * qnorm / rho));

  /* eq. (3) and (5): nu_tot, nu_t, alpha_tot, tau_alpha_tot */
  double nu_tot = (tau - 0.5) / 3.0;
  double nu_t = nu_tot - nu;
  double alpha_tot = alpha + nu_t / c->pr_t;
  double tau_a = 0.5 + 2.0 * alpha_tot;

  /* axisymmetric sources F1 (theta), F2 = (F_x, F_r), S */
  double theta = -rho * ur / r;
  double kv = 1.0 - 1.0 / (2.0 * tau);
  double hoop_den = (c->hoop == 1) ? (r * r + 2.0 * nu_tot) : (r * r);
  double Fx = -rho * ux * ur / r - kv * qxr / r + rho * c->body_force_x;
  double Fr = -rho * ur * ur / r - kv * qrr / r - 2.0 * rho * nu_tot * ur / hoop_den;
  double jr_neq = (g[1] - geq[1]) - (g[3] - geq[3]); /* sum_k e_kr g^neq */
  double ka = 1.0 - 1.0 / (2.0 * tau_a);
  double S = -T * ur / r - ka * jr_neq / r;

  /* eq. (1), right-hand sides */
  for (int k = 0; k < 9; ++k)
    fout[k] = f[k] - (f[k] - feq[k]) / tau + W9[k] * theta +
              (EX9[k] * Fx + ER9[k] * Fr) / 6.0;
  for (int k = 0; k < 4; ++k)
    gout[k] = g[k] - (g[k] - geq[k]) / tau_a + 0.25 * S;

  if (diag) {
    double d[20] = {rho,   ux,    ur,     T,         nu,  alpha, tau_nu,
                    qxx,   qxr,   qrr,    qnorm,     tau, nu_tot, nu_t,
                    alpha_tot, tau_a, theta, Fx,     Fr,  S};
    memcpy(diag, d, sizeof d);
  }
  return LBM_REF_OK;
}

/* ---- streaming: value pulled by node (i, j) along link k ----------------- */
static inline size_t idx(const lbm_ref_handle *h, int k, int i, int j) {
  return ((size_t)k * (size_t)h->c.nr + (size_t)j) * (size_t)h->c.nx + (size_t)i;
}

static inline double stored(const lbm_ref_handle *h, int P, int k, int i, int j) {
  return (P == FLOW ? h->f[h->cur] : h->g[h->cur])[idx(h, k, i, j)];
}

static inline double eq_link(int P, int k, double rho, double ux, double ur,
                             double T) {
  if (P == FLOW) {
    double e[9];
    lbm_ref_feq(rho, ux, ur, e);
    return e[k];
  }
  double e[4];
  lbm_ref_geq(T, ux, ur, e);
  return e[k];
}

/* half-way bounce-back at node (i, j): the node's own opposite population;
 * for g with a Dirichlet wall temperature, anti-bounce-back. */
static double bounce(const lbm_ref_handle *h, int P, int k, int i, int j, int side) {
  int kk = (P == FLOW) ? OPP9[k] : OPP4[k];
  double v = stored(h, P, kk, i, j);
  double tw = h->c.wall_T[side];
  if (P == HEAT && !isnan(tw)) v = -v + 2.0 * 0.25 * tw;
  return v;
}

/* x-side rule for population k taken from column ip of row jr; (i_land,
 * j_land) is the node that receives it (the pulling node, or for a mirrored
 * pull the node of the edge row). */
static double pull_x(const lbm_ref_handle *h, int P, int k, int ip, int jr,
                     int i_land, int j_land) {
  const lbm_ref_config *c = &h->c;
  if (ip >= 0 && ip < c->nx) return stored(h, P, k, ip, jr);
  int side = ip < 0 ? SX0 : SX1;
  switch (c->bc[side]) {
    case LBM_REF_BC_PERIODIC:
      return stored(h, P, k, ((ip % c->nx) + c->nx) % c->nx, jr);
    case LBM_REF_BC_OUTFLOW:
      return stored(h, P, k, c->nx - 1, jr);
    case LBM_REF_BC_INLET: {
      /* eq. (7) profiles enter as inlet rows; ghost at equilibrium, rho = 1 */
      size_t row = (size_t)(h->step % h->n_t) * (size_t)c->nr + (size_t)jr;
      return eq_link(P, k, 1.0, h->in_ux[row], h->in_ur[row], h->in_T[row]);
    }
    case LBM_REF_BC_WALL:
      return bounce(h, P, k, i_land, j_land, side);
    case LBM_REF_BC_EQ: {
      const double *e = c->eq_state[side];
      return eq_link(P, k, e[0], e[1], e[2], e[3]);
    }
  }
  return NAN;
}

static double pull(const lbm_ref_handle *h, int P, int k, int i, int j) {
  const lbm_ref_config *c = &h->c;
  int ex = (P == FLOW) ? EX9[k] : EX4[k];
  int er = (P == FLOW) ? ER9[k] : ER4[k];
  int ip = i - ex, jp = j - er;
  if (jp >= 0 && jp < c->nr) return pull_x(h, P, k, ip, jp, i, j);
  int side = jp < 0 ? SR0 : SR1;
  int jedge = jp < 0 ? 0 : c->nr - 1;
  switch (c->bc[side]) {
    case LBM_REF_BC_AXIS:
    case LBM_REF_BC_FREESLIP: {
      int km = (P == FLOW) ? MIR9[k] : MIR4[k];
      return pull_x(h, P, km, ip, jedge, i, jedge);
    }
    case LBM_REF_BC_WALL:
      return bounce(h, P, k, i, j, side);
    case LBM_REF_BC_EQ: {
      const double *e = c->eq_state[side];
      return eq_link(P, k, e[0], e[1], e[2], e[3]);
    }
  }
  return NAN;
}

static void pull_node(const lbm_ref_handle *h, int i, int j, double f[9], double g[4]) {
  for (int k = 0; k < 9; ++k) f[k] = pull(h, FLOW, k, i, j);
  for (int k = 0; k < 4; ++k) g[k] = pull(h, HEAT, k, i, j);
}

static inline double radius(const lbm_ref_handle *h, int j) {
  return h->c.r0 + (double)j + 0.5;
}

/* ---- validation ---------------------------------------------------------- */
static int valid_pair(const int32_t bc[4], double r0) {
  int x0 = bc[SX0], x1 = bc[SX1], a = bc[SR0], b = bc[SR1];
  int xper = (x0 == LBM_REF_BC_PERIODIC) + (x1 == LBM_REF_BC_PERIODIC);
  if (xper == 1) return 0;
  if (x0 != LBM_REF_BC_INLET && x0 != LBM_REF_BC_PERIODIC &&
      x0 != LBM_REF_BC_WALL && x0 != LBM_REF_BC_EQ)
    return 0;
  if (x1 != LBM_REF_BC_OUTFLOW && x1 != LBM_REF_BC_PERIODIC &&
      x1 != LBM_REF_BC_WALL && x1 != LBM_REF_BC_EQ)
    return 0;
  if (a != LBM_REF_BC_AXIS && a != LBM_REF_BC_FREESLIP && a != LBM_REF_BC_WALL &&
      a != LBM_REF_BC_EQ)
    return 0;
  if (b != LBM_REF_BC_FREESLIP && b != LBM_REF_BC_WALL && b != LBM_REF_BC_EQ)
    return 0;
  if (a == LBM_REF_BC_AXIS && r0 != 0.0) return 0;
  if (r0 < 0.0) return 0;
  return 1;
}

static int validate(const lbm_ref_config *c) {
  if (!c) return 0;
  if (c->nx < 2 || c->nr < 2) return 0;
  if (!(c->tau_nu > 0.5) || !(c->tau_alpha > 0.5)) return 0;
  if (!(c->pr_t > 0.0) || !(c->cs >= 0.0) || !(c->delta > 0.0)) return 0;
  if (!isfinite(c->r0) || !isfinite(c->body_force_x)) return 0;
  if (c->table_n != 0) {
    if (c->table_n < 2 || !c->nu_mult || !c->alpha_mult) return 0;
    if (!(c->t_hi > c->t_lo)) return 0;
    for (int i = 0; i < c->table_n; ++i)
      if (!(c->nu_mult[i] > 0.0) || !(c->alpha_mult[i] > 0.0) ||
          !isfinite(c->nu_mult[i]) || !isfinite(c->alpha_mult[i]))
        return 0;
  }
  if (!valid_pair(c->bc, c->r0)) return 0;
  if (c->hoop != 0 && c->hoop != 1) return 0;
  if (!(c->rho0 > 0.0) || !isfinite(c->ux0) || !isfinite(c->ur0) || !isfinite(c->T0))
    return 0;
  for (int s = 0; s < 4; ++s)
    if (c->bc[s] == LBM_REF_BC_EQ &&
        (!(c->eq_state[s][0] > 0.0) || !isfinite(c->eq_state[s][1]) ||
         !isfinite(c->eq_state[s][2]) || !isfinite(c->eq_state[s][3])))
      return 0;
  return 1;
}

/* ---- API ------------------------------------------------------------------ */
void lbm_ref_destroy(lbm_ref_handle *h) {
  if (!h) return;
  free(h->tab_nu);
  free(h->tab_alpha);
  for (int b = 0; b < 2; ++b) {
    free(h->f[b]);
    free(h->g[b]);
  }
  free(h->in_ux);
  free(h->in_ur);
  free(h->in_T);
  free(h);
}

static void fill_equilibrium(lbm_ref_handle *h, const double *rho,
                             const double *ux, const double *ur, const double *T) {
  const int nx = h->c.nx, nr = h->c.nr;
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t n = (size_t)j * nx + i;
      double fe[9], ge[4];
      lbm_ref_feq(rho ? rho[n] : h->c.rho0, ux ? ux[n] : h->c.ux0,
                  ur ? ur[n] : h->c.ur0, fe);
      lbm_ref_geq(T ? T[n] : h->c.T0, ux ? ux[n] : h->c.ux0,
                  ur ? ur[n] : h->c.ur0, ge);
      for (int k = 0; k < 9; ++k) h->f[h->cur][idx(h, k, i, j)] = fe[k];
      for (int k = 0; k < 4; ++k) h->g[h->cur][idx(h, k, i, j)] = ge[k];
    }
}

int lbm_ref_create(const lbm_ref_config *cfg, lbm_ref_handle **out) {
  if (!out) return LBM_REF_EINVAL;
  *out = NULL;
  if (!validate(cfg)) return LBM_REF_EINVAL;
  lbm_ref_handle *h = (lbm_ref_handle *)calloc(1, sizeof *h);
  if (!h) return LBM_REF_ENOMEM;
  h->c = *cfg;
  h->nu0 = (cfg->tau_nu - 0.5) / 3.0;
  h->alpha0 = (cfg->tau_alpha - 0.5) / 2.0;
  size_t nodes = (size_t)cfg->nx * (size_t)cfg->nr;
  int ok = 1;
  if (cfg->table_n > 0) {
    h->tab_nu = (double *)malloc(sizeof(double) * cfg->table_n);
    h->tab_alpha = (double *)malloc(sizeof(double) * cfg->table_n);
    ok = ok && h->tab_nu && h->tab_alpha;
    if (ok) {
      memcpy(h->tab_nu, cfg->nu_mult, sizeof(double) * cfg->table_n);
      memcpy(h->tab_alpha, cfg->alpha_mult, sizeof(double) * cfg->table_n);
    }
  }
  h->c.nu_mult = h->tab_nu;
  h->c.alpha_mult = h->tab_alpha;
  for (int b = 0; b < 2; ++b) {
    h->f[b] = (double *)malloc(sizeof(double) * 9 * nodes);
    h->g[b] = (double *)malloc(sizeof(double) * 4 * nodes);
    ok = ok && h->f[b] && h->g[b];
  }
  /* default inlet row: ambient state */
  h->n_t = 1;
  h->in_ux = (double *)calloc((size_t)cfg->nr, sizeof(double));
  h->in_ur = (double *)calloc((size_t)cfg->nr, sizeof(double));
  h->in_T = (double *)malloc(sizeof(double) * cfg->nr);
  ok = ok && h->in_ux && h->in_ur && h->in_T;
  if (!ok) {
    lbm_ref_destroy(h);
    return LBM_REF_ENOMEM;
  }
  for (int j = 0; j < cfg->nr; ++j) h->in_T[j] = cfg->T0;
  h->cur = 0;
  h->step = 0;
  fill_equilibrium(h, NULL, NULL, NULL, NULL);
  *out = h;
  return LBM_REF_OK;
}

int lbm_ref_set_inlet(lbm_ref_handle *h, int32_t n_t, const double *ux,
                      const double *ur, const double *T) {
  if (!h || n_t < 1 || !ux || !ur || !T) return LBM_REF_EINVAL;
  size_t n = (size_t)n_t * (size_t)h->c.nr;
  for (size_t q = 0; q < n; ++q)
    if (!isfinite(ux[q]) || !isfinite(ur[q]) || !isfinite(T[q])) return LBM_REF_EINVAL;
  double *a = (double *)malloc(sizeof(double) * n);
  double *b = (double *)malloc(sizeof(double) * n);
  double *t = (double *)malloc(sizeof(double) * n);
  if (!a || !b || !t) {
    free(a);
    free(b);
    free(t);
    return LBM_REF_ENOMEM;
  }
  memcpy(a, ux, sizeof(double) * n);
  memcpy(b, ur, sizeof(double) * n);
  memcpy(t, T, sizeof(double) * n);
  free(h->in_ux);
  free(h->in_ur);
  free(h->in_T);
  h->in_ux = a;
  h->in_ur = b;
  h->in_T = t;
  h->n_t = n_t;
  return LBM_REF_OK;
}

int lbm_ref_step(lbm_ref_handle *h, int64_t n_steps) {
  if (!h || n_steps < 0) return LBM_REF_EINVAL;
  if (h->unstable) return LBM_REF_EUNSTABLE;
  const int nx = h->c.nx, nr = h->c.nr;
  if (h->c.threads > 0) {
#ifdef _OPENMP
    omp_set_num_threads(h->c.threads);
#endif
  }
  for (int64_t s = 0; s < n_steps; ++s) {
    const int nb = 1 - h->cur;
    double *fo = h->f[nb], *go = h->g[nb];
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < nr; ++j) {
      const double r = radius(h, j);
      for (int i = 0; i < nx; ++i) {
        double f[9], g[4], fs[9], gs[4];
        pull_node(h, i, j, f, g);
        lbm_ref_collide_node(h, f, g, r, fs, gs, NULL);
        double rho = 0.0;
        for (int k = 0; k < 9; ++k) {
          rho += f[k];
          fo[idx(h, k, i, j)] = fs[k];
          if (!isfinite(fs[k])) bad = 1;
        }
        for (int k = 0; k < 4; ++k) {
          go[idx(h, k, i, j)] = gs[k];
          if (!isfinite(gs[k])) bad = 1;
        }
        if (!(rho > 0.0)) bad = 1;
      }
    }
    h->cur = nb;
    h->step += 1;
    if (bad) {
      h->unstable = 1;
      return LBM_REF_EUNSTABLE;
    }
  }
  return LBM_REF_OK;
}

int64_t lbm_ref_step_count(const lbm_ref_handle *h) { return h ? h->step : -1; }

int lbm_ref_moments(lbm_ref_handle *h, double *rho, double *ux, double *ur, double *T) {
  if (!h) return LBM_REF_EINVAL;
  const int nx = h->c.nx, nr = h->c.nr;
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < nx; ++i) {
      double f[9], g[4];
      pull_node(h, i, j, f, g);
      double d = 0.0, mx = 0.0, mr = 0.0, t = 0.0;
      for (int k = 0; k < 9; ++k) {
        d += f[k];
        mx += EX9[k] * f[k];
        mr += ER9[k] * f[k];
      }
      for (int k = 0; k < 4; ++k) t += g[k];
      size_t n = (size_t)j * nx + i;
      if (rho) rho[n] = d;
      if (ux) ux[n] = mx / d;
      if (ur) ur[n] = mr / d;
      if (T) T[n] = t;
    }
  return h->unstable ? LBM_REF_EUNSTABLE : LBM_REF_OK;
}

int lbm_ref_conservation(lbm_ref_handle *h, double *mass3d, double *energy3d) {
  if (!h || !mass3d || !energy3d) return LBM_REF_EINVAL;
  const int nx = h->c.nx, nr = h->c.nr;
  size_t nodes = (size_t)nx * nr;
  double *rho = (double *)malloc(sizeof(double) * nodes);
  double *T = (double *)malloc(sizeof(double) * nodes);
  if (!rho || !T) {
    free(rho);
    free(T);
    return LBM_REF_ENOMEM;
  }
  int rc = lbm_ref_moments(h, rho, NULL, NULL, T);
  double m = 0.0, e = 0.0;
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < nx; ++i) {
      m += radius(h, j) * rho[(size_t)j * nx + i];
      e += radius(h, j) * T[(size_t)j * nx + i];
    }
  free(rho);
  free(T);
  *mass3d = m;
  *energy3d = e;
  return rc;
}

int lbm_ref_profiles(lbm_ref_handle *h, double *ux_axis, double *T_axis,
                     double *ux_exit, double *T_exit) {
  if (!h) return LBM_REF_EINVAL;
  const int nx = h->c.nx, nr = h->c.nr;
  size_t nodes = (size_t)nx * nr;
  double *ux = (double *)malloc(sizeof(double) * nodes);
  double *T = (double *)malloc(sizeof(double) * nodes);
  if (!ux || !T) {
    free(ux);
    free(T);
    return LBM_REF_ENOMEM;
  }
  int rc = lbm_ref_moments(h, NULL, ux, NULL, T);
  for (int i = 0; i < nx; ++i) {
    if (ux_axis) ux_axis[i] = ux[i];
    if (T_axis) T_axis[i] = T[i];
  }
  for (int j = 0; j < nr; ++j) {
    if (ux_exit) ux_exit[j] = ux[(size_t)j * nx + nx - 1];
    if (T_exit) T_exit[j] = T[(size_t)j * nx + nx - 1];
  }
  free(ux);
  free(T);
  return rc;
}

int lbm_ref_set_state(lbm_ref_handle *h, const double *rho, const double *ux,
                      const double *ur, const double *T) {
  if (!h || !rho || !ux || !ur || !T) return LBM_REF_EINVAL;
  size_t nodes = (size_t)h->c.nx * h->c.nr;
  for (size_t n = 0; n < nodes; ++n)
    if (!(rho[n] > 0.0) || !isfinite(rho[n]) || !isfinite(ux[n]) ||
        !isfinite(ur[n]) || !isfinite(T[n]))
      return LBM_REF_EINVAL;
  fill_equilibrium(h, rho, ux, ur, T);
  h->unstable = 0;
  return LBM_REF_OK;
}

int lbm_ref_get_populations(const lbm_ref_handle *h, double *f, double *g) {
  if (!h) return LBM_REF_EINVAL;
  size_t nodes = (size_t)h->c.nx * h->c.nr;
  if (f) memcpy(f, h->f[h->cur], sizeof(double) * 9 * nodes);
  if (g) memcpy(g, h->g[h->cur], sizeof(double) * 4 * nodes);
  return LBM_REF_OK;
}

int lbm_ref_set_populations(lbm_ref_handle *h, const double *f, const double *g,
                            int64_t step) {
  if (!h || !f || !g || step < 0) return LBM_REF_EINVAL;
  size_t nodes = (size_t)h->c.nx * h->c.nr;
  for (size_t n = 0; n < 9 * nodes; ++n)
    if (!isfinite(f[n])) return LBM_REF_EINVAL;
  for (size_t n = 0; n < 4 * nodes; ++n)
    if (!isfinite(g[n])) return LBM_REF_EINVAL;
  memcpy(h->f[h->cur], f, sizeof(double) * 9 * nodes);
  memcpy(h->g[h->cur], g, sizeof(double) * 4 * nodes);
  h->step = step;
  h->unstable = 0;
  return LBM_REF_OK;
}
