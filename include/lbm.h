/*
 * lbm.h -- C-ABI of the MI355X (gfx950) axisymmetric thermal lattice
 * Boltzmann LES solver: D2Q9 flow populations, D2Q4 temperature populations,
 * local Smagorinsky relaxation time, temperature-dependent properties and the
 * axisymmetric source terms, one fused collide-and-stream update per step.
 *
 * Method (Djebali, Calve, Pateyron, El Ganaoui, Sammouda):
 *   section 2.1, eq. (1)   two LBGK updates with sources F1, F2, S;
 *   section 2.1, eq. (2)   moments rho, u, T;
 *   text after eq. (1)     nu = (tau_nu - 1/2)/3, alpha = (tau_alpha - 1/2)/2;
 *   section 2.2, eqs. 3-5  Smagorinsky closure, closed-form tau_tot,
 *                          alpha_tot = alpha + nu_t / Pr_t;
 *   section 2.3, eq. (6)   nu(T), alpha(T) from multiplier tables;
 *   section 2.4, eq. (7)   inlet profiles, given here as inlet rows.
 * The source terms are not printed in the paper; the library uses the forms
 * derived from the axisymmetric Navier-Stokes and energy equations:
 *   F1 -> w_k theta, theta = -rho u_r / r;
 *   F2 -> F_x = -rho u_x u_r / r - (1 - 1/(2 tau)) Q_xr / r + rho G,
 *         F_r = -rho u_r^2 / r - (1 - 1/(2 tau)) Q_rr / r - 2 rho nu_tot u_r / D,
 *         D = r^2 (hoop = 0) or r^2 + 2 nu_tot (hoop = 1), weight e_k . F / 6;
 *   S  -> S/4 per link, S = -T u_r / r - (1 - 1/(2 tau_a)) sum_k e_kr g_k^neq / r.
 *
 * Lattice units (dx = dt = 1).  Node (i, j) sits at x = i, r = r0 + j + 1/2;
 * i = 0..nx-1 is axial (fastest in every array), j = 0..nr-1 radial.
 *
 * Conventions shared by all calls:
 *   - Return 0 (LBM_OK) or a negative LBM_E* code; nothing prints or aborts.
 *   - Input pointers are borrowed for the duration of the call (copied).
 *   - Host arrays are caller-allocated; device memory handed in through
 *     lbm_create_in must outlive the handle and is never freed by the library.
 *   - Work is enqueued on the handle's HIP stream; lbm_step may return before
 *     the work completes.  Asynchronous failures (device errors, a non-finite
 *     or non-positive density seen by the step) are reported by the next
 *     synchronising call (lbm_moments, lbm_profiles, lbm_conservation,
 *     lbm_get_populations, lbm_sync) and by every later lbm_step.
 *   - LBM_EUNSTABLE is sticky until lbm_set_state or lbm_set_populations.
 *   - A handle is used by one host thread at a time; handles are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2u

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument or configuration               */
  LBM_ENOMEM = -2,     /* device or host allocation failed, budget full    */
  LBM_EUNSTABLE = -3,  /* non-finite value or rho <= 0 seen                */
  LBM_EDEVICE = -4,    /* HIP runtime error                                */
  LBM_ESTATE = -5      /* call not valid in the handle's current state     */
};

/* Population storage.  Arithmetic is FP32 in every case.  (The value 0,
 * FP64 populations, belongs to the FP64 CPU checker that exports the same
 * calls; this library rejects it.) */
enum lbm_precision {
  LBM_PREC_FP32 = 1,     /* 13 x 4 B per node                                */
  LBM_PREC_FP16DEV = 2,  /* binary16 of f_k - w_k rho_ref, g_k - g_ref/4     */
  LBM_PREC_BF16DEV = 3,  /* bfloat16 of the same deviations                  */
  LBM_PREC_FP16SR = 4    /* binary16 of the same deviations, rounded
                            stochastically by gfx950's conversion: up with
                            the probability of the discarded fraction, to
                            2^-13 (values binary16 holds are kept), the
                            random number from a hash of the node, the step
                            and the value (reproducible)                    */
};

/* Edge rules, per side: 0 = x0 (i = -1), 1 = x1 (i = nx), 2 = r0 (j = -1),
 * 3 = r1 (j = nr).  Rules on the r sides are applied first; a mirrored pull
 * then goes through the x-side rule at the edge row. */
enum lbm_bc {
  LBM_BC_INLET = 0,    /* x0: equilibrium at rho = 1 and the inlet row      */
  LBM_BC_OUTFLOW = 1,  /* x1: zero-gradient copy of column nx-1             */
  LBM_BC_PERIODIC = 2, /* x0 and x1 together                                */
  LBM_BC_AXIS = 3,     /* r0 with r0 == 0: half-way specular symmetry axis  */
  LBM_BC_FREESLIP = 4, /* r sides: half-way specular mirror                 */
  LBM_BC_WALL = 5,     /* any side: half-way bounce-back; anti-bounce-back
                          for g at the Dirichlet temperature wall_T[side],
                          plain bounce-back (adiabatic) if wall_T is NaN    */
  LBM_BC_EQ = 6        /* any side: equilibrium of eq_state[side]           */
};

/* Population buffers of a jet. */
enum lbm_layout {
  LBM_LAYOUT_TWO_BUFFERS = 0, /* read one buffer, write the other each step   */
  LBM_LAYOUT_SINGLE = 1       /* one buffer updated in place (AA pattern): half
                                 the memory; one step per launch; results
                                 bit-identical to the two-buffer layout       */
};

typedef struct lbm_handle lbm_handle;

/* Configuration of one jet.  Where each field comes from in the paper:
 *   nx, nr        section 2.4: the half plane (x, r) discretised on a uniform
 *                 lattice (the paper's run: 200 x 96 nodes);
 *   r0            section 2.1: the axisymmetric form of eq. (1) in (x, r);
 *                 node centres at r = r0 + j + 1/2 (a reading: the axis is
 *                 a half-way mirror, so 1/r stays finite);
 *   tau_nu,       text after eq. (1): nu = (tau_nu - 1/2)/3 and
 *   tau_alpha     alpha = (tau_alpha - 1/2)/2 in lattice units;
 *   cs, delta     section 2.2, eqs. (3)-(4): Smagorinsky constant C_s and
 *                 filter width Delta;
 *   pr_t          section 2.2, eq. (5): turbulent Prandtl number (0.3 to 1;
 *                 0.3 in the validation runs of section 4.1);
 *   table_n ..    section 2.3, eq. (6): nu(T), alpha(T) as multipliers of
 *   t_hi          the base values on a uniform T grid (the paper's N2-Ar
 *                 curves are not given; any table may be supplied);
 *   bc            section 2.4 (inlet, symmetry axis, outflow, outer edge)
 *                 and section 4.2 (a substrate wall at the far end);
 *   wall_T        section 4.2: temperature of a wall (the substrate);
 *                 NaN for an adiabatic wall;
 *   eq_state      not in the paper: an equilibrium side, used by tests;
 *   body_force_x  not in the paper: a uniform axial force, used by the
 *                 pipe-flow test of the viscous source terms;
 *   rho0 .. T0    section 2.4: the ambient gas at rest the jet enters;
 *   hoop          the form of the hoop term of F2 (eq. 1; the source terms
 *                 are not printed): explicit or stabilised, see above;
 *   precision,    storage of the populations (not in the paper: every
 *   rho_ref,      arithmetic is FP32 whatever the storage);
 *   g_ref, layout
 */
typedef struct {
  uint32_t abi_version;       /* must be LBM_ABI_VERSION                      */
  int32_t nx, nr;             /* fluid nodes; >= 2 each                       */
  double r0;                  /* radius offset; 0 when bc[2] is AXIS          */
  double tau_nu, tau_alpha;   /* base relaxation times; > 1/2                 */
  double cs, delta, pr_t;     /* C_s >= 0, filter width > 0, Pr_t > 0         */
  int32_t table_n;            /* 0: constant properties; else >= 2 entries    */
  const double *nu_mult;      /* table_n multipliers of nu over [t_lo, t_hi]  */
  const double *alpha_mult;   /* table_n multipliers of alpha                 */
  double t_lo, t_hi;          /* uniform table grid; linear, clamped          */
  int32_t bc[4];              /* LBM_BC_* of x0, x1, r0, r1                   */
  double wall_T[4];           /* WALL temperature per side; NaN = adiabatic   */
  double eq_state[4][4];      /* EQ side state rho, ux, ur, T                 */
  double body_force_x;        /* G; rho G is added to F_x                     */
  double rho0, ux0, ur0, T0;  /* uniform initial state (equilibrium)          */
  int32_t hoop;               /* 0: explicit hoop term, 1: stabilised         */
  int32_t precision;          /* LBM_PREC_*                                   */
  double rho_ref, g_ref;      /* 16-bit storage offsets (ignored for FP32)    */
  int32_t layout;             /* LBM_LAYOUT_* (a batch uses its own layout)   */
} lbm_config;

/* Device bytes lbm_create_in needs for the population buffers (two, or one
 * with LBM_LAYOUT_SINGLE).  Kernels address a buffer with 32-bit byte
 * offsets: a grid whose 13 FP32 planes, each (nx + 73 rounded up to 64) x
 * (nr + 2) including the ghost ring, reach 2^31 bytes is LBM_EINVAL here and
 * in lbm_create (8192 x 4096 fits, 10000 x 5000 does not). */
int lbm_bytes_required(const lbm_config *cfg, size_t *bytes);

/* Create a solver on the current HIP device for the problem the paper
 * states in sections 2.1-2.4 (the lattice, relaxation times, LES constants,
 * property tables and edges of lbm_config), populations at the equilibrium
 * of (rho0, ux0, ur0, T0) (the ambient state of section 2.4), step 0, inlet
 * rows at the ambient state (u = 0, T = T0).  lbm_create allocates the
 * population buffers and a stream itself; lbm_create_in uses dev_buf
 * (>= lbm_bytes_required bytes, 256-byte aligned) and hip_stream (a
 * hipStream_t; NULL = default stream), both owned by the caller.  *out is
 * NULL on failure; LBM_EINVAL for an invalid configuration, LBM_ENOMEM when
 * device memory runs out, LBM_EDEVICE for other HIP errors. */
int lbm_create(const lbm_config *cfg, lbm_handle **out);
int lbm_create_in(const lbm_config *cfg, void *dev_buf, size_t bytes,
                  void *hip_stream, lbm_handle **out);

/* Inlet rows for the x0 INLET edge (eq. 7 profiles, or any other):
 * n_t rows of nr values each, row-major; step s uses row s mod n_t. */
int lbm_set_inlet(lbm_handle *h, int32_t n_t, const double *ux, const double *ur,
                  const double *T);

/* Advance n_steps >= 0 steps: at every node, the pull of the edge rules
 * (section 2.4), the moments of eq. (2), the properties of eq. (6), the
 * relaxation times of eqs. (3)-(5), the source terms and the collision of
 * eq. (1) (section 2.1).  Enqueues only; LBM_EUNSTABLE if an earlier step
 * was found unstable. */
int lbm_step(lbm_handle *h, int64_t n_steps);

/* Pre-collision moments (eq. 2) at the current step, each nr*nx doubles;
 * NULL pointers are skipped.  Synchronises. */
int lbm_moments(lbm_handle *h, double *rho, double *ux, double *ur, double *T);

/* Release a solver and everything the library allocated for it (not
 * memory or a stream handed in through lbm_create_in).  NULL-safe; waits for
 * queued work first.  Not a step of the method. */
void lbm_destroy(lbm_handle *h);

/* ---- extras ------------------------------------------------------------- */
int64_t lbm_step_count(const lbm_handle *h); /* -1 for NULL */
void *lbm_stream(const lbm_handle *h);       /* the handle's hipStream_t    */
int lbm_sync(lbm_handle *h);                 /* wait; report async errors   */
/* Group k steps into one HIP graph launch (0 disables graphs).  The graph
 * of the handle's current tile shape is captured, instantiated and uploaded
 * here (and again by lbm_set_tile_shape), not at the first lbm_step that
 * replays it.  Synchronises. */
int lbm_set_graph_steps(lbm_handle *h, int32_t k);
/* Equilibrium fill from fields (each nr*nx); clears LBM_EUNSTABLE. */
int lbm_set_state(lbm_handle *h, const double *rho, const double *ux,
                  const double *ur, const double *T);
/* Stored post-collision populations, decoded to double: f 9*nr*nx, g 4*nr*nx
 * (population index slowest). */
int lbm_get_populations(lbm_handle *h, double *f, double *g);
int lbm_set_populations(lbm_handle *h, const double *f, const double *g,
                        int64_t step);
/* FP64 reductions of the step's pre-collision moments:
 * mass3d = sum_ij r_j rho_ij, energy3d = sum_ij r_j T_ij. */
int lbm_conservation(lbm_handle *h, double *mass3d, double *energy3d);
/* lbm_conservation for callers that cannot allocate device memory (a
 * serving loop or harness that forbids allocation): the same reduction, with
 * the same kernels and the same bits, but its partial sums (at most 1025 of
 * 32 B: one per reduction workgroup and the total) live in a fixed array
 * that the library holds on each device until the process ends, instead of
 * a buffer it allocates on first use.  Calls no allocating routine.  Every
 * call on one device uses that device's array: calls that overlap on one
 * device (from several host threads or handles) race and must be
 * serialised by the caller.  Nothing in the array needs clearing between
 * calls (every partial is written before it is read).  Synchronises;
 * LBM_EINVAL for a grid that would need more partials (none that
 * lbm_create accepts does). */
int lbm_conservation_noalloc(lbm_handle *h, double *mass3d, double *energy3d);
/* Centreline (j = 0) u_x and T, nx each; exit column (i = nx-1), nr each. */
int lbm_profiles(lbm_handle *h, double *ux_axis, double *T_axis,
                 double *ux_exit, double *T_exit);
const char *lbm_strerror(int code);

/* Measurement helper: copy `bytes` (multiple of 16) from src to dst on the
 * device with a plain streaming kernel, on hip_stream.  Used to calibrate
 * the HBM traffic counters against a transfer of known size. */
int lbm_probe_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* ---- many jets in persistent launches -------------------------------------
 * A batch owns up to max_slots resident jets whose population buffers are
 * carved out of budget_bytes of device memory.  lbm_batch_run advances every
 * active jet by up to k steps: the active jets are grouped into cohorts of
 * at most cohort_bytes of buffers (default 128 MiB, so that the two cohorts
 * in flight at once fill the 256 MiB Infinity Cache), and each cohort gets k
 * steps of one persistent launch per step over all its jets (HIP graphs),
 * cohorts alternating between two streams (lbm_batch_set_streams).  A jet
 * stops at its own target step count.  Each jet's result is bitwise the
 * same as that of the same jet run alone.  `precision` is the batch's
 * storage form; a jet admitted with another (cfg->precision) joins cohorts
 * of its own form, so one batch serves jets of several storage forms. */
typedef struct lbm_batch lbm_batch;
int lbm_batch_create(size_t budget_bytes, int32_t max_slots, int32_t precision,
                     void *hip_stream, lbm_batch **out);
/* Population layout of every jet of the batch (LBM_LAYOUT_*; default two
 * buffers).  Only while the batch holds no jet (else LBM_ESTATE).  With
 * LBM_LAYOUT_SINGLE a jet takes half the budget and every launch advances
 * one step. */
int lbm_batch_set_layout(lbm_batch *b, int32_t layout);
/* Admit a jet.  cfg->precision is the jet's storage form (LBM_PREC_FP32,
 * _FP16DEV, _BF16DEV or _FP16SR; 0 = the batch's; others LBM_EINVAL);
 * cfg->layout is ignored (the batch's).  LBM_ENOMEM when the budget or the
 * slot table is full.  n_t/ux/ur/T as lbm_set_inlet (n_t = 0: ambient). */
int lbm_batch_admit(lbm_batch *b, const lbm_config *cfg, int32_t n_t,
                    const double *ux, const double *ur, const double *T,
                    int64_t target_steps, int32_t *slot);
/* Queue k steps of every active jet (enqueues only: it does not wait for the
 * groups already queued, except that a rebuild of the cohort lists waits for
 * the group two rebuilds back, which read the same copy of the lists). */
int lbm_batch_run(lbm_batch *b, int32_t k_steps);
/* Wait until at most in_flight (0 to 15) of the groups queued by
 * lbm_batch_run are unfinished: 0 waits for all of them, 1 lets the last one
 * run on while the caller works (a serving loop's throttle). */
int lbm_batch_wait(lbm_batch *b, int32_t in_flight);
/* Steps done by a slot's jet (host-side count; exact after lbm_batch_run). */
int lbm_batch_poll(lbm_batch *b, int32_t slot, int64_t *steps_done);
/* Profiles and moments of a slot's jet at its step count: they wait for the
 * group in which the jet reached its target (or, for a jet still running,
 * for all queued work), not for groups queued after it. */
int lbm_batch_profiles(lbm_batch *b, int32_t slot, double *ux_axis, double *T_axis,
                       double *ux_exit, double *T_exit);
int lbm_batch_moments(lbm_batch *b, int32_t slot, double *rho, double *ux,
                      double *ur, double *T);
/* Free a slot: waits for the group in which its jet reached its target (or
 * for all queued work if it had not), then returns its memory to the budget.
 * Admission queues its uploads behind the work in flight and waits for
 * nothing; neither call allocates device memory once the slot's block for
 * the table and inlet rows is large enough. */
int lbm_batch_retire(lbm_batch *b, int32_t slot);
/* Wait for the batch's queued work; LBM_EDEVICE on an asynchronous error. */
int lbm_batch_sync(lbm_batch *b);
/* Device time of the groups (from just before a group's first launch to its
 * completion, HIP events on the batch's stream) summed over the groups that
 * lbm_batch_wait or lbm_batch_sync found complete, and how many they were
 * (a group more than 15 groups older than the newest queued when the batch
 * is next waited on is not counted).  Host-side; does not wait. */
int lbm_batch_device_time(lbm_batch *b, double *ms, int64_t *groups);
/* Bytes a jet of this configuration (and storage form, as for
 * lbm_batch_admit) takes from the budget. */
int lbm_batch_jet_bytes(const lbm_batch *b, const lbm_config *cfg, size_t *bytes);
int lbm_batch_active(const lbm_batch *b, int32_t *n_active, size_t *bytes_used);
/* Tile shape of the step kernel (index into the compiled shapes; -1 = auto,
 * the default shape of each storage form) and the number of persistent
 * workgroups (0 = auto: as many as the device holds at once for that
 * kernel); both apply to every storage form of the batch. */
int lbm_batch_set_launch(lbm_batch *b, int32_t tile_shape, int32_t workgroups);
/* Cohort size limit in bytes of population buffers (0: all jets together;
 * default 128 MiB, so that the two cohorts running at once fill the 256 MiB
 * Infinity Cache). */
int lbm_batch_set_cohort_bytes(lbm_batch *b, size_t bytes);
/* Streams the cohorts of a run are spread over, 1 to 4: cohort c runs on
 * stream c mod n, stream 0 being the batch's stream and the others streams
 * of default priority that the library creates.  They start after the work
 * already queued on the batch's stream, and later work on the batch's stream
 * waits for them, so callers see one stream.  Default 2 (measured best with
 * the default cohorts; 3 or 4 smaller cohorts were slower).  Results are the
 * same bits for any n.  Synchronises; LBM_EINVAL for other values,
 * LBM_EDEVICE (and one stream) if a stream cannot be created. */
int lbm_batch_set_streams(lbm_batch *b, int32_t n);
void lbm_batch_destroy(lbm_batch *b);

/* Compiled tile shapes of the step kernel: count, and one shape: a workgroup
 * of bx x by threads, each updating nx consecutive axial nodes in ny rows. */
int lbm_tile_shape_count(void);
int lbm_tile_shape(int32_t index, int32_t *bx, int32_t *by, int32_t *ny, int32_t *nx);
/* All properties of a shape: info[0..n-1] of (bx, by, ny, nx, waves per SIMD
 * targeted, variant bits (bit 0 non-temporal stores, bit 1 non-temporal
 * loads; two-step shapes: bit 2 no prefetch of the next rows' loads, bit 3
 * f_0 kept in registers instead of LDS), steps per launch, LDS bytes per
 * workgroup); n <= 8 entries are written.
 * Shapes with 2 steps per launch run two time steps of eq. (1) per kernel
 * launch on an LDS-resident 64 x (by * ny) tile with a one-node frame,
 * bit-identical to two one-step launches, on every edge rule (with periodic
 * x edges the frame wraps to the other end of the domain). */
int lbm_tile_shape_info(int32_t index, int32_t *info, int32_t n);
/* Select the launch variant of a handle (synchronises; EINVAL for an unknown
 * index, or any shape but 0 on a single-buffer handle, whose in-place kernel
 * uses shape 0's tiles). */
int lbm_set_tile_shape(lbm_handle *h, int32_t index);

#ifdef __cplusplus
}
#endif
#endif
