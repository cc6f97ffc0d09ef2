// lbm_kernels.hip -- kernel instantiations, launch helpers and the host-side
// configuration checks shared by the single-jet and batch runtimes.
#include "lbm_kernels.hpp"
#include "lbm_runtime.hpp"

namespace lbmx {

// ---- validation (same rules the paper's setting implies: tau > 1/2 so that
// nu, alpha > 0; Pr_t > 0; a symmetry axis only at r = 0) ------------------
static bool side_ok(int side, int bc) {
  switch (side) {
    case 0: return bc == BC_INLET || bc == BC_PERIODIC || bc == BC_WALL || bc == BC_EQ;
    case 1: return bc == BC_OUTFLOW || bc == BC_PERIODIC || bc == BC_WALL || bc == BC_EQ;
    case 2: return bc == BC_AXIS || bc == BC_FREESLIP || bc == BC_WALL || bc == BC_EQ;
    default: return bc == BC_FREESLIP || bc == BC_WALL || bc == BC_EQ;
  }
}

int validate_config(const lbm_config *c, bool check_precision) {
  if (!c || c->abi_version != LBM_ABI_VERSION) return LBM_EINVAL;
  if (c->nx < 2 || c->nr < 2) return LBM_EINVAL;
  // every byte offset inside a buffer must fit the 32-bit buffer offsets
  if ((int64_t)NPOP * layout_plane(c->nx, c->nr) * 4 >= ((int64_t)1 << 31)) return LBM_EINVAL;
  if (!(c->tau_nu > 0.5) || !(c->tau_alpha > 0.5) || !std::isfinite(c->tau_nu) ||
      !std::isfinite(c->tau_alpha))
    return LBM_EINVAL;
  if (!(c->pr_t > 0.0) || !(c->cs >= 0.0) || !(c->delta > 0.0) || !std::isfinite(c->cs) ||
      !std::isfinite(c->delta) || !std::isfinite(c->pr_t))
    return LBM_EINVAL;
  if (!std::isfinite(c->r0) || c->r0 < 0.0 || !std::isfinite(c->body_force_x)) return LBM_EINVAL;
  if (c->table_n != 0) {
    if (c->table_n < 2 || !c->nu_mult || !c->alpha_mult || !(c->t_hi > c->t_lo) ||
        !std::isfinite(c->t_lo) || !std::isfinite(c->t_hi))
      return LBM_EINVAL;
    for (int q = 0; q < c->table_n; ++q)
      if (!(c->nu_mult[q] > 0.0) || !(c->alpha_mult[q] > 0.0) || !std::isfinite(c->nu_mult[q]) ||
          !std::isfinite(c->alpha_mult[q]))
        return LBM_EINVAL;
  }
  for (int s = 0; s < 4; ++s)
    if (!side_ok(s, c->bc[s])) return LBM_EINVAL;
  if ((c->bc[0] == BC_PERIODIC) != (c->bc[1] == BC_PERIODIC)) return LBM_EINVAL;
  if (c->bc[2] == BC_AXIS && c->r0 != 0.0) return LBM_EINVAL;
  for (int s = 0; s < 4; ++s)
    if (c->bc[s] == BC_EQ &&
        (!(c->eq_state[s][0] > 0.0) || !std::isfinite(c->eq_state[s][0]) ||
         !std::isfinite(c->eq_state[s][1]) || !std::isfinite(c->eq_state[s][2]) ||
         !std::isfinite(c->eq_state[s][3])))
      return LBM_EINVAL;
  if (c->hoop != 0 && c->hoop != 1) return LBM_EINVAL;
  if (c->layout != LBM_LAYOUT_TWO_BUFFERS && c->layout != LBM_LAYOUT_SINGLE) return LBM_EINVAL;
  if (!(c->rho0 > 0.0) || !std::isfinite(c->rho0) || !std::isfinite(c->ux0) ||
      !std::isfinite(c->ur0) || !std::isfinite(c->T0))
    return LBM_EINVAL;
  if (check_precision) {
    if (c->precision != LBM_PREC_FP32 && c->precision != LBM_PREC_FP16DEV &&
        c->precision != LBM_PREC_BF16DEV && c->precision != LBM_PREC_FP16SR)
      return LBM_EINVAL;
    if (c->precision != LBM_PREC_FP32 &&
        (!std::isfinite(c->rho_ref) || !std::isfinite(c->g_ref)))
      return LBM_EINVAL;
  }
  return LBM_OK;
}

std::vector<float4> make_table(const lbm_config *c) {
  std::vector<float4> t;
  if (c->table_n == 0) {
    t.assign(2, make_float4(1.f, 0.f, 1.f, 0.f));
    return t;
  }
  const int n = c->table_n;
  t.resize(n);
  for (int q = 0; q < n; ++q) {
    const double a = c->nu_mult[q], b = c->alpha_mult[q];
    const double da = q + 1 < n ? c->nu_mult[q + 1] - a : 0.0;
    const double db = q + 1 < n ? c->alpha_mult[q + 1] - b : 0.0;
    t[q] = make_float4((float)a, (float)da, (float)b, (float)db);
  }
  return t;
}

void fill_desc(JetDesc &d, const lbm_config *c) {
  d.nx = c->nx;
  d.nr = c->nr;
  d.pitch = layout_pitch(c->nx);
  d.plane = layout_plane(c->nx, c->nr);
  d.table_n = c->table_n == 0 ? 2 : c->table_n;
  d.hoop = c->hoop;
  for (int s = 0; s < 4; ++s) {
    d.bc[s] = c->bc[s];
    d.wallT[s] = (float)c->wall_T[s];
    for (int q = 0; q < 4; ++q) d.eq[s][q] = (float)c->eq_state[s][q];
  }
  d.r0 = (float)c->r0;
  d.nu0 = (float)((c->tau_nu - 0.5) / 3.0);
  d.alpha0 = (float)((c->tau_alpha - 0.5) / 2.0);
  const double csd = c->cs * c->delta;
  d.c18 = (float)(18.0 * csd * csd);
  d.inv_prt = (float)(1.0 / c->pr_t);
  d.G = (float)c->body_force_x;
  d.t_lo = c->table_n == 0 ? 0.f : (float)c->t_lo;
  d.t_scale = c->table_n == 0 ? 0.f : (float)((c->table_n - 1) / (c->t_hi - c->t_lo));
  d.rho_ref = (float)c->rho_ref;
  d.g4_ref = (float)(0.25 * c->g_ref);
  d.flip = 0;
}

int make_inlet(const lbm_config *c, int32_t n_t, const double *ux, const double *ur,
               const double *T, std::vector<float4> &out) {
  if (n_t < 0) return LBM_EINVAL;
  if (n_t == 0) {
    out.assign((size_t)c->nr, make_float4(0.f, 0.f, (float)c->T0, 0.f));
    return LBM_OK;
  }
  if (!ux || !ur || !T) return LBM_EINVAL;
  const size_t n = (size_t)n_t * (size_t)c->nr;
  out.resize(n);
  for (size_t q = 0; q < n; ++q) {
    if (!std::isfinite(ux[q]) || !std::isfinite(ur[q]) || !std::isfinite(T[q])) return LBM_EINVAL;
    out[q] = make_float4((float)ux[q], (float)ur[q], (float)T[q], 0.f);
  }
  return LBM_OK;
}

// ---- tile shapes -------------------------------------------------------------
#define LBM_SHAPE(BX, BY, NY, NX, W, CP)                                         \
  {BX, BY, NY, NX, W, CP, 1, 0,                                                  \
   {(const void *)&step_kernel<CodecF32, BX, BY, NY, NX, W, CP>,                 \
    (const void *)&step_kernel<CodecF16, BX, BY, NY, NX, W, CP>,                 \
    (const void *)&step_kernel<CodecBF16, BX, BY, NY, NX, W, CP>,                \
    (const void *)&step_kernel<CodecF16SR, BX, BY, NY, NX, W, CP>}}
// two steps per launch: 64 x TY tiles, block 64 x NW (lds: the LDS image of
// FP32 storage; the 16-bit forms keep theirs in the storage type, half that)
#define LBM_PAIR(TY, NW, W, CP)                                                  \
  {64, NW, (TY) / (NW), 1, W, CP, 2, (NPOP - ((CP) & 8 ? 1 : 0)) * ((TY) + 2) * PAIR_W * 4, \
   {(const void *)&pair_kernel<CodecF32, TY, NW, W, CP>,                         \
    (const void *)&pair_kernel<CodecF16, TY, NW, W, CP>,                         \
    (const void *)&pair_kernel<CodecBF16, TY, NW, W, CP>,                        \
    (const void *)&pair_kernel<CodecF16SR, TY, NW, W, CP>}}

static const TileShape kShapes[] = {
    LBM_SHAPE(64, 4, 1, 1, 1, 0),  LBM_SHAPE(128, 2, 1, 1, 1, 0), LBM_SHAPE(256, 1, 1, 1, 1, 0),
    LBM_SHAPE(64, 8, 1, 1, 1, 0),  LBM_SHAPE(64, 4, 2, 1, 1, 0),  LBM_SHAPE(64, 4, 1, 2, 1, 0),
    LBM_SHAPE(128, 2, 1, 2, 1, 0), LBM_SHAPE(64, 4, 1, 1, 1, 1),  LBM_SHAPE(64, 4, 1, 1, 1, 2),
    LBM_SHAPE(64, 4, 1, 1, 1, 3),  LBM_SHAPE(64, 4, 2, 1, 1, 1),  LBM_SHAPE(64, 4, 2, 1, 1, 3),
    LBM_SHAPE(128, 2, 1, 1, 1, 1), LBM_SHAPE(64, 8, 2, 1, 1, 0),
    LBM_PAIR(8, 4, 4, 0),          LBM_PAIR(12, 4, 3, 0),         LBM_PAIR(16, 4, 2, 0),
    LBM_PAIR(8, 4, 4, 1),          LBM_PAIR(12, 4, 3, 1),         LBM_PAIR(8, 4, 4, 4),
    LBM_PAIR(12, 4, 3, 4),         LBM_PAIR(8, 4, 4, 5),          LBM_PAIR(16, 4, 2, 4),
    LBM_PAIR(8, 4, 5, 8),          LBM_PAIR(8, 4, 5, 9),          LBM_PAIR(8, 4, 5, 12),
    LBM_PAIR(12, 4, 3, 8),
    // 16-bit storage: a 64 x 16 tile's image (28.5 KB) leaves room for five
    // workgroups per CU, and the 1 024 tiles of a 2048 x 512 jet then fit
    // the resident workgroups at once (no second, partly idle round)
    LBM_PAIR(16, 4, 5, 8),         LBM_PAIR(16, 4, 5, 12),
};
#undef LBM_SHAPE
#undef LBM_PAIR

const TileShape *tile_shapes(int *count) {
  *count = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
  return kShapes;
}
// FP32 storage: the two-step kernel on 64 x 8 tiles with f_0 kept in
// registers (12-plane image, 5 workgroups per CU): the HBM traffic per step
// halves and the arithmetic still fits under it.  16-bit storage, whose step
// is arithmetic-limited already: one step per launch.
int default_tile_shape(int prec) {
  if (prec != LBM_PREC_FP32) return 0;
  int n;
  const TileShape *s = tile_shapes(&n);
  for (int q = 0; q < n; ++q)
    if (s[q].steps == 2 && s[q].by == 4 && s[q].by * s[q].ny == 8 && s[q].cache == 8) return q;
  return 0;
}

int tiles_of(const lbm_config *c, int shape, int32_t *tiles_x) {
  const TileShape &s = kShapes[shape];
  const int tx = (c->nx + s.bx * s.nx - 1) / (s.bx * s.nx);
  const int ty = (c->nr + s.by * s.ny - 1) / (s.by * s.ny);
  if (tiles_x) *tiles_x = tx;
  return tx * ty;
}

int launch_step(int shape, int prec, int grid, hipStream_t st, const JetDesc *jets,
                const int32_t *tiles, const BatchHdr *hdr, int32_t koff, int32_t tog,
                int32_t nsteps, int32_t *flags) {
  const TileShape &s = kShapes[shape];
  void *args[] = {(void *)&jets, (void *)&tiles, (void *)&hdr,   (void *)&koff,
                  (void *)&tog,  (void *)&nsteps, (void *)&flags};
  LBM_HIP(hipLaunchKernel(s.fn[codec_index(prec)], dim3(grid), dim3(s.bx, s.by), args, 0, st));
  return LBM_OK;
}

static const void *aa_fn(int prec) {
  static const void *fn[4] = {(const void *)&aa_kernel<CodecF32>,
                              (const void *)&aa_kernel<CodecF16>,
                              (const void *)&aa_kernel<CodecBF16>,
                              (const void *)&aa_kernel<CodecF16SR>};
  return fn[codec_index(prec)];
}

int resident_workgroups(int shape, int prec, bool single_buffer) {
  const TileShape &s = kShapes[shape];
  const void *fn = single_buffer ? aa_fn(prec) : s.fn[codec_index(prec)];
  const int threads = single_buffer ? 256 : s.bx * s.by;
  int per_cu = 0, cus = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      per_cu <= 0 || cus <= 0)
    return 2048;
  return (per_cu * cus + 7) / 8 * 8;
}

int launch_aa_step(int prec, int grid, hipStream_t st, const JetDesc *jets, const int32_t *tiles,
                   const BatchHdr *hdr, int32_t koff, int32_t *flags) {
  int32_t tog = 0, nsteps = 1;
  void *args[] = {(void *)&jets, (void *)&tiles, (void *)&hdr,   (void *)&koff,
                  (void *)&tog,  (void *)&nsteps, (void *)&flags};
  LBM_HIP(hipLaunchKernel(aa_fn(prec), dim3(grid), dim3(64, 4), args, 0, st));
  return LBM_OK;
}

int launch_advance(hipStream_t st, JetDesc *jets, const BatchHdr *hdr, int32_t njets_max,
                   int32_t delta, int32_t npair) {
  const int blocks = (njets_max + 63) / 64;
  hipLaunchKernelGGL(advance_kernel, dim3(blocks), dim3(64), 0, st, jets, hdr, delta, npair);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void init_t(hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                   const float4 *state, float4 u0) {
  hipLaunchKernelGGL(init_kernel<C>, dim3((c->nx + 255) / 256, c->nr), dim3(256), 0, st, d,
                     step, view, state, u0);
}
int launch_init(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                const float4 *state, float4 u0) {
  if (prec == LBM_PREC_FP32) init_t<CodecF32>(st, d, c, step, view, state, u0);
  else if (prec == LBM_PREC_FP16DEV) init_t<CodecF16>(st, d, c, step, view, state, u0);
  else if (prec == LBM_PREC_FP16SR) init_t<CodecF16SR>(st, d, c, step, view, state, u0);
  else init_t<CodecBF16>(st, d, c, step, view, state, u0);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void ghost_t(hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view) {
  const int n = 2 * (c->nx + 2) + 2 * c->nr;
  hipLaunchKernelGGL(ghost_fill_kernel<C>, dim3((n + 255) / 256), dim3(256), 0, st, d, step, view);
}
int launch_ghost_fill(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c,
                      int64_t step, int32_t view) {
  if (prec == LBM_PREC_FP32) ghost_t<CodecF32>(st, d, c, step, view);
  else if (prec == LBM_PREC_FP16DEV) ghost_t<CodecF16>(st, d, c, step, view);
  else if (prec == LBM_PREC_FP16SR) ghost_t<CodecF16SR>(st, d, c, step, view);
  else ghost_t<CodecBF16>(st, d, c, step, view);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void moments_t(hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                      float4 *out) {
  hipLaunchKernelGGL(moments_kernel<C>, dim3((c->nx + 255) / 256, c->nr), dim3(256), 0, st, d,
                     step, view, out);
}
int launch_moments(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c,
                   int64_t step, int32_t view, float4 *out) {
  if (prec == LBM_PREC_FP32) moments_t<CodecF32>(st, d, c, step, view, out);
  else if (prec == LBM_PREC_FP16DEV) moments_t<CodecF16>(st, d, c, step, view, out);
  else if (prec == LBM_PREC_FP16SR) moments_t<CodecF16SR>(st, d, c, step, view, out);
  else moments_t<CodecBF16>(st, d, c, step, view, out);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void profiles_t(hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                       float2 *out) {
  const int n = c->nx + c->nr;
  hipLaunchKernelGGL(profiles_kernel<C>, dim3((n + 255) / 256), dim3(256), 0, st, d, step, view, out);
}
int launch_profiles(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c,
                    int64_t step, int32_t view, float2 *out) {
  if (prec == LBM_PREC_FP32) profiles_t<CodecF32>(st, d, c, step, view, out);
  else if (prec == LBM_PREC_FP16DEV) profiles_t<CodecF16>(st, d, c, step, view, out);
  else if (prec == LBM_PREC_FP16SR) profiles_t<CodecF16SR>(st, d, c, step, view, out);
  else profiles_t<CodecBF16>(st, d, c, step, view, out);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void cons_t(hipStream_t st, const JetDesc *d, int64_t step, int32_t view, RedPartial *partial,
                   int nblocks) {
  hipLaunchKernelGGL(conservation_kernel<C>, dim3(nblocks), dim3(RED_THREADS), 0, st, d, step, view,
                     partial);
}
int launch_conservation(int prec, hipStream_t st, const JetDesc *d, int64_t nodes, int64_t step, int32_t view,
                        RedPartial *partial, int nblocks, RedPartial *out) {
  (void)nodes;
  if (prec == LBM_PREC_FP32) cons_t<CodecF32>(st, d, step, view, partial, nblocks);
  else if (prec == LBM_PREC_FP16DEV) cons_t<CodecF16>(st, d, step, view, partial, nblocks);
  else if (prec == LBM_PREC_FP16SR) cons_t<CodecF16SR>(st, d, step, view, partial, nblocks);
  else cons_t<CodecBF16>(st, d, step, view, partial, nblocks);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(RED_THREADS), 0, st, partial, nblocks,
                     out);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void decode_t(hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                     float *out) {
  hipLaunchKernelGGL(decode_kernel<C>, dim3((c->nx + 255) / 256, c->nr, NPOP), dim3(256), 0, st,
                     d, step, view, out);
}
int launch_decode(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                  float *out) {
  if (prec == LBM_PREC_FP32) decode_t<CodecF32>(st, d, c, step, view, out);
  else if (prec == LBM_PREC_FP16DEV) decode_t<CodecF16>(st, d, c, step, view, out);
  else if (prec == LBM_PREC_FP16SR) decode_t<CodecF16SR>(st, d, c, step, view, out);
  else decode_t<CodecBF16>(st, d, c, step, view, out);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <class C>
static void encode_t(hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                     const float *in) {
  hipLaunchKernelGGL(encode_kernel<C>, dim3((c->nx + 255) / 256, c->nr, NPOP), dim3(256), 0, st,
                     d, step, view, in);
}
int launch_encode(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step, int32_t view,
                  const float *in) {
  if (prec == LBM_PREC_FP32) encode_t<CodecF32>(st, d, c, step, view, in);
  else if (prec == LBM_PREC_FP16DEV) encode_t<CodecF16>(st, d, c, step, view, in);
  else if (prec == LBM_PREC_FP16SR) encode_t<CodecF16SR>(st, d, c, step, view, in);
  else encode_t<CodecBF16>(st, d, c, step, view, in);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

}  // namespace lbmx

extern "C" int lbm_probe_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (!dst || !src || bytes % 16 != 0) return LBM_EINVAL;
  const int64_t n = (int64_t)(bytes / 16);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 256 * 32);
  if (n == 0) return LBM_OK;
  hipLaunchKernelGGL(lbmx::copy_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     (const float4 *)src, (float4 *)dst, n);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

extern "C" int lbm_tile_shape_count(void) {
  int n;
  lbmx::tile_shapes(&n);
  return n;
}

extern "C" int lbm_tile_shape(int32_t index, int32_t *bx, int32_t *by, int32_t *ny,
                              int32_t *nx) {
  int n;
  const lbmx::TileShape *s = lbmx::tile_shapes(&n);
  if (index < 0 || index >= n || !bx || !by || !ny || !nx) return LBM_EINVAL;
  *bx = s[index].bx;
  *by = s[index].by;
  *ny = s[index].ny;
  *nx = s[index].nx;
  return LBM_OK;
}

extern "C" int lbm_tile_shape_info(int32_t index, int32_t *info, int32_t n) {
  int count;
  const lbmx::TileShape *s = lbmx::tile_shapes(&count);
  if (index < 0 || index >= count || !info || n < 0) return LBM_EINVAL;
  const lbmx::TileShape &t = s[index];
  const int32_t v[8] = {t.bx, t.by, t.ny, t.nx, t.waves, t.cache, t.steps, t.lds};
  for (int32_t q = 0; q < n && q < 8; ++q) info[q] = v[q];
  return LBM_OK;
}
