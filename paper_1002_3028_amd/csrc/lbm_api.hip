// lbm_api.hip -- single-jet C-ABI (include/lbm.h) on one HIP device.
//
// A handle owns (or borrows) two population buffers and a stream, plus a few
// small device arrays: the descriptor, a one-entry tile list, the property
// table, the inlet rows and an instability flag.  Steps are enqueued as one
// launch of the step kernel each, or as HIP graphs of k launches followed
// by the descriptor advance.
#include <mutex>

#include "lbm_runtime.hpp"

using namespace lbmx;

namespace {
// Workgroups of the FP64 conservation reduction at most (each strides over
// nodes, so every grid fits).
constexpr int kMaxRedBlocks = 1024;
}  // namespace

// Partial sums of the no-allocation FP64 conservation reduction
// (lbm_conservation_noalloc): one per reduction workgroup, then the total.
// 32.8 KB.  Each device holds its own copy until the process ends.  In host
// code the name stands for no device address: host code reaches the array
// only through the pointer that hipGetSymbolAddress returns for the current
// device (scratch_on).
static __device__ __align__(256) RedPartial scratch[kMaxRedBlocks + 1];

struct lbm_handle {
  int device = 0;
  lbm_config cfg{};
  std::vector<double> nu_tab, al_tab;
  int prec = LBM_PREC_FP32;
  int layout = LBM_LAYOUT_TWO_BUFFERS;
  void *buf = nullptr;
  bool own_buf = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device arrays
  JetDesc *d_desc = nullptr;
  int32_t *d_tiles = nullptr;
  BatchHdr *d_hdr = nullptr;
  int32_t *d_flag = nullptr;
  float4 *d_table = nullptr;
  float4 *d_inlet = nullptr;
  Scratch scratch;
  JetDesc desc{};
  int64_t step = 0;  // steps done
  int32_t flip = 0;  // state after s steps in buf[(s + flip) & 1]
  // step0 and flip held by the device descriptor: they may lag step and flip
  // (directly launched steps pass the difference as koff and tog; a graph,
  // whose arguments are fixed, first brings them up to date)
  int64_t base = 0;
  int32_t dflip = 0;
  int shape = 0;
  int32_t ntiles = 0, grid = 0;
  bool unstable = false;
  int32_t graph_k = 0;
  hipGraphExec_t gexec = nullptr;
  int32_t gexec_k = 0, gexec_shape = -1;
};

namespace {

int32_t view_of(const lbm_handle *h, int64_t step) {
  return state_view_of(h->layout, step, h->flip);
}

int upload_desc(lbm_handle *h) {
  h->base = h->step;
  h->dflip = h->flip;
  h->desc.step0 = h->base;
  h->desc.flip = h->flip;
  LBM_HIP(hipMemcpyAsync(h->d_desc, &h->desc, sizeof(JetDesc), hipMemcpyHostToDevice, h->stream));
  LBM_HIP(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int set_shape(lbm_handle *h, int shape) {
  int n;
  tile_shapes(&n);
  if (shape < 0 || shape >= n) return LBM_EINVAL;
  if (h->layout == LBM_LAYOUT_SINGLE && shape != 0) return LBM_EINVAL;
  int32_t tx;
  h->ntiles = tiles_of(&h->cfg, shape, &tx);
  h->grid = (h->ntiles + 7) / 8 * 8;
  h->shape = shape;
  h->desc.tiles_x = tx;
  int32_t tl[2] = {0, h->ntiles};
  LBM_HIP(hipMemcpyAsync(h->d_tiles, tl, sizeof tl, hipMemcpyHostToDevice, h->stream));
  return upload_desc(h);
}

void drop_graph(lbm_handle *h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  h->gexec_k = 0;
  h->gexec_shape = -1;
}

// Sync, then fold the device instability flag into the sticky state.
int sync_and_check(lbm_handle *h) {
  LBM_HIP(hipStreamSynchronize(h->stream));
  LBM_HIP(hipGetLastError());
  int32_t flag = 0;
  LBM_HIP(hipMemcpy(&flag, h->d_flag, sizeof flag, hipMemcpyDeviceToHost));
  if (flag) h->unstable = true;
  return h->unstable ? LBM_EUNSTABLE : LBM_OK;
}

int clear_flag(lbm_handle *h) {
  const int32_t zero = 0;
  LBM_HIP(hipMemcpy(h->d_flag, &zero, sizeof zero, hipMemcpyHostToDevice));
  h->unstable = false;
  return LBM_OK;
}

void release(lbm_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  drop_graph(h);
  h->scratch.release();
  if (h->d_desc) (void)hipFree(h->d_desc);
  if (h->d_tiles) (void)hipFree(h->d_tiles);
  if (h->d_hdr) (void)hipFree(h->d_hdr);
  if (h->d_flag) (void)hipFree(h->d_flag);
  if (h->d_table) (void)hipFree(h->d_table);
  if (h->d_inlet) (void)hipFree(h->d_inlet);
  if (h->own_buf && h->buf) (void)hipFree(h->buf);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

int upload_inlet(lbm_handle *h, const std::vector<float4> &rows, int32_t n_t) {
  float4 *p = nullptr;
  LBM_HIP(hipStreamSynchronize(h->stream));
  if (hipMalloc(&p, rows.size() * sizeof(float4)) != hipSuccess) return LBM_ENOMEM;
  if (hipMemcpy(p, rows.data(), rows.size() * sizeof(float4), hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(p);
    return LBM_EDEVICE;
  }
  if (h->d_inlet) (void)hipFree(h->d_inlet);
  h->d_inlet = p;
  h->desc.inlet = p;
  h->desc.n_t = n_t;
  int rc = upload_desc(h);
  if (rc) return rc;
  // the inlet ghosts of the current buffer follow the new rows
  if ((rc = launch_ghost_fill(h->prec, h->stream, h->d_desc, &h->cfg, h->step, view_of(h, h->step)))) return rc;
  LBM_HIP(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int create_common(const lbm_config *cfg, void *dev_buf, size_t bytes, void *stream,
                  lbm_handle **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  int rc = validate_config(cfg, true);
  if (rc) return rc;
  lbm_handle *h = new (std::nothrow) lbm_handle();
  if (!h) return LBM_ENOMEM;
  h->cfg = *cfg;
  if (cfg->table_n > 0) {
    h->nu_tab.assign(cfg->nu_mult, cfg->nu_mult + cfg->table_n);
    h->al_tab.assign(cfg->alpha_mult, cfg->alpha_mult + cfg->table_n);
    h->cfg.nu_mult = h->nu_tab.data();
    h->cfg.alpha_mult = h->al_tab.data();
  }
  h->prec = cfg->precision;
  h->layout = cfg->layout;
  if (hipGetDevice(&h->device) != hipSuccess) {
    release(h);
    return LBM_EDEVICE;
  }
  const size_t one = buffer_bytes(cfg, h->prec);
  const size_t total = n_buffers(h->layout) * one;
  if (dev_buf) {
    if (bytes < total || ((uintptr_t)dev_buf & 255)) {
      release(h);
      return LBM_EINVAL;
    }
    h->buf = dev_buf;
    h->stream = (hipStream_t)stream;
  } else {
    if (hipMalloc(&h->buf, total) != hipSuccess) {
      release(h);
      return LBM_ENOMEM;
    }
    h->own_buf = true;
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      release(h);
      return LBM_EDEVICE;
    }
    h->own_stream = true;
  }
  std::vector<float4> table = make_table(&h->cfg);
  bool ok = hipMalloc(&h->d_desc, sizeof(JetDesc)) == hipSuccess &&
            hipMalloc(&h->d_tiles, 2 * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&h->d_hdr, sizeof(BatchHdr)) == hipSuccess &&
            hipMalloc(&h->d_flag, sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&h->d_table, table.size() * sizeof(float4)) == hipSuccess;
  if (!ok) {
    release(h);
    return LBM_ENOMEM;
  }
  BatchHdr hdr{1, {0, 0, 0}};
  const int32_t zero = 0;
  ok = hipMemcpy(h->d_table, table.data(), table.size() * sizeof(float4),
                 hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(h->d_hdr, &hdr, sizeof hdr, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(h->d_flag, &zero, sizeof zero, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    release(h);
    return LBM_EDEVICE;
  }
  JetDesc &d = h->desc;
  fill_desc(d, &h->cfg);
  d.buf[0] = h->buf;
  d.buf[1] = h->layout == LBM_LAYOUT_SINGLE ? h->buf : (char *)h->buf + one;
  d.table = h->d_table;
  d.target = NO_TARGET;
  d.slot = 0;
  std::vector<float4> rows;
  make_inlet(&h->cfg, 0, nullptr, nullptr, nullptr, rows);
  if ((rc = upload_inlet(h, rows, 1)) ||
      (rc = set_shape(h, h->layout == LBM_LAYOUT_SINGLE ? 0 : default_tile_shape(h->prec)))) {
    release(h);
    return rc;
  }
  // both buffers at the initial equilibrium, each with its ghost ring (the
  // constant ghosts of equilibrium sides are only ever written here; the
  // single buffer's step rewrites them itself)
  const float4 u0 =
      make_float4((float)cfg->rho0, (float)cfg->ux0, (float)cfg->ur0, (float)cfg->T0);
  for (int64_t q = n_buffers(h->layout) - 1; q >= 0 && !rc; --q) {
    const int32_t v = view_of(h, q);
    rc = launch_init(h->prec, h->stream, h->d_desc, &h->cfg, q, v, nullptr, u0);
    if (!rc) rc = launch_ghost_fill(h->prec, h->stream, h->d_desc, &h->cfg, q, v);
  }
  if (rc || hipStreamSynchronize(h->stream) != hipSuccess) {
    release(h);
    return rc ? rc : LBM_EDEVICE;
  }
  *out = h;
  return LBM_OK;
}

// One launch of one step: the in-place kernel for a single buffer, else the
// handle's shape.
int one_step(lbm_handle *h, int32_t koff, int32_t tog) {
  if (h->layout == LBM_LAYOUT_SINGLE)
    return launch_aa_step(h->prec, h->grid, h->stream, h->d_desc, h->d_tiles, h->d_hdr, koff,
                          h->d_flag);
  return launch_step(h->shape, h->prec, h->grid, h->stream, h->d_desc, h->d_tiles, h->d_hdr,
                     koff, tog, 1, h->d_flag);
}

// The launches of a group of k steps on `st`: with a two-step shape, k / 2
// pair launches (and one single step if k is odd), starting koff0 steps past
// the descriptor's step0 with its flip toggled by tog0; then, if `advance`,
// the descriptor advance (koff0 = tog0 = 0 then).
int enqueue_group(lbm_handle *h, int32_t k, bool pair, hipStream_t st, int32_t koff0 = 0,
                  int32_t tog0 = 0, bool advance = true) {
  int rc = LBM_OK;
  const int32_t np = pair ? k / 2 : 0;
  for (int32_t q = 0; q < np && !rc; ++q)
    rc = launch_step(h->shape, h->prec, h->grid, st, h->d_desc, h->d_tiles, h->d_hdr,
                     koff0 + 2 * q, tog0 ^ (q & 1), 2, h->d_flag);
  for (int32_t q = 2 * np; q < k && !rc; ++q)
    rc = h->layout == LBM_LAYOUT_SINGLE
             ? launch_aa_step(h->prec, h->grid, st, h->d_desc, h->d_tiles, h->d_hdr, koff0 + q,
                              h->d_flag)
             : launch_step(h->shape, h->prec, h->grid, st, h->d_desc, h->d_tiles, h->d_hdr,
                           koff0 + q, tog0 ^ (np & 1), 1, h->d_flag);
  if (!rc && advance) rc = launch_advance(st, h->d_desc, h->d_hdr, 1, k, np);
  return rc;
}

// Capture k steps as one graph (enqueue_group's launches).
int capture_group(lbm_handle *h, int32_t k, bool pair) {
  hipGraph_t g;
  LBM_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  const int crc = enqueue_group(h, k, pair, h->stream);
  const hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (crc || e != hipSuccess) return crc ? crc : LBM_EDEVICE;
  const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    h->gexec = nullptr;
    return LBM_EDEVICE;
  }
  h->gexec_k = k;
  h->gexec_shape = h->shape;
  return LBM_OK;
}

// Capture and upload the graph of the handle's group size and shape now, so
// that the first lbm_step that replays it pays no capture or instantiation.
int prepare_graph(lbm_handle *h) {
  if (h->graph_k <= 0) return LBM_OK;
  if (h->gexec && h->gexec_k == h->graph_k && h->gexec_shape == h->shape) return LBM_OK;
  drop_graph(h);
  int nsh;
  const int rc = capture_group(h, h->graph_k, tile_shapes(&nsh)[h->shape].steps == 2);
  if (rc) return rc;
  // (an optimisation only: the graph also uploads itself at its first launch)
  (void)hipGraphUpload(h->gexec, h->stream);
  // One dry replay, so that the first lbm_step does not pay the graph's
  // first launch: with the descriptor's target at its step0 every tile is
  // skipped and the advance leaves step0 and flip as they are, so the state
  // does not change.
  h->desc.target = h->step;  // (upload_desc sets step0 to the step count)
  int rc2 = upload_desc(h);
  if (!rc2 && hipGraphLaunch(h->gexec, h->stream) != hipSuccess) rc2 = LBM_EDEVICE;
  if (!rc2 && hipStreamSynchronize(h->stream) != hipSuccess) rc2 = LBM_EDEVICE;
  h->desc.target = NO_TARGET;
  const int rc3 = upload_desc(h);
  return rc2 ? rc2 : rc3;
}

// Brings the device descriptor's step0 and flip to the host's.
int catch_up(lbm_handle *h) {
  if (h->base == h->step && h->dflip == h->flip) return LBM_OK;
  const int rc = launch_advance(h->stream, h->d_desc, h->d_hdr, 1, (int32_t)(h->step - h->base),
                                h->flip ^ h->dflip);
  if (rc) return rc;
  h->base = h->step;
  h->dflip = h->flip;
  return LBM_OK;
}

int launch_steps(lbm_handle *h, int64_t n) {
  int nsh;
  const bool pair = tile_shapes(&nsh)[h->shape].steps == 2;
  int rc;
  while (n > 0) {
    const bool graph = h->graph_k > 0 && n >= h->graph_k;
    // (the lag is kept below 2^30 steps, so koff fits its 32 bits)
    if ((graph || h->step - h->base > (1 << 30)) && (rc = catch_up(h))) return rc;
    if (graph) {
      if (!h->gexec || h->gexec_k != h->graph_k || h->gexec_shape != h->shape) {
        drop_graph(h);
        if ((rc = capture_group(h, h->graph_k, pair))) return rc;
      }
      LBM_HIP(hipGraphLaunch(h->gexec, h->stream));
      h->step += h->graph_k;
      h->base += h->graph_k;
      if (pair) {
        h->flip ^= (h->graph_k / 2) & 1;
        h->dflip ^= (h->graph_k / 2) & 1;
      }
      n -= h->graph_k;
    } else if (pair) {
      // the rest (fewer steps than a graph holds) as directly launched
      // steps: a graph's launches, offset from the descriptor, and no
      // advance (the device starts on the first kernel while the host
      // enqueues the rest)
      const int32_t m = (int32_t)std::min<int64_t>(n, 1 << 20);
      if ((rc = enqueue_group(h, m, true, h->stream, (int32_t)(h->step - h->base),
                              h->flip ^ h->dflip, false)))
        return rc;
      h->step += m;
      h->flip ^= (m / 2) & 1;
      n -= m;
    } else {
      rc = one_step(h, (int32_t)(h->step - h->base), h->flip ^ h->dflip);
      if (rc) return rc;
      h->step += 1;
      n -= 1;
    }
  }
  return LBM_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
RedPartial *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, resolved once per device with
// that device current.
int scratch_on(int device, RedPartial **out) {
  if (device < 0 || device >= kMaxDevices) return LBM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    LBM_HIP(hipGetDevice(&cur));
    if (cur != device) LBM_HIP(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return LBM_EDEVICE;
    g_scratch_ptr[device] = (RedPartial *)p;
  }
  *out = g_scratch_ptr[device];
  return LBM_OK;
}

// Reduction workgroups of the conservation kernels for a grid (the same
// count in both conservation entry points, so their sums agree bit for bit).
int red_blocks(const lbm_handle *h) {
  const int64_t nodes = (int64_t)h->cfg.nx * h->cfg.nr;
  return (int)std::min<int64_t>(kMaxRedBlocks, (nodes + RED_THREADS - 1) / RED_THREADS);
}

// Both conservation entry points: reduce into `part` (nblocks partials and
// the total after them), wait, read the total back.
int conservation_into(lbm_handle *h, RedPartial *part, int nblocks, double *mass3d,
                      double *energy3d) {
  const int64_t nodes = (int64_t)h->cfg.nx * h->cfg.nr;
  int rc;
  if ((rc = launch_conservation(h->prec, h->stream, h->d_desc, nodes, h->step,
                                view_of(h, h->step), part, nblocks, part + nblocks)))
    return rc;
  const int st = sync_and_check(h);
  if (st == LBM_EDEVICE) return st;
  RedPartial r;
  LBM_HIP(hipMemcpy(&r, part + nblocks, sizeof r, hipMemcpyDeviceToHost));
  *mass3d = r.mass;
  *energy3d = r.energy;
  if (r.bad != 0.0) h->unstable = true;
  return h->unstable ? LBM_EUNSTABLE : LBM_OK;
}

}  // namespace

extern "C" {

int lbm_bytes_required(const lbm_config *cfg, size_t *bytes) {
  if (!bytes) return LBM_EINVAL;
  const int rc = validate_config(cfg, true);
  if (rc) return rc;
  *bytes = n_buffers(cfg->layout) * buffer_bytes(cfg, cfg->precision);
  return LBM_OK;
}

int lbm_create(const lbm_config *cfg, lbm_handle **out) {
  return create_common(cfg, nullptr, 0, nullptr, out);
}

int lbm_create_in(const lbm_config *cfg, void *dev_buf, size_t bytes, void *hip_stream,
                  lbm_handle **out) {
  if (!dev_buf) return out ? (*out = nullptr, LBM_EINVAL) : LBM_EINVAL;
  return create_common(cfg, dev_buf, bytes, hip_stream, out);
}

void lbm_destroy(lbm_handle *h) { release(h); }

int lbm_set_inlet(lbm_handle *h, int32_t n_t, const double *ux, const double *ur,
                  const double *T) {
  if (!h || n_t < 1) return LBM_EINVAL;
  std::vector<float4> rows;
  const int rc = make_inlet(&h->cfg, n_t, ux, ur, T, rows);
  if (rc) return rc;
  return upload_inlet(h, rows, n_t);
}

int lbm_step(lbm_handle *h, int64_t n_steps) {
  if (!h || n_steps < 0) return LBM_EINVAL;
  if (h->unstable) return LBM_EUNSTABLE;
  return launch_steps(h, n_steps);
}

int64_t lbm_step_count(const lbm_handle *h) { return h ? h->step : -1; }

void *lbm_stream(const lbm_handle *h) { return h ? (void *)h->stream : nullptr; }

int lbm_sync(lbm_handle *h) {
  if (!h) return LBM_EINVAL;
  return sync_and_check(h);
}

int lbm_set_graph_steps(lbm_handle *h, int32_t k) {
  if (!h || k < 0) return LBM_EINVAL;
  LBM_HIP(hipStreamSynchronize(h->stream));
  h->graph_k = k;
  if (k == 0) drop_graph(h);
  return prepare_graph(h);
}

int lbm_set_tile_shape(lbm_handle *h, int32_t index) {
  if (!h) return LBM_EINVAL;
  LBM_HIP(hipStreamSynchronize(h->stream));
  // bring the descriptor's step0 up to date before re-uploading it
  h->base = h->step;
  const int rc = set_shape(h, index);
  drop_graph(h);
  return rc ? rc : prepare_graph(h);
}

int lbm_moments(lbm_handle *h, double *rho, double *ux, double *ur, double *T) {
  if (!h) return LBM_EINVAL;
  const int64_t nodes = (int64_t)h->cfg.nx * h->cfg.nr;
  void *p;
  int rc = h->scratch.get(nodes * sizeof(float4), &p);
  if (rc) return rc;
  if ((rc = launch_moments(h->prec, h->stream, h->d_desc, &h->cfg, h->step, view_of(h, h->step),
                             (float4 *)p)))
    return rc;
  const int st = sync_and_check(h);
  if (st == LBM_EDEVICE) return st;
  std::vector<float4> m((size_t)nodes);
  LBM_HIP(hipMemcpy(m.data(), p, nodes * sizeof(float4), hipMemcpyDeviceToHost));
  bool finite = true;
  for (int64_t n = 0; n < nodes; ++n) {
    if (rho) rho[n] = m[n].x;
    if (ux) ux[n] = m[n].y;
    if (ur) ur[n] = m[n].z;
    if (T) T[n] = m[n].w;
    finite = finite && std::isfinite(m[n].x) && std::isfinite(m[n].w) && m[n].x > 0.f;
  }
  if (!finite) h->unstable = true;
  return h->unstable ? LBM_EUNSTABLE : LBM_OK;
}

int lbm_profiles(lbm_handle *h, double *ux_axis, double *T_axis, double *ux_exit,
                 double *T_exit) {
  if (!h) return LBM_EINVAL;
  const int n = h->cfg.nx + h->cfg.nr;
  void *p;
  int rc = h->scratch.get(n * sizeof(float2), &p);
  if (rc) return rc;
  if ((rc = launch_profiles(h->prec, h->stream, h->d_desc, &h->cfg, h->step, view_of(h, h->step),
                              (float2 *)p)))
    return rc;
  const int st = sync_and_check(h);
  if (st == LBM_EDEVICE) return st;
  std::vector<float2> v(n);
  LBM_HIP(hipMemcpy(v.data(), p, n * sizeof(float2), hipMemcpyDeviceToHost));
  for (int i = 0; i < h->cfg.nx; ++i) {
    if (ux_axis) ux_axis[i] = v[i].x;
    if (T_axis) T_axis[i] = v[i].y;
  }
  for (int j = 0; j < h->cfg.nr; ++j) {
    if (ux_exit) ux_exit[j] = v[h->cfg.nx + j].x;
    if (T_exit) T_exit[j] = v[h->cfg.nx + j].y;
  }
  return st;
}

int lbm_conservation(lbm_handle *h, double *mass3d, double *energy3d) {
  if (!h || !mass3d || !energy3d) return LBM_EINVAL;
  const int nblocks = red_blocks(h);
  void *p;
  const int rc = h->scratch.get((nblocks + 1) * sizeof(RedPartial), &p);
  if (rc) return rc;
  return conservation_into(h, (RedPartial *)p, nblocks, mass3d, energy3d);
}

int lbm_conservation_noalloc(lbm_handle *h, double *mass3d, double *energy3d) {
  if (!h || !mass3d || !energy3d) return LBM_EINVAL;
  const int nblocks = red_blocks(h);
  if (nblocks > kMaxRedBlocks) return LBM_EINVAL;
  RedPartial *part;
  const int rc = scratch_on(h->device, &part);
  if (rc) return rc;
  return conservation_into(h, part, nblocks, mass3d, energy3d);
}

int lbm_set_state(lbm_handle *h, const double *rho, const double *ux, const double *ur,
                  const double *T) {
  if (!h || !rho || !ux || !ur || !T) return LBM_EINVAL;
  const int64_t nodes = (int64_t)h->cfg.nx * h->cfg.nr;
  std::vector<float4> s((size_t)nodes);
  for (int64_t n = 0; n < nodes; ++n) {
    if (!(rho[n] > 0.0) || !std::isfinite(rho[n]) || !std::isfinite(ux[n]) ||
        !std::isfinite(ur[n]) || !std::isfinite(T[n]))
      return LBM_EINVAL;
    s[n] = make_float4((float)rho[n], (float)ux[n], (float)ur[n], (float)T[n]);
  }
  void *p;
  int rc = h->scratch.get(nodes * sizeof(float4), &p);
  if (rc) return rc;
  LBM_HIP(hipStreamSynchronize(h->stream));
  LBM_HIP(hipMemcpy(p, s.data(), nodes * sizeof(float4), hipMemcpyHostToDevice));
  if ((rc = launch_init(h->prec, h->stream, h->d_desc, &h->cfg, h->step, view_of(h, h->step),
                        (const float4 *)p, make_float4(0, 0, 0, 0))))
    return rc;
  if ((rc = launch_ghost_fill(h->prec, h->stream, h->d_desc, &h->cfg, h->step, view_of(h, h->step)))) return rc;
  LBM_HIP(hipStreamSynchronize(h->stream));
  return clear_flag(h);
}

int lbm_get_populations(lbm_handle *h, double *f, double *g) {
  if (!h) return LBM_EINVAL;
  const int64_t nodes = (int64_t)h->cfg.nx * h->cfg.nr;
  void *p;
  int rc = h->scratch.get(NPOP * nodes * sizeof(float), &p);
  if (rc) return rc;
  if ((rc = launch_decode(h->prec, h->stream, h->d_desc, &h->cfg, h->step, view_of(h, h->step),
                           (float *)p)))
    return rc;
  const int st = sync_and_check(h);
  if (st == LBM_EDEVICE) return st;
  std::vector<float> v((size_t)(NPOP * nodes));
  LBM_HIP(hipMemcpy(v.data(), p, v.size() * sizeof(float), hipMemcpyDeviceToHost));
  for (int64_t q = 0; q < 9 * nodes; ++q)
    if (f) f[q] = v[q];
  for (int64_t q = 0; q < 4 * nodes; ++q)
    if (g) g[q] = v[9 * nodes + q];
  return st;
}

int lbm_set_populations(lbm_handle *h, const double *f, const double *g, int64_t step) {
  if (!h || !f || !g || step < 0) return LBM_EINVAL;
  const int64_t nodes = (int64_t)h->cfg.nx * h->cfg.nr;
  std::vector<float> v((size_t)(NPOP * nodes));
  for (int64_t q = 0; q < 9 * nodes; ++q) {
    if (!std::isfinite(f[q])) return LBM_EINVAL;
    v[q] = (float)f[q];
  }
  for (int64_t q = 0; q < 4 * nodes; ++q) {
    if (!std::isfinite(g[q])) return LBM_EINVAL;
    v[9 * nodes + q] = (float)g[q];
  }
  void *p;
  int rc = h->scratch.get(v.size() * sizeof(float), &p);
  if (rc) return rc;
  LBM_HIP(hipStreamSynchronize(h->stream));
  LBM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice));
  h->step = step;
  h->base = step;
  if ((rc = upload_desc(h))) return rc;
  if ((rc = launch_encode(h->prec, h->stream, h->d_desc, &h->cfg, step, view_of(h, step),
                           (const float *)p)))
    return rc;
  if ((rc = launch_ghost_fill(h->prec, h->stream, h->d_desc, &h->cfg, step, view_of(h, step)))) return rc;
  LBM_HIP(hipStreamSynchronize(h->stream));
  return clear_flag(h);
}

const char *lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument or configuration";
    case LBM_ENOMEM: return "out of memory or budget";
    case LBM_EUNSTABLE: return "unstable: non-finite value or non-positive density";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_ESTATE: return "call not valid in the current state";
    default: return "unknown error";
  }
}

}  // extern "C"
