// lbm_runtime.hpp -- host-side pieces shared by the single-jet and batch
// runtimes: validation, descriptor setup, kernel tables, small helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

namespace lbmx {

#define LBM_HIP(expr)                              \
  do {                                             \
    if ((expr) != hipSuccess) return LBM_EDEVICE;  \
  } while (0)

constexpr int64_t NO_TARGET = INT64_MAX / 4;

inline int storage_bytes(int prec) { return prec == LBM_PREC_FP32 ? 4 : 2; }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of one population buffer (13 planes with their ghost rings).
inline size_t buffer_bytes(const lbm_config *c, int prec) {
  return align256((size_t)NPOP * (size_t)layout_plane(c->nx, c->nr) * storage_bytes(prec));
}

// Buffers per jet: two, or one in place.
inline int n_buffers(int layout) { return layout == LBM_LAYOUT_SINGLE ? 1 : 2; }

// The view (see State in lbm_device.hpp) of the state after `step` steps.
inline int32_t state_view_of(int layout, int64_t step, int32_t flip) {
  if (layout == LBM_LAYOUT_SINGLE) return 2 + (int32_t)(step & 1);
  return (int32_t)((step + flip) & 1);
}

int validate_config(const lbm_config *c, bool check_precision);

// Host copy of the property tables as (M, dM) pairs at each grid point.
std::vector<float4> make_table(const lbm_config *c);

// Fill the physics fields of a descriptor (no buffers, table or inlet).
void fill_desc(JetDesc &d, const lbm_config *c);

// Inlet rows as float4 (ux, ur, T, 0); n_t == 0 gives one ambient row.
int make_inlet(const lbm_config *c, int32_t n_t, const double *ux, const double *ur,
               const double *T, std::vector<float4> &out);

// ---- kernel tables ---------------------------------------------------------
// A launch variant: block (bx, by), tile (bx * nx) x (by * ny) nodes, the
// occupancy target, the cache policy, and the steps one launch advances
// (2: the LDS-blocked two-step kernel).
struct TileShape {
  int bx, by, ny, nx, waves, cache, steps, lds;
  const void *fn[4];  // FP32, FP16-dev, BF16-dev, FP16-dev rounded stochastically
};
const TileShape *tile_shapes(int *count);
int default_tile_shape(int prec);

inline int codec_index(int prec) { return prec - LBM_PREC_FP32; }

// One launch of tile shape `shape`: the step (or pair) at step0 + koff, with
// `tog` the parity of two-step launches since the last advance and nsteps
// (1 or 2) the steps a two-step kernel may take.
int launch_step(int shape, int prec, int grid, hipStream_t st, const JetDesc *jets,
                const int32_t *tiles, const BatchHdr *hdr, int32_t koff, int32_t tog,
                int32_t nsteps, int32_t *flags);
// Advance after a group of delta steps whose first npair launches were
// two-step launches.
int launch_advance(hipStream_t st, JetDesc *jets, const BatchHdr *hdr, int32_t njets_max,
                   int32_t delta, int32_t npair);
// Single-buffer step over shape 0's tile list.
int launch_aa_step(int prec, int grid, hipStream_t st, const JetDesc *jets, const int32_t *tiles,
                   const BatchHdr *hdr, int32_t koff, int32_t *flags);
// Helpers on the state after `step` steps, seen through `view`
// (state_view_of).
int launch_init(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step,
                int32_t view, const float4 *state, float4 u0);
int launch_ghost_fill(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c,
                      int64_t step, int32_t view);
int launch_moments(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c,
                   int64_t step, int32_t view, float4 *out);
int launch_profiles(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c,
                    int64_t step, int32_t view, float2 *out);
int launch_conservation(int prec, hipStream_t st, const JetDesc *d, int64_t nodes, int64_t step,
                        int32_t view, RedPartial *partial, int nblocks, RedPartial *out);
int launch_decode(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step,
                  int32_t view, float *out);
int launch_encode(int prec, hipStream_t st, const JetDesc *d, const lbm_config *c, int64_t step,
                  int32_t view, const float *in);

int tiles_of(const lbm_config *c, int shape, int32_t *tiles_x);

// Workgroups of the step kernel of `shape` (or of the single-buffer kernel)
// that the current device holds at once: one full wave of a persistent grid.
int resident_workgroups(int shape, int prec, bool single_buffer);

// Simple device scratch that grows on demand.
struct Scratch {
  void *p = nullptr;
  size_t bytes = 0;
  int get(size_t need, void **out) {
    if (need > bytes) {
      if (p) (void)hipFree(p);
      p = nullptr;
      bytes = 0;
      if (hipMalloc(&p, need) != hipSuccess) return LBM_ENOMEM;
      bytes = need;
    }
    *out = p;
    return LBM_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

}  // namespace lbmx
