// lbm_kernels.hpp -- kernels of the gfx950 LBM-LES step and its helpers.
#pragma once

#include "lbm_device.hpp"

namespace lbmx {

// ---------------------------------------------------------------------------
// The fused collide-and-stream step over a flat tile list covering every
// active jet.  A tile is BX x (BY * NY) nodes; thread (tx, ty) handles column
// tile_x * BX + tx and rows tile_y * BY * NY + ty + q * BY, q < NY.
// Workgroups walk the tile list with a grid stride; within each round the
// tiles handed to one XCD (workgroup id mod 8) are contiguous, so the
// neighbouring columns that the shifted pulls share stay in one L2.
// The jet's state after s steps lives in buf[s & 1]; the step taken here is
// step0 + koff, skipped once the jet reaches its target.
// ---------------------------------------------------------------------------
template <class C, int BX, int BY, int NY>
__global__ __launch_bounds__(BX *BY) void step_kernel(const JetDesc *__restrict__ jets,
                                                      const int32_t *__restrict__ tile_start,
                                                      const BatchHdr *__restrict__ hdr,
                                                      int32_t koff, int32_t *__restrict__ flags) {
  const int32_t njets = hdr->njets;
  const int32_t ntiles = tile_start[njets];
  const int32_t G = gridDim.x;  // a multiple of 8
  const int32_t per_xcd = G >> 3;
  const int32_t b = blockIdx.x;
  for (int32_t t = (b & 7) * per_xcd + (b >> 3); t < ntiles; t += G) {
    int32_t jid = 0;
    if (njets > 1) {  // last jet whose first tile is <= t
      int32_t lo = 0, hi = njets - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
      }
      jid = lo;
    }
    const JetDesc &d = jets[jid];
    const int64_t step = d.step0 + koff;
    if (step >= d.target) continue;
    const int32_t lt = t - tile_start[jid];
    const int32_t ty = lt / d.tiles_x;
    const int32_t tx = lt - ty * d.tiles_x;
    const int i = tx * BX + (int)threadIdx.x;
    Src<C> s{static_cast<const typename C::T *>(d.buf[step & 1]), d.plane, d.pitch};
    typename C::T *__restrict__ dst = static_cast<typename C::T *>(d.buf[(step + 1) & 1]);
    const float4 *inrow = d.inlet + (int64_t)(step % d.n_t) * d.nr;
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NY; ++q) {
      const int j = ty * (BY * NY) + (int)threadIdx.y + q * BY;
      if (i >= d.nx || j >= d.nr) continue;
      float f[9], g[4];
      pull_node<C>(d, s, i, j, inrow, f, g);
      const float r = d.r0 + (float)j + 0.5f;
      ok &= collide(d, fast_rcp(r), r * r, f, g);
      typename C::T *o = dst + (int64_t)j * d.pitch + i;
#pragma unroll
      for (int p = 0; p < NPOP; ++p)
        o[(int64_t)p * d.plane] = C::enc(p < 9 ? f[p] : g[p - 9], pop_offset<C>(d, p));
    }
    if (!ok) flags[d.slot] = 1;
  }
}

// Moves every jet's step0 by delta (clamped at the target); ends a captured
// group of steps so that the same graph serves the next group.
__global__ void advance_kernel(JetDesc *__restrict__ jets, const BatchHdr *__restrict__ hdr,
                               int32_t delta) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < hdr->njets) {
    const int64_t s = jets[q].step0 + delta;
    jets[q].step0 = s < jets[q].target ? s : jets[q].target;
  }
}

// Equilibrium fill of buf[step & 1] from fields (float4 rho, ux, ur, T per
// node, i fastest) or, with state == nullptr, from the uniform u0.
template <class C>
__global__ void init_kernel(const JetDesc *__restrict__ dp, int64_t step,
                            const float4 *__restrict__ state, float4 u0) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= d.nx) return;
  const float4 q = state ? state[(int64_t)j * d.nx + i] : u0;
  typename C::T *o = static_cast<typename C::T *>(d.buf[step & 1]) + (int64_t)j * d.pitch + i;
#pragma unroll
  for (int p = 0; p < NPOP; ++p)
    o[(int64_t)p * d.plane] = C::enc(eq_plane(p, q.x, q.y, q.z, q.w), pop_offset<C>(d, p));
}

// Pre-collision moments (eq. 2) of buf[step & 1] at step `step`:
// float4 (rho, ux, ur, T) per node, i fastest.
template <class C>
__global__ void moments_kernel(const JetDesc *__restrict__ dp, int64_t step,
                               float4 *__restrict__ out) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= d.nx) return;
  Src<C> s{static_cast<const typename C::T *>(d.buf[step & 1]), d.plane, d.pitch};
  const float4 *inrow = d.inlet + (int64_t)(step % d.n_t) * d.nr;
  float f[9], g[4];
  pull_node<C>(d, s, i, j, inrow, f, g);
  const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const float mx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const float mr = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const float T = (g[0] + g[1]) + (g[2] + g[3]);
  out[(int64_t)j * d.nx + i] = make_float4(rho, mx / rho, mr / rho, T);
}

// Centreline (j = 0) and exit column (i = nx-1): (ux, T) pairs, nx + nr.
template <class C>
__global__ void profiles_kernel(const JetDesc *__restrict__ dp, int64_t step,
                                float2 *__restrict__ out) {
  const JetDesc &d = *dp;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.nx + d.nr) return;
  const int i = t < d.nx ? t : d.nx - 1;
  const int j = t < d.nx ? 0 : t - d.nx;
  Src<C> s{static_cast<const typename C::T *>(d.buf[step & 1]), d.plane, d.pitch};
  const float4 *inrow = d.inlet + (int64_t)(step % d.n_t) * d.nr;
  float f[9], g[4];
  pull_node<C>(d, s, i, j, inrow, f, g);
  const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const float mx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  out[t] = make_float2(mx / rho, (g[0] + g[1]) + (g[2] + g[3]));
}

// FP64 conservation sums of the pre-collision moments: each workgroup takes
// a fixed strided set of nodes, sums r_j rho and r_j T in double in a fixed
// order, reduces in LDS with a fixed tree and writes one partial; a second
// kernel reduces the partials the same way.  Results are bitwise
// reproducible for a given grid.  Also counts nodes with rho <= 0 or a
// non-finite rho or T.
template <class C>
__global__ __launch_bounds__(RED_THREADS) void conservation_kernel(
    const JetDesc *__restrict__ dp, int64_t step, RedPartial *__restrict__ partial) {
  const JetDesc &d = *dp;
  Src<C> s{static_cast<const typename C::T *>(d.buf[step & 1]), d.plane, d.pitch};
  const float4 *inrow = d.inlet + (int64_t)(step % d.n_t) * d.nr;
  const int64_t nodes = (int64_t)d.nx * d.nr;
  double m = 0.0, e = 0.0, bad = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; n < nodes;
       n += (int64_t)gridDim.x * RED_THREADS) {
    const int j = (int)(n / d.nx), i = (int)(n - (int64_t)j * d.nx);
    float f[9], g[4];
    pull_node<C>(d, s, i, j, inrow, f, g);
    const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const float T = (g[0] + g[1]) + (g[2] + g[3]);
    const double r = (double)d.r0 + (double)j + 0.5;
    m += r * (double)rho;
    e += r * (double)T;
    if (!((rho > 0.0f) && (rho < __builtin_inff()) && (fabsf(T) < __builtin_inff()))) bad += 1.0;
  }
  __shared__ double sm[RED_THREADS], se[RED_THREADS], sb[RED_THREADS];
  sm[threadIdx.x] = m;
  se[threadIdx.x] = e;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sm[threadIdx.x] += sm[threadIdx.x + w];
      se[threadIdx.x] += se[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = RedPartial{sm[0], se[0], sb[0], 0.0};
}

__global__ __launch_bounds__(RED_THREADS) void reduce_partials_kernel(
    const RedPartial *__restrict__ partial, int32_t n, RedPartial *__restrict__ out) {
  double m = 0.0, e = 0.0, bad = 0.0;
  for (int q = threadIdx.x; q < n; q += RED_THREADS) {
    m += partial[q].mass;
    e += partial[q].energy;
    bad += partial[q].bad;
  }
  __shared__ double sm[RED_THREADS], se[RED_THREADS], sb[RED_THREADS];
  sm[threadIdx.x] = m;
  se[threadIdx.x] = e;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sm[threadIdx.x] += sm[threadIdx.x + w];
      se[threadIdx.x] += se[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = RedPartial{sm[0], se[0], sb[0], 0.0};
}

// Stored populations <-> dense FP32 planes (13 x nr x nx, no pitch).
template <class C>
__global__ void decode_kernel(const JetDesc *__restrict__ dp, int64_t step,
                              float *__restrict__ out) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, p = blockIdx.z;
  if (i >= d.nx) return;
  const typename C::T *b = static_cast<const typename C::T *>(d.buf[step & 1]);
  out[((int64_t)p * d.nr + j) * d.nx + i] =
      C::dec(b[(int64_t)p * d.plane + (int64_t)j * d.pitch + i], pop_offset<C>(d, p));
}

template <class C>
__global__ void encode_kernel(const JetDesc *__restrict__ dp, int64_t step,
                              const float *__restrict__ in) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, p = blockIdx.z;
  if (i >= d.nx) return;
  typename C::T *b = static_cast<typename C::T *>(d.buf[step & 1]);
  b[(int64_t)p * d.plane + (int64_t)j * d.pitch + i] =
      C::enc(in[((int64_t)p * d.nr + j) * d.nx + i], pop_offset<C>(d, p));
}

// Plain streaming copy, 16 B per lane per iteration.
__global__ __launch_bounds__(256) void copy_kernel(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    dst[q] = src[q];
}

}  // namespace lbmx
