// lbm_kernels.hpp -- kernels of the gfx950 LBM-LES step and its helpers.
#pragma once

#include "lbm_device.hpp"

namespace lbmx {

// Raw buffer access of B bytes per lane (buffer instructions: the base sits in
// a scalar resource, one 32-bit VGPR offset is shared by all planes).
constexpr int32_t BUF_WORD3 = 0x00020000;  // 32-bit data format, gfx9 family

template <int B> struct Raw;
template <> struct Raw<2> { typedef uint16_t type; };
template <> struct Raw<4> { typedef uint32_t type; };
template <> struct Raw<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct Raw<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

// AUX is the cache-policy field of the instruction (2: non-temporal).
template <int B, int AUX>
__device__ __forceinline__ typename Raw<B>::type buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                          uint32_t soff) {
  if constexpr (B == 2) return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, AUX);
  else if constexpr (B == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX);
  else if constexpr (B == 8) return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
  else return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX);
}
template <int B, int AUX>
__device__ __forceinline__ void buf_store(typename Raw<B>::type v, __amdgpu_buffer_rsrc_t r,
                                          uint32_t voff, uint32_t soff) {
  if constexpr (B == 2) __builtin_amdgcn_raw_buffer_store_b16(v, r, voff, soff, AUX);
  else if constexpr (B == 4) __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, AUX);
  else if constexpr (B == 8) __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, AUX);
  else __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, AUX);
}
constexpr int CACHE_NT = 2;

// NX elements of storage type T packed in one raw word
template <class T, int NX>
struct Pack {
  typedef T vec __attribute__((ext_vector_type(NX)));
};
template <class T>
struct Pack<T, 1> {
  typedef T vec;
};

template <class T, int NX>
__device__ __forceinline__ T elem(const typename Pack<T, NX>::vec &v, int e) {
  if constexpr (NX == 1) return v;
  else return v[e];
}

// Tile walk of every step kernel.  The dispatcher deals workgroups round-robin
// over the eight XCDs, so workgroup b runs on XCD b mod 8.  Each XCD takes an
// equal contiguous share of the tile list, [ntiles x / 8, ntiles (x + 1) / 8),
// and its gridDim.x / 8 workgroups walk it with that stride.  The tiles whose
// x-shifted pulls share columns then sit in one L2, and no XCD idles while
// the others still hold tiles, whatever ntiles is against the grid size.
// With one workgroup per tile (rounded up to a multiple of 8) a workgroup gets
// at most one tile.  The grid is a multiple of 8.
struct TileWalk {
  int32_t first, end, stride;
};
__device__ __forceinline__ TileWalk tile_walk(int32_t ntiles) {
  const int32_t b = (int32_t)blockIdx.x, x = b & 7;
  const int32_t lo = (int32_t)(((int64_t)ntiles * x) >> 3);
  const int32_t hi = (int32_t)(((int64_t)ntiles * (x + 1)) >> 3);
  return {lo + (b >> 3), hi, (int32_t)(gridDim.x >> 3)};
}

// ---------------------------------------------------------------------------
// The fused collide-and-stream step over a flat tile list covering every
// active jet.  A tile is (BX * NX) x (BY * NY) nodes: thread (tx, ty) handles
// NX consecutive columns starting at (tile_x * BX + tx) * NX and rows
// tile_y * BY * NY + ty + q * BY, q < NY.  The source buffer's ghost ring is
// current, so every thread reads each plane with one buffer load of NX
// elements and writes with one buffer store; edge nodes then write the
// ghost values of the next step that they are the source of.
// Workgroups walk the tile list as tile_walk() assigns it.  W is the
// occupancy target (waves per SIMD) for register allocation; CP selects non-temporal stores (bit 0) and loads (bit 1).
// The jet's state after s steps lives in buf[(s + flip) & 1], where flip is
// the descriptor's value toggled by `tog` (the parity of the two-step
// launches issued since the descriptor was last advanced); the step taken
// here is step0 + koff, skipped once the jet reaches its target.  `nsteps`
// is unused (the two-step kernel below shares this signature).
// ---------------------------------------------------------------------------
template <class C, int BX, int BY, int NY, int NX, int W, int CP>
__global__ __launch_bounds__(BX *BY) __attribute__((amdgpu_waves_per_eu(W, 8))) void step_kernel(
    const JetDesc *__restrict__ jets, const int32_t *__restrict__ tile_start,
    const BatchHdr *__restrict__ hdr, int32_t koff, int32_t tog, int32_t nsteps,
    int32_t *__restrict__ flags) {
  using T = typename C::T;
  constexpr int ES = (int)sizeof(T);
  constexpr int VB = ES * NX;  // bytes per lane per plane
  using VT = typename Pack<T, NX>::vec;
  const int32_t njets = hdr->njets;
  const int32_t ntiles = tile_start[njets];
  const TileWalk tw = tile_walk(ntiles);
  for (int32_t t = tw.first; t < tw.end; t += tw.stride) {
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
    const int i0 = (tx * BX + (int)threadIdx.x) * NX;
    const int64_t sel = step + (d.flip ^ tog);
    T *src_raw = static_cast<T *>(d.buf[sel & 1]);
    T *dst_raw = static_cast<T *>(d.buf[(sel + 1) & 1]);
    const uint32_t pitch_b = (uint32_t)d.pitch * ES, plane_b = (uint32_t)d.plane * ES;
    const uint32_t span = (uint32_t)NPOP * plane_b;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(src_raw, 0, (int)span, BUF_WORD3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(dst_raw, 0, (int)span, BUF_WORD3);
    const int j_lo = ty * (BY * NY);
    const bool tile_edge = (tx == 0) | ((tx + 1) * BX * NX >= d.nx) | (j_lo == 0) |
                           (j_lo + BY * NY >= d.nr);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NY; ++q) {
      const int j = j_lo + (int)threadIdx.y + q * BY;
      if (i0 >= d.nx || j >= d.nr) continue;
      float f[NX][9], g[NX][4];
      const uint32_t voff = (uint32_t)node_index(d.pitch, i0, j) * ES;
#pragma unroll
      for (int p = 0; p < NPOP; ++p) {
        // pulled from node (i - e_x, j - e_r); the offset is never negative
        // because plane p >= 1 starts at least a plane after the buffer
        const uint32_t soff = (uint32_t)p * plane_b - (uint32_t)(per(p) * (int)pitch_b) -
                              (uint32_t)(pex(p) * ES);
        const VT v = __builtin_bit_cast(VT, buf_load<VB, (CP & 2) ? CACHE_NT : 0>(rs, voff, soff));
        const float off = pop_offset<C>(d, p);
#pragma unroll
        for (int e = 0; e < NX; ++e) {
          const float x = C::dec(elem<T, NX>(v, e), off);
          if (p < 9) f[e][p] = x; else g[e][p - 9] = x;
        }
      }
      const float r = d.r0 + (float)j + 0.5f;
      const float rinv = fast_rcp(r), r2 = r * r;
#pragma unroll
      for (int e = 0; e < NX; ++e) {
        const bool okn = collide(d, rinv, r2, f[e], g[e]);
        ok &= okn | (i0 + e >= d.nx);
      }
      uint32_t key[NX];
#pragma unroll
      for (int e = 0; e < NX; ++e) key[e] = sr_key(i0 + e, j, step + 1);
      if (i0 + NX <= d.nx) {
#pragma unroll
        for (int p = 0; p < NPOP; ++p) {
          const float off = pop_offset<C>(d, p);
          VT v;
#pragma unroll
          for (int e = 0; e < NX; ++e) {
            const T x = C::enc(p < 9 ? f[e][p] : g[e][p - 9], off, plane_key(key[e], p));
            if constexpr (NX == 1) v = x; else v[e] = x;
          }
          buf_store<VB, (CP & 1) ? CACHE_NT : 0>(__builtin_bit_cast(typename Raw<VB>::type, v), rd,
                                                 voff, (uint32_t)p * plane_b);
        }
      } else {
        const gptr<T> o = as_global(dst_raw) + node_index(d.pitch, i0, j);
#pragma unroll
        for (int e = 0; e < NX; ++e)
          if (i0 + e < d.nx)
#pragma unroll
            for (int p = 0; p < NPOP; ++p)
              o[(int64_t)p * d.plane + e] = C::enc(p < 9 ? f[e][p] : g[e][p - 9],
                                                   pop_offset<C>(d, p), plane_key(key[e], p));
      }
      if (tile_edge) {
        const Dst<C> o{as_global(dst_raw), d.plane, d.pitch};
        const float4 *in_next =
            (tx == 0 && d.bc[0] == BC_INLET) ? d.inlet + (int64_t)((step + 1) % d.n_t) * d.nr
                                              : d.inlet;
#pragma unroll
        for (int e = 0; e < NX; ++e) {
          const int i = i0 + e;
          if (i < d.nx && ((i == 0) | (i == d.nx - 1) | (j == 0) | (j == d.nr - 1)))
            ghost_epilogue<C>(d, o, i, j, f[e], g[e], in_next, key[e]);
        }
      }
    }
    if (!ok) flags[d.slot] = 1;
  }
}

// ---------------------------------------------------------------------------
// Node-wise pieces of the two-step kernel (one node per lane).
// ---------------------------------------------------------------------------
// The 13 raw storage words node (voff) pulls from a buffer whose ghost ring
// is current, then their decoded values.  Kept apart so that all 13 loads
// are in flight before the first is used.
template <class C, int AUX>
__device__ __forceinline__ void load_raw(__amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                         uint32_t plane_b, uint32_t pitch_b,
                                         typename Raw<sizeof(typename C::T)>::type (&raw)[NPOP]) {
  constexpr int ES = (int)sizeof(typename C::T);
#pragma unroll
  for (int p = 0; p < NPOP; ++p) {
    const uint32_t soff =
        (uint32_t)p * plane_b - (uint32_t)(per(p) * (int)pitch_b) - (uint32_t)(pex(p) * ES);
    raw[p] = buf_load<ES, AUX>(rs, voff, soff);
  }
}

template <class C>
__device__ __forceinline__ void decode_raw(const JetDesc &d,
                                           const typename Raw<sizeof(typename C::T)>::type (&raw)[NPOP],
                                           float (&f)[9], float (&g)[4]) {
  using T = typename C::T;
#pragma unroll
  for (int p = 0; p < NPOP; ++p) {
    const float x = C::dec(__builtin_bit_cast(T, raw[p]), pop_offset<C>(d, p));
    if (p < 9) f[p] = x; else g[p - 9] = x;
  }
}

template <class C, int AUX>
__device__ __forceinline__ void load_pulled(const JetDesc &d, __amdgpu_buffer_rsrc_t rs,
                                            uint32_t voff, uint32_t plane_b, uint32_t pitch_b,
                                            float (&f)[9], float (&g)[4]) {
  typename Raw<sizeof(typename C::T)>::type raw[NPOP];
  load_raw<C, AUX>(rs, voff, plane_b, pitch_b, raw);
  __builtin_amdgcn_sched_barrier(0);
  decode_raw<C>(d, raw, f, g);
}

template <class C, int AUX>
__device__ __forceinline__ void store_node(const JetDesc &d, __amdgpu_buffer_rsrc_t rd,
                                           uint32_t voff, uint32_t plane_b, const float (&f)[9],
                                           const float (&g)[4], uint32_t key) {
  using T = typename C::T;
  constexpr int ES = (int)sizeof(T);
#pragma unroll
  for (int p = 0; p < NPOP; ++p) {
    const T x = C::enc(p < 9 ? f[p] : g[p - 9], pop_offset<C>(d, p), plane_key(key, p));
    buf_store<ES, AUX>(__builtin_bit_cast(typename Raw<ES>::type, x), rd, voff,
                       (uint32_t)p * plane_b);
  }
}

__device__ __forceinline__ bool is_edge(const JetDesc &d, int i, int j) {
  return (i == 0) | (i == d.nx - 1) | (j == 0) | (j == d.nr - 1);
}

// LDS image of the intermediate state of a two-step launch: per plane,
// EH = TY + 2 rows of PAIR_W = 66 columns, position (x, y) holding node
// (ia - 1 + x, ja - 1 + y).  Values are kept in the storage type, encoded as
// a store to memory would encode them, and decoded when step 2 pulls them,
// so the image of 16-bit storage takes half the LDS of FP32's.  put() is the
// epilogue's destination: writes outside the image are dropped.
constexpr int PAIR_W = 66;

// Planes below P0 are not kept (P0 = 1: the rest population stays in the
// registers of the thread that computed it, see pair_kernel).
template <class C>
__device__ __forceinline__ float storage_round(const JetDesc &d, int p, float v, uint32_t k) {
  const float off = pop_offset<C>(d, p);
  return C::dec(C::enc(v, off, k), off);
}

template <class C, int EH, int P0>
struct LdsImage {
  typename C::T *s;
  int ia, ja;
  int wrap;  // nx for periodic x edges (a column nx away is the same column), else 0
  __device__ __forceinline__ void set(const JetDesc &d, int p, int x, int y, float v,
                                     uint32_t k) const {
    if (p >= P0) s[((p - P0) * EH + y) * PAIR_W + x] = C::enc(v, pop_offset<C>(d, p), k);
  }
  __device__ __forceinline__ void put(const JetDesc &d, int p, int i, int j, float v,
                                     uint32_t k) const {
    int x = i - ia + 1;
    const int y = j - ja + 1;
    if (wrap) x += x < 0 ? wrap : (x >= PAIR_W ? -wrap : 0);
    if (((unsigned)x < (unsigned)PAIR_W) & ((unsigned)y < (unsigned)EH)) set(d, p, x, y, v, k);
  }
};

// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking).  A workgroup of 64 x NW threads
// (NW waves, one per block row) owns a tile of 64 x TY nodes.
//  1. Every fluid node of the tile and of a one-node frame around it pulls
//     from the source buffer and collides; the results, and the ghost values
//     that edge nodes among them produce, go to the LDS image.  With an
//     equilibrium side, frame positions on the ghost ring first get the
//     ring's current (constant) values.
//  2. Every node of the tile pulls from the image, collides and stores to
//     the other buffer, followed by the ghost epilogue of the next step.
// Each stored population crosses HBM once per two steps instead of once per
// step; the frame is computed by both tiles that share it.  The intermediate
// values are rounded through the storage codec, so the result is
// bit-identical to two launches of the one-step kernel.
// After a full pair the state sits in the buffer that the one-step rule
// assigns to the odd step count, so each full pair toggles the jet's flip:
// the advance kernel applies it, `tog` accounts for the pairs issued since.
// A jet one step short of its target (or nsteps == 1) takes one step.
// With periodic x edges the frame columns beyond the domain are computed as
// the nodes at its other end, and the epilogue's ghost writes are wrapped into
// the image the same way, so the tile sees what the ghost ring would hold.
// ---------------------------------------------------------------------------
template <class C, int TY, int NW, int W, int CP>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(W, 8))) void pair_kernel(
    const JetDesc *__restrict__ jets, const int32_t *__restrict__ tile_start,
    const BatchHdr *__restrict__ hdr, int32_t koff, int32_t tog, int32_t nsteps,
    int32_t *__restrict__ flags) {
  using T = typename C::T;
  constexpr int ES = (int)sizeof(T);
  constexpr int EH = TY + 2;
  constexpr int AUX_L = (CP & 2) ? CACHE_NT : 0, AUX_S = (CP & 1) ? CACHE_NT : 0;
  constexpr bool PF = !(CP & 4);  // bit 2: no prefetch of the next task's loads
  // bit 3: the rest population f_0 of the tile's nodes stays in registers (the
  // wave that computes image row y in step 1 updates tile row y - 1 in step
  // 2), so the image holds 12 planes
  constexpr int P0 = (CP & 8) ? 1 : 0;
  static_assert(TY % NW == 0 && 2 * EH <= 64, "tile rows");
  __shared__ T img[(NPOP - P0) * EH * PAIR_W];
  const int lane = (int)threadIdx.x, wave = (int)threadIdx.y;
  const int32_t njets = hdr->njets;
  const int32_t ntiles = tile_start[njets];
  const TileWalk tw = tile_walk(ntiles);
  for (int32_t t = tw.first; t < tw.end; t += tw.stride) {
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
    const bool two = (nsteps > 1) & (step + 1 < d.target);
    const int32_t lt = t - tile_start[jid];
    const int32_t ty = lt / d.tiles_x;
    const int32_t tx = lt - ty * d.tiles_x;
    const int ia = tx * 64, ja = ty * TY;
    const int nx = d.nx, nr = d.nr;
    const int64_t sel = step + (d.flip ^ tog);
    T *src_raw = static_cast<T *>(d.buf[sel & 1]);
    T *dst_raw = static_cast<T *>(d.buf[(sel + 1) & 1]);
    const uint32_t pitch_b = (uint32_t)d.pitch * ES, plane_b = (uint32_t)d.plane * ES;
    const uint32_t span = (uint32_t)NPOP * plane_b;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(src_raw, 0, (int)span, BUF_WORD3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(dst_raw, 0, (int)span, BUF_WORD3);
    const bool tile_edge = (ia == 0) | (ia + 64 >= nx) | (ja == 0) | (ja + TY >= nr);
    const bool inlet = d.bc[0] == BC_INLET;
    const float4 *in1 = inlet ? d.inlet + (int64_t)((step + 1) % d.n_t) * nr : d.inlet;
    const float4 *in2 = inlet ? d.inlet + (int64_t)((step + 2) % d.n_t) * nr : d.inlet;
    const Dst<C> out{as_global(dst_raw), d.plane, d.pitch};
    bool ok = true;
    if (!two) {
      for (int r = wave; r < TY; r += NW) {
        const int i = ia + lane, j = ja + r;
        if ((i < nx) & (j < nr)) {
          float f[9], g[4];
          const uint32_t voff = (uint32_t)node_index(d.pitch, i, j) * ES;
          load_pulled<C, AUX_L>(d, rs, voff, plane_b, pitch_b, f, g);
          const float rr = d.r0 + (float)j + 0.5f;
          ok &= collide(d, fast_rcp(rr), rr * rr, f, g);
          const uint32_t key = sr_key(i, j, step + 1);
          store_node<C, AUX_S>(d, rd, voff, plane_b, f, g, key);
          if (is_edge(d, i, j)) ghost_epilogue<C>(d, out, i, j, f, g, in1, key);
        }
      }
    } else {
      // Periodic x edges: the frame columns beyond the domain are the
      // columns at its other end, computed in step 1 like any other node
      // (their values, and the ghost values their epilogue writes, are those
      // of the same nodes at the other end, so duplicates agree).
      const bool px = d.bc[0] == BC_PERIODIC;
      // (frame columns lie in -1 .. ia + 64; more than one turn only when nx < 65)
      const auto wrap_i = [&](int i) {
        return i < 0 ? i + nx : (i < nx ? i : (i - nx < nx ? i - nx : i % nx));
      };
      const LdsImage<C, EH, P0> im{img, ia, ja, px ? nx : 0};
      // Constant ghosts (equilibrium sides) are never rewritten by the
      // epilogue: copy the ring positions of the image from the source
      // buffer first.  Every other ghost value the tile pulls is produced in
      // step 1 by an edge node of the image.
      const bool eq_side = (d.bc[0] == BC_EQ) | (d.bc[1] == BC_EQ) | (d.bc[2] == BC_EQ) |
                           (d.bc[3] == BC_EQ);
      if (tile_edge & eq_side) {
        const Src<C> src{as_global(static_cast<const T *>(src_raw)), d.plane, d.pitch};
        for (int n = lane + 64 * wave; n < EH * PAIR_W; n += 64 * NW) {
          const int y = n / PAIR_W, x = n - y * PAIR_W;
          const int j = ja - 1 + y;
          // with periodic x only the rows j = -1, nr are ring (any column, wrapped)
          const int i = px ? wrap_i(ia - 1 + x) : ia - 1 + x;
          const bool ring = (i >= -1) & (i <= nx) & (j >= -1) & (j <= nr) &
                            ((!px & ((i == -1) | (i == nx))) | (j == -1) | (j == nr));
          if (ring) {
            T v[NPOP];
#pragma unroll
            for (int p = P0; p < NPOP; ++p)
              v[p] = src.base[(int64_t)p * src.plane + node_index(src.pitch, i, j)];
#pragma unroll
            for (int p = P0; p < NPOP; ++p) img[((p - P0) * EH + y) * PAIR_W + x] = v[p];
          }
        }
      }
      // step 1: rows 0..EH-1 of the image (columns 1..64), then the two side
      // columns (0 and 65) as one task of 2 EH lanes: EH + 1 tasks, task q
      // done by wave q % NW in round q / NW.  Software pipelined over the
      // (unrolled) rounds: a wave issues the loads of its next task right
      // after the property gather of this one.  Positions are clamped into
      // the domain so that every lane loads valid data; lanes off the fluid
      // skip the writes.  Every round but the last is valid for every wave.
      using R = typename Raw<ES>::type;
      constexpr int NROUND = (EH + NW) / NW;
      R raw[2][NPOP];
      float keep0[NROUND];  // f_0 of image rows 1..TY, by round (P0 == 1)
      const auto task_xy = [&](int q, int &x, int &y) {
        x = q < EH ? lane + 1 : ((lane & 1) ? PAIR_W - 1 : 0);
        y = q < EH ? q : lane >> 1;
      };
      // idle lanes of the side task load a row of the image (no new lines)
      const auto task_voff = [&](int q) {
        int x, y;
        task_xy(q, x, y);
        const int i = px ? wrap_i(ia - 1 + x) : min(max(ia - 1 + x, 0), nx - 1);
        const int j = min(max(ja - 1 + min(y, EH - 1), 0), nr - 1);
        return (uint32_t)node_index(d.pitch, i, j) * ES;
      };
      load_raw<C, AUX_L>(rs, task_voff(wave), plane_b, pitch_b, raw[0]);
      if (tile_edge & eq_side) __syncthreads();  // ring copy in LDS
#pragma unroll
      for (int k = 0; k < NROUND; ++k) {
        const int q = wave + NW * k;
        if (k + 1 < NROUND || q <= EH) {
          if (!PF && k > 0) {
            load_raw<C, AUX_L>(rs, task_voff(q), plane_b, pitch_b, raw[k & 1]);
            __builtin_amdgcn_sched_barrier(0);
          }
          const auto prefetch = [&] {
            if (k + 1 < NROUND)
              load_raw<C, AUX_L>(rs, task_voff(min(q + NW, EH)), plane_b, pitch_b,
                                 raw[(k + 1) & 1]);
          };
          int x, y;
          task_xy(q, x, y);
          const int i = px ? wrap_i(ia - 1 + x) : ia - 1 + x, j = ja - 1 + y;
          float f[9], g[4];
          decode_raw<C>(d, raw[k & 1], f, g);
          const float rr = d.r0 + (float)min(max(j, 0), nr - 1) + 0.5f;
          bool okn;
          if constexpr (PF) okn = collide(d, fast_rcp(rr), rr * rr, f, g, prefetch);
          else okn = collide(d, fast_rcp(rr), rr * rr, f, g);
          const uint32_t key = sr_key(i, j, step + 1);
          if ((y < EH) & (i >= 0) & (i < nx) & (j >= 0) & (j < nr)) {
            ok &= okn;
#pragma unroll
            for (int p = 0; p < NPOP; ++p)
              im.set(d, p, x, y, p < 9 ? f[p] : g[p - 9], plane_key(key, p));
            if (is_edge(d, i, j)) ghost_epilogue<C>(d, im, i, j, f, g, in1, key);
          }
          if (P0 == 1) keep0[k] = storage_round<C>(d, 0, f[0], plane_key(key, 0));
        }
      }
      __syncthreads();
      // step 2: the tile, from the image
      const auto out_row = [&](int r, float f0) {
        const int i = ia + lane, j = ja + r;
        if ((i < nx) & (j < nr)) {
          float f[9], g[4];
          f[0] = f0;
#pragma unroll
          for (int p = P0; p < NPOP; ++p) {
            const float v = C::dec(
                img[((p - P0) * EH + r + 1 - per(p)) * PAIR_W + lane + 1 - pex(p)],
                pop_offset<C>(d, p));
            if (p < 9) f[p] = v; else g[p - 9] = v;
          }
          const float rr = d.r0 + (float)j + 0.5f;
          ok &= collide(d, fast_rcp(rr), rr * rr, f, g);
          const uint32_t voff = (uint32_t)node_index(d.pitch, i, j) * ES;
          const uint32_t key = sr_key(i, j, step + 2);
          store_node<C, AUX_S>(d, rd, voff, plane_b, f, g, key);
          if (tile_edge && is_edge(d, i, j)) ghost_epilogue<C>(d, out, i, j, f, g, in2, key);
        }
      };
      if constexpr (P0 == 1) {
#pragma unroll
        for (int k = 0; k < NROUND; ++k) {
          const int y = wave + NW * k;  // image row of step 1 -> tile row y - 1
          if ((y >= 1) & (y <= TY)) out_row(y - 1, keep0[k]);
        }
      } else {
        for (int r = wave; r < TY; r += NW) out_row(r, 0.0f);
      }
    }
    __syncthreads();  // the image is reused by the next tile
    if (!ok) flags[d.slot] = 1;
  }
}

// ---------------------------------------------------------------------------
// Single-buffer (AA) step over the same 64 x 4 tiles as the one-step kernel's
// default shape, one node per lane.  After an even number of steps the buffer
// is in the swapped layout: a node pulls from its neighbours (plane opp(p) at
// x - e_p), collides and pushes f*_p into plane p at x + e_p, leaving the
// natural layout.  After an odd number it reads its own 13 values, collides
// and writes f*_p into plane opp(p) of its own node, leaving the swapped
// layout.  Edge nodes then write what the next step pulls from outside the
// domain.  Each location is read and written by a single thread in a step,
// so the update is in place; the per-node arithmetic is the one-step
// kernel's, so the results are bit-identical to the two-buffer scheme.
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(256) void aa_kernel(
    const JetDesc *__restrict__ jets, const int32_t *__restrict__ tile_start,
    const BatchHdr *__restrict__ hdr, int32_t koff, int32_t tog, int32_t nsteps,
    int32_t *__restrict__ flags) {
  using T = typename C::T;
  constexpr int ES = (int)sizeof(T);
  const int lane = (int)threadIdx.x, wave = (int)threadIdx.y;
  const int32_t njets = hdr->njets;
  const int32_t ntiles = tile_start[njets];
  const TileWalk tw = tile_walk(ntiles);
  for (int32_t t = tw.first; t < tw.end; t += tw.stride) {
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
    const int i = tx * 64 + lane, j = ty * 4 + wave;
    if ((i < d.nx) & (j < d.nr)) {
      T *raw = static_cast<T *>(d.buf[0]);
      const uint32_t pitch_b = (uint32_t)d.pitch * ES, plane_b = (uint32_t)d.plane * ES;
      const __amdgpu_buffer_rsrc_t r =
          __builtin_amdgcn_make_buffer_rsrc(raw, 0, (int)((uint32_t)NPOP * plane_b), BUF_WORD3);
      const uint32_t voff = (uint32_t)node_index(d.pitch, i, j) * ES;
      const bool swapped = (step & 1) == 0;
      typename Raw<ES>::type w[NPOP];
      if (swapped) {
#pragma unroll
        for (int p = 0; p < NPOP; ++p)
          w[p] = buf_load<ES, 0>(r, voff,
                                 (uint32_t)opp_plane(p) * plane_b -
                                     (uint32_t)(per(p) * (int)pitch_b) -
                                     (uint32_t)(pex(p) * ES));
      } else {
#pragma unroll
        for (int p = 0; p < NPOP; ++p) w[p] = buf_load<ES, 0>(r, voff, (uint32_t)p * plane_b);
      }
      float f[9], g[4];
      decode_raw<C>(d, w, f, g);
      const float rr = d.r0 + (float)j + 0.5f;
      const bool ok = collide(d, fast_rcp(rr), rr * rr, f, g);
      const uint32_t key = sr_key(i, j, step + 1);
#pragma unroll
      for (int p = 0; p < NPOP; ++p) {
        const T x = C::enc(p < 9 ? f[p] : g[p - 9], pop_offset<C>(d, p), plane_key(key, p));
        const uint32_t soff =
            swapped ? (uint32_t)p * plane_b + (uint32_t)(per(p) * (int)pitch_b) +
                          (uint32_t)(pex(p) * ES)
                    : (uint32_t)opp_plane(p) * plane_b;
        buf_store<ES, 0>(__builtin_bit_cast(typename Raw<ES>::type, x), r, voff, soff);
      }
      if (is_edge(d, i, j)) {
        const float4 *in1 = d.bc[0] == BC_INLET
                                ? d.inlet + (int64_t)((step + 1) % d.n_t) * d.nr
                                : d.inlet;
        const State<C> o{as_global(raw), d.plane, d.pitch, swapped ? 2 : 1};
        aa_epilogue<C>(d, o, i, j, f, g, in1, key);
      }
      if (!ok) flags[d.slot] = 1;
    }
  }
}

// Ghost values of the state after `step` steps (seen through `view`) from its
// interior and the inlet row of `step`, by the pull-side edge rules: every
// ghost slot (ghost node, link p) whose puller (ghost + e_p) is a fluid node
// gets the value that node pulls.  Run after any change of the interior or
// of the inlet made outside the step.  The rounding key is the ghost
// position's at step 0, whatever the step: the constant ghosts of
// equilibrium sides then hold the same bits in both buffers, which the
// single-buffer kernel rewrites with the same key every step.
// One thread per ghost node: row -1 and row nr (nx + 2 each, corners
// included), then columns -1 and nx (nr each).
template <class C>
__global__ void ghost_fill_kernel(const JetDesc *__restrict__ dp, int64_t step, int32_t view) {
  const JetDesc &d = *dp;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = d.nx, nr = d.nr;
  int gi, gj;
  if (q < nx + 2) { gi = q - 1; gj = -1; }
  else if (q < 2 * (nx + 2)) { gi = q - (nx + 2) - 1; gj = nr; }
  else if (q < 2 * (nx + 2) + nr) { gi = -1; gj = q - 2 * (nx + 2); }
  else if (q < 2 * (nx + 2) + 2 * nr) { gi = nx; gj = q - 2 * (nx + 2) - nr; }
  else return;
  const State<C> st = state_view<C>(d, view);
  const float4 *inrow = d.inlet + (int64_t)(step % d.n_t) * d.nr;
#pragma unroll
  for (int p = 1; p < NPOP; ++p) {
    const int pi = gi + pex(p), pj = gj + per(p);
    if (pi >= 0 && pi < nx && pj >= 0 && pj < nr)
      st.put(d, p, gi, gj, pull_edge<C>(d, st, p, pi, pj, inrow),
             plane_key(sr_key(gi, gj, 0), p));
  }
}

// Moves every jet's step0 by delta (clamped at the target); ends a captured
// group of steps so that the same graph serves the next group.  The group
// began with npair two-step launches: each that a jet took in full (both
// steps before its target) swapped the roles of its buffers.
__global__ void advance_kernel(JetDesc *__restrict__ jets, const BatchHdr *__restrict__ hdr,
                               int32_t delta, int32_t npair) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < hdr->njets) {
    const int64_t s0 = jets[q].step0, tg = jets[q].target;
    if (npair > 0 && tg - s0 >= 2) {
      const int64_t full = (tg - s0) / 2 < npair ? (tg - s0) / 2 : npair;
      jets[q].flip ^= (int32_t)(full & 1);
    }
    const int64_t s = s0 + delta;
    jets[q].step0 = s < tg ? s : tg;
  }
}

// Equilibrium fill of the state (through `view`) from fields (float4 rho, ux,
// ur, T per node, i fastest) or, with state == nullptr, from the uniform u0.
template <class C>
__global__ void init_kernel(const JetDesc *__restrict__ dp, int64_t step, int32_t view,
                            const float4 *__restrict__ state, float4 u0) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= d.nx) return;
  const float4 q = state ? state[(int64_t)j * d.nx + i] : u0;
  const State<C> st = state_view<C>(d, view);
  const uint32_t key = sr_key(i, j, step);
#pragma unroll
  for (int p = 0; p < NPOP; ++p)
    st.put(d, p, i, j, eq_plane(p, q.x, q.y, q.z, q.w), plane_key(key, p));
}

// Pre-collision moments (eq. 2) of the state after `step` steps:
// float4 (rho, ux, ur, T) per node, i fastest.
template <class C>
__global__ void moments_kernel(const JetDesc *__restrict__ dp, int64_t step, int32_t view,
                               float4 *__restrict__ out) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= d.nx) return;
  const State<C> s = state_view<C>(d, view);
  float f[9], g[4];
  pulled_node<C>(d, s, i, j, f, g);
  const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const float mx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const float mr = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const float T = (g[0] + g[1]) + (g[2] + g[3]);
  out[(int64_t)j * d.nx + i] = make_float4(rho, mx / rho, mr / rho, T);
}

// Centreline (j = 0) and exit column (i = nx-1): (ux, T) pairs, nx + nr.
template <class C>
__global__ void profiles_kernel(const JetDesc *__restrict__ dp, int64_t step, int32_t view,
                                float2 *__restrict__ out) {
  const JetDesc &d = *dp;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.nx + d.nr) return;
  const int i = t < d.nx ? t : d.nx - 1;
  const int j = t < d.nx ? 0 : t - d.nx;
  const State<C> s = state_view<C>(d, view);
  float f[9], g[4];
  pulled_node<C>(d, s, i, j, f, g);
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
    const JetDesc *__restrict__ dp, int64_t step, int32_t view, RedPartial *__restrict__ partial) {
  const JetDesc &d = *dp;
  const State<C> s = state_view<C>(d, view);
  const int64_t nodes = (int64_t)d.nx * d.nr;
  double m = 0.0, e = 0.0, bad = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; n < nodes;
       n += (int64_t)gridDim.x * RED_THREADS) {
    const int j = (int)(n / d.nx), i = (int)(n - (int64_t)j * d.nx);
    float f[9], g[4];
    pulled_node<C>(d, s, i, j, f, g);
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
__global__ void decode_kernel(const JetDesc *__restrict__ dp, int64_t step, int32_t view,
                              float *__restrict__ out) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, p = blockIdx.z;
  if (i >= d.nx) return;
  out[((int64_t)p * d.nr + j) * d.nx + i] = state_view<C>(d, view).load(d, p, i, j);
}

template <class C>
__global__ void encode_kernel(const JetDesc *__restrict__ dp, int64_t step, int32_t view,
                              const float *__restrict__ in) {
  const JetDesc &d = *dp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, p = blockIdx.z;
  if (i >= d.nx) return;
  state_view<C>(d, view).put(d, p, i, j, in[((int64_t)p * d.nr + j) * d.nx + i],
                            plane_key(sr_key(i, j, step), p));
}

// Plain streaming copy, 16 B per lane per iteration.
__global__ __launch_bounds__(256) void copy_kernel(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    dst[q] = src[q];
}

}  // namespace lbmx
