// lbm_device.hpp -- device side of the gfx950 axisymmetric D2Q9 + D2Q4
// LBGK-LES step: lattice constants, 16-bit storage codecs, the FP32 node
// collision and the pull (streaming) with the edge rules.
//
// Method: Djebali, Calve, Pateyron, El Ganaoui, Sammouda, sections 2.1-2.4,
// eqs. (1)-(7).  The source terms F1, F2 and S are the forms derived from the
// axisymmetric equations, stated in include/lbm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

// ---------------------------------------------------------------------------
// Lattices.  D2Q9 links k = 0..8 as (e_x, e_r):
//   0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1) 7 (-1,-1) 8 (1,-1)
// D2Q4 links (the paper's k = 1..4) stored as 0..3: +x, +r, -x, -r.
// Storage planes: 0..8 hold f_k, 9..12 hold g_0..g_3.
// ---------------------------------------------------------------------------
constexpr int NPOP = 13;

__host__ __device__ constexpr int ex9(int k) {
  return (k == 1 || k == 5 || k == 8) ? 1 : (k == 3 || k == 6 || k == 7) ? -1 : 0;
}
__host__ __device__ constexpr int er9(int k) {
  return (k == 2 || k == 5 || k == 6) ? 1 : (k == 4 || k == 7 || k == 8) ? -1 : 0;
}
__host__ __device__ constexpr float w9(int k) {
  return k == 0 ? 4.0f / 9.0f : (k <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr int opp9(int k) {
  return k == 0 ? 0 : (k <= 4 ? ((k + 1) & 3) + 1 : ((k - 3) & 3) + 5);
}
__host__ __device__ constexpr int mir9(int k) {  // e_r -> -e_r
  return k == 2 ? 4 : k == 4 ? 2 : k == 5 ? 8 : k == 8 ? 5 : k == 6 ? 7 : k == 7 ? 6 : k;
}
__host__ __device__ constexpr int ex4(int k) { return k == 0 ? 1 : k == 2 ? -1 : 0; }
__host__ __device__ constexpr int er4(int k) { return k == 1 ? 1 : k == 3 ? -1 : 0; }
__host__ __device__ constexpr int opp4(int k) { return (k + 2) & 3; }
__host__ __device__ constexpr int mir4(int k) { return k == 1 ? 3 : k == 3 ? 1 : k; }

// plane p -> (e_x, e_r)
__host__ __device__ constexpr int pex(int p) { return p < 9 ? ex9(p) : ex4(p - 9); }
__host__ __device__ constexpr int per(int p) { return p < 9 ? er9(p) : er4(p - 9); }

enum : int32_t { BC_INLET = 0, BC_OUTFLOW = 1, BC_PERIODIC = 2, BC_AXIS = 3,
                 BC_FREESLIP = 4, BC_WALL = 5, BC_EQ = 6 };

// ---------------------------------------------------------------------------
// Per-jet descriptor, read by every kernel through a device pointer.
// ---------------------------------------------------------------------------
struct alignas(16) JetDesc {
  void *buf[2];            // population buffers; state after s steps in buf[s & 1]
  const float4 *table;     // (M_nu, dM_nu, M_alpha, dM_alpha) at each grid point
  const float4 *inlet;     // n_t rows of nr (ux, ur, T, 0)
  int64_t plane;           // elements per population plane (pitch * nr)
  int64_t step0;           // step count of the launch with koff = 0
  int64_t target;          // the jet stops at this step count
  int32_t nx, nr, pitch, tiles_x;
  int32_t n_t, table_n, hoop, slot;
  int32_t bc[4];
  float r0, nu0, alpha0, c18;      // c18 = 18 (C_s Delta)^2
  float inv_prt, G, t_lo, t_scale; // t_scale = (table_n - 1) / (t_hi - t_lo)
  float rho_ref, g4_ref, pad0, pad1;
  float wallT[4];                  // NaN: adiabatic
  float eq[4][4];                  // EQ side: rho, ux, ur, T
};

// Batch header in device memory: number of jets in the tile list.  The tile
// list itself is tile_start[0..njets] (prefix sums of the jets' tile counts).
struct BatchHdr {
  int32_t njets;
  int32_t pad[3];
};

// Partial sums of the FP64 conservation reduction.
constexpr int RED_THREADS = 256;

struct RedPartial {
  double mass, energy;
  double bad, pad;
};

// ---------------------------------------------------------------------------
// Storage codecs.  FP32 stores populations as they are; the 16-bit codecs
// store the deviation from a reference (w_k rho_ref for f, g_ref/4 for g)
// rounded to nearest even, and decode to FP32.
// ---------------------------------------------------------------------------
struct CodecF32 {
  using T = float;
  static constexpr bool dev = false;
  __device__ static __forceinline__ float dec(T v, float) { return v; }
  __device__ static __forceinline__ T enc(float v, float) { return v; }
};
struct CodecF16 {
  using T = _Float16;
  static constexpr bool dev = true;
  __device__ static __forceinline__ float dec(T v, float off) { return (float)v + off; }
  __device__ static __forceinline__ T enc(float v, float off) { return (T)(v - off); }
};
struct CodecBF16 {
  using T = __bf16;
  static constexpr bool dev = true;
  __device__ static __forceinline__ float dec(T v, float off) { return (float)v + off; }
  __device__ static __forceinline__ T enc(float v, float off) { return (T)(v - off); }
};

template <class C>
__device__ __forceinline__ float pop_offset(const JetDesc &d, int p) {
  if constexpr (!C::dev) return 0.0f;
  else return p < 9 ? w9(p) * d.rho_ref : d.g4_ref;
}

// ---------------------------------------------------------------------------
// Equilibria (moments fixed by eq. 2): second-order D2Q9, c_s^2 = 1/3;
// first-order D2Q4, c_s^2 = 1/2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float feq_link(int k, float rho, float ux, float ur) {
  const float eu = (float)ex9(k) * ux + (float)er9(k) * ur;
  const float uu = ux * ux + ur * ur;
  return w9(k) * rho * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
}
__device__ __forceinline__ float geq_link(int k, float T, float ux, float ur) {
  const float eu = (float)ex4(k) * ux + (float)er4(k) * ur;
  return 0.25f * T * (1.0f + 2.0f * eu);
}
// equilibrium of storage plane p
__device__ __forceinline__ float eq_plane(int p, float rho, float ux, float ur, float T) {
  return p < 9 ? feq_link(p, rho, ux, ur) : geq_link(p - 9, T, ux, ur);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------------------
// One node: eq. (2) moments, eq. (6) properties, eq. (4) tau_tot, eq. (5)
// alpha_tot, the axisymmetric sources, eq. (1) collision.  f and g hold the
// pulled (pre-collision) populations on entry and f*, g* on exit.  Returns
// false if rho <= 0 or rho, T are not finite.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool collide(const JetDesc &d, float rinv, float r2,
                                        float (&f)[9], float (&g)[4]) {
  // eq. (2)
  const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const float mx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const float mr = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const float T = (g[0] + g[1]) + (g[2] + g[3]);
  const float irho = fast_rcp(rho);
  const float ux = mx * irho, ur = mr * irho;

  // non-equilibrium parts
  float fn[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) fn[k] = f[k] - feq_link(k, rho, ux, ur);
  float gn[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) gn[k] = g[k] - geq_link(k, T, ux, ur);

  // eq. (6): multiplier tables, linear on a uniform grid, clamped
  float x = fmaxf((T - d.t_lo) * d.t_scale, 0.0f);  // NaN -> 0
  x = fminf(x, (float)(d.table_n - 1));
  const int i0 = max(min((int)x, d.table_n - 2), 0);
  const float w = x - (float)i0;
  const float4 te = d.table[i0];
  const float nu = d.nu0 * (te.x + w * te.y);
  const float alpha = d.alpha0 * (te.z + w * te.w);
  const float tau_nu = 0.5f + 3.0f * nu;

  // eq. (4): Q_ij and the local relaxation time
  const float qxx = (fn[1] + fn[3]) + ((fn[5] + fn[6]) + (fn[7] + fn[8]));
  const float qrr = (fn[2] + fn[4]) + ((fn[5] + fn[6]) + (fn[7] + fn[8]));
  const float qxr = (fn[5] + fn[7]) - (fn[6] + fn[8]);
  const float qn = fast_sqrt(2.0f * (qxx * qxx + 2.0f * qxr * qxr + qrr * qrr));
  const float tau = 0.5f * (tau_nu + fast_sqrt(tau_nu * tau_nu + d.c18 * qn * irho));
  // eqs. (3), (5)
  const float nu_tot = (tau - 0.5f) * (1.0f / 3.0f);
  const float alpha_tot = alpha + (nu_tot - nu) * d.inv_prt;
  const float tau_a = 0.5f + 2.0f * alpha_tot;
  const float itau = fast_rcp(tau), itau_a = fast_rcp(tau_a);

  // axisymmetric sources
  const float kv = 1.0f - 0.5f * itau;
  const float ka = 1.0f - 0.5f * itau_a;
  const float theta = -rho * ur * rinv;
  const float hden = d.hoop ? fast_rcp(r2 + 2.0f * nu_tot) : rinv * rinv;
  const float Fx = (-rho * ux * ur - kv * qxr) * rinv + rho * d.G;
  const float Fr = (-rho * ur * ur - kv * qrr) * rinv - 2.0f * rho * nu_tot * ur * hden;
  const float S = (-T * ur - ka * (gn[1] - gn[3])) * rinv;

  // eq. (1)
  const float fx6 = Fx * (1.0f / 6.0f), fr6 = Fr * (1.0f / 6.0f);
#pragma unroll
  for (int k = 0; k < 9; ++k)
    f[k] = f[k] - fn[k] * itau + w9(k) * theta + (float)ex9(k) * fx6 + (float)er9(k) * fr6;
  const float s4 = 0.25f * S;
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = g[k] - gn[k] * itau_a + s4;

  return (rho > 0.0f) && (rho < __builtin_inff()) && (fabsf(T) < __builtin_inff());
}

// ---------------------------------------------------------------------------
// Pull.  load(p, i, j) reads plane p of the source buffer at node (i, j).
// ---------------------------------------------------------------------------
template <class C>
struct Src {
  const typename C::T *__restrict__ base;
  int64_t plane;
  int32_t pitch;
  __device__ __forceinline__ float load(const JetDesc &d, int p, int i, int j) const {
    return C::dec(base[(int64_t)p * plane + (int64_t)j * pitch + i], pop_offset<C>(d, p));
  }
};

// x-side rule for plane p taken from column ip of row jr; i_land is the
// column of the receiving node.
template <class C>
__device__ __forceinline__ float pull_x(const JetDesc &d, const Src<C> &s, int p, int ip,
                                        int jr, int i_land, const float4 *inrow) {
  if (ip >= 0 && ip < d.nx) return s.load(d, p, ip, jr);
  const int side = ip < 0 ? 0 : 1;
  switch (d.bc[side]) {
    case BC_PERIODIC:
      return s.load(d, p, ip < 0 ? ip + d.nx : ip - d.nx, jr);
    case BC_OUTFLOW:
      return s.load(d, p, d.nx - 1, jr);
    case BC_INLET: {
      const float4 q = inrow[jr];
      return eq_plane(p, 1.0f, q.x, q.y, q.z);
    }
    case BC_WALL: {
      const int po = p < 9 ? opp9(p) : 9 + opp4(p - 9);
      float v = s.load(d, po, i_land, jr);
      const float tw = d.wallT[side];
      if (p >= 9 && tw == tw) v = -v + 0.5f * tw;
      return v;
    }
    default: {  // BC_EQ
      const float *e = d.eq[side];
      return eq_plane(p, e[0], e[1], e[2], e[3]);
    }
  }
}

// Value pulled by node (i, j) along plane p when the source node lies outside
// the domain (or may): r-side rule first, then the x-side rule.
template <class C>
__device__ __forceinline__ float pull_edge(const JetDesc &d, const Src<C> &s, int p, int i,
                                           int j, const float4 *inrow) {
  const int ip = i - pex(p), jp = j - per(p);
  if (jp >= 0 && jp < d.nr) return pull_x<C>(d, s, p, ip, jp, i, inrow);
  const int side = jp < 0 ? 2 : 3;
  const int bc = d.bc[side];
  if (bc == BC_AXIS || bc == BC_FREESLIP) {
    const int pm = p < 9 ? mir9(p) : 9 + mir4(p - 9);
    return pull_x<C>(d, s, pm, ip, jp < 0 ? 0 : d.nr - 1, i, inrow);
  }
  if (bc == BC_WALL) {
    const int po = p < 9 ? opp9(p) : 9 + opp4(p - 9);
    float v = s.load(d, po, i, j);
    const float tw = d.wallT[side];
    if (p >= 9 && tw == tw) v = -v + 0.5f * tw;
    return v;
  }
  const float *e = d.eq[side];
  return eq_plane(p, e[0], e[1], e[2], e[3]);
}

// All 13 pulled values of node (i, j); interior nodes take direct loads.
template <class C>
__device__ __forceinline__ void pull_node(const JetDesc &d, const Src<C> &s, int i, int j,
                                          const float4 *inrow, float (&f)[9], float (&g)[4]) {
  const bool interior = (i >= 1) & (i <= d.nx - 2) & (j >= 1) & (j <= d.nr - 2);
  if (interior) {
    const typename C::T *b = s.base + (int64_t)j * s.pitch + i;
#pragma unroll
    for (int p = 0; p < NPOP; ++p) {
      const float v = C::dec(b[(int64_t)p * s.plane - (int64_t)per(p) * s.pitch - pex(p)],
                             pop_offset<C>(d, p));
      if (p < 9) f[p] = v; else g[p - 9] = v;
    }
  } else {
#pragma unroll
    for (int p = 0; p < NPOP; ++p) {
      const float v = pull_edge<C>(d, s, p, i, j, inrow);
      if (p < 9) f[p] = v; else g[p - 9] = v;
    }
  }
}

}  // namespace lbmx
