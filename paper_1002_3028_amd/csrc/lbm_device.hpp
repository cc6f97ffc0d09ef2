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

// Storage layout of one population plane: (nr + 2) rows of `pitch` elements.
// Node (i, j), i = -1..nx, j = -1..nr, sits at (j + 1) * pitch + XOFF + i:
// row -1, row nr, column -1 and column nx form the ghost ring that holds the
// values the edge nodes pull at the next step.  XOFF keeps interior rows
// aligned; the row end leaves room for vector reads past column nx.
constexpr int32_t XOFF = 64;
__host__ __device__ inline int32_t layout_pitch(int32_t nx) {
  return (XOFF + nx + 1 + 8 + 63) / 64 * 64;
}
__host__ __device__ inline int64_t layout_plane(int32_t nx, int32_t nr) {
  return (int64_t)layout_pitch(nx) * (nr + 2);
}
__host__ __device__ inline int64_t node_index(int32_t pitch, int i, int j) {
  return (int64_t)(j + 1) * pitch + XOFF + i;
}

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

// Pointers into device memory that the compiler must treat as global (not
// flat) address space: the buffers are reached through the descriptor, so
// their address space cannot be inferred.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T *p) {
  return (gptr<T>)p;
}
template <class T>
__device__ __forceinline__ gptr<const T> as_global(const T *p) {
  return (gptr<const T>)p;
}

// ---------------------------------------------------------------------------
// Per-jet descriptor, read by every kernel through a device pointer.
// ---------------------------------------------------------------------------
struct alignas(16) JetDesc {
  void *buf[2];            // population buffers; state after s steps in buf[(s + flip) & 1]
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
  float rho_ref, g4_ref;
  int32_t flip;                    // toggled by every launch that advances two steps
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
// store the deviation from a reference (w_k rho_ref for f, g_ref/4 for g).
// dec(stored, off) -> population; enc(population, off, key) -> stored.
// `key` is the population's rounding key (sr_key, plane_key); only
// stochastic rounding uses it.
// ---------------------------------------------------------------------------
// The 16-bit codecs convert and add on decode, subtract and convert on
// encode.  The deviation f - offset is exact in FP32 whenever f lies within
// a factor two of the offset (Sterbenz), as the populations of these flows
// do, so the conversion to binary16 (to nearest even) is its only rounding.
// The mixed-precision FMA would do each in one instruction and round the
// exact deviation once in every case, but it measured 5 % slower per step.
struct CodecF32 {
  using T = float;
  static constexpr bool dev = false;
  __device__ static __forceinline__ float dec(T v, float) { return v; }
  __device__ static __forceinline__ T enc(float v, float, uint32_t) { return v; }
};
struct CodecF16 {
  using T = _Float16;
  static constexpr bool dev = true;
  __device__ static __forceinline__ float dec(T v, float off) { return (float)v + off; }
  __device__ static __forceinline__ T enc(float v, float off, uint32_t) { return (T)(v - off); }
};
// Rounding keys of stochastic rounding.  sr_key hashes a node's position
// and the step of the state being written (the lowbias32 mixer of C.
// Wellons' hash-prospector over (j << 16 | i) xor step * 2^32/phi; nx, nr
// < 2^16); plane_key gives each population its own rotation of it.  Every
// kernel that writes a population of node (i, j) for the state of step s
// uses plane_key(sr_key(i, j, s), k), k the population's index (a ghost copy
// of population k takes k's key, so that it equals the stored value), so the
// two-step, single-buffer and batched paths round exactly as the one-step
// kernel does.  Ghost values not produced by a step (the ghost fill, and the
// constant ghosts of equilibrium sides) take the ghost position's key at
// step 0.
__device__ __forceinline__ uint32_t sr_key(int i, int j, int64_t step) {
  uint32_t x = ((uint32_t)j << 16) | ((uint32_t)i & 0xffffu);
  x ^= (uint32_t)step * 0x9e3779b9u;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ uint32_t plane_key(uint32_t key, int p) {
  return __builtin_amdgcn_alignbit(key, key, (uint32_t)(7 * p) & 31u);
}

// binary16 deviations with stochastic rounding, by gfx950's conversion for
// it (v_cvt_sr_f16_f32): the magnitude of the deviation rounds toward zero
// after adding r / 2^13 of the binary16 spacing at that magnitude, r the top
// 13 bits of the second operand, for normal and subnormal binary16 results
// alike (and the sign is kept).  The operand is the value's bits xor its
// rounding key, so over keys drawn uniformly r is uniform whatever the value
// and the value rounds up with the probability of its discarded fraction (to
// 2^-13); values binary16 holds are stored unchanged.  The key changes with
// the node and the step, so a value that recurs at one node rounds
// independently at every step and the systematic error that rounding to
// nearest leaves in nearly steady regions averages out.  Populations of one
// node with equal top bits share the key's bits in part (rotations of one
// 32-bit key): their roundings are correlated but each is unbiased.  All
// thirteen planes are rounded this way (the flow populations need it too:
// rounded to nearest they shift the mean flow of a long run).  Decoding is
// binary16's.
struct CodecF16SR {
  using T = _Float16;
  static constexpr bool dev = true;
  __device__ static __forceinline__ float dec(T v, float off) { return (float)v + off; }
  __device__ static __forceinline__ T enc(float v, float off, uint32_t key) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const float x = v - off;
    const uint32_t r = __builtin_bit_cast(uint32_t, x) ^ key;
    return __builtin_amdgcn_cvt_sr_f16_f32(half2_t{0, 0}, x, r, false)[0];
  }
};
struct CodecBF16 {
  using T = __bf16;
  static constexpr bool dev = true;
  __device__ static __forceinline__ float dec(T v, float off) { return (float)v + off; }
  __device__ static __forceinline__ T enc(float v, float off, uint32_t) { return (T)(v - off); }
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
// e . v for lattice components in {-1, 0, 1}: operands are selected, not
// multiplied, so that zero components add no instruction once k is known.
__device__ __forceinline__ float proj(int ex, int er, float vx, float vr) {
  if (ex == 0 && er == 0) return 0.0f;
  if (ex == 0) return er > 0 ? vr : -vr;
  if (er == 0) return ex > 0 ? vx : -vx;
  return (ex > 0 ? vx : -vx) + (er > 0 ? vr : -vr);
}

// Written as w rho (b + eu (3 + 4.5 eu)), b = 1 - 1.5 u.u shared by all
// links: three instructions per link (plus the sum for a diagonal).
__device__ __forceinline__ float feq_link(int k, float rho, float ux, float ur) {
  const float base = 1.0f - 1.5f * (ux * ux + ur * ur);
  if (k == 0) return w9(0) * rho * base;
  const float eu = proj(ex9(k), er9(k), ux, ur);
  return (w9(k) * rho) * __builtin_fmaf(eu, __builtin_fmaf(4.5f, eu, 3.0f), base);
}
__device__ __forceinline__ float geq_link(int k, float T, float ux, float ur) {
  const float eu = proj(ex4(k), er4(k), ux, ur);
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
// A hook, if given, is issued right after the property-table gather and
// nothing is moved across it: a caller can put loads for later work there,
// behind the gather in the memory counter's order.
// ---------------------------------------------------------------------------
struct NoHook {
  __device__ void operator()() const {}
};

template <class H = NoHook>
__device__ __forceinline__ bool collide(const JetDesc &d, float rinv, float r2,
                                        float (&f)[9], float (&g)[4], const H &hook = H()) {
  // eq. (2)
  // (partial sums shared between rho, m and Q)
  const float s13 = f[1] + f[3], s24 = f[2] + f[4];
  const float s58 = f[5] + f[8], s67 = f[6] + f[7];
  const float sd = s58 + s67;  // the four diagonal links
  const float rho = ((f[0] + s13) + s24) + sd;
  const float mx = (f[1] - f[3]) + (s58 - s67);
  const float mr = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
  const float T = (g[0] + g[1]) + (g[2] + g[3]);
  const float irho = fast_rcp(rho);
  const float ux = mx * irho, ur = mr * irho;

  // eq. (6): multiplier tables, linear on a uniform grid, clamped; the gather
  // goes out first, the work below that does not need it hides its latency
  float x = fmaxf((T - d.t_lo) * d.t_scale, 0.0f);  // NaN -> 0
  x = fminf(x, (float)(d.table_n - 1));
  const int i0 = max(min((int)x, d.table_n - 2), 0);
  const float w = x - (float)i0;
  const gptr<const float> tp = as_global((const float *)d.table) + 4 * i0;
  const float4 te = make_float4(tp[0], tp[1], tp[2], tp[3]);
  if constexpr (!__is_same(H, NoHook)) {
    __builtin_amdgcn_sched_barrier(0);
    hook();
    __builtin_amdgcn_sched_barrier(0);
  }

  // b of the equilibria (feq_link): 1 - 1.5 u.u
  const float base = 1.0f - 1.5f * (ux * ux + ur * ur);

  // eq. (4): Q_ij = sum_k e_ki e_kj (f_k - f_k^eq), with the second moments of
  // the equilibrium in closed form: rho/3 delta_ij + rho u_i u_j
  const float qxx = (s13 + sd) - rho * __builtin_fmaf(ux, ux, 1.0f / 3.0f);
  const float qrr = (s24 + sd) - rho * __builtin_fmaf(ur, ur, 1.0f / 3.0f);
  const float qxr = ((f[5] + f[7]) - (f[6] + f[8])) - mx * ur;
  // sum_k e_kr g_k^neq = (g_+r - g_-r) - T u_r
  const float jr = (g[1] - g[3]) - T * ur;
  const float qn = fast_sqrt(2.0f * (qxx * qxx + 2.0f * qxr * qxr + qrr * qrr));

  const float nu = d.nu0 * (te.x + w * te.y);
  const float alpha = d.alpha0 * (te.z + w * te.w);
  const float tau_nu = 0.5f + 3.0f * nu;

  // eq. (4): local relaxation time
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
  const float S = (-T * ur - ka * jr) * rinv;

  // eq. (1), as f (1 - 1/tau) + f^eq / tau + source, relaxing opposite links
  // together.  For k and k' = opp(k) (e_k' = -e_k) the equilibria share their
  // even part w rho (b + 4.5 (e.u)^2) and differ in the sign of the odd part
  // 3 w rho e.u; the sources likewise (w theta even, e.F / 6 odd):
  //   f*_k = f_k (1 - 1/tau) + E + O,   f*_k' = f_k' (1 - 1/tau) + E - O,
  //   E = w rho (b + 4.5 (e.u)^2) / tau + w theta,  O = 3 w rho (e.u) / tau + e.F / 6.
  const float fx6 = Fx * (1.0f / 6.0f), fr6 = Fr * (1.0f / 6.0f);
  const float omf = 1.0f - itau, omg = 1.0f - itau_a;
  const float rt = rho * itau;
  const auto relax_pair = [&](int k, int kp, float w, float eu, float ef) {
    const float cw = w * rt;
    const float E = __builtin_fmaf(cw, __builtin_fmaf(4.5f * eu, eu, base), w * theta);
    const float O = __builtin_fmaf(3.0f * cw, eu, ef);
    f[k] = __builtin_fmaf(f[k], omf, E + O);
    f[kp] = __builtin_fmaf(f[kp], omf, E - O);
  };
  f[0] = __builtin_fmaf(f[0], omf, __builtin_fmaf(w9(0) * rt, base, w9(0) * theta));
  relax_pair(1, 3, w9(1), ux, fx6);                 // (+-1, 0)
  relax_pair(2, 4, w9(2), ur, fr6);                 // (0, +-1)
  relax_pair(5, 7, w9(5), ux + ur, fx6 + fr6);      // +-(1, 1)
  relax_pair(6, 8, w9(6), ur - ux, fr6 - fx6);      // +-(-1, 1)
  // D2Q4: g^eq_k / tau_a = T / (4 tau_a) + (e_k.u) T / (2 tau_a); the source
  // S / 4 is even
  const float cT = T * itau_a;
  const float Eg = __builtin_fmaf(0.25f, cT, 0.25f * S);
  const float hx = 0.5f * cT * ux, hr = 0.5f * cT * ur;
  g[0] = __builtin_fmaf(g[0], omg, Eg + hx);  // +x
  g[2] = __builtin_fmaf(g[2], omg, Eg - hx);  // -x
  g[1] = __builtin_fmaf(g[1], omg, Eg + hr);  // +r
  g[3] = __builtin_fmaf(g[3], omg, Eg - hr);  // -r

  return (rho > 0.0f) && (rho < __builtin_inff()) && (fabsf(T) < __builtin_inff());
}

// ---------------------------------------------------------------------------
// Pull.  load(p, i, j) reads plane p of the source buffer at node (i, j).
// ---------------------------------------------------------------------------
template <class C>
struct Src {
  gptr<const typename C::T> base;
  int64_t plane;
  int32_t pitch;
  __device__ __forceinline__ float load(const JetDesc &d, int p, int i, int j) const {
    return C::dec(base[(int64_t)p * plane + node_index(pitch, i, j)], pop_offset<C>(d, p));
  }
};

template <class C>
struct Dst {
  gptr<typename C::T> base;
  int64_t plane;
  int32_t pitch;
  __device__ __forceinline__ void put(const JetDesc &d, int p, int i, int j, float v,
                                     uint32_t k) const {
    base[(int64_t)p * plane + node_index(pitch, i, j)] = C::enc(v, pop_offset<C>(d, p), k);
  }
};

// x-side rule for plane p taken from column ip of row jr; (i_land, j_land)
// is the receiving node (for a mirrored pull, the node of the edge row).
template <class C, class S>
__device__ __forceinline__ float pull_x(const JetDesc &d, const S &s, int p, int ip,
                                        int jr, int i_land, int j_land, const float4 *inrow) {
  if (ip >= 0 && ip < d.nx) return s.load(d, p, ip, jr);
  const int side = ip < 0 ? 0 : 1;
  switch (d.bc[side]) {
    case BC_PERIODIC:
      return s.load(d, p, ip < 0 ? ip + d.nx : ip - d.nx, jr);
    case BC_OUTFLOW:
      return s.load(d, p, d.nx - 1, jr);
    case BC_INLET: {
      const gptr<const float> qp = as_global((const float *)inrow) + 4 * jr;
      const float4 q = make_float4(qp[0], qp[1], qp[2], qp[3]);
      return eq_plane(p, 1.0f, q.x, q.y, q.z);
    }
    case BC_WALL: {
      const int po = p < 9 ? opp9(p) : 9 + opp4(p - 9);
      float v = s.load(d, po, i_land, j_land);
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
template <class C, class S>
__device__ __forceinline__ float pull_edge(const JetDesc &d, const S &s, int p, int i,
                                           int j, const float4 *inrow) {
  const int ip = i - pex(p), jp = j - per(p);
  if (jp >= 0 && jp < d.nr) return pull_x<C, S>(d, s, p, ip, jp, i, j, inrow);
  const int side = jp < 0 ? 2 : 3;
  const int bc = d.bc[side];
  if (bc == BC_AXIS || bc == BC_FREESLIP) {
    const int pm = p < 9 ? mir9(p) : 9 + mir4(p - 9);
    const int je = jp < 0 ? 0 : d.nr - 1;
    return pull_x<C, S>(d, s, pm, ip, je, i, je, inrow);
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

// All 13 pulled values of node (i, j) from a buffer whose ghost ring is
// current: every pull is a plain load.
template <class C, class S>
__device__ __forceinline__ void pull_node(const JetDesc &d, const S &s, int i, int j,
                                          float (&f)[9], float (&g)[4]) {
#pragma unroll
  for (int p = 0; p < NPOP; ++p) {
    const float v = s.load(d, p, i - pex(p), j - per(p));
    if (p < 9) f[p] = v; else g[p - 9] = v;
  }
}

// ---------------------------------------------------------------------------
// Views of a stored state.  In the two-buffer scheme a buffer holds, at a
// fluid node y and plane p, the post-collision value f*_p(y) of the last
// step, and at a ghost position g the value that node g + e_p pulls along p.
// The single-buffer (AA) scheme keeps one buffer in one of two layouts:
//   swapped (after an even number of steps): the two-buffer array with
//     planes p and opp(p) exchanged, f*_p(y) in plane opp(p) at y;
//   natural (after an odd number of steps): every population already
//     streamed, plane p at node x holding the value x pulls along p.
// A step from the swapped layout pulls from the neighbours and pushes to
// them; a step from the natural layout reads and writes only its own node.
// In both, every location is read and written by one thread, so a single
// buffer suffices.
//   load(p, i, j):      the two-buffer value at (i, j);
//   put(p, i, j, v):    write it (for a ghost position: the value pulled by
//                       (i, j) + e_p along p), i.e. the epilogue's and the
//                       ghost fill's destination;
//   pulled(p, i, j):    the value fluid node (i, j) pulls along p.
// view: 0, 1 = buffer 0 or 1 of the two-buffer scheme; 2 = swapped,
// 3 = natural layout of the single buffer (buf[0]).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int opp_plane(int p) { return p < 9 ? opp9(p) : 9 + opp4(p - 9); }

template <class C>
struct State {
  using T = typename C::T;
  gptr<T> base;
  int64_t plane;
  int32_t pitch;
  int32_t kind;  // 0: two-buffer, 1: swapped, 2: natural
  __device__ __forceinline__ gptr<T> at(int p, int i, int j) const {
    if (kind == 1) p = opp_plane(p);
    if (kind == 2) { i += pex(p); j += per(p); }
    return base + ((int64_t)p * plane + node_index(pitch, i, j));
  }
  __device__ __forceinline__ float load(const JetDesc &d, int p, int i, int j) const {
    return C::dec(*at(p, i, j), pop_offset<C>(d, p));
  }
  __device__ __forceinline__ void put(const JetDesc &d, int p, int i, int j, float v,
                                     uint32_t k) const {
    *at(p, i, j) = C::enc(v, pop_offset<C>(d, p), k);
  }
  __device__ __forceinline__ float pulled(const JetDesc &d, int p, int i, int j) const {
    const gptr<T> q = kind == 2 ? base + ((int64_t)p * plane + node_index(pitch, i, j))
                                : at(p, i - pex(p), j - per(p));
    return C::dec(*q, pop_offset<C>(d, p));
  }
};

template <class C>
__device__ __forceinline__ State<C> state_view(const JetDesc &d, int32_t view) {
  return State<C>{as_global(static_cast<typename C::T *>(d.buf[view == 1 ? 1 : 0])), d.plane,
                  d.pitch, view < 2 ? 0 : view - 1};
}

// The 13 values node (i, j) pulls, through a view.
template <class C>
__device__ __forceinline__ void pulled_node(const JetDesc &d, const State<C> &s, int i, int j,
                                            float (&f)[9], float (&g)[4]) {
#pragma unroll
  for (int p = 0; p < NPOP; ++p) {
    const float v = s.pulled(d, p, i, j);
    if (p < 9) f[p] = v; else g[p - 9] = v;
  }
}

// If the value node (i, j) pulls along p comes from outside the domain and
// the edge rules (r side first, as pull_edge) resolve it to an equilibrium
// side, set v to it and return true.
__device__ __forceinline__ bool eq_pull(const JetDesc &d, int p, int i, int j, float &v) {
  const int ip = i - pex(p), jp = j - per(p);
  int pp = p;
  if (jp < 0 || jp >= d.nr) {
    const int side = jp < 0 ? 2 : 3;
    const int bc = d.bc[side];
    if (bc == BC_EQ) {
      const float *e = d.eq[side];
      v = eq_plane(p, e[0], e[1], e[2], e[3]);
      return true;
    }
    if (bc != BC_AXIS && bc != BC_FREESLIP) return false;
    pp = p < 9 ? mir9(p) : 9 + mir4(p - 9);  // the mirrored link, x rule
  }
  if (ip >= 0 && ip < d.nx) return false;
  const int side = ip < 0 ? 0 : 1;
  if (d.bc[side] != BC_EQ) return false;
  const float *e = d.eq[side];
  v = eq_plane(pp, e[0], e[1], e[2], e[3]);
  return true;
}

// Thermal wall: anti-bounce-back towards the wall temperature, or plain
// bounce-back (adiabatic) when it is NaN.
__device__ __forceinline__ float wall_g(const JetDesc &d, int side, float v) {
  const float tw = d.wallT[side];
  return tw == tw ? -v + 0.5f * tw : v;
}

// Inlet row entry j as (ux, ur, T, 0), read through a global pointer.
__device__ __forceinline__ float4 inlet_at(const float4 *in, int j) {
  const gptr<const float> q = as_global((const float *)in) + 4 * j;
  return make_float4(q[0], q[1], q[2], 0.0f);
}

// After the collision of node (i, j), write the ghost values of the next
// step that this node is the source of, following the edge rules (r side
// first; a mirrored pull goes through the x rule at the edge row).  Ghosts
// of equilibrium sides are constant and written once by the ghost fill.
// `in` is the inlet row of the next step.
// O is any destination with put(d, p, i, j, v): the next buffer, or the
// LDS image of the intermediate state of a two-step launch.
template <class C, class O>
__device__ __forceinline__ void ghost_epilogue(const JetDesc &d, const O &o, int i, int j,
                                               const float (&f)[9], const float (&g)[4],
                                               const float4 *in, uint32_t key) {
  // a copy of population k takes k's key; a computed value its own plane's
  const auto K = [&](int k) { return plane_key(key, k); };
  const int nx = d.nx, nr = d.nr;
  const int x0 = d.bc[0], x1 = d.bc[1], r0 = d.bc[2], r1 = d.bc[3];
  const bool mir0 = (r0 == BC_AXIS) | (r0 == BC_FREESLIP);
  const bool mir1 = r1 == BC_FREESLIP;
  if (j == 0) {  // ghost row -1: links 2, 5, 6 and g1 (+r)
    if (mir0) {
      o.put(d, 2, i, -1, f[4], K(4));
      o.put(d, 5, i, -1, f[8], K(8));
      o.put(d, 6, i, -1, f[7], K(7));
      o.put(d, 10, i, -1, g[3], K(12));
    } else if (r0 == BC_WALL) {
      o.put(d, 2, i, -1, f[4], K(4));
      o.put(d, 5, i - 1, -1, f[7], K(7));
      o.put(d, 6, i + 1, -1, f[8], K(8));
      o.put(d, 10, i, -1, wall_g(d, 2, g[3]), K(10));
    }
  }
  if (j == nr - 1) {  // ghost row nr: links 4, 7, 8 and g3 (-r)
    if (mir1) {
      o.put(d, 4, i, nr, f[2], K(2));
      o.put(d, 7, i, nr, f[6], K(6));
      o.put(d, 8, i, nr, f[5], K(5));
      o.put(d, 12, i, nr, g[1], K(10));
    } else if (r1 == BC_WALL) {
      o.put(d, 4, i, nr, f[2], K(2));
      o.put(d, 7, i + 1, nr, f[5], K(5));
      o.put(d, 8, i - 1, nr, f[6], K(6));
      o.put(d, 12, i, nr, wall_g(d, 3, g[1]), K(12));
    }
  }
  if (i == 0) {  // ghost column -1 (rows 0..nr-1): links 1, 5, 8 and g0 (+x)
    if (x0 == BC_INLET) {
      const float4 q = inlet_at(in, j);
      o.put(d, 1, -1, j, feq_link(1, 1.0f, q.x, q.y), K(1));
      o.put(d, 5, -1, j, feq_link(5, 1.0f, q.x, q.y), K(5));
      o.put(d, 8, -1, j, feq_link(8, 1.0f, q.x, q.y), K(8));
      o.put(d, 9, -1, j, geq_link(0, q.z, q.x, q.y), K(9));
    } else if (x0 == BC_WALL) {
      o.put(d, 1, -1, j, f[3], K(3));
      if (j >= 1) o.put(d, 5, -1, j - 1, f[7], K(7));
      if (j + 1 < nr) o.put(d, 8, -1, j + 1, f[6], K(6));
      o.put(d, 9, -1, j, wall_g(d, 0, g[2]), K(9));
    }
    if (x1 == BC_PERIODIC) {  // column nx repeats column 0
      o.put(d, 3, nx, j, f[3], K(3));
      o.put(d, 6, nx, j, f[6], K(6));
      o.put(d, 7, nx, j, f[7], K(7));
      o.put(d, 11, nx, j, g[2], K(11));
    }
  }
  if (i == nx - 1) {  // ghost column nx: links 3, 6, 7 and g2 (-x)
    if (x1 == BC_OUTFLOW) {
      o.put(d, 3, nx, j, f[3], K(3));
      o.put(d, 6, nx, j, f[6], K(6));
      o.put(d, 7, nx, j, f[7], K(7));
      o.put(d, 11, nx, j, g[2], K(11));
    } else if (x1 == BC_WALL) {
      o.put(d, 3, nx, j, f[1], K(1));
      if (j >= 1) o.put(d, 6, nx, j - 1, f[8], K(8));
      if (j + 1 < nr) o.put(d, 7, nx, j + 1, f[5], K(5));
      o.put(d, 11, nx, j, wall_g(d, 1, g[0]), K(11));
    }
    if (x0 == BC_PERIODIC) {  // column -1 repeats column nx-1
      o.put(d, 1, -1, j, f[1], K(1));
      o.put(d, 5, -1, j, f[5], K(5));
      o.put(d, 8, -1, j, f[8], K(8));
      o.put(d, 9, -1, j, g[0], K(9));
    }
  }
  // corner ghosts under a mirror edge: the mirrored link goes through the
  // x rule at the edge row
  if (j == 0 && mir0) {
    // (-1, -1) link 5 <- x rule of link 8 at column -1, row 0
    if (i == nx - 1 && x0 == BC_PERIODIC) o.put(d, 5, -1, -1, f[8], K(8));
    if (i == 0 && x0 == BC_INLET) {
      const float4 q = inlet_at(in, 0);
      o.put(d, 5, -1, -1, feq_link(8, 1.0f, q.x, q.y), K(5));
    }
    if (i == 0 && x0 == BC_WALL) o.put(d, 5, -1, -1, f[6], K(6));
    // (nx, -1) link 6 <- x rule of link 7 at column nx, row 0
    if (i == 0 && x1 == BC_PERIODIC) o.put(d, 6, nx, -1, f[7], K(7));
    if (i == nx - 1 && x1 == BC_OUTFLOW) o.put(d, 6, nx, -1, f[7], K(7));
    if (i == nx - 1 && x1 == BC_WALL) o.put(d, 6, nx, -1, f[5], K(5));
  }
  if (j == nr - 1 && mir1) {
    // (-1, nr) link 8 <- x rule of link 5 at column -1, row nr-1
    if (i == nx - 1 && x0 == BC_PERIODIC) o.put(d, 8, -1, nr, f[5], K(5));
    if (i == 0 && x0 == BC_INLET) {
      const float4 q = inlet_at(in, nr - 1);
      o.put(d, 8, -1, nr, feq_link(5, 1.0f, q.x, q.y), K(8));
    }
    if (i == 0 && x0 == BC_WALL) o.put(d, 8, -1, nr, f[7], K(7));
    // (nx, nr) link 7 <- x rule of link 6 at column nx, row nr-1
    if (i == 0 && x1 == BC_PERIODIC) o.put(d, 7, nx, nr, f[6], K(6));
    if (i == nx - 1 && x1 == BC_OUTFLOW) o.put(d, 7, nx, nr, f[6], K(6));
    if (i == nx - 1 && x1 == BC_WALL) o.put(d, 7, nx, nr, f[8], K(8));
  }
}

// Epilogue of a single-buffer step: the producer-written ghost values, plus
// the constant values of equilibrium sides that this edge node pulls (the
// single buffer does not keep them between steps).  `o` is the view of the
// state the step produces.
template <class C>
__device__ __forceinline__ void aa_epilogue(const JetDesc &d, const State<C> &o, int i, int j,
                                            const float (&f)[9], const float (&g)[4],
                                            const float4 *in, uint32_t key) {
  ghost_epilogue<C>(d, o, i, j, f, g, in, key);
  if ((d.bc[0] == BC_EQ) | (d.bc[1] == BC_EQ) | (d.bc[2] == BC_EQ) | (d.bc[3] == BC_EQ)) {
#pragma unroll
    for (int p = 1; p < NPOP; ++p) {
      const int gi = i - pex(p), gj = j - per(p);
      float v;
      if ((gi < 0 || gi >= d.nx || gj < 0 || gj >= d.nr) && eq_pull(d, p, i, j, v))
        o.put(d, p, gi, gj, v, plane_key(sr_key(gi, gj, 0), p));  // as ghost_fill_kernel
    }
  }
}

}  // namespace lbmx
