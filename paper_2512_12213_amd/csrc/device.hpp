// Device-side building blocks shared by the forward step kernels and the
// adjoint kernels: storage formats, row-blocked A-A addressing with halfway
// bounce-back, and per-tile FP64 reductions.
//
// Distributions live in one in-place array per lattice, blocked by x-row:
// element (q, row, x) at (row Q + q) nx + x.  All quantities are
// dimensionless: velocities in units of c = dx/dt, body force as a dt / c.
#pragma once
#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------
// Cache hints (measured on MI355X, D3Q19 duct 256x128x128): 4- and 2-byte
// stores are plain (temporal), so that the partial 128-byte lines of the
// x-shifted A-A writes are merged in L2 before they are written back
// (non-temporal stores cost 4 % in FP32, 7 % on odd steps); 8-byte stores stay
// non-temporal (plain ones cost FP64 5 %).  4- and 8-byte loads are
// non-temporal, 2-byte loads plain (7 % faster for the 16-bit formats).
template <int P>
struct Stor;
template <>
struct Stor<S_F64> {
  using E = double;
  using T = double;
  static __device__ __forceinline__ T ld(const E* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(E* p, T v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Stor<S_F32> {
  using E = float;
  using T = float;
  static __device__ __forceinline__ T ld(const E* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(E* p, T v) { *p = v; }
};
template <>
struct Stor<S_F16> {
  using E = _Float16;
  using T = float;
  static __device__ __forceinline__ T ld(const E* p) { return (float)*p; }
  static __device__ __forceinline__ void st(E* p, T v) { *p = (_Float16)v; }
};
template <>
struct Stor<S_BF16> {
  using E = uint16_t;
  using T = float;
  static __device__ __forceinline__ T ld(const E* p) {
    return __uint_as_float(uint32_t(*p) << 16);
  }
  // round to nearest even (the hardware conversion; the same bits as the
  // integer form u + 0x7FFF + lsb for every finite value)
  static __device__ __forceinline__ void st(E* p, T v) { *p = __builtin_bit_cast(uint16_t, (__bf16)v); }
};

// A parameter in the arithmetic type T: the FP64 value, or its FP32 copy
// (rounded by the host exactly as the conversion here would round it).
template <class T>
__device__ __forceinline__ T par(double v, float) {
  return (T)v;
}
template <>
__device__ __forceinline__ float par<float>(double, float v) {
  return v;
}

template <class T>
__device__ __forceinline__ T rcp(T x) {
  return T(1) / x;
}
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// Square root: FP64 correctly rounded; FP32 the hardware instruction (within
// 1 ulp, without the correction steps of the correctly rounded expansion).
template <class T>
__device__ __forceinline__ T vsqrt(T x) {
  return sqrt(x);
}
template <>
__device__ __forceinline__ float vsqrt<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}

// The same formats through a buffer resource (scalar base and range,
// wave-uniform scalar byte offset, per-lane byte offset), with the same cache
// hints (aux bit 1: non-temporal).
template <int P>
struct BufIO;
template <>
struct BufIO<S_F64> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 2));
  }
  static __device__ __forceinline__ void st(double x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, v, s, 2);
  }
};
template <>
struct BufIO<S_F32> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, v, s, 2));
  }
  // plain (cached) load, for AddrBP
  static __device__ __forceinline__ float ldp(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(float x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, v, s, 0);
  }
};
template <>
struct BufIO<S_F16> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(float x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (_Float16)x), r, v, s, 0);
  }
};
template <>
struct BufIO<S_BF16> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __uint_as_float(uint32_t((uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0)) << 16);
  }
  static __device__ __forceinline__ void st(float x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (__bf16)x), r, v, s, 0);
  }
};

// ---------------------------------------------------------------------------
// index helpers
// ---------------------------------------------------------------------------
// Element offsets to the six axis neighbours (periodic wrap) in a row-blocked
// array whose rows hold P planes (row stride rs = P nx).
struct Offs {
  int xp, xm;
  int64_t yp, ym, zp, zm;
};

__device__ __forceinline__ void coords(const Geom& g, uint32_t n, uint32_t& x, uint32_t& y, uint32_t& z, uint32_t& r) {
  r = g.nx == 1 ? n : (uint32_t)__umul64hi((uint64_t)n, g.mnx);
  x = n - r * g.nx;
  z = g.ny == 1 ? r : (uint32_t)__umul64hi((uint64_t)r, g.mny);
  y = r - z * g.ny;
}

__device__ __forceinline__ Offs offsets(const Geom& g, uint32_t x, uint32_t y, uint32_t z, uint64_t rs) {
  Offs o;
  const int nx = (int)g.nx;
  const int64_t ry = (int64_t)rs, rz = (int64_t)rs * g.ny;
  o.xp = (x + 1 == g.nx) ? 1 - nx : 1;
  o.xm = (x == 0) ? nx - 1 : -1;
  o.yp = (y + 1 == g.ny) ? (1 - (int64_t)g.ny) * ry : ry;
  o.ym = (y == 0) ? ((int64_t)g.ny - 1) * ry : -ry;
  o.zp = (z + 1 == g.nz) ? (1 - (int64_t)g.nz) * rz : rz;
  o.zm = (z == 0) ? ((int64_t)g.nz - 1) * rz : -rz;
  return o;
}

// Offset from a node to its neighbour along e_q.
template <class L>
__device__ __forceinline__ int64_t off_of(int q, const Offs& o) {
  int64_t s = 0;
  if (L::ex(q) > 0) s += o.xp;
  if (L::ex(q) < 0) s += o.xm;
  if (L::ey(q) > 0) s += o.yp;
  if (L::ey(q) < 0) s += o.ym;
  if (L::ez(q) > 0) s += o.zp;
  if (L::ez(q) < 0) s += o.zm;
  return s;
}

// Addressing of one node's slots in a row-blocked array with P planes:
// ptr<L>(f, plane, q) points at `plane` of the neighbour x + e_q (q < 0: the
// node itself).
//
// Generic form: a per-lane element index of the node plus neighbour offsets.
struct AddrG {
  uint64_t b;
  Offs o;
  uint32_t nx;
  template <class L, class E>
  __device__ __forceinline__ E* ptr(E* f, int plane, int q) const {
    return f + ((q < 0 ? b : b + off_of<L>(q, o)) + (uint32_t)plane * nx);
  }
  template <class L, int P>
  __device__ __forceinline__ typename Stor<P>::T ld(const typename Stor<P>::E* f, int plane, int q) const;
  template <class L, int P>
  __device__ __forceinline__ void st(typename Stor<P>::E* f, int plane, int q, typename Stor<P>::T v) const;
};

// Row-uniform form, used when nx is a multiple of 64: a wavefront then never
// leaves its x-row, so y, z and every neighbour-row base are wave-uniform
// (scalar registers) and each lane only adds its 32-bit x byte offset
// (scalar base + vector offset addressing).  The row bases are recomputed in
// ptr() rather than kept in an array, so that the compiler never turns a
// per-lane choice between two slots into a dynamic index of private memory.
struct AddrR {
  uint32_t y, z, ny, nz;
  uint32_t x, xm, xp;  // x, x - 1, x + 1 (periodic), per lane
  uint32_t nx;
  uint64_t rs;         // row stride, planes * nx
  template <class L, class E>
  __device__ __forceinline__ E* ptr(E* f, int plane, int q) const {
    const int dx = q < 0 ? 0 : L::ex(q), dy = q < 0 ? 0 : L::ey(q), dz = q < 0 ? 0 : L::ez(q);
    const uint32_t yy = dy < 0 ? (y == 0 ? ny - 1 : y - 1) : (dy > 0 ? (y + 1 == ny ? 0 : y + 1) : y);
    const uint32_t zz = dz < 0 ? (z == 0 ? nz - 1 : z - 1) : (dz > 0 ? (z + 1 == nz ? 0 : z + 1) : z);
    E* base = f + (((uint64_t)zz * ny + yy) * rs + (uint32_t)plane * nx);  // wave-uniform
    const uint32_t xs = dx < 0 ? xm : (dx > 0 ? xp : x);
    return (E*)((char*)base + xs * (uint32_t)sizeof(E));  // 32-bit byte offset
  }
  template <class L, int P>
  __device__ __forceinline__ typename Stor<P>::T ld(const typename Stor<P>::E* f, int plane, int q) const;
  template <class L, int P>
  __device__ __forceinline__ void st(typename Stor<P>::E* f, int plane, int q, typename Stor<P>::T v) const;
};

// Row-uniform buffer form, used when nx is a multiple of 64 and the array
// is below 4 GiB: the array is a buffer resource (four scalar registers), the
// row and plane offset a wave-uniform scalar, and each lane adds only its x
// byte offset; no 64-bit per-lane addresses are formed (they cost two vector
// registers and a vector add per access in the pointer form).  Only for rows
// without boundary links (no per-lane choice between slots).
struct AddrB {
  __amdgpu_buffer_rsrc_t rs;
  uint32_t y, z, ny, nz;
  uint32_t vx, vxm, vxp;  // byte offsets of x, x - 1, x + 1 (periodic), per lane
  uint32_t nxb, rsb;      // bytes of one plane of a row, of one row block
  template <class L>
  __device__ __forceinline__ uint32_t soff(int plane, int q) const {
    const int dy = q < 0 ? 0 : L::ey(q), dz = q < 0 ? 0 : L::ez(q);
    const uint32_t yy = dy < 0 ? (y == 0 ? ny - 1 : y - 1) : (dy > 0 ? (y + 1 == ny ? 0 : y + 1) : y);
    const uint32_t zz = dz < 0 ? (z == 0 ? nz - 1 : z - 1) : (dz > 0 ? (z + 1 == nz ? 0 : z + 1) : z);
    return (zz * ny + yy) * rsb + (uint32_t)plane * nxb;  // wave-uniform
  }
  template <class L>
  __device__ __forceinline__ uint32_t voff(int q) const {
    const int dx = q < 0 ? 0 : L::ex(q);
    return dx < 0 ? vxm : (dx > 0 ? vxp : vx);
  }
  template <class L, int P>
  __device__ __forceinline__ typename Stor<P>::T ld(const typename Stor<P>::E*, int plane, int q) const {
    return BufIO<P>::ld(rs, voff<L>(q), soff<L>(plane, q));
  }
  template <class L, int P>
  __device__ __forceinline__ void st(typename Stor<P>::E*, int plane, int q, typename Stor<P>::T v) const {
    BufIO<P>::st(v, rs, voff<L>(q), soff<L>(plane, q));
  }
  // the same rows as ld / st along e_q, but the lane's own x (no x shift)
  template <class L, int P>
  __device__ __forceinline__ typename Stor<P>::T ldx(int plane, int q) const {
    return BufIO<P>::ld(rs, vx, soff<L>(plane, q));
  }
  template <class L, int P>
  __device__ __forceinline__ void stx(int plane, int q, typename Stor<P>::T v) const {
    BufIO<P>::st(v, rs, vx, soff<L>(plane, q));
  }
};

// The same addressing with plain (cached) FP32 loads instead of non-temporal
// ones.  On lattices far beyond the last-level cache the odd step reads each
// line it later writes, and keeping it cached measured 3 % faster there
// (512x256x256 duct, odd step 968 -> 939 us); on the 256x128x128 duct, whose
// state partly stays in that cache between steps, non-temporal loads are
// 4.5 % faster, so the host picks this form for large states only.
struct AddrBP : AddrB {
  template <class L, int P>
  __device__ __forceinline__ typename Stor<P>::T ld(const typename Stor<P>::E*, int plane, int q) const {
    static_assert(P == S_F32, "plain loads: FP32 storage");
    return BufIO<P>::ldp(rs, voff<L>(q), soff<L>(plane, q));
  }
  template <class L, int P>
  __device__ __forceinline__ typename Stor<P>::T ldx(int plane, int q) const {
    static_assert(P == S_F32, "plain loads: FP32 storage");
    return BufIO<P>::ldp(rs, vx, soff<L>(plane, q));
  }
};

template <class L, int P>
__device__ __forceinline__ typename Stor<P>::T AddrG::ld(const typename Stor<P>::E* f, int plane, int q) const {
  return Stor<P>::ld(ptr<L>(f, plane, q));
}
template <class L, int P>
__device__ __forceinline__ void AddrG::st(typename Stor<P>::E* f, int plane, int q, typename Stor<P>::T v) const {
  Stor<P>::st(ptr<L>(f, plane, q), v);
}
template <class L, int P>
__device__ __forceinline__ typename Stor<P>::T AddrR::ld(const typename Stor<P>::E* f, int plane, int q) const {
  return Stor<P>::ld(ptr<L>(f, plane, q));
}
template <class L, int P>
__device__ __forceinline__ void AddrR::st(typename Stor<P>::E* f, int plane, int q, typename Stor<P>::T v) const {
  Stor<P>::st(ptr<L>(f, plane, q), v);
}

__device__ __forceinline__ AddrG addr_g(const Geom& g, uint32_t x, uint32_t y, uint32_t z, uint32_t r, uint32_t P) {
  AddrG a;
  a.b = (uint64_t)r * (P * g.nx) + x;
  a.o = offsets(g, x, y, z, (uint64_t)P * g.nx);
  a.nx = g.nx;
  return a;
}

// y, z must be wave-uniform.
__device__ __forceinline__ AddrR addr_r(const Geom& g, uint32_t x, uint32_t y, uint32_t z, uint32_t P) {
  AddrR a;
  a.y = y;
  a.z = z;
  a.ny = g.ny;
  a.nz = g.nz;
  a.x = x;
  a.xm = x == 0 ? g.nx - 1 : x - 1;
  a.xp = x + 1 == g.nx ? 0 : x + 1;
  a.nx = g.nx;
  a.rs = (uint64_t)P * g.nx;
  return a;
}

// y, z must be wave-uniform; bytes (the whole array) below 4 GiB.
template <class E>
__device__ __forceinline__ AddrB addr_b(const Geom& g, uint32_t x, uint32_t y, uint32_t z, uint32_t P, const void* f,
                                        uint32_t bytes) {
  AddrB a;
  a.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(f), 0, bytes, 0x00020000);
  a.y = y;
  a.z = z;
  a.ny = g.ny;
  a.nz = g.nz;
  a.vx = x * (uint32_t)sizeof(E);
  a.vxm = (x == 0 ? g.nx - 1 : x - 1) * (uint32_t)sizeof(E);
  a.vxp = (x + 1 == g.nx ? 0 : x + 1) * (uint32_t)sizeof(E);
  a.nxb = g.nx * (uint32_t)sizeof(E);
  a.rsb = P * a.nxb;
  return a;
}

// Per-lane choice between two addresses, written as mask arithmetic on the
// address values so that it is not folded into an indexed access of the
// address objects' fields.
template <class E>
__device__ __forceinline__ E* pick(bool c, E* a, E* b) {
  const uint64_t m = 0ull - (uint64_t)c;
  return (E*)(((uint64_t)a & m) | ((uint64_t)b & ~m));
}

// Sums start from -0, the exact additive identity (x + -0 = x for every x,
// while 0 + -0 = +0), so that the compiler can drop the first addition.
template <class T>
constexpr T ZERO = T(-0.0);

template <class L, class T>
__device__ __forceinline__ T edot(int q, T vx, T vy, T vz) {
  T s = ZERO<T>;
  if (L::ex(q) > 0) s += vx;
  if (L::ex(q) < 0) s -= vx;
  if (L::ey(q) > 0) s += vy;
  if (L::ey(q) < 0) s -= vy;
  if (L::ez(q) > 0) s += vz;
  if (L::ez(q) < 0) s -= vz;
  return s;
}

__device__ __forceinline__ uint32_t nibble(const uint4& r, int q) {
  const uint32_t w = q < 8 ? r.y : (q < 16 ? r.z : r.w);
  return (w >> (4 * (q & 7))) & 15u;
}

// ---------------------------------------------------------------------------
// A-A reads and writes of one node's distributions
// ---------------------------------------------------------------------------
// Reading the state f_q(x, t):
//   even parity (natural layout): slot q of x;
//   odd parity: slot opp(q) of x - e_q, or, when the link from x along
//   -e_q ends in a wall, slot q of x (where the bounce-back value was put).
// (SCALE = false: 16-bit values are returned as stored, without the
// per-direction factor of their format.)
template <class L, int P, int PAR, bool BND, class AD, bool SCALE = true>
__device__ __forceinline__ void read_f(const typename Stor<P>::E* __restrict__ f, const AD& A, uint32_t mask,
                                       const Phys& p, typename Stor<P>::T (&d)[L::Q]) {
  using S = Stor<P>;
  using T = typename S::T;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const int qb = opp(q);
    T v;
    if constexpr (PAR == 0) {
      v = A.template ld<L, P>(f, q, -1);
    } else if constexpr (BND) {
      // a wall link: the value was put in the node's own slot q
      v = S::ld(pick((mask >> qb) & 1u, A.template ptr<L>(f, q, -1), A.template ptr<L>(f, qb, qb)));
    } else {
      v = A.template ld<L, P>(f, qb, qb);
    }
    if (SCALE && (P == S_F16 || P == S_BF16)) v *= (T)p.inv_scale[q];
    d[q] = v;
  }
}

// Writing the post-collision value v_q of node x (v_q already holds the
// bounce-back value, including the moving-wall term, for wall links):
//   even parity: slot opp(q) of x;
//   odd parity: slot q of x + e_q, or slot opp(q) of x for a wall link.
// One direction at a time.
// (SCALE = false: v is already in the stored units of a 16-bit format.)
template <class L, int P, int PAR, bool BND, class AD, bool SCALE = true>
__device__ __forceinline__ void write_f1(typename Stor<P>::E* __restrict__ f, const AD& A, uint32_t mask, const Phys& p,
                                         int q, typename Stor<P>::T v) {
  using S = Stor<P>;
  using T = typename S::T;
  const int qb = opp(q);
  T s = v;
  if (SCALE && (P == S_F16 || P == S_BF16)) s *= (T)p.scale[q];
  if constexpr (PAR == 0) {
    A.template st<L, P>(f, qb, -1, s);
  } else if constexpr (BND) {
    // wall link: back into the node's own slot
    S::st(pick((mask >> q) & 1u, A.template ptr<L>(f, qb, -1), A.template ptr<L>(f, q, q)), s);
  } else {
    A.template st<L, P>(f, q, q, s);
  }
}

// Same pattern for the induction planes (K directions x NB components,
// plane NB k + i).
template <class L, int P, int PAR, bool BND, class AD>
__device__ __forceinline__ void read_g(const typename Stor<P>::E* __restrict__ g, const AD& A, uint32_t mask,
                                       typename Stor<P>::T (&h)[Ind<L>::K][Ind<L>::NB]) {
  using S = Stor<P>;
  constexpr int NB = Ind<L>::NB;
#pragma unroll
  for (int k = 0; k < Ind<L>::K; ++k) {
    const int kb = opp(k);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if constexpr (PAR == 0) {
        h[k][i] = A.template ld<L, P>(g, NB * k + i, -1);
      } else if constexpr (BND) {
        h[k][i] = S::ld(pick((mask >> kb) & 1u, A.template ptr<L>(g, NB * k + i, -1),
                             A.template ptr<L>(g, NB * kb + i, kb)));
      } else {
        h[k][i] = A.template ld<L, P>(g, NB * kb + i, kb);
      }
    }
  }
}

template <class L, int P, int PAR, bool BND, class AD>
__device__ __forceinline__ void write_g(typename Stor<P>::E* __restrict__ g, const AD& A, uint32_t mask,
                                        const typename Stor<P>::T (&h)[Ind<L>::K][Ind<L>::NB]) {
  using S = Stor<P>;
  constexpr int NB = Ind<L>::NB;
#pragma unroll
  for (int k = 0; k < Ind<L>::K; ++k) {
    const int kb = opp(k);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if constexpr (PAR == 0) {
        A.template st<L, P>(g, NB * kb + i, -1, h[k][i]);
      } else if constexpr (BND) {
        S::st(pick((mask >> k) & 1u, A.template ptr<L>(g, NB * kb + i, -1), A.template ptr<L>(g, NB * k + i, k)),
              h[k][i]);
      } else {
        A.template st<L, P>(g, NB * k + i, k, h[k][i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// Sum of v over the 256-thread tile (deterministic order) into
// out[k * stride], k < NV, stored (ADD = false) or added to what is there
// (ADD = true).  Every thread of the tile must call it.
// x from another lane of the same row of 16 (DPP lane pattern CTRL), both
// 32-bit halves moved by the vector ALU (no LDS round trip).  Every lane of
// the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Sum over the 64 lanes (the same value in every lane, fixed order): pairs,
// quads and halves of each row of 16 by DPP (lane i with i ^ 1, i ^ 2, then
// the mirrored lane of its half row and of its row), then the four row sums.
__device__ __forceinline__ double wave_sum_f64(double s) {
  s += dpp_f64<0xB1>(s);   // quad_perm [1,0,3,2]
  s += dpp_f64<0x4E>(s);   // quad_perm [2,3,0,1]
  s += dpp_f64<0x141>(s);  // row_half_mirror
  s += dpp_f64<0x140>(s);  // row_mirror
  return (readlane_f64(s, 0) + readlane_f64(s, 16)) + (readlane_f64(s, 32) + readlane_f64(s, 48));
}

template <int NV, bool ADD = false>
__device__ __forceinline__ void tile_sum_store(double (&v)[NV], double* __restrict__ out, uint64_t stride = 1) {
  __shared__ double sh[NTHREADS / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_f64(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    const double t = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    out[k * stride] = ADD ? out[k * stride] + t : t;
  }
}

}  // namespace lbm
