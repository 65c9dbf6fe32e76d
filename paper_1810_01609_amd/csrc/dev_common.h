// Device-side building blocks shared by the HIP kernels of libmdwf:
// precision traits, the internal field layouts, site geometry and complex
// arithmetic.  gfx950 only.
//
// Internal layouts (one parity, "half-field"; cb = lexicographic 4D index
// of the site divided by 2, which enumerates one parity when Lx is even):
//   spinor F64 : double2 [s][12 groups][cb]      group g = complex comp g
//   spinor F32 : float4  [s][6 groups][cb]       group g = comps 2g, 2g+1
//   spinor F16/BF16/I16 : 16-byte groups of 8 16-bit values [s][3][cb]
//              (comps 4g..4g+3), then (256-byte aligned) float scale [s][cb]:
//              value = half*scale, or int16/32767*scale (fixed point)
//   gauge  : 12 reals (rows 0,1) per link, [parity][mu][group][cb]
//            F64 6 x double2, F32 3 x float4, F16/BF16/I16 3 x 4 x 16 bits (8 bytes);
//            I16 links are int16/32767 (|U_ij| <= 1 needs no scale)
// Complex component index comp = spin*3 + colour, reals interleaved re,im.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace mdwf {

enum Prec : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3, I16 = 4 };

template <int P> struct PrecTraits;
template <> struct PrecTraits<F64> { using Real = double; };
template <> struct PrecTraits<F32> { using Real = float; };
template <> struct PrecTraits<F16> { using Real = float; };
template <> struct PrecTraits<BF16> { using Real = float; };
template <> struct PrecTraits<I16> { using Real = float; };

__host__ __device__ __forceinline__ size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Spinor fields are stored in tiles of kSiteTile consecutive sites: a tile
// holds all L5 slices and all 16-byte groups of its sites, site fastest
// ([tile][s][group][site in tile]).  With 16-site tiles (the stencil's
// workgroup width) the loads of one wavefront (16 sites x 4 slices) cover one
// contiguous block of memory, and a workgroup's whole 5D column is one
// contiguous block, instead of one short run per (slice, group) stream.
#ifndef MDWF_SITE_TILE
#define MDWF_SITE_TILE 16
#endif
constexpr int kSiteTile = MDWF_SITE_TILE;  // a power of two
__host__ __device__ __forceinline__ size_t padded_vh(int Vh) { return round_up((size_t)Vh, kSiteTile); }
// index, in 16-byte units, of group g of slice s of site cb (G groups per site).
// 64-bit arithmetic: the constant group offsets fold into the loads'
// immediate offsets (32-bit unsigned arithmetic, which may wrap, blocks that
// and cost the 16-bit stencils 5-11 %).
__host__ __device__ __forceinline__ size_t tile_index(int cb, int s, int g, int L5, int G) {
  return ((size_t)(cb / kSiteTile) * L5 + s) * (size_t)(G * kSiteTile) + (size_t)g * kSiteTile + (cb % kSiteTile);
}
// index of the per-site scale of (cb, s) in the 16-bit scale array
__host__ __device__ __forceinline__ size_t tile_scale_index(int cb, int s, int L5) {
  return ((size_t)(cb / kSiteTile) * L5 + s) * kSiteTile + (cb % kSiteTile);
}

// Byte offset of the per-site scale array inside a 16-bit spinor field.
__host__ __device__ __forceinline__ size_t half_scale_offset(int L5, int Vh) {
  return round_up((size_t)L5 * padded_vh(Vh) * 48u, 256u);
}

// Bytes of one spinor half-field of precision p.
__host__ __device__ __forceinline__ size_t spinor_field_bytes(int p, int L5, int Vh) {
  const size_t n = (size_t)L5 * padded_vh(Vh);
  switch (p) {
    case F64: return n * 192u;
    case F32: return n * 96u;
    default: return half_scale_offset(L5, Vh) + n * 4u;
  }
}

// Bytes one spinor site costs in HBM traffic (data + scale).
__host__ __device__ __forceinline__ int spinor_site_bytes(int p) { return p == F64 ? 192 : p == F32 ? 96 : 52; }
__host__ __device__ __forceinline__ int link_real_bytes(int p) { return p == F64 ? 8 : p == F32 ? 4 : 2; }

// Bytes of one gauge field (both parities, 4 directions, 12 reals per link).
__host__ __device__ __forceinline__ size_t gauge_field_bytes(int p, int Vh) {
  return (size_t)2 * 4 * 12 * padded_vh(Vh) * link_real_bytes(p);
}

// Links are tiled like spinors: [parity][tile][mu][group][site in tile], G
// groups of 16 (FP64, FP32) or 8 (16-bit) bytes per link; index in groups.
__host__ __device__ __forceinline__ size_t link_index(int par, int mu, int g, int cb, int Vh, int G) {
  const size_t ntile = padded_vh(Vh) / kSiteTile;
  return (((size_t)par * ntile + cb / kSiteTile) * 4 + mu) * (size_t)(G * kSiteTile) + (size_t)g * kSiteTile +
         (cb % kSiteTile);
}

struct Geom {
  int Lx, Ly, Lz, Lt;  // lattice extents (Lx even)
  int Lxh;             // Lx / 2
  int Vh;              // sites per parity
  int L5;
  int tap;             // 1: antiperiodic in t
  // division by Lxh, Ly, Lz as a multiply-high: q = mulhi(n, m) with
  // m = floor(2^32 / d) + 1 is exact for n * d < 2^32 (checked when the
  // action is validated); m = 0 stands for d = 1
  uint32_t mLxh, mLy, mLz;
};

__host__ __device__ __forceinline__ uint32_t fastdiv_magic(uint32_t d) {
  return d <= 1 ? 0u : (uint32_t)((1ull << 32) / d + 1ull);
}
__device__ __forceinline__ int fastdiv(int n, uint32_t m) { return m == 0 ? n : (int)__umulhi((uint32_t)n, m); }

// 4D coordinates of the site with checkerboard index cb and parity par.
__device__ __forceinline__ void site_coords(const Geom& g, int par, int cb, int& x, int& y, int& z, int& t) {
  int r = fastdiv(cb, g.mLxh);
  const int xh = cb - r * g.Lxh;
  const int r2 = fastdiv(r, g.mLy);
  y = r - r2 * g.Ly;
  t = fastdiv(r2, g.mLz);
  z = r2 - t * g.Lz;
  x = 2 * xh + ((par + y + z + t) & 1);
}

__device__ __forceinline__ int cb_index(const Geom& g, int x, int y, int z, int t) {
  return (((t * g.Lz + z) * g.Ly + y) * g.Lx + x) >> 1;
}

// Workgroups are dealt to the 8 XCDs round-robin; remap so that each XCD
// processes one contiguous range of logical blocks (neighbouring sites and
// all right-hand sides of a site stay in one XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  if (nb & 7) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Global-memory accesses.  Field pointers come out of device pointer tables,
// so the compiler cannot tell they are global; without the explicit address
// space it emits generic (flat) loads that wait on both memory counters.
// ---------------------------------------------------------------------------
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
#if defined(__HIP_DEVICE_COMPILE__)
#define MDWF_GLOBAL __attribute__((address_space(1)))
#else
#define MDWF_GLOBAL
#endif
template <class V> __device__ __forceinline__ V ldg(const void* p) { return *(const MDWF_GLOBAL V*)(p); }
// nt: a streaming (non-temporal) store, for fields the launch writes once and
// no workgroup of it reads back: it keeps the caches for the neighbour reads.
template <class V> __device__ __forceinline__ void stg(void* p, V v, bool nt = false) {
  if (nt) __builtin_nontemporal_store(v, (MDWF_GLOBAL V*)(p));
  else *(MDWF_GLOBAL V*)(p) = v;
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 sum over each 16-lane row of a wavefront with DPP moves
// (v_mov_b32_dpp on the two 32-bit halves): pairs (quad_perm 1,0,3,2),
// quads (quad_perm 2,3,0,1), half rows (row_half_mirror), rows (row_mirror).
// Every lane of a row ends with the row's sum, and each step adds two values
// that all lanes of the group already agree on, so the result equals the
// xor-butterfly over lane distances 1, 2, 4, 8 bit for bit.
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <class R> struct Cplx { R re, im; };

template <class R> __device__ __forceinline__ Cplx<R> cmul(Cplx<R> a, Cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <class R> __device__ __forceinline__ Cplx<R> cjmul(Cplx<R> a, Cplx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// ---------------------------------------------------------------------------
// 16-bit conversions (IEEE bit manipulation; round to nearest even)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_float(uint32_t bits16) { return __uint_as_float(bits16 << 16); }
__device__ __forceinline__ uint32_t float_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float f16_to_float(uint32_t bits16) {
  return __half2float(__ushort_as_half((unsigned short)bits16));
}
__device__ __forceinline__ uint32_t float_to_f16(float f) {
  return (uint32_t)__half_as_ushort(__float2half_rn(f));
}

// 16-bit fixed point on [-1, 1]: q = rint(f * 32767), f = q / 32767
__device__ __forceinline__ float i16_to_float(uint32_t bits16) {
  return (float)(int16_t)(uint16_t)bits16 * (1.0f / 32767.0f);
}
__device__ __forceinline__ uint32_t float_to_i16(float f) {
  const float c = fminf(fmaxf(f, -1.0f), 1.0f) * 32767.0f;
  return (uint32_t)(uint16_t)(int16_t)__float2int_rn(c);
}

template <int P> __device__ __forceinline__ float h_to_f(uint32_t b) {
  if constexpr (P == F16) return f16_to_float(b);
  else if constexpr (P == I16) return i16_to_float(b);
  else return bf16_to_float(b);
}
template <int P> __device__ __forceinline__ uint32_t f_to_h(float f) {
  if constexpr (P == F16) return float_to_f16(f);
  else if constexpr (P == I16) return float_to_i16(f);
  else return float_to_bf16(f);
}
template <int P> __device__ __forceinline__ void unpack2(uint32_t w, float& a, float& b) {
  a = h_to_f<P>(w & 0xffffu);
  b = h_to_f<P>(w >> 16);
}
// two values rounded to nearest-even into one 32-bit word (first value in the
// low half); F16 and BF16 use the packed conversion instructions
template <int P> __device__ __forceinline__ uint32_t pack2(float a, float b) {
  if constexpr (P == F16) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, h2{(_Float16)a, (_Float16)b});
  } else if constexpr (P == BF16) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, b2{(__bf16)a, (__bf16)b});
  } else {
    return f_to_h<P>(a) | (f_to_h<P>(b) << 16);
  }
}

// ---------------------------------------------------------------------------
// Spinor storage.  A site is 24 reals v[k], k = 2*comp + (0 re | 1 im).
// ---------------------------------------------------------------------------
struct FieldDesc {
  int Vh, L5;
};

template <int P> struct SpinorIO;

template <> struct SpinorIO<F64> {
  using R = double;
  static __device__ __forceinline__ void load(const char* base, const FieldDesc& f, int cb, int s, R v[24]) {
    const double2* p = reinterpret_cast<const double2*>(base) + tile_index(cb, s, 0, f.L5, 12);
#pragma unroll
    for (int g = 0; g < 12; ++g) {
      const v2d d = ldg<v2d>(p + (size_t)g * kSiteTile);
      v[2 * g] = d.x;
      v[2 * g + 1] = d.y;
    }
  }
  // h = 0: comps 0..5 (spins 0,1); h = 1: comps 6..11 (spins 2,3)
  static __device__ __forceinline__ void load_half(const char* base, const FieldDesc& f, int cb, int s, int h, R v[12]) {
    const double2* p = reinterpret_cast<const double2*>(base) + tile_index(cb, s, 6 * h, f.L5, 12);
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      const v2d d = ldg<v2d>(p + (size_t)g * kSiteTile);
      v[2 * g] = d.x;
      v[2 * g + 1] = d.y;
    }
  }
  static __device__ __forceinline__ void store(char* base, const FieldDesc& f, int cb, int s, const R v[24],
                                                bool nt = false) {
    double2* p = reinterpret_cast<double2*>(base) + tile_index(cb, s, 0, f.L5, 12);
#pragma unroll
    for (int g = 0; g < 12; ++g) stg<v2d>(p + (size_t)g * kSiteTile, v2d{v[2 * g], v[2 * g + 1]}, nt);
  }
};

template <> struct SpinorIO<F32> {
  using R = float;
  static __device__ __forceinline__ void load(const char* base, const FieldDesc& f, int cb, int s, R v[24]) {
    const float4* p = reinterpret_cast<const float4*>(base) + tile_index(cb, s, 0, f.L5, 6);
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      const v4f d = ldg<v4f>(p + (size_t)g * kSiteTile);
      v[4 * g] = d.x;
      v[4 * g + 1] = d.y;
      v[4 * g + 2] = d.z;
      v[4 * g + 3] = d.w;
    }
  }
  static __device__ __forceinline__ void load_half(const char* base, const FieldDesc& f, int cb, int s, int h, R v[12]) {
    const float4* p = reinterpret_cast<const float4*>(base) + tile_index(cb, s, 3 * h, f.L5, 6);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const v4f d = ldg<v4f>(p + (size_t)g * kSiteTile);
      v[4 * g] = d.x;
      v[4 * g + 1] = d.y;
      v[4 * g + 2] = d.z;
      v[4 * g + 3] = d.w;
    }
  }
  static __device__ __forceinline__ void store(char* base, const FieldDesc& f, int cb, int s, const R v[24],
                                                bool nt = false) {
    float4* p = reinterpret_cast<float4*>(base) + tile_index(cb, s, 0, f.L5, 6);
#pragma unroll
    for (int g = 0; g < 6; ++g) stg<v4f>(p + (size_t)g * kSiteTile, v4f{v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]}, nt);
  }
};

constexpr float kMinNormalF32 = 1.17549435e-38f;

template <int P> struct SpinorIO16 {
  using R = float;
  static __device__ __forceinline__ float scale(const char* base, const FieldDesc& f, int cb, int s) {
    return ldg<float>(reinterpret_cast<const float*>(base + half_scale_offset(f.L5, f.Vh)) + tile_scale_index(cb, s, f.L5));
  }
  static __device__ __forceinline__ void group(const char* base, const FieldDesc& f, int cb, int s, int g, float sc, R* v) {
    const v4u q = ldg<v4u>(reinterpret_cast<const uint4*>(base) + tile_index(cb, s, g, f.L5, 3));
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
    if constexpr (P == I16) {
      // q/32767 * sc as q * (sc/32767): one multiply per value
      const float scq = sc * (1.0f / 32767.0f);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[2 * k] = (float)(int16_t)(uint16_t)(w[k] & 0xffffu) * scq;
        v[2 * k + 1] = (float)(int16_t)(uint16_t)(w[k] >> 16) * scq;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) unpack2<P>(w[k], v[2 * k], v[2 * k + 1]);
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] *= sc;
    }
  }
  static __device__ __forceinline__ void load(const char* base, const FieldDesc& f, int cb, int s, R v[24]) {
    const float sc = scale(base, f, cb, s);
#pragma unroll
    for (int g = 0; g < 3; ++g) group(base, f, cb, s, g, sc, v + 8 * g);
  }
  // the 12 stored complex numbers as (re, im) 16-bit pairs, and the site's scale
  static __device__ __forceinline__ void load_packed(const char* base, const FieldDesc& f, int cb, int s, uint32_t q[12],
                                                     float& sc) {
    sc = scale(base, f, cb, s);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const v4u d = ldg<v4u>(reinterpret_cast<const uint4*>(base) + tile_index(cb, s, g, f.L5, 3));
      q[4 * g] = d.x;
      q[4 * g + 1] = d.y;
      q[4 * g + 2] = d.z;
      q[4 * g + 3] = d.w;
    }
  }
  static __device__ __forceinline__ void load_half(const char* base, const FieldDesc& f, int cb, int s, int h, R v[12]) {
    const float sc = scale(base, f, cb, s);
    R t[16];
    // reals 0..11 live in groups 0 and 1 (first half), reals 12..23 in group 1 (second half) and 2
    group(base, f, cb, s, h, sc, t);
    group(base, f, cb, s, h + 1, sc, t + 8);
    if (h == 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = t[k];
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = t[k + 4];
    }
  }
  static __device__ __forceinline__ void store(char* base, const FieldDesc& f, int cb, int s, const R v[24],
                                                bool nt = false) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf(v[k]));
    // a site whose largest component is below the smallest normal FP32 value
    // is stored as zero: 1/m would overflow (and 0 * inf is NaN)
    const bool keep = m >= kMinNormalF32;
    const float inv = keep ? 1.0f / m : 0.f;
    if (!keep) m = 0.f;
    uint4* p = reinterpret_cast<uint4*>(base) + tile_index(cb, s, 0, f.L5, 3);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const R* w = v + 8 * g;
      const v4u q{pack2<P>(w[0] * inv, w[1] * inv), pack2<P>(w[2] * inv, w[3] * inv),
                  pack2<P>(w[4] * inv, w[5] * inv), pack2<P>(w[6] * inv, w[7] * inv)};
      stg<v4u>(p + (size_t)g * kSiteTile, q, nt);
    }
    stg<float>(reinterpret_cast<float*>(base + half_scale_offset(f.L5, f.Vh)) + tile_scale_index(cb, s, f.L5), m, nt);
  }
};
template <> struct SpinorIO<F16> : SpinorIO16<F16> {};
template <> struct SpinorIO<BF16> : SpinorIO16<BF16> {};
template <> struct SpinorIO<I16> : SpinorIO16<I16> {};

// ---------------------------------------------------------------------------
// Gauge links: 12 stored reals, row 2 = conj(row0 x row1).
// ---------------------------------------------------------------------------
template <class R> __device__ __forceinline__ void reconstruct_row2(Cplx<R> U[3][3]) {
  // u2j = conj(u0k u1l - u0l u1k), (j,k,l) cyclic
  Cplx<R> a, b;
  a = cmul(U[0][1], U[1][2]); b = cmul(U[0][2], U[1][1]);
  U[2][0] = {a.re - b.re, -(a.im - b.im)};
  a = cmul(U[0][2], U[1][0]); b = cmul(U[0][0], U[1][2]);
  U[2][1] = {a.re - b.re, -(a.im - b.im)};
  a = cmul(U[0][0], U[1][1]); b = cmul(U[0][1], U[1][0]);
  U[2][2] = {a.re - b.re, -(a.im - b.im)};
}

// U from its 12 stored reals r = (row 0, row 1) as (re, im) pairs
template <class R> __device__ __forceinline__ void link_from_raw(const R r[12], Cplx<R> U[3][3]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) U[k / 3][k % 3] = {r[2 * k], r[2 * k + 1]};
  reconstruct_row2(U);
}

template <int P> struct LinkIO;

template <> struct LinkIO<F64> {
  using R = double;
  static __device__ __forceinline__ void load_raw(const char* gbase, int Vh, int par, int mu, int cb, R r[12]) {
    const double2* p = reinterpret_cast<const double2*>(gbase) + link_index(par, mu, 0, cb, Vh, 6);
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      const v2d d = ldg<v2d>(p + (size_t)g * kSiteTile);
      r[2 * g] = d.x;
      r[2 * g + 1] = d.y;
    }
  }
  static __device__ __forceinline__ void load(const char* gbase, int Vh, int par, int mu, int cb, Cplx<R> U[3][3]) {
    const double2* p = reinterpret_cast<const double2*>(gbase) + link_index(par, mu, 0, cb, Vh, 6);
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      const v2d d = ldg<v2d>(p + (size_t)g * kSiteTile);
      U[g / 3][g % 3] = {d.x, d.y};
    }
    reconstruct_row2(U);
  }
};

template <> struct LinkIO<F32> {
  using R = float;
  static __device__ __forceinline__ void load_raw(const char* gbase, int Vh, int par, int mu, int cb, R r[12]) {
    const float4* p = reinterpret_cast<const float4*>(gbase) + link_index(par, mu, 0, cb, Vh, 3);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const v4f d = ldg<v4f>(p + (size_t)g * kSiteTile);
      r[4 * g] = d.x; r[4 * g + 1] = d.y; r[4 * g + 2] = d.z; r[4 * g + 3] = d.w;
    }
  }
  static __device__ __forceinline__ void load(const char* gbase, int Vh, int par, int mu, int cb, Cplx<R> U[3][3]) {
    const float4* p = reinterpret_cast<const float4*>(gbase) + link_index(par, mu, 0, cb, Vh, 3);
    float r[12];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const v4f d = ldg<v4f>(p + (size_t)g * kSiteTile);
      r[4 * g] = d.x; r[4 * g + 1] = d.y; r[4 * g + 2] = d.z; r[4 * g + 3] = d.w;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) U[k / 3][k % 3] = {r[2 * k], r[2 * k + 1]};
    reconstruct_row2(U);
  }
};

template <int P> struct LinkIO16 {
  using R = float;
  static __device__ __forceinline__ void load_raw(const char* gbase, int Vh, int par, int mu, int cb, R r[12]) {
    const uint2* p = reinterpret_cast<const uint2*>(gbase) + link_index(par, mu, 0, cb, Vh, 3);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const v2u d = ldg<v2u>(p + (size_t)g * kSiteTile);
      unpack2<P>(d.x, r[4 * g], r[4 * g + 1]);
      unpack2<P>(d.y, r[4 * g + 2], r[4 * g + 3]);
    }
  }
  static __device__ __forceinline__ void load(const char* gbase, int Vh, int par, int mu, int cb, Cplx<R> U[3][3]) {
    const uint2* p = reinterpret_cast<const uint2*>(gbase) + link_index(par, mu, 0, cb, Vh, 3);
    float r[12];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const v2u d = ldg<v2u>(p + (size_t)g * kSiteTile);
      unpack2<P>(d.x, r[4 * g], r[4 * g + 1]);
      unpack2<P>(d.y, r[4 * g + 2], r[4 * g + 3]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) U[k / 3][k % 3] = {r[2 * k], r[2 * k + 1]};
    reconstruct_row2(U);
  }
};
template <> struct LinkIO<F16> : LinkIO16<F16> {};
template <> struct LinkIO<BF16> : LinkIO16<BF16> {};
template <> struct LinkIO<I16> : LinkIO16<I16> {};

// ---------------------------------------------------------------------------
// 5th-dimension coefficients of one right-hand side (built on the host).
//   M_phi = b5 + c5 P5,  M5 = alpha + beta P5,  kappa = beta / alpha,
//   M5^-1 on one chirality: y_0 = (x_0 + sum_{k>=1} (-kappa)^k (-mq) x_{L5-k}) * inv_c,
//   y_i = x_i - kappa y_{i-1}, result y * inv_alpha, inv_c = 1/(1 + mq (-kappa)^L5).
// ---------------------------------------------------------------------------
struct Coef5 {
  double b5, c5, mq, alpha, beta, kappa, inv_alpha, inv_c;
};

// CG scalars of one right-hand side, resident on the device.
struct CGState {
  int active;   // 1: iterate; 0: frozen (waiting for the host) or finished
  int flags;    // CG_FLAG_*
  int iters;
  int max_iter;
  double rho;       // |r|^2 of the current residual
  double rho_new;   // |r|^2 after the latest update
  double pq;        // <p, A p>
  double alpha, beta;
  double rmax;      // max |r| since the last reliable update
  double bb;        // |b|^2
  double tol2;      // tol^2 |b|^2
  double delta;     // reliable-update threshold (0: only at convergence)
};

enum : int {
  CG_FLAG_UPDATE = 1,     // host: recompute the FP64 residual
  CG_FLAG_BREAKDOWN = 2,  // <p, Ap> <= 0
  CG_FLAG_NAN = 4,
  CG_FLAG_MAXIT = 8,
};

}  // namespace mdwf
