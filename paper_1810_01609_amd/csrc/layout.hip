// Layout, precision and source kernels: user complex128 fields <-> internal
// half-fields, gauge compression to 12 reals, point and Z2 sources.
#include "dev_common.h"
#include "kernels.h"

namespace mdwf {

__device__ __forceinline__ int lex_index(const Geom& g, int par, int cb) {
  int x, y, z, t;
  site_coords(g, par, cb, x, y, z, t);
  return ((t * g.Lz + z) * g.Ly + y) * g.Lx + x;
}

template <int P>
__global__ __launch_bounds__(256) void k_user_to_half(Geom g, const char* const* user, char* const* half, int par) {
  using R = typename PrecTraits<P>::Real;
  const int cb = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  const int slot = blockIdx.z;
  if (cb >= g.Vh) return;
  const size_t V4 = (size_t)g.Vh * 2;
  const int i4 = lex_index(g, par, cb);
  const double2* u = reinterpret_cast<const double2*>(user[slot]) + ((size_t)s * V4 + i4) * 12;
  R v[24];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 d = u[k];
    v[2 * k] = (R)d.x;
    v[2 * k + 1] = (R)d.y;
  }
  SpinorIO<P>::store(half[slot], FieldDesc{g.Vh, g.L5}, cb, s, v);
}

template <int P>
__global__ __launch_bounds__(256) void k_half_to_user(Geom g, const char* const* half, char* const* user, int par) {
  using R = typename PrecTraits<P>::Real;
  const int cb = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  const int slot = blockIdx.z;
  if (cb >= g.Vh) return;
  const size_t V4 = (size_t)g.Vh * 2;
  const int i4 = lex_index(g, par, cb);
  double2* u = reinterpret_cast<double2*>(user[slot]) + ((size_t)s * V4 + i4) * 12;
  R v[24];
  if (half[slot] != nullptr) {
    SpinorIO<P>::load(half[slot], FieldDesc{g.Vh, g.L5}, cb, s, v);
  } else {
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) u[k] = make_double2((double)v[2 * k], (double)v[2 * k + 1]);
}

template <int P>
__global__ __launch_bounds__(256) void k_gauge(Geom g, const double* user, char* out) {
  const int cb = blockIdx.x * 256 + threadIdx.x;
  const int mu = blockIdx.y;
  const int par = blockIdx.z;
  if (cb >= g.Vh) return;
  const int i4 = lex_index(g, par, cb);
  const double* u = user + ((size_t)i4 * 4 + mu) * 18;  // rows 0,1 = 12 doubles
  if constexpr (P == F64) {
    double2* o = reinterpret_cast<double2*>(out) + link_index(par, mu, 0, cb, g.Vh, 6);
#pragma unroll
    for (int k = 0; k < 6; ++k) o[(size_t)k * kSiteTile] = make_double2(u[2 * k], u[2 * k + 1]);
  } else if constexpr (P == F32) {
    float4* o = reinterpret_cast<float4*>(out) + link_index(par, mu, 0, cb, g.Vh, 3);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      o[(size_t)k * kSiteTile] = make_float4((float)u[4 * k], (float)u[4 * k + 1], (float)u[4 * k + 2], (float)u[4 * k + 3]);
  } else {
    uint2* o = reinterpret_cast<uint2*>(out) + link_index(par, mu, 0, cb, g.Vh, 3);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint2 q;
      q.x = pack2<P>((float)u[4 * k], (float)u[4 * k + 1]);
      q.y = pack2<P>((float)u[4 * k + 2], (float)u[4 * k + 3]);
      o[(size_t)k * kSiteTile] = q;
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint4* p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}
__global__ void k_fill_zero_tail(unsigned char* p, size_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

// one thread writes the wall entries of a unit 4D point source: in the chiral
// basis P+ keeps spins 0,1 (slice L5-1), P- keeps spins 2,3 (slice 0)
__global__ void k_source_point(Geom g, double* eta, int x, int y, int z, int t, int spin, int colour) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const size_t V4 = (size_t)g.Vh * 2;
  const size_t i4 = (size_t)((t * g.Lz + z) * g.Ly + y) * g.Lx + x;
  const int s = spin < 2 ? g.L5 - 1 : 0;
  eta[(((size_t)s * V4 + i4) * 12 + spin * 3 + colour) * 2] = 1.0;
}

// SplitMix64 (Steele, Lea, Flood 2014): output number k of the generator
// seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_source_z2(Geom g, double* eta, uint64_t seed, int rhs) {
  const size_t V4 = (size_t)g.Vh * 2;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;  // (i4*4 + spin)*3 + colour
  if (idx >= V4 * 12) return;
  const size_t i4 = idx / 12;
  const int sc = (int)(idx % 12);
  const int spin = sc / 3;
  const uint64_t z = splitmix64(seed, (uint64_t)rhs * V4 * 12 + idx);
  const double r = 0.70710678118654752440;
  const double re = (z & 1) ? -r : r;
  const double im = (z & 2) ? -r : r;
  const int s = spin < 2 ? g.L5 - 1 : 0;
  double2* e = reinterpret_cast<double2*>(eta);
  e[((size_t)s * V4 + i4) * 12 + sc] = make_double2(re, im);
}

hipError_t layout_user_to_half(const Geom& g, const char* const* user, char* const* half, int par, int p,
                               int nslots, hipStream_t st) {
  const dim3 grid((g.Vh + 255) / 256, g.L5, nslots), blk(256);
  switch (p) {
    case F64: launch_k(k_user_to_half<F64>, grid, blk, 0, st, g, user, half, par); break;
    case F32: launch_k(k_user_to_half<F32>, grid, blk, 0, st, g, user, half, par); break;
    case F16: launch_k(k_user_to_half<F16>, grid, blk, 0, st, g, user, half, par); break;
    case BF16: launch_k(k_user_to_half<BF16>, grid, blk, 0, st, g, user, half, par); break;
    case I16: launch_k(k_user_to_half<I16>, grid, blk, 0, st, g, user, half, par); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t layout_half_to_user(const Geom& g, const char* const* half, char* const* user, int par, int p,
                               int nslots, hipStream_t st) {
  const dim3 grid((g.Vh + 255) / 256, g.L5, nslots), blk(256);
  switch (p) {
    case F64: launch_k(k_half_to_user<F64>, grid, blk, 0, st, g, half, user, par); break;
    case F32: launch_k(k_half_to_user<F32>, grid, blk, 0, st, g, half, user, par); break;
    case F16: launch_k(k_half_to_user<F16>, grid, blk, 0, st, g, half, user, par); break;
    case BF16: launch_k(k_half_to_user<BF16>, grid, blk, 0, st, g, half, user, par); break;
    case I16: launch_k(k_half_to_user<I16>, grid, blk, 0, st, g, half, user, par); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t layout_gauge(const Geom& g, const double* user, char* out, int p, hipStream_t st) {
  const dim3 grid((g.Vh + 255) / 256, 4, 2), blk(256);
  switch (p) {
    case F64: launch_k(k_gauge<F64>, grid, blk, 0, st, g, user, out); break;
    case F32: launch_k(k_gauge<F32>, grid, blk, 0, st, g, user, out); break;
    case F16: launch_k(k_gauge<F16>, grid, blk, 0, st, g, user, out); break;
    case BF16: launch_k(k_gauge<BF16>, grid, blk, 0, st, g, user, out); break;
    case I16: launch_k(k_gauge<I16>, grid, blk, 0, st, g, user, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fill_zero(void* ptr, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  if (n16 > 0) {
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    launch_k(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(ptr), n16);
  }
  const size_t tail = bytes - n16 * 16;
  if (tail > 0)
    launch_k(k_fill_zero_tail, dim3(1), dim3(16), 0, st,
                       reinterpret_cast<unsigned char*>(ptr) + n16 * 16, tail);
  return hipGetLastError();
}

hipError_t source_point(const Geom& g, double* eta, const int x0[4], int spin, int colour, hipStream_t st) {
  const size_t bytes = (size_t)g.Vh * 2 * g.L5 * 12 * 16;
  hipError_t e = fill_zero(eta, bytes, st);
  if (e != hipSuccess) return e;
  launch_k(k_source_point, dim3(1), dim3(64), 0, st, g, eta, x0[0], x0[1], x0[2], x0[3], spin, colour);
  return hipGetLastError();
}

hipError_t source_z2(const Geom& g, double* eta, uint64_t seed, int rhs_index, hipStream_t st) {
  const size_t V4 = (size_t)g.Vh * 2;
  const size_t bytes = V4 * g.L5 * 12 * 16;
  hipError_t e = fill_zero(eta, bytes, st);
  if (e != hipSuccess) return e;
  const size_t n = V4 * 12;
  launch_k(k_source_z2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, eta, seed, rhs_index);
  return hipGetLastError();
}

}  // namespace mdwf
