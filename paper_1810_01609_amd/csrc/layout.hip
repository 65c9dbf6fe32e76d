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

// ---------------------------------------------------------------------------
// Feynman-Hellmann sequential source (user layouts, FP64).
// 4D quark field read off the walls: q = P- psi_0 + P+ psi_{L5-1}; in the
// chiral basis spins 0,1 come from slice L5-1 and spins 2,3 from slice 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_propagator_4d(Geom g, const double2* psi, double2* q) {
  const size_t V4 = (size_t)g.Vh * 2;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;  // i4 * 12 + spin * 3 + colour
  const size_t r = blockIdx.y;
  if (idx >= V4 * 12) return;
  const int spin = (int)(idx % 12) / 3;
  const int s = spin < 2 ? g.L5 - 1 : 0;
  q[r * V4 * 12 + idx] = psi[(r * g.L5 + s) * V4 * 12 + idx];
}

// eta = wall injection of Gamma q: Gamma is a signed permutation in the
// chiral basis, row a of Gamma q = i^phase[a] q[perm[a]]; eta_0 takes the P-
// spins (2,3), eta_{L5-1} the P+ spins (0,1), every other slice is zero.
struct SpinPerm {
  int perm[4];
  int phase[4];  // power of i
};

__global__ __launch_bounds__(256) void k_current_source(Geom g, SpinPerm G, const double2* q, double2* eta) {
  const size_t V4 = (size_t)g.Vh * 2;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;  // i4 * 12 + spin * 3 + colour
  const int s = blockIdx.y;
  const size_t r = blockIdx.z;
  if (idx >= V4 * 12) return;
  const size_t i4 = idx / 12;
  const int spin = (int)(idx % 12) / 3;
  const int colour = (int)(idx % 3);
  const bool wall = (s == 0 && spin >= 2) || (s == g.L5 - 1 && spin < 2);
  double2 v = make_double2(0.0, 0.0);
  if (wall) {
    const double2 x = q[r * V4 * 12 + i4 * 12 + G.perm[spin] * 3 + colour];
    switch (G.phase[spin] & 3) {
      case 0: v = x; break;
      case 1: v = make_double2(-x.y, x.x); break;   // i x
      case 2: v = make_double2(-x.x, -x.y); break;  // -x
      default: v = make_double2(x.y, -x.x); break;  // -i x
    }
  }
  eta[(r * g.L5 + s) * V4 * 12 + idx] = v;
}

// The gamma matrices (chiral DeGrand-Rossi basis, mu = x, y, z, t) as signed
// permutations: row a of g_mu has its one entry i^ph[mu][a] in column col[mu][a].
static const int kGammaCol[4][4] = {{3, 2, 1, 0}, {3, 2, 1, 0}, {2, 3, 0, 1}, {2, 3, 0, 1}};
static const int kGammaPh[4][4] = {{1, 1, 3, 3}, {2, 0, 0, 2}, {1, 3, 3, 1}, {0, 0, 0, 0}};

// Gamma = g_x^b0 g_y^b1 g_z^b2 g_t^b3 for mask = b0 + 2 b1 + 4 b2 + 8 b3.
// (A B) has row a in column colB[colA[a]] with phase phA[a] + phB[colA[a]].
static SpinPerm gamma_perm(int mask) {
  SpinPerm G;
  for (int a = 0; a < 4; ++a) {
    G.perm[a] = a;
    G.phase[a] = 0;
  }
  for (int mu = 0; mu < 4; ++mu) {
    if (!((mask >> mu) & 1)) continue;
    SpinPerm P;
    for (int a = 0; a < 4; ++a) {
      const int j = G.perm[a];
      P.perm[a] = kGammaCol[mu][j];
      P.phase[a] = (G.phase[a] + kGammaPh[mu][j]) & 3;
    }
    G = P;
  }
  return G;
}

// ---------------------------------------------------------------------------
// Source of the physical 4D propagator of the Moebius action: the 4D field
// Gamma xi enters on the walls of the opposite chirality to the read-out
// (P+ on slice 0, P- on slice L5-1) and is multiplied by the 4D factor
// (1 - c5 D_W) = beta + (c5/2) H, beta = 1 - c5 (4 - M5), that turns the
// Moebius operator into its Shamir-like form.  One thread per 4D site and
// right-hand side, FP64, user layouts; every other slice is written zero.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 times_i_pow(double2 x, int ph) {
  switch (ph & 3) {
    case 0: return x;
    case 1: return make_double2(-x.y, x.x);
    case 2: return make_double2(-x.x, -x.y);
    default: return make_double2(x.y, -x.x);
  }
}

struct GammaTab {
  int col[4][4];  // row a of g_mu has its entry i^ph[mu][a] in column col[mu][a]
  int ph[4][4];
};

// P_w Gamma xi at site i4 (w = 0: spins 0,1; w = 1: spins 2,3), 12 complex numbers
__device__ __forceinline__ void chi_at(const double2* x, size_t i4, const SpinPerm& G, int w, double2 v[12]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const bool keep = (w == 0) == (a < 2);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      v[a * 3 + c] = keep ? times_i_pow(x[i4 * 12 + G.perm[a] * 3 + c], G.phase[a]) : make_double2(0.0, 0.0);
  }
}

__global__ __launch_bounds__(128) void k_source_physical(Geom g, SpinPerm G, GammaTab T, const char* gauge,
                                                         const double2* xi, double2* eta, double beta, double hc) {
  const size_t V4 = (size_t)g.Vh * 2;
  const size_t i4 = (size_t)blockIdx.x * 128 + threadIdx.x;
  const size_t r = blockIdx.y;
  if (i4 >= V4) return;
  const double2* x = xi + r * V4 * 12;
  int X[4];
  size_t rem = i4;
  X[0] = (int)(rem % g.Lx); rem /= g.Lx;
  X[1] = (int)(rem % g.Ly); rem /= g.Ly;
  X[2] = (int)(rem % g.Lz); rem /= g.Lz;
  X[3] = (int)rem;
  const int par = (X[0] + X[1] + X[2] + X[3]) & 1;
  const int cb = (int)(i4 >> 1);
  const int Ls[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
  double2 out[2][12], v[12];
  for (int w = 0; w < 2; ++w) {
    chi_at(x, i4, G, w, v);
    for (int k = 0; k < 12; ++k) out[w][k] = make_double2(beta * v[k].x, beta * v[k].y);
  }
  for (int mu = 0; mu < 4; ++mu) {
    for (int fb = 0; fb < 2; ++fb) {
      int Y[4] = {X[0], X[1], X[2], X[3]};
      double sg = 1.0;
      if (fb == 0) {
        Y[mu] = X[mu] + 1 == Ls[mu] ? 0 : X[mu] + 1;
        if (mu == 3 && g.tap && X[3] == g.Lt - 1) sg = -1.0;
      } else {
        Y[mu] = X[mu] == 0 ? Ls[mu] - 1 : X[mu] - 1;
        if (mu == 3 && g.tap && X[3] == 0) sg = -1.0;
      }
      const size_t j4 = (((size_t)Y[3] * g.Lz + Y[2]) * g.Ly + Y[1]) * g.Lx + Y[0];
      Cplx<double> U[3][3];
      // forward: U_mu(x) on the site's own parity; backward: U_mu(x - mu)^dag
      if (fb == 0) LinkIO<F64>::load(gauge, g.Vh, par, mu, cb, U);
      else LinkIO<F64>::load(gauge, g.Vh, 1 - par, mu, (int)(j4 >> 1), U);
      const double s1 = fb == 0 ? -1.0 : 1.0;  // (1 - g_mu) forward, (1 + g_mu) backward
      for (int w = 0; w < 2; ++w) {
        chi_at(x, j4, G, w, v);
        double2 y[12];
        for (int a = 0; a < 4; ++a)
          for (int c = 0; c < 3; ++c) {
            double re = 0, im = 0;
            for (int b = 0; b < 3; ++b) {
              const Cplx<double> u = fb == 0 ? U[c][b] : Cplx<double>{U[b][c].re, -U[b][c].im};
              const double2 z = v[a * 3 + b];
              re += u.re * z.x - u.im * z.y;
              im += u.re * z.y + u.im * z.x;
            }
            y[a * 3 + c] = make_double2(re, im);
          }
        for (int a = 0; a < 4; ++a)
          for (int c = 0; c < 3; ++c) {
            const double2 gy = times_i_pow(y[T.col[mu][a] * 3 + c], T.ph[mu][a]);
            const double zr = y[a * 3 + c].x + s1 * gy.x, zi = y[a * 3 + c].y + s1 * gy.y;
            out[w][a * 3 + c].x += hc * sg * zr;
            out[w][a * 3 + c].y += hc * sg * zi;
          }
      }
    }
  }
  double2* e = eta + r * g.L5 * V4 * 12;
  for (int s = 0; s < g.L5; ++s) {
    for (int k = 0; k < 12; ++k) {
      double2 val = make_double2(0.0, 0.0);
      if (s == 0) val = out[0][k];
      if (s == g.L5 - 1) val = make_double2(val.x + out[1][k].x, val.y + out[1][k].y);
      e[((size_t)s * V4 + i4) * 12 + k] = val;
    }
  }
}

hipError_t propagator_4d(const Geom& g, int nrhs, const double* psi, double* q, hipStream_t st) {
  const size_t n = (size_t)g.Vh * 2 * 12;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)nrhs), blk(256);
  launch_k(k_propagator_4d, grid, blk, 0, st, g, reinterpret_cast<const double2*>(psi),
           reinterpret_cast<double2*>(q));
  return hipGetLastError();
}

hipError_t current_source(const Geom& g, int nrhs, int mask, const double* q, double* eta, hipStream_t st) {
  const size_t n = (size_t)g.Vh * 2 * 12;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)g.L5, (unsigned)nrhs), blk(256);
  launch_k(k_current_source, grid, blk, 0, st, g, gamma_perm(mask), reinterpret_cast<const double2*>(q),
           reinterpret_cast<double2*>(eta));
  return hipGetLastError();
}

hipError_t source_physical(const Geom& g, int nrhs, int mask, const char* gauge64, const double* xi, double* eta,
                           double beta, double hc, hipStream_t st) {
  GammaTab T;
  for (int mu = 0; mu < 4; ++mu)
    for (int a = 0; a < 4; ++a) {
      T.col[mu][a] = kGammaCol[mu][a];
      T.ph[mu][a] = kGammaPh[mu][a];
    }
  const size_t V4 = (size_t)g.Vh * 2;
  const dim3 grid((unsigned)((V4 + 127) / 128), (unsigned)nrhs), blk(128);
  launch_k(k_source_physical, grid, blk, 0, st, g, gamma_perm(mask), T, gauge64, reinterpret_cast<const double2*>(xi),
           reinterpret_cast<double2*>(eta), beta, hc);
  return hipGetLastError();
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
