// Fused BLAS-1 updates and deterministic FP64 reductions of the CG solver.
//
// The paper ("Performance Measurement Method", Linear Solver Performance)
// counts 50-100 flops per site for these operations, i.e. they are purely
// bandwidth bound, and does every reduction in double precision.  Here each
// thread owns one 4D site and walks its L5 slices (coalesced [s][group][cb]
// accesses across the wavefront), the updates are fused so each vector is
// read and written once, and every reduction accumulates in FP64 with a
// fixed summation tree (DPP moves within each 16-lane row, shuffles across
// the four rows of a wavefront, then LDS across wavefronts, then one
// workgroup per right-hand side over the block partials), so results are
// bitwise reproducible.
#include "dev_common.h"
#include "kernels.h"

namespace mdwf {

// Sum over a 256-thread block in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v) {
  __shared__ double red[kBlasThreads / 64];
  v = row_sum16(v);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlasThreads / 64; ++w) t += red[w];
  return t;
}

// p = r + beta p on every slice of a 4D site, and pt = M_phi p from the
// new p: (M_phi p)_s = b5 p_s + c5 (P5 p)_s, P5 taking spins 0,1 from slice
// s - 1 and spins 2,3 from slice s + 1, the wall hop carrying -mq.  pt is the
// input of the first stencil launch of the next iteration, which then needs
// no fifth-dimension prologue on its eight neighbours.
template <int PS>
__global__ __launch_bounds__(kBlasThreads) void k_cg_p(BlasArgs A) {
  using RS = typename PrecTraits<PS>::Real;
  const int slot = blockIdx.y;
  const CGState& S = A.st[slot];
  if (!S.active) return;
  const int cb = blockIdx.x * kBlasThreads + threadIdx.x;
  if (cb >= A.g.Vh) return;
  const FieldDesc f{A.g.Vh, A.g.L5};
  const int L5 = A.g.L5;
  const RS beta = (RS)S.beta;
  const Coef5 c = A.coef[slot];
  const RS b5 = (RS)c.b5, c5 = (RS)c.c5, wall = (RS)(-c.c5 * c.mq);
  char* p = A.a[slot];
  const char* r = A.b[slot];
  char* pt = A.c[slot];
  RS cur[24], rv[24];
  // spins 0,1 of the new p on slice L5 - 1 feed slice 0 across the wall
  SpinorIO<PS>::load(p, f, cb, L5 - 1, cur);
  SpinorIO<PS>::load(r, f, cb, L5 - 1, rv);
  RS up[12];  // c5 (P5 p)_s, spins 0,1
#pragma unroll
  for (int k = 0; k < 12; ++k) up[k] = wall * (rv[k] + beta * cur[k]);
  RS first_dn[12], pend[24];
  for (int s = 0; s < L5; ++s) {
    SpinorIO<PS>::load(p, f, cb, s, cur);
    SpinorIO<PS>::load(r, f, cb, s, rv);
#pragma unroll
    for (int k = 0; k < 24; ++k) cur[k] = rv[k] + beta * cur[k];
    SpinorIO<PS>::store(p, f, cb, s, cur, A.nt_store);
    if (s == 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) first_dn[k] = cur[12 + k];
    } else {
      // finish pt_{s-1}: spins 2,3 take c5 p_s
#pragma unroll
      for (int k = 0; k < 12; ++k) pend[12 + k] += c5 * cur[12 + k];
      SpinorIO<PS>::store(pt, f, cb, s - 1, pend, A.nt_store);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      pend[k] = b5 * cur[k] + up[k];
      pend[12 + k] = b5 * cur[12 + k];
      up[k] = c5 * cur[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) pend[12 + k] += wall * first_dn[k];
  SpinorIO<PS>::store(pt, f, cb, L5 - 1, pend, A.nt_store);
}

template <int PI, int PO>
__global__ __launch_bounds__(kBlasThreads) void k_axpby(BlasArgs A) {
  using RI = typename PrecTraits<PI>::Real;
  using RO = typename PrecTraits<PO>::Real;
  using RC = typename PrecTraits<(PI == F64 || PO == F64) ? F64 : F32>::Real;
  const int slot = blockIdx.y;
  if (A.st != nullptr && !A.st[slot].active) return;
  const int cb = blockIdx.x * kBlasThreads + threadIdx.x;
  const FieldDesc f{A.g.Vh, A.g.L5};
  double loc = 0;
  if (cb < A.g.Vh) {
    const char* in = A.a[slot];
    char* out = A.b[slot];
    const RC ca = (RC)A.ca, cbeta = (RC)A.cb;
    for (int s = 0; s < A.g.L5; ++s) {
      RI iv[24];
      RO ov[24];
      SpinorIO<PI>::load(in, f, cb, s, iv);
      if (A.cb != 0.0) {
        SpinorIO<PO>::load(out, f, cb, s, ov);
#pragma unroll
        for (int k = 0; k < 24; ++k) ov[k] = (RO)(ca * (RC)iv[k] + cbeta * (RC)ov[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) ov[k] = (RO)(ca * (RC)iv[k]);
      }
#pragma unroll
      for (int k = 0; k < 24; ++k) loc += (double)ov[k] * (double)ov[k];
      SpinorIO<PO>::store(out, f, cb, s, ov);
    }
  }
  if (A.partials != nullptr) {
    const double t = block_sum_256(loc);
    if (threadIdx.x == 0) A.partials[(size_t)slot * A.nblk + blockIdx.x] = t;
  }
}

template <int P>
__global__ __launch_bounds__(kBlasThreads) void k_norm_diff(BlasArgs A) {
  using R = typename PrecTraits<P>::Real;
  const int slot = blockIdx.y;
  const int cb = blockIdx.x * kBlasThreads + threadIdx.x;
  const FieldDesc f{A.g.Vh, A.g.L5};
  double loc = 0;
  if (cb < A.g.Vh) {
    const char* a = A.a[slot];
    const char* b = A.b != nullptr ? A.b[slot] : nullptr;
    for (int s = 0; s < A.g.L5; ++s) {
      R av[24], bv[24];
      SpinorIO<P>::load(a, f, cb, s, av);
      if (b != nullptr) {
        SpinorIO<P>::load(b, f, cb, s, bv);
#pragma unroll
        for (int k = 0; k < 24; ++k) av[k] -= bv[k];
      }
#pragma unroll
      for (int k = 0; k < 24; ++k) loc += (double)av[k] * (double)av[k];
    }
  }
  const double t = block_sum_256(loc);
  if (threadIdx.x == 0) A.partials[(size_t)slot * A.nblk + blockIdx.x] = t;
}

int blas_nblk(const Geom& g) { return (g.Vh + kBlasThreads - 1) / kBlasThreads; }

static dim3 blas_grid(BlasArgs& A) {
  A.nblk = blas_nblk(A.g);
  return dim3(A.nblk, A.nslots);
}


hipError_t blas_cg_p(BlasArgs A, int ps, hipStream_t st) {
  const dim3 grid = blas_grid(A);
  const dim3 blk(kBlasThreads);
  switch (ps) {
    case F64: launch_k(k_cg_p<F64>, grid, blk, 0, st, A); break;
    case F32: launch_k(k_cg_p<F32>, grid, blk, 0, st, A); break;
    case F16: launch_k(k_cg_p<F16>, grid, blk, 0, st, A); break;
    case BF16: launch_k(k_cg_p<BF16>, grid, blk, 0, st, A); break;
    case I16: launch_k(k_cg_p<I16>, grid, blk, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PI>
static hipError_t axpby_out(BlasArgs A, int pout, dim3 grid, hipStream_t st) {
  const dim3 blk(kBlasThreads);
  switch (pout) {
    case F64: launch_k((k_axpby<PI, F64>), grid, blk, 0, st, A); break;
    case F32: launch_k((k_axpby<PI, F32>), grid, blk, 0, st, A); break;
    case F16: launch_k((k_axpby<PI, F16>), grid, blk, 0, st, A); break;
    case BF16: launch_k((k_axpby<PI, BF16>), grid, blk, 0, st, A); break;
    case I16: launch_k((k_axpby<PI, I16>), grid, blk, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t blas_axpby(BlasArgs A, int pin, int pout, hipStream_t st) {
  const dim3 grid = blas_grid(A);
  switch (pin) {
    case F64: return axpby_out<F64>(A, pout, grid, st);
    case F32: return axpby_out<F32>(A, pout, grid, st);
    case F16: return axpby_out<F16>(A, pout, grid, st);
    case BF16: return axpby_out<BF16>(A, pout, grid, st);
    case I16: return axpby_out<I16>(A, pout, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t blas_norm_diff(BlasArgs A, int p, hipStream_t st) {
  const dim3 grid = blas_grid(A);
  const dim3 blk(kBlasThreads);
  switch (p) {
    case F64: launch_k(k_norm_diff<F64>, grid, blk, 0, st, A); break;
    case F32: launch_k(k_norm_diff<F32>, grid, blk, 0, st, A); break;
    case F16: launch_k(k_norm_diff<F16>, grid, blk, 0, st, A); break;
    case BF16: launch_k(k_norm_diff<BF16>, grid, blk, 0, st, A); break;
    case I16: launch_k(k_norm_diff<I16>, grid, blk, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// STREAM-style copy, the achievable-bandwidth reference the stencil's HBM
// figures are read against: each thread moves four 16-byte vectors, one per
// 256-thread stride (every wavefront access is 1 KB contiguous), with
// non-temporal loads and stores (nothing is re-read).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy16(const uint4* src, uint4* dst, size_t n) {
  const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
  v4u a[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t i = base + 256 * (size_t)j;
    if (i < n) a[j] = __builtin_nontemporal_load((const MDWF_GLOBAL v4u*)(src + i));
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t i = base + 256 * (size_t)j;
    if (i < n) __builtin_nontemporal_store(a[j], (MDWF_GLOBAL v4u*)(dst + i));
  }
}

hipError_t copy16(const void* src, void* dst, size_t n16, hipStream_t st) {
  if (n16 == 0) return hipErrorInvalidValue;
  const size_t blocks = (n16 + 1023) / 1024;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  launch_k(k_copy16, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const uint4*>(src), static_cast<uint4*>(dst),
           n16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scalar kernels: one 1024-thread workgroup per right-hand side
// ---------------------------------------------------------------------------
constexpr int kScalarThreads = 1024;

// Sum of one slot's n partials in a fixed order (four independent strided
// accumulators per thread, then a fixed tree); valid in thread 0.
__device__ __forceinline__ double slot_sum(const double* partials, int n, int slot) {
  const double* q = partials + (size_t)slot * n;
  constexpr int T = kScalarThreads;
  double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
  int j = threadIdx.x;
  for (; j + 3 * T < n; j += 4 * T) {
    v0 += q[j];
    v1 += q[j + T];
    v2 += q[j + 2 * T];
    v3 += q[j + 3 * T];
  }
  for (; j < n; j += T) v0 += q[j];
  double v = (v0 + v1) + (v2 + v3);
  __shared__ double red[T / 64];
  v = row_sum16(v);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < T / 64; ++w) t += red[w];
  return t;
}

__global__ __launch_bounds__(kScalarThreads) void k_reduce(const double* partials, int n, double* out) {
  const double t = slot_sum(partials, n, blockIdx.x);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

__global__ __launch_bounds__(kScalarThreads) void k_cg_alpha(CGState* S, const double* partials, int n) {
  const int slot = blockIdx.x;
  if (!S[slot].active) return;
  const double pq = slot_sum(partials, n, slot);
  if (threadIdx.x == 0) {
    CGState& s = S[slot];
    s.pq = pq;
    if (!finite_d(pq)) {
      s.flags |= CG_FLAG_NAN;
      s.active = 0;
    } else if (!(pq > 0.0)) {
      s.flags |= CG_FLAG_BREAKDOWN;
      s.active = 0;
    } else {
      s.alpha = s.rho / pq;
    }
  }
}

__global__ __launch_bounds__(kScalarThreads) void k_cg_beta(CGState* S, const double* partials, int n) {
  const int slot = blockIdx.x;
  if (!S[slot].active) return;
  const double rr = slot_sum(partials, n, slot);
  if (threadIdx.x == 0) {
    CGState& s = S[slot];
    s.iters += 1;
    s.rho_new = rr;
    const double rn = sqrt(rr);
    if (!finite_d(rr)) {
      s.flags |= CG_FLAG_NAN;
      s.active = 0;
    } else if (rr <= s.tol2 || (s.delta > 0.0 && rn < s.delta * s.rmax)) {
      // converged in the inner precision, or the residual fell by delta:
      // the host recomputes the FP64 residual (reliable update)
      s.flags |= CG_FLAG_UPDATE;
      s.active = 0;
    } else if (s.iters >= s.max_iter) {
      s.flags |= CG_FLAG_MAXIT | CG_FLAG_UPDATE;
      s.active = 0;
    } else {
      s.beta = rr / s.rho;
      s.rho = rr;
      if (rn > s.rmax) s.rmax = rn;
    }
  }
}

hipError_t scalar_reduce(const double* partials, int n, int nslots, double* out, hipStream_t st) {
  launch_k(k_reduce, dim3(nslots), dim3(kScalarThreads), 0, st, partials, n, out);
  return hipGetLastError();
}
hipError_t scalar_cg_alpha(CGState* S, const double* partials, int n, int nslots, hipStream_t st) {
  launch_k(k_cg_alpha, dim3(nslots), dim3(kScalarThreads), 0, st, S, partials, n);
  return hipGetLastError();
}
hipError_t scalar_cg_beta(CGState* S, const double* partials, int n, int nslots, hipStream_t st) {
  launch_k(k_cg_beta, dim3(nslots), dim3(kScalarThreads), 0, st, S, partials, n);
  return hipGetLastError();
}

}  // namespace mdwf
