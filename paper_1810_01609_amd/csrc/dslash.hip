// Fused domain-wall stencil kernel for gfx950.
//
// One workgroup owns CB consecutive sites of the output parity and all L5
// fifth-dimension slices of them: thread (cbl, s) computes the 4D Wilson hop
// on slice s of site cbl (spin projection to half-spinors, SU(3) x two colour
// vectors, reconstruction, 8 directions), with the links rebuilt from 12
// stored reals.  The site-local 5th-dimension operators M_phi, M5, M5^-1
// (and transposes) that surround the hop in the even-odd operator are fused
// as a prologue (M_phi on the input, applied while loading neighbours) and
// as epilogue chains that run in LDS on whole fifth-dimension columns.  The
// xpay of M^ = 1 - (...) and the |.|^2 reduction CG needs are fused too.
// Fusing these steps into one pass over the fields, with the operator never
// stored as a matrix, is the approach the paper's performance discussion
// takes for this operator (Current State of the Art, Performance related).
#include "dev_common.h"
#include "kernels.h"

#include <algorithm>

namespace mdwf {

// One LDS row per site, so a thread's reads are its row base plus immediate
// offsets; odd row strides keep consecutive sites on distinct banks.
constexpr int kStageLinkStride = 8 * 18 + 1;  // link reals per site row
constexpr int kStageNbrStride = 9;            // neighbour indices per site row

// ---------------------------------------------------------------------------
// spin projection.  h = spins 0,1 of (1 + SIG g_mu) psi; with w = U h the
// spins 2,3 of the result follow from w (chiral DeGrand-Rossi basis):
//   x: r2 = -SIG i w1, r3 = -SIG i w0     y: r2 =  SIG w1, r3 = -SIG w0
//   z: r2 = -SIG i w0, r3 =  SIG i w1     t: r2 =  SIG w0, r3 =  SIG w1
// ---------------------------------------------------------------------------
template <class R> __device__ __forceinline__ Cplx<R> add(Cplx<R> a, Cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ __forceinline__ Cplx<R> sub(Cplx<R> a, Cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
// a + sg * i * b
template <class R> __device__ __forceinline__ Cplx<R> addi(Cplx<R> a, Cplx<R> b, int sg) {
  return sg > 0 ? Cplx<R>{a.re - b.im, a.im + b.re} : Cplx<R>{a.re + b.im, a.im - b.re};
}

// the same operations on packed 16-bit (re, im) pairs, each result rounded
// once to the storage format
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f16x2 add(f16x2 a, f16x2 b) { return a + b; }
__device__ __forceinline__ f16x2 sub(f16x2 a, f16x2 b) { return a - b; }
__device__ __forceinline__ f16x2 addi(f16x2 a, f16x2 b, int sg) {
  return sg > 0 ? a + f16x2{-b.y, b.x} : a + f16x2{b.y, -b.x};
}
__device__ __forceinline__ bf16x2 add(bf16x2 a, bf16x2 b) { return a + b; }
__device__ __forceinline__ bf16x2 sub(bf16x2 a, bf16x2 b) { return a - b; }
__device__ __forceinline__ bf16x2 addi(bf16x2 a, bf16x2 b, int sg) {
  return sg > 0 ? a + bf16x2{-b.y, b.x} : a + bf16x2{b.y, -b.x};
}

template <int MU, int SIG, class C>
__device__ __forceinline__ void project(const C p[4][3], C h[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (MU == 0) {  // g_x psi = (i p3, i p2, -i p1, -i p0)
      h[0][c] = addi(p[0][c], p[3][c], SIG);
      h[1][c] = addi(p[1][c], p[2][c], SIG);
    } else if constexpr (MU == 1) {  // g_y psi = (-p3, p2, p1, -p0)
      h[0][c] = SIG > 0 ? sub(p[0][c], p[3][c]) : add(p[0][c], p[3][c]);
      h[1][c] = SIG > 0 ? add(p[1][c], p[2][c]) : sub(p[1][c], p[2][c]);
    } else if constexpr (MU == 2) {  // g_z psi = (i p2, -i p3, -i p0, i p1)
      h[0][c] = addi(p[0][c], p[2][c], SIG);
      h[1][c] = addi(p[1][c], p[3][c], -SIG);
    } else {  // g_t psi = (p2, p3, p0, p1)
      h[0][c] = SIG > 0 ? add(p[0][c], p[2][c]) : sub(p[0][c], p[2][c]);
      h[1][c] = SIG > 0 ? add(p[1][c], p[3][c]) : sub(p[1][c], p[3][c]);
    }
  }
}

template <int MU, int SIG, class R>
__device__ __forceinline__ void accumulate(Cplx<R> acc[4][3], const Cplx<R> w[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] = add(acc[0][c], w[0][c]);
    acc[1][c] = add(acc[1][c], w[1][c]);
    if constexpr (MU == 0) {
      acc[2][c] = addi(acc[2][c], w[1][c], -SIG);
      acc[3][c] = addi(acc[3][c], w[0][c], -SIG);
    } else if constexpr (MU == 1) {
      acc[2][c] = SIG > 0 ? add(acc[2][c], w[1][c]) : sub(acc[2][c], w[1][c]);
      acc[3][c] = SIG > 0 ? sub(acc[3][c], w[0][c]) : add(acc[3][c], w[0][c]);
    } else if constexpr (MU == 2) {
      acc[2][c] = addi(acc[2][c], w[0][c], -SIG);
      acc[3][c] = addi(acc[3][c], w[1][c], SIG);
    } else {
      acc[2][c] = SIG > 0 ? add(acc[2][c], w[0][c]) : sub(acc[2][c], w[0][c]);
      acc[3][c] = SIG > 0 ? add(acc[3][c], w[1][c]) : sub(acc[3][c], w[1][c]);
    }
  }
}

// acc += sc * (spin reconstruction of w): the accumulate above with the
// neighbour's per-site scale applied in the FP32 sum
template <int MU, int SIG>
__device__ __forceinline__ void accumulate_scaled(Cplx<float> acc[4][3], const Cplx<float> w[2][3], float sc) {
  const float ps = SIG > 0 ? sc : -sc;  // +SIG*sc
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] = {fmaf(sc, w[0][c].re, acc[0][c].re), fmaf(sc, w[0][c].im, acc[0][c].im)};
    acc[1][c] = {fmaf(sc, w[1][c].re, acc[1][c].re), fmaf(sc, w[1][c].im, acc[1][c].im)};
    if constexpr (MU == 0) {  // acc2 += -SIG i w1, acc3 += -SIG i w0
      acc[2][c] = {fmaf(ps, w[1][c].im, acc[2][c].re), fmaf(-ps, w[1][c].re, acc[2][c].im)};
      acc[3][c] = {fmaf(ps, w[0][c].im, acc[3][c].re), fmaf(-ps, w[0][c].re, acc[3][c].im)};
    } else if constexpr (MU == 1) {  // acc2 += SIG w1, acc3 -= SIG w0
      acc[2][c] = {fmaf(ps, w[1][c].re, acc[2][c].re), fmaf(ps, w[1][c].im, acc[2][c].im)};
      acc[3][c] = {fmaf(-ps, w[0][c].re, acc[3][c].re), fmaf(-ps, w[0][c].im, acc[3][c].im)};
    } else if constexpr (MU == 2) {  // acc2 += -SIG i w0, acc3 += SIG i w1
      acc[2][c] = {fmaf(ps, w[0][c].im, acc[2][c].re), fmaf(-ps, w[0][c].re, acc[2][c].im)};
      acc[3][c] = {fmaf(-ps, w[1][c].im, acc[3][c].re), fmaf(ps, w[1][c].re, acc[3][c].im)};
    } else {  // acc2 += SIG w0, acc3 += SIG w1
      acc[2][c] = {fmaf(ps, w[0][c].re, acc[2][c].re), fmaf(ps, w[0][c].im, acc[2][c].im)};
      acc[3][c] = {fmaf(ps, w[1][c].re, acc[3][c].re), fmaf(ps, w[1][c].im, acc[3][c].im)};
    }
  }
}

// w = U h (fwd) or U^dag h (bwd), two colour vectors.  Each row is one
// multiply-add chain per real and imaginary part (4 FMAs per complex product
// after the first), not products rounded and then added.
template <bool ADJ, class R>
__device__ __forceinline__ void colour_mul(const Cplx<R> U[3][3], const Cplx<R> h[2][3], Cplx<R> w[2][3]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R re = 0, im = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const Cplx<R> u = ADJ ? U[b][a] : U[a][b];
        const Cplx<R> x = h[k][b];
        if (b == 0) {
          re = u.re * x.re;
          im = u.re * x.im;
        } else {
          re = u.re * x.re + re;
          im = u.re * x.im + im;
        }
        if constexpr (ADJ) {  // conj(u) x
          re = u.im * x.im + re;
          im = im - u.im * x.re;
        } else {
          re = re - u.im * x.im;
          im = u.im * x.re + im;
        }
      }
      w[k][a] = {re, im};
    }
  }
}

// ---------------------------------------------------------------------------
// Packed 16-bit hop (F16 and BF16 storage).  A neighbour's 12 complex numbers
// stay in their stored (re, im) 16-bit pairs; the spin projection is formed on
// the pairs (its sum rounded once to the storage format) and the colour
// product uses dot2 instructions, whose 16 x 16-bit products are exact in FP32
// and are summed in FP32.  The neighbour's per-site scale enters in the FP32
// accumulation.  The staged link of a direction is V = U (forward) or U^dag
// (backward), with the antiperiodic sign, as two pairs per entry:
// (Re V, -Im V) and (Im V, Re V), so Re(V h) and Im(V h) are plain dot2 sums.
// ---------------------------------------------------------------------------

template <int P> struct Packed {
  static constexpr bool enabled = false;
};
template <> struct Packed<F16> {
  static constexpr bool enabled = true;
  using T2 = f16x2;
  static __device__ __forceinline__ float dot(T2 a, T2 b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }
  // the first product of a chain: the three-operand form with a zero addend
  // (the builtin becomes a register clear plus the accumulating form)
  static __device__ __forceinline__ float dot0(T2 a, T2 b) {
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
  }
  static __device__ __forceinline__ T2 make(float re, float im) { return T2{(_Float16)re, (_Float16)im}; }
};
template <> struct Packed<BF16> {
  static constexpr bool enabled = true;
  using T2 = bf16x2;
  static __device__ __forceinline__ float dot(T2 a, T2 b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(a, b, c, false);
  }
  static __device__ __forceinline__ float dot0(T2 a, T2 b) {
    float r;
    asm("v_dot2_f32_bf16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
  }
  static __device__ __forceinline__ T2 make(float re, float im) { return T2{(__bf16)re, (__bf16)im}; }
};

// w = V h for the two projected colour vectors, V from the packed stage
template <int P>
__device__ __forceinline__ void colour_mul_packed(const uint32_t* lnk, int dir, int CB, int cbl,
                                                  const typename Packed<P>::T2 h[2][3], Cplx<float> w[2][3]) {
  using K = Packed<P>;
  using T2 = typename K::T2;
  const uint32_t* row = lnk + cbl * kStageLinkStride + dir * 18;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T2 p1[3], p2[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      p1[b] = __builtin_bit_cast(T2, row[2 * (a * 3 + b)]);
      p2[b] = __builtin_bit_cast(T2, row[2 * (a * 3 + b) + 1]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      w[k][a].re = K::dot(p1[2], h[k][2], K::dot(p1[1], h[k][1], K::dot0(p1[0], h[k][0])));
      w[k][a].im = K::dot(p2[2], h[k][2], K::dot(p2[1], h[k][1], K::dot0(p2[0], h[k][0])));
    }
  }
}

// a*x_s + b*(P5 x)_s (dag = 0) or a*x_s + b*(P5^T x)_s (dag = 1), loaded from
// one site's fifth-dimension column.  P5: spins 0,1 from s-1, spins 2,3 from
// s+1; P5^T the other way round; the wall hop carries -mq.
template <int P>
__device__ __forceinline__ void load_bidiag(const char* base, const FieldDesc& f, int cb, int s, int L5,
                                   typename PrecTraits<P>::Real a, typename PrecTraits<P>::Real b,
                                   typename PrecTraits<P>::Real mq, bool dag,
                                   typename PrecTraits<P>::Real v[24]) {
  using R = typename PrecTraits<P>::Real;
  SpinorIO<P>::load(base, f, cb, s, v);
  int s_up = dag ? s + 1 : s - 1;  // source slice of spins 0,1
  int s_dn = dag ? s - 1 : s + 1;  // source slice of spins 2,3
  R b_up = b, b_dn = b;
  if (s_up < 0) { s_up = L5 - 1; b_up = -b * mq; }
  if (s_up >= L5) { s_up = 0; b_up = -b * mq; }
  if (s_dn < 0) { s_dn = L5 - 1; b_dn = -b * mq; }
  if (s_dn >= L5) { s_dn = 0; b_dn = -b * mq; }
  R u[12], d[12];
  SpinorIO<P>::load_half(base, f, cb, s_up, 0, u);
  SpinorIO<P>::load_half(base, f, cb, s_dn, 1, d);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[k] = a * v[k] + b_up * u[k];
    v[12 + k] = a * v[12 + k] + b_dn * d[k];
  }
}

// Compiler fence that also pins the accumulator: the arithmetic of one
// direction must be finished before the next direction's loads are issued,
// so at most one neighbour's spinor and link are live in registers.
template <class R>
__device__ __forceinline__ void pin_acc(Cplx<R> acc[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
    asm volatile("" : "+v"(acc[a][0].re), "+v"(acc[a][0].im), "+v"(acc[a][1].re), "+v"(acc[a][1].im),
                 "+v"(acc[a][2].re), "+v"(acc[a][2].im) : : "memory");
}

// Per-workgroup staging of the stencil's geometry and links in LDS: for each
// of the CB sites and 8 directions (mu forward 0..3, backward 4..7) the
// neighbour's index and the full 3x3 link (row 2 rebuilt once here instead of
// once per slice thread), loaded once and shared by the site's L5 slice
// threads.  A hop across the antiperiodic t boundary carries its -1 in the
// staged link: U(-h) and (-U)h round identically.
template <class R> struct Stage {
  int* nbr;  // [CB][9]: dir
  R* lnk;    // [CB][145]: dir * 18 + 2 * (3a + b) + (re | im)
};

template <class R>
__device__ __forceinline__ void stage_link(const Stage<R>& st, int dir, int CB, int cbl, Cplx<R> U[3][3]) {
  const R* row = st.lnk + cbl * kStageLinkStride + dir * 18;
#pragma unroll
  for (int k = 0; k < 9; ++k) U[k / 3][k % 3] = {row[2 * k], row[2 * k + 1]};
}
__device__ __forceinline__ int stage_nbr(const int* nbr, int dir, int cbl) { return nbr[cbl * kStageNbrStride + dir]; }
__host__ __device__ __forceinline__ size_t stage_nbr_bytes(int CB) {
  return round_up((size_t)CB * kStageNbrStride * sizeof(int), 16);
}

// SPLIT: a hop across the boundary of a split dimension is staged with
// neighbour index -1 (and a zero link); the hop skips it.
template <int P, bool SPLIT>
__device__ __forceinline__ void stage_fill(const DslashArgs& A, Stage<typename PrecTraits<P>::Real> st, int CB,
                                           int cb_log2, int cb0, int tid, int nthr) {
  using R = typename PrecTraits<P>::Real;
  const Geom& g = A.g;
  for (int task = tid; task < CB * 8; task += nthr) {
    const int cbl = task & (CB - 1);
    const int dir = task >> cb_log2;
    const int cb = cb0 + cbl;
    int nb = 0;
    R r[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) r[k] = 0;
    bool flip = false;
    if (cb < g.Vh) {
      int X[4];
      site_coords(g, A.out_par, cb, X[0], X[1], X[2], X[3]);
      const int mu = dir & 3;
      const int Lmu = mu == 0 ? g.Lx : mu == 1 ? g.Ly : mu == 2 ? g.Lz : g.Lt;
      const bool cut = SPLIT && ((A.split_mask >> mu) & 1) && (dir < 4 ? X[mu] + 1 == Lmu : X[mu] == 0);
      if (cut) {
        nb = -1;
      } else if (dir < 4) {
        flip = mu == 3 && g.tap && X[3] == g.Lt - 1;
        X[mu] = X[mu] + 1 == Lmu ? 0 : X[mu] + 1;
        nb = cb_index(g, X[0], X[1], X[2], X[3]);
        LinkIO<P>::load_raw(A.gauge, g.Vh, A.out_par, mu, cb, r);
      } else {
        flip = mu == 3 && g.tap && X[3] == 0;
        X[mu] = X[mu] == 0 ? Lmu - 1 : X[mu] - 1;
        nb = cb_index(g, X[0], X[1], X[2], X[3]);
        LinkIO<P>::load_raw(A.gauge, g.Vh, 1 - A.out_par, mu, nb, r);
      }
    }
    Cplx<R> U[3][3];
    link_from_raw(r, U);
    const R sg = flip ? R(-1) : R(1);
    st.nbr[cbl * kStageNbrStride + dir] = nb;
    R* row = st.lnk + cbl * kStageLinkStride + dir * 18;
    if constexpr (Packed<P>::enabled) {
      // V = U or U^dag as the pairs (Re V, -Im V), (Im V, Re V)
      using K = Packed<P>;
      uint32_t* pk = reinterpret_cast<uint32_t*>(row);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int a = k / 3, b = k % 3;
        const Cplx<R> u = dir < 4 ? U[a][b] : Cplx<R>{U[b][a].re, -U[b][a].im};
        const R vr = sg * u.re, vi = sg * u.im;
        pk[2 * k] = __builtin_bit_cast(uint32_t, K::make(vr, -vi));
        pk[2 * k + 1] = __builtin_bit_cast(uint32_t, K::make(vi, vr));
      }
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        row[2 * k] = sg * U[k / 3][k % 3].re;
        row[2 * k + 1] = sg * U[k / 3][k % 3].im;
      }
    }
  }
}

// load_bidiag (dag = 0) for 16-bit storage, with the three sites' scales
// divided by their maximum m, which is returned: the combination stays O(1)
// whatever the field's magnitude, so it can be rounded back to 16 bits.
template <int P>
__device__ __forceinline__ float load_bidiag_norm(const char* base, const FieldDesc& f, int cb, int s, int L5, float a,
                                                  float b, float mq, float v[24]) {
  int s_up = s - 1, s_dn = s + 1;
  float b_up = b, b_dn = b;
  if (s_up < 0) { s_up = L5 - 1; b_up = -b * mq; }
  if (s_dn >= L5) { s_dn = 0; b_dn = -b * mq; }
  using IO = SpinorIO<P>;
  const float c0 = IO::scale(base, f, cb, s), cu = IO::scale(base, f, cb, s_up), cd = IO::scale(base, f, cb, s_dn);
  const float m = fmaxf(c0, fmaxf(cu, cd));
  const float im = m >= kMinNormalF32 ? 1.0f / m : 0.f;  // stored scales are 0 or normal
#pragma unroll
  for (int g = 0; g < 3; ++g) IO::group(base, f, cb, s, g, a * c0 * im, v + 8 * g);
  float t[16];
  IO::group(base, f, cb, s_up, 0, b_up * cu * im, t);
  IO::group(base, f, cb, s_up, 1, b_up * cu * im, t + 8);
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] += t[k];
  IO::group(base, f, cb, s_dn, 1, b_dn * cd * im, t);
  IO::group(base, f, cb, s_dn, 2, b_dn * cd * im, t + 8);
#pragma unroll
  for (int k = 0; k < 12; ++k) v[12 + k] += t[4 + k];
  return m;
}

template <int P, bool DAG, bool PRO, int MU, bool SPLIT>
__device__ __forceinline__ void hop_dir_packed(const DslashArgs& A, const FieldDesc& f, const char* in, int s,
                                               const Coef5& c, Cplx<float> acc[4][3], Stage<float> st, int CB,
                                               int cbl) {
  using K = Packed<P>;
  using T2 = typename K::T2;
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  const uint32_t* lnk = reinterpret_cast<const uint32_t*>(st.lnk);
#pragma unroll
  for (int fb = 0; fb < 2; ++fb) {
    const int nb = stage_nbr(st.nbr, MU + 4 * fb, cbl);
    if constexpr (SPLIT) {
      if (nb < 0) continue;
    }
    T2 h[2][3];
    float sc;
    if constexpr (PRO) {
      float v[24];
      sc = load_bidiag_norm<P>(in, f, nb, s, A.g.L5, (float)c.b5, (float)c.c5, (float)c.mq, v);
      Cplx<float> pf[4][3], hf[2][3];
#pragma unroll
      for (int k = 0; k < 12; ++k) pf[k / 3][k % 3] = {v[2 * k], v[2 * k + 1]};
      if (fb == 0) project<MU, SF>(pf, hf);
      else project<MU, SB>(pf, hf);
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[k][a] = K::make(hf[k][a].re, hf[k][a].im);
    } else {
      uint32_t q[12];
      SpinorIO<P>::load_packed(in, f, nb, s, q, sc);
      T2 psi[4][3];
#pragma unroll
      for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = __builtin_bit_cast(T2, q[k]);
      if (fb == 0) project<MU, SF>(psi, h);
      else project<MU, SB>(psi, h);
    }
    Cplx<float> w[2][3];
    colour_mul_packed<P>(lnk, MU + 4 * fb, CB, cbl, h, w);
    if (fb == 0) accumulate_scaled<MU, SF>(acc, w, sc);
    else accumulate_scaled<MU, SB>(acc, w, sc);
    pin_acc(acc);
  }
}

template <int P, bool DAG, bool PRO, bool STAGE, int MU, bool SPLIT>
__device__ __forceinline__ void hop_dir_single(const DslashArgs& A, const FieldDesc& f, const char* in, int cb, int s,
                                        const int X[4], const Coef5& c, Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                        Stage<typename PrecTraits<P>::Real> st, int CB, int cbl) {
  using R = typename PrecTraits<P>::Real;
  const Geom& g = A.g;
  const int Lmu = MU == 0 ? g.Lx : MU == 1 ? g.Ly : MU == 2 ? g.Lz : g.Lt;
  constexpr int SF = DAG ? +1 : -1;  // forward projector 1 + SF g_mu
  constexpr int SB = -SF;            // backward projector
  Cplx<R> U[3][3], psi[4][3], h[2][3], w[2][3];
  R v[24];
#pragma unroll
  for (int fb = 0; fb < 2; ++fb) {
    // fb = 0 forward: (1 -+ g) U_mu(x) psi(x + mu); fb = 1 backward: (1 +- g) U_mu(x - mu)^dag psi(x - mu)
    int nb;
    bool flip;
    if constexpr (STAGE) {
      nb = stage_nbr(st.nbr, MU + 4 * fb, cbl);
      if constexpr (SPLIT) {
        if (nb < 0) continue;
      }
      flip = false;  // carried by the staged link
      stage_link(st, MU + 4 * fb, CB, cbl, U);
    } else {
      int Y[4] = {X[0], X[1], X[2], X[3]};
      if (fb == 0) {
        Y[MU] = X[MU] + 1 == Lmu ? 0 : X[MU] + 1;
        flip = MU == 3 && g.tap && X[3] == g.Lt - 1;
      } else {
        Y[MU] = X[MU] == 0 ? Lmu - 1 : X[MU] - 1;
        flip = MU == 3 && g.tap && X[3] == 0;
      }
      nb = cb_index(g, Y[0], Y[1], Y[2], Y[3]);
      if (fb == 0) LinkIO<P>::load(A.gauge, g.Vh, A.out_par, MU, cb, U);
      else LinkIO<P>::load(A.gauge, g.Vh, 1 - A.out_par, MU, nb, U);
    }
    // int16 storage: the stored integers enter the projection and the colour
    // product unscaled; the site's scale (and 1/32767) joins in the
    // accumulation, one multiply-add per result instead of one multiply per
    // loaded value
    constexpr bool kI16Raw = P == I16 && STAGE && !PRO;
    float sc16 = 1.f;
    if constexpr (kI16Raw) {
      uint32_t q[12];
      SpinorIO<P>::load_packed(in, f, nb, s, q, sc16);
      sc16 *= 1.0f / 32767.0f;
#pragma unroll
      for (int k = 0; k < 12; ++k)
        psi[k / 3][k % 3] = {(R)(int16_t)(uint16_t)(q[k] & 0xffffu), (R)(int16_t)(uint16_t)(q[k] >> 16)};
    } else {
      if constexpr (PRO) load_bidiag<P>(in, f, nb, s, g.L5, (R)c.b5, (R)c.c5, (R)c.mq, false, v);
      else SpinorIO<P>::load(in, f, nb, s, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = {v[2 * k], v[2 * k + 1]};
    }
    if (fb == 0) project<MU, SF>(psi, h);
    else project<MU, SB>(psi, h);
    if (flip) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[k][a] = {-h[k][a].re, -h[k][a].im};
    }
    if (fb == 0) colour_mul<false>(U, h, w);
    else colour_mul<true>(U, h, w);
    if constexpr (kI16Raw) {
      if (fb == 0) accumulate_scaled<MU, SF>(acc, w, sc16);
      else accumulate_scaled<MU, SB>(acc, w, sc16);
    } else {
      if (fb == 0) accumulate<MU, SF>(acc, w);
      else accumulate<MU, SB>(acc, w);
    }
    pin_acc(acc);
  }
}


// ---------------------------------------------------------------------------
// The staged hop with the neighbour loads of NB directions issued together:
// the eight directions (mu-major, forward then backward, the order of the
// one-at-a-time form, so the sums round identically) are taken in batches of
// NB; a batch first loads its NB neighbours (NB loads in flight per thread),
// then projects, multiplies and accumulates them one by one.  Used for the
// staged hop without the M_phi prologue.
// ---------------------------------------------------------------------------
template <int P> struct NbrLoad {
  using R = typename PrecTraits<P>::Real;
  // 16-bit storage keeps the stored pairs and the scale
  static constexpr bool kRaw = Packed<P>::enabled || P == I16;
  uint32_t q[kRaw ? 12 : 1];
  R v[kRaw ? 1 : 24];
  float sc;
  bool skip;
};

template <int P, bool SPLIT, int D>
__device__ __forceinline__ void nbr_load(const FieldDesc& f, const char* in, int s, const int* nbr, int cbl,
                                         NbrLoad<P>& n) {
  constexpr int MU = D / 2, FB = D % 2;
  const int nb = stage_nbr(nbr, MU + 4 * FB, cbl);
  n.skip = SPLIT && nb < 0;
  n.sc = 1.f;
  if (n.skip) return;
  if constexpr (NbrLoad<P>::kRaw) SpinorIO<P>::load_packed(in, f, nb, s, n.q, n.sc);
  else SpinorIO<P>::load(in, f, nb, s, n.v);
}

// Compiler fence after a batch's loads: every loaded register passes through
// an empty asm, so no load of the batch can sink below it and no arithmetic
// of the batch can rise above it.
template <class T, int N> __device__ __forceinline__ void pin_regs(T (&v)[N]) {
#pragma unroll
  for (int k = 0; k + 3 < N; k += 4) asm volatile("" : "+v"(v[k]), "+v"(v[k + 1]), "+v"(v[k + 2]), "+v"(v[k + 3]) : : "memory");
  if constexpr (N % 4 != 0) {
#pragma unroll
    for (int k = N - N % 4; k < N; ++k) asm volatile("" : "+v"(v[k]) : : "memory");
  }
}
template <int P> __device__ __forceinline__ void pin_load(NbrLoad<P>& n) {
  if constexpr (NbrLoad<P>::kRaw) pin_regs(n.q);
  else pin_regs(n.v);
  asm volatile("" : "+v"(n.sc) : : "memory");
}

template <int P, bool DAG, int D>
__device__ __forceinline__ void nbr_compute(const Stage<typename PrecTraits<P>::Real>& st, int CB, int cbl,
                                            const NbrLoad<P>& n, Cplx<typename PrecTraits<P>::Real> acc[4][3]) {
  using R = typename PrecTraits<P>::Real;
  constexpr int MU = D / 2, FB = D % 2;
  constexpr int SG = (FB == 0) == DAG ? +1 : -1;  // projector 1 + SG g_mu
  if (n.skip) return;
  if constexpr (Packed<P>::enabled) {
    using K = Packed<P>;
    using T2 = typename K::T2;
    T2 psi[4][3], h[2][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = __builtin_bit_cast(T2, n.q[k]);
    project<MU, SG>(psi, h);
    Cplx<float> w[2][3];
    colour_mul_packed<P>(reinterpret_cast<const uint32_t*>(st.lnk), MU + 4 * FB, CB, cbl, h, w);
    accumulate_scaled<MU, SG>(acc, w, n.sc);
  } else {
    Cplx<R> U[3][3], psi[4][3], h[2][3], w[2][3];
    stage_link(st, MU + 4 * FB, CB, cbl, U);
    if constexpr (NbrLoad<P>::kRaw) {  // int16: unscaled integers, the scale joins the accumulation
#pragma unroll
      for (int k = 0; k < 12; ++k)
        psi[k / 3][k % 3] = {(R)(int16_t)(uint16_t)(n.q[k] & 0xffffu), (R)(int16_t)(uint16_t)(n.q[k] >> 16)};
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = {n.v[2 * k], n.v[2 * k + 1]};
    }
    project<MU, SG>(psi, h);
    colour_mul<FB == 1>(U, h, w);
    if constexpr (NbrLoad<P>::kRaw) accumulate_scaled<MU, SG>(acc, w, n.sc * (1.0f / 32767.0f));
    else accumulate<MU, SG>(acc, w);
  }
}

template <int P, bool DAG, bool SPLIT, int D, int END> struct HopBatch {
  static __device__ __forceinline__ void load(const FieldDesc& f, const char* in, int s, const int* nbr, int cbl,
                                              NbrLoad<P>* n) {
    if constexpr (D < END) {
      nbr_load<P, SPLIT, D>(f, in, s, nbr, cbl, n[0]);
      HopBatch<P, DAG, SPLIT, D + 1, END>::load(f, in, s, nbr, cbl, n + 1);
    }
  }
  static __device__ __forceinline__ void compute(const Stage<typename PrecTraits<P>::Real>& st, int CB, int cbl,
                                                 const NbrLoad<P>* n, Cplx<typename PrecTraits<P>::Real> acc[4][3]) {
    if constexpr (D < END) {
      nbr_compute<P, DAG, D>(st, CB, cbl, n[0], acc);
      HopBatch<P, DAG, SPLIT, D + 1, END>::compute(st, CB, cbl, n + 1, acc);
    }
  }
};

template <int P, bool DAG, bool SPLIT, int NB, int B0>
__device__ __forceinline__ void hop_batches(const FieldDesc& f, const char* in, int s,
                                            Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                            const Stage<typename PrecTraits<P>::Real>& st, int CB, int cbl) {
  if constexpr (B0 < 8) {
    NbrLoad<P> n[NB];
    HopBatch<P, DAG, SPLIT, B0, B0 + NB>::load(f, in, s, st.nbr, cbl, n);
#pragma unroll
    for (int j = 0; j < NB; ++j) pin_load(n[j]);
    HopBatch<P, DAG, SPLIT, B0, B0 + NB>::compute(st, CB, cbl, n, acc);
    pin_acc(acc);
    hop_batches<P, DAG, SPLIT, NB, B0 + NB>(f, in, s, acc, st, CB, cbl);
  }
}

// Neighbours loaded together per thread (0: the one-at-a-time form) in the
// staged hop without the M_phi prologue; the build options MDWF_HOP_BATCH and
// MDWF_HOP_BATCH_CGU (launches with the fused CG update) set it.  FP64 stays
// at one.
#ifndef MDWF_HOP_BATCH
#define MDWF_HOP_BATCH 2
#endif
#ifndef MDWF_HOP_BATCH_CGU
#define MDWF_HOP_BATCH_CGU 0
#endif
template <int P, bool PRO, bool CGU> constexpr int kHopBatch =
    (P == F64 || PRO) ? 0 : CGU ? MDWF_HOP_BATCH_CGU : MDWF_HOP_BATCH;

template <int P, bool DAG, bool PRO, bool STAGE, int MU, bool SPLIT>
__device__ __forceinline__ void hop_dir(const DslashArgs& A, const FieldDesc& f, const char* in, int cb, int s,
                                        const int X[4], const Coef5& c, Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                        Stage<typename PrecTraits<P>::Real> st, int CB, int cbl) {
  if constexpr (STAGE && Packed<P>::enabled) hop_dir_packed<P, DAG, PRO, MU, SPLIT>(A, f, in, s, c, acc, st, CB, cbl);
  else hop_dir_single<P, DAG, PRO, STAGE, MU, SPLIT>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
}

// ---------------------------------------------------------------------------
// fifth-dimension chains on one complex component column held in LDS.
// lds layout: [(s*CB + cbl) * 25 + 2*comp + reim] (one padded row per
// 5D site: immediate offsets, conflict-free rows).
// "lower" orientation: the operator couples s to s-1 (P+ of P5, or P- of
// P5^T); otherwise the column is walked from the top with i = L5-1-s.
// ---------------------------------------------------------------------------
constexpr int kChainStride = 25;
// A column walked from i = 0 (s = 0 when "lower", s = L5 - 1 otherwise).
template <class R> struct Column {
  R* p0;
  int step;  // signed distance between consecutive i, in elements
  int L5;
  __device__ __forceinline__ Cplx<R> get(int i) const { const R* q = p0 + i * step; return {q[0], q[1]}; }
  __device__ __forceinline__ void set(int i, Cplx<R> v) const { R* q = p0 + i * step; q[0] = v.re; q[1] = v.im; }
};

// y = M5^-1 x on a column, in place; with BIDIAG the column is then replaced
// by z = a*y + b*(shift y) (the lower bidiagonal with the -mq wall), fused
// into the same sweep: z_i needs y_i and y_{i-1}, z_0 needs y_{L5-1}.
// The sweeps read four column entries before writing any, so the LDS reads
// of a batch are in flight together (the in-place writes would otherwise
// order every read behind the previous write).
template <class R, bool BIDIAG>
__device__ __forceinline__ void col_m5inv(const Column<R>& col, const Coef5& c, R a, R b) {
  const R kappa = (R)c.kappa, mq = (R)c.mq;
  const int L5 = col.L5;
  R pw = 1, wr = 0, wi = 0;
  for (int k = 1; k < L5; ++k) {
    pw *= -kappa;
    const Cplx<R> x = col.get(L5 - k);
    wr += pw * x.re;
    wi += pw * x.im;
  }
  const Cplx<R> x0 = col.get(0);
  const R ic = (R)c.inv_c, ia = (R)c.inv_alpha;
  Cplx<R> prev = {(x0.re - mq * wr) * ic, (x0.im - mq * wi) * ic};
  const Cplx<R> y0 = {prev.re * ia, prev.im * ia};
  Cplx<R> ym = y0;
  if constexpr (!BIDIAG) col.set(0, y0);
  auto step = [&](int i, Cplx<R> x) {
    prev = {x.re - kappa * prev.re, x.im - kappa * prev.im};
    const Cplx<R> y = {prev.re * ia, prev.im * ia};
    if constexpr (BIDIAG) col.set(i, {a * y.re + b * ym.re, a * y.im + b * ym.im});
    else col.set(i, y);
    ym = y;
  };
  int i = 1;
  for (; i + 3 < L5; i += 4) {
    const Cplx<R> x1 = col.get(i), x2 = col.get(i + 1), x3 = col.get(i + 2), x4 = col.get(i + 3);
    step(i, x1);
    step(i + 1, x2);
    step(i + 2, x3);
    step(i + 3, x4);
  }
  for (; i < L5; ++i) step(i, col.get(i));
  if constexpr (BIDIAG) col.set(0, {a * y0.re - b * mq * ym.re, a * y0.im - b * mq * ym.im});
}

// z = a*y + b*(shift y), shift the lower bidiagonal with the -mq wall, in place
template <class R> __device__ __forceinline__ void col_bidiag(const Column<R>& col, R a, R b, R mq) {
  const int L5 = col.L5;
  const Cplx<R> last = col.get(L5 - 1);
  Cplx<R> y = last;
  auto step = [&](int i, Cplx<R> ym) {
    col.set(i, {a * y.re + b * ym.re, a * y.im + b * ym.im});
    y = ym;
  };
  int i = L5 - 1;
  for (; i - 3 >= 1; i -= 4) {
    const Cplx<R> y1 = col.get(i - 1), y2 = col.get(i - 2), y3 = col.get(i - 3), y4 = col.get(i - 4);
    step(i, y1);
    step(i - 1, y2);
    step(i - 2, y3);
    step(i - 3, y4);
  }
  for (; i >= 1; --i) step(i, col.get(i - 1));
  col.set(0, {a * y.re - b * mq * last.re, a * y.im - b * mq * last.im});
}

template <class R>
__device__ __forceinline__ void run_chain(R* lds, int op, int CB, int cb_log2, int L5, const Coef5& c, int tid, int nthr) {
  const bool dag = op == CH_M5INV_DAG || op == CH_MPHI_DAG || op == CH_M5_DAG || op == CH_MPHIDAG_M5INVDAG;
  for (int task = tid; task < CB * 12; task += nthr) {
    const int cbl = task & (CB - 1);
    const int j = task >> cb_log2;
    const bool plus = j < 6;
    const int stride = kChainStride * CB;
    R* base = lds + cbl * kChainStride + 2 * j;
    const Column<R> col = (plus != dag) ? Column<R>{base, stride, L5} : Column<R>{base + (L5 - 1) * stride, -stride, L5};
    switch (op) {
      case CH_M5INV:
      case CH_M5INV_DAG:
        col_m5inv<R, false>(col, c, R(0), R(0));
        break;
      case CH_MPHI:
      case CH_MPHI_DAG:
        col_bidiag(col, (R)c.b5, (R)c.c5, (R)c.mq);
        break;
      case CH_M5:
      case CH_M5_DAG:
        col_bidiag(col, (R)c.alpha, (R)c.beta, (R)c.mq);
        break;
      case CH_MPHI_M5INV:
      case CH_MPHIDAG_M5INVDAG:
        col_m5inv<R, true>(col, c, (R)c.b5, (R)c.c5);
        break;
      default:
        break;
    }
  }
}

template <class R> __device__ __forceinline__ void lds_put(R* lds, int CB, int cbl, int s, const R v[24]) {
  R* row = lds + (s * CB + cbl) * kChainStride;
#pragma unroll
  for (int k = 0; k < 24; ++k) row[k] = v[k];
}
template <class R> __device__ __forceinline__ void lds_get(const R* lds, int CB, int cbl, int s, R v[24]) {
  const R* row = lds + (s * CB + cbl) * kChainStride;
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = row[k];
}

// ---------------------------------------------------------------------------
// The kernel.  HOP = false turns it into a pure fifth-dimension operator
// (input and output of the same parity).
// ---------------------------------------------------------------------------
// First site of workgroup q.  order_bt = 0: consecutive workgroups take
// consecutive ranges of cb (t is the slowest index, so a site's t-neighbours
// are a whole time slice away in the access stream).  order_bt = Bt > 0 (Bt
// divides Lt): the lattice is cut into order_yb bands of Ly/order_yb y-rows
// (the band's xy-rectangle holds a whole number of workgroups); inside a band
// the (z, t) rectangles are visited in blocks of Bt time slices, z inside a
// block, t fastest.  The z- and t-neighbour rectangles of a rectangle are then
// at most Bt rectangles away in the access stream, and a narrower band keeps
// that distance (in bytes) inside the XCD's L2.  Sites inside a rectangle stay
// consecutive (same reduction tiles).
__device__ __forceinline__ int block_first_site(const DslashArgs& A, int q, int CB) {
  if (A.order_bt <= 0) return q * CB;
  const Geom& g = A.g;
  const int rows = g.Ly / A.order_yb;
  const int bpp = g.Lxh * rows / CB;  // workgroups per rectangle
  const int k = q % bpp;
  int r = q / bpp;
  const int tt = r % A.order_bt;
  r /= A.order_bt;
  const int z = r % g.Lz;
  r /= g.Lz;
  const int ntb = g.Lt / A.order_bt;
  const int t = (r % ntb) * A.order_bt + tt;
  const int yb = r / ntb;
  return ((t * g.Lz + z) * g.Ly + yb * rows) * g.Lxh + k * CB;
}

// x += alpha p on one (checkerboard index, slice) of the CG's x and p
template <int P>
__device__ __forceinline__ void x_update(const DslashArgs& A, const FieldDesc& f, int slot, int cb, int s,
                                         typename PrecTraits<P>::Real alpha) {
  constexpr int PX = P == F64 ? F64 : F32;
  typename PrecTraits<P>::Real pv[24];
  typename PrecTraits<PX>::Real xv[24];
  SpinorIO<P>::load(A.cg_p[slot], f, cb, s, pv);
  SpinorIO<PX>::load(A.cg_x[slot], f, cb, s, xv);
#pragma unroll
  for (int k = 0; k < 24; ++k) xv[k] += alpha * pv[k];
  SpinorIO<PX>::store(A.cg_x[slot], f, cb, s, xv, A.nt_store);
}

// (RHS slot, site block) of logical workgroup lb in the launch's RHS order.
// The XCD remap hands XCD k the logical range [k, k + 1) * gridDim.x / 8, so
// order 2 keeps one eighth of the site blocks on each XCD and walks its RHS
// one after another there: one RHS's neighbour planes at a time in that L2.
__device__ __forceinline__ void block_slot(const DslashArgs& A, int lb, int& slot, int& blk) {
  if (A.rhs_order == 1) {
    slot = lb / A.nblk;
    blk = lb - slot * A.nblk;
  } else if (A.rhs_order == 2) {
    const int per = A.nblk >> 3;  // site blocks per XCD
    const int range = per * A.nslots;
    const int k = lb / range, j = lb - k * range;
    slot = j / per;
    blk = k * per + (j - slot * per);
  } else {
    slot = lb % A.nslots;
    blk = lb / A.nslots;
  }
}

// FP64 needs ~180 VGPRs per thread (2 waves per SIMD), the 32-bit
// arithmetic variants fit 128 (4 waves per SIMD).
template <int P> constexpr int kMaxThreads = P == F64 ? 512 : 1024;

// Resident waves per SIMD the register allocation must leave room for.  The
// 16-bit kernels are asked for 6 (67-80 VGPRs instead of 83-102, no spills in
// FP16, a few in BF16/int16): 6-9 % faster on 32^3 x 64, 0-3 % on 24^3 x 64.
// The FP32 and FP64 kernels are asked for the floor their launch bound
// implies (FP32 at 6 spills and ran 9 % slower).  The build option
// MDWF_WAVES_PER_EU sets the 16-bit request.
#ifndef MDWF_WAVES_PER_EU
#define MDWF_WAVES_PER_EU 0
#endif
template <int P> constexpr int kWavesPerEU =
    (P == F16 || P == BF16 || P == I16) ? (MDWF_WAVES_PER_EU > 0 ? MDWF_WAVES_PER_EU : 6) : kMaxThreads<P> / 256;

template <int P, bool HOP, bool DAG, bool PRO, bool STAGE, bool CGU, bool SPLIT>
__global__ __launch_bounds__(kMaxThreads<P>) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<P>))) void dslash5_kernel(
    DslashArgs A) {
  using R = typename PrecTraits<P>::Real;
  extern __shared__ __align__(16) unsigned char smem[];
  const int CB = 1 << A.cb_log2;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int cbl = tid & (CB - 1);
  const int s = tid >> A.cb_log2;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= A.nslots * A.nblk) return;
  int slot, blk;
  block_slot(A, lb, slot, blk);
  const int cb0 = block_first_site(A, blk, CB);
  if (A.active != nullptr && A.active[(size_t)slot * A.active_stride] == 0) return;
  const int cb = cb0 + cbl;
  const bool valid = cb < A.g.Vh;
  const Coef5 c = A.coef[slot];
  const FieldDesc f{A.g.Vh, A.g.L5};
  const int L5 = A.g.L5;

  Stage<R> st{reinterpret_cast<int*>(smem + A.lds_stage_off),
              reinterpret_cast<R*>(smem + A.lds_stage_off + stage_nbr_bytes(CB))};
  if constexpr (HOP && STAGE) {
    stage_fill<P, SPLIT>(A, st, CB, A.cb_log2, cb0, tid, nthr);
    __syncthreads();
  }

  R v[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = 0;
  if (valid) {
    if constexpr (HOP) {
      int X[4] = {0, 0, 0, 0};
      if constexpr (!STAGE) site_coords(A.g, A.out_par, cb, X[0], X[1], X[2], X[3]);
      Cplx<R> acc[4][3];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a][b] = {0, 0};
      const char* in = A.in[slot];
      if constexpr (STAGE && kHopBatch<P, PRO, CGU> > 0) {
        hop_batches<P, DAG, SPLIT, kHopBatch<P, PRO, CGU>, 0>(f, in, s, acc, st, CB, cbl);
      } else {
        hop_dir<P, DAG, PRO, STAGE, 0, SPLIT>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
        hop_dir<P, DAG, PRO, STAGE, 1, SPLIT>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
        hop_dir<P, DAG, PRO, STAGE, 2, SPLIT>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
        hop_dir<P, DAG, PRO, STAGE, 3, SPLIT>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        v[2 * k] = acc[k / 3][k % 3].re;
        v[2 * k + 1] = acc[k / 3][k % 3].im;
      }
    } else {
      SpinorIO<P>::load(A.in[slot], f, cb, s, v);
    }
  }

  R* lds = reinterpret_cast<R*>(smem);
  if (A.c1 != CH_NONE) {
    if constexpr (HOP && STAGE) __syncthreads();  // the chain columns overlay the stage
    lds_put(lds, CB, cbl, s, v);
    __syncthreads();
    run_chain(lds, A.c1, CB, A.cb_log2, L5, c, tid, nthr);
    __syncthreads();
    lds_get(lds, CB, cbl, s, v);
  }

  // combine: v = coef_y * v + aux term (one multiply-add per value)
  const R cy = (R)A.coef_y;
  if (A.aux_mode != AUX_NONE && valid) {
    R w[24];
    const char* aux = A.aux[slot];
    if (A.aux_mode == AUX_PLAIN) SpinorIO<P>::load(aux, f, cb, s, w);
    else load_bidiag<P>(aux, f, cb, s, L5, (R)c.alpha, (R)c.beta, (R)c.mq, A.aux_mode == AUX_M5DAG, w);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = cy * v[k] + w[k];
  } else if (A.coef_y != 1.0) {
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] *= cy;
  }

  if constexpr (CGU) {
    // r -= alpha q with q = v (and x += alpha p unless a previous launch of
    // the iteration did it); v becomes r for the reduction
    if (valid) {
      const R alpha = (R)A.cg_st[slot].alpha;
      R rv[24];
      SpinorIO<P>::load(A.cg_r[slot], f, cb, s, rv);
#pragma unroll
      for (int k = 0; k < 24; ++k) {
        rv[k] -= alpha * v[k];
        v[k] = rv[k];
      }
      SpinorIO<P>::store(A.cg_r[slot], f, cb, s, rv, A.nt_store);
      if (A.cg_update == 1) x_update<P>(A, f, slot, cb, s, alpha);
    }
  }

  if (A.reduce) {
    // a thread's 24 squares are summed in its arithmetic precision (FP32 for
    // the 32- and 16-bit kernels: relative error < 2e-6 on one site-slice);
    // everything from the slice sums upwards is accumulated in FP64
    R lr = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) lr += v[k] * v[k];
    const double loc = (double)lr;
    // overlaid on the chain columns / stage: every thread has read its row first
    if (A.lds_chain_bytes == 0) __syncthreads();
    double* red = reinterpret_cast<double*>(smem + A.lds_chain_bytes);
    red[s * CB + cbl] = loc;
    __syncthreads();
    double site = 0;
    if (s == 0)
      for (int ss = 0; ss < L5; ++ss) site += red[ss * CB + cbl];
    // fixed 16-site tree (one DPP row = one 16-site tile): the same
    // summation order whatever CB is
    site = row_sum16(site);
    if (s == 0 && (cbl & 15) == 0) {
      const int tile = cb >> 4;
      if (tile < A.ntiles) A.partials[(size_t)slot * A.ntiles + tile] = site;
    }
  }

  if (A.c2 != CH_NONE) {
    __syncthreads();
    lds_put(lds, CB, cbl, s, v);
    __syncthreads();
    run_chain(lds, A.c2, CB, A.cb_log2, L5, c, tid, nthr);
    __syncthreads();
    lds_get(lds, CB, cbl, s, v);
  }
  if (valid && !CGU) SpinorIO<P>::store(A.out[slot], f, cb, s, v, A.nt_store);
  if (!CGU && A.cg_update == 3 && valid) x_update<P>(A, f, slot, cb, s, (R)A.cg_st[slot].alpha);
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
template <int P, bool HOP, bool DAG, bool PRO, bool STAGE, bool CGU = false, bool SPLIT = false>
static hipError_t launch_t(const DslashArgs& A, int threads, size_t smem, int grid, hipStream_t st) {
  auto k = dslash5_kernel<P, HOP, DAG, PRO, STAGE, CGU, SPLIT>;
  if (smem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  launch_k(k, dim3(grid), dim3(threads), smem, st, A);
  return hipGetLastError();
}

template <int P, bool STAGE>
static hipError_t launch_s(const DslashArgs& A, bool dag, bool pro, int threads, size_t smem, int grid,
                           hipStream_t st) {
  // the CG update is fused into M^+ only: r (and x) into its second launch
  // (B2), x alone possibly into its first (B1)
  if (dag && (A.cg_update == 1 || A.cg_update == 2))
    return launch_t<P, true, true, false, STAGE, true>(A, threads, smem, grid, st);
  if (A.cg_update != 0 && !(dag && A.cg_update == 3)) return hipErrorInvalidValue;
  if (dag) return launch_t<P, true, true, false, STAGE>(A, threads, smem, grid, st);
  if (pro) return launch_t<P, true, false, true, STAGE>(A, threads, smem, grid, st);
  return launch_t<P, true, false, false, STAGE>(A, threads, smem, grid, st);
}

template <int P>
static hipError_t launch_p(const DslashArgs& A, bool hop, bool dag, bool pro, int threads, size_t smem, int grid,
                           hipStream_t st) {
  if (A.split_mask != 0) {
    // the split interior exists for the plain staged hop only
    if (!hop || dag || pro || !A.stage || A.cg_update) return hipErrorInvalidValue;
    return launch_t<P, true, false, false, true, false, true>(A, threads, smem, grid, st);
  }
  if (!hop) return A.cg_update ? hipErrorInvalidValue : launch_t<P, false, false, false, false>(A, threads, smem, grid, st);
  if (A.stage) return launch_s<P, true>(A, dag, pro, threads, smem, grid, st);
  return launch_s<P, false>(A, dag, pro, threads, smem, grid, st);
}

int dslash_max_threads(int prec) { return prec == F64 ? kMaxThreads<F64> : kMaxThreads<F32>; }

// LDS: [stage (neighbours + links) | fifth-dimension chain columns][reduction].
// The stage is dead once the hop is done, so the chain columns overlay it.
static void lds_layout(const DslashArgs& A, int prec, int cb_log2, bool hop, size_t& chain, size_t& red,
                       size_t& stage) {
  const size_t CB = (size_t)1 << cb_log2;
  const size_t rb = prec == F64 ? 8 : 4;
  chain = (A.c1 != CH_NONE || A.c2 != CH_NONE) ? round_up(CB * A.g.L5 * kChainStride * rb, 16) : 0;
  red = A.reduce ? round_up(CB * A.g.L5 * 8, 16) : 0;
  stage = (hop && A.stage) ? round_up(stage_nbr_bytes((int)CB) + CB * kStageLinkStride * rb, 16) : 0;
}

// The reduction area overlays the chain columns and the stage when it fits in
// them (both are dead by then, after one more barrier): the launches with a
// reduction then need no more LDS than the others, and on 32^3 x 64 x 12 in
// FP16 they hold 8 workgroups per CU instead of 7 (M^ halves 2.5 % and the
// fused CG-update launch 3.7 % faster; FP32, bound by registers, unchanged).
// The build option MDWF_RED_OVERLAY=0 gives the reduction an area of its own.
#ifndef MDWF_RED_OVERLAY
#define MDWF_RED_OVERLAY 1
#endif
static bool red_overlays(size_t chain, size_t red, size_t stage) {
  return MDWF_RED_OVERLAY && red > 0 && red <= std::max(chain, stage);
}

size_t dslash_lds_bytes(const DslashArgs& A, int prec, int cb_log2, bool hop) {
  size_t chain, red, stage;
  lds_layout(A, prec, cb_log2, hop, chain, red, stage);
  return std::max(chain, stage) + (red_overlays(chain, red, stage) ? 0 : red);
}

// A traversal the kernel's block_first_site can follow: Bt > 0 must divide
// Lt and the xy-plane must hold whole workgroups; y-bands must split Ly into
// whole workgroups.  Anything else (including negative values) falls back to
// the linear order / one band.
void clamp_traversal(const Geom& g, int CB, int& bt, int& yb) {
  if (yb < 1 || g.Ly % yb != 0 || (g.Lxh * (g.Ly / yb)) % CB != 0) yb = 1;
  if (bt < 0 || (bt > 0 && ((g.Lxh * g.Ly) % CB != 0 || g.Lt % bt != 0))) bt = 0;
}

hipError_t dslash_launch(DslashArgs A, int prec, bool hop, bool dag, bool pro, int cb_log2, hipStream_t st) {
  const int CB = 1 << cb_log2;
  A.cb_log2 = cb_log2;
  A.nblk = (A.g.Vh + CB - 1) / CB;
  clamp_traversal(A.g, CB, A.order_bt, A.order_yb);
  size_t chain, red, stage;
  lds_layout(A, prec, cb_log2, hop, chain, red, stage);
  const bool overlay = red_overlays(chain, red, stage);
  A.lds_chain_bytes = overlay ? 0 : (int)std::max(chain, stage);  // offset of the reduction area
  A.lds_stage_off = 0;
  const size_t smem = std::max(chain, stage) + (overlay ? 0 : red);
  const int threads = CB * A.g.L5;
  const long long blocks = (long long)A.nblk * A.nslots;
  const int grid = (int)round_up((size_t)blocks, 8);
  if (A.rhs_order < 0 || A.rhs_order > 2 || A.nslots == 1 || (A.rhs_order == 2 && A.nblk % 8 != 0)) A.rhs_order = 0;
  if (threads > dslash_max_threads(prec) || blocks <= 0) return hipErrorInvalidValue;
  switch (prec) {
    case F64: return launch_p<F64>(A, hop, dag, pro, threads, smem, grid, st);
    case F32: return launch_p<F32>(A, hop, dag, pro, threads, smem, grid, st);
    case F16: return launch_p<F16>(A, hop, dag, pro, threads, smem, grid, st);
    case BF16: return launch_p<BF16>(A, hop, dag, pro, threads, smem, grid, st);
    case I16: return launch_p<I16>(A, hop, dag, pro, threads, smem, grid, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Domain decomposition on one GPU: face packing and the exterior update.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dd_extent(const Geom& g, int d) {
  return d == 0 ? g.Lx : d == 1 ? g.Ly : d == 2 ? g.Lz : g.Lt;
}

// Face index of site X on the face orthogonal to mu: the lexicographic index
// of the other three coordinates (x, y, z, t order, the first fastest), / 2.
__device__ __forceinline__ int dd_face_index(const Geom& g, int mu, const int X[4]) {
  int idx = 0;
#pragma unroll
  for (int d = 3; d >= 0; --d)
    if (d != mu) idx = idx * dd_extent(g, d) + X[d];
  return idx >> 1;
}

// The site of parity par with X[mu] = xm and face index f.  The fastest of
// the other coordinates has an even extent (checked on the host), so 2f and
// 2f + 1 differ only in it and one of the two has the right parity.
__device__ __forceinline__ void dd_face_site(const Geom& g, int mu, int xm, int par, int f, int X[4]) {
  int r = 2 * f;
  int first = -1, sum = xm;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d == mu) continue;
    const int L = dd_extent(g, d);
    X[d] = r % L;
    r /= L;
    if (first < 0) first = d;
    else sum += X[d];
  }
  X[first] += (sum + par + X[first]) & 1;
  X[mu] = xm;
}

template <int SIG, class R>
__device__ __forceinline__ void project_mu(int mu, const Cplx<R> p[4][3], Cplx<R> h[2][3]) {
  switch (mu) {
    case 0: project<0, SIG>(p, h); break;
    case 1: project<1, SIG>(p, h); break;
    case 2: project<2, SIG>(p, h); break;
    default: project<3, SIG>(p, h); break;
  }
}
template <int SIG, class R>
__device__ __forceinline__ void accumulate_mu(int mu, Cplx<R> acc[4][3], const Cplx<R> w[2][3]) {
  switch (mu) {
    case 0: accumulate<0, SIG>(acc, w); break;
    case 1: accumulate<1, SIG>(acc, w); break;
    case 2: accumulate<2, SIG>(acc, w); break;
    default: accumulate<3, SIG>(acc, w); break;
  }
}

// One thread per (face site, slice) of face kind blockIdx.y, RHS blockIdx.z.
// The projectors are those of the plain hop H: (1 - g_mu) forward,
// (1 + g_mu) backward.
template <int P>
__global__ __launch_bounds__(256) void k_dd_pack(DDArgs A) {
  using R = typename PrecTraits<P>::Real;
  const int kind = blockIdx.y, mu = kind >> 1, fb = kind & 1, slot = blockIdx.z;
  if (!((A.split_mask >> mu) & 1)) return;
  const int n = A.face_n[mu];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * A.g.L5) return;
  const int f = t % n, s = t / n;
  const int par = 1 - A.out_par;
  int X[4];
  dd_face_site(A.g, mu, fb == 0 ? 0 : dd_extent(A.g, mu) - 1, par, f, X);
  const int cb = cb_index(A.g, X[0], X[1], X[2], X[3]);
  R v[24];
  SpinorIO<P>::load(A.in[slot], FieldDesc{A.g.Vh, A.g.L5}, cb, s, v);
  Cplx<R> psi[4][3], h[2][3];
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = {v[2 * k], v[2 * k + 1]};
  if (fb == 0) {
    project_mu<-1>(mu, psi, h);
  } else {
    Cplx<R> p2[2][3], U[3][3];
    project_mu<+1>(mu, psi, p2);
    LinkIO<P>::load(A.gauge, A.g.Vh, par, mu, cb, U);
    colour_mul<true>(U, p2, h);
  }
  R* dst = reinterpret_cast<R*>(A.send[slot] + A.face_off[kind]) + (size_t)s * 12 * n + f;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    dst[(size_t)(2 * k) * n] = h[k / 3][k % 3].re;
    dst[(size_t)(2 * k + 1) * n] = h[k / 3][k % 3].im;
  }
}

// One thread per (output site, slice), RHS blockIdx.y: adds the hops across
// split boundaries from the received faces (the forward ones multiplied by
// the site's own link here, the antiperiodic sign applied at the t boundary).
template <int P>
__global__ __launch_bounds__(256) void k_dd_exterior(DDArgs A) {
  using R = typename PrecTraits<P>::Real;
  const int slot = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const Geom& g = A.g;
  if (t >= g.Vh * g.L5) return;
  const int cb = t % g.Vh, s = t / g.Vh;
  int X[4];
  site_coords(g, A.out_par, cb, X[0], X[1], X[2], X[3]);
  Cplx<R> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = {0, 0};
  bool any = false;
  for (int mu = 0; mu < 4; ++mu) {
    if (!((A.split_mask >> mu) & 1)) continue;
    const int L = dd_extent(g, mu), n = A.face_n[mu];
    for (int fb = 0; fb < 2; ++fb) {
      if (fb == 0 ? X[mu] != L - 1 : X[mu] != 0) continue;
      const R* src = reinterpret_cast<const R*>(A.recv[slot] + A.face_off[2 * mu + fb]) + (size_t)s * 12 * n +
                     dd_face_index(g, mu, X);
      Cplx<R> h[2][3], w[2][3];
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k / 3][k % 3] = {src[(size_t)(2 * k) * n], src[(size_t)(2 * k + 1) * n]};
      if (fb == 0) {
        Cplx<R> U[3][3];
        LinkIO<P>::load(A.gauge, g.Vh, A.out_par, mu, cb, U);
        colour_mul<false>(U, h, w);
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k / 3][k % 3] = h[k / 3][k % 3];
      }
      if (mu == 3 && g.tap) {
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k / 3][k % 3] = {-w[k / 3][k % 3].re, -w[k / 3][k % 3].im};
      }
      if (fb == 0) accumulate_mu<-1>(mu, acc, w);
      else accumulate_mu<+1>(mu, acc, w);
      any = true;
    }
  }
  if (!any) return;
  const FieldDesc fd{g.Vh, g.L5};
  R v[24];
  SpinorIO<P>::load(A.out[slot], fd, cb, s, v);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[2 * k] += acc[k / 3][k % 3].re;
    v[2 * k + 1] += acc[k / 3][k % 3].im;
  }
  SpinorIO<P>::store(A.out[slot], fd, cb, s, v);
}

hipError_t dd_pack(const DDArgs& A, int prec, hipStream_t st) {
  int nmax = 0;
  for (int mu = 0; mu < 4; ++mu)
    if ((A.split_mask >> mu) & 1) nmax = std::max(nmax, A.face_n[mu]);
  if (nmax == 0 || A.nslots < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(((size_t)nmax * A.g.L5 + 255) / 256), 8, (unsigned)A.nslots), blk(256);
  switch (prec) {
    case F64: launch_k(k_dd_pack<F64>, grid, blk, 0, st, A); break;
    case F32: launch_k(k_dd_pack<F32>, grid, blk, 0, st, A); break;
    case F16: launch_k(k_dd_pack<F16>, grid, blk, 0, st, A); break;
    case BF16: launch_k(k_dd_pack<BF16>, grid, blk, 0, st, A); break;
    case I16: launch_k(k_dd_pack<I16>, grid, blk, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t dd_exterior(const DDArgs& A, int prec, hipStream_t st) {
  if (A.nslots < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(((size_t)A.g.Vh * A.g.L5 + 255) / 256), (unsigned)A.nslots), blk(256);
  switch (prec) {
    case F64: launch_k(k_dd_exterior<F64>, grid, blk, 0, st, A); break;
    case F32: launch_k(k_dd_exterior<F32>, grid, blk, 0, st, A); break;
    case F16: launch_k(k_dd_exterior<F16>, grid, blk, 0, st, A); break;
    case BF16: launch_k(k_dd_exterior<BF16>, grid, blk, 0, st, A); break;
    case I16: launch_k(k_dd_exterior<I16>, grid, blk, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mdwf
