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
// This is the paper's "kernel fusion to minimise memory traffic, matrix-free
// stencil kernels" (Current State of the Art, Performance related) on the
// operator that paragraph names.
#include "dev_common.h"
#include "kernels.h"

namespace mdwf {

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

template <int MU, int SIG, class R>
__device__ __forceinline__ void project(const Cplx<R> p[4][3], Cplx<R> h[2][3]) {
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

// w = U h (fwd) or U^dag h (bwd), two colour vectors
template <bool ADJ, class R>
__device__ __forceinline__ void colour_mul(const Cplx<R> U[3][3], const Cplx<R> h[2][3], Cplx<R> w[2][3]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cplx<R> s = {0, 0};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const Cplx<R> t = ADJ ? cjmul(U[b][a], h[k][b]) : cmul(U[a][b], h[k][b]);
        s = add(s, t);
      }
      w[k][a] = s;
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
// neighbour's index (bit 31 = crosses the antiperiodic t boundary) and the
// link's 12 reals, loaded once and shared by the site's L5 slice threads.
template <class R> struct Stage {
  int* nbr;  // [8][CB]
  R* lnk;    // [8*12][CB]
};

template <int P>
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
    if (cb < g.Vh) {
      int X[4];
      site_coords(g, A.out_par, cb, X[0], X[1], X[2], X[3]);
      const int mu = dir & 3;
      const int Lmu = mu == 0 ? g.Lx : mu == 1 ? g.Ly : mu == 2 ? g.Lz : g.Lt;
      bool flip;
      if (dir < 4) {
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
      if (flip) nb |= (int)0x80000000u;
    }
    st.nbr[dir * CB + cbl] = nb;
#pragma unroll
    for (int k = 0; k < 12; ++k) st.lnk[(dir * 12 + k) * CB + cbl] = r[k];
  }
}

template <int P, bool DAG, bool PRO, bool STAGE, int MU>
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
      const int e = st.nbr[(MU + 4 * fb) * CB + cbl];
      nb = e & 0x7fffffff;
      flip = e < 0;
      R r[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) r[k] = st.lnk[((MU + 4 * fb) * 12 + k) * CB + cbl];
      link_from_raw(r, U);
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
    if constexpr (PRO) load_bidiag<P>(in, f, nb, s, g.L5, (R)c.b5, (R)c.c5, (R)c.mq, false, v);
    else SpinorIO<P>::load(in, f, nb, s, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = {v[2 * k], v[2 * k + 1]};
    if (fb == 0) project<MU, SF>(psi, h);
    else project<MU, SB>(psi, h);
    if (flip) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[k][a] = {-h[k][a].re, -h[k][a].im};
    }
    if (fb == 0) {
      colour_mul<false>(U, h, w);
      accumulate<MU, SF>(acc, w);
    } else {
      colour_mul<true>(U, h, w);
      accumulate<MU, SB>(acc, w);
    }
    pin_acc(acc);
  }
}


// Both neighbours of direction mu (forward and backward) loaded before either
// is used: two spinor loads in flight per thread instead of one.  Links come
// from the LDS stage in the compute phase, so only the spinors are buffered.
template <int P, bool DAG, bool PRO, int MU>
__device__ __forceinline__ void hop_dir_pair(const DslashArgs& A, const FieldDesc& f, const char* in, int s,
                                             const Coef5& c, Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                             Stage<typename PrecTraits<P>::Real> st, int CB, int cbl) {
  using R = typename PrecTraits<P>::Real;
  const Geom& g = A.g;
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  R v0[24], v1[24];
  const int e0 = st.nbr[MU * CB + cbl];
  const int e1 = st.nbr[(MU + 4) * CB + cbl];
  if constexpr (PRO) {
    load_bidiag<P>(in, f, e0 & 0x7fffffff, s, g.L5, (R)c.b5, (R)c.c5, (R)c.mq, false, v0);
    load_bidiag<P>(in, f, e1 & 0x7fffffff, s, g.L5, (R)c.b5, (R)c.c5, (R)c.mq, false, v1);
  } else {
    SpinorIO<P>::load(in, f, e0 & 0x7fffffff, s, v0);
    SpinorIO<P>::load(in, f, e1 & 0x7fffffff, s, v1);
  }
  Cplx<R> U[3][3], psi[4][3], h[2][3], w[2][3];
#pragma unroll
  for (int fb = 0; fb < 2; ++fb) {
    const R* v = fb == 0 ? v0 : v1;
    R r[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) r[k] = st.lnk[((MU + 4 * fb) * 12 + k) * CB + cbl];
    link_from_raw(r, U);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = {v[2 * k], v[2 * k + 1]};
    if (fb == 0) project<MU, SF>(psi, h);
    else project<MU, SB>(psi, h);
    if ((fb == 0 ? e0 : e1) < 0) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[k][a] = {-h[k][a].re, -h[k][a].im};
    }
    if (fb == 0) {
      colour_mul<false>(U, h, w);
      accumulate<MU, SF>(acc, w);
    } else {
      colour_mul<true>(U, h, w);
      accumulate<MU, SB>(acc, w);
    }
  }
  pin_acc(acc);
}

// Software-pipelined hop over the 8 neighbours (mu forward, mu backward, ...):
// the spinor of neighbour k+1 is requested before neighbour k is computed, so
// each thread always has one neighbour load in flight behind its arithmetic.
// Links and neighbour indices come from the LDS stage.
template <int P, bool PRO>
__device__ __forceinline__ void pipe_load(const DslashArgs& A, const FieldDesc& f, const char* in, int s,
                                          const Coef5& c, int e, typename PrecTraits<P>::Real v[24]) {
  using R = typename PrecTraits<P>::Real;
  if constexpr (PRO) load_bidiag<P>(in, f, e & 0x7fffffff, s, A.g.L5, (R)c.b5, (R)c.c5, (R)c.mq, false, v);
  else SpinorIO<P>::load(in, f, e & 0x7fffffff, s, v);
}

template <int P, bool DAG, int K>
__device__ __forceinline__ void pipe_compute(const typename PrecTraits<P>::Real v[24], int e,
                                             Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                             Stage<typename PrecTraits<P>::Real> st, int CB, int cbl) {
  using R = typename PrecTraits<P>::Real;
  constexpr int MU = K >> 1;
  constexpr int FB = K & 1;  // 0 forward, 1 backward
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SIG = FB == 0 ? SF : -SF;
  Cplx<R> U[3][3], psi[4][3], h[2][3], w[2][3];
  R r[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) r[k] = st.lnk[((MU + 4 * FB) * 12 + k) * CB + cbl];
  link_from_raw(r, U);
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k / 3][k % 3] = {v[2 * k], v[2 * k + 1]};
  project<MU, SIG>(psi, h);
  if (e < 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int a = 0; a < 3; ++a) h[k][a] = {-h[k][a].re, -h[k][a].im};
  }
  colour_mul<FB == 1>(U, h, w);
  accumulate<MU, SIG>(acc, w);
}

template <int P, bool DAG, bool PRO, int K>
__device__ __forceinline__ void pipe_step(const DslashArgs& A, const FieldDesc& f, const char* in, int s,
                                          const Coef5& c, Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                          Stage<typename PrecTraits<P>::Real> st, int CB, int cbl,
                                          typename PrecTraits<P>::Real cur[24], typename PrecTraits<P>::Real nxt[24]) {
  // neighbour order K = 2*mu + fb; stage index = mu + 4*fb
  const int e = st.nbr[((K >> 1) + 4 * (K & 1)) * CB + cbl];
  if constexpr (K < 7) {
    constexpr int K1 = K + 1;
    const int e1 = st.nbr[((K1 >> 1) + 4 * (K1 & 1)) * CB + cbl];
    pipe_load<P, PRO>(A, f, in, s, c, e1, nxt);
  }
  pipe_compute<P, DAG, K>(cur, e, acc, st, CB, cbl);
  pin_acc(acc);
}

template <int P, bool DAG, bool PRO>
__device__ __forceinline__ void hop_pipelined(const DslashArgs& A, const FieldDesc& f, const char* in, int s,
                                              const Coef5& c, Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                              Stage<typename PrecTraits<P>::Real> st, int CB, int cbl) {
  using R = typename PrecTraits<P>::Real;
  R a[24], b[24];
  pipe_load<P, PRO>(A, f, in, s, c, st.nbr[0 * CB + cbl], a);
  pipe_step<P, DAG, PRO, 0>(A, f, in, s, c, acc, st, CB, cbl, a, b);
  pipe_step<P, DAG, PRO, 1>(A, f, in, s, c, acc, st, CB, cbl, b, a);
  pipe_step<P, DAG, PRO, 2>(A, f, in, s, c, acc, st, CB, cbl, a, b);
  pipe_step<P, DAG, PRO, 3>(A, f, in, s, c, acc, st, CB, cbl, b, a);
  pipe_step<P, DAG, PRO, 4>(A, f, in, s, c, acc, st, CB, cbl, a, b);
  pipe_step<P, DAG, PRO, 5>(A, f, in, s, c, acc, st, CB, cbl, b, a);
  pipe_step<P, DAG, PRO, 6>(A, f, in, s, c, acc, st, CB, cbl, a, b);
  pipe_step<P, DAG, PRO, 7>(A, f, in, s, c, acc, st, CB, cbl, b, a);
}

#ifndef MDWF_HOP_PIPE
#define MDWF_HOP_PIPE 0
#endif

#ifndef MDWF_HOP_PAIR
#define MDWF_HOP_PAIR 0
#endif

template <int P, bool DAG, bool PRO, bool STAGE, int MU>
__device__ __forceinline__ void hop_dir(const DslashArgs& A, const FieldDesc& f, const char* in, int cb, int s,
                                        const int X[4], const Coef5& c, Cplx<typename PrecTraits<P>::Real> acc[4][3],
                                        Stage<typename PrecTraits<P>::Real> st, int CB, int cbl) {
  if constexpr (STAGE && MDWF_HOP_PAIR) hop_dir_pair<P, DAG, PRO, MU>(A, f, in, s, c, acc, st, CB, cbl);
  else hop_dir_single<P, DAG, PRO, STAGE, MU>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
}

// ---------------------------------------------------------------------------
// fifth-dimension chains on one complex component column held in LDS.
// lds layout: [(s*24 + 2*comp + reim) * CB + cbl].
// "lower" orientation: the operator couples s to s-1 (P+ of P5, or P- of
// P5^T); otherwise the column is walked from the top with i = L5-1-s.
// ---------------------------------------------------------------------------
template <class R> struct Column {
  R* lds;
  int base;  // offset of (s = 0, comp) for this cbl
  int CB;
  int L5;
  bool lower;
  __device__ __forceinline__ int off(int i) const { return base + (lower ? i : (L5 - 1 - i)) * 24 * CB; }
  __device__ __forceinline__ Cplx<R> get(int i) const { const int o = off(i); return {lds[o], lds[o + CB]}; }
  __device__ __forceinline__ void set(int i, Cplx<R> v) const { const int o = off(i); lds[o] = v.re; lds[o + CB] = v.im; }
};

// y = M5^-1 x on a column, in place
template <class R> __device__ __forceinline__ void col_m5inv(const Column<R>& col, const Coef5& c) {
  const R kappa = (R)c.kappa, mq = (R)c.mq;
  R pw = 1, wr = 0, wi = 0;
  for (int k = 1; k < col.L5; ++k) {
    pw *= -kappa;
    const Cplx<R> x = col.get(col.L5 - k);
    wr += pw * x.re;
    wi += pw * x.im;
  }
  const Cplx<R> x0 = col.get(0);
  const R ic = (R)c.inv_c, ia = (R)c.inv_alpha;
  Cplx<R> prev = {(x0.re - mq * wr) * ic, (x0.im - mq * wi) * ic};
  col.set(0, {prev.re * ia, prev.im * ia});
  for (int i = 1; i < col.L5; ++i) {
    const Cplx<R> x = col.get(i);
    prev = {x.re - kappa * prev.re, x.im - kappa * prev.im};
    col.set(i, {prev.re * ia, prev.im * ia});
  }
}

// z = a*y + b*(shift y), shift the lower bidiagonal with the -mq wall, in place
template <class R> __device__ __forceinline__ void col_bidiag(const Column<R>& col, R a, R b, R mq) {
  const Cplx<R> last = col.get(col.L5 - 1);
  for (int i = col.L5 - 1; i >= 1; --i) {
    const Cplx<R> y = col.get(i), ym = col.get(i - 1);
    col.set(i, {a * y.re + b * ym.re, a * y.im + b * ym.im});
  }
  const Cplx<R> y0 = col.get(0);
  col.set(0, {a * y0.re - b * mq * last.re, a * y0.im - b * mq * last.im});
}

template <class R>
__device__ __forceinline__ void run_chain(R* lds, int op, int CB, int cb_log2, int L5, const Coef5& c, int tid, int nthr) {
  const bool dag = op == CH_M5INV_DAG || op == CH_MPHI_DAG || op == CH_M5_DAG || op == CH_MPHIDAG_M5INVDAG;
  for (int task = tid; task < CB * 12; task += nthr) {
    const int cbl = task & (CB - 1);
    const int j = task >> cb_log2;
    const bool plus = j < 6;
    Column<R> col{lds, 2 * j * CB + cbl, CB, L5, plus != dag};
    switch (op) {
      case CH_M5INV:
      case CH_M5INV_DAG:
        col_m5inv(col, c);
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
        col_m5inv(col, c);
        col_bidiag(col, (R)c.b5, (R)c.c5, (R)c.mq);
        break;
      default:
        break;
    }
  }
}

template <class R> __device__ __forceinline__ void lds_put(R* lds, int CB, int cbl, int s, const R v[24]) {
#pragma unroll
  for (int k = 0; k < 24; ++k) lds[(s * 24 + k) * CB + cbl] = v[k];
}
template <class R> __device__ __forceinline__ void lds_get(const R* lds, int CB, int cbl, int s, R v[24]) {
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = lds[(s * 24 + k) * CB + cbl];
}

// ---------------------------------------------------------------------------
// The kernel.  HOP = false turns it into a pure fifth-dimension operator
// (input and output of the same parity).
// ---------------------------------------------------------------------------
// First site of workgroup q.  order_bt = 0: consecutive workgroups take
// consecutive ranges of cb (t is the slowest index, so a site's t-neighbours
// are a whole time slice away in the access stream).  order_bt = Bt > 0 (the
// xy-plane holds a whole number of workgroups, Bt divides Lt): xy-planes are
// visited in blocks of Bt time slices, z inside a block, t fastest, so the
// z- and t-neighbour planes of a plane are at most Bt planes away and stay in
// the XCD's L2.  Sites inside a plane stay consecutive (same reduction tiles).
__device__ __forceinline__ int block_first_site(const DslashArgs& A, int q, int CB) {
  if (A.order_bt == 0) return q * CB;
  const Geom& g = A.g;
  const int plane = g.Lxh * g.Ly;
  const int bpp = plane / CB;  // workgroups per plane
  const int k = q % bpp;
  int r = q / bpp;
  const int tt = r % A.order_bt;
  r /= A.order_bt;
  const int z = r % g.Lz;
  const int tb = r / g.Lz;
  const int t = tb * A.order_bt + tt;
  return (t * g.Lz + z) * plane + k * CB;
}

// FP64 needs ~180 VGPRs per thread (2 waves per SIMD), the 32-bit
// arithmetic variants fit 128 (4 waves per SIMD).
template <int P> constexpr int kMaxThreads = P == F64 ? 512 : 1024;

template <int P, bool HOP, bool DAG, bool PRO, bool STAGE, bool CGU>
__global__ __launch_bounds__(kMaxThreads<P>) void dslash5_kernel(DslashArgs A) {
  using R = typename PrecTraits<P>::Real;
  extern __shared__ __align__(16) unsigned char smem[];
  const int CB = 1 << A.cb_log2;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int cbl = tid & (CB - 1);
  const int s = tid >> A.cb_log2;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= A.nslots * A.nblk) return;
  const int slot = lb % A.nslots;
  const int cb0 = block_first_site(A, lb / A.nslots, CB);
  if (A.active != nullptr && A.active[(size_t)slot * A.active_stride] == 0) return;
  const int cb = cb0 + cbl;
  const bool valid = cb < A.g.Vh;
  const Coef5 c = A.coef[slot];
  const FieldDesc f{A.g.Vh, A.g.L5};
  const int L5 = A.g.L5;

  Stage<R> st{reinterpret_cast<int*>(smem + A.lds_stage_off),
              reinterpret_cast<R*>(smem + A.lds_stage_off + (size_t)8 * CB * sizeof(int))};
  if constexpr (HOP && STAGE) {
    stage_fill<P>(A, st, CB, A.cb_log2, cb0, tid, nthr);
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
      if constexpr (STAGE && MDWF_HOP_PIPE) {
        hop_pipelined<P, DAG, PRO>(A, f, in, s, c, acc, st, CB, cbl);
      } else {
        hop_dir<P, DAG, PRO, STAGE, 0>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
        hop_dir<P, DAG, PRO, STAGE, 1>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
        hop_dir<P, DAG, PRO, STAGE, 2>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
        hop_dir<P, DAG, PRO, STAGE, 3>(A, f, in, cb, s, X, c, acc, st, CB, cbl);
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
    lds_put(lds, CB, cbl, s, v);
    __syncthreads();
    run_chain(lds, A.c1, CB, A.cb_log2, L5, c, tid, nthr);
    __syncthreads();
    lds_get(lds, CB, cbl, s, v);
  }

  // combine: v = coef_y * v + aux term
  const R cy = (R)A.coef_y;
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] *= cy;
  if (A.aux_mode != AUX_NONE && valid) {
    R w[24];
    const char* aux = A.aux[slot];
    if (A.aux_mode == AUX_PLAIN) SpinorIO<P>::load(aux, f, cb, s, w);
    else load_bidiag<P>(aux, f, cb, s, L5, (R)c.alpha, (R)c.beta, (R)c.mq, A.aux_mode == AUX_M5DAG, w);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] += w[k];
  }

  if constexpr (CGU) {
    // x += alpha p, r -= alpha q with q = v; v becomes r for the reduction
    constexpr int PX = P == F64 ? F64 : F32;
    if (valid) {
      const R alpha = (R)A.cg_st[slot].alpha;
      R pv[24], rv[24];
      typename PrecTraits<PX>::Real xv[24];
      SpinorIO<P>::load(A.cg_p[slot], f, cb, s, pv);
      SpinorIO<P>::load(A.cg_r[slot], f, cb, s, rv);
      SpinorIO<PX>::load(A.cg_x[slot], f, cb, s, xv);
#pragma unroll
      for (int k = 0; k < 24; ++k) {
        xv[k] += alpha * pv[k];
        rv[k] -= alpha * v[k];
        v[k] = rv[k];
      }
      SpinorIO<PX>::store(A.cg_x[slot], f, cb, s, xv);
      SpinorIO<P>::store(A.cg_r[slot], f, cb, s, rv);
    }
  }

  if (A.reduce) {
    double loc = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) loc += (double)v[k] * (double)v[k];
    double* red = reinterpret_cast<double*>(smem + A.lds_chain_bytes);
    red[s * CB + cbl] = loc;
    __syncthreads();
    double site = 0;
    if (s == 0)
      for (int ss = 0; ss < L5; ++ss) site += red[ss * CB + cbl];
    // fixed 16-site tree: the same summation order whatever CB is
    site += __shfl_xor(site, 8);
    site += __shfl_xor(site, 4);
    site += __shfl_xor(site, 2);
    site += __shfl_xor(site, 1);
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
  if (valid && !CGU) SpinorIO<P>::store(A.out[slot], f, cb, s, v);
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
template <int P, bool HOP, bool DAG, bool PRO, bool STAGE, bool CGU = false>
static hipError_t launch_t(const DslashArgs& A, int threads, size_t smem, int grid, hipStream_t st) {
  auto k = dslash5_kernel<P, HOP, DAG, PRO, STAGE, CGU>;
  if (smem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(threads), smem, st, A);
  return hipGetLastError();
}

template <int P, bool STAGE>
static hipError_t launch_s(const DslashArgs& A, bool dag, bool pro, int threads, size_t smem, int grid,
                           hipStream_t st) {
  if (dag && A.cg_update) return launch_t<P, true, true, false, STAGE, true>(A, threads, smem, grid, st);
  if (A.cg_update) return hipErrorInvalidValue;  // the CG update is fused into M^+ (B2) only
  if (dag) return launch_t<P, true, true, false, STAGE>(A, threads, smem, grid, st);
  if (pro) return launch_t<P, true, false, true, STAGE>(A, threads, smem, grid, st);
  return launch_t<P, true, false, false, STAGE>(A, threads, smem, grid, st);
}

template <int P>
static hipError_t launch_p(const DslashArgs& A, bool hop, bool dag, bool pro, int threads, size_t smem, int grid,
                           hipStream_t st) {
  if (!hop) return A.cg_update ? hipErrorInvalidValue : launch_t<P, false, false, false, false>(A, threads, smem, grid, st);
  if (A.stage) return launch_s<P, true>(A, dag, pro, threads, smem, grid, st);
  return launch_s<P, false>(A, dag, pro, threads, smem, grid, st);
}

int dslash_max_threads(int prec) { return prec == F64 ? kMaxThreads<F64> : kMaxThreads<F32>; }

// LDS: [fifth-dimension chain columns][reduction][stage: neighbours + links]
static void lds_layout(const DslashArgs& A, int prec, int cb_log2, bool hop, size_t& chain, size_t& red,
                       size_t& stage) {
  const size_t CB = (size_t)1 << cb_log2;
  const size_t rb = prec == F64 ? 8 : 4;
  chain = (A.c1 != CH_NONE || A.c2 != CH_NONE) ? round_up(CB * A.g.L5 * 24 * rb, 16) : 0;
  red = A.reduce ? round_up(CB * A.g.L5 * 8, 16) : 0;
  stage = (hop && A.stage) ? round_up(CB * 8 * 4, 16) + CB * 8 * 12 * rb : 0;
}

size_t dslash_lds_bytes(const DslashArgs& A, int prec, int cb_log2, bool hop) {
  size_t chain, red, stage;
  lds_layout(A, prec, cb_log2, hop, chain, red, stage);
  return chain + red + stage;
}

hipError_t dslash_launch(DslashArgs A, int prec, bool hop, bool dag, bool pro, int cb_log2, hipStream_t st) {
  const int CB = 1 << cb_log2;
  A.cb_log2 = cb_log2;
  A.nblk = (A.g.Vh + CB - 1) / CB;
  const int plane = A.g.Lxh * A.g.Ly;
  if (A.order_bt > 0 && (plane % CB != 0 || A.g.Lt % A.order_bt != 0)) A.order_bt = 0;
  size_t chain, red, stage;
  lds_layout(A, prec, cb_log2, hop, chain, red, stage);
  A.lds_chain_bytes = (int)chain;
  A.lds_stage_off = (int)(chain + red);
  const size_t smem = chain + red + stage;
  const int threads = CB * A.g.L5;
  const long long blocks = (long long)A.nblk * A.nslots;
  const int grid = (int)round_up((size_t)blocks, 8);
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

}  // namespace mdwf
