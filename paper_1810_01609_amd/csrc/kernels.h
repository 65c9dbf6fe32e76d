// Launch interface of the libmdwf HIP kernels (internal to the library).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dev_common.h"

namespace mdwf {

// Kernel-time profiling without marker packets: while a profiled library
// call is in flight on this thread, the first kernel it launches carries the
// start event and every kernel it launches records the stop event, both
// inside the dispatch itself.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  int launches = 0;
};
LaunchTiming& launch_timing();

// A failed launch is left in the runtime's last-error state: every caller
// returns hipGetLastError() after its launches.
template <class F, class... Args>
inline void launch_k(F kernel, dim3 grid, dim3 block, size_t smem, hipStream_t st, Args... args) {
  LaunchTiming& t = launch_timing();
  hipEvent_t e0 = (t.stop != nullptr && t.launches == 0) ? t.start : nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)smem, st, e0, t.stop, 0u, args...);
  if (t.stop != nullptr) ++t.launches;
}

// Fifth-dimension chains applied to whole columns of a site.
enum Chain : int {
  CH_NONE = 0,
  CH_M5INV = 1,
  CH_M5INV_DAG = 2,
  CH_MPHI = 3,
  CH_MPHI_DAG = 4,
  CH_M5 = 5,
  CH_M5_DAG = 6,
  CH_MPHI_M5INV = 7,        // M_phi M5^-1
  CH_MPHIDAG_M5INVDAG = 8,  // M_phi^T M5^-T
};

// Term added to coef_y * (chained hop result).
enum AuxMode : int {
  AUX_NONE = 0,
  AUX_PLAIN = 1,  // + aux
  AUX_M5 = 2,     // + M5 aux
  AUX_M5DAG = 3,  // + M5^T aux
};

// out = c2( coef_y * c1( H (or H^dag) ( M_phi in if PRO ) ) + auxterm )
// with an optional |.|^2 reduction of the value before c2.
struct DslashArgs {
  Geom g;
  int out_par;
  const char* gauge;       // gauge field of this precision
  char* const* in;         // [nslots] input half-fields (parity 1-out_par; out_par if no hop)
  char* const* aux;        // [nslots] or nullptr
  char* const* out;        // [nslots]
  const Coef5* coef;       // [nslots]
  const int* active;       // nullptr or active flag of slot i at active[i*active_stride]
  int active_stride;
  double* partials;        // [nslots][ntiles] (16-site tiles) when reduce
  int ntiles;
  int nslots;
  int nblk;                // filled by the launcher
  int cb_log2;             // filled by the launcher
  int lds_chain_bytes;     // filled by the launcher: offset of the reduction area
  int lds_stage_off;       // filled by the launcher
  int stage;               // 1: stage neighbour indices and links in LDS once per workgroup
  int order_bt;            // > 0: blocked (z, t) plane traversal with Bt time slices per block
  int order_yb;            // with order_bt > 0: the xy-plane is cut into order_yb bands of Ly/order_yb rows
  int nt_store;            // 1: the launch's field stores are streaming (non-temporal)
  // Order of (RHS, site block) over the workgroups of a multi-RHS launch:
  // 0 = the RHS of one site block consecutive; 1 = RHS by RHS over the whole
  // grid; 2 = each XCD's eighth of the site blocks, RHS by RHS inside it
  // (needs nblk % 8 == 0; the launcher falls back to 0 otherwise).
  int rhs_order;
  int split_mask;          // bit mu: hops across the mu boundary come from halo buffers (skipped here)
  int c1, c2, aux_mode, reduce;
  double coef_y;
  // CG update fused into the epilogue.  cg_update = 1: with q the combined
  // value, x += alpha p, r -= alpha q, and the reduction takes |r|^2; q and
  // `out` are not written.  2: the same without x (r -= alpha q only).  3:
  // `out` is written as usual, and x += alpha p is applied on the launch's
  // (checkerboard index, slice) pairs of x and p (fields of the other parity).
  // x is FP64 for an FP64 kernel, FP32 otherwise.
  int cg_update;
  char* const* cg_x;
  char* const* cg_r;
  char* const* cg_p;
  const CGState* cg_st;
};

hipError_t dslash_launch(DslashArgs A, int prec, bool hop, bool dag, bool pro, int cb_log2, hipStream_t st);
// The traversal a launch of CB-site workgroups actually takes (invalid Bt or
// band counts fall back to the linear order / one band).
void clamp_traversal(const Geom& g, int CB, int& bt, int& yb);

// ---- domain decomposition, rehearsed on one GPU ---------------------------
// A rank owning a block of the lattice computes the hop in three steps: pack
// the faces its neighbours need (spin-projected half spinors, the backward
// ones already multiplied by U^dag), the interior hop with every hop across a
// split boundary left out (dslash5_kernel with split_mask), and the exterior
// update adding the received faces.  Face kind k = 2 mu + fb: fb = 0 holds
// (1 - g_mu) psi of the sites with x_mu = 0 (needed by the neighbour below as
// its forward term), fb = 1 holds U_mu^dag (1 + g_mu) psi of the sites with
// x_mu = L_mu - 1.  Layout per kind: [s][12 reals][face site], face sites of
// one parity indexed by the lexicographic index of the other three
// coordinates divided by two.
struct DDArgs {
  Geom g;
  int out_par;           // parity of the hop's output sites
  int split_mask;
  const char* gauge;
  char* const* in;       // [nslots] input half-fields (parity 1 - out_par)
  char* const* out;      // [nslots] output half-fields (updated in place by the exterior step)
  char* const* send;     // [nslots] packed faces
  char* const* recv;     // [nslots] faces received from the neighbours
  int nslots;
  size_t face_off[8];    // byte offset of face kind k inside a slot's buffer
  int face_n[4];         // sites of one parity on a face orthogonal to mu
};
hipError_t dd_pack(const DDArgs& A, int prec, hipStream_t st);
hipError_t dd_exterior(const DDArgs& A, int prec, hipStream_t st);
size_t dslash_lds_bytes(const DslashArgs& A, int prec, int cb_log2, bool hop);
int dslash_max_threads(int prec);

// ---- BLAS-1 / reductions (one thread per 4D site, loop over s) ------------
struct BlasArgs {
  Geom g;
  char* const* a;   // [nslots]
  char* const* b;
  char* const* c;
  char* const* d;
  CGState* st;      // [nslots] (CG kernels)
  double* partials; // [nslots][nblk]
  int nblk;         // filled by launcher
  int nslots;
  double ca, cb;    // coefficients for axpby
  const Coef5* coef; // [nslots] (k_cg_p)
  int nt_store;      // k_cg_p: streaming stores of p and pt
};
constexpr int kBlasThreads = 256;

// CG: p = r + beta p and pt = M_phi p.   a=p b=r c=pt, coef
hipError_t blas_cg_p(BlasArgs A, int ps, hipStream_t st);
// out = ca * in + cb * out  (cb == 0: out is not read).  a=in(pin) b=out(pout);
// partials of |out|^2 if A.partials.
hipError_t blas_axpby(BlasArgs A, int pin, int pout, hipStream_t st);
// partials of |a - b|^2 (b may be nullptr table: |a|^2).  both precision p
hipError_t blas_norm_diff(BlasArgs A, int p, hipStream_t st);
int blas_nblk(const Geom& g);
// STREAM-style copy of n16 16-byte vectors (achievable-bandwidth reference)
hipError_t copy16(const void* src, void* dst, size_t n16, hipStream_t st);

// ---- scalar kernels (one workgroup per slot, fixed summation order) -------
// out[i] = sum_j partials[i*n + j]
hipError_t scalar_reduce(const double* partials, int n, int nslots, double* out, hipStream_t st);
// alpha = rho / <p,Ap>, with breakdown / NaN checks
hipError_t scalar_cg_alpha(CGState* st_, const double* partials, int n, int nslots, hipStream_t st);
// rho_new = |r|^2; freeze for the host or form beta
hipError_t scalar_cg_beta(CGState* st_, const double* partials, int n, int nslots, hipStream_t st);

// ---- layout, precision, sources --------------------------------------------
// user complex128 full field [s][t][z][y][x][spin][col] -> half-field of parity par (prec p)
hipError_t layout_user_to_half(const Geom& g, const char* const* user, char* const* half, int par, int p,
                               int nslots, hipStream_t st);
// half-field (prec p; nullptr entry in table: zeros) -> user sites of parity par
hipError_t layout_half_to_user(const Geom& g, const char* const* half, char* const* user, int par, int p,
                               int nslots, hipStream_t st);
// user gauge complex128 [t][z][y][x][mu][3][3] (device) -> internal 12-real, prec p
hipError_t layout_gauge(const Geom& g, const double* user, char* out, int p, hipStream_t st);
hipError_t fill_zero(void* ptr, size_t bytes, hipStream_t st);
hipError_t source_point(const Geom& g, double* eta, const int x0[4], int spin, int colour, hipStream_t st);
hipError_t source_z2(const Geom& g, double* eta, uint64_t seed, int rhs_index, hipStream_t st);
// Feynman-Hellmann sequential source, user layouts, nrhs fields back to back
hipError_t propagator_4d(const Geom& g, int nrhs, const double* psi, double* q, hipStream_t st);
hipError_t current_source(const Geom& g, int nrhs, int mask, const double* q, double* eta, hipStream_t st);
// physical 4D-propagator source: eta = (beta + hc H) inject'(Gamma_mask xi), inject' = P+ on slice 0,
// P- on slice L5-1; gauge64 the FP64 internal gauge field
hipError_t source_physical(const Geom& g, int nrhs, int mask, const char* gauge64, const double* xi, double* eta,
                           double beta, double hc, hipStream_t st);

}  // namespace mdwf
