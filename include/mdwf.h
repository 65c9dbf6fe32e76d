/*
 * mdwf.h -- C ABI of libmdwf, an MI355X (gfx950) solver for the Moebius
 * domain-wall fermion (MDWF) Dirac equation.
 *
 * The paper this library follows ("Simulating the weak death of the neutron
 * in a femtoscale universe with near-Exascale computing", arXiv:1810.01609)
 * states the problem in its "Current State of the Art" section: quark
 * propagators are solutions of a large sparse linear system, the MDWF Dirac
 * operator acting on L^3 x T x L5 x 3 colours x 4 spins, a radius-one
 * stencil, solved by conjugate gradient on the normal equations with
 * red-black (even-odd) preconditioning, mixed precision and reliable updates.
 * Its "Performance Measurement Method" section describes the workflow this
 * interface mirrors: read a gauge configuration, solve for propagators from
 * sources, hand the propagators on.
 *
 * Operator (standard Moebius form; the paper names it but does not write it):
 *   D   = (b5 D_W + 1) + (c5 D_W - 1) P5,   D_W = (4 - M5) - H/2
 *   H   = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
 *   P5  = P- (shift s+1) + P+ (shift s-1), walls carry -mq,
 *   DeGrand-Rossi chiral gammas (g5 = diag(1,1,-1,-1)), periodic x,y,z,
 *   antiperiodic t when t_antiperiodic != 0.
 *   Even-odd: M^ = 1 - 1/4 M5^-1 H_eo M_phi M5^-1 H_oe M_phi on even sites,
 *   M_phi = b5 + c5 P5, M5 = (b5(4-M5)+1) + (c5(4-M5)-1) P5.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layouts (user layout; the library's device layouts are internal):
 *   gauge  : complex128 (interleaved re,im doubles) [t][z][y][x][mu][row][col],
 *            mu = 0,1,2,3 <-> x,y,z,t; U_mu(x) must be SU(3) (det = 1).
 *   spinor : complex128 [rhs][s][t][z][y][x][spin][colour], full lattice,
 *            both parities, nrhs right-hand sides back to back.
 * Spinor pointers are DEVICE pointers (for example from a torch tensor);
 * the gauge pointer may be host or device (argument `where`).
 * Ownership: the library never frees caller memory; handles are created and
 * destroyed only through this ABI; mdwf_gauge_load copies the links.  A
 * context must outlive the gauge fields and jobs made with it.
 * Errors: every call returns an mdwf_status; on failure the context's
 * last-error string says why (mdwf_last_error).  Arguments are validated
 * before any device work; nothing aborts the process and no C++ exception
 * crosses the ABI.
 * Streams: each context owns one HIP stream (or adopts the caller's);
 * mdwf_dslash is asynchronous on it, mdwf_solve and mdwf_job_step block.
 * Threads: one context per host thread at a time.
 */
#ifndef MDWF_H
#define MDWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDWF_ABI_VERSION 1

#if defined(__GNUC__)
#define MDWF_API __attribute__((visibility("default")))
#else
#define MDWF_API
#endif

typedef struct mdwf_ctx mdwf_ctx;     /* device + stream + workspaces + tune table */
typedef struct mdwf_gauge mdwf_gauge; /* resident gauge field, per precision      */
typedef struct mdwf_job mdwf_job;     /* an in-flight multi-RHS solve             */

typedef enum {
  MDWF_OK = 0,
  MDWF_EINVAL = -1,     /* bad argument (shape, parameter, null pointer)       */
  MDWF_ENOMEM = -2,     /* device allocation failed                            */
  MDWF_EHIP = -3,       /* a HIP runtime call failed                           */
  MDWF_ENOCONV = -4,    /* max_iter reached before the tolerance               */
  MDWF_EBREAKDOWN = -5, /* CG breakdown: <p, A p> <= 0                         */
  MDWF_ENAN = -6,       /* NaN or Inf met in the iteration                     */
  MDWF_EBUSY = -7       /* resource limit (e.g. job jobs/slots per step)       */
} mdwf_status;

/* Storage precisions.  F16 / BF16 / I16 store spinors as 16-bit values with
 * one FP32 scale per 5D site (max |component|; I16 is the paper's fixed-point
 * "half": value = int16 / 32767 * scale) and links as 16-bit values (I16:
 * int16 / 32767); their arithmetic is FP32. */
typedef enum { MDWF_F64 = 0, MDWF_F32 = 1, MDWF_F16 = 2, MDWF_BF16 = 3, MDWF_I16 = 4 } mdwf_prec;

/* Operators for mdwf_dslash.  Half-field operators read the parity they act
 * on from `in` and write the parity they produce into `out`; the other
 * parity of `out` is set to zero. */
typedef enum {
  MDWF_OP_D = 0,         /* out = D in                                    */
  MDWF_OP_DDAG = 1,      /* out = D^+ in                                  */
  MDWF_OP_MHAT = 2,      /* out_e = M^ in_e                               */
  MDWF_OP_MHATDAG = 3,   /* out_e = M^+ in_e                              */
  MDWF_OP_NORMAL = 4,    /* out_e = M^+ M^ in_e                           */
  MDWF_OP_HOP_EO = 5,    /* out_e = H_eo in_o                             */
  MDWF_OP_HOP_OE = 6,    /* out_o = H_oe in_e                             */
  MDWF_OP_HOP = 7,       /* out = H in (both parities)                    */
  MDWF_OP_HOPDAG = 8,    /* out = g5 H g5 in = H^+ in                     */
  MDWF_OP_M5 = 9,        /* out = M5 in (5th-dimension, 4D-site local)    */
  MDWF_OP_M5INV = 10,    /* out = M5^-1 in                                */
  MDWF_OP_MPHI = 11,     /* out = M_phi in                                */
  MDWF_OP_PREP = 12      /* out_e = M5^-1 (in_e + 1/2 H_eo M_phi M5^-1 in_o) */
} mdwf_op;

typedef enum { MDWF_HOST = 0, MDWF_DEVICE = 1 } mdwf_where;

/* Action parameters.  Lx must be even, every L >= 2, L5 >= 1, mq >= 0,
 * b5, c5, M5 finite. */
typedef struct {
  int32_t L[4];           /* Lx, Ly, Lz, Lt                               */
  int32_t L5;
  int32_t t_antiperiodic; /* 1: antiperiodic in t (default), 0: periodic  */
  double b5, c5, M5, mq;
} mdwf_action;

/* CG options.  tol is the relative residual of the normal equations,
 * |b - A x| <= tol |b|, decided on the FP64 residual.  inner is the storage
 * precision of the inner iteration (F64: plain FP64 CG; F32: FP32; F16/BF16/
 * I16: 16-bit storage with a per-site FP32 scale and FP32 arithmetic); every
 * reliable update recomputes the FP64 residual when |r| < delta * max|r|
 * since the previous update.  check_every: iterations between host polls. */
typedef struct {
  double tol;
  double delta;
  int32_t max_iter;
  int32_t inner;
  int32_t use_initial_guess; /* 1: psi holds the starting guess on entry */
  int32_t check_every;       /* <= 0: by size (8; 2 for iterations of >= 8 GB) */
} mdwf_cg_opts;

/* Per right-hand-side result. */
typedef struct {
  int32_t status;           /* mdwf_status of this RHS                     */
  int32_t converged;
  int32_t iters;            /* inner CG iterations                         */
  int32_t reliable_updates; /* FP64 residual recomputations                */
  double rel_res_normal;    /* |b - A x| / |b|, FP64                       */
  double rel_res_full;      /* |eta - D psi| / |eta|, FP64, full 5D        */
  double seconds;           /* wall time from job begin to this RHS's end  */
  double bytes;             /* modelled compulsory HBM bytes moved         */
  double flops;             /* modelled flops                              */
} mdwf_cg_stats;

/* ---- version / context -------------------------------------------------- */

/* Returns MDWF_ABI_VERSION of the built library. */
MDWF_API int32_t mdwf_abi_version(void);

/* Host-only validation of an action (no device work).  MDWF_EINVAL names the
 * offending field in the message written to `msg` (if msg != NULL, up to
 * msg_len bytes, NUL-terminated). */
MDWF_API mdwf_status mdwf_check_action(const mdwf_action *act, char *msg, size_t msg_len);

/* Host-only query (no device work): the workgroup traversal the fused
 * stencil takes for this action, storage precision `prec`, `nrhs` fused
 * right-hand sides and workgroups of 2^cb_log2 sites (cb_log2 in [4, 7]):
 * *bt = time slices per (z, t) block (0: linear order), *yb = y-bands of the
 * xy-plane.  It applies the environment overrides MDWF_BT (>= 0) and MDWF_YB
 * (>= 1) -- other values are ignored -- and falls back to the linear order /
 * one band where the lattice does not admit the requested blocking.
 * MDWF_EINVAL on a bad action, precision, count or NULL output. */
MDWF_API mdwf_status mdwf_query_traversal(const mdwf_action *act, int32_t prec, int32_t nrhs, int32_t cb_log2,
                                          int32_t *bt, int32_t *yb);

/* Create a context on HIP device `device` (the unit that holds one GPU's
 * share of the paper's workflow, "Performance Measurement Method": gauge
 * fields, solves and their workspaces).  stream: a hipStream_t to adopt (not
 * owned), or NULL to create a private blocking stream (default
 * priority).  *out receives the handle (NULL on failure).  EINVAL for a bad
 * device or NULL out, EHIP when the runtime fails, ENOMEM on host exhaustion. */
MDWF_API mdwf_status mdwf_create(int32_t device, void *stream, mdwf_ctx **out);

/* Destroy a context and its workspaces (not its gauge fields or jobs: free
 * those first). */
MDWF_API mdwf_status mdwf_destroy(mdwf_ctx *ctx);

/* Last error message of this context ("" when none).  Valid until the next
 * call on the context. */
MDWF_API const char *mdwf_last_error(const mdwf_ctx *ctx);

/* The context's stream (hipStream_t). */
MDWF_API void *mdwf_stream(const mdwf_ctx *ctx);

/* ---- gauge field (paper: a gluonic field configuration is read per
 *      ensemble member, "Performance Measurement Method", Overview) -------- */

/* Copy and compress the links to the device: rows 0 and 1 of each SU(3)
 * matrix (12 reals) are stored; row 2 is rebuilt as conj(row0 x row1), so
 * the links must have det = 1.  prec_mask: bit (1 << mdwf_prec) for every
 * storage precision to keep resident (FP64 is always kept).  `links` is
 * complex128 [t][z][y][x][mu][3][3] in host or device memory (where). */
MDWF_API mdwf_status mdwf_gauge_load(mdwf_ctx *ctx, const int32_t L[4], const void *links, int32_t where,
                            uint32_t prec_mask, mdwf_gauge **out);
MDWF_API mdwf_status mdwf_gauge_free(mdwf_gauge *g);
/* Device bytes held by a gauge field. */
MDWF_API size_t mdwf_gauge_bytes(const mdwf_gauge *g);

/* ---- sources -------------------------------------------------------------- */

/* The sources of the propagator solves the paper computes ("Current State
 * of the Art", Background: propagators are solutions of the Dirac equation
 * for given sources).  eta (device, user layout, one RHS, caller-allocated,
 * every entry written) = unit 4D point source at x0 = (x,y,z,t) with the
 * given spin and colour, placed on the domain walls: eta_0 = P- xi,
 * eta_{L5-1} = P+ xi.  EINVAL on a bad action, x0 outside the lattice, spin
 * outside [0, 4), colour outside [0, 3) or NULL eta.  Asynchronous. */
MDWF_API mdwf_status mdwf_source_point(mdwf_ctx *ctx, const mdwf_action *act, const int32_t x0[4], int32_t spin,
                              int32_t colour, void *eta);

/* Stochastic source (same passage): eta (device, user layout, one RHS,
 * every entry written) = complex Z2 noise ((+-1) + i(+-1))/sqrt(2) per (4D
 * site, spin, colour), wall-injected as above.  The draws are
 * SplitMix64(seed) outputs with counter ((rhs_index*V4 + i4)*4 + spin)*3 +
 * colour, i4 the lexicographic 4D index; bit 0 gives the real sign, bit 1 the
 * imaginary.  EINVAL on a bad action, rhs_index < 0 or NULL eta.
 * Asynchronous. */
MDWF_API mdwf_status mdwf_source_z2(mdwf_ctx *ctx, const mdwf_action *act, uint64_t seed, int32_t rhs_index,
                           void *eta);

/* ---- Feynman-Hellmann sequential propagator ------------------------------- */
/* The paper's propagator with a current inserted at every time slice
 * ("Current State of the Art", Physics algorithms related): from a solved
 * 5D propagator psi, the 4D quark field q is read off the walls, a current
 * Gamma is applied at every site, the result is wall-injected as a new 5D
 * source, and mdwf_solve gives the sequential propagator. */

/* q (device, complex128 [rhs][t][z][y][x][spin][colour], caller-allocated,
 * nrhs 4D fields back to back) = P- psi_0 + P+ psi_{L5-1} for each of the
 * nrhs 5D fields in psi (device, user layout, back to back).  Asynchronous on
 * the context stream.  EINVAL on a bad action, nrhs < 1 or NULL pointers. */
MDWF_API mdwf_status mdwf_propagator_4d(mdwf_ctx *ctx, const mdwf_action *act, int32_t nrhs, const void *psi,
                                       void *q);

/* eta (device, user layout, nrhs 5D fields, caller-allocated; every entry is
 * written) = wall injection of Gamma q: eta_0 = P- Gamma q,
 * eta_{L5-1} = P+ Gamma q, zero on the other slices.  Gamma =
 * g_x^b0 g_y^b1 g_z^b2 g_t^b3 with gamma_mask = b0 + 2 b1 + 4 b2 + 8 b3
 * (0: identity, 15: gamma5; the axial current g_z g5 is mask 11 up to sign).
 * Asynchronous.  EINVAL on a bad action, mask outside [0, 15], nrhs < 1 or
 * NULL pointers; q and eta must not overlap. */
MDWF_API mdwf_status mdwf_current_source(mdwf_ctx *ctx, const mdwf_action *act, int32_t nrhs, int32_t gamma_mask,
                                        const void *q, void *eta);

/* The physical 4D propagator of the Moebius action (Brower-Neff-Orginos; the
 * quark propagators the paper's Feynman-Hellmann method combines, "Current
 * State of the Art", Physics algorithms related).  eta (device, user layout,
 * nrhs 5D fields, caller-allocated, every entry written) =
 * (1 - c5 D_W) inject(Gamma xi): Gamma xi (gamma_mask as in
 * mdwf_current_source; 0 = identity) enters on the walls of the opposite
 * chirality to the read-out of mdwf_propagator_4d, eta_0 = P+ Gamma xi,
 * eta_{L5-1} = P- Gamma xi (both on slice 0 when L5 = 1), and the 4D factor
 * (1 - c5 D_W), D_W = (4 - M5) - H/2, is applied on those slices.  Solving
 * D psi = eta and reading q = P- psi_0 + P+ psi_{L5-1} then gives
 * q = S Gamma xi with S = (D_eff^-1 - 1) / (1 - mq), D_eff the truncated
 * overlap operator of the Moebius kernel.  xi: device, complex128
 * [rhs][t][z][y][x][spin][colour], nrhs 4D fields back to back (for the
 * sequential source pass the propagator q and the current's mask).  FP64,
 * asynchronous on the context stream.  EINVAL on a bad action, mask outside
 * [0, 15], nrhs < 1, NULL pointers, a gauge field of another lattice or not
 * loaded in FP64; xi and eta must not overlap. */
MDWF_API mdwf_status mdwf_source_physical(mdwf_ctx *ctx, const mdwf_gauge *g, const mdwf_action *act, int32_t nrhs,
                                          int32_t gamma_mask, const void *xi, void *eta);

/* ---- operator application ------------------------------------------------- */

/* The Dirac operator and its even-odd pieces ("Current State of the Art",
 * Background: the MDWF operator, a radius-one stencil in 4D with dense
 * blocks in the fifth dimension; Performance related: its red-black form).
 * out = op(in) for nrhs fields (device, user layout, caller-allocated; every
 * entry of out is written).  The operator is evaluated in storage precision
 * `prec` (inputs rounded to it on entry, FP64 results written back); the
 * gauge field must hold `prec`.  Temporaries live in the context's
 * workspace (allocated on first use, grown when needed).  EINVAL on a bad
 * action, operator, precision, nrhs < 1, NULL or overlapping in/out, or a
 * gauge field of another lattice; ENOMEM when the workspace cannot grow.
 * Asynchronous on the context stream. */
MDWF_API mdwf_status mdwf_dslash(mdwf_ctx *ctx, const mdwf_gauge *g, const mdwf_action *act, int32_t op, int32_t prec,
                        int32_t nrhs, const void *in, void *out);

/* mdwf_dslash without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operators, arguments, layouts and results
 * (bitwise) as mdwf_dslash; every temporary -- the device pointer tables, the
 * per-RHS coefficients and the five internal half-fields per RHS -- lives in
 * one fixed scratch array of 256 MiB per GPU that the library holds until
 * the process ends, so the call performs no hipMalloc, hipFree or other
 * allocation.  Limits: nrhs <= 16 and
 * 64 KiB + 5 * nrhs * (one half-field in `prec`, padded to 256 B) <= 256 MiB
 * (e.g. 16^3 x 32 x L5 = 12 in FP16 with one RHS); beyond them EINVAL with
 * the sizes in the message.  Calls on one stream are ordered; calls on one
 * GPU that overlap in time (two streams or contexts) share the array and
 * race.  No kernel timing is recorded for this call.  Asynchronous on the
 * context stream. */
MDWF_API mdwf_status mdwf_dslash_noalloc(mdwf_ctx *ctx, const mdwf_gauge *g, const mdwf_action *act, int32_t op,
                                         int32_t prec, int32_t nrhs, const void *in, void *out);

/* out_e = H_eo in_o (as MDWF_OP_HOP_EO; the odd parity of out is set to zero)
 * computed the way one rank of a 4D domain-decomposed run computes it (paper,
 * "Current State of the Art": pack the halo, communicate it, apply the
 * interior stencil, then complete the halo part).  Bit mu of split_mask
 * (0..15) marks dimension mu as split between ranks; the lattice is its own
 * neighbour in each split dimension, so the faces a neighbour would send are
 * the ones this call packs.  Steps: (1) pack, per split mu, the spin-projected
 * half spinors (12 reals per site and slice) of the odd sites with x_mu = 0
 * (projector 1 - g_mu) and, already multiplied by U_mu^+, of those with
 * x_mu = L_mu - 1 (projector 1 + g_mu), in the arithmetic precision of prec
 * (FP64 for MDWF_F64, FP32 otherwise); (2) the fused stencil over all even
 * sites without the hops that cross a split boundary; (3) add those hops from
 * the packed faces (the forward ones multiplied by the site's own link, the
 * antiperiodic sign at the t boundary).  split_mask = 0 is MDWF_OP_HOP_EO.
 * Split dimensions need even extents, and splitting x needs an even Ly.  The
 * face buffers live in the context's workspace.  in, out: device, user
 * layout, nrhs fields, not overlapping.  phase_ms: NULL, or 3 doubles that
 * receive the GPU time of (1), (2) and (3) in milliseconds (the call then
 * waits for the stream).  Asynchronous on the context stream otherwise.
 * Errors: MDWF_EINVAL for a bad mask, extent or argument, MDWF_EHIP for a
 * failed launch. */
MDWF_API mdwf_status mdwf_hop_split(mdwf_ctx *ctx, const mdwf_gauge *g, const mdwf_action *act, int32_t prec,
                                    int32_t split_mask, int32_t nrhs, const void *in, void *out, double *phase_ms);

/* ---- propagator solve ----------------------------------------------------- */

/* psi = D^-1 eta for nrhs right-hand sides, by even-odd CG on the normal
 * equations (paper, "Performance related": red-black preconditioned CG,
 * most work in low precision, occasional reliable updates to FP64).  All
 * RHS run fused through the same kernels.  Blocks until every RHS has
 * finished; fills stats[nrhs].  Returns MDWF_OK if all converged, otherwise
 * the first failing RHS's status (the others' results are still written).
 * The solver state (mdwf_job_footprint bytes) stays allocated in the
 * context after the call and is reused by the context's next mdwf_solve of
 * the same or a smaller size (MDWF_SOLVE_CACHE=0 frees it at once;
 * mdwf_trim or mdwf_destroy release it). */
MDWF_API mdwf_status mdwf_solve(mdwf_ctx *ctx, const mdwf_gauge *g, const mdwf_action *act, const mdwf_cg_opts *opts,
                       int32_t nrhs, const void *eta, void *psi, mdwf_cg_stats *stats);

/* Release the device memory the context keeps between calls (the last
 * solve's state, the operator and FP64 workspaces); the next call that needs
 * them allocates again.  Waits for the context stream.  EINVAL on NULL. */
MDWF_API mdwf_status mdwf_trim(mdwf_ctx *ctx);

/* ---- stepping interface for continuous batching --------------------------- */

/* The stepping interface for continuous batching: the one-GPU analogue of
 * the paper's job manager matching ready work to free resources
 * ("Innovations", management and backfilling of tasks).  Device bytes a job
 * of nrhs RHS allocates, including the context's FP64 temporaries (for
 * admission control); 0 for a bad action, options or nrhs < 1. */
MDWF_API size_t mdwf_job_footprint(const mdwf_action *act, const mdwf_cg_opts *opts, int32_t nrhs);

/* Start a solve of nrhs RHS (same solver as mdwf_solve): prepares the
 * even-odd sources and CG state on the device, allocates the job's block
 * (mdwf_job_footprint bytes), returns without iterating.  eta, psi: device,
 * user layout, nrhs fields, not overlapping; they must stay valid until
 * mdwf_job_end (psi receives each RHS when it finishes).  *out receives the
 * job (NULL on failure).  EINVAL on bad arguments, ENOMEM when the block
 * cannot be allocated. */
MDWF_API mdwf_status mdwf_job_begin(mdwf_ctx *ctx, const mdwf_gauge *g, const mdwf_action *act,
                           const mdwf_cg_opts *opts, int32_t nrhs, const void *eta, void *psi,
                           mdwf_job **out);

/* Advance every job in jobs[0..njobs) by up to `iters` CG iterations, all
 * their unfinished RHS fused into the same kernel launches.  Jobs stepped
 * together must share the gauge field, L5, lattice and inner precision
 * (mq may differ).  RHS that converge are reconstructed, verified and
 * written to psi before this returns.  A RHS's arithmetic does not depend
 * on which other jobs it is stepped with. */
MDWF_API mdwf_status mdwf_job_step(mdwf_ctx *ctx, mdwf_job *const *jobs, int32_t njobs, int32_t iters);

/* done = 1 when every RHS of the job has finished (converged or failed);
 * stats (may be NULL) receives nrhs entries.  Host only; EINVAL on NULL job. */
MDWF_API mdwf_status mdwf_job_poll(const mdwf_job *job, int32_t *done, mdwf_cg_stats *stats);

/* Wait for the job's work on its context stream and release its device
 * memory; the handle is invalid afterwards.  EINVAL on NULL. */
MDWF_API mdwf_status mdwf_job_end(mdwf_job *job);

/* ---- measurement ---------------------------------------------------------- */

/* Kernel classes timed with HIP events on the context stream. */
typedef enum {
  MDWF_PROF_DSLASH_INNER = 0, /* fused hop+5th-dimension kernels of the inner CG */
  MDWF_PROF_DSLASH_F64 = 1,   /* FP64 operator kernels (setup, reliable updates) */
  MDWF_PROF_BLAS = 2,         /* fused BLAS-1 + reduction kernels               */
  MDWF_PROF_SCALAR = 3,       /* CG scalar kernels                              */
  MDWF_PROF_OTHER = 4,        /* layout / precision conversion, sources         */
  MDWF_PROF_NCLASS = 5
} mdwf_prof_class;

/* Per-launch kernel timing: on = 0 off (the default), 1 every launch, N > 1
 * every launch outside the CG iteration loop and the launches of one CG
 * iteration in N (the others are counted, not timed).  The start and stop
 * events ride in the kernel dispatches (no marker packets); EINVAL if on < 0. */
MDWF_API mdwf_status mdwf_profile_enable(mdwf_ctx *ctx, int32_t on);
MDWF_API mdwf_status mdwf_profile_reset(mdwf_ctx *ctx);
/* Synchronises the stream, then returns, for one class, all launches, the
 * kernel time in ms and the summed modelled compulsory bytes.  The time is
 * the plain sum when every launch is timed; when sampling, launches inside
 * and outside the CG loop are kept apart and each group's timed mean is
 * multiplied by that group's launch count. */
MDWF_API mdwf_status mdwf_profile_read(mdwf_ctx *ctx, int32_t cls, int64_t *launches, double *ms, double *bytes);

/* Achievable-bandwidth reference: copies `bytes` (a multiple of 16) from
 * device buffer src to device buffer dst with the library's STREAM-style copy
 * kernel (16-byte non-temporal loads and stores, 1 KB contiguous per
 * wavefront access), once untimed and then `reps` times between two HIP
 * events on the context stream; writes 2 * bytes * reps / elapsed in GB/s
 * (read + write).  Blocks until done.  Buffers are the caller's; EINVAL on
 * NULL pointers, overlapping buffers, reps < 1 or a size that is zero or not
 * a multiple of 16. */
MDWF_API mdwf_status mdwf_copy_bandwidth(mdwf_ctx *ctx, const void *src, void *dst, size_t bytes, int32_t reps,
                                         double *gb_per_s);

/* ---- launch autotuner (paper, "GPU Kernel Autotuning") -------------------- */

/* mode 0: fixed default launch shapes; 1: brute-force search of the launch
 * shape the first time a (kernel, lattice, L5, RHS count, precision) key is
 * met, kept in the context's table.  Tuning never changes results: every
 * candidate performs the same arithmetic in the same order per site. */
MDWF_API mdwf_status mdwf_tune_mode(mdwf_ctx *ctx, int32_t mode);
/* Save / load the tune table as text ("key value..." lines). */
MDWF_API mdwf_status mdwf_tune_save(const mdwf_ctx *ctx, const char *path);
MDWF_API mdwf_status mdwf_tune_load(mdwf_ctx *ctx, const char *path);
/* Number of entries in the tune table. */
MDWF_API int32_t mdwf_tune_entries(const mdwf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MDWF_H */
