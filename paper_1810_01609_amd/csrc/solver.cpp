// CG on the normal equations of the even-odd preconditioned Moebius operator,
// with mixed precision and reliable updates, fused over many right-hand sides.
//
// The paper ("Current State of the Art", Performance related) solves the
// red-black preconditioned system with a "double-half" CG: most work in
// 16-bit storage with FP32 arithmetic, with occasional reliable updates to
// full double precision.  Here:
//   * the inner iteration runs in FP64, FP32, or 16-bit storage (FP16, BF16
//     or the paper's int16 fixed point) with a per-site scale (FP32 arithmetic); its solution increment x is FP32
//     (FP64 for the plain solver) and all reductions are FP64;
//   * a reliable update (Sleijpen & van der Vorst 1996) folds x into the FP64
//     solution xh and recomputes the FP64 residual rh = M^+(eta^ - M^ xh)
//     whenever |r| < delta max|r| since the last update, and whenever the
//     inner residual meets the tolerance; convergence is declared only on rh;
//   * alpha, beta and the stopping tests live on the device, so the host
//     polls the per-RHS state only every `check_every` iterations; a RHS that
//     needs the host freezes itself until then;
//   * every RHS of every job stepped together shares the same kernel
//     launches (one workgroup column per RHS): one launch per operator step
//     for the whole batch, each RHS with its own coefficients and state; the
//     workgroups of different RHS on the same sites stage the same links,
//     which the L2 cache serves after the first of them reads them.
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>

#include "internal.h"

using namespace mdwf;

namespace mdwf {
Prog prog_D(int par);
Prog prog_A1();
Prog prog_A1_pt();
Prog prog_A2(bool with_c2, bool reduce);
Prog prog_B1();
Prog prog_B2();
Prog prog_PRE(int par);
Prog prog_5D(int chain);
}  // namespace mdwf

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int inner_x_prec(int ps) { return ps == F64 ? F64 : F32; }

struct SlotLayout {
  size_t fs, fx, fxh, feh, total;
};

SlotLayout slot_layout(const Geom& g, int ps) {
  SlotLayout L;
  L.fs = round_up(spinor_field_bytes(ps, g.L5, g.Vh), 256);
  L.fx = round_up(spinor_field_bytes(inner_x_prec(ps), g.L5, g.Vh), 256);
  L.fxh = ps == F64 ? 0 : round_up(spinor_field_bytes(F64, g.L5, g.Vh), 256);
  L.feh = round_up(spinor_field_bytes(F64, g.L5, g.Vh), 256);  // eta^_e, kept for reliable updates
  L.total = 5 * L.fs + L.fx + L.fxh + L.feh;  // r, p, M_phi p, t, v
  return L;
}

// modelled compulsory bytes / flops of one CG iteration, per RHS
void iter_model(const Geom& g, int ps, double& bytes, double& flops) {
  const double ne = (double)g.Vh * g.L5;
  const double sb = spinor_site_bytes(ps), sx = spinor_site_bytes(inner_x_prec(ps));
  const double links = 8.0 * g.Vh * 12.0 * link_real_bytes(ps);
  // A1 2, A2 3, B1 2, B2 with the fused update 5 spinor transfers + x read/write,
  // 4 link sweeps; p = r + beta p with M_phi p 4 transfers
  bytes = ne * sb * 12 + 2 * ne * sx + 4 * links + ne * 4 * sb;
  // hop 1320/site x4, M_phi 72 x4 (A1, B1, B2, p-update), M5^-1 96 x4, M5 72,
  // xpay 48 x2, CG BLAS 192
  flops = ne * (4 * 1320.0 + 4 * 72 + 4 * 96 + 72 + 2 * 48 + 192);
}

// one fused slot of a step
struct Slot {
  mdwf_job* job;
  int r;
};

struct FP64Temps {
  char *t1, *t2, *t3;
};

}  // namespace

namespace mdwf {

static mdwf_status get_temps(mdwf_ctx* c, const Geom& g, FP64Temps& T) {
  const size_t fb = round_up(spinor_field_bytes(F64, g.L5, g.Vh), 256);
  for (int k = 0; k < 3; ++k) {
    mdwf_status s = ensure(c, c->tmp64[k], fb);
    if (s != MDWF_OK) return s;
  }
  T.t1 = static_cast<char*>(c->tmp64[0].p);
  T.t2 = static_cast<char*>(c->tmp64[1].p);
  T.t3 = static_cast<char*>(c->tmp64[2].p);
  return MDWF_OK;
}

// |a - b|^2 (or |a|^2) of single half-fields in FP64, to the host
static mdwf_status norms_f64(mdwf_ctx* c, const Geom& g, const std::vector<const void*>& a,
                             const std::vector<const void*>* b, std::vector<double>& out) {
  const int n = (int)a.size();
  BlasArgs B{};
  B.g = g;
  B.nslots = n;
  const int nblk = blas_nblk(g);
  mdwf_status s = ensure(c, c->partials_b, (size_t)nblk * n * sizeof(double));
  if (s != MDWF_OK) return s;
  s = ensure(c, c->red_out, (size_t)n * sizeof(double));
  if (s != MDWF_OK) return s;
  B.a = upload_table(c, a);
  B.b = b != nullptr ? upload_table(c, *b) : nullptr;
  B.partials = static_cast<double*>(c->partials_b.p);
  hipEvent_t ev;
  prof_begin(c, &ev);
  hipError_t e = blas_norm_diff(B, F64, c->stream);
  if (e == hipSuccess) e = scalar_reduce(B.partials, nblk, n, static_cast<double*>(c->red_out.p), c->stream);
  prof_end(c, MDWF_PROF_BLAS, (double)g.Vh * g.L5 * 192.0 * (b ? 2 : 1) * n, ev);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->red_host, c->red_out.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_err(c, e, "FP64 norm");
  out.assign(c->red_host, c->red_host + n);
  return MDWF_OK;
}

// single-slot helpers (tables of one entry)
struct One {
  mdwf_ctx* c;
  const mdwf_gauge* g;
  Geom geom;
  const Coef5* coef_d;
  hipError_t e = hipSuccess;
  // a one-entry device pointer table; a failed upload turns into an error
  // here instead of a null table reaching a kernel
  char* const* tab(const void* p) {
    char* const* t = upload_table(c, std::vector<const void*>{p});
    if (t == nullptr && e == hipSuccess) e = hipErrorOutOfMemory;
    return t;
  }
  void prog(const Prog& p, const void* in, const void* aux, void* out) {
    prog_in(p, F64, in, aux, out, MDWF_PROF_DSLASH_F64);
  }
  // a program in precision prec on fields of one job
  void prog_in(const Prog& p, int prec, const void* in, void* out) {
    prog_in(p, prec, in, nullptr, out, MDWF_PROF_DSLASH_INNER);
  }
  void prog_in(const Prog& p, int prec, const void* in, const void* aux, void* out, int cls) {
    if (e != hipSuccess) return;
    if (coef_d == nullptr) { e = hipErrorInvalidValue; return; }
    char* const* I = tab(in);
    char* const* A = aux ? tab(aux) : nullptr;
    char* const* O = tab(out);
    if (e != hipSuccess) return;
    e = run_prog(c, g, geom, prec, p, I, A, O, coef_d, 1, nullptr, 0, nullptr, 0, cls, in != out && aux != out);
  }
  void to_half(const void* user, void* half, int par) {
    if (e != hipSuccess) return;
    char* const* U = tab(user);
    char* const* H = tab(half);
    if (e != hipSuccess) return;
    hipEvent_t ev;
    prof_begin(c, &ev);
    e = layout_user_to_half(geom, U, H, par, F64, 1, c->stream);
    prof_end(c, MDWF_PROF_OTHER, 0, ev);
  }
  void to_user(const void* half, void* user, int par) {
    if (e != hipSuccess) return;
    char* const* H = tab(half);
    char* const* U = tab(user);
    if (e != hipSuccess) return;
    hipEvent_t ev;
    prof_begin(c, &ev);
    e = layout_half_to_user(geom, H, U, par, F64, 1, c->stream);
    prof_end(c, MDWF_PROF_OTHER, 0, ev);
  }
  // out = ca * in + cb * out (precisions pin -> pout)
  void axpby(const void* in, int pin, void* out, int pout, double ca, double cb) {
    if (e != hipSuccess) return;
    BlasArgs B{};
    B.g = geom;
    B.nslots = 1;
    B.a = tab(in);
    B.b = tab(out);
    if (e != hipSuccess) return;
    B.ca = ca;
    B.cb = cb;
    hipEvent_t ev;
    prof_begin(c, &ev);
    e = blas_axpby(B, pin, pout, c->stream);
    const double ne = (double)geom.Vh * geom.L5;
    prof_end(c, MDWF_PROF_BLAS, ne * (spinor_site_bytes(pin) + spinor_site_bytes(pout) * (cb != 0 ? 2 : 1)), ev);
  }
  void zero(void* p, size_t bytes) {
    if (e != hipSuccess) return;
    e = fill_zero(p, bytes, c->stream);
  }
};

// rh (in T.t1) = M^+ (eta^ - M^ xh), with eta^_e kept by the job
static void true_residual(One& o, const FP64Temps& T, const char* eta_hat, const char* xh) {
  o.axpby(eta_hat, F64, T.t1, F64, 1.0, 0.0);               // eta^_e
  o.prog(prog_A1(), xh, nullptr, T.t2);                      // M_phi M5^-1 H_oe M_phi xh
  o.prog(prog_A2(false, false), T.t2, xh, T.t3);             // M^ xh
  o.axpby(T.t3, F64, T.t1, F64, -1.0, 1.0);                  // y = eta^ - M^ xh
  o.prog(prog_5D(CH_M5INV_DAG), T.t1, nullptr, T.t3);        // v = M5^-T y
  o.prog(prog_B1(), T.t3, nullptr, T.t2);
  o.prog(prog_B2(), T.t2, T.t3, T.t1);                       // rh = M^+ y
}

}  // namespace mdwf

// ===========================================================================

static mdwf_status check_opts(mdwf_ctx* c, const mdwf_cg_opts* o) {
  if (o == nullptr) return set_err(c, MDWF_EINVAL, "cg options are NULL");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return set_err(c, MDWF_EINVAL, "tol must be > 0");
  if (o->max_iter < 1) return set_err(c, MDWF_EINVAL, "max_iter must be >= 1");
  if (o->inner < MDWF_F64 || o->inner > MDWF_I16) return set_err(c, MDWF_EINVAL, "bad inner precision");
  if (!(o->delta >= 0.0 && o->delta < 1.0)) return set_err(c, MDWF_EINVAL, "delta must be in [0, 1)");
  if (o->use_initial_guess != 0 && o->use_initial_guess != 1)
    return set_err(c, MDWF_EINVAL, "use_initial_guess must be 0 or 1");
  return MDWF_OK;
}

extern "C" size_t mdwf_job_footprint(const mdwf_action* act, const mdwf_cg_opts* opts, int32_t nrhs) {
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK || opts == nullptr || nrhs < 1) return 0;
  if (opts->inner < MDWF_F64 || opts->inner > MDWF_I16) return 0;
  const Geom g = make_geom(act);
  const SlotLayout L = slot_layout(g, opts->inner);
  // the job's own block, plus the context's three FP64 temporaries
  return L.total * (size_t)nrhs + 3 * round_up(spinor_field_bytes(F64, g.L5, g.Vh), 256);
}

static void finish_slot(mdwf_job* j, int r, int status) {
  j->finished[r] = 1;
  mdwf_cg_stats& s = j->stats[r];
  s.status = status;
  s.converged = status == MDWF_OK ? 1 : 0;
  s.iters = j->st[r].iters;
  s.seconds = now_s() - j->t0;
}

// psi from xh: reconstruct the odd half, write the user field, FP64 full
// residual |eta - D psi| / |eta|.
static mdwf_status finalize(mdwf_ctx* c, mdwf_job* j, int r) {
  FP64Temps T;
  mdwf_status st = get_temps(c, j->geom, T);
  if (st != MDWF_OK) return st;
  One o{c, j->g, j->geom, nullptr};
  std::vector<Coef5> cf(1, j->coef);
  o.coef_d = static_cast<const Coef5*>(upload_bytes(c, cf.data(), sizeof(Coef5)));
  const char* eta = j->eta + j->user_bytes * r;
  char* psi = j->psi + j->user_bytes * r;
  char* xh = j->ps == F64 ? j->fx[r] : j->fxh[r];
  o.to_half(eta, T.t1, 1);
  o.prog(prog_PRE(1), xh, T.t1, T.t2);  // psi_o = M5^-1 (eta_o + 1/2 H_oe M_phi psi_e)
  o.to_user(xh, psi, 0);
  o.to_user(T.t2, psi, 1);
  o.prog(prog_D(0), T.t2, xh, T.t3);    // (D psi)_e
  o.to_half(eta, T.t1, 0);
  if (o.e != hipSuccess) return hip_err(c, o.e, "finalize");
  std::vector<double> n1, n2;
  std::vector<const void*> a{T.t1}, b{T.t3};
  st = norms_f64(c, j->geom, a, &b, n1);
  if (st != MDWF_OK) return st;
  st = norms_f64(c, j->geom, a, nullptr, n2);
  if (st != MDWF_OK) return st;
  double res = n1[0], nrm = n2[0];
  o.prog(prog_D(1), xh, T.t2, T.t3);    // (D psi)_o
  o.to_half(eta, T.t1, 1);
  if (o.e != hipSuccess) return hip_err(c, o.e, "finalize");
  st = norms_f64(c, j->geom, a, &b, n1);
  if (st != MDWF_OK) return st;
  st = norms_f64(c, j->geom, a, nullptr, n2);
  if (st != MDWF_OK) return st;
  res += n1[0];
  nrm += n2[0];
  j->stats[r].rel_res_full = nrm > 0 ? std::sqrt(res / nrm) : 0.0;
  return MDWF_OK;
}

// Reliable update of one RHS: xh += x, x = 0, rh = M^+(eta^ - M^ xh) in FP64,
// r = lo(rh).  Returns |rh|^2 in rr.
static mdwf_status reliable_update(mdwf_ctx* c, mdwf_job* j, int r, double& rr) {
  FP64Temps T;
  mdwf_status st = get_temps(c, j->geom, T);
  if (st != MDWF_OK) return st;
  One o{c, j->g, j->geom, nullptr};
  std::vector<Coef5> cf(1, j->coef);
  o.coef_d = static_cast<const Coef5*>(upload_bytes(c, cf.data(), sizeof(Coef5)));
  char* xh = j->ps == F64 ? j->fx[r] : j->fxh[r];
  if (j->ps != F64) {
    o.axpby(j->fx[r], j->px, xh, F64, 1.0, 1.0);
    o.zero(j->fx[r], spinor_field_bytes(j->px, j->geom.L5, j->geom.Vh));
  }
  true_residual(o, T, j->feh[r], xh);
  o.axpby(T.t1, F64, j->fr[r], j->ps, 1.0, 0.0);
  if (o.e != hipSuccess) return hip_err(c, o.e, "reliable update");
  std::vector<double> n;
  std::vector<const void*> a{T.t1};
  st = norms_f64(c, j->geom, a, nullptr, n);
  rr = n.empty() ? 0.0 : n[0];
  j->stats[r].reliable_updates += 1;
  return st;
}

extern "C" mdwf_status mdwf_job_begin(mdwf_ctx* c, const mdwf_gauge* g, const mdwf_action* act,
                                      const mdwf_cg_opts* opts, int32_t nrhs, const void* eta, void* psi,
                                      mdwf_job** out) {
  if (c == nullptr) return MDWF_EINVAL;
  if (out == nullptr) return set_err(c, MDWF_EINVAL, "mdwf_job_begin: out is NULL");
  *out = nullptr;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_job_begin: %s", msg.c_str());
  mdwf_status st = check_opts(c, opts);
  if (st != MDWF_OK) return st;
  if (g == nullptr || eta == nullptr || psi == nullptr) return set_err(c, MDWF_EINVAL, "mdwf_job_begin: NULL argument");
  if (nrhs < 1) return set_err(c, MDWF_EINVAL, "mdwf_job_begin: nrhs must be >= 1");
  for (int m = 0; m < 4; ++m)
    if (g->L[m] != act->L[m]) return set_err(c, MDWF_EINVAL, "mdwf_job_begin: gauge lattice differs from the action's");
  if (g->data[opts->inner] == nullptr)
    return set_err(c, MDWF_EINVAL, "mdwf_job_begin: gauge field not loaded in the inner precision %d", opts->inner);
  const Geom geom = make_geom(act);
  const size_t ub = (size_t)geom.Vh * 2 * geom.L5 * 12 * 16;
  {
    const char* a = static_cast<const char*>(eta);
    const char* b = static_cast<const char*>(psi);
    if (a < b + ub * nrhs && b < a + ub * nrhs) return set_err(c, MDWF_EINVAL, "mdwf_job_begin: eta and psi overlap");
  }
  (void)hipSetDevice(c->device);
  reset_tables(c);
  mdwf_job* j = new (std::nothrow) mdwf_job();
  if (j == nullptr) return set_err(c, MDWF_ENOMEM, "host allocation");
  j->ctx = c;
  j->g = g;
  j->act = *act;
  j->opts = *opts;
  if (j->opts.check_every <= 0) {
    // host polls: every 8 iterations, or every 2 once an iteration moves 8 GB
    // or more (some 2 ms): a poll costs ~50 us, and a RHS frozen for a
    // reliable update waits for the next poll -- on 32^3 x 64 x 12 with 12
    // RHS polling every 2 iterations made the solve 0.9 % faster, on 16^3 x
    // 32 x 12 every 16 was already slower than every 8
    double bi = 0, fi = 0;
    iter_model(geom, opts->inner, bi, fi);
    j->opts.check_every = bi * nrhs >= 8e9 ? 2 : 8;
  }
  j->nrhs = nrhs;
  j->geom = geom;
  j->ps = opts->inner;
  j->px = inner_x_prec(j->ps);
  j->eta = static_cast<const char*>(eta);
  j->psi = static_cast<char*>(psi);
  j->user_bytes = ub;
  j->coef = make_coef(act);
  iter_model(geom, j->ps, j->bytes_iter, j->flops_iter);
  const SlotLayout L = slot_layout(geom, j->ps);
  j->block_bytes = L.total * (size_t)nrhs;
  hipError_t e = hipSuccess;
  if (c->solve_cache && c->job_cache.p != nullptr && c->job_cache.n >= j->block_bytes) {
    // mdwf_solve: the previous solve's block (same or larger size)
    j->block = c->job_cache.p;
    j->block_bytes = c->job_cache.n;
    c->job_cache.p = nullptr;
    c->job_cache.n = 0;
  } else {
    if (c->solve_cache) release(c->job_cache);  // too small: give its memory back first
    e = hipMalloc(&j->block, j->block_bytes);
  }
  if (e != hipSuccess) {
    j->block = nullptr;
    delete j;
    return hip_err(c, e, "mdwf_job_begin: hipMalloc");
  }
  j->keep_block = c->solve_cache;
  char* p = static_cast<char*>(j->block);
  for (int r = 0; r < nrhs; ++r) {
    j->fr.push_back(p); p += L.fs;
    j->fp.push_back(p); p += L.fs;
    j->fpt.push_back(p); p += L.fs;
    j->ft.push_back(p); p += L.fs;
    j->fv.push_back(p); p += L.fs;
    j->fx.push_back(p); p += L.fx;
    j->fxh.push_back(L.fxh ? p : nullptr); p += L.fxh;
    j->feh.push_back(p); p += L.feh;
  }
  j->st.assign(nrhs, CGState{});
  j->stats.assign(nrhs, mdwf_cg_stats{});
  j->finished.assign(nrhs, 0);
  j->t0 = now_s();

  FP64Temps T;
  st = get_temps(c, geom, T);
  if (st != MDWF_OK) {
    mdwf_job_end(j);
    return st;
  }
  One o{c, g, geom, nullptr};
  std::vector<Coef5> cf(1, j->coef);
  o.coef_d = static_cast<const Coef5*>(upload_bytes(c, cf.data(), sizeof(Coef5)));
  for (int r = 0; r < nrhs && st == MDWF_OK; ++r) {
    const char* er = j->eta + ub * r;
    char* xh = j->ps == F64 ? j->fx[r] : j->fxh[r];
    // b = M^+ eta^, eta^_e = M5^-1 (eta_e + 1/2 H_eo M_phi M5^-1 eta_o)
    o.to_half(er, T.t1, 0);
    o.to_half(er, T.t2, 1);
    o.prog(prog_5D(CH_M5INV), T.t2, nullptr, T.t2);
    o.prog(prog_PRE(0), T.t2, T.t1, T.t1);
    o.axpby(T.t1, F64, j->feh[r], F64, 1.0, 0.0);  // keep eta^_e
    o.prog(prog_5D(CH_M5INV_DAG), T.t1, nullptr, T.t3);
    o.prog(prog_B1(), T.t3, nullptr, T.t2);
    o.prog(prog_B2(), T.t2, T.t3, T.t1);
    if (o.e != hipSuccess) { st = hip_err(c, o.e, "job setup"); break; }
    std::vector<double> n;
    std::vector<const void*> a{T.t1};
    st = norms_f64(c, geom, a, nullptr, n);
    if (st != MDWF_OK) break;
    const double bb = n[0];
    double rr = bb;
    if (opts->use_initial_guess) {
      o.to_half(j->psi + ub * r, xh, 0);
      true_residual(o, T, j->feh[r], xh);
      if (o.e != hipSuccess) { st = hip_err(c, o.e, "job setup"); break; }
      st = norms_f64(c, geom, a, nullptr, n);
      if (st != MDWF_OK) break;
      rr = n[0];
    } else {
      o.zero(xh, spinor_field_bytes(F64, geom.L5, geom.Vh));
    }
    if (j->ps != F64) o.zero(j->fx[r], spinor_field_bytes(j->px, geom.L5, geom.Vh));
    o.axpby(T.t1, F64, j->fr[r], j->ps, 1.0, 0.0);      // r = lo(rh)
    o.axpby(j->fr[r], j->ps, j->fp[r], j->ps, 1.0, 0.0);  // p = r
    o.prog_in(prog_5D(CH_MPHI), j->ps, j->fp[r], j->fpt[r]);
    if (o.e != hipSuccess) { st = hip_err(c, o.e, "job setup"); break; }
    CGState& s = j->st[r];
    s.active = 1;
    s.flags = 0;
    s.iters = 0;
    s.max_iter = opts->max_iter;
    s.rho = rr;
    s.rho_new = rr;
    s.rmax = std::sqrt(rr);
    s.bb = bb;
    s.tol2 = opts->tol * opts->tol * bb;
    s.delta = j->ps == F64 ? 0.0 : opts->delta;
    j->stats[r].rel_res_normal = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (bb == 0.0 || rr <= s.tol2) {
      // zero source (psi = 0) or the initial guess already solves it
      s.active = 0;
      j->stats[r].rel_res_normal = bb > 0 ? std::sqrt(rr / bb) : 0.0;
      st = finalize(c, j, r);
      finish_slot(j, r, MDWF_OK);
    }
  }
  if (st != MDWF_OK) {
    mdwf_job_end(j);
    return st;
  }
  *out = j;
  return MDWF_OK;
}

extern "C" mdwf_status mdwf_job_step(mdwf_ctx* c, mdwf_job* const* jobs, int32_t njobs, int32_t iters) {
  if (c == nullptr) return MDWF_EINVAL;
  if (jobs == nullptr || njobs < 1 || iters < 0) return set_err(c, MDWF_EINVAL, "mdwf_job_step: bad arguments");
  const mdwf_job* j0 = jobs[0];
  for (int k = 0; k < njobs; ++k) {
    const mdwf_job* j = jobs[k];
    if (j == nullptr) return set_err(c, MDWF_EINVAL, "mdwf_job_step: NULL job");
    if (j->ctx != c) return set_err(c, MDWF_EINVAL, "mdwf_job_step: job belongs to another context");
    if (j->g != j0->g || j->ps != j0->ps || j->geom.L5 != j0->geom.L5 || j->geom.tap != j0->geom.tap ||
        j->act.b5 != j0->act.b5 || j->act.c5 != j0->act.c5 || j->act.M5 != j0->act.M5)
      return set_err(c, MDWF_EINVAL, "mdwf_job_step: jobs differ in gauge, L5, precision or Moebius parameters");
    for (int k2 = 0; k2 < k; ++k2)
      if (jobs[k2] == j) return set_err(c, MDWF_EINVAL, "mdwf_job_step: job listed twice");
  }
  (void)hipSetDevice(c->device);
  reset_tables(c);
  const Geom geom = j0->geom;
  const int ps = j0->ps;
  const int ntiles = (geom.Vh + 15) / 16;
  const int nblk = blas_nblk(geom);
  mdwf_status st = MDWF_OK;
  mdwf_status first_fail = MDWF_OK;

  std::vector<Slot> slots;
  auto gather = [&]() {
    slots.clear();
    for (int k = 0; k < njobs; ++k)
      for (int r = 0; r < jobs[k]->nrhs; ++r)
        if (!jobs[k]->finished[r]) slots.push_back(Slot{jobs[k], r});
  };
  gather();
  if (slots.empty() || iters == 0) return MDWF_OK;

  using Tab = char* const*;
  Tab X = nullptr, R = nullptr, P = nullptr, PT = nullptr, T = nullptr, V = nullptr;
  const Coef5* coef_d = nullptr;
  CGState* S_d = nullptr;
  double* pd = nullptr;
  double* pb = nullptr;
  auto build = [&]() -> mdwf_status {
    const int n = (int)slots.size();
    std::vector<const void*> x(n), r(n), p(n), pt(n), t(n), v(n);
    std::vector<Coef5> cf(n);
    for (int i = 0; i < n; ++i) {
      mdwf_job* j = slots[i].job;
      const int k = slots[i].r;
      x[i] = j->fx[k]; r[i] = j->fr[k]; p[i] = j->fp[k]; pt[i] = j->fpt[k];
      t[i] = j->ft[k]; v[i] = j->fv[k];
      cf[i] = j->coef;
    }
    X = upload_table(c, x); R = upload_table(c, r); P = upload_table(c, p); PT = upload_table(c, pt);
    T = upload_table(c, t); V = upload_table(c, v);
    coef_d = static_cast<const Coef5*>(upload_bytes(c, cf.data(), n * sizeof(Coef5)));
    if (!X || !R || !P || !PT || !T || !V || !coef_d) return set_err(c, MDWF_EHIP, "mdwf_job_step: table upload");
    mdwf_status s2 = ensure(c, c->states, n * sizeof(CGState));
    if (s2 == MDWF_OK) s2 = ensure(c, c->partials_d, (size_t)n * ntiles * sizeof(double));
    if (s2 == MDWF_OK) s2 = ensure(c, c->partials_b, (size_t)n * nblk * sizeof(double));
    if (s2 != MDWF_OK) return s2;
    if (c->st_host_n < (size_t)n) {
      if (c->st_host) (void)hipHostFree(c->st_host);
      c->st_host = nullptr;
      c->st_host_n = 0;
      if (hipHostMalloc(reinterpret_cast<void**>(&c->st_host), (n + 64) * sizeof(CGState), hipHostMallocDefault) !=
          hipSuccess)
        return set_err(c, MDWF_ENOMEM, "pinned allocation");
      c->st_host_n = n + 64;
    }
    S_d = static_cast<CGState*>(c->states.p);
    pd = static_cast<double*>(c->partials_d.p);
    pb = static_cast<double*>(c->partials_b.p);
    return MDWF_OK;
  };
  auto upload_states = [&]() -> hipError_t {
    for (size_t i = 0; i < slots.size(); ++i) c->st_host[i] = slots[i].job->st[slots[i].r];
    return hipMemcpyAsync(S_d, c->st_host, slots.size() * sizeof(CGState), hipMemcpyHostToDevice, c->stream);
  };
  st = build();
  if (st != MDWF_OK) return st;
  c->tables_floor = c->tables_used;  // the batch's tables stay put for the whole step
  hipError_t e = upload_states();
  if (e != hipSuccess) return hip_err(c, e, "state upload");

  const int stride = (int)(sizeof(CGState) / sizeof(int));
  const double ne = (double)geom.Vh * geom.L5;
  // x += alpha p rides in the first M^+ launch (B1), whose hop leaves memory
  // bandwidth unused, rather than in the second (B2), already bound by its
  // streams of r and x: single RHS FP16 4 % and 12 fused FP32 RHS 1.4 % faster
  // per iteration on 32^3 x 64, L5 = 12; the same arithmetic, bitwise the same
  // solve (MDWF_X_IN_B1=0 keeps it in B2)
  const char* xe = getenv("MDWF_X_IN_B1");
  const bool x_in_b1 = !(xe != nullptr && xe[0] == '0');
  // One CG iteration is seven launches whose arguments stay fixed while the
  // batch does not change.  With MDWF_GRAPH=1 (and kernel timing and the
  // autotuner off) they are captured once into a HIP graph and replayed.
  // Measured on the smallest serving volume (8^3 x 16, L5 = 8, ~11 us per
  // launch): replaying the graph was 8-10 % slower than launching the seven
  // kernels one by one, so direct launches are the default.
  hipGraphExec_t gexec = nullptr;
  bool graph_failed = false;
  struct GraphGuard {  // early returns release the graph too
    hipGraphExec_t* g;
    hipStream_t s;
    ~GraphGuard() {
      if (*g != nullptr) {
        (void)hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(*g);
      }
    }
  } graph_guard{&gexec, c->stream};
  auto graphs_on = [&]() {
    const char* ev = getenv("MDWF_GRAPH");
    const bool wanted = ev != nullptr && ev[0] == '1';
    return wanted && !graph_failed && c->prof == 0 && c->tune_mode == 0;
  };
  auto drop_graph = [&]() {
    if (gexec != nullptr) {
      (void)hipStreamSynchronize(c->stream);
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
  };
  int remaining = iters;
  while (remaining > 0 && !slots.empty()) {
    const int n = (int)slots.size();
    const int chunk = std::min(remaining, slots[0].job->opts.check_every);
    const int* act = &S_d[0].active;
    std::vector<int> it0(n);
    for (int i = 0; i < n; ++i) it0[i] = slots[i].job->st[slots[i].r].iters;
    prof_chunk_begin(c, chunk);
    auto iteration = [&]() -> hipError_t {
      hipError_t e = run_prog(c, j0->g, geom, ps, prog_A1_pt(), PT, nullptr, T, coef_d, n, act, stride, nullptr, 0,
                              MDWF_PROF_DSLASH_INNER, true);
      if (e == hipSuccess)
        e = run_prog(c, j0->g, geom, ps, prog_A2(true, true), T, P, V, coef_d, n, act, stride, pd, ntiles,
                     MDWF_PROF_DSLASH_INNER, true);
      hipEvent_t ev;
      if (e == hipSuccess) {  // alpha = rho / <p, A p>, <p, A p> = |M^ p|^2 from A2
        prof_begin(c, &ev);
        e = scalar_cg_alpha(S_d, pd, ntiles, n, c->stream);
        prof_end(c, MDWF_PROF_SCALAR, 0, ev);
      }
      if (e == hipSuccess) {  // w_o = M_phi^T M5^-T H^+_oe v (and x += alpha p)
        const CgFuse fx{X, nullptr, P, S_d, 3};
        e = run_prog(c, j0->g, geom, ps, prog_B1(), V, nullptr, T, coef_d, n, act, stride, nullptr, 0,
                     MDWF_PROF_DSLASH_INNER, true, x_in_b1 ? &fx : nullptr);
      }
      if (e == hipSuccess) {  // q = M^+ M^ p, fused with r -= alpha q, |r|^2 (and x += alpha p)
        const CgFuse fz{X, R, P, S_d, x_in_b1 ? 2 : 1};
        Prog b2 = prog_B2();
        b2.reduce = 1;
        e = run_prog(c, j0->g, geom, ps, b2, T, V, T, coef_d, n, act, stride, pd, ntiles, MDWF_PROF_DSLASH_INNER,
                     false, &fz);
      }
      if (e == hipSuccess) {
        prof_begin(c, &ev);
        e = scalar_cg_beta(S_d, pd, ntiles, n, c->stream);
        prof_end(c, MDWF_PROF_SCALAR, 0, ev);
      }
      if (e == hipSuccess) {
        BlasArgs B{};
        B.g = geom;
        B.nslots = n;
        B.a = P; B.b = R; B.c = PT;
        B.st = S_d;
        B.coef = coef_d;
        B.nt_store = streaming_stores(geom, ps, n);
        prof_begin(c, &ev);
        e = blas_cg_p(B, ps, c->stream);
        prof_end(c, MDWF_PROF_BLAS, n * ne * 4.0 * spinor_site_bytes(ps), ev);
      }
      return e;
    };
    if (graphs_on() && gexec == nullptr) {
      hipGraph_t graph = nullptr;
      hipError_t ge = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
      if (ge == hipSuccess) {
        const hipError_t le = iteration();
        ge = hipStreamEndCapture(c->stream, &graph);
        if (le != hipSuccess) ge = le;
      }
      if (ge == hipSuccess) ge = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      if (graph != nullptr) (void)hipGraphDestroy(graph);
      if (ge != hipSuccess) {  // the stream cannot be captured: launch one by one
        (void)hipGetLastError();
        gexec = nullptr;
        graph_failed = true;
      }
    }
    for (int it = 0; it < chunk && e == hipSuccess; ++it) {
      if (gexec != nullptr) {
        e = hipGraphLaunch(gexec, c->stream);
      } else {
        c->prof_pos = it;
        c->prof_skip = c->prof > 1 && (c->prof_iter++ % c->prof) != 0;
        e = iteration();
      }
    }
    c->prof_skip = false;
    c->prof_pos = -1;
    if (e != hipSuccess) return hip_err(c, e, "CG iteration");
    remaining -= chunk;
    // poll the device state
    e = hipMemcpyAsync(c->st_host, S_d, n * sizeof(CGState), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_err(c, e, "state poll");
    for (int i = 0; i < n; ++i) slots[i].job->st[slots[i].r] = c->st_host[i];
    if (c->prof) {  // which iterations of the chunk did work, for the kernel-time accounting
      std::vector<double> frac(chunk, 0.0);
      for (int i = 0; i < n; ++i) {
        const int done = std::min(chunk, std::max(0, c->st_host[i].iters - it0[i]));
        for (int pos = 0; pos < done; ++pos) frac[pos] += 1.0 / n;
      }
      prof_chunk_commit(c, frac);
    }
    bool changed = false;
    for (int i = 0; i < n && st == MDWF_OK; ++i) {
      mdwf_job* j = slots[i].job;
      const int r = slots[i].r;
      CGState& s = j->st[r];
      if (s.active) continue;
      changed = true;
      if (s.flags & (CG_FLAG_NAN | CG_FLAG_BREAKDOWN)) {
        const mdwf_status fs = (s.flags & CG_FLAG_NAN) ? MDWF_ENAN : MDWF_EBREAKDOWN;
        j->stats[r].rel_res_normal = s.bb > 0 ? std::sqrt(std::fabs(s.rho) / s.bb) : 0.0;
        st = finalize(c, j, r);
        finish_slot(j, r, fs);
        if (first_fail == MDWF_OK) first_fail = fs;
        continue;
      }
      if (s.flags & CG_FLAG_UPDATE) {
        double rr = 0;
        st = reliable_update(c, j, r, rr);
        if (st != MDWF_OK) break;
        j->stats[r].rel_res_normal = s.bb > 0 ? std::sqrt(rr / s.bb) : 0.0;
        if (!std::isfinite(rr)) {
          st = finalize(c, j, r);
          finish_slot(j, r, MDWF_ENAN);
          if (first_fail == MDWF_OK) first_fail = MDWF_ENAN;
        } else if (rr <= s.tol2) {
          st = finalize(c, j, r);
          finish_slot(j, r, MDWF_OK);
        } else if (s.flags & CG_FLAG_MAXIT) {
          st = finalize(c, j, r);
          finish_slot(j, r, MDWF_ENOCONV);
          if (first_fail == MDWF_OK) first_fail = MDWF_ENOCONV;
        } else {
          // continue: beta from the true residual, p = r + beta p
          const double beta = rr / s.rho;
          One o{c, j->g, geom, nullptr};
          std::vector<Coef5> cf(1, j->coef);
          o.coef_d = static_cast<const Coef5*>(upload_bytes(c, cf.data(), sizeof(Coef5)));
          if (o.coef_d == nullptr) return set_err(c, MDWF_EHIP, "reliable update: coefficient upload");
          o.axpby(j->fr[r], ps, j->fp[r], ps, 1.0, beta);
          o.prog_in(prog_5D(CH_MPHI), ps, j->fp[r], j->fpt[r]);
          if (o.e != hipSuccess) return hip_err(c, o.e, "reliable update");
          s.rho = rr;
          s.rho_new = rr;
          s.rmax = std::sqrt(rr);
          s.flags = 0;
          s.active = 1;
        }
      }
    }
    if (st != MDWF_OK) return st;
    if (changed) {
      bool any_finished = false;
      for (auto& sl : slots) any_finished |= sl.job->finished[sl.r] != 0;
      if (any_finished) {
        gather();
        drop_graph();  // its launches name the old batch's tables
        if (slots.empty()) break;
        reset_tables(c);
        st = build();
        if (st != MDWF_OK) return st;
        c->tables_floor = c->tables_used;
      }
      e = upload_states();
      if (e != hipSuccess) return hip_err(c, e, "state upload");
    }
  }
  drop_graph();
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_err(c, e, "mdwf_job_step");
  // per-RHS modelled traffic
  for (int k = 0; k < njobs; ++k) {
    mdwf_job* j = jobs[k];
    for (int r = 0; r < j->nrhs; ++r) {
      j->stats[r].iters = j->st[r].iters;
      j->stats[r].bytes = j->bytes_iter * j->st[r].iters;
      j->stats[r].flops = j->flops_iter * j->st[r].iters;
    }
  }
  return first_fail;
}

extern "C" mdwf_status mdwf_job_poll(const mdwf_job* j, int32_t* done, mdwf_cg_stats* stats) {
  if (j == nullptr) return MDWF_EINVAL;
  int all = 1;
  for (int r = 0; r < j->nrhs; ++r) all &= j->finished[r] ? 1 : 0;
  if (done) *done = all;
  if (stats) {
    for (int r = 0; r < j->nrhs; ++r) {
      stats[r] = j->stats[r];
      stats[r].iters = j->st[r].iters;
    }
  }
  return MDWF_OK;
}

extern "C" mdwf_status mdwf_job_end(mdwf_job* j) {
  if (j == nullptr) return MDWF_EINVAL;
  if (j->ctx != nullptr) {
    (void)hipSetDevice(j->ctx->device);
    (void)hipStreamSynchronize(j->ctx->stream);
  }
  if (j->block != nullptr) {
    mdwf_ctx* c = j->ctx;
    if (j->keep_block && c != nullptr && c->job_cache.p == nullptr) {
      c->job_cache.p = j->block;  // kept for the context's next mdwf_solve
      c->job_cache.n = j->block_bytes;
    } else {
      (void)hipFree(j->block);
    }
  }
  delete j;
  return MDWF_OK;
}

extern "C" mdwf_status mdwf_solve(mdwf_ctx* c, const mdwf_gauge* g, const mdwf_action* act,
                                  const mdwf_cg_opts* opts, int32_t nrhs, const void* eta, void* psi,
                                  mdwf_cg_stats* stats) {
  if (c == nullptr) return MDWF_EINVAL;
  mdwf_job* j = nullptr;
  // a blocking solve reuses the previous solve's device block (hipMalloc of
  // tens of GB again for every solve costs time); MDWF_SOLVE_CACHE=0 frees it
  const char* ev = getenv("MDWF_SOLVE_CACHE");
  c->solve_cache = !(ev != nullptr && ev[0] == '0');
  mdwf_status st = mdwf_job_begin(c, g, act, opts, nrhs, eta, psi, &j);
  c->solve_cache = false;
  if (st != MDWF_OK) return st;
  mdwf_status sst = mdwf_job_step(c, &j, 1, INT_MAX);
  int32_t done = 0;
  mdwf_job_poll(j, &done, stats);
  mdwf_status ret = MDWF_OK;
  if (sst != MDWF_OK) ret = sst;
  if (ret == MDWF_OK && stats != nullptr)
    for (int r = 0; r < nrhs; ++r)
      if (stats[r].status != MDWF_OK) {
        ret = (mdwf_status)stats[r].status;
        break;
      }
  mdwf_job_end(j);
  return ret;
}
