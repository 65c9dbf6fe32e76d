// mdwf_dslash: the operators of the even-odd preconditioned Moebius
// domain-wall system, each built from the fused stencil kernel.
#include <cstring>
#include <mutex>

#include "internal.h"

using namespace mdwf;

namespace mdwf {

// The programs that compose the operators (see DslashArgs):
//   D_e  = M5 in_e - 1/2 H_eo M_phi in_o            (PRO, aux M5, coef -1/2)
//   D^+_e = M5^T in_e - 1/2 M_phi^T H^+_eo in_o       (DAG, c1 M_phi^T, aux M5^T)
//   A1   : t_o = M_phi M5^-1 H_oe M_phi p_e          (PRO, c1 M_phi M5^-1)
//   A2   : u = p - 1/4 M5^-1 H_eo t_o, out M5^-T u   (c1 M5^-1, aux p, c2 M5^-T)
//   B1   : w_o = M_phi^T M5^-T H^+_oe v_e            (DAG, c1 M_phi^T M5^-T)
//   B2   : q = M5^T v - 1/4 M_phi^T H^+_eo w_o       (DAG, c1 M_phi^T, aux M5^T)
//   PRE  : out = M5^-1 (aux + 1/2 H M_phi in)         (PRO, aux, c2 M5^-1)
// so that M^ p = A2 without c2, and M^+ y = B2(B1(M5^-T y)).
Prog prog_D(int par) { return Prog{true, false, true, CH_NONE, CH_NONE, AUX_M5, 0, -0.5, par}; }
Prog prog_Ddag(int par) { return Prog{true, true, false, CH_MPHI_DAG, CH_NONE, AUX_M5DAG, 0, -0.5, par}; }
Prog prog_A1() { return Prog{true, false, true, CH_MPHI_M5INV, CH_NONE, AUX_NONE, 0, 1.0, 1}; }
// A1 on an input that already holds M_phi p (the CG loop's p-update writes it)
Prog prog_A1_pt() { return Prog{true, false, false, CH_MPHI_M5INV, CH_NONE, AUX_NONE, 0, 1.0, 1}; }
Prog prog_A2(bool with_c2, bool reduce) {
  return Prog{true, false, false, CH_M5INV, with_c2 ? CH_M5INV_DAG : CH_NONE, AUX_PLAIN, reduce ? 1 : 0, -0.25, 0};
}
Prog prog_B1() { return Prog{true, true, false, CH_MPHIDAG_M5INVDAG, CH_NONE, AUX_NONE, 0, 1.0, 1}; }
Prog prog_B2() { return Prog{true, true, false, CH_MPHI_DAG, CH_NONE, AUX_M5DAG, 0, -0.25, 0}; }
Prog prog_PRE(int par) { return Prog{true, false, true, CH_NONE, CH_M5INV, AUX_PLAIN, 0, 0.5, par}; }
Prog prog_HOP(int par, bool dag) { return Prog{true, dag, false, CH_NONE, CH_NONE, AUX_NONE, 0, 1.0, par}; }
Prog prog_5D(int chain) { return Prog{false, false, false, chain, CH_NONE, AUX_NONE, 0, 1.0, 0}; }

}  // namespace mdwf

// Argument checks shared by mdwf_dslash and its no-allocation variant.
static mdwf_status dslash_check(mdwf_ctx* c, const char* who, const mdwf_gauge* g, const mdwf_action* act,
                                int32_t op, int32_t prec, int32_t nrhs, const void* in, void* out) {
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "%s: %s", who, msg.c_str());
  if (g == nullptr || in == nullptr || out == nullptr) return set_err(c, MDWF_EINVAL, "%s: NULL argument", who);
  for (int m = 0; m < 4; ++m)
    if (g->L[m] != act->L[m]) return set_err(c, MDWF_EINVAL, "%s: gauge lattice differs from the action's", who);
  if (prec < MDWF_F64 || prec > MDWF_I16) return set_err(c, MDWF_EINVAL, "%s: bad precision", who);
  if (g->data[prec] == nullptr)
    return set_err(c, MDWF_EINVAL, "%s: gauge field was not loaded in precision %d", who, prec);
  if (op < MDWF_OP_D || op > MDWF_OP_PREP) return set_err(c, MDWF_EINVAL, "%s: bad operator %d", who, op);
  if (nrhs < 1) return set_err(c, MDWF_EINVAL, "%s: nrhs must be >= 1", who);
  const Geom geom = make_geom(act);
  const size_t ub = (size_t)geom.Vh * 2 * geom.L5 * 12 * 16;  // user bytes per RHS
  const char* ib = static_cast<const char*>(in);
  const char* ob = static_cast<const char*>(out);
  if (ib < ob + ub * nrhs && ob < ib + ub * nrhs) return set_err(c, MDWF_EINVAL, "%s: in and out overlap", who);
  return MDWF_OK;
}

// The device tables one operator application reads: user fields, the five
// internal half-fields per RHS (in_e, in_o, out_e, out_o, temporary), a table
// of null pointers (a zero parity) and the per-RHS coefficients.
struct DslashTables {
  char* const* UIN;
  char* const* UOUT;
  char* const* IE;
  char* const* IO;
  char* const* OE;
  char* const* OO;
  char* const* T;
  char* const* NUL;
  const Coef5* coef;
};

static mdwf_status dslash_body(mdwf_ctx* c, const mdwf_gauge* g, const Geom& geom, int32_t op, int32_t prec,
                               int32_t nrhs, const DslashTables& t);

extern "C" mdwf_status mdwf_dslash(mdwf_ctx* c, const mdwf_gauge* g, const mdwf_action* act, int32_t op,
                                   int32_t prec, int32_t nrhs, const void* in, void* out) {
  if (c == nullptr) return MDWF_EINVAL;
  mdwf_status st = dslash_check(c, "mdwf_dslash", g, act, op, prec, nrhs, in, out);
  if (st != MDWF_OK) return st;
  const Geom geom = make_geom(act);
  const size_t ub = (size_t)geom.Vh * 2 * geom.L5 * 12 * 16;  // user bytes per RHS
  const char* ib = static_cast<const char*>(in);
  char* ob = static_cast<char*>(out);
  (void)hipSetDevice(c->device);
  reset_tables(c);
  const size_t fb = round_up(spinor_field_bytes(prec, geom.L5, geom.Vh), 256);
  st = ensure(c, c->dws, fb * 5 * nrhs);
  if (st != MDWF_OK) return st;
  const Coef5 coef = make_coef(act);
  std::vector<Coef5> coefs(nrhs, coef);
  const Coef5* coef_d = static_cast<const Coef5*>(upload_bytes(c, coefs.data(), coefs.size() * sizeof(Coef5)));
  std::vector<const void*> uin(nrhs), uout(nrhs), ie(nrhs), io(nrhs), oe(nrhs), oo(nrhs), tt(nrhs), nul(nrhs, nullptr);
  char* w = static_cast<char*>(c->dws.p);
  for (int r = 0; r < nrhs; ++r) {
    uin[r] = ib + ub * r;
    uout[r] = ob + ub * r;
    ie[r] = w + fb * (5 * r + 0);
    io[r] = w + fb * (5 * r + 1);
    oe[r] = w + fb * (5 * r + 2);
    oo[r] = w + fb * (5 * r + 3);
    tt[r] = w + fb * (5 * r + 4);
  }
  DslashTables t;
  t.UIN = upload_table(c, uin);
  t.UOUT = upload_table(c, uout);
  t.IE = upload_table(c, ie);
  t.IO = upload_table(c, io);
  t.OE = upload_table(c, oe);
  t.OO = upload_table(c, oo);
  t.T = upload_table(c, tt);
  t.NUL = upload_table(c, nul);
  t.coef = coef_d;
  if (!t.coef || !t.UIN || !t.UOUT || !t.IE || !t.IO || !t.OE || !t.OO || !t.T || !t.NUL)
    return set_err(c, MDWF_EHIP, "mdwf_dslash: table upload failed");
  return dslash_body(c, g, geom, op, prec, nrhs, t);
}

static mdwf_status dslash_body(mdwf_ctx* c, const mdwf_gauge* g, const Geom& geom, int32_t op, int32_t prec,
                               int32_t nrhs, const DslashTables& t) {
  char* const* UIN = t.UIN;
  char* const* UOUT = t.UOUT;
  char* const* IE = t.IE;
  char* const* IO = t.IO;
  char* const* OE = t.OE;
  char* const* OO = t.OO;
  char* const* T = t.T;
  char* const* NUL = t.NUL;
  const Coef5* coef_d = t.coef;
  const int cls = prec == MDWF_F64 ? MDWF_PROF_DSLASH_F64 : MDWF_PROF_DSLASH_INNER;
  hipError_t e = hipSuccess;
  hipEvent_t ev;
  auto conv_in = [&](int par, char* const* half) {
    if (e != hipSuccess) return;
    prof_begin(c, &ev);
    e = layout_user_to_half(geom, UIN, half, par, prec, nrhs, c->stream);
    prof_end(c, MDWF_PROF_OTHER, 0, ev);
  };
  auto run = [&](const Prog& p, char* const* i, char* const* a, char* const* o) {
    if (e != hipSuccess) return;
    e = run_prog(c, g, geom, prec, p, i, a, o, coef_d, nrhs, nullptr, 0, nullptr, 0, cls, i != o && a != o);
  };
  char* const* res_e = NUL;
  char* const* res_o = NUL;
  switch (op) {
    case MDWF_OP_D:
    case MDWF_OP_DDAG: {
      conv_in(0, IE);
      conv_in(1, IO);
      const bool dg = op == MDWF_OP_DDAG;
      run(dg ? prog_Ddag(0) : prog_D(0), IO, IE, OE);
      run(dg ? prog_Ddag(1) : prog_D(1), IE, IO, OO);
      res_e = OE;
      res_o = OO;
      break;
    }
    case MDWF_OP_MHAT:
      conv_in(0, IE);
      run(prog_A1(), IE, nullptr, T);
      run(prog_A2(false, false), T, IE, OE);
      res_e = OE;
      break;
    case MDWF_OP_MHATDAG:
      conv_in(0, IE);
      run(prog_5D(CH_M5INV_DAG), IE, nullptr, OO);
      run(prog_B1(), OO, nullptr, T);
      run(prog_B2(), T, OO, OE);
      res_e = OE;
      break;
    case MDWF_OP_NORMAL:
      conv_in(0, IE);
      run(prog_A1(), IE, nullptr, T);
      run(prog_A2(true, false), T, IE, OO);
      run(prog_B1(), OO, nullptr, T);
      run(prog_B2(), T, OO, OE);
      res_e = OE;
      break;
    case MDWF_OP_HOP_EO:
      conv_in(1, IO);
      run(prog_HOP(0, false), IO, nullptr, OE);
      res_e = OE;
      break;
    case MDWF_OP_HOP_OE:
      conv_in(0, IE);
      run(prog_HOP(1, false), IE, nullptr, OO);
      res_o = OO;
      break;
    case MDWF_OP_HOP:
    case MDWF_OP_HOPDAG: {
      conv_in(0, IE);
      conv_in(1, IO);
      const bool dg = op == MDWF_OP_HOPDAG;
      run(prog_HOP(0, dg), IO, nullptr, OE);
      run(prog_HOP(1, dg), IE, nullptr, OO);
      res_e = OE;
      res_o = OO;
      break;
    }
    case MDWF_OP_M5:
    case MDWF_OP_M5INV:
    case MDWF_OP_MPHI: {
      conv_in(0, IE);
      conv_in(1, IO);
      const int ch = op == MDWF_OP_M5 ? CH_M5 : op == MDWF_OP_M5INV ? CH_M5INV : CH_MPHI;
      run(prog_5D(ch), IE, nullptr, OE);
      run(prog_5D(ch), IO, nullptr, OO);
      res_e = OE;
      res_o = OO;
      break;
    }
    case MDWF_OP_PREP:
      conv_in(0, IE);
      conv_in(1, IO);
      run(prog_5D(CH_M5INV), IO, nullptr, T);
      run(prog_PRE(0), T, IE, OE);
      res_e = OE;
      break;
    default:
      return set_err(c, MDWF_EINVAL, "mdwf_dslash: bad operator");
  }
  if (e == hipSuccess) {
    prof_begin(c, &ev);
    e = layout_half_to_user(geom, res_e, UOUT, 0, prec, nrhs, c->stream);
    if (e == hipSuccess) e = layout_half_to_user(geom, res_o, UOUT, 1, prec, nrhs, c->stream);
    prof_end(c, MDWF_PROF_OTHER, 0, ev);
  }
  return hip_err(c, e, "mdwf_dslash");
}

// ---------------------------------------------------------------------------
// mdwf_dslash without allocation, for callers that cannot allocate: the
// pointer tables, the coefficients and the five internal half-fields per RHS
// live in `scratch`, one fixed array per GPU that the library holds for the
// life of the process.  Host code never names the array's symbol as an
// address: each device's address comes from hipGetSymbolAddress, taken once
// per device when a context is created on it.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per GPU
constexpr size_t kScratchTableBytes = (size_t)64 << 10;
constexpr int kScratchMaxRhs = 16;
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchMaxDevices] = {};
static hipError_t g_scratch_err[kScratchMaxDevices] = {};

// With `device` current: fetch this device's address of `scratch` (once).
void mdwf::scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kScratchMaxDevices || g_scratch_ptr[device] != nullptr) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  if (e == hipSuccess) g_scratch_ptr[device] = p;
}

static void* scratch_ptr(int device, hipError_t& err) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kScratchMaxDevices) {
    err = hipErrorInvalidDevice;
    return nullptr;
  }
  err = g_scratch_ptr[device] != nullptr ? hipSuccess : g_scratch_err[device];
  if (g_scratch_ptr[device] == nullptr && err == hipSuccess) err = hipErrorNotInitialized;
  return g_scratch_ptr[device];
}

// The tables travel by value in the kernel arguments and are written into the
// scratch by one small kernel on the caller's stream (no host-to-device copy).
struct ScratchTables {
  const char* ptr[8][kScratchMaxRhs];
  Coef5 coef[kScratchMaxRhs];
};
static_assert(sizeof(ScratchTables) <= 3072, "kernel argument size");
static_assert(8 * kScratchMaxRhs * sizeof(void*) + kScratchMaxRhs * sizeof(Coef5) <= kScratchTableBytes, "tables");

__global__ __launch_bounds__(256) void k_put_tables(ScratchTables t, char* dst) {
  const char** tab = reinterpret_cast<const char**>(dst);
  for (int i = threadIdx.x; i < 8 * kScratchMaxRhs; i += blockDim.x) tab[i] = t.ptr[i / kScratchMaxRhs][i % kScratchMaxRhs];
  Coef5* cf = reinterpret_cast<Coef5*>(dst + 8 * kScratchMaxRhs * sizeof(void*));
  for (int i = threadIdx.x; i < kScratchMaxRhs; i += blockDim.x) cf[i] = t.coef[i];
}

extern "C" mdwf_status mdwf_dslash_noalloc(mdwf_ctx* c, const mdwf_gauge* g, const mdwf_action* act, int32_t op,
                                           int32_t prec, int32_t nrhs, const void* in, void* out) {
  if (c == nullptr) return MDWF_EINVAL;
  mdwf_status st = dslash_check(c, "mdwf_dslash_noalloc", g, act, op, prec, nrhs, in, out);
  if (st != MDWF_OK) return st;
  if (nrhs > kScratchMaxRhs)
    return set_err(c, MDWF_EINVAL, "mdwf_dslash_noalloc: nrhs %d exceeds the maximum of %d", nrhs, kScratchMaxRhs);
  const Geom geom = make_geom(act);
  const size_t ub = (size_t)geom.Vh * 2 * geom.L5 * 12 * 16;
  const size_t fb = round_up(spinor_field_bytes(prec, geom.L5, geom.Vh), 256);
  const size_t need = kScratchTableBytes + fb * 5 * (size_t)nrhs;
  if (need > kScratchBytes)
    return set_err(c, MDWF_EINVAL, "mdwf_dslash_noalloc: needs %zu bytes of scratch, more than the %zu it holds", need,
                   kScratchBytes);
  (void)hipSetDevice(c->device);
  hipError_t e = hipSuccess;
  char* base = static_cast<char*>(scratch_ptr(c->device, e));
  if (base == nullptr) return hip_err(c, e, "mdwf_dslash_noalloc: scratch address");
  ScratchTables t{};
  const char* ib = static_cast<const char*>(in);
  const char* ob = static_cast<const char*>(out);
  char* w = base + kScratchTableBytes;
  const Coef5 coef = make_coef(act);
  for (int r = 0; r < nrhs; ++r) {
    t.ptr[0][r] = ib + ub * r;
    t.ptr[1][r] = ob + ub * r;
    for (int k = 0; k < 5; ++k) t.ptr[2 + k][r] = w + fb * (5 * r + k);
    t.ptr[7][r] = nullptr;
    t.coef[r] = coef;
  }
  launch_k(k_put_tables, dim3(1), dim3(256), 0, c->stream, t, base);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "mdwf_dslash_noalloc: table kernel");
  char* const* tab = reinterpret_cast<char* const*>(base);
  DslashTables d;
  d.UIN = tab + 0 * kScratchMaxRhs;
  d.UOUT = tab + 1 * kScratchMaxRhs;
  d.IE = tab + 2 * kScratchMaxRhs;
  d.IO = tab + 3 * kScratchMaxRhs;
  d.OE = tab + 4 * kScratchMaxRhs;
  d.OO = tab + 5 * kScratchMaxRhs;
  d.T = tab + 6 * kScratchMaxRhs;
  d.NUL = tab + 7 * kScratchMaxRhs;
  d.coef = reinterpret_cast<const Coef5*>(base + 8 * kScratchMaxRhs * sizeof(void*));
  // kernel timing would create HIP events: it is left off for this call
  const int prof = c->prof;
  c->prof = 0;
  st = dslash_body(c, g, geom, op, prec, nrhs, d);
  c->prof = prof;
  return st;
}

// The hop H_eo computed the way one rank of a domain-decomposed run computes
// it, with the lattice as its own neighbour in every split dimension: pack the
// faces, run the interior hop without the hops across split boundaries, and
// add those from the faces.  The faces are read back from the packing buffer
// itself (the exchange between ranks is the one step one GPU cannot show).
extern "C" mdwf_status mdwf_hop_split(mdwf_ctx* c, const mdwf_gauge* g, const mdwf_action* act, int32_t prec,
                                      int32_t split_mask, int32_t nrhs, const void* in, void* out,
                                      double* phase_ms) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: %s", msg.c_str());
  if (split_mask < 0 || split_mask > 15) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: split_mask must be in [0, 15]");
  for (int m = 0; m < 4; ++m)
    if (((split_mask >> m) & 1) && act->L[m] % 2 != 0)
      return set_err(c, MDWF_EINVAL, "mdwf_hop_split: a split dimension needs an even extent");
  if ((split_mask & 1) && act->L[1] % 2 != 0)
    return set_err(c, MDWF_EINVAL, "mdwf_hop_split: splitting x needs an even Ly (face indexing)");
  if (g == nullptr || in == nullptr || out == nullptr) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: NULL argument");
  for (int m = 0; m < 4; ++m)
    if (g->L[m] != act->L[m]) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: gauge lattice differs from the action's");
  if (prec < MDWF_F64 || prec > MDWF_I16) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: bad precision");
  if (g->data[prec] == nullptr)
    return set_err(c, MDWF_EINVAL, "mdwf_hop_split: gauge field was not loaded in precision %d", prec);
  if (nrhs < 1) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: nrhs must be >= 1");
  {
    const char* e = getenv("MDWF_STAGE");
    if (split_mask != 0 && e != nullptr && e[0] == '0')
      return set_err(c, MDWF_EINVAL, "mdwf_hop_split: the split interior needs the staged stencil (MDWF_STAGE=0)");
  }
  const Geom geom = make_geom(act);
  const size_t ub = (size_t)geom.Vh * 2 * geom.L5 * 12 * 16;
  const char* ib = static_cast<const char*>(in);
  char* ob = static_cast<char*>(out);
  if (ib < ob + ub * nrhs && ob < ib + ub * nrhs) return set_err(c, MDWF_EINVAL, "mdwf_hop_split: in and out overlap");
  (void)hipSetDevice(c->device);
  reset_tables(c);
  DDArgs D{};
  D.g = geom;
  D.out_par = 0;
  D.split_mask = split_mask;
  D.gauge = static_cast<const char*>(g->data[prec]);
  D.nslots = nrhs;
  const int Ls[4] = {geom.Lx, geom.Ly, geom.Lz, geom.Lt};
  const size_t rb = prec == MDWF_F64 ? 8 : 4;
  size_t hb = 0;  // face buffer bytes per RHS
  for (int m = 0; m < 4; ++m) {
    D.face_n[m] = (int)((size_t)geom.Vh * 2 / Ls[m] / 2);
    for (int fb = 0; fb < 2; ++fb) {
      D.face_off[2 * m + fb] = hb;
      if ((split_mask >> m) & 1) hb += round_up((size_t)D.face_n[m] * geom.L5 * 12 * rb, 256);
    }
  }
  const size_t fb = round_up(spinor_field_bytes(prec, geom.L5, geom.Vh), 256);
  const size_t hb_r = round_up(hb, 256);
  mdwf_status st = ensure(c, c->dws, (fb * 2 + hb_r) * nrhs);
  if (st != MDWF_OK) return st;
  const Coef5 coef = make_coef(act);
  std::vector<Coef5> coefs(nrhs, coef);
  const Coef5* coef_d = static_cast<const Coef5*>(upload_bytes(c, coefs.data(), coefs.size() * sizeof(Coef5)));
  std::vector<const void*> uin(nrhs), uout(nrhs), io(nrhs), oe(nrhs), hal(nrhs), nul(nrhs, nullptr);
  char* w = static_cast<char*>(c->dws.p);
  for (int r = 0; r < nrhs; ++r) {
    uin[r] = ib + ub * r;
    uout[r] = ob + ub * r;
    io[r] = w + (fb * 2 + hb_r) * r;
    oe[r] = w + (fb * 2 + hb_r) * r + fb;
    hal[r] = w + (fb * 2 + hb_r) * r + 2 * fb;
  }
  char* const* UIN = upload_table(c, uin);
  char* const* UOUT = upload_table(c, uout);
  char* const* IO = upload_table(c, io);
  char* const* OE = upload_table(c, oe);
  char* const* HAL = upload_table(c, hal);
  char* const* NUL = upload_table(c, nul);
  if (!coef_d || !UIN || !UOUT || !IO || !OE || !HAL || !NUL)
    return set_err(c, MDWF_EHIP, "mdwf_hop_split: table upload failed");
  D.in = IO;
  D.out = OE;
  D.send = HAL;
  D.recv = HAL;  // every split neighbour is the lattice itself
  const int cls = prec == MDWF_F64 ? MDWF_PROF_DSLASH_F64 : MDWF_PROF_DSLASH_INNER;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  if (phase_ms != nullptr)
    for (auto& x : ev) (void)hipEventCreate(&x);
  hipError_t e = layout_user_to_half(geom, UIN, IO, 1, prec, nrhs, c->stream);
  if (e == hipSuccess && ev[0]) e = hipEventRecord(ev[0], c->stream);
  if (e == hipSuccess && split_mask != 0) e = dd_pack(D, prec, c->stream);
  if (e == hipSuccess && ev[1]) e = hipEventRecord(ev[1], c->stream);
  if (e == hipSuccess) {
    Prog p = prog_HOP(0, false);
    p.split = split_mask;
    e = run_prog(c, g, geom, prec, p, IO, nullptr, OE, coef_d, nrhs, nullptr, 0, nullptr, 0, cls, false);
  }
  if (e == hipSuccess && ev[2]) e = hipEventRecord(ev[2], c->stream);
  if (e == hipSuccess && split_mask != 0) e = dd_exterior(D, prec, c->stream);
  if (e == hipSuccess && ev[3]) e = hipEventRecord(ev[3], c->stream);
  if (e == hipSuccess) {
    e = layout_half_to_user(geom, OE, UOUT, 0, prec, nrhs, c->stream);
    if (e == hipSuccess) e = layout_half_to_user(geom, NUL, UOUT, 1, prec, nrhs, c->stream);
  }
  if (phase_ms != nullptr) {
    if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
    for (int k = 0; k < 3; ++k) {
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      phase_ms[k] = ms;
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
  }
  return hip_err(c, e, "mdwf_hop_split");
}
