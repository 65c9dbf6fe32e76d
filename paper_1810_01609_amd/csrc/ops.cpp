// mdwf_dslash: the operators of the even-odd preconditioned Moebius
// domain-wall system, each built from the fused stencil kernel.
#include <cstring>

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

extern "C" mdwf_status mdwf_dslash(mdwf_ctx* c, const mdwf_gauge* g, const mdwf_action* act, int32_t op,
                                   int32_t prec, int32_t nrhs, const void* in, void* out) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_dslash: %s", msg.c_str());
  if (g == nullptr || in == nullptr || out == nullptr) return set_err(c, MDWF_EINVAL, "mdwf_dslash: NULL argument");
  for (int m = 0; m < 4; ++m)
    if (g->L[m] != act->L[m]) return set_err(c, MDWF_EINVAL, "mdwf_dslash: gauge lattice differs from the action's");
  if (prec < MDWF_F64 || prec > MDWF_I16) return set_err(c, MDWF_EINVAL, "mdwf_dslash: bad precision");
  if (g->data[prec] == nullptr)
    return set_err(c, MDWF_EINVAL, "mdwf_dslash: gauge field was not loaded in precision %d", prec);
  if (op < MDWF_OP_D || op > MDWF_OP_PREP) return set_err(c, MDWF_EINVAL, "mdwf_dslash: bad operator %d", op);
  if (nrhs < 1) return set_err(c, MDWF_EINVAL, "mdwf_dslash: nrhs must be >= 1");
  const Geom geom = make_geom(act);
  const size_t ub = (size_t)geom.Vh * 2 * geom.L5 * 12 * 16;  // user bytes per RHS
  const char* ib = static_cast<const char*>(in);
  char* ob = static_cast<char*>(out);
  if (ib < ob + ub * nrhs && ob < ib + ub * nrhs) return set_err(c, MDWF_EINVAL, "mdwf_dslash: in and out overlap");
  (void)hipSetDevice(c->device);
  reset_tables(c);
  const size_t fb = round_up(spinor_field_bytes(prec, geom.L5, geom.Vh), 256);
  mdwf_status st = ensure(c, c->dws, fb * 5 * nrhs);
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
  char* const* UIN = upload_table(c, uin);
  char* const* UOUT = upload_table(c, uout);
  char* const* IE = upload_table(c, ie);
  char* const* IO = upload_table(c, io);
  char* const* OE = upload_table(c, oe);
  char* const* OO = upload_table(c, oo);
  char* const* T = upload_table(c, tt);
  char* const* NUL = upload_table(c, nul);
  if (!coef_d || !UIN || !UOUT || !IE || !IO || !OE || !OO || !T || !NUL)
    return set_err(c, MDWF_EHIP, "mdwf_dslash: table upload failed");
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
