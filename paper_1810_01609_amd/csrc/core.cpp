// libmdwf host core: contexts, validation, device memory, pointer tables,
// profiling, the launch autotuner, gauge fields and sources.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "internal.h"

using namespace mdwf;

namespace mdwf {

mdwf_status set_err(mdwf_ctx* c, mdwf_status s, const char* fmt, ...) {
  if (c != nullptr) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

mdwf_status hip_err(mdwf_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return MDWF_OK;
  // a failed runtime call (a hipMalloc out of memory, say) also leaves the
  // thread's last-error state set; clear it, or the next launch's
  // hipGetLastError check would report this error again
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory) return set_err(c, MDWF_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_err(c, MDWF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

mdwf_status check_action_msg(const mdwf_action* a, std::string& msg) {
  if (a == nullptr) {
    msg = "action is NULL";
    return MDWF_EINVAL;
  }
  const char* nm[4] = {"Lx", "Ly", "Lz", "Lt"};
  for (int m = 0; m < 4; ++m) {
    if (a->L[m] < 2) {
      msg = std::string(nm[m]) + " must be >= 2";
      return MDWF_EINVAL;
    }
  }
  if (a->L[0] % 2 != 0) {
    msg = "Lx must be even (checkerboard indexing)";
    return MDWF_EINVAL;
  }
  const double v4 = (double)a->L[0] * a->L[1] * a->L[2] * a->L[3];
  if (v4 * (a->L5 > 0 ? a->L5 : 1) > 2.0e9) {
    msg = "lattice too large (V4*L5 must stay below 2^31)";
    return MDWF_EINVAL;
  }
  {
    // site coordinates divide checkerboard indices (< V4/2) by Lx/2, Ly, Lz
    // with 32-bit multiply-high, exact while index * divisor < 2^32
    const double dmax = std::max({(double)a->L[0] / 2, (double)a->L[1], (double)a->L[2]});
    if (v4 / 2 * dmax >= 4294967296.0) {
      msg = "lattice too large (V4/2 * max(Lx/2, Ly, Lz) must stay below 2^32)";
      return MDWF_EINVAL;
    }
  }
  if (a->L5 < 1 || a->L5 > 32) {
    msg = "L5 must be in [1, 32]";
    return MDWF_EINVAL;
  }
  if (!std::isfinite(a->b5) || !std::isfinite(a->c5) || !std::isfinite(a->M5) || !std::isfinite(a->mq)) {
    msg = "b5, c5, M5, mq must be finite";
    return MDWF_EINVAL;
  }
  if (a->mq < 0) {
    msg = "mq must be >= 0";
    return MDWF_EINVAL;
  }
  const double alpha = a->b5 * (4.0 - a->M5) + 1.0;
  if (alpha == 0.0) {
    msg = "b5*(4-M5)+1 must be nonzero";
    return MDWF_EINVAL;
  }
  const double kappa = (a->c5 * (4.0 - a->M5) - 1.0) / alpha;
  if (1.0 + a->mq * std::pow(-kappa, a->L5) == 0.0) {
    msg = "M5 is singular for these parameters";
    return MDWF_EINVAL;
  }
  if (a->t_antiperiodic != 0 && a->t_antiperiodic != 1) {
    msg = "t_antiperiodic must be 0 or 1";
    return MDWF_EINVAL;
  }
  return MDWF_OK;
}

Geom make_geom(const mdwf_action* a) {
  Geom g;
  g.Lx = a->L[0];
  g.Ly = a->L[1];
  g.Lz = a->L[2];
  g.Lt = a->L[3];
  g.Lxh = a->L[0] / 2;
  g.Vh = a->L[0] * a->L[1] * a->L[2] * a->L[3] / 2;
  g.L5 = a->L5;
  g.tap = a->t_antiperiodic;
  g.mLxh = fastdiv_magic((uint32_t)g.Lxh);
  g.mLy = fastdiv_magic((uint32_t)g.Ly);
  g.mLz = fastdiv_magic((uint32_t)g.Lz);
  return g;
}

Coef5 make_coef(const mdwf_action* a) {
  Coef5 c;
  c.b5 = a->b5;
  c.c5 = a->c5;
  c.mq = a->mq;
  c.alpha = a->b5 * (4.0 - a->M5) + 1.0;
  c.beta = a->c5 * (4.0 - a->M5) - 1.0;
  c.kappa = c.beta / c.alpha;
  c.inv_alpha = 1.0 / c.alpha;
  c.inv_c = 1.0 / (1.0 + a->mq * std::pow(-c.kappa, a->L5));
  return c;
}

mdwf_status ensure(mdwf_ctx* c, DevBuf& b, size_t n) {
  if (b.n >= n) return MDWF_OK;
  if (b.p != nullptr) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_err(c, e, "hipStreamSynchronize");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
  }
  const size_t want = round_up(n, 4096);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return hip_err(c, e, "hipMalloc (workspace)");
  }
  b.n = want;
  return MDWF_OK;
}

void release(DevBuf& b) {
  if (b.p != nullptr) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
}

static constexpr size_t kTableBytes = 1 << 20;

// Small uploads (pointer tables, coefficients) go through a pinned mirror of
// a device region, bump-allocated per top-level call.  A region offset is
// rewritten only after the copies of the previous call have executed
// (reset_tables waits for the event recorded after the latest upload).
void reset_tables(mdwf_ctx* c) {
  if (c->tables_ev != nullptr) (void)hipEventSynchronize(c->tables_ev);
  c->tables_used = 0;
  c->tables_floor = 0;
}

void* upload_bytes(mdwf_ctx* c, const void* data, size_t n) {
  const size_t bytes = round_up(n > 0 ? n : 1, 256);
  if (c->tables.p == nullptr) {
    if (ensure(c, c->tables, kTableBytes) != MDWF_OK) return nullptr;
    if (hipHostMalloc(&c->tables_host, kTableBytes, hipHostMallocDefault) != hipSuccess) {
      c->tables_host = nullptr;
      return nullptr;
    }
    if (hipEventCreateWithFlags(&c->tables_ev, hipEventDisableTiming) != hipSuccess) return nullptr;
  }
  if (bytes > kTableBytes) return nullptr;
  if (c->tables_used + bytes > kTableBytes) {
    // exhausted within one call: drain the stream, then start over above the
    // tables the running CG loop keeps reading (tables_floor)
    (void)hipStreamSynchronize(c->stream);
    c->tables_used = c->tables_floor;
    if (c->tables_used + bytes > kTableBytes) return nullptr;
  }
  char* dst = static_cast<char*>(c->tables.p) + c->tables_used;
  char* src = static_cast<char*>(c->tables_host) + c->tables_used;
  c->tables_used += bytes;
  memcpy(src, data, n);
  if (hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream) != hipSuccess) return nullptr;
  (void)hipEventRecord(c->tables_ev, c->stream);
  return dst;
}

char* const* upload_table(mdwf_ctx* c, const std::vector<const void*>& ptrs) {
  return static_cast<char* const*>(upload_bytes(c, ptrs.data(), ptrs.size() * sizeof(void*)));
}

static hipEvent_t get_event(mdwf_ctx* c) {
  if (!c->events.empty()) {
    hipEvent_t e = c->events.back();
    c->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

LaunchTiming& launch_timing() {
  static thread_local LaunchTiming t;
  return t;
}

void prof_begin(mdwf_ctx* c, hipEvent_t* e0) {
  *e0 = nullptr;
  if (!c->prof || c->prof_skip) return;
  *e0 = get_event(c);
  LaunchTiming& t = launch_timing();
  t.start = *e0;
  t.stop = get_event(c);
  t.launches = 0;
}

// fold the finished records whose chunk has been committed (all records when
// the loop is not running); returns their events to the pool
static void fold_records(mdwf_ctx* c) {
  std::vector<ProfRec> keep;
  for (auto& r : c->pending) {
    if (r.pos >= 0 && r.chunk > c->prof_committed) {
      keep.push_back(r);
      continue;
    }
    if (!r.idle) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, r.e0, r.e1);
      const int sr = r.pos >= 0 ? 1 : 0;
      if (sr == 0) {  // launches and bytes of the loop stratum come from the chunk commit
        c->prof_launches[r.cls][0] += 1;
        c->prof_bytes[r.cls][0] += r.bytes;
      }
      c->prof_timed[r.cls][sr] += 1;
      c->prof_ms[r.cls][sr] += ms;
    }
    c->events.push_back(r.e0);
    c->events.push_back(r.e1);
  }
  c->pending.swap(keep);
}

void prof_end(mdwf_ctx* c, int cls, double bytes, hipEvent_t e0) {
  if (!c->prof) return;
  const int pos = c->prof_pos;
  if (pos >= 0) {  // inside the CG loop: counted per position until the poll
    const size_t k = (size_t)pos * MDWF_PROF_NCLASS + cls;
    if (k < c->prof_chunk_n.size()) {
      c->prof_chunk_n[k] += 1;
      c->prof_chunk_b[k] += bytes;
    }
  }
  if (e0 == nullptr) return;  // an iteration that is not sampled: counted, not timed
  LaunchTiming& t = launch_timing();
  hipEvent_t e1 = t.stop;
  const int n = t.launches;
  t = LaunchTiming{};
  if (n == 0) {  // nothing was launched: no record
    c->events.push_back(e0);
    c->events.push_back(e1);
    return;
  }
  c->pending.push_back(ProfRec{cls, pos, c->prof_chunk, false, bytes, e0, e1});
  if (c->pending.size() > 8192) {
    // keep the event pool bounded
    (void)hipEventSynchronize(e1);
    fold_records(c);
  }
}

void prof_chunk_begin(mdwf_ctx* c, int chunk) {
  if (!c->prof) return;
  c->prof_chunk += 1;
  c->prof_chunk_n.assign((size_t)chunk * MDWF_PROF_NCLASS, 0.0);
  c->prof_chunk_b.assign((size_t)chunk * MDWF_PROF_NCLASS, 0.0);
}

void prof_chunk_commit(mdwf_ctx* c, const std::vector<double>& active_frac) {
  if (!c->prof) return;
  const int npos = (int)(c->prof_chunk_n.size() / MDWF_PROF_NCLASS);
  for (int pos = 0; pos < npos && pos < (int)active_frac.size(); ++pos) {
    const double f = active_frac[pos];
    if (f <= 0.0) continue;
    for (int cls = 0; cls < MDWF_PROF_NCLASS; ++cls) {
      const size_t k = (size_t)pos * MDWF_PROF_NCLASS + cls;
      c->prof_launches[cls][1] += (int64_t)c->prof_chunk_n[k];
      c->prof_bytes[cls][1] += c->prof_chunk_b[k] * f;
    }
  }
  for (auto& r : c->pending)
    if (r.pos >= 0 && r.chunk == c->prof_chunk && (r.pos >= (int)active_frac.size() || active_frac[r.pos] <= 0.0))
      r.idle = true;
  c->prof_committed = c->prof_chunk;
  c->prof_chunk_n.clear();
  c->prof_chunk_b.clear();
}

// ---------------------------------------------------------------------------
// Fused operator launch with the autotuner (the paper's "GPU Kernel
// Autotuning": brute-force search of the launch space the first time a
// kernel/problem key is met, kept in a std::map and looked up afterwards).
// The tunable parameter is the number of sites per workgroup; all candidates
// perform identical per-site arithmetic, and reductions use fixed 16-site
// tiles, so tuning never changes results.  Launches whose output aliases an
// input are not tuned (no backup/restore of destroyed data is needed then).
// ---------------------------------------------------------------------------
static int default_stage();

// The untuned traversal (MDWF_BT and MDWF_YB override; Bt = 0 is the linear
// order, one band is the whole xy-plane).  Measured on three lattices:
//  * fifth dimension up to 12 slices (a workgroup column of at most 192 5D
//    sites): bands of 4 y-rows, Bt = 2.  16^3 x 32: +3 % on the whole solve;
//    32^3 x 64: the stencil 10 % (FP32) / 3 % (FP16) faster for one
//    right-hand side, 24 % / 9 % for 12 fused ones; 1-, 2- and 8-row bands
//    gained less;
//  * longer columns (24^3 x 64, L5 = 16): 4-row bands were 2-3 % slower; whole
//    planes with the largest Bt of 8, 4, 2 whose (Bt + 2) planes of one RHS
//    fit in 3 MB of the XCD's 4 MB L2.
static void traversal(const Geom& g, int prec, int nslots, int& bt, int& yb, int& order) {
  // several RHS: each XCD keeps its eighth of the lattice and walks the RHS
  // one after another there (one RHS's neighbour planes at a time in its L2).
  // Against the RHS of a site block side by side, on 32^3 x 64, L5 = 12, 12
  // RHS: FP32 M^+M^ 7 % faster, FP16 2 %, HBM fetch of the hop 18 % lower.
  order = nslots > 1 ? 2 : 0;
  const bool bands = g.L5 <= 12 && g.Ly % 4 == 0 && g.Ly / 4 > 1 && g.Lt % 2 == 0;
  if (bands) {
    bt = 2;
    yb = g.Ly / 4;
  } else {
    yb = 1;
    bt = g.Lt % 2 == 0 ? 2 : 0;
    const double plane_bytes = (double)g.Lxh * g.Ly * g.L5 * spinor_site_bytes(prec);
    for (int b : {8, 4}) {
      if (g.Lt % b == 0 && (b + 2) * plane_bytes * (nslots > 4 ? 4 : nslots) <= 3.0e6) {
        bt = b;
        break;
      }
    }
  }
  // overrides: Bt >= 0 (0 = linear order), band count >= 1; other values are ignored
  const char* e = getenv("MDWF_BT");
  if (e != nullptr && e[0] != 0 && atoi(e) >= 0) bt = atoi(e);
  e = getenv("MDWF_YB");
  if (e != nullptr && e[0] != 0 && atoi(e) >= 1) yb = atoi(e);
  e = getenv("MDWF_RHS_ORDER");
  if (e != nullptr && e[0] != 0 && atoi(e) >= 0 && atoi(e) <= 2) order = atoi(e);
}

// Streaming stores once the launch's output fields no longer fit the 256 MB
// MALL together with the fields a CG iteration cycles through (MDWF_NT
// overrides): +2-4 % on the stencil at 24^3 x 64 and 32^3 x 64; on 16^3 x 32
// (37.7 MB per FP32 half-field) the fields stay cache-resident, and streaming
// stores would evict them.
int streaming_stores(const Geom& g, int prec, int nslots) {
  const char* e = getenv("MDWF_NT");
  if (e != nullptr && e[0] != 0) return atoi(e) != 0;
  const double half = (double)g.Vh * g.L5 * spinor_site_bytes(prec);
  return nslots * half > 48.0e6 ? 1 : 0;
}

static std::string tune_key(const Geom& g, int prec, const Prog& p, int nslots, int cg) {
  char buf[256];
  snprintf(buf, sizeof(buf), "dslash5 p%d h%d d%d pr%d c%d.%d a%d r%d u%d s%d L%dx%dx%dx%d L5=%d n%d gfx950",
           prec, (int)p.hop, (int)p.dag, (int)p.pro, p.c1, p.c2, p.aux, p.reduce, (int)cg,
           p.hop ? default_stage() : 0, g.Lx, g.Ly, g.Lz, g.Lt, g.L5, nslots);
  std::string k = buf;
  if (p.split != 0) k += " x" + std::to_string(p.split);
  return k;
}

// Launch candidates: log2 of sites per workgroup (bits 0-7); bit 8 carries
// the LDS staging of links / neighbour indices, which is fixed per process
// (MDWF_STAGE, default on) and not searched: the staged and unstaged kernels
// round differently in the last bit (their multiply-adds are contracted
// differently), and tuning must never change a result.
static int default_stage() {
  const char* e = getenv("MDWF_STAGE");
  return (e != nullptr && e[0] == '0') ? 0 : 1;
}

// A candidate's code: log2 sites per workgroup (bits 0-7), LDS staging (bit
// 8), and the traversal of the hop kernels: Bt + 1 (bits 12-15) and the y-band
// count (bits 16-23) and the RHS order + 1 (bits 24-25), where 0 keeps the
// size-based default.  The traversal only reorders whole workgroups, so every
// candidate gives the same result.
constexpr int kTravBtShift = 12, kTravYbShift = 16, kRhsOrderShift = 24;

static void candidates(const Geom& g, int prec, DslashArgs A, bool hop, std::vector<int>& out, int& dflt) {
  out.clear();
  dflt = -1;
  const int stage = hop ? default_stage() : 0;
  A.stage = stage;
  std::vector<int> trav{0};
  if (hop) {
    std::vector<int> ybs{1};
    if (g.Ly % 4 == 0 && g.Ly / 4 > 1) ybs.push_back(g.Ly / 4);
    for (int bt : {2, 4, 8}) {
      if (g.Lt % bt != 0) continue;
      for (int yb : ybs) trav.push_back(((bt + 1) << kTravBtShift) | (yb << kTravYbShift));
    }
    if (A.nslots > 1) {  // both RHS orders for every traversal
      const size_t n = trav.size();
      for (size_t i = 0; i < n; ++i)
        for (int o : {0, 2}) trav.push_back(trav[i] | ((o + 1) << kRhsOrderShift));
    }
  }
  for (int lg = 4; lg <= 7; ++lg) {
    const int CB = 1 << lg;
    if (CB * g.L5 > dslash_max_threads(prec)) break;
    if (CB > 2 * g.Vh && lg > 4) break;
    const size_t lds = dslash_lds_bytes(A, prec, lg, hop);
    if (lds > 160 * 1024) break;
    for (int t : trav) out.push_back(lg | (stage << 8) | t);
  }
  // untuned default: the smallest workgroup (16 sites x L5 slices) — it packs
  // the most resident waves per CU under the LDS and register limits, and the
  // tuner picks it for nearly every kernel and lattice measured — with the
  // size-based traversal.  MDWF_CB_LOG2 (4..7) picks another workgroup width
  // for the untuned launch when the kernel admits it (so every candidate the
  // tuner may choose can be run and checked on its own).
  if (!out.empty()) dflt = out.front();
  const char* e = getenv("MDWF_CB_LOG2");
  if (e != nullptr && e[0] != 0)
    for (int code : out)
      if ((code & 0xff) == atoi(e) && (code >> kTravBtShift) == 0) {
        dflt = code;
        break;
      }
}

static void apply_candidate(DslashArgs& A, int code) {
  A.stage = (code >> 8) & 1;
  const int bt1 = (code >> kTravBtShift) & 0xf;
  const int yb = (code >> kTravYbShift) & 0xff;
  const int ord1 = (code >> kRhsOrderShift) & 3;
  if (bt1 != 0) A.order_bt = bt1 - 1;
  if (yb != 0) A.order_yb = yb;
  if (ord1 != 0) A.rhs_order = ord1 - 1;
}

static double prog_bytes(const Geom& g, int prec, const Prog& p, int nslots, int cg) {
  const double ne = (double)g.Vh * g.L5;
  const double sb = spinor_site_bytes(prec);
  const double xs = spinor_site_bytes(prec == F64 ? F64 : F32) / sb;
  // in + out (+ aux); the fused CG update reads r and writes r instead of
  // out (+ reads p, reads and writes x), or adds p and x to a plain launch
  double per = 2.0 + (p.aux != AUX_NONE ? 1.0 : 0.0);
  if (cg == 1) per += 2.0 + 2.0 * xs;
  if (cg == 2) per += 1.0;
  if (cg == 3) per += 1.0 + 2.0 * xs;
  double b = nslots * ne * sb * per;
  if (p.hop) b += 8.0 * g.Vh * 12.0 * link_real_bytes(prec);
  return b;
}

hipError_t run_prog(mdwf_ctx* c, const mdwf_gauge* gf, const Geom& geom, int prec, const Prog& pr,
                    char* const* in, char* const* aux, char* const* out, const Coef5* coef_d, int nslots,
                    const int* active, int active_stride, double* partials, int ntiles, int cls, bool tunable,
                    const CgFuse* fuse) {
  DslashArgs A{};
  A.g = geom;
  A.out_par = pr.out_par;
  A.gauge = gf != nullptr ? static_cast<const char*>(gf->data[prec]) : nullptr;
  A.in = in;
  A.aux = aux;
  A.out = out;
  A.coef = coef_d;
  A.active = active;
  A.active_stride = active_stride;
  A.partials = partials;
  A.ntiles = ntiles;
  A.nslots = nslots;
  A.c1 = pr.c1;
  A.c2 = pr.c2;
  A.aux_mode = pr.aux;
  A.reduce = pr.reduce;
  A.coef_y = pr.coef;
  traversal(geom, prec, nslots, A.order_bt, A.order_yb, A.rhs_order);
  A.nt_store = streaming_stores(geom, prec, nslots);
  A.split_mask = pr.split;
  if (fuse != nullptr) {
    A.cg_update = fuse->mode;
    A.cg_x = fuse->x;
    A.cg_r = fuse->r;
    A.cg_p = fuse->p;
    A.cg_st = fuse->st;
  }
  std::vector<int> cand;
  int dflt = 4;
  candidates(geom, prec, A, pr.hop, cand, dflt);
  if (cand.empty()) return hipErrorInvalidValue;
  int lg = dflt;
  const std::string key = tune_key(geom, prec, pr, nslots, fuse != nullptr ? fuse->mode : 0);
  // the fused CG update is destructive (x, r in place): never tuned on live data
  if (fuse != nullptr) tunable = false;
  auto it = c->tune.find(key);
  if (it != c->tune.end()) {
    lg = it->second;
  } else if (c->tune_mode == 1 && tunable && cand.size() > 1) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    int best_lg = dflt;
    const DslashArgs A0 = A;
    for (int cl : cand) {
      DslashArgs B = A0;
      apply_candidate(B, cl);
      hipError_t e = dslash_launch(B, prec, pr.hop, pr.dag, pr.pro, cl & 0xff, c->stream);  // warm-up
      if (e != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < 3; ++r) (void)dslash_launch(B, prec, pr.hop, pr.dag, pr.pro, cl & 0xff, c->stream);
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        best_lg = cl;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    lg = best_lg;
    c->tune[key] = lg;
    c->tune_ms[key] = best / 3.0f;
  }
  hipEvent_t ev;
  prof_begin(c, &ev);
  apply_candidate(A, lg);
  hipError_t e = dslash_launch(A, prec, pr.hop, pr.dag, pr.pro, lg & 0xff, c->stream);
  prof_end(c, cls, prog_bytes(geom, prec, pr, nslots, fuse != nullptr ? fuse->mode : 0), ev);
  return e;
}

}  // namespace mdwf

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t mdwf_abi_version(void) { return MDWF_ABI_VERSION; }

mdwf_status mdwf_check_action(const mdwf_action* act, char* msg, size_t msg_len) {
  std::string m;
  mdwf_status s = check_action_msg(act, m);
  if (msg != nullptr && msg_len > 0) {
    snprintf(msg, msg_len, "%s", m.c_str());
  }
  return s;
}

mdwf_status mdwf_query_traversal(const mdwf_action* act, int32_t prec, int32_t nrhs, int32_t cb_log2, int32_t* bt,
                                 int32_t* yb) {
  std::string m;
  if (check_action_msg(act, m) != MDWF_OK || bt == nullptr || yb == nullptr) return MDWF_EINVAL;
  if (prec < MDWF_F64 || prec > MDWF_I16 || nrhs < 1 || cb_log2 < 4 || cb_log2 > 7) return MDWF_EINVAL;
  const Geom g = make_geom(act);
  int b = 0, y = 1, o = 0;
  traversal(g, prec, nrhs, b, y, o);
  clamp_traversal(g, 1 << cb_log2, b, y);
  *bt = b;
  *yb = y;
  return MDWF_OK;
}

mdwf_status mdwf_create(int32_t device, void* stream, mdwf_ctx** out) {
  if (out == nullptr) return MDWF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MDWF_EHIP;
  if (device < 0 || device >= n) return MDWF_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return MDWF_EHIP;
  mdwf_ctx* c = new (std::nothrow) mdwf_ctx();
  if (c == nullptr) return MDWF_ENOMEM;
  c->device = device;
  scratch_init(device);  // this device's address of the no-allocation scratch
  if (stream != nullptr) {
    c->stream = static_cast<hipStream_t>(stream);
    c->own_stream = false;
  } else {
    // a blocking stream: it stays ordered with the legacy default stream,
    // where torch enqueues its work unless told otherwise
    if (hipStreamCreateWithFlags(&c->stream, hipStreamDefault) != hipSuccess) {
      delete c;
      return MDWF_EHIP;
    }
    c->own_stream = true;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->red_host), 4096 * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MDWF_ENOMEM;
  }
  c->red_host_n = 4096;
  const char* tm = getenv("MDWF_TUNE");
  if (tm != nullptr && tm[0] == '1') c->tune_mode = 1;
  const char* tc = getenv("MDWF_TUNE_CACHE");
  if (tc != nullptr && tc[0] != 0) (void)mdwf_tune_load(c, tc);
  *out = c;
  return MDWF_OK;
}

mdwf_status mdwf_trim(mdwf_ctx* c) {
  if (c == nullptr) return MDWF_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  release(c->job_cache);
  release(c->dws);
  for (auto& b : c->tmp64) release(b);
  return MDWF_OK;
}

mdwf_status mdwf_destroy(mdwf_ctx* c) {
  if (c == nullptr) return MDWF_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& r : c->pending) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (auto e : c->events) (void)hipEventDestroy(e);
  release(c->tables);
  if (c->tables_host != nullptr) (void)hipHostFree(c->tables_host);
  if (c->tables_ev != nullptr) (void)hipEventDestroy(c->tables_ev);
  release(c->partials_d);
  release(c->partials_b);
  release(c->states);
  release(c->coefs);
  release(c->red_out);
  for (auto& b : c->tmp64) release(b);
  release(c->dws);
  release(c->job_cache);
  if (c->red_host != nullptr) (void)hipHostFree(c->red_host);
  if (c->st_host != nullptr) (void)hipHostFree(c->st_host);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  const char* tc = getenv("MDWF_TUNE_CACHE");
  if (tc != nullptr && tc[0] != 0 && !c->tune.empty()) (void)mdwf_tune_save(c, tc);
  delete c;
  return MDWF_OK;
}

const char* mdwf_last_error(const mdwf_ctx* c) { return c == nullptr ? "null context" : c->err.c_str(); }

void* mdwf_stream(const mdwf_ctx* c) { return c == nullptr ? nullptr : static_cast<void*>(c->stream); }

mdwf_status mdwf_gauge_load(mdwf_ctx* c, const int32_t L[4], const void* links, int32_t where, uint32_t prec_mask,
                            mdwf_gauge** out) {
  if (c == nullptr) return MDWF_EINVAL;
  if (out == nullptr || L == nullptr || links == nullptr)
    return set_err(c, MDWF_EINVAL, "mdwf_gauge_load: NULL argument");
  *out = nullptr;
  if (where != MDWF_HOST && where != MDWF_DEVICE) return set_err(c, MDWF_EINVAL, "mdwf_gauge_load: bad `where`");
  mdwf_action a{};
  for (int m = 0; m < 4; ++m) a.L[m] = L[m];
  a.L5 = 1;
  a.b5 = 1;
  a.c5 = 0;
  a.M5 = 1;
  a.mq = 0;
  std::string msg;
  if (check_action_msg(&a, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_gauge_load: %s", msg.c_str());
  if (prec_mask & ~0x1fu) return set_err(c, MDWF_EINVAL, "mdwf_gauge_load: prec_mask has unknown bits");
  prec_mask |= 1u << MDWF_F64;
  (void)hipSetDevice(c->device);
  const Geom g = make_geom(&a);
  const size_t user_bytes = (size_t)g.Vh * 2 * 4 * 18 * sizeof(double);
  mdwf_gauge* gf = new (std::nothrow) mdwf_gauge();
  if (gf == nullptr) return set_err(c, MDWF_ENOMEM, "host allocation");
  gf->ctx = c;
  for (int m = 0; m < 4; ++m) gf->L[m] = L[m];
  gf->Vh = g.Vh;
  const double* dev_links = static_cast<const double*>(links);
  void* staging = nullptr;
  hipError_t e;
  if (where == MDWF_HOST) {
    e = hipMalloc(&staging, user_bytes);
    if (e != hipSuccess) {
      delete gf;
      return hip_err(c, e, "hipMalloc (gauge staging)");
    }
    e = hipMemcpyAsync(staging, links, user_bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      (void)hipFree(staging);
      delete gf;
      return hip_err(c, e, "hipMemcpyAsync (gauge)");
    }
    dev_links = static_cast<const double*>(staging);
  }
  mdwf_status st = MDWF_OK;
  for (int p = 0; p < 5 && st == MDWF_OK; ++p) {
    if (!(prec_mask & (1u << p))) continue;
    const size_t nb = gauge_field_bytes(p, g.Vh);
    e = hipMalloc(&gf->data[p], nb);
    if (e != hipSuccess) {
      gf->data[p] = nullptr;
      st = hip_err(c, e, "hipMalloc (gauge)");
      break;
    }
    gf->bytes += nb;
    e = layout_gauge(g, dev_links, static_cast<char*>(gf->data[p]), p, c->stream);
    if (e != hipSuccess) st = hip_err(c, e, "gauge layout kernel");
  }
  e = hipStreamSynchronize(c->stream);
  if (st == MDWF_OK && e != hipSuccess) st = hip_err(c, e, "gauge load");
  if (staging != nullptr) (void)hipFree(staging);
  if (st != MDWF_OK) {
    for (int p = 0; p < 5; ++p)
      if (gf->data[p] != nullptr) (void)hipFree(gf->data[p]);
    delete gf;
    return st;
  }
  *out = gf;
  return MDWF_OK;
}

mdwf_status mdwf_gauge_free(mdwf_gauge* g) {
  if (g == nullptr) return MDWF_EINVAL;
  if (g->ctx != nullptr) {
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
  }
  for (int p = 0; p < 5; ++p)
    if (g->data[p] != nullptr) (void)hipFree(g->data[p]);
  delete g;
  return MDWF_OK;
}

size_t mdwf_gauge_bytes(const mdwf_gauge* g) { return g == nullptr ? 0 : g->bytes; }

mdwf_status mdwf_source_point(mdwf_ctx* c, const mdwf_action* act, const int32_t x0[4], int32_t spin, int32_t colour,
                              void* eta) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_source_point: %s", msg.c_str());
  if (x0 == nullptr || eta == nullptr) return set_err(c, MDWF_EINVAL, "mdwf_source_point: NULL argument");
  for (int m = 0; m < 4; ++m)
    if (x0[m] < 0 || x0[m] >= act->L[m]) return set_err(c, MDWF_EINVAL, "mdwf_source_point: x0 outside the lattice");
  if (spin < 0 || spin > 3 || colour < 0 || colour > 2)
    return set_err(c, MDWF_EINVAL, "mdwf_source_point: spin in [0,4), colour in [0,3)");
  (void)hipSetDevice(c->device);
  const Geom g = make_geom(act);
  int x[4] = {x0[0], x0[1], x0[2], x0[3]};
  hipEvent_t ev;
  prof_begin(c, &ev);
  hipError_t e = source_point(g, static_cast<double*>(eta), x, spin, colour, c->stream);
  prof_end(c, MDWF_PROF_OTHER, (double)g.Vh * 2 * g.L5 * 192, ev);
  return hip_err(c, e, "source_point");
}

mdwf_status mdwf_source_z2(mdwf_ctx* c, const mdwf_action* act, uint64_t seed, int32_t rhs_index, void* eta) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_source_z2: %s", msg.c_str());
  if (eta == nullptr || rhs_index < 0) return set_err(c, MDWF_EINVAL, "mdwf_source_z2: bad argument");
  (void)hipSetDevice(c->device);
  const Geom g = make_geom(act);
  hipEvent_t ev;
  prof_begin(c, &ev);
  hipError_t e = source_z2(g, static_cast<double*>(eta), seed, rhs_index, c->stream);
  prof_end(c, MDWF_PROF_OTHER, (double)g.Vh * 2 * g.L5 * 192, ev);
  return hip_err(c, e, "source_z2");
}

mdwf_status mdwf_propagator_4d(mdwf_ctx* c, const mdwf_action* act, int32_t nrhs, const void* psi, void* q) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_propagator_4d: %s", msg.c_str());
  if (psi == nullptr || q == nullptr || nrhs < 1) return set_err(c, MDWF_EINVAL, "mdwf_propagator_4d: bad argument");
  (void)hipSetDevice(c->device);
  const Geom g = make_geom(act);
  hipEvent_t ev;
  prof_begin(c, &ev);
  hipError_t e = propagator_4d(g, nrhs, static_cast<const double*>(psi), static_cast<double*>(q), c->stream);
  prof_end(c, MDWF_PROF_OTHER, (double)nrhs * g.Vh * 2 * 12 * 32, ev);
  return hip_err(c, e, "propagator_4d");
}

mdwf_status mdwf_current_source(mdwf_ctx* c, const mdwf_action* act, int32_t nrhs, int32_t gamma_mask, const void* q,
                                void* eta) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_current_source: %s", msg.c_str());
  if (q == nullptr || eta == nullptr || nrhs < 1) return set_err(c, MDWF_EINVAL, "mdwf_current_source: bad argument");
  if (gamma_mask < 0 || gamma_mask > 15) return set_err(c, MDWF_EINVAL, "mdwf_current_source: gamma_mask in [0, 15]");
  (void)hipSetDevice(c->device);
  const Geom g = make_geom(act);
  const size_t qb = (size_t)nrhs * g.Vh * 2 * 12 * 16, eb = qb * g.L5;
  const char* qa = static_cast<const char*>(q);
  const char* ea = static_cast<const char*>(eta);
  if (qa < ea + eb && ea < qa + qb) return set_err(c, MDWF_EINVAL, "mdwf_current_source: q and eta overlap");
  hipEvent_t ev;
  prof_begin(c, &ev);
  hipError_t e = current_source(g, nrhs, gamma_mask, static_cast<const double*>(q), static_cast<double*>(eta), c->stream);
  prof_end(c, MDWF_PROF_OTHER, (double)eb + qb, ev);
  return hip_err(c, e, "current_source");
}

mdwf_status mdwf_source_physical(mdwf_ctx* c, const mdwf_gauge* gf, const mdwf_action* act, int32_t nrhs,
                                 int32_t gamma_mask, const void* xi, void* eta) {
  if (c == nullptr) return MDWF_EINVAL;
  std::string msg;
  if (check_action_msg(act, msg) != MDWF_OK) return set_err(c, MDWF_EINVAL, "mdwf_source_physical: %s", msg.c_str());
  if (gf == nullptr || xi == nullptr || eta == nullptr || nrhs < 1)
    return set_err(c, MDWF_EINVAL, "mdwf_source_physical: bad argument");
  if (gamma_mask < 0 || gamma_mask > 15) return set_err(c, MDWF_EINVAL, "mdwf_source_physical: gamma_mask in [0, 15]");
  for (int m = 0; m < 4; ++m)
    if (gf->L[m] != act->L[m])
      return set_err(c, MDWF_EINVAL, "mdwf_source_physical: gauge lattice differs from the action's");
  if (gf->data[MDWF_F64] == nullptr)
    return set_err(c, MDWF_EINVAL, "mdwf_source_physical: the gauge field must be loaded in FP64");
  (void)hipSetDevice(c->device);
  const Geom g = make_geom(act);
  const size_t qb = (size_t)nrhs * g.Vh * 2 * 12 * 16, eb = qb * g.L5;
  const char* qa = static_cast<const char*>(xi);
  const char* ea = static_cast<const char*>(eta);
  if (qa < ea + eb && ea < qa + qb) return set_err(c, MDWF_EINVAL, "mdwf_source_physical: xi and eta overlap");
  const double beta = 1.0 - act->c5 * (4.0 - act->M5), hc = 0.5 * act->c5;
  hipEvent_t ev;
  prof_begin(c, &ev);
  hipError_t e = source_physical(g, nrhs, gamma_mask, static_cast<const char*>(gf->data[MDWF_F64]),
                                 static_cast<const double*>(xi), static_cast<double*>(eta), beta, hc, c->stream);
  prof_end(c, MDWF_PROF_OTHER, (double)eb + qb, ev);
  return hip_err(c, e, "source_physical");
}

mdwf_status mdwf_copy_bandwidth(mdwf_ctx* c, const void* src, void* dst, size_t bytes, int32_t reps, double* gbs) {
  if (c == nullptr) return MDWF_EINVAL;
  if (src == nullptr || dst == nullptr || gbs == nullptr || reps < 1 || bytes == 0 || bytes % 16 != 0)
    return set_err(c, MDWF_EINVAL, "mdwf_copy_bandwidth: bad argument");
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + bytes && b < a + bytes) return set_err(c, MDWF_EINVAL, "mdwf_copy_bandwidth: src and dst overlap");
  (void)hipSetDevice(c->device);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = copy16(src, dst, bytes / 16, c->stream);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = copy16(src, dst, bytes / 16, c->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_err(c, e, "mdwf_copy_bandwidth");
  *gbs = ms > 0 ? 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
  return MDWF_OK;
}

mdwf_status mdwf_profile_enable(mdwf_ctx* c, int32_t on) {
  if (c == nullptr) return MDWF_EINVAL;
  if (on < 0) return set_err(c, MDWF_EINVAL, "mdwf_profile_enable: negative mode");
  c->prof = on;
  c->prof_skip = false;
  c->prof_pos = -1;
  c->prof_iter = 0;
  return MDWF_OK;
}

static void fold_profile(mdwf_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  fold_records(c);
}

mdwf_status mdwf_profile_reset(mdwf_ctx* c) {
  if (c == nullptr) return MDWF_EINVAL;
  fold_profile(c);
  // records of a chunk that never reached its poll (an error path) are dropped
  for (auto& r : c->pending) {
    c->events.push_back(r.e0);
    c->events.push_back(r.e1);
  }
  c->pending.clear();
  c->prof_committed = c->prof_chunk;
  for (int k = 0; k < MDWF_PROF_NCLASS; ++k)
    for (int sr = 0; sr < 2; ++sr) {
      c->prof_launches[k][sr] = 0;
      c->prof_timed[k][sr] = 0;
      c->prof_ms[k][sr] = 0;
      c->prof_bytes[k][sr] = 0;
    }
  return MDWF_OK;
}

mdwf_status mdwf_profile_read(mdwf_ctx* c, int32_t cls, int64_t* launches, double* ms, double* bytes) {
  if (c == nullptr) return MDWF_EINVAL;
  if (cls < 0 || cls >= MDWF_PROF_NCLASS) return set_err(c, MDWF_EINVAL, "profile class out of range");
  fold_profile(c);
  // per stratum, the timed launches' mean times the stratum's launches (the
  // plain sum where every launch was timed)
  int64_t n = 0;
  double t_ms = 0, b = 0;
  for (int sr = 0; sr < 2; ++sr) {
    const int64_t t = c->prof_timed[cls][sr];
    n += c->prof_launches[cls][sr];
    b += c->prof_bytes[cls][sr];
    if (t > 0) t_ms += c->prof_ms[cls][sr] * ((double)c->prof_launches[cls][sr] / (double)t);
  }
  if (launches) *launches = n;
  if (ms) *ms = t_ms;
  if (bytes) *bytes = b;
  return MDWF_OK;
}

mdwf_status mdwf_tune_mode(mdwf_ctx* c, int32_t mode) {
  if (c == nullptr) return MDWF_EINVAL;
  if (mode != 0 && mode != 1) return set_err(c, MDWF_EINVAL, "tune mode must be 0 or 1");
  c->tune_mode = mode;
  return MDWF_OK;
}

mdwf_status mdwf_tune_save(const mdwf_ctx* c, const char* path) {
  if (c == nullptr || path == nullptr) return MDWF_EINVAL;
  std::ofstream f(path);
  if (!f) return MDWF_EINVAL;
  for (auto& kv : c->tune) {
    auto m = c->tune_ms.find(kv.first);
    f << kv.first << " | " << kv.second << " " << (m != c->tune_ms.end() ? m->second : 0.0f) << "\n";
  }
  return MDWF_OK;
}

mdwf_status mdwf_tune_load(mdwf_ctx* c, const char* path) {
  if (c == nullptr || path == nullptr) return MDWF_EINVAL;
  std::ifstream f(path);
  if (!f) return set_err(c, MDWF_EINVAL, "cannot open tune table %s", path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t bar = line.find(" | ");
    if (bar == std::string::npos) continue;
    std::istringstream rest(line.substr(bar + 3));
    int lg = -1;
    float ms = 0;
    rest >> lg >> ms;
    if ((lg & 0xff) >= 4 && (lg & 0xff) <= 7 && ((lg >> 9) & 7) == 0 && ((lg >> kTravBtShift) & 0xf) <= 9 &&
        ((lg >> kRhsOrderShift) & 3) != 2 && (lg >> 26) == 0) {
      c->tune[line.substr(0, bar)] = lg;
      c->tune_ms[line.substr(0, bar)] = ms;
    }
  }
  return MDWF_OK;
}

int32_t mdwf_tune_entries(const mdwf_ctx* c) { return c == nullptr ? 0 : (int32_t)c->tune.size(); }

}  // extern "C"
