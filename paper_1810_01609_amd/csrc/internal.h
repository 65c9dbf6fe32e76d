// Host-side objects of libmdwf (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <map>
#include <string>
#include <vector>

#include "../../include/mdwf.h"
#include "kernels.h"

namespace mdwf {

// grow-only device buffer
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

struct ProfRec {
  int cls;
  int pos;        // iteration position within its CG chunk, -1 outside the loop
  int64_t chunk;  // CG chunk the launch belongs to (pos >= 0)
  bool idle;      // every slot was frozen at that iteration (set at the poll)
  double bytes;
  hipEvent_t e0, e1;
};

// one fused-operator program (see DslashArgs)
struct Prog {
  bool hop, dag, pro;
  int c1, c2, aux, reduce;
  double coef;
  int out_par;
  int split = 0;  // split_mask of the domain-decomposed interior hop
};

}  // namespace mdwf

struct mdwf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // profiling
  int prof = 0;            // 0 off, 1 every launch, N > 1 one CG iteration in N
  bool prof_skip = false;  // inside a CG iteration that is not sampled
  int64_t prof_iter = 0;   // CG iterations seen while sampling
  // CG loop accounting: launches and bytes of the current chunk per iteration
  // position, committed at the poll with the fraction of slots that were
  // still iterating (launches where every slot was frozen do no work and are
  // left out of both the time and the byte totals)
  int prof_pos = -1;          // position in the current chunk, -1 outside the loop
  int64_t prof_chunk = 0;     // current chunk id
  int64_t prof_committed = 0; // chunks whose positions are known
  std::vector<double> prof_chunk_n, prof_chunk_b;  // [pos * NCLASS + cls]
  std::vector<mdwf::ProfRec> pending;
  std::vector<hipEvent_t> events;
  // per class and stratum (0 outside the CG loop, 1 inside): launches,
  // timed launches, timed ms, modelled bytes
  int64_t prof_launches[MDWF_PROF_NCLASS][2] = {};
  int64_t prof_timed[MDWF_PROF_NCLASS][2] = {};
  double prof_ms[MDWF_PROF_NCLASS][2] = {};
  double prof_bytes[MDWF_PROF_NCLASS][2] = {};
  // autotuner: key -> log2 of sites per workgroup
  int tune_mode = 0;
  std::map<std::string, int> tune;
  std::map<std::string, float> tune_ms;
  // device scratch
  mdwf::DevBuf tables;     // pointer tables / small arrays, bump-allocated per call
  void* tables_host = nullptr;  // pinned mirror of `tables`
  size_t tables_used = 0;
  size_t tables_floor = 0;  // bytes below which a wrapped region must not reuse (tables a running loop still reads)
  hipEvent_t tables_ev = nullptr;  // recorded after the latest table upload
  mdwf::DevBuf partials_d; // dslash 16-site tile partials
  mdwf::DevBuf partials_b; // blas block partials
  mdwf::DevBuf states;     // CGState per fused slot
  mdwf::DevBuf coefs;      // Coef5 per slot
  mdwf::DevBuf red_out;    // reduced doubles
  mdwf::DevBuf tmp64[3];   // FP64 half-field temporaries (setup, updates, finalize)
  mdwf::DevBuf dws;        // operator workspace of mdwf_dslash
  mdwf::DevBuf job_cache;  // the block of the last mdwf_solve, reused by the next one
  bool solve_cache = false;  // set while mdwf_solve begins its job
  double* red_host = nullptr;  // pinned
  size_t red_host_n = 0;
  mdwf::CGState* st_host = nullptr;  // pinned
  size_t st_host_n = 0;
};

struct mdwf_gauge {
  mdwf_ctx* ctx = nullptr;
  int L[4] = {0, 0, 0, 0};
  int Vh = 0;
  void* data[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // per precision
  size_t bytes = 0;
};

struct mdwf_job {
  mdwf_ctx* ctx = nullptr;
  const mdwf_gauge* g = nullptr;
  mdwf_action act{};
  mdwf_cg_opts opts{};
  int nrhs = 0;
  mdwf::Geom geom{};
  int ps = 0, px = 0;  // inner spinor precision, inner solution precision
  const char* eta = nullptr;
  char* psi = nullptr;
  size_t user_bytes = 0;  // bytes of one user-layout RHS
  mdwf::Coef5 coef{};
  void* block = nullptr;
  size_t block_bytes = 0;
  bool keep_block = false;  // mdwf_solve: on mdwf_job_end the block goes back to the context's cache
  std::vector<char*> fx, fr, fp, fpt, ft, fv, fxh, feh;  // fpt = M_phi p
  std::vector<mdwf::CGState> st;
  std::vector<mdwf_cg_stats> stats;
  std::vector<int> finished;
  double t0 = 0;
  double bytes_iter = 0, flops_iter = 0;  // model, per RHS per iteration
};

namespace mdwf {

// error helpers
mdwf_status set_err(mdwf_ctx* c, mdwf_status s, const char* fmt, ...);
mdwf_status hip_err(mdwf_ctx* c, hipError_t e, const char* what);

// validation
mdwf_status check_action_msg(const mdwf_action* a, std::string& msg);
Geom make_geom(const mdwf_action* a);
Coef5 make_coef(const mdwf_action* a);

// device memory
mdwf_status ensure(mdwf_ctx* c, DevBuf& b, size_t n);
void release(DevBuf& b);
// upload a pointer table / small array (stream-ordered); returns device address
char* const* upload_table(mdwf_ctx* c, const std::vector<const void*>& ptrs);
void* upload_bytes(mdwf_ctx* c, const void* data, size_t n);
void reset_tables(mdwf_ctx* c);

// CG update fused into a stencil launch (see DslashArgs::cg_update)
struct CgFuse {
  char* const* x;
  char* const* r;
  char* const* p;
  const CGState* st;
  int mode;  // DslashArgs::cg_update
};

// launches with profiling
hipError_t run_prog(mdwf_ctx* c, const mdwf_gauge* g, const Geom& geom, int prec, const Prog& pr,
                    char* const* in, char* const* aux, char* const* out, const Coef5* coef_d, int nslots,
                    const int* active, int active_stride, double* partials, int ntiles, int cls, bool tunable,
                    const CgFuse* fuse = nullptr);
// 1 when a launch over nslots fields of this size should store with
// streaming (non-temporal) writes
int streaming_stores(const Geom& g, int prec, int nslots);
void prof_begin(mdwf_ctx* c, hipEvent_t* e0);
void prof_end(mdwf_ctx* c, int cls, double bytes, hipEvent_t e0);
// CG loop accounting (see mdwf_ctx): a chunk of `chunk` iterations starts;
// after the poll, active_frac[pos] is the fraction of slots that iterated at
// position pos
void prof_chunk_begin(mdwf_ctx* c, int chunk);
void prof_chunk_commit(mdwf_ctx* c, const std::vector<double>& active_frac);
// With `device` current: record this device's address of the scratch array
// behind mdwf_dslash_noalloc (called once per context creation; idempotent).
void scratch_init(int device);

}  // namespace mdwf
