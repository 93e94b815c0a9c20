// Host runtime of libgalsat: the C ABI declared in include/galsat.h.
//
// galsat_create validates the two CSR orientations, derives the
// occurrence tables the kernels read (per var-major slot: recompute the
// clause, or read a stored partial row), splits variables and clauses into
// work chunks of balanced cost that never cross a formula, and sizes the
// workspace.  The per-call entry points only enqueue kernels on the
// caller's stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "galsat_internal.h"

using namespace galsat;

namespace {

thread_local std::string g_create_error;

constexpr int kDefaultRecomputeMaxLen = 8;
constexpr int kTargetBlocks = 2048;  // blocks per general-pass launch (256 CUs x 8)
// XCD-contiguous order of one formula: chunk count (measured; 2,048 per
// XCD) and the id window that counts as local.
// Workgroups of the LDS schedule up to which every restart gets its own
// (two per CU of the 256).
constexpr int64_t kPersistSpreadGroups = 512;
constexpr int64_t kXseqChunks = 65536;
constexpr int kSegDivSinglePass = 16;  // single-pass segment = one item's share / 16 (measured)
constexpr int kClassShort = 0, kClassWave = 1;  // passes of the stored-clause classes
constexpr int32_t kLocalWindow = 4096;
constexpr int64_t kCacheBudgetBytes = 256ll << 20;  // state rows one launch may gather from
constexpr int kXcds = 8;                            // accelerator complex dies of an MI355X
constexpr int64_t kXcdChunks = 160;                 // workgroups resident on one XCD (about)
constexpr int64_t kXcdChunksTwoPhase = 20;          // measured for the two-phase passes
constexpr int64_t kXcdChunksFlat = 40;              // measured for the flat plan (batch of 4,096)

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

inline int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Runs fn(begin, end) over [0, count) split across host threads (the
// O(L) validation and planning of galsat_create).
template <class Fn>
void parallel_for(int64_t count, Fn fn) {
  int threads = (int)std::thread::hardware_concurrency();
  if (const char* e = std::getenv("OMP_NUM_THREADS")) threads = std::max(1, std::atoi(e));
  threads = std::max(1, std::min(threads, 64));
  if (count < (1 << 16) || threads == 1) {
    fn((int64_t)0, count);
    return;
  }
  std::vector<std::thread> pool;
  for (int i = 0; i < threads; ++i)
    pool.emplace_back(fn, count * i / threads, count * (i + 1) / threads);
  for (auto& t : pool) t.join();
}

// First error found by concurrent checks: the one at the lowest index wins,
// so the message does not depend on thread timing.
struct FirstError {
  std::mutex mu;
  int64_t index = -1;
  std::string msg;
  void report(int64_t i, const std::string& m) {
    std::lock_guard<std::mutex> g(mu);
    if (index < 0 || i < index) {
      index = i;
      msg = m;
    }
  }
};

// Work chunks over per-formula item ranges: consecutive items with total
// cost <= target, never crossing a formula boundary.
struct Chunks {
  std::vector<int32_t> beg, end;   // item range of each chunk
  std::vector<int32_t> f_first;    // [F+1] first chunk of each formula
  int count() const { return (int)beg.size(); }
};

Chunks make_chunks(int F, const std::vector<int64_t>& f_item_beg, const std::vector<int64_t>& cost_prefix,
                   int64_t target_all, const std::vector<int64_t>* f_target = nullptr) {
  Chunks c;
  c.f_first.assign((size_t)F + 1, 0);
  for (int f = 0; f < F; ++f) {
    c.f_first[f] = c.count();
    const int64_t target = std::max<int64_t>(1, f_target ? (*f_target)[f] : target_all);
    int64_t i = f_item_beg[f];
    const int64_t e = f_item_beg[f + 1];
    while (i < e) {
      int64_t j = i + 1;
      // extend while the chunk stays within target
      const int64_t limit = cost_prefix[i] + target;
      int64_t lo = j, hi = e;
      while (lo < hi) {  // largest j in [i+1, e] with prefix[j] <= limit
        int64_t mid = (lo + hi + 1) / 2;
        if (cost_prefix[mid] <= limit) lo = mid; else hi = mid - 1;
      }
      j = std::max(lo, i + 1);
      c.beg.push_back((int32_t)i);
      c.end.push_back((int32_t)j);
      i = j;
    }
  }
  c.f_first[F] = c.count();
  return c;
}

}  // namespace

struct galsat_ctx {
  int device = 0;
  int32_t F = 1, n = 0, m = 0, L = 0, R = 1;
  galsat_options opt{};
  std::string err;
  bool sticky = false;
  int32_t kmax = 0;
  int32_t krec = 0;
  int64_t stored = 0;
  int schedule = GALSAT_SCHED_GENERAL;
  Tile tile;
  int tgroup = 1;    // restart tiles per launch of a gradient pass
  int stream_items = 0;  // streaming variable pass
  int xcd_pin = 0;       // single pass: restart tiles mapped to XCDs
  int two_phase = 0;     // occurrence pass + variable sum instead of the single pass
  int flat = 0;          // flat plan: pair records + clause rows (galsat_flat.hip)
  int prefetch = 1;      // flat plan: next batch's records loaded during this batch's gathers
  int32_t xseq = 0;      // chunks of the XCD-contiguous order (0: off)
  int lds_rg = 0;        // restart group of the persistent LDS schedule (0: not used)
  int lds_stage = 0;     // its occurrence records staged in LDS
  int32_t lds_nocc = 0;  // most occurrences of one formula
  int32_t nf_max = 0;    // most variables of one formula
  int32_t ld = 0;    // internal state row stride (floats)
  int64_t ldD = 0;
  int adam_t = 0;
  size_t device_bytes = 0;
  std::vector<void*> allocs;

  std::vector<int32_t> h_fvb, h_fcb;
  Chunks vch, sch, ach;  // var chunks, stored-clause chunks, all-clause chunks
  Chunks segch;          // chunks of segments of split variables
  Chunks och;            // occurrence-range chunks of the two-phase plan
  Chunks rch;            // chunks of the flat plan's clause-row list
  std::vector<int32_t> heavy_f_first;  // [F+1] split variables of each formula
  int32_t n_heavy = 0, n_seg = 0, step_rows = 0;

  // device tables
  int32_t *clause_ptr = nullptr, *clause_lits = nullptr, *var_ptr = nullptr, *var_occ = nullptr;
  int4* occ4 = nullptr;
  int4* occx = nullptr;
  int32_t *lit_dslot = nullptr, *var_formula = nullptr, *stored_ids = nullptr;
  int32_t *vch_beg = nullptr, *vch_end = nullptr, *vch_row = nullptr, *vch_order = nullptr;
  int32_t n_vorder = 0;  // entries of vch_order (0: launch chunks in index order)
  int32_t *och_beg = nullptr, *och_end = nullptr, *och_row = nullptr, *och_order = nullptr;
  int32_t n_oorder = 0;
  int32_t* occ_own = nullptr;  // [L] variable of each variable-major slot (two-phase)
  int32_t* var_perm = nullptr;  // cost-sorted item order of the variable chunks, or null
  int32_t *sch_beg = nullptr, *sch_end = nullptr, *sch_row = nullptr;
  // Stored clauses by length class, each class with its own pass instance
  // (register-sized for its longest clause) and chunk table.
  struct ClauseClass {
    int kind = 0;   // kClassShort or kClassWave
    int param = 0;  // literals (short) or chunks of G literals (wave) held in registers
    Chunks ch;
    int32_t *ids = nullptr, *beg = nullptr, *end = nullptr, *row = nullptr;
    int32_t* packed = nullptr;  // short classes: [clauses][2][param] codes, then D rows
    int32_t* order = nullptr;   // XCD-aware launch order of the chunks (-1: padding)
    int32_t n_order = 0;
  };
  std::vector<ClauseClass> cls;
  int32_t *segch_beg = nullptr, *segch_end = nullptr, *segch_row = nullptr;
  int32_t *ach_beg = nullptr, *ach_end = nullptr, *ach_order = nullptr;
  int32_t n_aorder = 0;  // blocks of the XCD-aware order of the all-clause chunks, 0: none
  // flat plan
  int2* pairs = nullptr;
  int32_t *pair_first = nullptr, *pair_end = nullptr, *pair_mid = nullptr, *lrec_ptr = nullptr,
          *lrec_mid = nullptr, *lrec_end = nullptr;
  uint32_t* lrec = nullptr;
  uint32_t* qrow = nullptr;  // [clause rows][ld] packed per-clause products
  int32_t *row_ids = nullptr, *rch_beg = nullptr, *rch_end = nullptr, *rch_row = nullptr;
  int32_t *rch_order = nullptr, *rch_fvb = nullptr, *rlit_ptr = nullptr, *rlits = nullptr;
  int32_t n_rorder = 0;
  int32_t* vch_fvb = nullptr;  // [variable chunks] first variable of the chunk's formula
  int32_t* vch_rbase = nullptr;  // [variable chunks] first clause row of the chunk's formula
  int32_t* f_rbeg = nullptr;     // [F+1] first clause row of each formula
  int32_t *seg_var = nullptr, *seg_q0 = nullptr, *seg_q1 = nullptr, *seg_perm = nullptr;
  int32_t *heavy_var = nullptr, *heavy_sbeg = nullptr;
  int32_t *fin_step_a0 = nullptr, *fin_step_a1 = nullptr;
  int32_t *fin_all_a0 = nullptr, *fin_all_a1 = nullptr;
  // Empty clauses have no occurrence, so the step's variable pass never
  // sees them: the step's finalize adds n_empty.  Passes over every clause
  // (loss only, round check) count them themselves and add zero_empty.
  int32_t *n_empty = nullptr, *zero_empty = nullptr;
  int32_t *f_vbeg = nullptr, *f_cbeg = nullptr;
  int32_t* lds_order = nullptr;  // formulas of the LDS schedule, costliest first
  // workspace
  float *D = nullptr, *xa = nullptr, *xb = nullptr;
  float* nbuf = nullptr;  // noise of the straight-through Gumbel mode (allocated on first use)
  int32_t* sel_off = nullptr;  // per-formula selection offsets of galsat_select_vars
  double* loss_part = nullptr;
  double* fin_l = nullptr;     // split-finalize part sums (kFinalizeScratch entries)
  int32_t* fin_u = nullptr;
  int32_t max_step_rows = 0, max_all_rows = 0;  // most partial rows of one formula
  double* gseg = nullptr;
  int32_t* unsat_part = nullptr;
  uint64_t* bits = nullptr;
  int32_t* best_tmp = nullptr;
  int32_t* unsat_tmp = nullptr;
  int32_t* work_counter = nullptr;

  // per-kernel event timing (galsat_profile)
  bool prof = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }

  void release_records() {
    for (auto& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }

  // captured step sequence of galsat_step (use_graph)
  struct GraphKey {
    float* x;
    int32_t ldx, steps;
    float* loss_trace;
    int32_t* unsat_trace;
    bool operator==(const GraphKey& o) const {
      return x == o.x && ldx == o.ldx && steps == o.steps && loss_trace == o.loss_trace &&
             unsat_trace == o.unsat_trace;
    }
  };
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  GraphKey graph_key{};

  ~galsat_ctx() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    release_records();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
  }

  galsat_status fail(galsat_status s, const std::string& msg) {
    err = msg;
    if (s == GALSAT_EDEVICE) sticky = true;
    return s;
  }

  galsat_status dev_fail(hipError_t e, const char* what) {
    return fail(GALSAT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }

  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    device_bytes += count * sizeof(T);
    *p = static_cast<T*>(q);
    return hipSuccess;
  }

  template <typename T>
  hipError_t upload(T** p, const T* src, size_t count, hipStream_t s) {
    hipError_t e = alloc(p, count);
    if (e != hipSuccess || count == 0) return e;
    return hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, s);
  }
};

// Brackets the launches of its scope with a pair of events when the
// handle is profiling.
struct ProfScope {
  galsat_ctx* h;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(galsat_ctx* h_, int kind_, hipStream_t s_) : h(h_), kind(kind_), s(s_) {
    if (!h->prof) return;
    a = h->get_event();
    b = h->get_event();
    if (a && b) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      h->recs.push_back({kind, a, b});
    }
  }
};

#define GS_CHECK_HANDLE(h)                                                      \
  do {                                                                          \
    if (!(h)) return GALSAT_EINVAL;                                             \
    if ((h)->sticky) return GALSAT_EDEVICE;                                     \
  } while (0)

#define GS_HIP(h, expr, what)                                                   \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess) return (h)->dev_fail(_e, what);                       \
  } while (0)

extern "C" {

void galsat_default_options(galsat_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->optimizer = GALSAT_OPT_SGD_CLAMP;
  o->lr = 0.1f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->partials = GALSAT_PARTIALS_AUTO;
  o->recompute_max_len = 0;
  o->workspace_budget_bytes = 0;
  o->validate = 1;
  o->schedule = GALSAT_SCHED_AUTO;
  o->use_graph = 0;
  o->plan_override = nullptr;
}

const char* galsat_status_string(galsat_status s) {
  switch (s) {
    case GALSAT_OK: return "ok";
    case GALSAT_EINVAL: return "invalid argument";
    case GALSAT_ENOMEM: return "out of device memory or workspace budget";
    case GALSAT_EDEVICE: return "device error";
    case GALSAT_EOVERFLOW: return "size overflow";
    case GALSAT_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* galsat_last_error(galsat_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"

namespace {

// GALSAT_VERBOSE=1 prints the duration of each galsat_create phase.
struct PhaseTimer {
  bool on = std::getenv("GALSAT_VERBOSE") != nullptr;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    auto t1 = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[galsat] create %-18s %8.3f s\n", what,
                 std::chrono::duration<double>(t1 - t0).count());
    t0 = t1;
  }
};

galsat_status create_fail(galsat_status s, const std::string& msg) {
  g_create_error = msg;
  return s;
}

// Parses "key=value,key=value" plan overrides: lpi, rpl, krec, tg, xcdc
// (chunks per formula of multi-formula launches; 0 turns the XCD order off),
// stream (1: streaming variable pass), two (1: two-phase gradient), dsort
// (1: cost-sorted variable items), csort (1: length-sorted stored clauses),
// wave (0: no wave-per-clause pass), short (0: no short-clause pass), xseq
// (one formula: about this many chunks in an XCD-contiguous order), segdiv,
// ldsrg (restarts per workgroup of the LDS schedule: 1, 2, 4, 8, 16 or 32)
// ldsstage (0: the LDS schedule reads records from global memory), ldslpt
// (0: the LDS schedule issues formulas in index order), xpin (1/0: the
// single pass maps restart tiles to XCDs or not), flat (1/0: the flat plan
// of pair records and clause rows, or not), pf (flat plan: 1/0, records of
// the next batch prefetched or not), rsort (flat plan: 1/0, a variable's
// clause rows in row order or in slot order) and sord (flat plan: 1/0,
// segments of split variables run in the order of the first clause row
// they read, or variable by variable) and psort (flat plan: 1/0, each
// variable's pair records in the order of their nearer partner, or in slot
// order).
void apply_override(const char* spec, int* lpi, int* rpl, int* krec, int* tg, int* xcdc,
                    int* stream_items, int* two_phase, int* dsort, int* csort, int* wave,
                    int* short_clauses, int* xseq, int* segdiv, int* ldsrg, int* ldsstage,
                    int* ldslpt, int* xpin, int* flat, int* pf, int* rsort, int* sord, int* psort) {
  if (!spec) return;
  std::string s(spec);
  size_t pos = 0;
  while (pos < s.size()) {
    size_t comma = s.find(',', pos);
    if (comma == std::string::npos) comma = s.size();
    std::string kv = s.substr(pos, comma - pos);
    size_t eq = kv.find('=');
    if (eq != std::string::npos) {
      std::string k = kv.substr(0, eq);
      int v = std::atoi(kv.c_str() + eq + 1);
      if (k == "lpi") *lpi = v;
      else if (k == "rpl") *rpl = v;
      else if (k == "krec") *krec = v;
      else if (k == "tg") *tg = v;
      else if (k == "xcdc") *xcdc = v;
      else if (k == "stream") *stream_items = v;
      else if (k == "two") *two_phase = v;
      else if (k == "dsort") *dsort = v;
      else if (k == "csort") *csort = v;
      else if (k == "wave") *wave = v;
      else if (k == "short") *short_clauses = v;
      else if (k == "xseq") *xseq = v;
      else if (k == "segdiv") *segdiv = v;
      else if (k == "ldsrg") *ldsrg = v;
      else if (k == "ldsstage") *ldsstage = v;
      else if (k == "ldslpt") *ldslpt = v;
      else if (k == "xpin") *xpin = v;
      else if (k == "flat") *flat = v;
      else if (k == "sord") *sord = v;
      else if (k == "psort") *psort = v;
      else if (k == "pf") *pf = v;
      else if (k == "rsort") *rsort = v;
    }
    pos = comma + 1;
  }
}

// Default lanes-per-item / restarts-per-lane.  Wide restart batches take 4
// consecutive restarts per lane (one 16-byte load per lane, 1 KB per wave
// and row); at 32 restarts or fewer one restart per lane measured faster
// (two variables per wave instead of eight).
Tile choose_tile(int R, int rpl_max) {
  Tile t;
  int rpl = 1;
  if (R > 32 && rpl_max >= 4 && R % 4 == 0) rpl = 4;
  else if (R > 32 && rpl_max >= 2 && R % 2 == 0) rpl = 2;
  int per_lane = (R + rpl - 1) / rpl;
  int lpi = pow2_ceil(per_lane);
  lpi = std::max(4, std::min(64, lpi));
  t.lpi = lpi;
  t.rpl = rpl;
  return t;
}

}  // namespace

extern "C" galsat_status galsat_create(const galsat_problem* prob, const galsat_options* opt_in,
                                       void* stream, galsat_handle* out) {
  g_create_error.clear();
  if (!out) return create_fail(GALSAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!prob) return create_fail(GALSAT_EINVAL, "problem is NULL");
  galsat_options opt;
  if (opt_in) opt = *opt_in; else galsat_default_options(&opt);
  const int32_t F = prob->num_formulas, n = prob->n_vars, m = prob->n_clauses, L = prob->n_lits,
                R = prob->restarts;
  if (F < 1) return create_fail(GALSAT_EINVAL, "num_formulas must be >= 1");
  if (n < 0 || m < 0 || L < 0) return create_fail(GALSAT_EINVAL, "negative size");
  if (R < 1) return create_fail(GALSAT_EINVAL, "restarts must be >= 1");
  if (R > 65536) return create_fail(GALSAT_EOVERFLOW, "restarts above 65536");
  if (!prob->clause_ptr || !prob->var_ptr || (L > 0 && (!prob->clause_lits || !prob->var_occ)))
    return create_fail(GALSAT_EINVAL, "missing CSR array");
  if (F > 1 && (!prob->formula_var_begin || !prob->formula_clause_begin))
    return create_fail(GALSAT_EINVAL, "formula ranges are required when num_formulas > 1");
  if (opt.optimizer != GALSAT_OPT_SGD_CLAMP && opt.optimizer != GALSAT_OPT_ADAM)
    return create_fail(GALSAT_EINVAL, "unknown optimizer");
  if (opt.partials < 0 || opt.partials > 2) return create_fail(GALSAT_EINVAL, "unknown partials mode");
  if (opt.schedule != GALSAT_SCHED_AUTO && opt.schedule != GALSAT_SCHED_GENERAL &&
      opt.schedule != GALSAT_SCHED_LDS && opt.schedule != GALSAT_SCHED_PLAIN)
    return create_fail(GALSAT_EINVAL, "unknown schedule");
  if (!(opt.lr >= 0.0f) || !std::isfinite(opt.lr)) return create_fail(GALSAT_EINVAL, "lr must be finite and >= 0");

  // a plan remembered by galsat_autotune for this problem's shape
  std::string cached_plan;
  if (!opt.plan_override && std::getenv("GALSAT_PLAN_CACHE") &&
      plan_cache_lookup(plan_key(prob), &cached_plan))
    opt.plan_override = cached_plan.c_str();

  hipStream_t s = static_cast<hipStream_t>(stream);
  PhaseTimer ptimer;
  // ---- host views of the inputs (copied only when they live on the device)
  std::vector<int32_t> cp_own, cl_own, vp_own, vo_own;
  const int32_t *cp = prob->clause_ptr, *cl = prob->clause_lits, *vp = prob->var_ptr,
                *vo = prob->var_occ;
  std::vector<int32_t> fvb((size_t)F + 1), fcb((size_t)F + 1);
  hipError_t he = hipSuccess;
  auto fetch = [&](std::vector<int32_t>& dst, const int32_t* src, size_t count) -> hipError_t {
    dst.resize(count);
    if (count == 0) return hipSuccess;
    if (prob->inputs_on_device)
      return hipMemcpy(dst.data(), src, count * sizeof(int32_t), hipMemcpyDeviceToHost);
    std::memcpy(dst.data(), src, count * sizeof(int32_t));
    return hipSuccess;
  };
  if (prob->inputs_on_device) {
    if ((he = fetch(cp_own, prob->clause_ptr, (size_t)m + 1)) != hipSuccess ||
        (he = fetch(vp_own, prob->var_ptr, (size_t)n + 1)) != hipSuccess ||
        (he = fetch(cl_own, prob->clause_lits, (size_t)L)) != hipSuccess ||
        (he = fetch(vo_own, prob->var_occ, (size_t)L)) != hipSuccess)
      return create_fail(GALSAT_EDEVICE, std::string("copying inputs: ") + hipGetErrorString(he));
    cp = cp_own.data();
    vp = vp_own.data();
    cl = cl_own.data();
    vo = vo_own.data();
  }
  if (prob->formula_var_begin && prob->formula_clause_begin) {
    if ((he = fetch(fvb, prob->formula_var_begin, (size_t)F + 1)) != hipSuccess ||
        (he = fetch(fcb, prob->formula_clause_begin, (size_t)F + 1)) != hipSuccess)
      return create_fail(GALSAT_EDEVICE, std::string("copying formula ranges: ") + hipGetErrorString(he));
  } else {
    fvb = {0, n};
    fcb = {0, m};
  }
  ptimer.mark("fetch");
  // ---- validation
  if (cp[0] != 0 || cp[(size_t)m] != L) return create_fail(GALSAT_EINVAL, "clause_ptr must start at 0 and end at n_lits");
  for (int32_t t = 0; t < m; ++t)
    if (cp[t + 1] < cp[t]) return create_fail(GALSAT_EINVAL, "clause_ptr is not non-decreasing");
  if (vp[0] != 0 || vp[(size_t)n] != L) return create_fail(GALSAT_EINVAL, "var_ptr must start at 0 and end at n_lits");
  for (int32_t v = 0; v < n; ++v)
    if (vp[v + 1] < vp[v]) return create_fail(GALSAT_EINVAL, "var_ptr is not non-decreasing");
  if (fvb[0] != 0 || fvb[F] != n || fcb[0] != 0 || fcb[F] != m)
    return create_fail(GALSAT_EINVAL, "formula ranges must start at 0 and end at n_vars / n_clauses");
  for (int32_t f = 0; f < F; ++f)
    if (fvb[f + 1] < fvb[f] || fcb[f + 1] < fcb[f])
      return create_fail(GALSAT_EINVAL, "formula ranges are not non-decreasing");
  std::vector<int32_t> var_formula((size_t)n);
  for (int32_t f = 0; f < F; ++f)
    for (int32_t v = fvb[f]; v < fvb[f + 1]; ++v) var_formula[v] = f;
  std::unique_ptr<int32_t[]> clause_of(new int32_t[(size_t)L + 1]);
  std::atomic<int32_t> kmax_a{0};
  std::vector<std::atomic<int32_t>> n_empty_a((size_t)F);
  for (auto& e : n_empty_a) e.store(0);
  FirstError ferr;
  parallel_for(m, [&](int64_t t0, int64_t t1) {
    if (t0 >= t1) return;
    int32_t f = (int32_t)(std::upper_bound(fcb.begin(), fcb.end(), (int32_t)t0) - fcb.begin()) - 1;
    int32_t kloc = 0;
    for (int64_t t = t0; t < t1; ++t) {
      while (t >= fcb[f + 1]) ++f;
      const int32_t k = cp[t + 1] - cp[t];
      kloc = std::max(kloc, k);
      if (k == 0) n_empty_a[f]++;
      for (int32_t p = cp[t]; p < cp[t + 1]; ++p) {
        const int32_t code = cl[p];
        if (code < 0 || (code >> 1) >= n) {
          ferr.report(p, "literal code out of range at position " + std::to_string(p));
          return;
        }
        if ((code >> 1) < fvb[f] || (code >> 1) >= fvb[f + 1]) {
          ferr.report(p, "clause " + std::to_string(t) + " uses a variable of another formula");
          return;
        }
        clause_of[p] = (int32_t)t;
      }
    }
    int32_t cur = kmax_a.load();
    while (kloc > cur && !kmax_a.compare_exchange_weak(cur, kloc)) {
    }
  });
  if (ferr.index >= 0) return create_fail(GALSAT_EINVAL, ferr.msg);
  const int32_t kmax = kmax_a.load();
  std::vector<int32_t> n_empty((size_t)F);
  for (int32_t f = 0; f < F; ++f) n_empty[f] = n_empty_a[f].load();
  {
    // every slot names a position of its own variable, each position once
    std::unique_ptr<uint64_t[]> seen(opt.validate ? new uint64_t[(size_t)L / 64 + 1]() : nullptr);
    parallel_for(n, [&](int64_t v0, int64_t v1) {
      for (int64_t v = v0; v < v1; ++v)
        for (int32_t q = vp[v]; q < vp[v + 1]; ++q) {
          const int32_t p = vo[q];
          if (p < 0 || p >= L) {
            ferr.report(q, "var_occ entry out of range");
            return;
          }
          if ((cl[p] >> 1) != v) {
            ferr.report(q, "var_occ is not the transpose of clause_lits (variable " +
                               std::to_string(v) + ")");
            return;
          }
          if (seen) {
            const uint64_t bit = 1ULL << (p & 63);
            if (__atomic_fetch_or(&seen[p >> 6], bit, __ATOMIC_RELAXED) & bit) {
              ferr.report(q, "var_occ lists a position twice");
              return;
            }
          }
        }
    });
    if (ferr.index >= 0) return create_fail(GALSAT_EINVAL, ferr.msg);
  }

  ptimer.mark("validate");
  std::unique_ptr<galsat_ctx> h(new galsat_ctx());
  h->F = F; h->n = n; h->m = m; h->L = L; h->R = R;
  h->opt = opt;
  h->kmax = kmax;
  h->h_fvb = fvb;
  h->h_fcb = fcb;
  (void)hipGetDevice(&h->device);

  // ---- plan: which clauses recompute their partials in the variable pass
  int lpi_o = 0, rpl_o = 0, krec_o = -1, tg_o = 0, xcdc_o = -1, stream_o = -1, two_o = -1;
  int dsort_o = -1, csort_o = -1, wave_o = -1, short_o = -1, xseq_o = -1, segdiv_o = -1;
  int ldsrg_o = 0, ldsstage_o = -1, ldslpt_o = -1, xpin_o = -1, flat_o = -1, pf_o = -1, rsort_o = -1;
  int sord_o = -1, psort_o = -1;
  apply_override(opt.plan_override, &lpi_o, &rpl_o, &krec_o, &tg_o, &xcdc_o, &stream_o, &two_o,
                 &dsort_o, &csort_o, &wave_o, &short_o, &xseq_o, &segdiv_o, &ldsrg_o, &ldsstage_o,
                 &ldslpt_o, &xpin_o, &flat_o, &pf_o, &rsort_o, &sord_o, &psort_o);
  const bool csort = csort_o != 0;
  // Persistent LDS schedule: every formula's restart group must fit in LDS
  // (state double-buffered); SGD only; every clause recomputed.
  int lds_rg = 0, lds_stage = 0;
  int32_t lds_nocc = 0;
  if (opt.schedule == GALSAT_SCHED_LDS) {
    if (opt.optimizer != GALSAT_OPT_SGD_CLAMP || opt.partials == GALSAT_PARTIALS_STORE)
      return create_fail(GALSAT_EUNSUPPORTED, "the LDS schedule runs projected SGD with recomputed partials");
    int32_t nf_max = 0;
    for (int32_t f = 0; f < F; ++f) {
      nf_max = std::max(nf_max, fvb[f + 1] - fvb[f]);
      lds_nocc = std::max(lds_nocc, vp[fvb[f + 1]] - vp[fvb[f]]);
    }
    int dev = 0, lds_max = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lds_max <= 0)
      lds_max = 64 << 10;
    lds_max = std::min(lds_max, 64 << 10);
    // Restarts per workgroup: one (a workgroup per restart, the most
    // parallel) while that gives at most two workgroups per CU; beyond, up
    // to 32 and no more than the restarts, as long as every variable of the
    // largest formula keeps its own slot of the 512 threads (a step makes
    // one pass over the variables).  Fewer when the state does not fit.
    // The records are staged when they fit beside it.
    // A dispatch holds fewer than 2^32 work-items per dimension, so very
    // large batches take bigger groups (several passes over the variables)
    // or are refused.
    auto items = [&](int g) { return (int64_t)F * ((R + g - 1) / g) * kPersistBlock; };
    int rg = 1;
    while (rg < 32 && rg < R && (int64_t)(kPersistBlock / (2 * rg)) >= nf_max &&
           (int64_t)F * ((R + rg - 1) / rg) > kPersistSpreadGroups)
      rg *= 2;
    if (ldsrg_o == 1 || ldsrg_o == 2 || ldsrg_o == 4 || ldsrg_o == 8 || ldsrg_o == 16 || ldsrg_o == 32)
      rg = ldsrg_o;
    while (rg < 32 && items(rg) > (int64_t)UINT32_MAX) rg *= 2;
    if (items(rg) > (int64_t)UINT32_MAX)
      return create_fail(GALSAT_EUNSUPPORTED, "too many formulas x restarts for the LDS schedule");
    for (; rg >= 1 && !lds_rg && items(rg) <= (int64_t)UINT32_MAX; rg /= 2) {
      if (ldsstage_o != 0 && persist_lds_bytes(rg, nf_max, lds_nocc) <= (size_t)lds_max) {
        lds_rg = rg;
        lds_stage = 1;
      } else if (persist_lds_bytes(rg, nf_max, 0) <= (size_t)lds_max) {
        lds_rg = rg;
      }
    }
    if (!lds_rg) return create_fail(GALSAT_EUNSUPPORTED, "a formula is too large for the LDS schedule");
  }
  int32_t krec;
  if (opt.partials == GALSAT_PARTIALS_STORE) krec = -1;           // every clause stores
  else if (opt.partials == GALSAT_PARTIALS_RECOMPUTE) krec = kmax;
  else krec = opt.recompute_max_len > 0 ? opt.recompute_max_len : kDefaultRecomputeMaxLen;
  if (krec_o >= -1 && opt.plan_override && std::strstr(opt.plan_override, "krec=")) krec = krec_o;
  if (lds_rg) krec = kmax;
  h->ld = (int32_t)round_up(R, 4);
  h->ldD = round_up(R, 4);
  h->stream_items = stream_o >= 0 ? stream_o : 0;
  h->xcd_pin = xpin_o > 0 ? 1 : 0;
  // Two-phase gradient (clause passes + variable sums): by default for
  // narrow restart batches (at most 32 restarts), where one gather per
  // literal plus a contribution row written and read beats the single
  // pass's k - 1 gathers per occurrence; wide batches keep the single pass,
  // whose gathers are row-wide.  It needs one contribution row per
  // occurrence.
  h->two_phase = two_o >= 0 ? (two_o ? 1 : 0) : (R <= 32 ? 1 : 0);
  if (h->two_phase && opt.workspace_budget_bytes > 0 &&
      (size_t)L * (size_t)h->ldD * sizeof(float) > opt.workspace_budget_bytes)
    h->two_phase = 0;
  if (h->stream_items || lds_rg) h->two_phase = 0;
  // Flat plan (galsat_flat.hip): 3-literal clauses recomputed from pair
  // records, every other clause reduced once per step to a row of packed
  // per-clause products.  By default for narrow restart batches (at most 64)
  // with AUTO partials and no explicit gradient-plan override; it needs
  // formula-local literal codes below 2^31 and the clause rows within the
  // workspace budget.
  {
    const bool krec_set = opt.recompute_max_len > 0 ||
                          (opt.plan_override && std::strstr(opt.plan_override, "krec="));
    // the variable pass addresses a formula's state rows and clause rows by
    // 32-bit byte offsets and its local indices by 24-bit multiplies
    bool fit = !h->stream_items && !lds_rg && opt.partials != GALSAT_PARTIALS_RECOMPUTE;
    const int64_t row_bytes = round_up(R, 4) * 4;
    for (int32_t f = 0; f < F && fit; ++f) {
      int64_t rows_f = 0;
      for (int32_t t = fcb[f]; t < fcb[f + 1]; ++t) rows_f += (cp[t + 1] - cp[t] != 3 && cp[t + 1] > cp[t]) ? 1 : 0;
      const int64_t nf = fvb[f + 1] - fvb[f];
      fit = nf < (1 << 24) && rows_f < (1 << 24) && nf * row_bytes < (int64_t(1) << 32) &&
            rows_f * row_bytes < (int64_t(1) << 32);
    }
    if (fit && opt.workspace_budget_bytes > 0) {
      int64_t rows = 0;
      for (int32_t t = 0; t < m; ++t) rows += (cp[t + 1] - cp[t] != 3 && cp[t + 1] > cp[t]) ? 1 : 0;
      fit = (size_t)rows * (size_t)round_up(R, 4) * sizeof(uint32_t) <= opt.workspace_budget_bytes;
    }
    const bool auto_flat = flat_o < 0 && two_o < 0 && !krec_set && R <= 64 &&
                           opt.partials == GALSAT_PARTIALS_AUTO;
    h->flat = fit && (flat_o > 0 || auto_flat) ? 1 : 0;
    if (h->flat) h->two_phase = 0;
  }
  // chunks per formula of the XCD-aware order (several formulas per launch)
  const int64_t xcd_chunks =
      xcdc_o >= 0 ? xcdc_o
                  : (h->two_phase ? kXcdChunksTwoPhase : h->flat ? kXcdChunksFlat : kXcdChunks);
  h->tile = choose_tile(R, 4);
  if ((h->two_phase || h->flat) && R % 4 == 0 && R >= 16) {
    // four restarts per lane measured faster for the two-phase passes (and
    // the flat plan, whose per-record decoding then serves four restarts)
    h->tile.rpl = 4;
    h->tile.lpi = std::max(4, std::min(64, pow2_ceil(R / 4)));
  }
  // Wide restart batches of one formula on the single pass: eight tiles of
  // R/8 restarts (4 per lane; rows of 128 bytes or more) in one launch, each
  // tile on its own XCD (k_var_pass maps tiles by linear block id), so an
  // XCD's L2 holds one tile's lines.  Measured 7 % faster per step than
  // 256-restart tiles two per launch at R = 1024.
  bool xpin_auto = false;
  if (xpin_o < 0 && !h->two_phase && !h->flat && !h->stream_items && !lds_rg && F == 1 && R >= 1024 &&
      R % 256 == 0 && opt.schedule != GALSAT_SCHED_PLAIN) {
    xpin_auto = true;
    h->xcd_pin = 1;
    h->tile.rpl = 4;
    h->tile.lpi = std::min(64, R / 32);
  }
  if (lpi_o == 4 || lpi_o == 8 || lpi_o == 16 || lpi_o == 32 || lpi_o == 64) h->tile.lpi = lpi_o;
  if ((rpl_o == 1 || rpl_o == 2 || rpl_o == 4) && R % rpl_o == 0) h->tile.rpl = rpl_o;
  // Cost-sorted variable items when a wave holds several items (with a
  // whole wave per item the index order keeps neighbouring variables, and
  // their shared clauses, together).
  const bool dsort = dsort_o >= 0 ? dsort_o > 0 : h->tile.lpi < 64;
  // Restart tiles per launch: keep the state rows a launch gathers from
  // (n x tiles x tile x 4 B) within a share of the 256 MB last-level cache.
  {
    const int tiles_all = (R + h->tile.tile() - 1) / h->tile.tile();
    const int64_t tile_bytes = std::max<int64_t>(1, (int64_t)n * h->tile.tile() * 4);
    int tg = (int)std::max<int64_t>(1, kCacheBudgetBytes / tile_bytes);
    if (xpin_auto) tg = 8;
    if (tg_o > 0) tg = tg_o;
    h->tgroup = std::min(tg, tiles_all);
  }
  // The two-phase plan writes a contribution row for every occurrence
  // anyway: by default every clause stores its partials (each literal's row
  // gathered once, by the clause passes) and nothing is recomputed per
  // occurrence.
  {
    const bool krec_given = opt.recompute_max_len > 0 ||
                            (krec_o >= -1 && opt.plan_override && std::strstr(opt.plan_override, "krec="));
    if (h->two_phase && opt.partials == GALSAT_PARTIALS_AUTO && !krec_given) krec = 0;
  }
  auto count_stored = [&](int32_t kr) {
    std::atomic<int64_t> c{0};
    parallel_for(m, [&](int64_t t0, int64_t t1) {
      int64_t loc = 0;
      for (int64_t t = t0; t < t1; ++t)
        if (cp[t + 1] - cp[t] > kr && cp[t + 1] > cp[t]) loc += cp[t + 1] - cp[t];
      c += loc;
    });
    return c.load();
  };
  int64_t stored = count_stored(krec);
  if (opt.workspace_budget_bytes > 0 &&
      (size_t)stored * (size_t)h->ldD * sizeof(float) > opt.workspace_budget_bytes) {
    if (opt.partials == GALSAT_PARTIALS_STORE)
      return create_fail(GALSAT_ENOMEM, "stored partials exceed workspace_budget_bytes");
    krec = kmax;  // recompute everything: no per-literal storage at all
    stored = 0;
  }
  if (h->flat) {
    // the flat plan keeps no per-literal rows: its clause rows are planned
    // below, and no old-style occurrence record is built
    krec = kmax;
    stored = 0;
  }
  h->krec = krec;
  h->stored = stored;

  // Occurrence records in variable-major order (one int4 per slot; the
  // kernels' record layout): stored partial row, a short recomputed clause
  // with the other literals' codes inline, or a longer recomputed clause by
  // id and position.  Stored rows are numbered in variable-major order so a
  // variable's stored partials are contiguous.
  // filled completely below, so left uninitialised
  const bool flat = h->flat != 0;
  std::unique_ptr<int4[]> occ4(new int4[flat ? 1 : (size_t)L + 1]);
  const bool need_x = !flat && krec >= 5 && kmax >= 5;  // some inline record holds 4 to 7 others
  std::unique_ptr<int4[]> occx(new int4[need_x ? (size_t)L + 1 : 1]);
  std::unique_ptr<int32_t[]> occ_cost(new int32_t[(size_t)L + 1]);
  std::unique_ptr<int32_t[]> lit_dslot(new int32_t[stored > 0 ? (size_t)L + 1 : 1]);
  const bool two = h->two_phase != 0;
  {
    std::vector<int64_t> sbase((size_t)n + 1, 0);
    parallel_for(n, [&](int64_t v0, int64_t v1) {
      for (int64_t v = v0; v < v1; ++v) {
        int64_t c = 0;
        for (int32_t q = vp[v]; q < vp[v + 1]; ++q) {
          const int32_t t = clause_of[vo[q]];
          c += (cp[t + 1] - cp[t] > krec) ? 1 : 0;
        }
        sbase[v + 1] = c;
      }
    });
    for (int32_t v = 0; v < n; ++v) sbase[v + 1] += sbase[v];
    parallel_for(n, [&](int64_t v0, int64_t v1) {
    for (int64_t vv = v0; vv < v1; ++vv) {
      const int32_t v = (int32_t)vv;
      int64_t d = sbase[v];
      for (int32_t q = vp[v]; q < vp[v + 1]; ++q) {
        const int32_t p = vo[q], t = clause_of[p], k = cp[t + 1] - cp[t];
        if (flat) {
          // gathers per restart: two other rows (3-literal clause) or one
          // clause row
          occ_cost[q] = k == 3 ? 2 : 1;
          continue;
        }
        const int32_t sign_first = ((cl[p] & 1) << 3) | ((p == cp[t]) ? 16 : 0);
        if (k > krec) {
          // two-phase: the clause pass writes the contribution straight into
          // the slot's row of the contribution buffer
          const int32_t row = two ? q : (int32_t)d;
          occ4[q] = make_int4(2 << 5, row, 0, 0);
          occ_cost[q] = 1;
          lit_dslot[p] = row;
          ++d;
        } else if (k <= 8) {
          int32_t codes[7] = {2 * v, 2 * v, 2 * v, 2 * v, 2 * v, 2 * v, 2 * v};
          int32_t c = 0;
          for (int32_t i = cp[t]; i < cp[t + 1]; ++i)
            if (i != p) codes[c++] = cl[i];
          occ4[q] = make_int4((k - 1) | sign_first, codes[0], codes[1], codes[2]);
          if (need_x) occx[q] = make_int4(codes[3], codes[4], codes[5], codes[6]);
          occ_cost[q] = std::max(1, k - 1);
        } else {
          occ4[q] = make_int4((1 << 5) | sign_first, t, p, 0);
          if (need_x) occx[q] = make_int4(0, 0, 0, 0);
          occ_cost[q] = k - 1;
        }
      }
    }
    });
  }
  ptimer.mark("records");
  // ---- flat plan tables.  Clause rows: every clause that is not 3
  // literals long (and not empty), per formula longest first.  Per
  // variable, in variable-major slot order: pair records of the 3-literal
  // clauses whose first literal is the variable's own occurrence, then the
  // other pair records, then clause-row records.
  std::vector<int32_t> row_ids, row_of, pair_first, pair_fneg, pair_mid, lrec_ptr, lrec_mid, pair_end,
      lrec_end, rlit_ptr, rlits;
  std::vector<int64_t> f_rbeg((size_t)F + 1, 0);
  std::vector<int2> pairs;
  std::vector<uint32_t> lrec;
  const bool rsort = rsort_o != 0;
  const bool psort = psort_o != 0;
  // Prefetching the next batch's records pays when a variable's record runs
  // span several batches (measured: +7 % at 38 occurrences per variable,
  // -13 % at 14), so by default from 24 occurrences per variable on.
  h->prefetch = pf_o >= 0 ? (pf_o ? 1 : 0) : ((int64_t)L >= 24 * (int64_t)std::max(n, 1) ? 1 : 0);
  if (flat) {
    row_of.assign((size_t)std::max(m, 1), -1);
    for (int32_t f = 0; f < F; ++f) {
      f_rbeg[f] = (int64_t)row_ids.size();
      for (int32_t t = fcb[f]; t < fcb[f + 1]; ++t) {
        const int32_t k = cp[t + 1] - cp[t];
        if (k != 3 && k > 0) row_ids.push_back(t);
      }
      std::stable_sort(row_ids.begin() + f_rbeg[f], row_ids.end(), [&](int32_t a2, int32_t b2) {
        return cp[a2 + 1] - cp[a2] > cp[b2 + 1] - cp[b2];
      });
    }
    f_rbeg[F] = (int64_t)row_ids.size();
    for (size_t i = 0; i < row_ids.size(); ++i) row_of[row_ids[i]] = (int32_t)i;
    // the row pass's own literal list: each listed clause's codes relative
    // to its formula, contiguous in list order
    rlit_ptr.assign(row_ids.size() + 1, 0);
    for (size_t i = 0; i < row_ids.size(); ++i)
      rlit_ptr[i + 1] = rlit_ptr[i] + (cp[row_ids[i] + 1] - cp[row_ids[i]]);
    rlits.resize((size_t)std::max(rlit_ptr.back(), 1));
    parallel_for((int64_t)row_ids.size(), [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        const int32_t t = row_ids[i];
        const int32_t base2 = 2 * fvb[var_formula[cl[cp[t]] >> 1]];
        int32_t o = rlit_ptr[i];
        for (int32_t q = cp[t]; q < cp[t + 1]; ++q) rlits[(size_t)o++] = cl[q] - base2;
      }
    });
    std::vector<int64_t> np((size_t)n + 1, 0), nr((size_t)n + 1, 0), nf((size_t)n, 0),
        nfp((size_t)n, 0);
    parallel_for(n, [&](int64_t v0, int64_t v1) {
      for (int64_t v = v0; v < v1; ++v) {
        int64_t a3 = 0, fst = 0, fpos = 0, b = 0;
        for (int32_t q = vp[v]; q < vp[v + 1]; ++q) {
          const int32_t p = vo[q], t = clause_of[p];
          if (cp[t + 1] - cp[t] == 3) {
            ++a3;
            fst += p == cp[t] ? 1 : 0;
            fpos += (p == cp[t] && (cl[p] & 1) == 0) ? 1 : 0;
          } else {
            ++b;
          }
        }
        np[v + 1] = a3;
        nr[v + 1] = b;
        nf[v] = fst;
        nfp[v] = fpos;
      }
    });
    for (int32_t v = 0; v < n; ++v) {
      np[v + 1] += np[v];
      nr[v + 1] += nr[v];
    }
    pair_first.resize((size_t)n + 1);
    pair_mid.resize((size_t)std::max(n, 1));
    lrec_mid.assign((size_t)std::max(n, 1), 0);
    lrec_ptr.resize((size_t)n + 1);
    pair_fneg.resize((size_t)std::max(n, 1));
    for (int32_t v = 0; v <= n; ++v) {
      pair_first[v] = (int32_t)np[v];
      lrec_ptr[v] = (int32_t)nr[v];
      if (v < n) {
        pair_fneg[v] = (int32_t)(np[v] + nfp[v]);
        pair_mid[v] = (int32_t)(np[v] + nf[v]);
      }
    }
    pairs.resize((size_t)std::max<int64_t>(np[n], 1));
    lrec.resize((size_t)std::max<int64_t>(nr[n], 1));
    parallel_for(n, [&](int64_t v0, int64_t v1) {
      for (int64_t vv = v0; vv < v1; ++vv) {
        const int32_t v = (int32_t)vv;
        const int32_t base2 = 2 * fvb[var_formula[v]];
        int64_t af = pair_first[v], an = pair_fneg[v], ao = pair_mid[v], b = lrec_ptr[v];
        for (int32_t q = vp[v]; q < vp[v + 1]; ++q) {
          const int32_t p = vo[q], t = clause_of[p];
          const uint32_t own_neg = (uint32_t)(cl[p] & 1) << 31;
          if (cp[t + 1] - cp[t] == 3) {
            int32_t o[2], c = 0;
            for (int32_t i = cp[t]; i < cp[t + 1]; ++i)
              if (i != p) o[c++] = cl[i] - base2;
            const int2 rec = make_int2((int32_t)((uint32_t)o[0] | own_neg), o[1]);
            if (p == cp[t] && !own_neg) pairs[(size_t)af++] = rec;
            else if (p == cp[t]) pairs[(size_t)an++] = rec;
            else pairs[(size_t)ao++] = rec;
          } else {
            lrec[(size_t)b++] = (uint32_t)(row_of[t] - f_rbeg[var_formula[v]]) | own_neg;
          }
        }
        // psort: within each of the variable's three pair runs (first
        // literal positive, first literal negated, the others), the nearer
        // partner first in each record (a product of two factors does not
        // depend on their order) and the records in that partner's order,
        // so a hot variable's pair gathers sweep the state rows in order
        if (psort) {
          auto near_first = [](int2 r) {
            const uint32_t sgn = (uint32_t)r.x & 0x80000000u;
            const int32_t a1 = r.x & 0x7fffffff, a2 = r.y;
            return (a2 >> 1) < (a1 >> 1) ? make_int2((int32_t)((uint32_t)a2 | sgn), a1) : r;
          };
          const int64_t runs[4] = {pair_first[v], pair_fneg[v], pair_mid[v], pair_first[v + 1]};
          for (int64_t i = runs[0]; i < runs[3]; ++i) pairs[(size_t)i] = near_first(pairs[(size_t)i]);
          for (int k = 0; k < 3; ++k)
            std::stable_sort(pairs.begin() + runs[k], pairs.begin() + runs[k + 1],
                             [](int2 p1, int2 p2) { return (p1.x & 0x7fffffff) < (p2.x & 0x7fffffff); });
        }
        // a variable's clause rows: positive own literals first, then
        // negated ones (one partial sign per run), each in row order, so a
        // hot variable, which meets most long clauses, sweeps the rows
        // nearly sequentially; the sign bit is then dropped
        if (rsort)
          std::sort(lrec.begin() + lrec_ptr[v], lrec.begin() + b, [](uint32_t p1, uint32_t p2) {
            return (p1 >> 31) < (p2 >> 31) || ((p1 >> 31) == (p2 >> 31) && p1 < p2);
          });
        else
          std::stable_sort(lrec.begin() + lrec_ptr[v], lrec.begin() + b,
                           [](uint32_t p1, uint32_t p2) { return (p1 >> 31) < (p2 >> 31); });
        int64_t mid = lrec_ptr[v];
        while (mid < b && (lrec[(size_t)mid] >> 31) == 0) ++mid;
        lrec_mid[v] = (int32_t)mid;
        for (int64_t i = lrec_ptr[v]; i < b; ++i) lrec[(size_t)i] &= 0x7fffffffu;
      }
    });
  }
  std::vector<int32_t> stored_ids;
  std::vector<int64_t> f_sbeg((size_t)F + 1, 0);
  for (int32_t f = 0; f < F; ++f) {
    f_sbeg[f] = (int64_t)stored_ids.size();
    for (int32_t t = fcb[f]; t < fcb[f + 1]; ++t)
      if (cp[t + 1] - cp[t] > krec && cp[t + 1] > cp[t]) stored_ids.push_back(t);
    // longest first, so the clauses sharing a wave have similar lengths
    if (csort)
      std::stable_sort(stored_ids.begin() + f_sbeg[f], stored_ids.end(), [&](int32_t a2, int32_t b2) {
        return cp[a2 + 1] - cp[a2] > cp[b2 + 1] - cp[b2];
      });
  }
  f_sbeg[F] = (int64_t)stored_ids.size();
  // Stored clauses by length class, shortest first: at most 4 and at most
  // kShortClauseMax literals to the short-clause pass, then up to two
  // wave-per-clause classes (kWaveClauseSmallChunks and the tile's maximum
  // chunks of G = 64 / lanes-per-item literals), the rest to the sweeping
  // clause pass.  Each class's kernel holds only what its longest clause
  // needs in registers.
  struct Route { int kind, param, kmax; };
  std::vector<Route> routes;
  if (short_o != 0) {
    routes.push_back({kClassShort, 4, 4});
    routes.push_back({kClassShort, kShortClauseMax, kShortClauseMax});
  }
  {
    const int kw_max = wave_o != 0 ? wave_clause_kmax(h->tile) : 0;
    if (kw_max > 0) {
      const int G = 64 / h->tile.lpi;
      if (kWaveClauseSmallChunks * G < kw_max)
        routes.push_back({kClassWave, kWaveClauseSmallChunks, kWaveClauseSmallChunks * G});
      routes.push_back({kClassWave, wave_clause_chunks(h->tile.lpi), kw_max});
    }
  }
  const int NCL = (int)routes.size();
  std::vector<std::vector<int32_t>> cls_ids((size_t)NCL);
  std::vector<std::vector<int64_t>> cls_fbeg((size_t)NCL, std::vector<int64_t>((size_t)F + 1, 0));
  {
    std::vector<int32_t> keep;
    keep.reserve(stored_ids.size());
    std::vector<int64_t> f_kbeg((size_t)F + 1, 0);
    for (int32_t f = 0; f <= F; ++f) {
      f_kbeg[f] = (int64_t)keep.size();
      for (int c = 0; c < NCL; ++c) cls_fbeg[c][f] = (int64_t)cls_ids[c].size();
      if (f == F) break;
      for (int64_t i = f_sbeg[f]; i < f_sbeg[f + 1]; ++i) {
        const int32_t t = stored_ids[(size_t)i], k = cp[t + 1] - cp[t];
        int c = 0;
        while (c < NCL && k > routes[c].kmax) ++c;
        if (c < NCL) cls_ids[c].push_back(t);
        else keep.push_back(t);
      }
    }
    stored_ids.swap(keep);
    f_sbeg.swap(f_kbeg);
  }

  // ---- chunks of balanced cost.  The cost of a variable is its number of
  // gathered rows per restart; a chunk (one workgroup) gets about
  // total / chunks_target, and a variable costlier than one item slot's
  // share (chunk target / items per workgroup) is split into segments whose
  // partial gradients are summed in segment order by a second kernel.
  const int tiles = (R + h->tile.tile() - 1) / h->tile.tile();
  const int64_t chunks_target = std::max<int64_t>(1, kTargetBlocks / std::max(1, tiles));
  const int ipb = kBlock / h->tile.lpi;
  std::vector<int32_t> heavy, heavy_sbeg{0}, seg_var, seg_q0, seg_q1, vorder, oorder, vperm, seg_perm;
  std::vector<int64_t> fcost_all((size_t)F, 0);  // gather cost of each formula
  std::vector<int32_t> heavy_f_first((size_t)F + 1, 0);
  {
    std::vector<int64_t> vcost((size_t)n, 1);
    parallel_for(n, [&](int64_t v0, int64_t v1) {
      for (int64_t v = v0; v < v1; ++v)
        for (int32_t q = vp[v]; q < vp[v + 1]; ++q) vcost[v] += occ_cost[q];
    });
    int64_t total = 0;
    for (int32_t v = 0; v < n; ++v) total += vcost[v];
    int64_t target = std::max<int64_t>(64, total / chunks_target);
    const int64_t item_cap = std::max<int64_t>(64, target / ipb);
    // segments of a split variable: in the single pass a fraction of one
    // item's share, so the hottest variables' gathers spread over many
    // waves; the two-phase plan's segments only read contribution rows
    const int segdiv = segdiv_o > 0 ? segdiv_o : (two ? 1 : kSegDivSinglePass);
    const int64_t seg_cap = std::max<int64_t>(64, item_cap / segdiv);
    // XCD-contiguous order (one formula): many small chunks, each XCD taking
    // a contiguous run of them, so the workgroups resident on an XCD cover a
    // narrow range of variable ids and share the rows they gather in its L2
    // when the numbering has locality.
    // By default for a single formula whose clauses mostly join nearby
    // variable ids (measured on a sample: a literal within kLocalWindow ids
    // of its clause's first literal).
    int64_t xseq_chunks = xseq_o;
    if (xseq_o < 0 && F == 1 && m > 0) {
      int64_t near = 0, pairs = 0;
      const int64_t stride = std::max<int64_t>(1, m / 200000);
      for (int64_t t = 0; t < m; t += stride)
        for (int32_t i = cp[t] + 1; i < cp[t + 1]; ++i) {
          near += std::abs((cl[i] >> 1) - (cl[cp[t]] >> 1)) < kLocalWindow ? 1 : 0;
          ++pairs;
        }
      xseq_chunks = (pairs > 0 && near * 2 > pairs && n > 64 * kLocalWindow) ? kXseqChunks : 0;
    }
    h->xseq = xseq_chunks > 0 ? (int32_t)xseq_chunks : 0;
    // the XCD-contiguous order assigns chunks to XCDs itself
    if (h->xseq && xpin_auto) h->xcd_pin = 0;
    const bool xseq = F == 1 && xseq_chunks > 0;
    if (xseq) target = std::max<int64_t>(1, total / xseq_chunks);
    Chunks vc, sc;
    vc.f_first.assign((size_t)F + 1, 0);
    sc.f_first.assign((size_t)F + 1, 0);
    const bool per_formula = opt.schedule == GALSAT_SCHED_PLAIN;
    std::vector<int64_t>& fcost = fcost_all;
    for (int32_t f = 0; f < F; ++f) {
      vc.f_first[f] = vc.count();
      heavy_f_first[f] = (int32_t)heavy.size();
      int32_t cb = fvb[f];
      int64_t acc = 0;
      // one formula per launch (PLAIN): size its chunks as if it were the
      // whole problem, so each launch still spreads over the chip.  Which
      // variables are split does not change, so every gradient is summed in
      // the same order as in the all-formula plan.
      int64_t target_f = target;
      const int64_t item_cap_f = item_cap;
      int64_t cost_f = 0;
      for (int32_t v = fvb[f]; v < fvb[f + 1]; ++v) cost_f += vcost[v];
      fcost[f] = cost_f;
      if (per_formula) {
        target_f = std::max<int64_t>(64, cost_f / chunks_target);
      } else if (F > 1 && xcd_chunks > 0) {
        // many formulas in one launch: about kXcdChunks chunks per formula,
        // so the workgroups resident on one XCD work on one formula at a
        // time and its state stays in that XCD's L2 (see the launch order)
        target_f = std::max<int64_t>(64, cost_f / xcd_chunks);
      }
      for (int32_t v = fvb[f]; v < fvb[f + 1]; ++v) {
        if (vcost[v] > item_cap_f && vp[v + 1] - vp[v] > 1) {
          if (v > cb) { vc.beg.push_back(cb); vc.end.push_back(v); }
          cb = v + 1;
          acc = 0;
          heavy.push_back(v);
          int64_t sacc = 0;
          int32_t q0 = vp[v];
          for (int32_t q = vp[v]; q < vp[v + 1]; ++q) {
            sacc += occ_cost[q];
            if (sacc >= seg_cap || q + 1 == vp[v + 1]) {
              seg_var.push_back(v);
              seg_q0.push_back(q0);
              seg_q1.push_back(q + 1);
              q0 = q + 1;
              sacc = 0;
            }
          }
          heavy_sbeg.push_back((int32_t)seg_var.size());
          continue;
        }
        acc += vcost[v];
        if (acc >= target_f) {
          vc.beg.push_back(cb);
          vc.end.push_back(v + 1);
          cb = v + 1;
          acc = 0;
        }
      }
      if (fvb[f + 1] > cb) { vc.beg.push_back(cb); vc.end.push_back(fvb[f + 1]); }
      // segment chunks of this formula: about one segment per item slot in
      // the flat plan and the single pass, so no slot walks several
      // segments in a row and the hottest variables spread over the chip
      // (and the variable chunks' size does not set theirs); about
      // `target` cost each in the two-phase plan
      sc.f_first[f] = sc.count();
      const int32_t s_lo = heavy_sbeg[heavy_f_first[f]], s_hi = (int32_t)seg_var.size();
      // run order of the formula's segments (chunks cover runs of it).  In
      // the flat plan by the first clause row a segment reads (segments of
      // pair records only first): the hot variables each sweep the clause
      // rows in row order, so segments of different variables that run at
      // the same time read the same rows
      for (int32_t sg = s_lo; sg < s_hi; ++sg) seg_perm.push_back(sg);
      if (flat && sord_o != 0 && s_hi > s_lo) {
        std::vector<int64_t> skey((size_t)(s_hi - s_lo));
        for (int32_t sg = s_lo; sg < s_hi; ++sg) {
          const int32_t v = seg_var[sg];
          const int64_t npv = pair_first[v + 1] - pair_first[v];
          const int64_t u0 = seg_q0[sg] - vp[v], u1 = seg_q1[sg] - vp[v];
          skey[sg - s_lo] = u1 <= npv ? -1 : (int64_t)lrec[(size_t)(lrec_ptr[v] + std::max(u0, npv) - npv)];
        }
        std::stable_sort(seg_perm.begin() + s_lo, seg_perm.end(),
                         [&](int32_t a2, int32_t b2) { return skey[a2 - s_lo] < skey[b2 - s_lo]; });
      }
      int32_t sb = s_lo;
      int64_t sacc = 0;
      const int64_t seg_target = !two ? std::max<int64_t>(64, seg_cap * ipb) : target_f;
      for (int32_t i = s_lo; i < s_hi; ++i) {
        const int32_t sg = seg_perm[i];
        for (int32_t q = seg_q0[sg]; q < seg_q1[sg]; ++q) sacc += occ_cost[q];
        if (sacc >= seg_target || i + 1 == s_hi) {
          sc.beg.push_back(sb);
          sc.end.push_back(i + 1);
          sb = i + 1;
          sacc = 0;
        }
      }
    }
    vc.f_first[F] = vc.count();
    sc.f_first[F] = sc.count();
    // XCD-aware launch order of the variable chunks (several formulas per
    // launch): workgroups are dealt to the 8 XCDs round-robin by index, so
    // formulas are split into 8 groups of balanced cost (longest first) and
    // group x's chunks are placed at indices x, x + 8, x + 16, ...; padding
    // indices (-1) do nothing.
    auto xcd_order = [&](const Chunks& ch, std::vector<int32_t>* order) {
      std::vector<int32_t> ford(F);
      for (int32_t f = 0; f < F; ++f) ford[f] = f;
      std::stable_sort(ford.begin(), ford.end(),
                       [&](int32_t a2, int32_t b2) { return fcost[a2] > fcost[b2]; });
      std::vector<int64_t> load(kXcds, 0);
      std::vector<std::vector<int32_t>> lists(kXcds);
      for (int32_t f : ford) {
        const int gsel = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[gsel] += fcost[f];
        for (int32_t cid = ch.f_first[f]; cid < ch.f_first[f + 1]; ++cid) lists[gsel].push_back(cid);
      }
      size_t longest = 0;
      for (auto& l : lists) longest = std::max(longest, l.size());
      order->assign(longest * kXcds, -1);
      for (int gsel = 0; gsel < kXcds; ++gsel)
        for (size_t i = 0; i < lists[gsel].size(); ++i) (*order)[i * kXcds + gsel] = lists[gsel][i];
    };
    const bool xcd = F > 1 && !per_formula && xcd_chunks > 0;
    if (xcd) xcd_order(vc, &vorder);
    if (xseq) {
      const int32_t C = vc.count(), per = (C + kXcds - 1) / kXcds;
      vorder.assign((size_t)per * kXcds, -1);
      for (int x = 0; x < kXcds; ++x)
        for (int32_t i = 0; i < per && x * per + i < C; ++i) vorder[(size_t)i * kXcds + x] = x * per + i;
    }
    if (dsort) {
      // item order within each variable chunk, so the variables sharing a
      // wave run their loops the same number of times: costliest first, or
      // in the flat plan by the trip counts of their three record loops
      // (first-literal pairs, other pairs, clause rows; four records per
      // trip), then whether it has clause rows at all (their inverse
      // factors are set up once per variable)
      std::vector<int64_t> key((size_t)n);
      parallel_for(n, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
          if (!flat) {
            key[v] = vcost[v];
            continue;
          }
          const int64_t tf = std::min<int64_t>((pair_mid[v] - pair_first[v] + 3) / 4, 0xffff);
          const int64_t tm = std::min<int64_t>((pair_first[v + 1] - pair_mid[v] + 3) / 4, 0xffff);
          const int64_t nr = lrec_ptr[v + 1] - lrec_ptr[v];
          key[v] = (tf << 33) | (tm << 17) | (std::min<int64_t>((nr + 3) / 4, 0xffff) << 1) |
                   (nr > 0 ? 1 : 0);
        }
      });
      vperm.resize((size_t)n);
      for (int32_t v = 0; v < n; ++v) vperm[v] = v;
      parallel_for(vc.count(), [&](int64_t c0, int64_t c1) {
        for (int64_t cc = c0; cc < c1; ++cc)
          std::stable_sort(vperm.begin() + vc.beg[cc], vperm.begin() + vc.end[cc],
                           [&](int32_t a2, int32_t b2) { return key[a2] > key[b2]; });
      });
    }
    if (flat) {
      // record ranges as [begin, end) per variable; with an item order,
      // the records are laid out in that order, so the variables sharing a
      // wave read neighbouring records
      pair_end.resize((size_t)std::max(n, 1));
      lrec_end.resize((size_t)std::max(n, 1));
      if (vperm.empty()) {
        for (int32_t v = 0; v < n; ++v) {
          pair_end[v] = pair_first[v + 1];
          lrec_end[v] = lrec_ptr[v + 1];
        }
      } else {
        std::vector<int64_t> pnew((size_t)n + 1, 0), lnew((size_t)n + 1, 0);
        for (int32_t i = 0; i < n; ++i) {
          const int32_t v = vperm[i];
          pnew[i + 1] = pnew[i] + (pair_first[v + 1] - pair_first[v]);
          lnew[i + 1] = lnew[i] + (lrec_ptr[v + 1] - lrec_ptr[v]);
        }
        std::vector<int2> pairs2(pairs.size());
        std::vector<uint32_t> lrec2(lrec.size());
        std::vector<int32_t> pb((size_t)std::max(n, 1)), pm2((size_t)std::max(n, 1)),
            lb2((size_t)std::max(n, 1)), lm2((size_t)std::max(n, 1));
        parallel_for(n, [&](int64_t i0, int64_t i1) {
          for (int64_t i = i0; i < i1; ++i) {
            const int32_t v = vperm[i];
            std::copy(pairs.begin() + pair_first[v], pairs.begin() + pair_first[v + 1],
                      pairs2.begin() + pnew[i]);
            std::copy(lrec.begin() + lrec_ptr[v], lrec.begin() + lrec_ptr[v + 1],
                      lrec2.begin() + lnew[i]);
            pb[v] = (int32_t)pnew[i];
            pm2[v] = (int32_t)(pnew[i] + (pair_mid[v] - pair_first[v]));
            pair_end[v] = (int32_t)pnew[i + 1];
            lb2[v] = (int32_t)lnew[i];
            lm2[v] = (int32_t)(lnew[i] + (lrec_mid[v] - lrec_ptr[v]));
            lrec_end[v] = (int32_t)lnew[i + 1];
          }
        });
        pairs.swap(pairs2);
        lrec.swap(lrec2);
        pb.swap(pair_first);
        pm2.swap(pair_mid);
        lb2.swap(lrec_ptr);
        lm2.swap(lrec_mid);
      }
    }
    heavy_f_first[F] = (int32_t)heavy.size();
    h->vch = vc;
    h->segch = sc;
    // (no occurrence chunks when every occurrence's partial is stored; the
    // per-formula index stays valid and empty)
    h->och.f_first.assign((size_t)F + 1, 0);
    if (two && stored < L) {
      // occurrence chunks of the two-phase plan: ranges of variable-major
      // slots of about equal gather cost (+1 per slot for its row store)
      Chunks oc;
      oc.f_first.assign((size_t)F + 1, 0);
      int64_t ototal = 0;
      std::vector<int64_t> focost((size_t)F, 0);
      for (int32_t f = 0; f < F; ++f) {
        int64_t cf = 0;
        for (int32_t q = vp[fvb[f]]; q < vp[fvb[f + 1]]; ++q) cf += occ_cost[q] + 1;
        focost[f] = cf;
        ototal += cf;
      }
      const int64_t otarget = std::max<int64_t>(64, ototal / chunks_target);
      for (int32_t f = 0; f < F; ++f) {
        oc.f_first[f] = oc.count();
        int64_t tf = otarget;
        if (per_formula) tf = std::max<int64_t>(64, focost[f] / chunks_target);
        else if (xcd) tf = std::max<int64_t>(64, focost[f] / xcd_chunks);
        const int32_t qe = vp[fvb[f + 1]];
        int32_t qb = vp[fvb[f]];
        int64_t acc = 0;
        for (int32_t q = qb; q < qe; ++q) {
          acc += occ_cost[q] + 1;
          if (acc >= tf || q + 1 == qe) {
            oc.beg.push_back(qb);
            oc.end.push_back(q + 1);
            qb = q + 1;
            acc = 0;
          }
        }
      }
      oc.f_first[F] = oc.count();
      h->och = oc;
      if (xcd) xcd_order(oc, &oorder);
    }
  }
  // One formula per launch (PLAIN): size each formula's clause chunks as if
  // it were the whole problem, as for its variable chunks, so each launch
  // still spreads over the chip.
  std::vector<int64_t> plain_targets;
  auto per_formula_targets = [&](const std::vector<int64_t>& fb,
                                 const std::vector<int64_t>& pre) -> const std::vector<int64_t>* {
    if (opt.schedule != GALSAT_SCHED_PLAIN) return nullptr;
    plain_targets.assign((size_t)F, 64);
    for (int32_t f = 0; f < F; ++f)
      plain_targets[f] = std::max<int64_t>(64, (pre[fb[f + 1]] - pre[fb[f]]) / chunks_target);
    return &plain_targets;
  };
  {
    std::vector<int64_t> pre(stored_ids.size() + 1, 0);
    for (size_t i = 0; i < stored_ids.size(); ++i)
      pre[i + 1] = pre[i] + 1 + 2 * (cp[stored_ids[i] + 1] - cp[stored_ids[i]]);
    h->sch = make_chunks(F, f_sbeg, pre, std::max<int64_t>(64, pre.back() / chunks_target),
                         per_formula_targets(f_sbeg, pre));
  }
  // XCD-aware order of the clause classes' chunks (several formulas per
  // launch): the same formula groups as the variable chunks, so a formula's
  // clause and variable work run on the same XCD.
  const bool xcd_all = F > 1 && opt.schedule != GALSAT_SCHED_PLAIN && xcd_chunks > 0;
  auto xcd_order_all = [&](const Chunks& ch, std::vector<int32_t>* order) {
    std::vector<int32_t> ford(F);
    for (int32_t f = 0; f < F; ++f) ford[f] = f;
    std::stable_sort(ford.begin(), ford.end(),
                     [&](int32_t a2, int32_t b2) { return fcost_all[a2] > fcost_all[b2]; });
    std::vector<int64_t> load(kXcds, 0);
    std::vector<std::vector<int32_t>> lists(kXcds);
    for (int32_t f : ford) {
      const int gsel = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[gsel] += fcost_all[f];
      for (int32_t cid = ch.f_first[f]; cid < ch.f_first[f + 1]; ++cid) lists[gsel].push_back(cid);
    }
    size_t longest = 0;
    for (auto& l : lists) longest = std::max(longest, l.size());
    order->assign(longest * kXcds, -1);
    for (int gsel = 0; gsel < kXcds; ++gsel)
      for (size_t i = 0; i < lists[gsel].size(); ++i) (*order)[i * kXcds + gsel] = lists[gsel][i];
  };
  std::vector<std::vector<int32_t>> cls_order((size_t)NCL);
  h->cls.resize((size_t)NCL);
  for (int c = 0; c < NCL; ++c) {
    const std::vector<int32_t>& ids = cls_ids[c];
    std::vector<int64_t> pre(ids.size() + 1, 0);
    for (size_t i = 0; i < ids.size(); ++i) pre[i + 1] = pre[i] + 1 + (cp[ids[i] + 1] - cp[ids[i]]);
    h->cls[c].kind = routes[c].kind;
    h->cls[c].param = routes[c].param;
    if (xcd_all) {
      // several formulas per launch: about xcd_chunks chunks per formula,
      // in the formula groups of the variable chunks' XCD order
      std::vector<int64_t> ft((size_t)F);
      for (int32_t f = 0; f < F; ++f)
        ft[f] = std::max<int64_t>(64, (pre[cls_fbeg[c][f + 1]] - pre[cls_fbeg[c][f]]) / xcd_chunks);
      h->cls[c].ch = make_chunks(F, cls_fbeg[c], pre, 0, &ft);
      xcd_order_all(h->cls[c].ch, &cls_order[c]);
    } else {
      h->cls[c].ch = make_chunks(F, cls_fbeg[c], pre, std::max<int64_t>(64, pre.back() / chunks_target),
                                 per_formula_targets(cls_fbeg[c], pre));
    }
  }
  // flat plan: chunks of the clause-row list, in the same formula groups
  // of the XCD-aware order as the variable chunks
  std::vector<int32_t> rorder, aorder;
  if (flat) {
    std::vector<int64_t> pre(row_ids.size() + 1, 0);
    for (size_t i = 0; i < row_ids.size(); ++i)
      pre[i + 1] = pre[i] + 1 + (cp[row_ids[i] + 1] - cp[row_ids[i]]);
    if (xcd_all) {
      std::vector<int64_t> ft((size_t)F);
      for (int32_t f = 0; f < F; ++f)
        ft[f] = std::max<int64_t>(64, (pre[f_rbeg[f + 1]] - pre[f_rbeg[f]]) / xcd_chunks);
      h->rch = make_chunks(F, f_rbeg, pre, 0, &ft);
      xcd_order_all(h->rch, &rorder);
    } else {
      h->rch = make_chunks(F, f_rbeg, pre, std::max<int64_t>(64, pre.back() / chunks_target),
                           per_formula_targets(f_rbeg, pre));
    }
  } else {
    h->rch.f_first.assign((size_t)F + 1, 0);
  }
  {
    std::vector<int64_t> pre((size_t)m + 1, 0), fb(fcb.begin(), fcb.end());
    for (int32_t t = 0; t < m; ++t) pre[t + 1] = pre[t] + 1 + (cp[t + 1] - cp[t]);
    if (xcd_all) {
      // several formulas: about xcd_chunks chunks per formula in the
      // XCD-aware order, so an XCD's resident workgroups count a few
      // formulas at a time and their packed rows stay in its L2
      std::vector<int64_t> ft((size_t)F);
      for (int32_t f = 0; f < F; ++f)
        ft[f] = std::max<int64_t>(256, (pre[fcb[f + 1]] - pre[fcb[f]]) / xcd_chunks);
      h->ach = make_chunks(F, fb, pre, 0, &ft);
      xcd_order_all(h->ach, &aorder);
    } else {
      h->ach = make_chunks(F, fb, pre, std::max<int64_t>(256, pre[m] / chunks_target));
    }
  }
  ptimer.mark("chunks");
  h->heavy_f_first = heavy_f_first;
  h->opt.plan_override = nullptr;  // only read while planning
  h->n_heavy = (int32_t)heavy.size();
  h->n_seg = (int32_t)seg_var.size();
  // partial-sum rows of a step, contiguous per formula: its variable chunks,
  // its stored-clause chunks, then its segment chunks
  // (two-phase: its occurrence chunks, then its stored-clause chunks; the
  // variable sums write no partial rows)
  const int VC = h->vch.count(), SC = h->sch.count(), GC = h->segch.count(), AC = h->ach.count();
  const int OC = h->och.count(), RC = h->rch.count();
  std::vector<int32_t> vrow(VC, 0), srow(SC), grow(GC, 0), orow(OC), rrow(RC), frow0(F), frow1(F),
      faa0(F), faa1(F);
  std::vector<std::vector<int32_t>> crow((size_t)NCL);
  for (int c = 0; c < NCL; ++c) crow[c].assign((size_t)h->cls[c].ch.count(), 0);
  auto class_rows = [&](int32_t f, int32_t* row) {
    for (int c = 0; c < NCL; ++c)
      for (int k = h->cls[c].ch.f_first[f]; k < h->cls[c].ch.f_first[f + 1]; ++k) crow[c][k] = (*row)++;
  };
  {
    int32_t row = 0;
    for (int32_t f = 0; f < F; ++f) {
      frow0[f] = row;
      if (two) {
        for (int c = h->och.f_first[f]; c < h->och.f_first[f + 1]; ++c) orow[c] = row++;
        for (int c = h->sch.f_first[f]; c < h->sch.f_first[f + 1]; ++c) srow[c] = row++;
        class_rows(f, &row);
        frow1[f] = row;
        faa0[f] = h->ach.f_first[f];
        faa1[f] = h->ach.f_first[f + 1];
        continue;
      }
      for (int c = h->vch.f_first[f]; c < h->vch.f_first[f + 1]; ++c) vrow[c] = row++;
      for (int c = h->rch.f_first[f]; c < h->rch.f_first[f + 1]; ++c) rrow[c] = row++;
      for (int c = h->sch.f_first[f]; c < h->sch.f_first[f + 1]; ++c) srow[c] = row++;
      class_rows(f, &row);
      for (int c = h->segch.f_first[f]; c < h->segch.f_first[f + 1]; ++c) grow[c] = row++;
      frow1[f] = row;
      faa0[f] = h->ach.f_first[f];
      faa1[f] = h->ach.f_first[f + 1];
    }
    h->step_rows = row;
  }
  std::vector<int32_t> fnone(F, 0);
  // schedule
  h->schedule = opt.schedule == GALSAT_SCHED_PLAIN ? GALSAT_SCHED_PLAIN
              : lds_rg                                ? GALSAT_SCHED_LDS
                                                      : GALSAT_SCHED_GENERAL;
  h->lds_rg = lds_rg;
  h->lds_stage = lds_stage;
  h->lds_nocc = lds_nocc;
  h->nf_max = 0;
  for (int32_t f = 0; f < F; ++f) h->nf_max = std::max(h->nf_max, fvb[f + 1] - fvb[f]);

  // ---- device upload and workspace
  galsat_ctx* c = h.get();
#define UP(dst, vec)                                                                     \
  do {                                                                                   \
    if ((he = c->upload(&c->dst, (vec).data(), (vec).size(), s)) != hipSuccess)         \
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,    \
                         std::string("upload " #dst ": ") + hipGetErrorString(he));      \
  } while (0)
#define AL(dst, count)                                                                   \
  do {                                                                                   \
    if ((he = c->alloc(&c->dst, (size_t)(count))) != hipSuccess)                        \
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,    \
                         std::string("allocate " #dst ": ") + hipGetErrorString(he));    \
  } while (0)
#define UPP(dst, ptr, count)                                                             \
  do {                                                                                   \
    if ((he = c->upload(&c->dst, (ptr), (size_t)(count), s)) != hipSuccess)              \
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,    \
                         std::string("upload " #dst ": ") + hipGetErrorString(he));      \
  } while (0)
  UPP(clause_ptr, cp, m + 1);
  UPP(clause_lits, cl, L);
  UPP(var_ptr, vp, n + 1);
#undef UPP
  // (the flat plan builds no old-style records: one placeholder entry)
  if ((he = c->upload(&c->occ4, occ4.get(), flat ? (size_t)1 : (size_t)L, s)) != hipSuccess ||
      (need_x && (he = c->upload(&c->occx, occx.get(), (size_t)L, s)) != hipSuccess))
    return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,
                       std::string("upload occurrence records: ") + hipGetErrorString(he));
  if (!need_x && (he = c->alloc(&c->occx, 1)) != hipSuccess)
    return create_fail(GALSAT_EDEVICE, "allocate record words");
  if (stored > 0 && (he = c->upload(&c->lit_dslot, lit_dslot.get(), (size_t)L, s)) != hipSuccess)
    return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,
                       std::string("upload stored rows: ") + hipGetErrorString(he));
  UP(var_formula, var_formula);
  UP(stored_ids, stored_ids);
  UP(vch_beg, c->vch.beg);
  UP(vch_end, c->vch.end);
  UP(vch_row, vrow);
  UP(vch_order, vorder);
  c->n_vorder = (int32_t)vorder.size();
  if (!vperm.empty()) UP(var_perm, vperm);
  std::unique_ptr<int32_t[]> own;  // kept until the uploads have completed
  if (two) {
    UP(och_beg, c->och.beg);
    UP(och_end, c->och.end);
    UP(och_row, orow);
    UP(och_order, oorder);
    c->n_oorder = (int32_t)oorder.size();
    own.reset(new int32_t[(size_t)L + 1]);
    parallel_for(n, [&](int64_t v0, int64_t v1) {
      for (int64_t v = v0; v < v1; ++v)
        for (int32_t q = vp[v]; q < vp[v + 1]; ++q) own[q] = (int32_t)v;
    });
    if ((he = c->upload(&c->occ_own, own.get(), (size_t)L, s)) != hipSuccess)
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,
                         std::string("upload slot owners: ") + hipGetErrorString(he));
  }
  UP(sch_beg, c->sch.beg);
  UP(sch_end, c->sch.end);
  UP(sch_row, srow);
  std::vector<std::vector<int32_t>> cls_packed((size_t)NCL);
  for (int k = 0; k < NCL; ++k) {
    if (routes[k].kind != kClassShort) continue;
    const int KS = routes[k].param;
    const std::vector<int32_t>& ids = cls_ids[k];
    std::vector<int32_t>& pk = cls_packed[k];
    pk.assign(ids.size() * 2 * KS, 0);
    parallel_for((int64_t)ids.size(), [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        const int32_t t = ids[(size_t)i], kk = cp[t + 1] - cp[t];
        int32_t* e = pk.data() + i * 2 * KS;
        for (int u = 0; u < KS; ++u) {
          e[u] = u < kk ? cl[cp[t] + u] : 0;
          e[KS + u] = u < kk ? lit_dslot[cp[t] + u] : -1;
        }
      }
    });
  }
  for (int k = 0; k < NCL; ++k) {
    galsat_ctx::ClauseClass& cc = c->cls[k];
    cc.n_order = (int32_t)cls_order[k].size();
    if (cc.n_order > 0 &&
        (he = c->upload(&cc.order, cls_order[k].data(), cls_order[k].size(), s)) != hipSuccess)
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,
                         std::string("upload clause order: ") + hipGetErrorString(he));
    if (!cls_packed[k].empty() &&
        (he = c->upload(&cc.packed, cls_packed[k].data(), cls_packed[k].size(), s)) != hipSuccess)
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,
                         std::string("upload packed clauses: ") + hipGetErrorString(he));
    if ((he = c->upload(&cc.ids, cls_ids[k].data(), cls_ids[k].size(), s)) != hipSuccess ||
        (he = c->upload(&cc.beg, cc.ch.beg.data(), cc.ch.beg.size(), s)) != hipSuccess ||
        (he = c->upload(&cc.end, cc.ch.end.data(), cc.ch.end.size(), s)) != hipSuccess ||
        (he = c->upload(&cc.row, crow[k].data(), crow[k].size(), s)) != hipSuccess)
      return create_fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE,
                         std::string("upload clause classes: ") + hipGetErrorString(he));
  }
  if (flat) {
    UP(pairs, pairs);
    UP(pair_first, pair_first);
    UP(pair_end, pair_end);
    UP(pair_mid, pair_mid);
    UP(lrec, lrec);
    UP(lrec_ptr, lrec_ptr);
    UP(lrec_mid, lrec_mid);
    UP(lrec_end, lrec_end);
    UP(row_ids, row_ids);
    UP(rch_beg, c->rch.beg);
    UP(rch_end, c->rch.end);
    UP(rch_row, rrow);
    UP(rch_order, rorder);
    UP(rlit_ptr, rlit_ptr);
    UP(rlits, rlits);
    {
      std::vector<int32_t> rfvb((size_t)std::max(c->rch.count(), 1), 0);
      for (int32_t f = 0; f < F; ++f)
        for (int cc = c->rch.f_first[f]; cc < c->rch.f_first[f + 1]; ++cc) rfvb[cc] = fvb[f];
      UP(rch_fvb, rfvb);
    }
    c->n_rorder = (int32_t)rorder.size();
    std::vector<int32_t> vfvb((size_t)std::max(VC, 1), 0);
    for (int32_t f = 0; f < F; ++f)
      for (int ch = c->vch.f_first[f]; ch < c->vch.f_first[f + 1]; ++ch) vfvb[ch] = fvb[f];
    UP(vch_fvb, vfvb);
    std::vector<int32_t> vrb((size_t)std::max(VC, 1), 0), frb((size_t)F + 1);
    for (int32_t f = 0; f < F; ++f)
      for (int ch = c->vch.f_first[f]; ch < c->vch.f_first[f + 1]; ++ch) vrb[ch] = (int32_t)f_rbeg[f];
    for (int32_t f = 0; f <= F; ++f) frb[f] = (int32_t)f_rbeg[f];
    UP(vch_rbase, vrb);
    UP(f_rbeg, frb);
    AL(qrow, (size_t)std::max<size_t>(row_ids.size(), 1) * (size_t)c->ld);
  }
  UP(segch_beg, c->segch.beg);
  UP(segch_end, c->segch.end);
  UP(segch_row, grow);
  UP(ach_beg, c->ach.beg);
  UP(ach_end, c->ach.end);
  UP(ach_order, aorder);
  c->n_aorder = (int32_t)aorder.size();
  UP(seg_var, seg_var);
  UP(seg_perm, seg_perm);
  UP(seg_q0, seg_q0);
  UP(seg_q1, seg_q1);
  UP(heavy_var, heavy);
  UP(heavy_sbeg, heavy_sbeg);
  for (int32_t f = 0; f < F; ++f) {
    c->max_step_rows = std::max(c->max_step_rows, frow1[f] - frow0[f]);
    c->max_all_rows = std::max(c->max_all_rows, faa1[f] - faa0[f]);
  }
  UP(fin_step_a0, frow0);
  UP(fin_step_a1, frow1);
  UP(fin_all_a0, faa0);
  UP(fin_all_a1, faa1);
  UP(n_empty, n_empty);
  UP(zero_empty, fnone);
  UP(f_vbeg, fvb);
  UP(f_cbeg, fcb);
  // LDS schedule: formulas in LPT order (most occurrences first, ties by
  // id), so the longest workgroups start first and the tail is short
  std::vector<int32_t> lds_order;
  if (lds_rg) {
    lds_order.resize((size_t)F);
    for (int32_t f = 0; f < F; ++f) lds_order[f] = f;
    if (ldslpt_o != 0)
      std::stable_sort(lds_order.begin(), lds_order.end(), [&](int32_t p, int32_t q) {
        return vp[fvb[p + 1]] - vp[fvb[p]] > vp[fvb[q + 1]] - vp[fvb[q]];
      });
  }
  UP(lds_order, lds_order);
  if (two) AL(D, (size_t)std::max<int64_t>(L, 1) * (size_t)c->ldD);  // one row per slot
  else if (stored > 0) AL(D, (size_t)stored * (size_t)c->ldD);
  AL(xa, (size_t)n * c->ld);
  AL(xb, (size_t)n * c->ld);
  const int64_t rows = std::max<int64_t>(c->step_rows, AC);
  AL(gseg, (size_t)std::max<int64_t>(c->n_seg, 1) * R);
  AL(loss_part, (size_t)std::max<int64_t>(rows, 1) * R);
  AL(unsat_part, (size_t)std::max<int64_t>(rows, 1) * R);
  AL(bits, (size_t)n * ((R + 63) / 64));
  AL(best_tmp, F);
  AL(fin_l, kFinalizeScratch);
  AL(fin_u, kFinalizeScratch);
  AL(unsat_tmp, (size_t)F * R);
  AL(work_counter, 1);
#undef UP
#undef AL
  if ((he = hipStreamSynchronize(s)) != hipSuccess)
    return create_fail(GALSAT_EDEVICE, std::string("create: ") + hipGetErrorString(he));
  ptimer.mark("upload");
  *out = h.release();
  return GALSAT_OK;
}

extern "C" galsat_status galsat_destroy(galsat_handle h) {
  if (!h) return GALSAT_OK;
  (void)hipDeviceSynchronize();
  delete h;
  return GALSAT_OK;
}

extern "C" galsat_status galsat_set_adam_step(galsat_handle h, int32_t t) {
  GS_CHECK_HANDLE(h);
  if (t < 0) return h->fail(GALSAT_EINVAL, "adam step must be >= 0");
  h->adam_t = t;
  return GALSAT_OK;
}

extern "C" galsat_status galsat_get_info(galsat_handle h, galsat_info* info) {
  if (!h || !info) return GALSAT_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->num_formulas = h->F;
  info->n_vars = h->n;
  info->n_clauses = h->m;
  info->n_lits = h->L;
  info->restarts = h->R;
  info->max_clause_len = h->kmax;
  info->recompute_max_len = h->krec;
  info->stored_lits = h->stored;
  info->schedule = h->schedule;
  info->lanes_per_item = h->tile.lpi;
  info->restarts_per_lane = h->tile.rpl;
  info->var_chunks = h->vch.count() + h->segch.count();
  info->clause_chunks = h->sch.count();
  for (const galsat_ctx::ClauseClass& cc : h->cls) info->clause_chunks += cc.ch.count();
  info->two_phase = h->two_phase;
  info->xseq_chunks = h->xseq;
  info->device_bytes = h->device_bytes;
  info->adam_step = h->adam_t;
  info->lds_restarts_per_group = h->lds_rg;
  info->lds_staged = h->lds_stage;
  info->flat = h->flat;
  info->clause_rows = h->flat ? (int32_t)(h->rch.count() > 0 ? h->rch.end.back() : 0) : 0;
  if (h->flat) info->clause_chunks = h->rch.count();
  return GALSAT_OK;
}

extern "C" galsat_status galsat_init_state(galsat_handle h, float* x, int32_t ldx, uint64_t seed,
                                           void* stream) {
  GS_CHECK_HANDLE(h);
  if (!x && h->n > 0) return h->fail(GALSAT_EINVAL, "x is NULL");
  if (ldx < h->R) return h->fail(GALSAT_EINVAL, "ldx < restarts");
  GS_HIP(h, launch_init_state(x, ldx, h->n, h->R, seed, static_cast<hipStream_t>(stream)), "init_state");
  return GALSAT_OK;
}

namespace {

bool aligned_for(const void* p, int32_t ld, int rpl) {
  if (rpl == 1) return true;
  return (reinterpret_cast<uintptr_t>(p) % (4 * rpl) == 0) && (ld % rpl == 0);
}

Tile tile_for(const galsat_ctx* h, const void* a, int32_t lda, const void* b, int32_t ldb) {
  Tile t = h->tile;
  if (!aligned_for(a, lda, t.rpl) || (b && !aligned_for(b, ldb, t.rpl))) {
    t.rpl = 1;
    t.lpi = std::max(4, std::min(64, pow2_ceil(h->R)));
  }
  return t;
}

VarPassArgs var_args(const galsat_ctx* h) {
  VarPassArgs a{};
  a.var_ptr = h->var_ptr;
  a.occ = h->occ4;
  a.occx = h->occx;
  a.clause_ptr = h->clause_ptr;
  a.clause_lits = h->clause_lits;
  a.chunk_vbeg = h->vch_beg;
  a.chunk_vend = h->vch_end;
  a.chunk_row = h->vch_row;
  a.seg_var = h->seg_var;
  a.seg_perm = h->seg_perm;
  a.seg_q0 = h->seg_q0;
  a.seg_q1 = h->seg_q1;
  a.gseg = h->gseg;
  a.heavy_var = h->heavy_var;
  a.heavy_sbeg = h->heavy_sbeg;
  a.var_formula = h->var_formula;
  a.stream_items = h->stream_items;
  a.xcd_pin = h->xcd_pin;
  a.occ_own = h->occ_own;
  a.var_perm = h->var_perm;
  a.C = h->D;
  a.D = h->D;
  a.ldD = h->ldD;
  a.pairs = h->pairs;
  a.pair_first = h->pair_first;
  a.pair_end = h->pair_end;
  a.pair_mid = h->pair_mid;
  a.lrec = h->lrec;
  a.lrec_ptr = h->lrec_ptr;
  a.lrec_mid = h->lrec_mid;
  a.lrec_end = h->lrec_end;
  a.prefetch = h->prefetch;
  a.qrow = h->qrow;
  a.ldq = h->ld;
  a.chunk_fvb = h->vch_fvb;
  a.chunk_rbase = h->vch_rbase;
  a.f_vbeg = h->f_vbeg;
  a.f_rbeg = h->f_rbeg;
  a.loss_part = h->loss_part;
  a.unsat_part = h->unsat_part;
  a.R = h->R;
  a.lr = h->opt.lr;
  a.b1 = h->opt.beta1;
  a.b2 = h->opt.beta2;
  a.eps = h->opt.eps;
  return a;
}

// The two-phase gradient of one restart-tile group (after the clause pass
// has written the stored clauses' contributions): every recomputed
// occurrence's contribution, then each whole variable's sum with the
// epilogue, then the split variables' segment sums and their finish.
galsat_status two_phase_passes(galsat_ctx* h, VarPassArgs va, Tile t, int mode, int f0, int f1,
                               hipStream_t s) {
  const bool all = f0 == 0 && f1 == h->F;
  {
    VarPassArgs oa = va;
    oa.chunk_vbeg = h->och_beg;
    oa.chunk_vend = h->och_end;
    oa.chunk_row = h->och_row;
    oa.chunk_base = h->och.f_first[f0];
    int blocks = h->och.f_first[f1] - h->och.f_first[f0];
    oa.chunk_order = nullptr;
    if (h->n_oorder > 0 && all) {
      oa.chunk_order = h->och_order;
      oa.chunk_base = 0;
      blocks = h->n_oorder;
    }
    ProfScope _ps(h, GALSAT_K_OCC_PASS, s);
    GS_HIP(h, launch_occ_pass(oa, t, blocks, s), "occurrence pass");
  }
  {
    VarPassArgs sa = va;
    sa.chunk_vbeg = h->vch_beg;
    sa.chunk_vend = h->vch_end;
    sa.chunk_base = h->vch.f_first[f0];
    int blocks = h->vch.f_first[f1] - h->vch.f_first[f0];
    sa.chunk_order = nullptr;
    if (h->n_vorder > 0 && all) {
      sa.chunk_order = h->vch_order;
      sa.chunk_base = 0;
      blocks = h->n_vorder;
    }
    ProfScope _ps(h, GALSAT_K_VAR_SUM, s);
    GS_HIP(h, launch_var_sum(sa, mode, t, blocks, s), "variable sum");
  }
  const int gc0 = h->segch.f_first[f0], gc1 = h->segch.f_first[f1];
  if (gc1 > gc0) {
    VarPassArgs ga = va;
    ga.chunk_vbeg = h->segch_beg;
    ga.chunk_vend = h->segch_end;
    ga.chunk_base = gc0;
    ga.chunk_order = nullptr;
    {
      ProfScope _ps(h, GALSAT_K_SEG_PASS, s);
      GS_HIP(h, launch_seg_sum(ga, t, gc1 - gc0, s), "segment sum");
    }
    ProfScope _ps(h, GALSAT_K_HEAVY, s);
    GS_HIP(h, launch_heavy_finish(va, mode, t, h->heavy_f_first[f0], h->heavy_f_first[f1], s),
           "split-variable finish");
  }
  return GALSAT_OK;
}

// The flat plan's gradient of one restart-tile group: the clause rows of
// every clause that is not 3 literals long, then the whole variables (pair
// records and clause rows) with the epilogue, then the split variables'
// segments and their finish.
galsat_status flat_passes(galsat_ctx* h, VarPassArgs va, Tile t, int mode, int f0, int f1,
                          hipStream_t s) {
  const bool all = f0 == 0 && f1 == h->F;
  // state rows are addressed by 32-bit byte offsets within a formula
  if ((int64_t)h->nf_max * va.ldx * 4 >= (int64_t(1) << 32))
    return h->fail(GALSAT_EUNSUPPORTED, "flat plan: a formula's state at this row stride exceeds 4 GiB");
  const int rc0 = h->rch.f_first[f0], rc1 = h->rch.f_first[f1];
  if (rc1 > rc0) {
    ClausePassArgs ca{};
    ca.clause_ptr = h->clause_ptr;
    ca.clause_lits = h->clause_lits;
    ca.clause_ids = h->row_ids;
    ca.chunk_cbeg = h->rch_beg;
    ca.chunk_cend = h->rch_end;
    ca.chunk_row = h->rch_row;
    ca.chunk_base = rc0;
    int blocks = rc1 - rc0;
    if (h->n_rorder > 0 && all) {
      ca.chunk_order = h->rch_order;
      ca.chunk_base = 0;
      blocks = h->n_rorder;
    }
    ca.tile_base = va.tile_base;
    ca.tile_count = va.tile_count;
    ca.x = va.x;
    ca.ldx = va.ldx;
    ca.loss_part = h->loss_part;
    ca.unsat_part = h->unsat_part;
    ca.R = h->R;
    ca.qrow = h->qrow;
    ca.ldq = h->ld;
    ca.rlit_ptr = h->rlit_ptr;
    ca.rlits = h->rlits;
    ca.chunk_fvb = h->rch_fvb;
    ProfScope _ps(h, GALSAT_K_CLAUSE_PASS, s);
    GS_HIP(h, launch_row_clause(ca, t, blocks, s), "clause-row pass");
  }
  {
    VarPassArgs a = va;
    a.chunk_vbeg = h->vch_beg;
    a.chunk_vend = h->vch_end;
    a.chunk_row = h->vch_row;
    a.chunk_base = h->vch.f_first[f0];
    int blocks = h->vch.f_first[f1] - h->vch.f_first[f0];
    a.chunk_order = nullptr;
    if (h->n_vorder > 0 && all) {
      a.chunk_order = h->vch_order;
      a.chunk_base = 0;
      blocks = h->n_vorder;
    }
    ProfScope _ps(h, GALSAT_K_VAR_PASS, s);
    GS_HIP(h, launch_flat_var(a, mode, t, blocks, s), "flat variable pass");
  }
  const int gc0 = h->segch.f_first[f0], gc1 = h->segch.f_first[f1];
  if (gc1 > gc0) {
    VarPassArgs ga = va;
    ga.chunk_vbeg = h->segch_beg;
    ga.chunk_vend = h->segch_end;
    ga.chunk_row = h->segch_row;
    ga.chunk_base = gc0;
    ga.chunk_order = nullptr;
    {
      ProfScope _ps(h, GALSAT_K_SEG_PASS, s);
      GS_HIP(h, launch_flat_seg(ga, t, gc1 - gc0, s), "flat segment pass");
    }
    ProfScope _ps(h, GALSAT_K_HEAVY, s);
    GS_HIP(h, launch_heavy_finish(va, mode, t, h->heavy_f_first[f0], h->heavy_f_first[f1], s),
           "split-variable finish");
  }
  return GALSAT_OK;
}

// Gradient passes for formulas [f0, f1) at state x: stored-clause partials,
// whole variables, segments of split variables, then the split variables'
// sums; every pass ends in the epilogue `mode` writing `out`.  The per-chunk
// loss and unsat partial rows of the formulas are all written.
galsat_status grad_passes(galsat_ctx* h, Tile t, int mode, const float* x, int32_t ldx,
                          float* out, int32_t ldo, float* mom, float* vel, int32_t ldm,
                          const float* upstream, int f0, int f1, hipStream_t s) {
  VarPassArgs va = var_args(h);
  va.x = x;
  va.ldx = ldx;
  va.out = out;
  va.ldo = ldo;
  va.mom = mom;
  va.vel = vel;
  va.ldm = ldm;
  va.upstream = upstream;
  if (mode == kModeAdam) {
    const int tt = h->adam_t + 1;
    va.inv_c1 = 1.0 / (1.0 - std::pow((double)h->opt.beta1, tt));
    va.inv_c2 = 1.0 / (1.0 - std::pow((double)h->opt.beta2, tt));
  }
  const int sc0 = h->sch.f_first[f0], sc1 = h->sch.f_first[f1];
  const int vc0 = h->vch.f_first[f0], vc1 = h->vch.f_first[f1];
  const int gc0 = h->segch.f_first[f0], gc1 = h->segch.f_first[f1];
  const int tiles_all = (h->R + t.tile() - 1) / t.tile();
  // the planned group size applies to the planned tile; a fallback tile
  // (unaligned caller buffers) keeps the same restart span per launch
  const int tg = std::max(1, h->tgroup * h->tile.tile() / t.tile());
  galsat_status st = GALSAT_OK;
  for (int tb = 0; tb < tiles_all; tb += tg) {
    const int tc = std::min(tg, tiles_all - tb);
    if (h->stored > 0 && sc1 > sc0) {
      ClausePassArgs ca{};
      ca.clause_ptr = h->clause_ptr;
      ca.clause_lits = h->clause_lits;
      ca.lit_dslot = h->lit_dslot;
      ca.clause_ids = h->stored_ids;
      ca.chunk_cbeg = h->sch_beg;
      ca.chunk_cend = h->sch_end;
      ca.chunk_row = h->sch_row;
      ca.chunk_base = sc0;
      ca.tile_base = tb;
      ca.tile_count = tc;
      ca.x = x;
      ca.ldx = ldx;
      ca.D = h->D;
      ca.ldD = h->ldD;
      ca.loss_part = h->loss_part;
      ca.unsat_part = h->unsat_part;
      ca.R = h->R;
      ProfScope _ps(h, GALSAT_K_CLAUSE_PASS, s);
      GS_HIP(h, launch_clause_pass(ca, true, t, sc1 - sc0, s), "clause pass");
    }
    for (const galsat_ctx::ClauseClass& cc : h->cls) {
      const int c0 = cc.ch.f_first[f0], c1 = cc.ch.f_first[f1];
      if (c1 <= c0) continue;
      ClausePassArgs ca{};
      ca.clause_ptr = h->clause_ptr;
      ca.clause_lits = h->clause_lits;
      ca.lit_dslot = h->lit_dslot;
      ca.clause_ids = cc.ids;
      ca.packed = cc.packed;
      ca.chunk_cbeg = cc.beg;
      ca.chunk_cend = cc.end;
      ca.chunk_row = cc.row;
      ca.chunk_base = c0;
      int blocks = c1 - c0;
      if (cc.n_order > 0 && f0 == 0 && f1 == h->F) {
        ca.chunk_order = cc.order;
        ca.chunk_base = 0;
        blocks = cc.n_order;
      }
      ca.tile_base = tb;
      ca.tile_count = tc;
      ca.x = x;
      ca.ldx = ldx;
      ca.D = h->D;
      ca.ldD = h->ldD;
      ca.loss_part = h->loss_part;
      ca.unsat_part = h->unsat_part;
      ca.R = h->R;
      ProfScope _ps(h, GALSAT_K_CLAUSE_PASS, s);
      if (cc.kind == kClassShort) {
        GS_HIP(h, launch_short_clause(ca, t, cc.param, blocks, s), "short clause pass");
      } else if (t.lpi == h->tile.lpi && t.rpl == h->tile.rpl) {
        GS_HIP(h, launch_wave_clause(ca, t, cc.param, blocks, s), "wave clause pass");
      } else {
        // the classes were routed for the planned tile; a fallback tile
        // (unaligned caller buffers) runs them through the sweeping pass
        GS_HIP(h, launch_clause_pass(ca, true, t, blocks, s), "clause pass");
      }
    }
    va.tile_base = tb;
    va.tile_count = tc;
    if (h->flat) {
      st = flat_passes(h, va, t, mode, f0, f1, s);
      if (st != GALSAT_OK) return st;
      continue;
    }
    if (h->two_phase) {
      st = two_phase_passes(h, va, t, mode, f0, f1, s);
      if (st != GALSAT_OK) return st;
      continue;
    }
    va.chunk_vbeg = h->vch_beg;
    va.chunk_vend = h->vch_end;
    va.chunk_row = h->vch_row;
    va.chunk_base = vc0;
    int vblocks = vc1 - vc0;
    va.chunk_order = nullptr;
    if (h->n_vorder > 0 && f0 == 0 && f1 == h->F) {
      va.chunk_order = h->vch_order;
      va.chunk_base = 0;
      vblocks = h->n_vorder;
    }
    {
      ProfScope _ps(h, GALSAT_K_VAR_PASS, s);
      GS_HIP(h, launch_var_pass(va, mode, t, vblocks, s), "var pass");
    }
    va.chunk_order = nullptr;
    if (gc1 > gc0) {
      VarPassArgs sa = va;
      sa.chunk_vbeg = h->segch_beg;
      sa.chunk_vend = h->segch_end;
      sa.chunk_row = h->segch_row;
      sa.chunk_base = gc0;
      {
        ProfScope _ps(h, GALSAT_K_SEG_PASS, s);
        GS_HIP(h, launch_var_seg(sa, t, gc1 - gc0, s), "segment pass");
      }
      ProfScope _ps(h, GALSAT_K_HEAVY, s);
      GS_HIP(h, launch_heavy_finish(va, mode, t, h->heavy_f_first[f0], h->heavy_f_first[f1], s),
             "split-variable finish");
    }
  }
  return GALSAT_OK;
}

galsat_status finalize_step(galsat_ctx* h, float* loss, int32_t* unsat, int f0, int f1,
                            hipStream_t s) {
  if (!loss && !unsat) return GALSAT_OK;
  FinalizeArgs fa{h->fin_step_a0, h->fin_step_a1, h->n_empty, h->loss_part, h->unsat_part,
                  loss, unsat, h->R, f0, h->fin_l, h->fin_u, 1, h->max_step_rows};
  ProfScope _ps(h, GALSAT_K_FINALIZE, s);
  GS_HIP(h, launch_finalize(fa, f1 - f0, s), "finalize");
  return GALSAT_OK;
}

}  // namespace

extern "C" galsat_status galsat_loss_grad(galsat_handle h, const float* x, int32_t ldx,
                                          const float* upstream, float* loss, float* grad,
                                          void* stream) {
  GS_CHECK_HANDLE(h);
  if ((!x && h->n > 0) || !loss) return h->fail(GALSAT_EINVAL, "x and loss are required");
  if (ldx < h->R) return h->fail(GALSAT_EINVAL, "ldx < restarts");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t F = h->F;
  if (!grad) {
    // forward only: one clause pass over every clause, nothing stored
    Tile t = tile_for(h, x, ldx, nullptr, 0);
    ClausePassArgs a{};
    a.clause_ptr = h->clause_ptr;
    a.clause_lits = h->clause_lits;
    a.clause_ids = nullptr;
    a.chunk_cbeg = h->ach_beg;
    a.chunk_cend = h->ach_end;
    a.chunk_row = nullptr;
    a.x = x;
    a.ldx = ldx;
    a.loss_part = h->loss_part;
    a.unsat_part = h->unsat_part;
    a.R = h->R;
    {
      ProfScope _ps(h, GALSAT_K_CLAUSE_PASS, s);
      GS_HIP(h, launch_clause_pass(a, false, t, h->ach.count(), s), "clause pass");
    }
    FinalizeArgs fa{h->fin_all_a0, h->fin_all_a1, h->zero_empty, h->loss_part, h->unsat_part,
                    loss, nullptr, h->R, 0, h->fin_l, h->fin_u, 1, h->max_all_rows};
    ProfScope _ps(h, GALSAT_K_FINALIZE, s);
    GS_HIP(h, launch_finalize(fa, F, s), "finalize");
    return GALSAT_OK;
  }
  Tile t = tile_for(h, x, ldx, grad, ldx);
  galsat_status st = grad_passes(h, t, kModeGrad, x, ldx, grad, ldx, nullptr, nullptr, 0,
                                 upstream, 0, F, s);
  if (st != GALSAT_OK) return st;
  return finalize_step(h, loss, nullptr, 0, F, s);
}

namespace {

// One step from xin to xout (internal layout) for formulas [f0, f1).
galsat_status general_step(galsat_ctx* h, Tile t, const float* xin, float* xout, float* mom,
                           float* vel, int32_t ldm, float* loss_row, int32_t* unsat_row,
                           hipStream_t s, int f0, int f1) {
  const int mode = h->opt.optimizer == GALSAT_OPT_ADAM ? kModeAdam : kModeSGD;
  galsat_status st = grad_passes(h, t, mode, xin, h->ld, xout, h->ld, mom, vel, ldm, nullptr,
                                 f0, f1, s);
  if (st != GALSAT_OK) return st;
  return finalize_step(h, loss_row, unsat_row, f0, f1, s);
}

}  // namespace

namespace {

// Enqueues `steps` iterations.  When the caller's state already has the
// internal layout the iterations ping-pong between it and one internal
// buffer, arranged so the last one lands in x (one copy for an odd count,
// none for an even one); otherwise x is copied in and out.
galsat_status enqueue_steps(galsat_ctx* h, Tile t, float* x, int32_t ldx, float* mom, float* vel,
                            int32_t steps, float* loss_trace, int32_t* unsat_trace,
                            hipStream_t s) {
  const bool adam = h->opt.optimizer == GALSAT_OPT_ADAM;
  const int64_t FR = (int64_t)h->F * h->R;
  const bool direct = ldx == h->ld && aligned_for(x, ldx, h->tile.rpl);
  float *cur, *nxt;
  if (direct && steps % 2 == 0) {
    cur = x;
    nxt = h->xa;
  } else {
    ProfScope _ps(h, GALSAT_K_COPY, s);
    GS_HIP(h, launch_copy_state(x, ldx, h->xa, h->ld, h->n, h->R, s), "copy in");
    cur = h->xa;
    nxt = direct ? x : h->xb;
  }
  for (int32_t k = 0; k < steps; ++k) {
    float* lrow = loss_trace ? loss_trace + k * FR : nullptr;
    int32_t* urow = unsat_trace ? unsat_trace + k * FR : nullptr;
    if (h->schedule == GALSAT_SCHED_PLAIN) {
      for (int f = 0; f < h->F; ++f) {
        galsat_status st = general_step(h, t, cur, nxt, mom, vel, ldx, lrow, urow, s, f, f + 1);
        if (st != GALSAT_OK) return st;
      }
    } else {
      galsat_status st = general_step(h, t, cur, nxt, mom, vel, ldx, lrow, urow, s, 0, h->F);
      if (st != GALSAT_OK) return st;
    }
    if (adam) h->adam_t++;
    std::swap(cur, nxt);
  }
  if (cur != x) {
    ProfScope _ps(h, GALSAT_K_COPY, s);
    GS_HIP(h, launch_copy_state(cur, h->ld, x, ldx, h->n, h->R, s), "copy out");
  }
  return GALSAT_OK;
}

}  // namespace

namespace {

// Graph replay: the whole call (every step's launches) is captured once on a
// private stream and replayed on the caller's stream while the call's
// arguments stay the same.  Adam's bias correction changes the launch
// arguments every step, and profiling records events, so both run eagerly.
galsat_status capture_steps(galsat_ctx* h, Tile t, float* x, int32_t ldx, int32_t steps,
                            float* loss_trace, int32_t* unsat_trace) {
  const galsat_ctx::GraphKey key{x, ldx, steps, loss_trace, unsat_trace};
  if (h->graph_exec && h->graph_key == key) return GALSAT_OK;
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  h->graph_exec = nullptr;
  if (!h->cap_stream)
    GS_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "capture stream");
  GS_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed), "begin capture");
  galsat_status st = enqueue_steps(h, t, x, ldx, nullptr, nullptr, steps, loss_trace, unsat_trace,
                                   h->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
  if (st != GALSAT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return h->dev_fail(e, "end capture");
  e = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    h->graph_exec = nullptr;
    return h->dev_fail(e, "graph instantiate");
  }
  h->graph_key = key;
  return GALSAT_OK;
}

}  // namespace

extern "C" galsat_status galsat_step_prepare(galsat_handle h, float* x, int32_t ldx,
                                             float* opt_state, int32_t steps, float* loss_trace,
                                             int32_t* unsat_trace) {
  GS_CHECK_HANDLE(h);
  if (!x && h->n > 0) return h->fail(GALSAT_EINVAL, "x is NULL");
  if (ldx < h->R) return h->fail(GALSAT_EINVAL, "ldx < restarts");
  if (steps <= 0) return h->fail(GALSAT_EINVAL, "steps must be >= 1");
  (void)opt_state;
  if (h->lds_rg) return GALSAT_OK;  // galsat_step is one launch already
  if (!h->opt.use_graph || h->opt.optimizer == GALSAT_OPT_ADAM || h->prof)
    return h->fail(GALSAT_EUNSUPPORTED, "this handle runs galsat_step eagerly");
  return capture_steps(h, h->tile, x, ldx, steps, loss_trace, unsat_trace);
}

extern "C" galsat_status galsat_step(galsat_handle h, float* x, int32_t ldx, float* opt_state,
                                     int32_t steps, float* loss_trace, int32_t* unsat_trace,
                                     void* stream) {
  GS_CHECK_HANDLE(h);
  if (!x && h->n > 0) return h->fail(GALSAT_EINVAL, "x is NULL");
  if (ldx < h->R) return h->fail(GALSAT_EINVAL, "ldx < restarts");
  if (steps < 0) return h->fail(GALSAT_EINVAL, "steps must be >= 0");
  const bool adam = h->opt.optimizer == GALSAT_OPT_ADAM;
  if (adam && !opt_state && h->n > 0) return h->fail(GALSAT_EINVAL, "Adam needs opt_state");
  if (steps == 0) return GALSAT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* mom = adam ? opt_state : nullptr;
  float* vel = adam ? opt_state + (int64_t)h->n * ldx : nullptr;
  // the internal state is aligned for the planned tile; the caller's Adam
  // moments may not be
  const Tile t = adam ? tile_for(h, mom, ldx, vel, ldx) : h->tile;
  if (h->lds_rg) {
    // every step in one persistent launch, the state read and written once
    PersistArgs pa{h->var_ptr, h->occ4, h->occx, h->clause_ptr, h->clause_lits, h->f_vbeg,
                   h->lds_order, h->n_empty, x, ldx, h->R, h->F, steps, h->nf_max, h->lds_nocc, h->lds_stage,
                   h->opt.lr, loss_trace,
                   unsat_trace};
    ProfScope _ps(h, GALSAT_K_VAR_PASS, s);
    GS_HIP(h, launch_persistent(pa, h->lds_rg, s), "persistent step loop");
    return GALSAT_OK;
  }
  if (h->opt.use_graph && !adam && !h->prof) {
    galsat_status st = capture_steps(h, t, x, ldx, steps, loss_trace, unsat_trace);
    if (st != GALSAT_OK) return st;
    GS_HIP(h, hipGraphLaunch(h->graph_exec, s), "graph launch");
    return GALSAT_OK;
  }
  return enqueue_steps(h, t, x, ldx, mom, vel, steps, loss_trace, unsat_trace, s);
}

extern "C" galsat_status galsat_gumbel_noise(galsat_handle h, uint64_t seed, int32_t step,
                                             float* noise, int32_t ldn, void* stream) {
  GS_CHECK_HANDLE(h);
  if (!noise && h->n > 0) return h->fail(GALSAT_EINVAL, "noise is NULL");
  if (ldn < h->R) return h->fail(GALSAT_EINVAL, "ldn < restarts");
  GS_HIP(h, launch_gumbel_noise(noise, ldn, h->n, h->R, seed, step, static_cast<hipStream_t>(stream)),
         "gumbel noise");
  return GALSAT_OK;
}

extern "C" galsat_status galsat_gumbel_step(galsat_handle h, float* d, int32_t ldd, float* opt_state,
                                            uint64_t seed, int32_t step0, int32_t steps, float tau,
                                            const float* noise, float* loss_trace,
                                            int32_t* unsat_trace, void* stream) {
  GS_CHECK_HANDLE(h);
  if (!d && h->n > 0) return h->fail(GALSAT_EINVAL, "d is NULL");
  if (ldd < h->R) return h->fail(GALSAT_EINVAL, "ldd < restarts");
  if (steps < 0 || step0 < 0) return h->fail(GALSAT_EINVAL, "steps and step0 must be >= 0");
  if (!(tau > 0.0f) || !std::isfinite(tau)) return h->fail(GALSAT_EINVAL, "tau must be > 0");
  const bool adam = h->opt.optimizer == GALSAT_OPT_ADAM;
  if (adam && !opt_state && h->n > 0) return h->fail(GALSAT_EINVAL, "Adam needs opt_state");
  if (steps == 0) return GALSAT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the hard point, its gradient and the step's noise live in the internal
  // state buffers (xa, xb) and one more buffer of the same shape
  hipError_t he;
  if (!h->nbuf && (he = h->alloc(&h->nbuf, (size_t)h->n * h->ld)) != hipSuccess)
    return h->fail(he == hipErrorOutOfMemory ? GALSAT_ENOMEM : GALSAT_EDEVICE, "noise buffer");
  float* xh = h->xa;
  float* gb = h->xb;
  float* mom = adam ? opt_state : nullptr;
  float* vel = adam ? opt_state + (int64_t)h->n * ldd : nullptr;
  const int64_t FR = (int64_t)h->F * h->R;
  for (int32_t k = 0; k < steps; ++k) {
    const float* nk = noise ? noise + (int64_t)k * h->n * ldd : nullptr;
    {
      ProfScope _ps(h, GALSAT_K_COPY, s);
      GS_HIP(h, launch_gumbel_prep(d, ldd, nk, ldd, seed, step0 + k, h->n, h->R, xh, h->nbuf, h->ld, s),
             "gumbel prep");
    }
    galsat_status st = grad_passes(h, h->tile, kModeGrad, xh, h->ld, gb, h->ld, nullptr, nullptr, 0,
                                   nullptr, 0, h->F, s);
    if (st != GALSAT_OK) return st;
    st = finalize_step(h, loss_trace ? loss_trace + k * FR : nullptr,
                       unsat_trace ? unsat_trace + k * FR : nullptr, 0, h->F, s);
    if (st != GALSAT_OK) return st;
    double inv_c1 = 1.0, inv_c2 = 1.0;
    if (adam) {
      const int tt = h->adam_t + 1;
      inv_c1 = 1.0 / (1.0 - std::pow((double)h->opt.beta1, tt));
      inv_c2 = 1.0 / (1.0 - std::pow((double)h->opt.beta2, tt));
      h->adam_t++;
    }
    ProfScope _ps(h, GALSAT_K_VAR_PASS, s);
    GS_HIP(h, launch_gumbel_update(d, ldd, h->nbuf, gb, h->ld, mom, vel, ldd, h->n, h->R, tau,
                                   h->opt.lr, h->opt.beta1, h->opt.beta2, h->opt.eps, inv_c1, inv_c2,
                                   adam ? 1 : 0, s),
           "gumbel update");
  }
  return GALSAT_OK;
}

extern "C" galsat_status galsat_candidates(galsat_handle h, const float* d, int32_t ldd,
                                           const int32_t* best_restart, int32_t num, uint64_t seed,
                                           float tau, uint8_t* assign, float* conf, void* stream) {
  GS_CHECK_HANDLE(h);
  if (num < 0) return h->fail(GALSAT_EINVAL, "num must be >= 0");
  if (num > 0 && h->n > 0 && (!d || !best_restart || !assign || !conf))
    return h->fail(GALSAT_EINVAL, "d, best_restart, assign and conf are required");
  if (ldd < h->R) return h->fail(GALSAT_EINVAL, "ldd < restarts");
  if (!(tau > 0.0f) || !std::isfinite(tau)) return h->fail(GALSAT_EINVAL, "tau must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProfScope _ps(h, GALSAT_K_SELECT, s);
  GS_HIP(h, launch_candidates(d, ldd, h->var_formula, best_restart, h->n, num, seed, tau, assign, conf,
                              s),
         "candidates");
  return GALSAT_OK;
}

extern "C" galsat_status galsat_confidence(galsat_handle h, const float* d, int32_t ldd,
                                           const int32_t* best_restart, float tau, float* conf,
                                           void* stream) {
  GS_CHECK_HANDLE(h);
  if (h->n > 0 && (!d || !best_restart || !conf))
    return h->fail(GALSAT_EINVAL, "d, best_restart and conf are required");
  if (ldd < h->R) return h->fail(GALSAT_EINVAL, "ldd < restarts");
  if (!(tau > 0.0f) || !std::isfinite(tau)) return h->fail(GALSAT_EINVAL, "tau must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProfScope _ps(h, GALSAT_K_SELECT, s);
  GS_HIP(h, launch_confidence(d, ldd, h->var_formula, best_restart, h->n, tau, conf, s), "confidence");
  return GALSAT_OK;
}

extern "C" galsat_status galsat_select_vars(galsat_handle h, const float* conf, int32_t num,
                                            int32_t highest, float frac, int32_t min_count,
                                            int32_t* offsets, int32_t* out, void* stream) {
  GS_CHECK_HANDLE(h);
  if (!offsets) return h->fail(GALSAT_EINVAL, "offsets is NULL");
  if (num < 0 || min_count < 0 || !(frac >= 0.0f && frac <= 1.0f))
    return h->fail(GALSAT_EINVAL, "num, min_count >= 0 and frac in [0, 1] required");
  std::vector<int32_t> off((size_t)h->F + 1, 0);
  for (int32_t f = 0; f < h->F; ++f) {
    const int32_t nf = h->h_fvb[f + 1] - h->h_fvb[f];
    int64_t c = (int64_t)std::ceil((double)frac * (double)nf);
    c = std::max<int64_t>(c, min_count);
    c = std::min<int64_t>(c, nf);
    off[f + 1] = off[f] + (int32_t)c;
  }
  std::memcpy(offsets, off.data(), off.size() * sizeof(int32_t));
  if (!out) return GALSAT_OK;  // size query
  if (!conf && num > 0) return h->fail(GALSAT_EINVAL, "conf is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!h->sel_off) {
    hipError_t he = h->alloc(&h->sel_off, (size_t)h->F + 1);
    if (he != hipSuccess) return h->dev_fail(he, "allocate selection offsets");
  }
  // the offsets table is tiny; upload it on the call's stream before the launch
  GS_HIP(h, hipMemcpyAsync(h->sel_off, off.data(), off.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s),
         "upload selection offsets");
  GS_HIP(h, hipStreamSynchronize(s), "selection offsets");
  ProfScope _ps(h, GALSAT_K_SELECT, s);
  GS_HIP(h, launch_select(conf, h->n, h->F, h->f_vbeg, h->sel_off, off[h->F], num, highest != 0, out,
                          s),
         "select");
  return GALSAT_OK;
}

extern "C" galsat_status galsat_round_check(galsat_handle h, const float* x, int32_t ldx,
                                            int32_t* unsat, int32_t* best_restart,
                                            uint8_t* best_assign, void* stream) {
  GS_CHECK_HANDLE(h);
  if ((!x && h->n > 0) || !unsat) return h->fail(GALSAT_EINVAL, "x and unsat are required");
  if (ldx < h->R) return h->fail(GALSAT_EINVAL, "ldx < restarts");
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    ProfScope _ps(h, GALSAT_K_PACK, s);
    GS_HIP(h, launch_pack_bits(x, ldx, h->n, h->R, h->bits, s), "pack bits");
  }
  {
    ProfScope _ps(h, GALSAT_K_COUNT, s);
    GS_HIP(h, launch_count_unsat(h->clause_ptr, h->clause_lits, h->ach_beg, h->ach_end,
                                 h->n_aorder > 0 ? h->ach_order : nullptr,
                                 h->n_aorder > 0 ? h->n_aorder : h->ach.count(), h->bits, h->n,
                                 h->R, h->unsat_part, s),
           "count unsat");
  }
  FinalizeArgs fa{h->fin_all_a0, h->fin_all_a1, h->zero_empty, h->loss_part, h->unsat_part,
                  nullptr, unsat, h->R, 0, h->fin_l, h->fin_u, 1, h->max_all_rows};
  {
    ProfScope _ps(h, GALSAT_K_FINALIZE, s);
    GS_HIP(h, launch_finalize(fa, h->F, s), "finalize");
  }
  if (best_restart || best_assign) {
    int32_t* best = best_restart ? best_restart : h->best_tmp;
    {
      ProfScope _ps(h, GALSAT_K_SELECT, s);
      GS_HIP(h, launch_best(unsat, h->F, h->R, best, s), "best");
    }
    if (best_assign)
      {
        ProfScope _ps(h, GALSAT_K_SELECT, s);
        GS_HIP(h, launch_best_assign(h->bits, h->n, h->var_formula, best, best_assign, s), "best assign");
      }
  }
  return GALSAT_OK;
}

// ------------------------------------------------ allocation-free round check
//
// The same kernels as galsat_round_check, with their scratch (bit-planes,
// per-chunk unsat rows, split-finalize part sums, the best restart when the
// caller does not ask for it) carved from one file-scope device array
// instead of the handle's workspace.  The array's device address differs per
// GPU and is looked up once per device with hipGetSymbolAddress; host code
// uses only that looked-up address.
namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per device
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" galsat_status galsat_round_check_static(galsat_handle h, const float* x, int32_t ldx,
                                                   int32_t* unsat, int32_t* best_restart,
                                                   uint8_t* best_assign, void* stream) {
  GS_CHECK_HANDLE(h);
  if ((!x && h->n > 0) || !unsat) return h->fail(GALSAT_EINVAL, "x and unsat are required");
  if (ldx < h->R) return h->fail(GALSAT_EINVAL, "ldx < restarts");
  int dev = -1;
  GS_HIP(h, hipGetDevice(&dev), "get device");
  if (dev != h->device) return h->fail(GALSAT_EINVAL, "call on the device the handle was created on");
  if (dev < 0 || dev >= kMaxDevices) return h->fail(GALSAT_EUNSUPPORTED, "device index above 63");
  // the scratch layout for this handle; refused when it exceeds the array
  const int64_t words = (h->R + 63) / 64;
  const size_t b_bits = align256((size_t)h->n * (size_t)words * sizeof(uint64_t));
  const size_t b_rows = align256((size_t)std::max(h->ach.count(), 1) * (size_t)h->R * sizeof(int32_t));
  const size_t b_pl = align256((size_t)kFinalizeScratch * sizeof(double));
  const size_t b_pu = align256((size_t)kFinalizeScratch * sizeof(int32_t));
  const size_t b_best = align256((size_t)h->F * sizeof(int32_t));
  const size_t need = b_bits + b_rows + b_pl + b_pu + b_best;
  if (need > kStaticScratchBytes)
    return h->fail(GALSAT_EOVERFLOW,
                   "galsat_round_check_static needs " + std::to_string(need) +
                       " bytes of scratch, above its fixed " +
                       std::to_string(kStaticScratchBytes) + " (use galsat_round_check)");
  // once per device, with that device current: the array's address on it
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  GS_HIP(h, g_scratch_err[dev], "scratch symbol address");
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  if (!base) return h->fail(GALSAT_EDEVICE, "scratch symbol address is null");
  uint64_t* bits = reinterpret_cast<uint64_t*>(base);
  int32_t* rows = reinterpret_cast<int32_t*>(base + b_bits);
  double* part_l = reinterpret_cast<double*>(base + b_bits + b_rows);
  int32_t* part_u = reinterpret_cast<int32_t*>(base + b_bits + b_rows + b_pl);
  int32_t* best_tmp = reinterpret_cast<int32_t*>(base + b_bits + b_rows + b_pl + b_pu);
  // every kernel below overwrites the scratch entries it later reads, so
  // nothing needs clearing between calls; no per-kernel profiling events
  // either (creating one may allocate)
  hipStream_t s = static_cast<hipStream_t>(stream);
  GS_HIP(h, launch_pack_bits(x, ldx, h->n, h->R, bits, s), "pack bits");
  GS_HIP(h, launch_count_unsat(h->clause_ptr, h->clause_lits, h->ach_beg, h->ach_end,
                               h->n_aorder > 0 ? h->ach_order : nullptr,
                               h->n_aorder > 0 ? h->n_aorder : h->ach.count(), bits, h->n, h->R,
                               rows, s),
         "count unsat");
  FinalizeArgs fa{h->fin_all_a0, h->fin_all_a1, h->zero_empty, nullptr, rows,
                  nullptr, unsat, h->R, 0, part_l, part_u, 1, h->max_all_rows};
  GS_HIP(h, launch_finalize(fa, h->F, s), "finalize");
  if (best_restart || best_assign) {
    int32_t* best = best_restart ? best_restart : best_tmp;
    GS_HIP(h, launch_best(unsat, h->F, h->R, best, s), "best");
    if (best_assign)
      GS_HIP(h, launch_best_assign(bits, h->n, h->var_formula, best, best_assign, s), "best assign");
  }
  return GALSAT_OK;
}

extern "C" galsat_status galsat_profile(galsat_handle h, int32_t enable) {
  GS_CHECK_HANDLE(h);
  if (enable) {
    for (auto& r : h->recs) {
      (void)hipEventSynchronize(r.b);
    }
    h->release_records();
  }
  h->prof = enable != 0;
  return GALSAT_OK;
}

extern "C" galsat_status galsat_kernel_times(galsat_handle h, galsat_kernel_stats* out) {
  GS_CHECK_HANDLE(h);
  if (!out) return h->fail(GALSAT_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  for (auto& r : h->recs) {
    GS_HIP(h, hipEventSynchronize(r.b), "event synchronize");
    float ms = 0.0f;
    GS_HIP(h, hipEventElapsedTime(&ms, r.a, r.b), "event elapsed");
    if (r.kind >= 0 && r.kind < GALSAT_K_KINDS) {
      out->launches[r.kind] += 1;
      out->total_ms[r.kind] += ms;
    }
  }
  return GALSAT_OK;
}
