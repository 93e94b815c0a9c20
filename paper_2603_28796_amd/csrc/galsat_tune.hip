// Plan autotuner: candidate plans derived from the restart count and the
// clause-length histogram, each timed on the real step, the fastest kept
// (and optionally remembered in a plan cache file keyed by the problem's
// shape, which galsat_create consults).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "galsat_internal.h"

namespace {

int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Clause lengths of the problem (host or device inputs).
bool clause_lengths(const galsat_problem* prob, std::vector<int32_t>* len) {
  const int32_t m = prob->n_clauses;
  std::vector<int32_t> cp((size_t)m + 1);
  if (prob->inputs_on_device) {
    if (hipMemcpy(cp.data(), prob->clause_ptr, cp.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return false;
  } else {
    std::memcpy(cp.data(), prob->clause_ptr, cp.size() * sizeof(int32_t));
  }
  len->resize((size_t)m);
  for (int32_t t = 0; t < m; ++t) (*len)[t] = cp[t + 1] - cp[t];
  return true;
}

}  // namespace

namespace galsat {

// Key of a problem's shape for the plan cache: sizes, restarts and a hash
// of the clause-length histogram.
std::string plan_key(const galsat_problem* prob) {
  std::vector<int32_t> len;
  uint64_t hsh = 1469598103934665603ULL;
  if (clause_lengths(prob, &len)) {
    std::vector<int64_t> hist;
    for (int32_t k : len) {
      if ((size_t)k >= hist.size()) hist.resize((size_t)k + 1, 0);
      hist[k]++;
    }
    for (size_t k = 0; k < hist.size(); ++k) {
      hsh = (hsh ^ (uint64_t)k) * 1099511628211ULL;
      hsh = (hsh ^ (uint64_t)hist[k]) * 1099511628211ULL;
    }
  }
  char buf[160];
  std::snprintf(buf, sizeof(buf), "F=%d n=%d m=%d L=%d R=%d h=%016llx", prob->num_formulas,
                prob->n_vars, prob->n_clauses, prob->n_lits, prob->restarts,
                (unsigned long long)hsh);
  return buf;
}

// Looks the key up in the file named by GALSAT_PLAN_CACHE ("<key> | <plan>"
// lines, last one wins).
bool plan_cache_lookup(const std::string& key, std::string* plan) {
  const char* path = std::getenv("GALSAT_PLAN_CACHE");
  if (!path) return false;
  FILE* fh = std::fopen(path, "r");
  if (!fh) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), fh)) {
    std::string s(line);
    const size_t bar = s.find(" | ");
    if (bar == std::string::npos || s.compare(0, bar, key) != 0 || bar != key.size()) continue;
    std::string p = s.substr(bar + 3);
    while (!p.empty() && (p.back() == '\n' || p.back() == '\r')) p.pop_back();
    *plan = p;
    found = true;
  }
  std::fclose(fh);
  return found;
}

}  // namespace galsat

namespace galsat {

// Times each candidate plan on `steps` real steps from x0 (after one warm-up
// step) and keeps the fastest; candidates that do not fit the workspace are
// skipped.
galsat_status tune_plans(const galsat_problem* prob, const galsat_options& base, const float* x0,
                         int32_t ldx, int32_t steps, void* stream,
                         const std::vector<std::string>& plans, char* plan_out, int32_t plan_cap,
                         double* best_ms) {
  const int n = prob->n_vars;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* xs = nullptr;
  if (hipMalloc(&xs, (size_t)std::max(n, 1) * ldx * sizeof(float)) != hipSuccess) return GALSAT_ENOMEM;
  // Adam candidates step their own moments [2][n][ldx], zeroed before each
  const bool adam = base.optimizer == GALSAT_OPT_ADAM;
  const size_t mom_bytes = 2 * (size_t)std::max(n, 1) * ldx * sizeof(float);
  float* mom = nullptr;
  if (adam && hipMalloc(&mom, mom_bytes) != hipSuccess) {
    (void)hipFree(xs);
    return GALSAT_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e300;
  std::string best_plan;
  galsat_status result = GALSAT_OK;
  for (const auto& plan : plans) {
    galsat_options o = base;
    o.plan_override = plan.c_str();
    galsat_handle h = nullptr;
    galsat_status st = galsat_create(prob, &o, stream, &h);
    if (st != GALSAT_OK) {
      if (st == GALSAT_ENOMEM) continue;  // a storing plan may not fit: skip it
      result = st;
      break;
    }
    (void)hipMemcpyAsync(xs, x0, (size_t)n * ldx * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (adam) (void)hipMemsetAsync(mom, 0, mom_bytes, s);
    st = galsat_step(h, xs, ldx, mom, 1, nullptr, nullptr, stream);  // warm-up
    (void)hipEventRecord(e0, s);
    if (st == GALSAT_OK) st = galsat_step(h, xs, ldx, mom, steps, nullptr, nullptr, stream);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    galsat_destroy(h);
    if (st != GALSAT_OK) {
      result = st;
      break;
    }
    if (ms < best) {
      best = ms;
      best_plan = plan;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(xs);
  if (mom) (void)hipFree(mom);
  if (result != GALSAT_OK && best_plan.empty()) return result;
  if ((int32_t)best_plan.size() + 1 > plan_cap) return GALSAT_EINVAL;
  std::memcpy(plan_out, best_plan.c_str(), best_plan.size() + 1);
  if (best_ms) *best_ms = best / steps;
  if (const char* path = std::getenv("GALSAT_PLAN_CACHE")) {
    if (FILE* fh = std::fopen(path, "a")) {
      std::fprintf(fh, "%s | %s\n", galsat::plan_key(prob).c_str(), best_plan.c_str());
      std::fclose(fh);
    }
  }
  return GALSAT_OK;
}

}  // namespace galsat

extern "C" galsat_status galsat_autotune(const galsat_problem* prob, const galsat_options* opt_in,
                                         const float* x0, int32_t ldx, int32_t steps, void* stream,
                                         char* plan_out, int32_t plan_cap, double* best_ms) {
  if (!prob || !x0 || ldx < prob->restarts || steps < 1 || !plan_out || plan_cap < 64)
    return GALSAT_EINVAL;
  galsat_options base;
  if (opt_in) base = *opt_in; else galsat_default_options(&base);
  base.use_graph = 0;
  const int R = prob->restarts;
  std::vector<int32_t> len;
  if (!clause_lengths(prob, &len)) return GALSAT_EDEVICE;
  int kmax = 0;
  int64_t long_lits = 0;
  for (int32_t k : len) {
    kmax = std::max(kmax, k);
    if (k > 8) long_lits += k;
  }
  // Narrow restart batches with AUTO partials run the flat plan: the
  // candidates are both record-prefetch choices (one of them the plan's own
  // choice), other chunk counts per formula for batches, and the two-phase
  // plan.
  if (R <= 64 && base.partials == GALSAT_PARTIALS_AUTO && base.schedule != GALSAT_SCHED_LDS &&
      base.recompute_max_len == 0) {
    std::vector<std::string> plans = {"flat=1,pf=0", "flat=1,pf=1"};
    if (prob->num_formulas > 1 && base.schedule != GALSAT_SCHED_PLAIN) {
      plans.push_back("flat=1,xcdc=20");
      plans.push_back("flat=1,xcdc=80");
    }
    plans.push_back("two=1");
    return galsat::tune_plans(prob, base, x0, ldx, steps, stream, plans, plan_out, plan_cap, best_ms);
  }
  // tiles: wide restart batches favour 4 restarts per lane, small ones one
  std::vector<std::string> tiles;
  if (R > 32) {
    tiles = {"lpi=64,rpl=4"};
    if (R % 2 == 0) tiles.push_back("lpi=64,rpl=2");
    if (R >= 128) tiles.push_back("lpi=32,rpl=4");
  } else {
    const int p = std::max(4, std::min(64, pow2_at_least(R)));
    tiles = {"lpi=" + std::to_string(p) + ",rpl=1"};
    if (p != 64) tiles.push_back("lpi=64,rpl=1");
    if (R % 4 == 0 && p / 4 >= 4) tiles.push_back("lpi=" + std::to_string(p / 4) + ",rpl=4");
  }
  // recompute threshold from the clause-length histogram: with long clauses
  // present, storing their partials competes with recomputing them
  std::vector<std::string> krecs = {""};
  if (base.partials == GALSAT_PARTIALS_AUTO && kmax > 8 && long_lits > 0)
    krecs = {",krec=8", ",krec=" + std::to_string(kmax)};
  std::vector<std::string> xcd = {""};
  if (prob->num_formulas > 1 && base.schedule != GALSAT_SCHED_PLAIN) xcd = {"", ",xcdc=160", ",xcdc=20"};
  // narrow restart batches: the single pass against the two-phase gradient
  std::vector<std::string> twos = {""};
  if (R <= 64) twos = {",two=0", ",two=1"};

  std::vector<std::string> plans;
  for (const auto& t : tiles)
    for (const auto& k : krecs)
      for (const auto& x : xcd)
        for (const auto& w : twos) plans.push_back(t + k + x + w);
  if (base.schedule == GALSAT_SCHED_LDS) {
    // the persistent schedule has its own choices: restarts per workgroup
    // (up to the restarts rounded to a power of two) and record staging
    plans.clear();
    for (int g = 1; g <= 32 && g < 2 * R; g *= 2)
      for (const char* st : {"", ",ldsstage=0"}) plans.push_back("ldsrg=" + std::to_string(g) + st);
  }
  return galsat::tune_plans(prob, base, x0, ldx, steps, stream, plans, plan_out, plan_cap, best_ms);
}
