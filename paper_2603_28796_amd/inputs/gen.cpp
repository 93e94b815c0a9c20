// Seeded synthetic CNF generators and the clause-major -> variable-major
// transpose.  This module builds INPUTS only: it holds none of the method's
// arithmetic (no clause polynomial, no gradient, no update) and is shared by
// the test oracle and the HIP path as their common source of workloads.
//
// Every random draw comes from a counter-based stream keyed by
// (seed, tag, formula, clause), so the output does not depend on the number
// of threads that produce it.
//
// Workload families (standing in for the SAT Competition instances, which
// are not available): planted random k-SAT, mixed clause lengths, Zipf
// variable popularity over a seeded permutation of ids, and community
// structure with intra-community literals.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

// SplitMix64 output mix (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014), used as a 64-bit bijective hash.
inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ULL;
constexpr uint64_t TAG_LEN = 0x4c454e00ULL;
constexpr uint64_t TAG_LIT = 0x4c495400ULL;
constexpr uint64_t TAG_PLANT = 0x504c4e54ULL;
constexpr uint64_t TAG_PERM = 0x5045524dULL;
constexpr uint64_t TAG_CPERM = 0x4350524dULL;
constexpr uint64_t TAG_SIZE = 0x53495a45ULL;

struct Stream {
  uint64_t s;
  Stream(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
    s = mix64(seed ^ mix64(tag * kGolden ^ mix64((a << 40) ^ (a >> 24) ^ mix64(b + kGolden))));
  }
  uint64_t next() {
    s += kGolden;
    return mix64(s);
  }
  double unif() { return (double)(next() >> 11) * 0x1.0p-53; }
  // integer in [0, n) by 64x64->128 multiply (bias < n / 2^64)
  uint64_t below(uint64_t n) { return (uint64_t)(((__uint128_t)next() * n) >> 64); }
};

}  // namespace

extern "C" {

typedef struct {
  int32_t len_kind;  // 0: fixed k0; 1: 2 + Geometric(geom_p), redrawn while > kmax;
                     // 2: k0 with probability p0, else uniform in [ka, kb]
  int32_t k0, ka, kb, kmax;
  double p0, geom_p;
  int32_t var_kind;  // 0: uniform; 1: Zipf(zipf_s) over a seeded permutation of the
                     // formula's ids; 2: n_comm contiguous communities, Zipf within
  int32_t n_comm;
  double zipf_s;
  double p_intra;
  int32_t plant;     // 1: flip one literal of every clause the hidden assignment falsifies
  int32_t distinct;  // 1: the variables of a clause are pairwise distinct
} galsat_gen_spec;

// Per-formula sizes for an uneven batch: n_f uniform in [nmin, nmax],
// ratio uniform in [rmin, rmax), m_f = round(n_f * ratio).
void gen_batch_sizes(uint64_t seed, int32_t F, int32_t nmin, int32_t nmax, double rmin,
                     double rmax, int64_t* n_out, int64_t* m_out) {
  for (int32_t f = 0; f < F; ++f) {
    Stream st(seed, TAG_SIZE, (uint64_t)f, 0);
    int64_t n = nmin + (int64_t)st.below((uint64_t)(nmax - nmin + 1));
    double ratio = rmin + (rmax - rmin) * st.unif();
    n_out[f] = n;
    m_out[f] = (int64_t)std::llround((double)n * ratio);
  }
}

static int draw_len(const galsat_gen_spec* sp, Stream& st) {
  switch (sp->len_kind) {
    case 0:
      return sp->k0;
    case 1: {
      const double lq = std::log1p(-sp->geom_p);
      for (;;) {
        double u = st.unif();
        // failures before the first success: floor(log(1-u) / log(1-p))
        int g = (int)std::floor(std::log1p(-u) / lq);
        int k = 2 + g;
        if (k <= sp->kmax) return k;
      }
    }
    case 2: {
      if (st.unif() < sp->p0) return sp->k0;
      return sp->ka + (int)st.below((uint64_t)(sp->kb - sp->ka + 1));
    }
  }
  return sp->k0;
}

// Clause lengths for all formulas.  clause_begin[F+1] gives each formula's
// clause range in the global clause order.
int gen_lengths(const galsat_gen_spec* sp, uint64_t seed, int32_t F, const int64_t* clause_begin,
                int32_t* len_out) {
  for (int32_t f = 0; f < F; ++f) {
    const int64_t c0 = clause_begin[f], c1 = clause_begin[f + 1];
#pragma omp parallel for schedule(static)
    for (int64_t t = c0; t < c1; ++t) {
      Stream st(seed, TAG_LEN, (uint64_t)f, (uint64_t)(t - c0));
      len_out[t] = draw_len(sp, st);
    }
  }
  return 0;
}

static inline bool plant_bit(uint64_t seed, int64_t v) {
  Stream st(seed, TAG_PLANT, 0, (uint64_t)v);
  return (st.next() >> 63) & 1;
}

static void zipf_cdf(int64_t N, double s, std::vector<double>& cdf) {
  cdf.resize((size_t)N);
  double acc = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    acc += std::pow((double)(i + 1), -s);
    cdf[(size_t)i] = acc;
  }
}

static inline int64_t zipf_draw(const std::vector<double>& cdf, Stream& st) {
  double u = st.unif() * cdf.back();
  auto it = std::upper_bound(cdf.begin(), cdf.end(), u);
  int64_t r = (int64_t)(it - cdf.begin());
  if (r >= (int64_t)cdf.size()) r = (int64_t)cdf.size() - 1;
  return r;
}

static void seeded_perm(uint64_t seed, uint64_t tag, uint64_t key, int32_t* p, int64_t N) {
  for (int64_t i = 0; i < N; ++i) p[i] = (int32_t)i;
  Stream st(seed, tag, key, 0);
  for (int64_t i = N - 1; i > 0; --i) {
    int64_t j = (int64_t)st.below((uint64_t)(i + 1));
    std::swap(p[i], p[j]);
  }
}

// Literal codes (2*var + neg, global variable ids) for all formulas, plus the
// hidden assignment planted[v] in {0,1}.  clause_ptr[m+1] holds the global
// clause offsets built from gen_lengths.  Returns 0, or -1 when a clause
// cannot hold distinct variables (k > n_f) or the community split is uneven.
int gen_literals(const galsat_gen_spec* sp, uint64_t seed, int32_t F, const int64_t* var_begin,
                 const int64_t* clause_begin, const int32_t* clause_ptr, int32_t* lits_out,
                 uint8_t* planted_out) {
  const int64_t n_total = var_begin[F];
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n_total; ++v) planted_out[v] = plant_bit(seed, v) ? 1 : 0;

  std::vector<double> cdf;
  std::vector<int32_t> perm;
  int bad = 0;
  for (int32_t f = 0; f < F && !bad; ++f) {
    const int64_t v0 = var_begin[f], nf = var_begin[f + 1] - var_begin[f];
    const int64_t c0 = clause_begin[f], c1 = clause_begin[f + 1];
    if (c1 == c0) continue;
    int64_t csize = 0;
    if (sp->var_kind == 1) {
      zipf_cdf(nf, sp->zipf_s, cdf);
      perm.resize((size_t)nf);
      seeded_perm(seed, TAG_PERM, (uint64_t)f, perm.data(), nf);
    } else if (sp->var_kind == 2) {
      if (sp->n_comm <= 1 || nf % sp->n_comm != 0) return -1;
      csize = nf / sp->n_comm;
      zipf_cdf(csize, sp->zipf_s, cdf);
      perm.resize((size_t)nf);
#pragma omp parallel for schedule(static)
      for (int32_t c = 0; c < sp->n_comm; ++c)
        seeded_perm(seed, TAG_CPERM, ((uint64_t)f << 20) ^ (uint64_t)c, perm.data() + (int64_t)c * csize,
                    csize);
    }
#pragma omp parallel for schedule(dynamic, 4096) reduction(| : bad)
    for (int64_t t = c0; t < c1; ++t) {
      Stream st(seed, TAG_LIT, (uint64_t)f, (uint64_t)(t - c0));
      const int32_t p0 = clause_ptr[t], k = clause_ptr[t + 1] - clause_ptr[t];
      if (sp->distinct && k > nf) {
        bad = 1;
        continue;
      }
      int64_t home = 0;
      if (sp->var_kind == 2) home = (int64_t)st.below((uint64_t)sp->n_comm);
      for (int32_t j = 0; j < k; ++j) {
        int64_t v;
        for (;;) {
          if (sp->var_kind == 0) {
            v = (int64_t)st.below((uint64_t)nf);
          } else if (sp->var_kind == 1) {
            v = perm[(size_t)zipf_draw(cdf, st)];
          } else {
            int64_t c = home;
            if (st.unif() >= sp->p_intra) {
              c = (int64_t)st.below((uint64_t)(sp->n_comm - 1));
              if (c >= home) ++c;
            }
            v = perm[(size_t)(c * csize + zipf_draw(cdf, st))];
          }
          if (!sp->distinct) break;
          bool dup = false;
          for (int32_t i = 0; i < j; ++i)
            if ((lits_out[p0 + i] >> 1) == (int32_t)(v0 + v)) {
              dup = true;
              break;
            }
          if (!dup) break;
        }
        const int32_t neg = (int32_t)(st.next() >> 63);
        lits_out[p0 + j] = (int32_t)(2 * (v0 + v) + neg);
      }
      if (sp->plant && k > 0) {
        bool sat = false;
        for (int32_t j = 0; j < k && !sat; ++j) {
          const int32_t code = lits_out[p0 + j];
          const int hv = planted_out[code >> 1];
          sat = (code & 1) ? (hv == 0) : (hv == 1);
        }
        if (!sat) {
          const int32_t j = (int32_t)st.below((uint64_t)k);
          lits_out[p0 + j] ^= 1;
        }
      }
    }
  }
  return bad ? -1 : 0;
}

// Variable-major transpose: var_occ lists, for each variable in increasing
// id order, the clause-major positions p with lits[p] >> 1 == v, in
// increasing p.  var_begin/clause_begin (F formulas) let formulas be
// transposed independently; with F == 1 the variable range is split across
// threads instead.  var_ptr has n+1 entries.
int gen_transpose(int32_t F, const int64_t* var_begin, const int64_t* clause_begin,
                  const int32_t* clause_ptr, const int32_t* lits, int32_t* var_ptr,
                  int32_t* var_occ) {
  const int64_t n = var_begin[F];
  const int64_t L = clause_ptr[clause_begin[F]];
  std::vector<int32_t> cnt((size_t)n + 1, 0);
  // per-formula threads are race-free only while every literal names a
  // variable of its own formula; otherwise threads own variable ranges
  int bad = 0;
  if (F > 1) {
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int32_t f = 0; f < F; ++f) {
      const int64_t p0 = clause_ptr[clause_begin[f]], p1 = clause_ptr[clause_begin[f + 1]];
      for (int64_t p = p0; p < p1; ++p) {
        const int64_t v = lits[p] >> 1;
        if (lits[p] < 0 || v < var_begin[f] || v >= var_begin[f + 1]) bad = 1;
      }
    }
  }
  const bool by_formula = F > 1 && !bad;
  if (by_formula) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
      const int64_t p0 = clause_ptr[clause_begin[f]], p1 = clause_ptr[clause_begin[f + 1]];
      for (int64_t p = p0; p < p1; ++p) cnt[(size_t)(lits[p] >> 1)]++;
    }
  } else {
    const int nt = omp_get_max_threads();
#pragma omp parallel num_threads(nt)
    {
      const int64_t tid = omp_get_thread_num(), nth = omp_get_num_threads();
      const int64_t va = n * tid / nth, vb = n * (tid + 1) / nth;
      for (int64_t p = 0; p < L; ++p) {
        const int64_t v = lits[p] >> 1;
        if (v >= va && v < vb) cnt[(size_t)v]++;
      }
    }
  }
  int64_t acc = 0;
  for (int64_t v = 0; v < n; ++v) {
    var_ptr[v] = (int32_t)acc;
    acc += cnt[(size_t)v];
  }
  var_ptr[n] = (int32_t)acc;
  if (acc != L) return -1;
  std::vector<int32_t> fill(var_ptr, var_ptr + n);
  if (by_formula) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
      const int64_t p0 = clause_ptr[clause_begin[f]], p1 = clause_ptr[clause_begin[f + 1]];
      for (int64_t p = p0; p < p1; ++p) var_occ[fill[(size_t)(lits[p] >> 1)]++] = (int32_t)p;
    }
  } else {
    const int nt = omp_get_max_threads();
#pragma omp parallel num_threads(nt)
    {
      const int64_t tid = omp_get_thread_num(), nth = omp_get_num_threads();
      const int64_t va = n * tid / nth, vb = n * (tid + 1) / nth;
      for (int64_t p = 0; p < L; ++p) {
        const int64_t v = lits[p] >> 1;
        if (v >= va && v < vb) var_occ[fill[(size_t)v]++] = (int32_t)p;
      }
    }
  }
  return 0;
}

}  // extern "C"
