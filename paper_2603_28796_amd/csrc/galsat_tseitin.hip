// Host-side clause normalization to a fixed width: the chain encoding of
// Section 3.2 ("Clause Normalization for Vectorization", Eq. 6-7).
//
// A clause (l1 v l2 v ... v lu) longer than the width w becomes a chain of
// clauses linked by fresh auxiliary variables f1, f2, ...:
//   (l1 v ... v l_{w-1} v f1) ^ (~f1 v l_w v ... v f2) ^ ... ^ (~f_last v ... v lu)
// where every middle link carries w-2 original literals.  For w = 3 this is
// exactly Eq. (6): u-3 auxiliaries and u-2 clauses, equisatisfiable with the
// original clause (Eq. 7).  A clause shorter than w is padded by repeating
// its last literal, as in the appendix example (~x1 v x3) -> (~x1 v x3 v x3).
// Empty clauses stay empty (an unsatisfiable formula stays unsatisfiable).
// Auxiliary variables are numbered from n_vars upward in the order they are
// created, so the original variables keep their ids.
#include <cstdint>
#include <vector>

#include "galsat_internal.h"

namespace {

// Emits the normalized clauses of one clause into (ptr, lits); returns the
// number of auxiliary variables used.
int64_t normalize_clause(int32_t width, const int32_t* c, int32_t u, int64_t next_aux,
                         std::vector<int64_t>* ends, std::vector<int64_t>* lits, int64_t* n_out_clauses,
                         int64_t* n_out_lits) {
  auto emit = [&](const std::vector<int64_t>& cl) {
    if (lits) lits->insert(lits->end(), cl.begin(), cl.end());
    *n_out_lits += (int64_t)cl.size();
    *n_out_clauses += 1;
    if (ends) ends->push_back(*n_out_lits);
  };
  if (u == 0) {
    emit({});
    return 0;
  }
  if (u <= width) {
    std::vector<int64_t> cl(c, c + u);
    while ((int32_t)cl.size() < width) cl.push_back(c[u - 1]);
    emit(cl);
    return 0;
  }
  int64_t used = 0;
  int32_t i = 0;
  int64_t prev = -1;  // auxiliary variable linking to the previous link
  while (true) {
    std::vector<int64_t> cl;
    if (prev >= 0) cl.push_back(2 * prev + 1);  // ~f_prev
    const int32_t room = width - (int32_t)cl.size();
    const int32_t rest = u - i;
    if (rest <= room) {  // last link: the remaining literals (padded like a short clause)
      for (; i < u; ++i) cl.push_back(c[i]);
      while ((int32_t)cl.size() < width) cl.push_back(c[u - 1]);
      emit(cl);
      break;
    }
    for (int32_t t = 0; t < room - 1; ++t) cl.push_back(c[i++]);
    const int64_t f = next_aux + used++;
    cl.push_back(2 * f);  // f
    emit(cl);
    prev = f;
  }
  return used;
}

}  // namespace

extern "C" galsat_status galsat_tseitin(int32_t width, int32_t n_vars, int32_t n_clauses,
                                        const int32_t* clause_ptr, const int32_t* clause_lits,
                                        int32_t* out_n_vars, int32_t* out_n_clauses,
                                        int32_t* out_n_lits, int32_t* out_clause_ptr,
                                        int32_t* out_clause_lits) {
  if (width < 3 || n_vars < 0 || n_clauses < 0 || !clause_ptr || !out_n_vars || !out_n_clauses ||
      !out_n_lits)
    return GALSAT_EINVAL;
  if (clause_ptr[0] != 0) return GALSAT_EINVAL;
  for (int32_t t = 0; t < n_clauses; ++t)
    if (clause_ptr[t + 1] < clause_ptr[t]) return GALSAT_EINVAL;
  const int64_t L = clause_ptr[n_clauses];
  if (L > 0 && !clause_lits) return GALSAT_EINVAL;
  for (int64_t p = 0; p < L; ++p)
    if (clause_lits[p] < 0 || (clause_lits[p] >> 1) >= n_vars) return GALSAT_EINVAL;
  const bool fill = out_clause_ptr && out_clause_lits;
  std::vector<int64_t> ends, lits;
  int64_t aux = 0, m_out = 0, L_out = 0;
  for (int32_t t = 0; t < n_clauses; ++t)
    aux += normalize_clause(width, clause_lits + clause_ptr[t], clause_ptr[t + 1] - clause_ptr[t],
                            (int64_t)n_vars + aux, fill ? &ends : nullptr, fill ? &lits : nullptr,
                            &m_out, &L_out);
  if ((int64_t)n_vars + aux >= (1LL << 30) || m_out >= (1LL << 31) - 1 || L_out >= (1LL << 31) - 1)
    return GALSAT_EOVERFLOW;
  *out_n_vars = (int32_t)(n_vars + aux);
  *out_n_clauses = (int32_t)m_out;
  *out_n_lits = (int32_t)L_out;
  if (fill) {
    out_clause_ptr[0] = 0;
    for (int64_t i = 0; i < m_out; ++i) out_clause_ptr[i + 1] = (int32_t)ends[(size_t)i];
    for (int64_t i = 0; i < L_out; ++i) out_clause_lits[i] = (int32_t)lits[(size_t)i];
  }
  return GALSAT_OK;
}
