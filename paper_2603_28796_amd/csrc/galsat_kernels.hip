// HIP kernels of the general schedule for gfx950 (MI355X, wave64).
//
// Mapping: an item (a variable or a clause) is processed by LPI lanes, each
// lane owning RPL consecutive restarts, so the restarts of one variable row
// x[v][r0 .. r0+LPI*RPL) are read and written with contiguous, coalesced
// accesses while every index of the item is shared by its lanes (with
// LPI = 64 the whole wave works on one item and the index loads become
// scalar loads).  All sums run in a fixed order: per-thread in FP64, then
// across the items of a workgroup in slot order, then across workgroups in
// chunk order, so every result is bitwise reproducible without atomics.
//
// Paper passages: clause value U_t = prod_i (1 - s_i) (Section 3.2, Eq. 2)
// with the negation rule of Eq. (1); loss' = sum_t U_t (Eq. 5 shifted by
// the clause count); the gradient is the derivative of that sum
// (backpropagation through Eq. 2); rounding x_hat = [x > 0.5] is the argmax
// of Eq. (4) with ties to 0.
#include "galsat_internal.h"

namespace galsat {

// ---------------------------------------------------------------- helpers

// Clause factor (1 - s) of a literal at variable value xv: a negated
// literal has s = 1 - xv and factor xv, a positive one factor 1 - xv.
__device__ __forceinline__ float lit_factor(int code, float xv) {
  return (code & 1) ? xv : 1.0f - xv;
}

// Truth of a literal under the rounded assignment [xv > 0.5].
__device__ __forceinline__ bool lit_true(int code, float xv) {
  const bool one = xv > 0.5f;
  return (code & 1) ? !one : one;
}

template <int N>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float (&o)[N]) {
  if constexpr (N == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else if constexpr (N == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    o[0] = t.x; o[1] = t.y;
  } else {
    o[0] = p[0];
  }
}

template <int N>
__device__ __forceinline__ void store_row(float* __restrict__ p, const float (&o)[N]) {
  if constexpr (N == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  } else if constexpr (N == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(o[0], o[1]);
  } else {
    p[0] = o[0];
  }
}

// Streaming (non-temporal) row access for data written once and read once
// (the two-phase contribution rows), so it does not evict the gathered
// state rows from the caches.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));

template <int N>
__device__ __forceinline__ void store_row_nt(float* __restrict__ p, const float (&o)[N]) {
  if constexpr (N == 4) {
    nt_f4 t = {o[0], o[1], o[2], o[3]};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(p));
  } else if constexpr (N == 2) {
    nt_f2 t = {o[0], o[1]};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f2*>(p));
  } else {
    __builtin_nontemporal_store(o[0], p);
  }
}

template <int N>
__device__ __forceinline__ void load_row_nt(const float* __restrict__ p, float (&o)[N]) {
  if constexpr (N == 4) {
    const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else if constexpr (N == 2) {
    const nt_f2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    o[0] = t.x; o[1] = t.y;
  } else {
    o[0] = __builtin_nontemporal_load(p);
  }
}

// With a whole wave on one item, item indices are wave-uniform: moving them
// to a scalar register lets the compiler use scalar loads for the CSR.
template <int LPI>
__device__ __forceinline__ int uniform(int v) {
  if constexpr (LPI == 64) return __builtin_amdgcn_readfirstlane(v);
  return v;
}

// Loads from the read-only plan tables (CSR, occurrence records, chunk
// tables), which no kernel writes: reading them through the constant
// address space lets wave-uniform loads become scalar loads.
__device__ __forceinline__ int ldc(const int32_t* p, int64_t i) {
  return ((const __attribute__((address_space(4))) int32_t*)p)[i];
}

__device__ __forceinline__ int4 ldc4(const int4* p, int64_t i) {
  const int32_t* b = reinterpret_cast<const int32_t*>(p) + 4 * i;
  return make_int4(ldc(b, 0), ldc(b, 1), ldc(b, 2), ldc(b, 3));
}

__device__ __forceinline__ float clamp01(double y) {
  y = y < 0.0 ? 0.0 : y;
  y = y > 1.0 ? 1.0 : y;
  return (float)y;
}

// Sum per-thread partials over the item slots of the block in slot order
// and write one row of partial sums per (chunk, restart).
template <int LPI, int RPL>
__device__ __forceinline__ void block_partials(const double (&lsum)[RPL], const int (&usum)[RPL],
                                               int64_t row, int tile, int R, double* loss_part,
                                               int32_t* unsat_part) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  __shared__ double s_l[kBlock * RPL];
  __shared__ int s_u[kBlock * RPL];
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    s_l[slot * RT + lane * RPL + j] = lsum[j];
    s_u[slot * RT + lane * RPL + j] = usum[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RT; i += kBlock) {
    double acc = 0.0;
    int uacc = 0;
    for (int s = 0; s < IPB; ++s) {
      acc += s_l[s * RT + i];
      uacc += s_u[s * RT + i];
    }
    const int r = tile * RT + i;
    if (r < R) {
      loss_part[row * R + r] = acc;
      unsat_part[row * R + r] = uacc;
    }
  }
}

// ------------------------------------------------------- variable pass
//
// For a variable v and the restarts r of the lane, the gradient is
//   g[v][r] = sum over the occurrences q of v (var_occ order) of
//             dU_t/dx_v = slope_j * prod_{i != j} factor_i,
// with the product over the other literals taken either from the stored
// partial row or recomputed from x.  The
// occurrence that is the first literal of a recomputed clause also
// accounts for that clause's U_t and its rounded satisfaction, so each
// clause enters the loss and the unsat count exactly once.

// Occurrence records: per variable-major slot two int4 words, occ[q] and
// occx[q] (the second is read only for clauses of 5 to 8 literals).
// Header (occ[q].x): bits 0-2 the number of other literals (0..7), bit 3
// the own literal's sign (1 = negated), bit 4 whether the own literal is
// its clause's first, bits 5-6 the kind:
//   INLINE  recomputed clause of at most 8 literals; the other literals'
//           codes are occ[q].y, .z, .w, occx[q].x, .y, .z, .w (unused
//           entries repeat the own variable, so every load stays in
//           bounds);
//   GENERAL recomputed longer clause: occ[q].y = clause id, .z = own
//           position in clause_lits;
//   STORED  partial stored by the clause pass: occ[q].y = stored row.
constexpr int kRecInline = 0, kRecStored = 2;  // kind 1 is GENERAL
__device__ __forceinline__ int rec_kind(int hdr) { return hdr >> 5; }
__device__ __forceinline__ int rec_nother(int hdr) { return hdr & 7; }
__device__ __forceinline__ bool rec_neg(int hdr) { return (hdr & 8) != 0; }
__device__ __forceinline__ bool rec_first(int hdr) { return (hdr & 16) != 0; }

// Contribution of one occurrence whose other-literal product is prod: the
// slope of the own factor times prod, and, for the clause's first literal,
// the clause's U and rounded satisfaction (any_true: some other literal is
// true under rounding).
template <int RPL>
__device__ __forceinline__ void add_occurrence(bool own_neg, bool first, const float (&prod)[RPL],
                                               const bool (&any_true)[RPL], const float (&xv)[RPL],
                                               double (&g)[RPL], double (&lsum)[RPL],
                                               int (&usum)[RPL]) {
  const int own = own_neg ? 1 : 0;
#pragma unroll
  for (int j = 0; j < RPL; ++j) g[j] += (double)(own_neg ? prod[j] : -prod[j]);
  if (first) {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      lsum[j] += (double)(lit_factor(own, xv[j]) * prod[j]);
      usum[j] += (any_true[j] || lit_true(own, xv[j])) ? 0 : 1;
    }
  }
}

// Product of the first `nother` of NO gathered rows y[c] (codes[c]) and,
// when `first`, whether any of them is true under rounding.
template <int RPL, int NO>
__device__ __forceinline__ void combine(const int (&codes)[NO], const float (&y)[NO][RPL],
                                        int nother, bool first, float (&prod)[RPL],
                                        bool (&any_true)[RPL]) {
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    prod[j] = 1.0f;
    any_true[j] = false;
#pragma unroll
    for (int c = 0; c < NO; ++c) prod[j] *= c < nother ? lit_factor(codes[c], y[c][j]) : 1.0f;
  }
  if (first) {
#pragma unroll
    for (int j = 0; j < RPL; ++j)
#pragma unroll
      for (int c = 0; c < NO; ++c)
        any_true[j] = any_true[j] || (c < nother && lit_true(codes[c], y[c][j]));
  }
}

// Four consecutive INLINE occurrences with at most NO (<= 3) other literals
// each: every row gather is issued before any product is formed, so a wave
// keeps up to 4 * NO loads in flight.
template <int RPL, int NO>
__device__ __forceinline__ void inline4(const VarPassArgs& a, const int4 (&o)[4], int r0,
                                        const float (&xv)[RPL], double (&g)[RPL],
                                        double (&lsum)[RPL], int (&usum)[RPL]) {
  float y[4][NO][RPL];
  int codes[4][NO];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int all[3] = {o[k].y, o[k].z, o[k].w};
#pragma unroll
    for (int c = 0; c < NO; ++c) {
      codes[k][c] = all[c];
      load_row<RPL>(a.x + (int64_t)(all[c] >> 1) * a.ldx + r0, y[k][c]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int hdr = o[k].x;
    float prod[RPL];
    bool any_true[RPL];
    combine<RPL, NO>(codes[k], y[k], rec_nother(hdr), rec_first(hdr), prod, any_true);
    add_occurrence<RPL>(rec_neg(hdr), rec_first(hdr), prod, any_true, xv, g, lsum, usum);
  }
}

// One INLINE occurrence of up to 7 other literals, all gathers in flight.
template <int RPL>
__device__ __forceinline__ void inline_one(const VarPassArgs& a, const int4 o, int q, int r0,
                                           const float (&xv)[RPL], double (&g)[RPL],
                                           double (&lsum)[RPL], int (&usum)[RPL]) {
  const int hdr = o.x, nother = rec_nother(hdr);
  float prod[RPL];
  bool any_true[RPL];
  if (nother <= 3) {
    const int codes[3] = {o.y, o.z, o.w};
    float y[3][RPL];
#pragma unroll
    for (int c = 0; c < 3; ++c) load_row<RPL>(a.x + (int64_t)(codes[c] >> 1) * a.ldx + r0, y[c]);
    combine<RPL, 3>(codes, y, nother, rec_first(hdr), prod, any_true);
  } else {
    const int4 e = ldc4(a.occx, q);
    const int codes[7] = {o.y, o.z, o.w, e.x, e.y, e.z, e.w};
    float y[7][RPL];
#pragma unroll
    for (int c = 0; c < 7; ++c) load_row<RPL>(a.x + (int64_t)(codes[c] >> 1) * a.ldx + r0, y[c]);
    combine<RPL, 7>(codes, y, nother, rec_first(hdr), prod, any_true);
  }
  add_occurrence<RPL>(rec_neg(hdr), rec_first(hdr), prod, any_true, xv, g, lsum, usum);
}

// One GENERAL occurrence: the clause's other literals four at a time.
template <int RPL>
__device__ __forceinline__ void general_one(const VarPassArgs& a, const int4 o, int r0,
                                            const float (&xv)[RPL], double (&g)[RPL],
                                            double (&lsum)[RPL], int (&usum)[RPL]) {
  const int t = o.y, p = o.z;
  const int cs = ldc(a.clause_ptr, t), ce = ldc(a.clause_ptr, t + 1);
  const bool first = p == cs;
  float prod[RPL];
  bool any_true[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { prod[j] = 1.0f; any_true[j] = false; }
  for (int i = cs; i < ce; i += 4) {
    int codes[4];
    float y[4][RPL];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // positions past the clause read the clause's first literal again and
      // are masked out below, like the own position
      const int iu = i + u < ce ? i + u : cs;
      codes[u] = ldc(a.clause_lits, iu);
      load_row<RPL>(a.x + (int64_t)(codes[u] >> 1) * a.ldx + r0, y[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool use = i + u < ce && i + u != p;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        prod[j] *= use ? lit_factor(codes[u], y[u][j]) : 1.0f;
        any_true[j] = any_true[j] || (use && lit_true(codes[u], y[u][j]));
      }
    }
  }
  add_occurrence<RPL>((ldc(a.clause_lits, p) & 1) != 0, first, prod, any_true, xv, g, lsum, usum);
}

// Product over the other literals (and, for a first literal, whether one
// of them is true) of one INLINE or GENERAL occurrence.
template <int RPL>
__device__ __forceinline__ void occurrence_product(const VarPassArgs& a, const int4 o, int q, int r0,
                                                   float (&prod)[RPL], bool (&any_true)[RPL]) {
  const int hdr = o.x, nother = rec_nother(hdr);
  if (rec_kind(hdr) == kRecInline) {
    if (nother <= 3) {
      const int codes[3] = {o.y, o.z, o.w};
      float y[3][RPL];
#pragma unroll
      for (int c = 0; c < 3; ++c) load_row<RPL>(a.x + (int64_t)(codes[c] >> 1) * a.ldx + r0, y[c]);
      combine<RPL, 3>(codes, y, nother, rec_first(hdr), prod, any_true);
    } else {
      const int4 e = ldc4(a.occx, q);
      const int codes[7] = {o.y, o.z, o.w, e.x, e.y, e.z, e.w};
      float y[7][RPL];
#pragma unroll
      for (int c = 0; c < 7; ++c) load_row<RPL>(a.x + (int64_t)(codes[c] >> 1) * a.ldx + r0, y[c]);
      combine<RPL, 7>(codes, y, nother, rec_first(hdr), prod, any_true);
    }
    return;
  }
  const int t = o.y, p = o.z;
  const int cs = ldc(a.clause_ptr, t), ce = ldc(a.clause_ptr, t + 1);
#pragma unroll
  for (int j = 0; j < RPL; ++j) { prod[j] = 1.0f; any_true[j] = false; }
  for (int i = cs; i < ce; i += 4) {
    int codes[4];
    float y[4][RPL];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int iu = i + u < ce ? i + u : cs;
      codes[u] = ldc(a.clause_lits, iu);
      load_row<RPL>(a.x + (int64_t)(codes[u] >> 1) * a.ldx + r0, y[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool use = i + u < ce && i + u != p;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        prod[j] *= use ? lit_factor(codes[u], y[u][j]) : 1.0f;
        any_true[j] = any_true[j] || (use && lit_true(codes[u], y[u][j]));
      }
    }
  }
}

// One occurrence of any kind.
template <int RPL>
__device__ __forceinline__ void one_occurrence(const VarPassArgs& a, const int4 o, int q, int r0,
                                               const float (&xv)[RPL], double (&g)[RPL],
                                               double (&lsum)[RPL], int (&usum)[RPL]) {
  const int kind = rec_kind(o.x);
  if (kind == kRecStored) {
    float d[RPL];
    load_row<RPL>(a.D + (int64_t)o.y * a.ldD + r0, d);
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] += (double)d[j];
  } else if (kind == kRecInline) {
    inline_one<RPL>(a, o, q, r0, xv, g, lsum, usum);
  } else {
    general_one<RPL>(a, o, r0, xv, g, lsum, usum);
  }
}

// Adds the contributions of occurrences [q0, q1) (in that order) of the
// variable whose own state is xv.  r0 must be a valid column for every lane
// (lanes past the last restart pass a clamped one and discard the results),
// so the loop runs under wave-uniform control and its table loads can be
// scalar.
template <int RPL>
__device__ __forceinline__ void gather_occurrences(const VarPassArgs& a, int q0, int q1, int r0,
                                                   const float (&xv)[RPL], double (&g)[RPL],
                                                   double (&lsum)[RPL], int (&usum)[RPL]) {
  int q = q0;
  while (q < q1) {
    if (q + 4 <= q1) {
      const int4 o[4] = {ldc4(a.occ, q), ldc4(a.occ, q + 1), ldc4(a.occ, q + 2),
                         ldc4(a.occ, q + 3)};
      const int k0 = rec_kind(o[0].x), k1 = rec_kind(o[1].x), k2 = rec_kind(o[2].x),
                k3 = rec_kind(o[3].x);
      if ((k0 | k1 | k2 | k3) == kRecInline) {
        const int most = max(max(rec_nother(o[0].x), rec_nother(o[1].x)),
                             max(rec_nother(o[2].x), rec_nother(o[3].x)));
        if (most <= 2) {
          inline4<RPL, 2>(a, o, r0, xv, g, lsum, usum);
        } else if (most <= 3) {
          inline4<RPL, 3>(a, o, r0, xv, g, lsum, usum);
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) inline_one<RPL>(a, o[k], q + k, r0, xv, g, lsum, usum);
        }
        q += 4;
        continue;
      }
      if (k0 == kRecStored && k1 == kRecStored && k2 == kRecStored && k3 == kRecStored) {
        float d[4][RPL];
#pragma unroll
        for (int k = 0; k < 4; ++k) load_row<RPL>(a.D + (int64_t)o[k].y * a.ldD + r0, d[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int j = 0; j < RPL; ++j) g[j] += (double)d[k][j];
        q += 4;
        continue;
      }
    }
    one_occurrence<RPL>(a, ldc4(a.occ, q), q, r0, xv, g, lsum, usum);
    ++q;
  }
}

// The epilogue for one variable row: projected SGD or Adam update (writing
// the next state) or the (upstream-scaled) gradient.
template <int RPL, int MODE>
__device__ __forceinline__ void var_epilogue(const VarPassArgs& a, int v, int r0,
                                             const float (&xv)[RPL], const double (&g)[RPL]) {
  float o[RPL];
  if constexpr (MODE == kModeSGD) {
#pragma unroll
    for (int j = 0; j < RPL; ++j) o[j] = clamp01((double)xv[j] - (double)a.lr * g[j]);
  } else if constexpr (MODE == kModeAdam) {
    float m[RPL], s2[RPL];
    float* mp = a.mom + (int64_t)v * a.ldm + r0;
    float* vp = a.vel + (int64_t)v * a.ldm + r0;
    load_row<RPL>(mp, m);
    load_row<RPL>(vp, s2);
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const double mm = (double)a.b1 * (double)m[j] + (1.0 - (double)a.b1) * g[j];
      const double vv = (double)a.b2 * (double)s2[j] + (1.0 - (double)a.b2) * g[j] * g[j];
      m[j] = (float)mm;
      s2[j] = (float)vv;
      const double step = (double)a.lr * ((double)m[j] * a.inv_c1) /
                          (sqrt((double)s2[j] * a.inv_c2) + (double)a.eps);
      o[j] = clamp01((double)xv[j] - step);
    }
    store_row<RPL>(mp, m);
    store_row<RPL>(vp, s2);
  } else {
    const int R = a.R;
    const int f = a.upstream ? a.var_formula[v] : 0;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const double w = a.upstream ? (double)a.upstream[(int64_t)f * R + r0 + j] : 1.0;
      o[j] = (float)(w * g[j]);
    }
  }
  store_row<RPL>(a.out + (int64_t)v * a.ldo + r0, o);
}

// Variables of the chunk's range (the ranges exclude split variables): the
// whole gradient, then the epilogue.
template <int LPI, int RPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_var_pass(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk =
      a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x) : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;  // in-bounds column for lanes past the last restart
  const int vb = ldc(a.chunk_vbeg, chunk), ve = ldc(a.chunk_vend, chunk);
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  for (int v0 = vb + slot; v0 < ve; v0 += IPB) {
    const int v = uniform<LPI>(a.var_perm ? ldc(a.var_perm, v0) : v0);
    double g[RPL];
    float xv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    load_row<RPL>(a.x + (int64_t)v * a.ldx + rc, xv);
    gather_occurrences<RPL>(a, ldc(a.var_ptr, v), ldc(a.var_ptr, v + 1), rc, xv, g, lsum, usum);
    if (active) var_epilogue<RPL, MODE>(a, v, r0, xv, g);
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// Streaming variant for small restart tiles: each item slot walks the
// occurrences of a contiguous run of variables as one list, four records at
// a time across variable boundaries, so a variable's last few occurrences
// share a batch with the next variable's first ones instead of costing a
// memory round trip each.  Sums and their order per variable are those of
// k_var_pass.
template <int RPL, int NO>
__device__ __forceinline__ void inline4_products(const VarPassArgs& a, const int4 (&o)[4], int r0,
                                                 float (&prod)[4][RPL], bool (&any_true)[4][RPL]) {
  float y[4][NO][RPL];
  int codes[4][NO];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int all[3] = {o[k].y, o[k].z, o[k].w};
#pragma unroll
    for (int c = 0; c < NO; ++c) {
      codes[k][c] = all[c];
      load_row<RPL>(a.x + (int64_t)(all[c] >> 1) * a.ldx + r0, y[k][c]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    combine<RPL, NO>(codes[k], y[k], rec_nother(o[k].x), rec_first(o[k].x), prod[k], any_true[k]);
}

template <int LPI, int RPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_var_stream(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk =
      a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x) : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  const int vb = ldc(a.chunk_vbeg, chunk), ve = ldc(a.chunk_vend, chunk);
  // occurrence-balanced split of [vb, ve) into IPB contiguous runs
  const int qB = ldc(a.var_ptr, vb), qE = ldc(a.var_ptr, ve);
  auto split = [&](int s) -> int {  // first v in [vb, ve] with var_ptr[v] >= target
    if (s <= 0) return vb;
    if (s >= IPB) return ve;
    const int target = qB + (int)((int64_t)(qE - qB) * s / IPB);
    int lo = vb, hi = ve;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ldc(a.var_ptr, mid) < target) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  const int va = uniform<LPI>(split(slot)), vz = uniform<LPI>(split(slot + 1));
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  int v = va;
  int cur_end = v < vz ? ldc(a.var_ptr, v + 1) : 0;
  double g[RPL];
  float xv[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { g[j] = 0.0; xv[j] = 0.0f; }
  if (v < vz) load_row<RPL>(a.x + (int64_t)v * a.ldx + rc, xv);
  // finishes every variable whose occurrences end at or before position qpos
  auto finish_before = [&](int qpos) {
    while (v < vz && cur_end <= qpos) {
      if (active) var_epilogue<RPL, MODE>(a, v, r0, xv, g);
      ++v;
#pragma unroll
      for (int j = 0; j < RPL; ++j) g[j] = 0.0;
      if (v < vz) {
        cur_end = ldc(a.var_ptr, v + 1);
        load_row<RPL>(a.x + (int64_t)v * a.ldx + rc, xv);
      }
    }
  };
  int q = va < vz ? ldc(a.var_ptr, va) : 0;
  const int qz = va < vz ? ldc(a.var_ptr, vz) : 0;
  finish_before(q);
  while (q < qz) {
    if (q + 4 <= qz) {
      const int4 o[4] = {ldc4(a.occ, q), ldc4(a.occ, q + 1), ldc4(a.occ, q + 2),
                         ldc4(a.occ, q + 3)};
      const int kinds = rec_kind(o[0].x) | rec_kind(o[1].x) | rec_kind(o[2].x) | rec_kind(o[3].x);
      const int most = max(max(rec_nother(o[0].x), rec_nother(o[1].x)),
                           max(rec_nother(o[2].x), rec_nother(o[3].x)));
      if (kinds == kRecInline && most <= 3) {
        float prod[4][RPL];
        bool any_true[4][RPL];
        if (most <= 2)
          inline4_products<RPL, 2>(a, o, rc, prod, any_true);
        else
          inline4_products<RPL, 3>(a, o, rc, prod, any_true);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          finish_before(q + k);
          add_occurrence<RPL>(rec_neg(o[k].x), rec_first(o[k].x), prod[k], any_true[k], xv, g,
                              lsum, usum);
        }
        q += 4;
        continue;
      }
    }
    finish_before(q);
    one_occurrence<RPL>(a, ldc4(a.occ, q), q, rc, xv, g, lsum, usum);
    ++q;
  }
  finish_before(qz);
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// ---------------------------------------------------- two-phase plan
//
// For small restart tiles the variable-centric walk leaves each wave little
// data per memory round trip.  The two-phase plan splits it: an
// occurrence-parallel pass writes every recomputed contribution
// slope * prod_{i != j} a_i to its variable-major slot of C (the clause
// pass writes the long clauses' slots), then a variable pass sums each
// variable's contiguous slots in order.  The sums and their order equal the
// single-pass kernel's, so gradients are bitwise identical.

// Phase A: occurrences [qa, qz) of the chunk, item slot s taking
// q = qa + s, qa + s + IPB, ...; four of a slot's occurrences are handled
// together with all their gathers in flight.
template <int LPI, int RPL>
__global__ __launch_bounds__(kBlock) void k_occ_pass(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk =
      a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x) : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  const int qa = ldc(a.chunk_vbeg, chunk), qz = ldc(a.chunk_vend, chunk);
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }
  auto emit = [&](int q, int hdr, const float (&prod)[RPL], const bool (&any_true)[RPL]) {
    const bool neg = rec_neg(hdr);
    float c[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) c[j] = neg ? prod[j] : -prod[j];
    if (active) store_row_nt<RPL>(a.C + (int64_t)q * a.ldD + r0, c);
    if (rec_first(hdr)) {
      float xv[RPL];
      load_row<RPL>(a.x + (int64_t)ldc(a.occ_own, q) * a.ldx + rc, xv);
      const int own = neg ? 1 : 0;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        lsum[j] += (double)(lit_factor(own, xv[j]) * prod[j]);
        usum[j] += (any_true[j] || lit_true(own, xv[j])) ? 0 : 1;
      }
    }
  };
  int q = qa + slot;
  for (; q + 3 * IPB < qz; q += 4 * IPB) {
    const int4 o[4] = {ldc4(a.occ, q), ldc4(a.occ, q + IPB), ldc4(a.occ, q + 2 * IPB),
                       ldc4(a.occ, q + 3 * IPB)};
    const int kinds = rec_kind(o[0].x) | rec_kind(o[1].x) | rec_kind(o[2].x) | rec_kind(o[3].x);
    const int most = max(max(rec_nother(o[0].x), rec_nother(o[1].x)),
                         max(rec_nother(o[2].x), rec_nother(o[3].x)));
    if (kinds == kRecInline && most <= 3) {
      float prod[4][RPL];
      bool any_true[4][RPL];
      if (most <= 2)
        inline4_products<RPL, 2>(a, o, rc, prod, any_true);
      else
        inline4_products<RPL, 3>(a, o, rc, prod, any_true);
#pragma unroll
      for (int k = 0; k < 4; ++k) emit(q + k * IPB, o[k].x, prod[k], any_true[k]);
      continue;
    }
    for (int k = 0; k < 4; ++k) {
      const int qk = q + k * IPB;
      const int kind = rec_kind(o[k].x);
      if (kind == kRecStored) continue;
      float prod[RPL];
      bool any_true[RPL];
      occurrence_product<RPL>(a, o[k], qk, rc, prod, any_true);
      emit(qk, o[k].x, prod, any_true);
    }
  }
  for (; q < qz; q += IPB) {
    const int4 o = ldc4(a.occ, q);
    if (rec_kind(o.x) == kRecStored) continue;
    float prod[RPL];
    bool any_true[RPL];
    occurrence_product<RPL>(a, o, q, rc, prod, any_true);
    emit(q, o.x, prod, any_true);
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// Phase B: each variable of the chunk sums its slots of C in order (four
// independent row loads in flight), then the epilogue.
template <int LPI, int RPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_var_sum(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk =
      a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x) : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  const int vb = ldc(a.chunk_vbeg, chunk), ve = ldc(a.chunk_vend, chunk);
  for (int v0 = vb + slot; v0 < ve; v0 += IPB) {
    const int v = uniform<LPI>(a.var_perm ? ldc(a.var_perm, v0) : v0);
    double g[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    const int q0 = ldc(a.var_ptr, v), q1 = ldc(a.var_ptr, v + 1);
    int q = q0;
    for (; q + 4 <= q1; q += 4) {
      float c[4][RPL];
#pragma unroll
      for (int k = 0; k < 4; ++k) load_row_nt<RPL>(a.C + (int64_t)(q + k) * a.ldD + rc, c[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < RPL; ++j) g[j] += (double)c[k][j];
    }
    for (; q < q1; ++q) {
      float c[RPL];
      load_row_nt<RPL>(a.C + (int64_t)q * a.ldD + rc, c);
#pragma unroll
      for (int j = 0; j < RPL; ++j) g[j] += (double)c[j];
    }
    if (active) {
      float xv[RPL];
      load_row<RPL>(a.x + (int64_t)v * a.ldx + r0, xv);
      var_epilogue<RPL, MODE>(a, v, r0, xv, g);
    }
  }
}

// Phase B for split variables: each segment's slots summed in FP64 into
// gseg (then k_heavy_finish adds the segments in order).
template <int LPI, int RPL>
__global__ __launch_bounds__(kBlock) void k_seg_sum(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk = a.chunk_base + blockIdx.x;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  const int sb = ldc(a.chunk_vbeg, chunk), se = ldc(a.chunk_vend, chunk);
  for (int s0 = sb + slot; s0 < se; s0 += IPB) {
    const int sgi = uniform<LPI>(s0);
    const int q0 = ldc(a.seg_q0, sgi), q1 = ldc(a.seg_q1, sgi);
    double g[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    int q = q0;
    for (; q + 4 <= q1; q += 4) {
      float c[4][RPL];
#pragma unroll
      for (int k = 0; k < 4; ++k) load_row_nt<RPL>(a.C + (int64_t)(q + k) * a.ldD + rc, c[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < RPL; ++j) g[j] += (double)c[k][j];
    }
    for (; q < q1; ++q) {
      float c[RPL];
      load_row_nt<RPL>(a.C + (int64_t)q * a.ldD + rc, c);
#pragma unroll
      for (int j = 0; j < RPL; ++j) g[j] += (double)c[j];
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) a.gseg[(int64_t)sgi * a.R + r0 + j] = g[j];
    }
  }
}

// Segments of split variables (variables with more occurrences than one
// item should serialise): each segment's partial gradient goes to
// gseg[s][r] in FP64.
template <int LPI, int RPL>
__global__ __launch_bounds__(kBlock) void k_var_seg(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk = a.chunk_base + blockIdx.x;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  const int sb = ldc(a.chunk_vbeg, chunk), se = ldc(a.chunk_vend, chunk);
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  for (int s0 = sb + slot; s0 < se; s0 += IPB) {
    const int sgi = uniform<LPI>(s0);
    const int v = ldc(a.seg_var, sgi);
    double g[RPL];
    float xv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    load_row<RPL>(a.x + (int64_t)v * a.ldx + rc, xv);
    gather_occurrences<RPL>(a, ldc(a.seg_q0, sgi), ldc(a.seg_q1, sgi), rc, xv, g, lsum, usum);
    if (active) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) a.gseg[(int64_t)sgi * a.R + r0 + j] = g[j];
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// Split variables: their segments' partial gradients summed in segment
// order, then the same epilogue as k_var_pass.
template <int LPI, int RPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_heavy_finish(VarPassArgs a, int h0, int h1) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  if (r0 >= a.R) return;
  for (int i = h0 + blockIdx.x * IPB + slot; i < h1; i += gridDim.x * IPB) {
    const int v = a.heavy_var[i];
    double g[RPL];
    float xv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    load_row<RPL>(a.x + (int64_t)v * a.ldx + r0, xv);
    for (int sgi = a.heavy_sbeg[i]; sgi < a.heavy_sbeg[i + 1]; ++sgi) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) g[j] += a.gseg[(int64_t)sgi * a.R + r0 + j];
    }
    var_epilogue<RPL, MODE>(a, v, r0, xv, g);
  }
}

// -------------------------------------------------------- clause pass
//
// For each clause t of the chunk: U_t = prod_i factor_i, its rounded
// satisfaction, and (WRITE_D) the partial of every literal j,
//   D[slot(j)][r] = slope_j * prod_{i<j} factor_i * prod_{i>j} factor_i,
// from a forward prefix sweep (prefix stored in place) and a backward
// suffix sweep.  No division: exact zero factors need no special case.
template <int LPI, int RPL, bool WRITE_D>
__global__ __launch_bounds__(kBlock) void k_clause_pass(ClausePassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk = a.chunk_base + blockIdx.x;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;  // in-bounds column for lanes past the last restart
  const int cb = ldc(a.chunk_cbeg, chunk), ce = ldc(a.chunk_cend, chunk);
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  for (int c0 = cb + slot; c0 < ce; c0 += IPB) {
    const int t = uniform<LPI>(a.clause_ids ? ldc(a.clause_ids, c0) : c0);
    const int s = ldc(a.clause_ptr, t), e = ldc(a.clause_ptr, t + 1);
    float pre[RPL];
    bool any_true[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) { pre[j] = 1.0f; any_true[j] = false; }
    // forward sweep, four literals' rows in flight at a time; with WRITE_D
    // the prefix product before each literal is stored in its partial row
    int i = s;
    for (; i + 4 <= e; i += 4) {
      int code[4];
      float y[4][RPL];
#pragma unroll
      for (int u = 0; u < 4; ++u) code[u] = ldc(a.clause_lits, i + u);
#pragma unroll
      for (int u = 0; u < 4; ++u) load_row<RPL>(a.x + (int64_t)(code[u] >> 1) * a.ldx + rc, y[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if constexpr (WRITE_D) {
          if (active) store_row<RPL>(a.D + (int64_t)ldc(a.lit_dslot, i + u) * a.ldD + r0, pre);
        }
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          pre[j] *= lit_factor(code[u], y[u][j]);
          any_true[j] = any_true[j] || lit_true(code[u], y[u][j]);
        }
      }
    }
    for (; i < e; ++i) {
      const int code = ldc(a.clause_lits, i);
      float y[RPL];
      load_row<RPL>(a.x + (int64_t)(code >> 1) * a.ldx + rc, y);
      if constexpr (WRITE_D) {
        if (active) store_row<RPL>(a.D + (int64_t)ldc(a.lit_dslot, i) * a.ldD + r0, pre);
      }
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        pre[j] *= lit_factor(code, y[j]);
        any_true[j] = any_true[j] || lit_true(code, y[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      lsum[j] += (double)pre[j];
      usum[j] += any_true[j] ? 0 : 1;
    }
    if constexpr (WRITE_D) {
      // backward sweep: partial = slope * prefix * suffix
      float suf[RPL];
#pragma unroll
      for (int j = 0; j < RPL; ++j) suf[j] = 1.0f;
      int i2 = e - 1;
      for (; i2 - 3 >= s; i2 -= 4) {
        int code[4];
        float y[4][RPL], d[4][RPL];
#pragma unroll
        for (int u = 0; u < 4; ++u) code[u] = ldc(a.clause_lits, i2 - u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          load_row<RPL>(a.x + (int64_t)(code[u] >> 1) * a.ldx + rc, y[u]);
          load_row<RPL>(a.D + (int64_t)ldc(a.lit_dslot, i2 - u) * a.ldD + rc, d[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float slope = (code[u] & 1) ? 1.0f : -1.0f;
#pragma unroll
          for (int j = 0; j < RPL; ++j) {
            d[u][j] = slope * (d[u][j] * suf[j]);
            suf[j] *= lit_factor(code[u], y[u][j]);
          }
          if (active) store_row<RPL>(a.D + (int64_t)ldc(a.lit_dslot, i2 - u) * a.ldD + r0, d[u]);
        }
      }
      for (; i2 >= s; --i2) {
        const int code = ldc(a.clause_lits, i2);
        float y[RPL], d[RPL];
        load_row<RPL>(a.x + (int64_t)(code >> 1) * a.ldx + rc, y);
        float* dp = a.D + (int64_t)ldc(a.lit_dslot, i2) * a.ldD;
        load_row<RPL>(dp + rc, d);
        const float slope = (code & 1) ? 1.0f : -1.0f;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          d[j] = slope * (d[j] * suf[j]);
          suf[j] *= lit_factor(code, y[j]);
        }
        if (active) store_row<RPL>(dp + r0, d);
      }
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row ? ldc(a.chunk_row, chunk) : chunk, tile, a.R,
                           a.loss_part, a.unsat_part);
}

// ------------------------------------------------------------ finalize
//
// loss[f][r] = sum of the formula's partial rows (fixed order) + empty
// clauses; the same for the unsat count.
// W waves per block: wave w sums rows w, w + W, ... for 64 restarts, then
// the W partial sums are combined pairwise in a fixed tree.
template <int W>
__global__ __launch_bounds__(64 * W) void k_finalize(FinalizeArgs a) {
  const int f = a.f_base + blockIdx.x;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  const int R = a.R;
  double acc = 0.0;
  int uacc = 0;
  if (r < R) {
    const int rb = a.a_beg[f], re = a.a_end[f];
    for (int row = rb + w; row < re; row += W) {
      if (a.loss_out) acc += a.loss_part[(int64_t)row * R + r];
      if (a.unsat_out) uacc += a.unsat_part[(int64_t)row * R + r];
    }
  }
  __shared__ double sl[64 * W];
  __shared__ int su[64 * W];
  sl[threadIdx.x] = acc;
  su[threadIdx.x] = uacc;
  __syncthreads();
#pragma unroll
  for (int half = W / 2; half >= 1; half /= 2) {
    if (w < half) {
      sl[threadIdx.x] += sl[threadIdx.x + 64 * half];
      su[threadIdx.x] += su[threadIdx.x + 64 * half];
    }
    __syncthreads();
  }
  if (w == 0 && r < R) {
    const double tot = sl[lane] + (double)a.n_empty[f];
    const int utot = su[lane] + a.n_empty[f];
    if (a.loss_out) a.loss_out[(int64_t)f * R + r] = (float)tot;
    if (a.unsat_out) a.unsat_out[(int64_t)f * R + r] = utot;
  }
}

// ---------------------------------------------------------- init / copy

__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_init_state(float* x, int32_t ldx, int32_t n, int32_t R,
                                                    uint64_t seed) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4) {
    const uint64_t key = ((uint64_t)(uint32_t)v << 32) + (uint64_t)(uint32_t)r + 0x9e3779b97f4a7c15ULL;
    const uint64_t h = splitmix_mix(seed ^ splitmix_mix(key));
    x[v * ldx + r] = (float)(h >> 40) * (1.0f / 16777216.0f);
  }
}

__global__ __launch_bounds__(256) void k_copy_state(const float* src, int32_t lds, float* dst,
                                                    int32_t ldd, int32_t n, int32_t R) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int r = blockIdx.y * 64 + lane; r < R; r += gridDim.y * 64)
    for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4)
      dst[v * ldd + r] = src[v * lds + r];
}

__global__ void k_zero_i32(int32_t* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ------------------------------------------- straight-through Gumbel mode
//
// Two logits per (variable, restart) go through a temperature softmax after
// Gumbel(0,1) noise (Section 3.2, Eq. 3); the forward uses the hard argmax
// (Eq. 4) and the backward the soft probabilities.  With two states only the
// logit difference d = theta1 - theta0 and the noise difference
// l = g1 - g0 matter: y1 = sigma((d + l) / tau), x_hat = [d + l > 0].

// Noise difference of step t for (v, r): g_j = -log(-log(u_j)) with
// u_j = ((h_j >> 40) + 0.5) * 2^-24 and h_j the SplitMix64 mix of
// (seed, v * 2^32 + 2r + j, t), evaluated in FP64 and rounded once.
__device__ __forceinline__ float gumbel_diff(uint64_t seed, int t, int64_t v, int r) {
  const uint64_t ts = splitmix_mix((uint64_t)(uint32_t)t + 0x632be59bd9b4e019ULL);
  double g[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const uint64_t c = ((uint64_t)(uint32_t)v << 32) + 2 * (uint64_t)(uint32_t)r + (uint64_t)j;
    const uint64_t h = splitmix_mix(seed ^ splitmix_mix(c ^ ts));
    const double u = ((double)(h >> 40) + 0.5) * (1.0 / 16777216.0);
    g[j] = -log(-log(u));
  }
  return (float)(g[1] - g[0]);
}

__global__ __launch_bounds__(256) void k_gumbel_noise(float* out, int32_t ldo, int32_t n, int32_t R,
                                                      uint64_t seed, int32_t t) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4)
    out[v * ldo + r] = gumbel_diff(seed, t, v, r);
}

// Hard point of the step: xh = [d + l > 0] (FP32 sum; a tie goes to state
// 0), keeping l for the update.  noise: caller-given l or null to draw it.
__global__ __launch_bounds__(256) void k_gumbel_prep(const float* d, int32_t ldd, const float* noise,
                                                     int32_t ldn, uint64_t seed, int32_t t,
                                                     int32_t n, int32_t R, float* xh, float* nb,
                                                     int32_t ld) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4) {
    const float l = noise ? noise[v * ldn + r] : gumbel_diff(seed, t, v, r);
    const float s = d[v * ldd + r] + l;
    xh[v * ld + r] = s > 0.0f ? 1.0f : 0.0f;
    nb[v * ld + r] = l;
  }
}

// Soft backward and update: g1 = G * y1 (1 - y1) / tau reaches theta1 and
// -g1 reaches theta0, so d moves by twice theta1's step (SGD, or Adam whose
// theta0 moments are the exact negatives of theta1's).
__global__ __launch_bounds__(256) void k_gumbel_update(float* d, int32_t ldd, const float* nb,
                                                       const float* G, int32_t ld, float* mom,
                                                       float* vel, int32_t ldm, int32_t n,
                                                       int32_t R, float tau, float lr, float b1,
                                                       float b2, float eps, double inv_c1,
                                                       double inv_c2, int32_t adam) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4) {
    const double dv = d[v * ldd + r];
    const double z = (dv + (double)nb[v * ld + r]) / (double)tau;
    const double y1 = 1.0 / (1.0 + exp(-z));
    const double g1 = (double)G[v * ld + r] * y1 * (1.0 - y1) / (double)tau;
    double step;
    if (adam) {
      const double mm = (double)b1 * (double)mom[v * ldm + r] + (1.0 - (double)b1) * g1;
      const double vv = (double)b2 * (double)vel[v * ldm + r] + (1.0 - (double)b2) * g1 * g1;
      mom[v * ldm + r] = (float)mm;
      vel[v * ldm + r] = (float)vv;
      step = (double)lr * ((double)(float)mm * inv_c1) /
             (sqrt((double)(float)vv * inv_c2) + (double)eps);
    } else {
      step = (double)lr * g1;
    }
    d[v * ldd + r] = (float)(dv - 2.0 * step);
  }
}

// ---------------------------------------------------------- hand-off
//
// Candidate pool of Section 3.3.1, Eq. (8): candidate k of formula f adds
// the noise difference of "step" k, restart 0 to the logit difference of
// f's selected restart and takes the argmax; its confidence is the
// perturbed probability of the value taken.
__global__ __launch_bounds__(256) void k_candidates(const float* d, int32_t ldd,
                                                    const int32_t* var_formula, const int32_t* best,
                                                    int32_t n, uint64_t seed, float tau,
                                                    uint8_t* assign, float* conf) {
  const int k = blockIdx.y;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int r = best[var_formula[v]];
    const float dv = d[v * ldd + r];
    const float l = gumbel_diff(seed, k, v, 0);
    const bool one = dv + l > 0.0f;
    const double y1 = 1.0 / (1.0 + exp(-((double)dv + (double)l) / (double)tau));
    assign[(int64_t)k * n + v] = one ? 1 : 0;
    conf[(int64_t)k * n + v] = (float)(one ? y1 : 1.0 - y1);
  }
}

// Unperturbed confidence max(p, 1 - p), p = sigma(d / tau), of each
// variable at its formula's selected restart (Section 3.3.2).
__global__ __launch_bounds__(256) void k_confidence(const float* d, int32_t ldd,
                                                    const int32_t* var_formula, const int32_t* best,
                                                    int32_t n, float tau, float* conf) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const double p = 1.0 / (1.0 + exp(-(double)d[v * ldd + best[var_formula[v]]] / (double)tau));
    conf[v] = (float)(p > 0.5 ? p : 1.0 - p);
  }
}

// Selection of the S_f most (HIGH) or least confident variables of formula
// f in candidate k, ties to the lower index, written in increasing index
// order.  Keys are 64-bit: confidence bits (inverted for LOW) above the
// inverted local index, so every key is distinct and larger = preferred.
// An exact radix select (eight 8-bit digits, integer counts in LDS) finds
// the S-th largest key; a block scan then compacts the selected indices.
template <bool HIGH>
__device__ __forceinline__ uint64_t sel_key(float c, int local) {
  const uint32_t b = __float_as_uint(c);
  const uint64_t hi = HIGH ? b : ~b;
  return (hi << 32) | (uint64_t)(~(uint32_t)local);
}

template <bool HIGH>
__global__ __launch_bounds__(1024) void k_select(const float* conf, int32_t n,
                                                 const int32_t* f_vbeg, const int32_t* sel_off,
                                                 int32_t stot, int32_t* out) {
  const int f = blockIdx.x, k = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int v0 = f_vbeg[f], nf = f_vbeg[f + 1] - v0;
  const int S = sel_off[f + 1] - sel_off[f];
  if (S <= 0) return;
  const float* c = conf + (int64_t)k * n + v0;
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix, s_mask;
  __shared__ int s_rank;
  if (tid == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_rank = S;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int b = tid; b < 256; b += nt) hist[b] = 0;
    __syncthreads();
    const uint64_t prefix = s_prefix, mask = s_mask;
    for (int i = tid; i < nf; i += nt) {
      const uint64_t key = sel_key<HIGH>(c[i], i);
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      int rank = s_rank, acc = 0, chosen = 0;
      for (int b = 255; b >= 0; --b) {
        if (acc + (int)hist[b] >= rank) {
          chosen = b;
          rank -= acc;
          break;
        }
        acc += (int)hist[b];
      }
      s_prefix = prefix | ((uint64_t)chosen << shift);
      s_mask = mask | (0xFFULL << shift);
      s_rank = rank;
    }
    __syncthreads();
  }
  const uint64_t thr = s_prefix;  // the S-th largest key: keys >= thr are the selection
  __shared__ int cnt[1024];
  const int per = (nf + nt - 1) / nt;
  const int i0 = tid * per, i1 = min(nf, i0 + per);
  int mine = 0;
  for (int i = i0; i < i1; ++i) mine += sel_key<HIGH>(c[i], i) >= thr ? 1 : 0;
  cnt[tid] = mine;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int t = 0; t < nt; ++t) {
      const int x = cnt[t];
      cnt[t] = acc;
      acc += x;
    }
  }
  __syncthreads();
  int pos = cnt[tid];
  int32_t* o = out + (int64_t)k * stot + sel_off[f];
  for (int i = i0; i < i1; ++i)
    if (sel_key<HIGH>(c[i], i) >= thr) o[pos++] = v0 + i;
}

// ------------------------------------------------------- round & count
//
// bits[w][v]: bit l = [x[v][64w + l] > 0.5] packed by one wavefront ballot.
__global__ __launch_bounds__(256) void k_pack_bits(const float* x, int32_t ldx, int32_t n,
                                                   int32_t R, uint64_t* bits) {
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int word = blockIdx.y;
  const int r = word * 64 + lane;
  for (int64_t v = (int64_t)blockIdx.x * 4 + wv; v < n; v += (int64_t)gridDim.x * 4) {
    const bool one = (r < R) && (x[v * ldx + r] > 0.5f);
    const uint64_t m = __ballot(one);
    if (lane == 0) bits[(int64_t)word * n + v] = m;
  }
}

// Lanes take one clause each; for the 64 restarts of word w a clause's
// "unsatisfied" mask is the AND over its literals of "literal false".  The
// per-restart count over the wave's 64 clauses is then one ballot and one
// popcount per restart, accumulated by the lane that owns the restart.
__global__ __launch_bounds__(256) void k_count_unsat(const int32_t* clause_ptr,
                                                     const int32_t* clause_lits,
                                                     const int32_t* chunk_cbeg,
                                                     const int32_t* chunk_cend,
                                                     const uint64_t* bits, int32_t n, int32_t R,
                                                     int32_t* unsat_part) {
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int chunk = blockIdx.x, word = blockIdx.y;
  const int cb = chunk_cbeg[chunk], ce = chunk_cend[chunk];
  const int rem = R - word * 64;
  const uint64_t valid = rem >= 64 ? ~0ULL : ((1ULL << rem) - 1ULL);
  const uint64_t* bw = bits + (int64_t)word * n;
  int cnt = 0;
  for (int base = cb + wv * 64; base < ce; base += 256) {
    const int t = base + lane;
    uint64_t mask = 0;
    if (t < ce) {
      mask = valid;
      for (int p = clause_ptr[t]; p < clause_ptr[t + 1]; ++p) {
        const int code = clause_lits[p];
        const uint64_t b = bw[code >> 1];
        const uint64_t lit_is_true = (code & 1) ? ~b : b;
        mask &= ~lit_is_true;
      }
    }
    for (int j = 0; j < 64; ++j) {
      const uint64_t bal = __ballot((mask >> j) & 1ULL);
      if (lane == j) cnt += __popcll(bal);
    }
  }
  __shared__ int s[256];
  s[threadIdx.x] = cnt;
  __syncthreads();
  if (wv == 0) {
    const int r = word * 64 + lane;
    if (r < R) unsat_part[(int64_t)chunk * R + r] = s[lane] + s[64 + lane] + s[128 + lane] + s[192 + lane];
  }
}

// best[f] = argmin_r unsat[f][r], ties to the lowest r, via the packed key
// (unsat << 32) | r.
__global__ __launch_bounds__(256) void k_best(const int32_t* unsat, int32_t R, int32_t* best) {
  const int f = blockIdx.x;
  uint64_t key = ~0ULL;
  for (int r = threadIdx.x; r < R; r += 256) {
    const uint64_t k = ((uint64_t)(uint32_t)unsat[(int64_t)f * R + r] << 32) | (uint32_t)r;
    key = k < key ? k : key;
  }
  __shared__ uint64_t s[256];
  s[threadIdx.x] = key;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = s[threadIdx.x + w] < s[threadIdx.x] ? s[threadIdx.x + w] : s[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) best[f] = (int32_t)(s[0] & 0xffffffffULL);
}

__global__ void k_best_assign(const uint64_t* bits, int32_t n, const int32_t* var_formula,
                              const int32_t* best, uint8_t* out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int r = best[var_formula[v]];
    out[v] = (uint8_t)((bits[(int64_t)(r >> 6) * n + v] >> (r & 63)) & 1ULL);
  }
}

// ------------------------------------------------------------ launchers

namespace {

template <int LPI, int RPL>
hipError_t var_pass_rpl(const VarPassArgs& a, int mode, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  if (a.stream_items) {
    switch (mode) {
      case kModeSGD: hipLaunchKernelGGL((k_var_stream<LPI, RPL, kModeSGD>), grid, block, 0, s, a); break;
      case kModeAdam: hipLaunchKernelGGL((k_var_stream<LPI, RPL, kModeAdam>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_var_stream<LPI, RPL, kModeGrad>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
  }
  switch (mode) {
    case kModeSGD: hipLaunchKernelGGL((k_var_pass<LPI, RPL, kModeSGD>), grid, block, 0, s, a); break;
    case kModeAdam: hipLaunchKernelGGL((k_var_pass<LPI, RPL, kModeAdam>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_var_pass<LPI, RPL, kModeGrad>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

template <int LPI>
hipError_t var_pass_lpi(const VarPassArgs& a, int mode, Tile t, int chunks, int tiles, hipStream_t s) {
  switch (t.rpl) {
    case 4: return var_pass_rpl<LPI, 4>(a, mode, chunks, tiles, s);
    case 2: return var_pass_rpl<LPI, 2>(a, mode, chunks, tiles, s);
    default: return var_pass_rpl<LPI, 1>(a, mode, chunks, tiles, s);
  }
}

template <int LPI, int RPL>
hipError_t var_seg_rpl(const VarPassArgs& a, int chunks, int tiles, hipStream_t s) {
  hipLaunchKernelGGL((k_var_seg<LPI, RPL>), dim3(chunks, tiles), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int LPI>
hipError_t var_seg_lpi(const VarPassArgs& a, Tile t, int chunks, int tiles, hipStream_t s) {
  switch (t.rpl) {
    case 4: return var_seg_rpl<LPI, 4>(a, chunks, tiles, s);
    case 2: return var_seg_rpl<LPI, 2>(a, chunks, tiles, s);
    default: return var_seg_rpl<LPI, 1>(a, chunks, tiles, s);
  }
}

template <int LPI, int RPL>
hipError_t heavy_rpl(const VarPassArgs& a, int mode, int h0, int h1, int tiles, hipStream_t s) {
  constexpr int IPB = kBlock / LPI;
  int blocks = (h1 - h0 + IPB - 1) / IPB;
  blocks = blocks > 4096 ? 4096 : blocks;
  dim3 grid(blocks, tiles), block(kBlock);
  switch (mode) {
    case kModeSGD: hipLaunchKernelGGL((k_heavy_finish<LPI, RPL, kModeSGD>), grid, block, 0, s, a, h0, h1); break;
    case kModeAdam: hipLaunchKernelGGL((k_heavy_finish<LPI, RPL, kModeAdam>), grid, block, 0, s, a, h0, h1); break;
    default: hipLaunchKernelGGL((k_heavy_finish<LPI, RPL, kModeGrad>), grid, block, 0, s, a, h0, h1); break;
  }
  return hipGetLastError();
}

template <int LPI>
hipError_t heavy_lpi(const VarPassArgs& a, int mode, Tile t, int h0, int h1, int tiles, hipStream_t s) {
  switch (t.rpl) {
    case 4: return heavy_rpl<LPI, 4>(a, mode, h0, h1, tiles, s);
    case 2: return heavy_rpl<LPI, 2>(a, mode, h0, h1, tiles, s);
    default: return heavy_rpl<LPI, 1>(a, mode, h0, h1, tiles, s);
  }
}

template <int LPI, int RPL>
hipError_t clause_pass_rpl(const ClausePassArgs& a, bool write_d, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  if (write_d) hipLaunchKernelGGL((k_clause_pass<LPI, RPL, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_clause_pass<LPI, RPL, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int LPI>
hipError_t clause_pass_lpi(const ClausePassArgs& a, bool write_d, Tile t, int chunks, int tiles,
                           hipStream_t s) {
  switch (t.rpl) {
    case 4: return clause_pass_rpl<LPI, 4>(a, write_d, chunks, tiles, s);
    case 2: return clause_pass_rpl<LPI, 2>(a, write_d, chunks, tiles, s);
    default: return clause_pass_rpl<LPI, 1>(a, write_d, chunks, tiles, s);
  }
}

inline int grid_x_for(int64_t items_div4) {
  int64_t g = items_div4 < 1 ? 1 : items_div4;
  return (int)(g > 65536 ? 65536 : g);
}

}  // namespace

// Restart tiles of one launch: [tile_base, tile_base + tile_count), or all.
template <class Args>
inline int launch_tiles(const Args& a, Tile t) {
  const int all = (a.R + t.tile() - 1) / t.tile() - a.tile_base;
  return a.tile_count > 0 && a.tile_count < all ? a.tile_count : all;
}

hipError_t launch_var_pass(const VarPassArgs& a, int mode, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return var_pass_lpi<4>(a, mode, t, chunks, tiles, s);
    case 8: return var_pass_lpi<8>(a, mode, t, chunks, tiles, s);
    case 16: return var_pass_lpi<16>(a, mode, t, chunks, tiles, s);
    case 32: return var_pass_lpi<32>(a, mode, t, chunks, tiles, s);
    default: return var_pass_lpi<64>(a, mode, t, chunks, tiles, s);
  }
}

hipError_t launch_var_seg(const VarPassArgs& a, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return var_seg_lpi<4>(a, t, chunks, tiles, s);
    case 8: return var_seg_lpi<8>(a, t, chunks, tiles, s);
    case 16: return var_seg_lpi<16>(a, t, chunks, tiles, s);
    case 32: return var_seg_lpi<32>(a, t, chunks, tiles, s);
    default: return var_seg_lpi<64>(a, t, chunks, tiles, s);
  }
}

hipError_t launch_heavy_finish(const VarPassArgs& a, int mode, Tile t, int h0, int h1,
                               hipStream_t s) {
  if (h1 <= h0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return heavy_lpi<4>(a, mode, t, h0, h1, tiles, s);
    case 8: return heavy_lpi<8>(a, mode, t, h0, h1, tiles, s);
    case 16: return heavy_lpi<16>(a, mode, t, h0, h1, tiles, s);
    case 32: return heavy_lpi<32>(a, mode, t, h0, h1, tiles, s);
    default: return heavy_lpi<64>(a, mode, t, h0, h1, tiles, s);
  }
}

template <int LPI, int RPL>
hipError_t occ_rpl(const VarPassArgs& a, int chunks, int tiles, hipStream_t s) {
  hipLaunchKernelGGL((k_occ_pass<LPI, RPL>), dim3(chunks, tiles), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int LPI, int RPL>
hipError_t vsum_rpl(const VarPassArgs& a, int mode, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  switch (mode) {
    case kModeSGD: hipLaunchKernelGGL((k_var_sum<LPI, RPL, kModeSGD>), grid, block, 0, s, a); break;
    case kModeAdam: hipLaunchKernelGGL((k_var_sum<LPI, RPL, kModeAdam>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_var_sum<LPI, RPL, kModeGrad>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

template <int LPI, int RPL>
hipError_t ssum_rpl(const VarPassArgs& a, int chunks, int tiles, hipStream_t s) {
  hipLaunchKernelGGL((k_seg_sum<LPI, RPL>), dim3(chunks, tiles), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Dispatch over the runtime (lpi, rpl) of a tile to a template instance.
#define GALSAT_TILE_DISPATCH(FN, t, ...)                                             \
  switch ((t).lpi * 8 + (t).rpl) {                                                   \
    case 4 * 8 + 1: return FN<4, 1>(__VA_ARGS__);                                    \
    case 4 * 8 + 2: return FN<4, 2>(__VA_ARGS__);                                    \
    case 4 * 8 + 4: return FN<4, 4>(__VA_ARGS__);                                    \
    case 8 * 8 + 1: return FN<8, 1>(__VA_ARGS__);                                    \
    case 8 * 8 + 2: return FN<8, 2>(__VA_ARGS__);                                    \
    case 8 * 8 + 4: return FN<8, 4>(__VA_ARGS__);                                    \
    case 16 * 8 + 1: return FN<16, 1>(__VA_ARGS__);                                  \
    case 16 * 8 + 2: return FN<16, 2>(__VA_ARGS__);                                  \
    case 16 * 8 + 4: return FN<16, 4>(__VA_ARGS__);                                  \
    case 32 * 8 + 1: return FN<32, 1>(__VA_ARGS__);                                  \
    case 32 * 8 + 2: return FN<32, 2>(__VA_ARGS__);                                  \
    case 32 * 8 + 4: return FN<32, 4>(__VA_ARGS__);                                  \
    case 64 * 8 + 2: return FN<64, 2>(__VA_ARGS__);                                  \
    case 64 * 8 + 4: return FN<64, 4>(__VA_ARGS__);                                  \
    default: return FN<64, 1>(__VA_ARGS__);                                          \
  }

hipError_t launch_occ_pass(const VarPassArgs& a, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  GALSAT_TILE_DISPATCH(occ_rpl, t, a, chunks, tiles, s)
}

hipError_t launch_var_sum(const VarPassArgs& a, int mode, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  GALSAT_TILE_DISPATCH(vsum_rpl, t, a, mode, chunks, tiles, s)
}

hipError_t launch_seg_sum(const VarPassArgs& a, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  GALSAT_TILE_DISPATCH(ssum_rpl, t, a, chunks, tiles, s)
}

hipError_t launch_clause_pass(const ClausePassArgs& a, bool write_d, Tile t, int chunks,
                              hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return clause_pass_lpi<4>(a, write_d, t, chunks, tiles, s);
    case 8: return clause_pass_lpi<8>(a, write_d, t, chunks, tiles, s);
    case 16: return clause_pass_lpi<16>(a, write_d, t, chunks, tiles, s);
    case 32: return clause_pass_lpi<32>(a, write_d, t, chunks, tiles, s);
    default: return clause_pass_lpi<64>(a, write_d, t, chunks, tiles, s);
  }
}

hipError_t launch_finalize(const FinalizeArgs& a, int F, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  dim3 grid(F, (a.R + 63) / 64);
  // few large formulas: more waves per formula; many small ones: fewer
  if ((int64_t)F * grid.y < 256)
    hipLaunchKernelGGL((k_finalize<16>), grid, dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((k_finalize<4>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_state(float* x, int32_t ldx, int32_t n, int32_t R, uint64_t seed,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_init_state, grid, block, 0, s, x, ldx, n, R, seed);
  return hipGetLastError();
}

hipError_t launch_copy_state(const float* src, int32_t lds, float* dst, int32_t ldd, int32_t n,
                             int32_t R, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int gy = (R + 63) / 64 > 64 ? 64 : (R + 63) / 64;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), gy), block(256);
  hipLaunchKernelGGL(k_copy_state, grid, block, 0, s, src, lds, dst, ldd, n, R);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_x_for((count + 255) / 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_pack_bits(const float* x, int32_t ldx, int32_t n, int32_t R, uint64_t* bits,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_pack_bits, grid, block, 0, s, x, ldx, n, R, bits);
  return hipGetLastError();
}

hipError_t launch_count_unsat(const int32_t* clause_ptr, const int32_t* clause_lits,
                              const int32_t* chunk_cbeg, const int32_t* chunk_cend, int chunks,
                              const uint64_t* bits, int32_t n, int32_t R, int32_t* unsat_part,
                              hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  dim3 grid(chunks, (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_count_unsat, grid, block, 0, s, clause_ptr, clause_lits, chunk_cbeg,
                     chunk_cend, bits, n, R, unsat_part);
  return hipGetLastError();
}

hipError_t launch_gumbel_noise(float* out, int32_t ldo, int32_t n, int32_t R, uint64_t seed,
                               int32_t t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_gumbel_noise, grid, block, 0, s, out, ldo, n, R, seed, t);
  return hipGetLastError();
}

hipError_t launch_gumbel_prep(const float* d, int32_t ldd, const float* noise, int32_t ldn,
                              uint64_t seed, int32_t t, int32_t n, int32_t R, float* xh, float* nb,
                              int32_t ld, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_gumbel_prep, grid, block, 0, s, d, ldd, noise, ldn, seed, t, n, R, xh, nb, ld);
  return hipGetLastError();
}

hipError_t launch_gumbel_update(float* d, int32_t ldd, const float* nb, const float* G, int32_t ld,
                                float* mom, float* vel, int32_t ldm, int32_t n, int32_t R, float tau,
                                float lr, float b1, float b2, float eps, double inv_c1,
                                double inv_c2, int32_t adam, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_gumbel_update, grid, block, 0, s, d, ldd, nb, G, ld, mom, vel, ldm, n, R, tau,
                     lr, b1, b2, eps, inv_c1, inv_c2, adam);
  return hipGetLastError();
}

hipError_t launch_candidates(const float* d, int32_t ldd, const int32_t* var_formula,
                             const int32_t* best, int32_t n, int32_t num, uint64_t seed, float tau,
                             uint8_t* assign, float* conf, hipStream_t s) {
  if (n <= 0 || num <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 255) / 256), num), block(256);
  hipLaunchKernelGGL(k_candidates, grid, block, 0, s, d, ldd, var_formula, best, n, seed, tau, assign,
                     conf);
  return hipGetLastError();
}

hipError_t launch_confidence(const float* d, int32_t ldd, const int32_t* var_formula,
                             const int32_t* best, int32_t n, float tau, float* conf, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_confidence, dim3(grid_x_for(((int64_t)n + 255) / 256)), dim3(256), 0, s, d,
                     ldd, var_formula, best, n, tau, conf);
  return hipGetLastError();
}

hipError_t launch_select(const float* conf, int32_t n, int32_t F, const int32_t* f_vbeg,
                         const int32_t* sel_off, int32_t stot, int32_t num, bool highest,
                         int32_t* out, hipStream_t s) {
  if (F <= 0 || num <= 0 || stot <= 0) return hipSuccess;
  dim3 grid(F, num), block(1024);
  if (highest)
    hipLaunchKernelGGL((k_select<true>), grid, block, 0, s, conf, n, f_vbeg, sel_off, stot, out);
  else
    hipLaunchKernelGGL((k_select<false>), grid, block, 0, s, conf, n, f_vbeg, sel_off, stot, out);
  return hipGetLastError();
}

hipError_t launch_best(const int32_t* unsat, int32_t F, int32_t R, int32_t* best, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best, dim3(F), dim3(256), 0, s, unsat, R, best);
  return hipGetLastError();
}

hipError_t launch_best_assign(const uint64_t* bits, int32_t n, const int32_t* var_formula,
                              const int32_t* best, uint8_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best_assign, dim3(grid_x_for(((int64_t)n + 255) / 256)), dim3(256), 0, s,
                     bits, n, var_formula, best, out);
  return hipGetLastError();
}

}  // namespace galsat
