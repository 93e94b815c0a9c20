// Flat single pass of the general schedule (gfx950).
//
// The gradient of loss' = sum_t U_t, U_t = prod_i a_{t,i} (Section 3.2,
// Eq. 2 with the negation of Eq. 1, summed as in Eq. 5) needs, for every
// literal occurrence (t, j), the product of the clause's other factors.
// This plan obtains it two ways, chosen per clause by its length:
//
//  * 3-literal clauses: the variable pass recomputes the two other factors
//    from x ("pair records": the two other literal codes, relative to the
//    formula's first variable).  Nothing is stored between passes.
//  * every other clause: a row pass first reduces the clause, per restart,
//    to the FP64 product Q of its nonzero factors and the number of its
//    factors that are exactly zero, packed in 32 bits ("clause rows").  The
//    variable pass then forms each occurrence's partial without recomputing
//    the clause:  zero count 0 -> Q / a_own;  count 1 -> Q when the own
//    factor is the zero one, else 0;  count >= 2 -> 0.  Exact zeros (clamped
//    states) therefore need no special case in the arithmetic, and a clause
//    of k literals costs k gathers in the row pass plus one row gather per
//    occurrence, instead of k (k - 1) gathers (recomputing) or a stored row
//    per literal (prefix and suffix products).
//
// Packed clause value (32 bits): bit 31 is set when exactly one factor is
// zero; bits 0..30 hold the top 31 bits of the FP64 value (sign, the full
// 11-bit exponent and 19 mantissa bits, rounded to nearest), so any FP64
// product keeps its range and a relative precision of 2^-20; a clause with
// two or more zero factors stores 0.  The product is formed with its
// binary exponent carried separately (renormalised every four factors), so
// factors outside [0, 1] (states that loss_grad accepts) cannot overflow or
// underflow it midway.
//
// Sums run in a fixed order, so results are bitwise reproducible: per
// variable the first-literal pairs (positive own literals, then negated),
// then the other pairs, each in variable-major slot order, then the clause
// rows (positive, then negated), each in row order, accumulated in FP64.
#include "galsat_device.h"

namespace galsat {

namespace {

constexpr float kHalf = 0.5f;
constexpr float kHalfUp = 0.50000006f;  // the float after 0.5 (0.5 + 2^-24)

// A literal is false under rounding (x_hat = [x > 0.5], ties to 0) exactly
// when its factor f = 1 - s satisfies f >= 0.5 (positive literal: f = 1 - x
// is exact for x >= 0.5) or f > 0.5, i.e. f >= 0.5 + 2^-24 (negated
// literal: f = x).  The margin f - theta is >= 0 exactly when the literal
// is false; the clause is unsatisfied when the smallest margin is >= 0.
__device__ __forceinline__ float false_margin(int code, float f) {
  return f - ((code & 1) ? kHalfUp : kHalf);
}

__device__ __forceinline__ uint32_t clause_pack(double q, int zeros) {
  if (zeros >= 2) return 0u;
  uint64_t b = (uint64_t)__double_as_longlong(q);
  b += (uint64_t)1 << 32;  // round to nearest on the 33 dropped bits
  return (uint32_t)(b >> 33) | (zeros == 1 ? 0x80000000u : 0u);
}

template <int N>
__device__ __forceinline__ void load_urow(const uint32_t* __restrict__ p, uint32_t (&o)[N]) {
  if constexpr (N == 4) {
    const uint4 t = *reinterpret_cast<const uint4*>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else if constexpr (N == 2) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);
    o[0] = t.x; o[1] = t.y;
  } else {
    o[0] = p[0];
  }
}

template <int N>
__device__ __forceinline__ void store_urow(uint32_t* __restrict__ p, const uint32_t (&o)[N]) {
  if constexpr (N == 4) {
    *reinterpret_cast<uint4*>(p) = make_uint4(o[0], o[1], o[2], o[3]);
  } else if constexpr (N == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(o[0], o[1]);
  } else {
    p[0] = o[0];
  }
}

}  // namespace

// Byte offset of row idx (a formula-local index, below 2^24) at the given
// row stride, plus a column offset: one 24-bit multiply-add.
__device__ __forceinline__ uint32_t row_off(uint32_t idx, uint32_t stride_bytes, uint32_t col_bytes) {
  return __umul24(idx, stride_bytes) + col_bytes;
}

// ---------------------------------------------------------------- row pass
//
// One item per clause of the row list (every clause that is not 3 literals
// long, longest first within a formula), LPI lanes x RPL restarts: the
// clause's packed value per restart, and its U_t and unsat into the chunk's
// partial rows.
template <int LPI, int RPL>
__global__ __launch_bounds__(kBlock) void k_row_clause(ClausePassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  constexpr int B = 8;  // literals gathered per batch
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk =
      a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x) : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  const int cb = ldc(a.chunk_cbeg, chunk), ce = ldc(a.chunk_cend, chunk);
  // the chunk's clauses belong to one formula: rows by 32-bit offsets from
  // its first state row
  const char* xb = reinterpret_cast<const char*>(a.x + (int64_t)ldc(a.chunk_fvb, chunk) * a.ldx);
  const uint32_t ldx4 = (uint32_t)a.ldx * 4u, rc4 = (uint32_t)rc * 4u;
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  for (int i0 = cb + slot; i0 < ce; i0 += IPB) {
    const int i = uniform<LPI>(i0);
    const int ps = ldc(a.rlit_ptr, i), pe = ldc(a.rlit_ptr, i + 1);
    double qm[RPL];
    int qe[RPL], zeros[RPL];
    float mind[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) { qm[j] = 1.0; qe[j] = 0; zeros[j] = 0; mind[j] = __builtin_huge_valf(); }
    for (int p = ps; p < pe; p += B) {
      int codes[B];
      float y[B][RPL];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int pu = p + u < pe ? p + u : pe - 1;  // in bounds; masked below
        codes[u] = ldc(a.rlits, pu);
        load_row<RPL>(reinterpret_cast<const float*>(xb + row_off((uint32_t)codes[u] >> 1, ldx4, rc4)),
                      y[u]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        // the factor as one FMA, f = fma(y, sg, sb) (as in the pair loop);
        // a slot past the clause gets sg = 0, sb = 1, the factor exactly 1,
        // which leaves the product and the zero count unchanged, and the
        // margin 1 - 0.5 >= 0, which never decides the sign of the smallest
        // margin
        const bool use = p + u < pe;
        const bool neg = use && (codes[u] & 1) != 0;
        const float sg = use ? (neg ? 1.0f : -1.0f) : 0.0f;
        const float sb = neg ? 0.0f : 1.0f;
        const float th = neg ? kHalfUp : kHalf;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const float f = fmaf(y[u][j], sg, sb);
          const bool zero = f == 0.0f;
          zeros[j] += zero ? 1 : 0;
          qm[j] *= (double)(zero ? 1.0f : f);
          mind[j] = fminf(mind[j], f - th);
        }
        if (u % 4 == 3) {
          // at most four factors since the last renormalisation: |qm| stays
          // within [2^-597, 2^517], inside FP64's normal range
#pragma unroll
          for (int j = 0; j < RPL; ++j) {
            int e = 0;
            qm[j] = frexp(qm[j], &e);
            qe[j] += e;
          }
        }
      }
    }
    uint32_t packed[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const double q = ldexp(qm[j], qe[j]);
      packed[j] = clause_pack(q, zeros[j]);
      lsum[j] += zeros[j] ? 0.0 : q;
      usum[j] += mind[j] >= 0.0f ? 1 : 0;
    }
    if (active) store_urow<RPL>(a.qrow + (int64_t)i * a.ldq + r0, packed);
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row ? a.chunk_row[chunk] : chunk, tile, a.R,
                           a.loss_part, a.unsat_part);
}

// ------------------------------------------------------------ variable side
//
// Rows are addressed by 32-bit byte offsets from the base of their formula
// (the plan keeps a formula's state and clause rows below 4 GiB and its
// local indices below 2^24), so each gather costs one 24-bit multiply-add
// and the load takes its base from scalar registers.  Record streams are
// read once per step and are loaded non-temporally, and so is the next
// state stored, so the gathered rows keep the L2.

// Pair records of [b, e) (consecutive pair slots of one variable), four at a
// time with all eight row gathers in flight.  A literal's factor is one FMA,
// fma(y, +1, 0) = y for a negated literal and fma(y, -1, 1) = 1 - y for a
// positive one (each rounded once, as 1 - y is).  The four contributions are
// summed in FP32 and that sum is added to the FP64 accumulator; a record
// past the end has weight 0.  The own literal's sign is the first code's
// bit 31.  FIRST: the own literal is its clause's first, so the occurrence
// also accounts for U_t = a_own * f1 * f2 and the clause's rounded
// satisfaction: unsatisfied when all three literals are false, a literal
// being false when f >= 0.5 (positive) or f > 0.5, i.e. f >= 0.5 + 2^-24
// (negated).
template <int RPL, bool FIRST, bool PF>
__device__ __forceinline__ void flat_pairs(const VarPassArgs& a, const char* xb, uint32_t ldx4,
                                           uint32_t rc4, int b, int e, const float (&ap)[RPL],
                                           const float (&an)[RPL], double (&g)[RPL],
                                           double (&lsum)[RPL], int (&usum)[RPL]) {
  if (b >= e) return;
  bool fp[RPL], fn[RPL];  // own literal false (first-literal loop only)
  if constexpr (FIRST) {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      fp[j] = ap[j] >= kHalf;
      fn[j] = an[j] >= kHalfUp;
    }
  }
  const long long* pr = reinterpret_cast<const long long*>(a.pairs);
  // PF: records of the next batch are loaded while this batch's gathers are
  // in flight (indices clamped into [b, e), so every load stays in bounds)
  long long nxt[4];
  if constexpr (PF) {
#pragma unroll
    for (int k = 0; k < 4; ++k) nxt[k] = __builtin_nontemporal_load(pr + (b + k < e ? b + k : e - 1));
  }
  for (int q = b; q < e; q += 4) {
    uint32_t c1[4], c2[4];
    float y[4][2][RPL];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (!PF) nxt[k] = __builtin_nontemporal_load(pr + (q + k < e ? q + k : e - 1));
      c1[k] = (uint32_t)nxt[k];
      c2[k] = (uint32_t)((unsigned long long)nxt[k] >> 32);
      load_row<RPL>(reinterpret_cast<const float*>(xb + row_off((c1[k] & 0x7fffffffu) >> 1, ldx4, rc4)),
                    y[k][0]);
      load_row<RPL>(reinterpret_cast<const float*>(xb + row_off(c2[k] >> 1, ldx4, rc4)), y[k][1]);
    }
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        nxt[k] = __builtin_nontemporal_load(pr + (q + 4 + k < e ? q + 4 + k : e - 1));
    }
    // every gather of the batch is issued before any of them is used
    __builtin_amdgcn_sched_barrier(0);
    float tg[RPL], tl[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) { tg[j] = 0.0f; tl[j] = 0.0f; }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool use = q + k < e;
      const bool own_neg = (c1[k] >> 31) != 0;
      const bool n1 = (c1[k] & 1) != 0, n2 = (c2[k] & 1) != 0;
      const float sg1 = n1 ? 1.0f : -1.0f, sb1 = n1 ? 0.0f : 1.0f;
      const float sg2 = n2 ? 1.0f : -1.0f, sb2 = n2 ? 0.0f : 1.0f;
      const float w = use ? (own_neg ? 1.0f : -1.0f) : 0.0f;
      const float th1 = n1 ? kHalfUp : kHalf, th2 = n2 ? kHalfUp : kHalf;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const float f1 = fmaf(y[k][0][j], sg1, sb1), f2 = fmaf(y[k][1][j], sg2, sb2);
        const float p = f1 * f2;
        tg[j] = fmaf(w, p, tg[j]);
        if constexpr (FIRST) {
          const float ao = own_neg ? an[j] : ap[j];
          tl[j] = fmaf(use ? 1.0f : 0.0f, ao * p, tl[j]);
          const bool own_false = own_neg ? fn[j] : fp[j];
          usum[j] += (use && own_false && f1 >= th1 && f2 >= th2) ? 1 : 0;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      g[j] += (double)tg[j];
      if constexpr (FIRST) lsum[j] += (double)tl[j];
    }
  }
}

// 1/a in FP64 for a nonzero FP32 factor a (always a normal FP64 number):
// the hardware reciprocal refined by two Newton steps, far below the
// FP32 rounding of the final gradient.
__device__ __forceinline__ double recip64(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(fma(-a, r, 1.0), r, r);
  return fma(fma(-a, r, 1.0), r, r);
}

// Clause-row records of [b, e): record = row within the formula; records
// before m belong to positive own literals, the rest to negated ones (the
// plan keeps a variable's positive-literal rows first).  With a the own
// factor, the partial is Q / a when the clause has no zero factor, Q when a
// is its only zero, and 0 otherwise; dU/dx_v carries the sign s (-1 for a
// positive own literal, +1 for a negated one), folded into the inverse.  A
// zero own factor with the one-zero flag clear means two or more zeros,
// whose stored Q is 0, so only "flag set and own factor nonzero" needs
// masking.
template <int RPL, bool PF>
__device__ __forceinline__ void flat_rows(const VarPassArgs& a, const char* qb, uint32_t ldq4,
                                          uint32_t rc4, int b, int m, int e,
                                          const float (&ap)[RPL], const float (&an)[RPL],
                                          double (&g)[RPL]) {
  if (b >= e) return;
  double inv_p[RPL], inv_n[RPL];
  uint32_t nz_p[RPL], nz_n[RPL];  // all ones when the own factor is nonzero
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const bool zp = ap[j] == 0.0f, zn = an[j] == 0.0f;
    nz_p[j] = zp ? 0u : ~0u;
    nz_n[j] = zn ? 0u : ~0u;
    inv_p[j] = zp ? -1.0 : -recip64((double)ap[j]);
    inv_n[j] = zn ? 1.0 : recip64((double)an[j]);
  }
  constexpr int B = 4;
  uint32_t nxt[B];  // PF: records of the next batch, loaded during this one's gathers
  if constexpr (PF) {
#pragma unroll
    for (int k = 0; k < B; ++k) nxt[k] = __builtin_nontemporal_load(a.lrec + (b + k < e ? b + k : e - 1));
  }
  for (int q = b; q < e; q += B) {
    uint32_t rec[B];
    uint32_t u[B][RPL];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      if constexpr (!PF) nxt[k] = __builtin_nontemporal_load(a.lrec + (q + k < e ? q + k : e - 1));
      rec[k] = nxt[k];
      load_urow<RPL>(reinterpret_cast<const uint32_t*>(qb + row_off(rec[k], ldq4, rc4)), u[k]);
    }
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < B; ++k)
        nxt[k] = __builtin_nontemporal_load(a.lrec + (q + B + k < e ? q + B + k : e - 1));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const uint32_t keep = q + k < e ? ~0u : 0u;
      const bool own_neg = q + k >= m;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        // high word of the FP64 value: the 31 stored bits shifted past the
        // flag; cleared when masked (the low word is always 0)
        const uint32_t skip = (uint32_t)((int32_t)u[k][j] >> 31) & (own_neg ? nz_n[j] : nz_p[j]);
        const uint32_t hi = (u[k][j] << 1) & ~skip & keep;
        g[j] = fma(__hiloint2double((int)hi, 0), own_neg ? inv_n[j] : inv_p[j], g[j]);
      }
    }
  }
}

// Unified index range [u0, u1) of variable v's contributions: first-literal
// pairs (positive own literal, then negated), the other pairs, then clause
// rows (positive, then negated): together exactly one entry per occurrence
// of v.  xb, qb: the bases of v's
// formula's state rows and clause rows.
template <int RPL, bool PF>
__device__ __forceinline__ void flat_range(const VarPassArgs& a, const char* xb, const char* qb,
                                           int v, int u0, int u1, int rc, const float (&xv)[RPL],
                                           double (&g)[RPL], double (&lsum)[RPL],
                                           int (&usum)[RPL]) {
  const uint32_t ldx4 = (uint32_t)a.ldx * 4u, ldq4 = (uint32_t)a.ldq * 4u, rc4 = (uint32_t)rc * 4u;
  float ap[RPL], an[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    ap[j] = 1.0f - xv[j];
    an[j] = xv[j];
  }
  const int pf = ldc(a.pair_first, v), pm = ldc(a.pair_mid, v), pz = ldc(a.pair_end, v);
  const int lb = ldc(a.lrec_ptr, v), lm = ldc(a.lrec_mid, v), lz = ldc(a.lrec_end, v);
  const int nf = pm - pf, np = pz - pf, nl = lz - lb;
  flat_pairs<RPL, true, PF>(a, xb, ldx4, rc4, pf + max(u0, 0), pf + min(u1, nf), ap, an, g, lsum,
                            usum);
  flat_pairs<RPL, false, PF>(a, xb, ldx4, rc4, pf + max(u0, nf), pf + min(u1, np), ap, an, g, lsum,
                             usum);
  flat_rows<RPL, PF>(a, qb, ldq4, rc4, lb + max(u0 - np, 0), lm, lb + min(u1 - np, nl), ap, an, g);
}

// Whole variables of the chunk's range: the gradient, then the epilogue.
template <int LPI, int RPL, int MODE, bool PF>
__global__ __launch_bounds__(kBlock) void k_flat_var(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int chunk = a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x)
                                  : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;  // in-bounds column for lanes past the last restart
  const int vb = ldc(a.chunk_vbeg, chunk), ve = ldc(a.chunk_vend, chunk);
  const char* xb = reinterpret_cast<const char*>(a.x + (int64_t)ldc(a.chunk_fvb, chunk) * a.ldx);
  const char* qb = reinterpret_cast<const char*>(a.qrow + (int64_t)ldc(a.chunk_rbase, chunk) * a.ldq);
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
    flat_range<RPL, PF>(a, xb, qb, v, 0, 0x7fffffff, rc, xv, g, lsum, usum);
    if (active) var_epilogue<RPL, MODE, true>(a, v, r0, xv, g);
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// Segments of split variables: each segment's partial gradient (its
// unified range [seg_q0 - var_ptr[v], seg_q1 - var_ptr[v])) goes to
// gseg[s][r] in FP64; k_heavy_finish adds them in segment order.
template <int LPI, int RPL, bool PF>
__global__ __launch_bounds__(kBlock) void k_flat_seg(VarPassArgs a) {
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
    const int sgi = uniform<LPI>(ldc(a.seg_perm, s0));
    const int v = ldc(a.seg_var, sgi);
    const int qv = ldc(a.var_ptr, v);
    const int f = ldc(a.var_formula, v);
    const char* xb = reinterpret_cast<const char*>(a.x + (int64_t)ldc(a.f_vbeg, f) * a.ldx);
    const char* qb = reinterpret_cast<const char*>(a.qrow + (int64_t)ldc(a.f_rbeg, f) * a.ldq);
    double g[RPL];
    float xv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    load_row<RPL>(a.x + (int64_t)v * a.ldx + rc, xv);
    flat_range<RPL, PF>(a, xb, qb, v, ldc(a.seg_q0, sgi) - qv, ldc(a.seg_q1, sgi) - qv, rc, xv, g,
                        lsum, usum);
    if (active) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) a.gseg[(int64_t)sgi * a.R + r0 + j] = g[j];
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// ------------------------------------------------------------ launchers

namespace {

template <int LPI, int RPL, bool PF>
hipError_t flat_var_pf(const VarPassArgs& a, int mode, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  switch (mode) {
    case kModeSGD: hipLaunchKernelGGL((k_flat_var<LPI, RPL, kModeSGD, PF>), grid, block, 0, s, a); break;
    case kModeAdam: hipLaunchKernelGGL((k_flat_var<LPI, RPL, kModeAdam, PF>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_flat_var<LPI, RPL, kModeGrad, PF>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

template <int LPI, int RPL>
hipError_t flat_var_rpl(const VarPassArgs& a, int mode, int chunks, int tiles, hipStream_t s) {
  return a.prefetch ? flat_var_pf<LPI, RPL, true>(a, mode, chunks, tiles, s)
                    : flat_var_pf<LPI, RPL, false>(a, mode, chunks, tiles, s);
}

template <int LPI>
hipError_t flat_var_lpi(const VarPassArgs& a, int mode, Tile t, int chunks, int tiles,
                        hipStream_t s) {
  switch (t.rpl) {
    case 4: return flat_var_rpl<LPI, 4>(a, mode, chunks, tiles, s);
    case 2: return flat_var_rpl<LPI, 2>(a, mode, chunks, tiles, s);
    default: return flat_var_rpl<LPI, 1>(a, mode, chunks, tiles, s);
  }
}

template <int LPI>
hipError_t flat_seg_lpi(const VarPassArgs& a, Tile t, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  if (a.prefetch) {
    switch (t.rpl) {
      case 4: hipLaunchKernelGGL((k_flat_seg<LPI, 4, true>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_flat_seg<LPI, 2, true>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_flat_seg<LPI, 1, true>), grid, block, 0, s, a); break;
    }
  } else {
    switch (t.rpl) {
      case 4: hipLaunchKernelGGL((k_flat_seg<LPI, 4, false>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_flat_seg<LPI, 2, false>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_flat_seg<LPI, 1, false>), grid, block, 0, s, a); break;
    }
  }
  return hipGetLastError();
}

template <int LPI>
hipError_t row_clause_lpi(const ClausePassArgs& a, Tile t, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  switch (t.rpl) {
    case 4: hipLaunchKernelGGL((k_row_clause<LPI, 4>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_row_clause<LPI, 2>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_row_clause<LPI, 1>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_flat_var(const VarPassArgs& a, int mode, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return flat_var_lpi<4>(a, mode, t, chunks, tiles, s);
    case 8: return flat_var_lpi<8>(a, mode, t, chunks, tiles, s);
    case 16: return flat_var_lpi<16>(a, mode, t, chunks, tiles, s);
    case 32: return flat_var_lpi<32>(a, mode, t, chunks, tiles, s);
    default: return flat_var_lpi<64>(a, mode, t, chunks, tiles, s);
  }
}

hipError_t launch_flat_seg(const VarPassArgs& a, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return flat_seg_lpi<4>(a, t, chunks, tiles, s);
    case 8: return flat_seg_lpi<8>(a, t, chunks, tiles, s);
    case 16: return flat_seg_lpi<16>(a, t, chunks, tiles, s);
    case 32: return flat_seg_lpi<32>(a, t, chunks, tiles, s);
    default: return flat_seg_lpi<64>(a, t, chunks, tiles, s);
  }
}

hipError_t launch_row_clause(const ClausePassArgs& a, Tile t, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  const int tiles = launch_tiles(a, t);
  switch (t.lpi) {
    case 4: return row_clause_lpi<4>(a, t, chunks, tiles, s);
    case 8: return row_clause_lpi<8>(a, t, chunks, tiles, s);
    case 16: return row_clause_lpi<16>(a, t, chunks, tiles, s);
    case 32: return row_clause_lpi<32>(a, t, chunks, tiles, s);
    default: return row_clause_lpi<64>(a, t, chunks, tiles, s);
  }
}

}  // namespace galsat
