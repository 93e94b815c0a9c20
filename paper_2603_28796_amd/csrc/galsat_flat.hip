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
// variable the first-literal pairs, then the other pairs, then the clause
// rows, each in variable-major slot order, accumulated in FP64.
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

__device__ __forceinline__ double clause_value(uint32_t u) {
  return __longlong_as_double((long long)((uint64_t)(u & 0x7fffffffu) << 33));
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

// Row of a formula-local literal code: the formula's rows start at xb.
template <int RPL>
__device__ __forceinline__ void load_local(const float* xb, int32_t ldx, int code, int rc,
                                           float (&o)[RPL]) {
  load_row<RPL>(xb + (int64_t)((uint32_t)code >> 1) * ldx + rc, o);
}

}  // namespace

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
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  for (int i0 = cb + slot; i0 < ce; i0 += IPB) {
    const int i = uniform<LPI>(i0);
    const int t = ldc(a.clause_ids, i);
    const int ps = ldc(a.clause_ptr, t), pe = ldc(a.clause_ptr, t + 1);
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
        codes[u] = ldc(a.clause_lits, pu);
        load_row<RPL>(a.x + (int64_t)(codes[u] >> 1) * a.ldx + rc, y[u]);
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const bool use = p + u < pe;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const float f = lit_factor(codes[u], y[u][j]);
          const bool zero = f == 0.0f;
          zeros[j] += (use && zero) ? 1 : 0;
          qm[j] *= (use && !zero) ? (double)f : 1.0;
          mind[j] = use ? fminf(mind[j], false_margin(codes[u], f)) : mind[j];
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

// Pair records of [b, e) (consecutive pair slots of one variable), four at a
// time with all eight row gathers in flight.  FIRST: the own literal is its
// clause's first, so the occurrence also accounts for U_t = a_own * f1 * f2
// and the clause's rounded satisfaction.
template <int RPL, bool FIRST>
__device__ __forceinline__ void flat_pairs(const VarPassArgs& a, const float* xb, int b, int e,
                                           int rc, const float (&xv)[RPL], double (&g)[RPL],
                                           double (&lsum)[RPL], int (&usum)[RPL]) {
  for (int q = b; q < e; q += 4) {
    int2 rec[4];
    float y[4][2][RPL];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int qk = q + k < e ? q + k : e - 1;  // in bounds; masked below
      const int32_t* rp = reinterpret_cast<const int32_t*>(a.pairs) + 2 * (int64_t)qk;
      rec[k] = make_int2(ldc(rp, 0), ldc(rp, 1));
      load_local<RPL>(xb, a.ldx, rec[k].x & 0x7fffffff, rc, y[k][0]);
      load_local<RPL>(xb, a.ldx, rec[k].y, rc, y[k][1]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool use = q + k < e;
      const int c1 = rec[k].x & 0x7fffffff, c2 = rec[k].y;
      const bool own_neg = rec[k].x < 0;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const float f1 = lit_factor(c1, y[k][0][j]), f2 = lit_factor(c2, y[k][1][j]);
        const float p = f1 * f2;
        g[j] += use ? (double)(own_neg ? p : -p) : 0.0;
        if constexpr (FIRST) {
          const float ao = own_neg ? xv[j] : 1.0f - xv[j];
          lsum[j] += use ? (double)(ao * p) : 0.0;
          const float m = fminf(fminf(false_margin(c1, f1), false_margin(c2, f2)),
                                false_margin(own_neg ? 1 : 0, ao));
          usum[j] += (use && m >= 0.0f) ? 1 : 0;
        }
      }
    }
  }
}

// Clause-row records of [b, e): record = row | own_neg << 31.  The partial
// of the occurrence is the row's product divided by the own factor (count
// 0), the row's product when the own factor is its only zero, else 0; the
// sign of dU/dx_v (- for a positive own literal, + for a negated one) is
// folded into the inverse.
template <int RPL>
__device__ __forceinline__ void flat_rows(const VarPassArgs& a, int b, int e, int rc,
                                          const float (&xv)[RPL], double (&g)[RPL]) {
  if (b >= e) return;
  double inv_p[RPL], inv_n[RPL];
  bool zp[RPL], zn[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const float ap = 1.0f - xv[j], an = xv[j];
    zp[j] = ap == 0.0f;
    zn[j] = an == 0.0f;
    inv_p[j] = zp[j] ? -1.0 : -1.0 / (double)ap;
    inv_n[j] = zn[j] ? 1.0 : 1.0 / (double)an;
  }
  constexpr int B = 8;
  for (int q = b; q < e; q += B) {
    uint32_t rec[B];
    uint32_t u[B][RPL];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int qk = q + k < e ? q + k : e - 1;  // in bounds; masked below
      rec[k] = (uint32_t)ldc(reinterpret_cast<const int32_t*>(a.lrec), qk);
      load_urow<RPL>(a.qrow + (int64_t)(rec[k] & 0x7fffffffu) * a.ldq + rc, u[k]);
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const bool use = q + k < e;
      const bool own_neg = (rec[k] >> 31) != 0;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const bool one_zero = (u[k][j] >> 31) != 0;
        const bool own_zero = own_neg ? zn[j] : zp[j];
        const double qv = (one_zero && !own_zero) ? 0.0 : clause_value(u[k][j]);
        const double s = own_neg ? inv_n[j] : inv_p[j];
        g[j] += use ? qv * s : 0.0;
      }
    }
  }
}

// Unified index range [u0, u1) of variable v's contributions: first-literal
// pairs, then the other pairs, then clause rows (the three together have
// exactly one entry per occurrence of v).
template <int RPL>
__device__ __forceinline__ void flat_range(const VarPassArgs& a, const float* xb, int v, int u0,
                                           int u1, int rc, const float (&xv)[RPL],
                                           double (&g)[RPL], double (&lsum)[RPL],
                                           int (&usum)[RPL]) {
  const int pf = ldc(a.pair_first, v), pm = ldc(a.pair_mid, v), pz = ldc(a.pair_first, v + 1);
  const int lb = ldc(a.lrec_ptr, v);
  const int nf = pm - pf, np = pz - pf;
  flat_pairs<RPL, true>(a, xb, pf + max(u0, 0), pf + min(u1, nf), rc, xv, g, lsum, usum);
  flat_pairs<RPL, false>(a, xb, pf + max(u0, nf), pf + min(u1, np), rc, xv, g, lsum, usum);
  const int nl = ldc(a.lrec_ptr, v + 1) - lb;
  flat_rows<RPL>(a, lb + max(u0 - np, 0), lb + min(u1 - np, nl), rc, xv, g);
}

// Whole variables of the chunk's range: the gradient, then the epilogue.
template <int LPI, int RPL, int MODE>
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
  const float* xb = a.x + (int64_t)ldc(a.chunk_fvb, chunk) * a.ldx;
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
    flat_range<RPL>(a, xb, v, 0, 0x7fffffff, rc, xv, g, lsum, usum);
    if (active) var_epilogue<RPL, MODE>(a, v, r0, xv, g);
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// Segments of split variables: each segment's partial gradient (its
// unified range [seg_q0 - var_ptr[v], seg_q1 - var_ptr[v])) goes to
// gseg[s][r] in FP64; k_heavy_finish adds them in segment order.
template <int LPI, int RPL>
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
    const int sgi = uniform<LPI>(s0);
    const int v = ldc(a.seg_var, sgi);
    const int qb = ldc(a.var_ptr, v);
    const float* xb = a.x + (int64_t)ldc(a.f_vbeg, ldc(a.var_formula, v)) * a.ldx;
    double g[RPL];
    float xv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    load_row<RPL>(a.x + (int64_t)v * a.ldx + rc, xv);
    flat_range<RPL>(a, xb, v, ldc(a.seg_q0, sgi) - qb, ldc(a.seg_q1, sgi) - qb, rc, xv, g, lsum,
                    usum);
    if (active) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) a.gseg[(int64_t)sgi * a.R + r0 + j] = g[j];
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// ------------------------------------------------------------ launchers

namespace {

template <int LPI, int RPL>
hipError_t flat_var_rpl(const VarPassArgs& a, int mode, int chunks, int tiles, hipStream_t s) {
  dim3 grid(chunks, tiles), block(kBlock);
  switch (mode) {
    case kModeSGD: hipLaunchKernelGGL((k_flat_var<LPI, RPL, kModeSGD>), grid, block, 0, s, a); break;
    case kModeAdam: hipLaunchKernelGGL((k_flat_var<LPI, RPL, kModeAdam>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_flat_var<LPI, RPL, kModeGrad>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
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
  switch (t.rpl) {
    case 4: hipLaunchKernelGGL((k_flat_seg<LPI, 4>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_flat_seg<LPI, 2>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_flat_seg<LPI, 1>), grid, block, 0, s, a); break;
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
