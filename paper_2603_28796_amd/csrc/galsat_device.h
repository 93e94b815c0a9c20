// Device helpers shared by the HIP kernels of the general schedule
// (gfx950, wave64): literal factors and rounding, row loads and stores,
// scalar-path table loads, the per-block partial sums, the occurrence
// record format, and the variable epilogue (fused update or gradient).
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
#pragma once

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

// Four occurrences' other-literal products at once (INLINE records with at
// most NO <= 3 other literals each): every row gather is issued before any
// product is formed.
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

// The epilogue for one variable row: projected SGD or Adam update (writing
// the next state) or the (upstream-scaled) gradient.
// NT: the output row is stored non-temporally (it is not read again in the
// same pass, so it should not evict rows that are).
template <int RPL, int MODE, bool NT = false>
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
  if constexpr (NT) store_row_nt<RPL>(a.out + (int64_t)v * a.ldo + r0, o);
  else store_row<RPL>(a.out + (int64_t)v * a.ldo + r0, o);
}

// SplitMix64 output mixing (the finalizer of Steele, Lea and Flood's
// SplitMix64), the counter hash of the state init and the Gumbel noise.
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Restart tiles of one launch: [tile_base, tile_base + tile_count), or all.
template <class Args>
inline int launch_tiles(const Args& a, Tile t) {
  const int all = (a.R + t.tile() - 1) / t.tile() - a.tile_base;
  return a.tile_count > 0 && a.tile_count < all ? a.tile_count : all;
}

// Grid width for grid-stride launches (at most 65536 blocks).
inline int grid_x_for(int64_t items_div4) {
  int64_t g = items_div4 < 1 ? 1 : items_div4;
  return (int)(g > 65536 ? 65536 : g);
}

}  // namespace galsat
