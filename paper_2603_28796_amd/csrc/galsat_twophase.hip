// Two-phase gradient plan (gfx950): an occurrence-parallel pass writes
// every occurrence's contribution row, then per-variable sums in the
// single pass's order (backpropagation through Eq. 2 of Section 3.2).
#include "galsat_device.h"

namespace galsat {

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
#pragma unroll
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

// ------------------------------------------------------------ launchers

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

}  // namespace galsat
