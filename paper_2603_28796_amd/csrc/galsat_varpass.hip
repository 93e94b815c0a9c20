// Variable pass of the general schedule (gfx950): for every variable and
// restart, the gradient summed over the variable's occurrences in a fixed
// order, fused with the projected SGD / Adam update or the gradient output
// (backpropagation through Eq. 2 of Section 3.2); the streaming variant;
// segments of split variables and their finish.
#include "galsat_device.h"

namespace galsat {

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

// The product of a record's exactly K other literals (the first K of
// `all`), all K gathers in flight; no slot is padding, so combine's masks
// fold away.
template <int RPL, int K>
__device__ __forceinline__ void others_k(const VarPassArgs& a, const int (&all)[7], bool first,
                                         int r0, float (&prod)[RPL], bool (&any_true)[RPL]) {
  int codes[K];
  float y[K][RPL];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    codes[c] = all[c];
    load_row<RPL>(a.x + (int64_t)(codes[c] >> 1) * a.ldx + r0, y[c]);
  }
  combine<RPL, K>(codes, y, K, first, prod, any_true);
}

// One INLINE occurrence of up to 7 other literals, all gathers in flight.
// U: the record is the same for the whole wave (one item per wave), so a
// record of 4 to 7 other literals branches, without divergence, to the
// instance of exactly its size instead of padding to seven.
template <int RPL, bool U = false>
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
  } else if constexpr (U) {
    const int4 e = ldc4(a.occx, q);
    const int all[7] = {o.y, o.z, o.w, e.x, e.y, e.z, e.w};
    const bool first = rec_first(hdr);
    if (nother == 4) others_k<RPL, 4>(a, all, first, r0, prod, any_true);
    else if (nother == 5) others_k<RPL, 5>(a, all, first, r0, prod, any_true);
    else if (nother == 6) others_k<RPL, 6>(a, all, first, r0, prod, any_true);
    else others_k<RPL, 7>(a, all, first, r0, prod, any_true);
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

// W consecutive literal positions [i, i + W) of a GENERAL record's clause
// (ce: the clause's end, p: the own position) multiplied into prod, all W
// gathers in flight; positions past ce (when W overruns it) read the
// clause's first literal again and, like the own position, count as 1.
template <int RPL, int W>
__device__ __forceinline__ void general_batch(const VarPassArgs& a, int i, int cs, int ce, int p,
                                              int r0, float (&prod)[RPL], bool (&any_true)[RPL]) {
  int codes[W];
  float y[W][RPL];
#pragma unroll
  for (int u = 0; u < W; ++u) {
    const int iu = i + u < ce ? i + u : cs;
    codes[u] = ldc(a.clause_lits, iu);
    load_row<RPL>(a.x + (int64_t)(codes[u] >> 1) * a.ldx + r0, y[u]);
  }
#pragma unroll
  for (int u = 0; u < W; ++u) {
    const bool use = i + u < ce && i + u != p;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      prod[j] *= use ? lit_factor(codes[u], y[u][j]) : 1.0f;
      any_true[j] = any_true[j] || (use && lit_true(codes[u], y[u][j]));
    }
  }
}

// One GENERAL occurrence: the clause's other literals four at a time.  U
// (one item per wave): the last one to three positions run as an instance
// of exactly that width instead of four.
template <int RPL, bool U = false>
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
  if constexpr (U) {
    int i = cs;
    for (; i + 4 <= ce; i += 4) general_batch<RPL, 4>(a, i, cs, ce, p, r0, prod, any_true);
    const int rem = ce - i;
    if (rem == 1) general_batch<RPL, 1>(a, i, cs, ce, p, r0, prod, any_true);
    else if (rem == 2) general_batch<RPL, 2>(a, i, cs, ce, p, r0, prod, any_true);
    else if (rem == 3) general_batch<RPL, 3>(a, i, cs, ce, p, r0, prod, any_true);
  } else {
    for (int i = cs; i < ce; i += 4) {
      int codes[4];
      float y[4][RPL];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // positions past the clause read the clause's first literal again
        // and are masked out below, like the own position
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
  add_occurrence<RPL>((ldc(a.clause_lits, p) & 1) != 0, first, prod, any_true, xv, g, lsum, usum);
}

// One occurrence of any kind (U: as for inline_one).
template <int RPL, bool U = false>
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
    inline_one<RPL, U>(a, o, q, r0, xv, g, lsum, usum);
  } else {
    general_one<RPL, U>(a, o, r0, xv, g, lsum, usum);
  }
}

// Adds the contributions of occurrences [q0, q1) (in that order) of the
// variable whose own state is xv.  r0 must be a valid column for every lane
// (lanes past the last restart pass a clamped one and discard the results),
// so the loop runs under wave-uniform control and its table loads can be
// scalar.
template <int RPL, bool U = false>
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
          for (int k = 0; k < 4; ++k) inline_one<RPL, U>(a, o[k], q + k, r0, xv, g, lsum, usum);
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
    one_occurrence<RPL, U>(a, ldc4(a.occ, q), q, r0, xv, g, lsum, usum);
    ++q;
  }
}

// Variables of the chunk's range (the ranges exclude split variables): the
// whole gradient, then the epilogue.
template <int LPI, int RPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_var_pass(VarPassArgs a) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  int bx = blockIdx.x, by = blockIdx.y;
  if (a.xcd_pin) {
    // tile = linear block id mod tiles: workgroups are dealt to the 8 XCDs
    // round-robin in that order, so with 8 tiles per launch an XCD's L2
    // serves one tile's lines only
    const int lin = blockIdx.y * gridDim.x + blockIdx.x;
    by = lin % gridDim.y;
    bx = lin / gridDim.y;
  }
  const int chunk = a.chunk_order ? ldc(a.chunk_order, a.chunk_base + bx) : a.chunk_base + bx;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
  const int tile = a.tile_base + by;
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

// Segments of split variables (variables with more occurrences than one
// item should serialise): each segment's partial gradient goes to
// gseg[s][r] in FP64.  With one item per wave the segment walks are
// latency-bound chains of gathers, and six waves per SIMD (a few spilled
// registers) beat five without spills; records then take their exact-size
// instances (in the whole-variable kernel the extra registers of those
// instances cost more than they save).
template <int LPI, int RPL>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(LPI == 64 ? 6 : 1))) void k_var_seg(VarPassArgs a) {
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
    gather_occurrences<RPL, LPI == 64>(a, ldc(a.seg_q0, sgi), ldc(a.seg_q1, sgi), rc, xv, g, lsum, usum);
    if (active) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) a.gseg[(int64_t)sgi * a.R + r0 + j] = g[j];
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row[chunk], tile, a.R, a.loss_part, a.unsat_part);
}

// Split variables, one workgroup each: item slot s sums the variable's
// segments s, s + IPB, ... in FP64, the slots' sums are added in slot
// order, then the same epilogue as k_var_pass.  The shape of this sum is
// fixed by the plan, so the result is reproducible; segment partials of
// the hottest variables (thousands of segments) are read in parallel.
template <int LPI, int RPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_heavy_finish(VarPassArgs a, int h0, int h1) {
  constexpr int IPB = kBlock / LPI;
  constexpr int RT = LPI * RPL;
  __shared__ double s_g[IPB][RT];
  const int lane = threadIdx.x % LPI, slot = threadIdx.x / LPI;
  const int tile = a.tile_base + blockIdx.y;
  const int r0 = tile * RT + lane * RPL;
  const bool active = r0 < a.R;
  const int rc = active ? r0 : 0;
  for (int i = h0 + blockIdx.x; i < h1; i += gridDim.x) {
    const int sb = ldc(a.heavy_sbeg, i), se = ldc(a.heavy_sbeg, i + 1);
    double g[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) g[j] = 0.0;
    // eight of the slot's segments per trip, all loads issued first (indices
    // clamped into range), then added in segment order
    for (int sgi = sb + slot; sgi < se; sgi += 8 * IPB) {
      double d[8][RPL];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int s2 = min(sgi + u * IPB, se - 1);
#pragma unroll
        for (int j = 0; j < RPL; ++j) d[u][j] = a.gseg[(int64_t)s2 * a.R + rc + j];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (sgi + u * IPB < se) {
#pragma unroll
          for (int j = 0; j < RPL; ++j) g[j] += d[u][j];
        }
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j) s_g[slot][lane * RPL + j] = g[j];
    __syncthreads();
    if (slot == 0 && active) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) g[j] = 0.0;
#pragma unroll 4
      for (int t = 0; t < IPB; ++t)
#pragma unroll
        for (int j = 0; j < RPL; ++j) g[j] += s_g[t][lane * RPL + j];
      const int v = ldc(a.heavy_var, i);
      float xv[RPL];
      load_row<RPL>(a.x + (int64_t)v * a.ldx + r0, xv);
      var_epilogue<RPL, MODE>(a, v, r0, xv, g);
    }
    __syncthreads();
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
  int blocks = h1 - h0;  // one workgroup per split variable
  blocks = blocks > 65536 ? 65536 : blocks;
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

}  // namespace

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

}  // namespace galsat
