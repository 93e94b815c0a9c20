// Clause pass, fixed-order reductions, state init / copy and the exact
// rounded unsat count of the general schedule (gfx950).
//
// Paper passages: clause value U_t = prod_i (1 - s_i) (Section 3.2, Eq. 2)
// with the negation rule of Eq. (1); loss' = sum_t U_t (Eq. 5 shifted by
// the clause count); rounding x_hat = [x > 0.5] is the argmax of Eq. (4)
// with ties to 0.
#include "galsat_device.h"

namespace galsat {

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
  const int chunk =
      a.chunk_order ? ldc(a.chunk_order, a.chunk_base + blockIdx.x) : a.chunk_base + blockIdx.x;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
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

// ---------------------------------------------- short-clause partials
//
// Stored clauses of at most KS literals, one item (LPI lanes) per clause,
// read from the class's packed table (codes and D rows, -1 marking unused
// positions): the clause's rows are gathered once into registers, the
// exclusive prefix and suffix products formed there, and every literal's
// partial
//   slope_j * prefix_j * suffix_j
// written to its row of D.  One gather and one store per literal.
template <int LPI, int RPL, int KS>
__global__ __launch_bounds__(kBlock) void k_short_clause(ClausePassArgs a) {
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
  const int cb = ldc(a.chunk_cbeg, chunk), ce = ldc(a.chunk_cend, chunk);
  double lsum[RPL];
  int usum[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) { lsum[j] = 0.0; usum[j] = 0; }

  for (int c0 = cb + slot; c0 < ce; c0 += IPB) {
    // the class's packed table: the clause's codes and D rows side by side,
    // so its row gathers depend on one table load only
    const int32_t* pk = a.packed + (int64_t)uniform<LPI>(c0) * 2 * KS;
    int code[KS], drow[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      code[u] = ldc(pk, u);
      drow[u] = ldc(pk, KS + u);
    }
    float f[KS][RPL];
    bool any_true[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) any_true[j] = false;
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const bool in = drow[u] >= 0;
      float y[RPL];
      if (in) {
        load_row<RPL>(a.x + (int64_t)(code[u] >> 1) * a.ldx + rc, y);
      } else {
#pragma unroll
        for (int j = 0; j < RPL; ++j) y[j] = 0.0f;  // factor 1 below
      }
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        f[u][j] = in ? lit_factor(code[u], y[j]) : 1.0f;
        any_true[j] = any_true[j] || (in && lit_true(code[u], y[j]));
      }
    }
    float pre[KS][RPL];
    float run[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) run[j] = 1.0f;
#pragma unroll
    for (int u = 0; u < KS; ++u)
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        pre[u][j] = run[j];
        run[j] *= f[u][j];
      }
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      lsum[j] += (double)run[j];
      usum[j] += any_true[j] ? 0 : 1;
    }
    float suf[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) suf[j] = 1.0f;
#pragma unroll
    for (int u = KS - 1; u >= 0; --u) {
      float dv[RPL];
      const float slope = (code[u] & 1) ? 1.0f : -1.0f;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        dv[j] = slope * (pre[u][j] * suf[j]);
        suf[j] *= f[u][j];
      }
      if (active && drow[u] >= 0) store_row<RPL>(a.D + (int64_t)drow[u] * a.ldD + r0, dv);
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row ? ldc(a.chunk_row, chunk) : chunk, tile, a.R,
                           a.loss_part, a.unsat_part);
}

// ------------------------------------------------ wave-per-clause pass
//
// Stored clauses of G..KMAX literals, one wavefront per clause: the wave's
// 64 lanes form G = 64 / LPI literal groups of LPI lanes, each group
// covering the tile's restarts, and group g takes the clause's literals
// [g * m, g * m + m) with m = ceil(k / G) <= MAXC.  Every literal's row is
// gathered once and its factor kept in registers; a lane forms the prefix
// and suffix products within its run serially, and one exclusive scan of
// the run products across the groups (shuffles by multiples of LPI lanes,
// so a lane only combines values of its own restarts) supplies the
// products of the runs before and after.  The partial of literal j is
//   slope_j * (before * prefix_in_run) * (suffix_in_run * after),
// written to its row of D: one gather and one store per literal, nothing
// stored in between.  No division: exact zero factors need no special case.
template <int LPI, int RPL, int MAXC>
__global__ __launch_bounds__(kBlock) void k_wave_clause(ClausePassArgs a) {
  constexpr int G = 64 / LPI;
  constexpr int RT = LPI * RPL;
  constexpr int WPB = kBlock / 64;
  const int wave = threadIdx.x / 64, lw = threadIdx.x % 64;
  const int grp = lw / LPI, lane = lw % LPI;
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

  // the next clause's header is loaded while the current one is processed
  auto header = [&](int i, int* s, int* k) {
    const int t = __builtin_amdgcn_readfirstlane(a.clause_ids ? ldc(a.clause_ids, i) : i);
    *s = ldc(a.clause_ptr, t);
    *k = ldc(a.clause_ptr, t + 1) - *s;
  };
  int s_next = 0, k_next = 0;
  if (cb + wave < ce) header(cb + wave, &s_next, &k_next);
  for (int i = cb + wave; i < ce; i += WPB) {
    const int s = s_next, k = k_next;
    if (i + WPB < ce) header(i + WPB, &s_next, &k_next);
    const int m = (k + G - 1) / G;  // run length (the plan keeps m <= MAXC)
    const int lb = grp * m;         // first literal of this group's run
    float f[MAXC][RPL];
    int code[MAXC];
    int any_true[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) any_true[j] = 0;
    // gather the run: all its rows in flight together
#pragma clang loop unroll(full)
    for (int c = 0; c < MAXC; ++c) {
      const int li = lb + c;
      const bool in = c < m && li < k;
      code[c] = c < m ? ldc(a.clause_lits, s + (in ? li : 0)) : 0;
      float y[RPL];
      if (c < m) {
        // positions past the clause read its first literal's row again
        // and use factor 1
        load_row<RPL>(a.x + (int64_t)(code[c] >> 1) * a.ldx + rc, y);
      } else {
#pragma unroll
        for (int j = 0; j < RPL; ++j) y[j] = 0.0f;
      }
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        f[c][j] = in ? lit_factor(code[c], y[j]) : 1.0f;
        any_true[j] |= (in && lit_true(code[c], y[j])) ? 1 : 0;
      }
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      // any literal true (per restart): OR over the groups
#pragma unroll
      for (int d = LPI; d < 64; d <<= 1) any_true[j] |= __shfl_xor(any_true[j], d);
    }
    // prefix within the run (exclusive), overwriting nothing: pre[c]
    float pre[MAXC][RPL];
    float run[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) run[j] = 1.0f;
#pragma clang loop unroll(full)
    for (int c = 0; c < MAXC; ++c) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        pre[c][j] = run[j];
        run[j] *= f[c][j];
      }
    }
    // products of the runs before (inclusive scan, then shift) and after
    float before[RPL], after[RPL], total[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      float inc = run[j];
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const float o = __shfl_up(inc, d * LPI);
        inc = grp >= d ? inc * o : inc;
      }
      const float ex = __shfl_up(inc, LPI);
      before[j] = grp > 0 ? ex : 1.0f;
      total[j] = __shfl(inc, (G - 1) * LPI + lane);  // U_t: the product of all factors
      float sinc = run[j];
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const float o = __shfl_down(sinc, d * LPI);
        sinc = grp + d < G ? sinc * o : sinc;
      }
      const float sex = __shfl_down(sinc, LPI);
      after[j] = grp < G - 1 ? sex : 1.0f;
    }
    if (grp == 0) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        lsum[j] += (double)total[j];
        usum[j] += any_true[j] ? 0 : 1;
      }
    }
    // suffix within the run, then the partials
    float suf[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) suf[j] = after[j];
#pragma clang loop unroll(full)
    for (int c = MAXC - 1; c >= 0; --c) {
      float dv[RPL];
      const float slope = (code[c] & 1) ? 1.0f : -1.0f;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        dv[j] = slope * ((before[j] * pre[c][j]) * suf[j]);
        suf[j] *= f[c][j];
      }
      const int li = lb + c;
      if (active && c < m && li < k)
        store_row<RPL>(a.D + (int64_t)ldc(a.lit_dslot, s + li) * a.ldD + r0, dv);
    }
  }
  block_partials<LPI, RPL>(lsum, usum, a.chunk_row ? ldc(a.chunk_row, chunk) : chunk, tile, a.R,
                           a.loss_part, a.unsat_part);
}

// ------------------------------------------------------------ finalize
//
// loss[f][r] = sum of the formula's partial rows (fixed order) + empty
// clauses; the same for the unsat count.
// W waves per block: wave w sums rows w, w + W, ... for 64 restarts into
// eight interleaved accumulators (eight rows in flight), which are added in
// a fixed order; then the W partial sums are combined pairwise in a fixed
// tree.
// With a.split > 1, block x handles part x % split of formula x / split and
// writes its sums (without the empty clauses) to part_l / part_u.
template <int W>
__global__ __launch_bounds__(64 * W) void k_finalize(FinalizeArgs a) {
  constexpr int U = 8;
  const int fl = blockIdx.x / a.split, part = blockIdx.x % a.split;
  const int f = a.f_base + fl;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  const int R = a.R;
  double acc = 0.0;
  int uacc = 0;
  if (r < R) {
    const int fb = a.a_beg[f], fe = a.a_end[f];
    const int rb = fb + (int)((int64_t)(fe - fb) * part / a.split);
    const int re = fb + (int)((int64_t)(fe - fb) * (part + 1) / a.split);
    double al[U];
    int au[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { al[u] = 0.0; au[u] = 0; }
    int row = rb + w;
    for (; row + (U - 1) * W < re; row += U * W) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = (int64_t)(row + u * W) * R + r;
        if (a.loss_out) al[u] += a.loss_part[i];
        if (a.unsat_out) au[u] += a.unsat_part[i];
      }
    }
    for (int u = 0; row < re; row += W, ++u) {
      const int64_t i = (int64_t)row * R + r;
      if (a.loss_out) al[u] += a.loss_part[i];
      if (a.unsat_out) au[u] += a.unsat_part[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc += al[u];
      uacc += au[u];
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
    if (a.split > 1) {
      a.part_l[(int64_t)blockIdx.x * R + r] = sl[lane];
      a.part_u[(int64_t)blockIdx.x * R + r] = su[lane];
    } else {
      const double tot = sl[lane] + (double)a.n_empty[f];
      const int utot = su[lane] + a.n_empty[f];
      if (a.loss_out) a.loss_out[(int64_t)f * R + r] = (float)tot;
      if (a.unsat_out) a.unsat_out[(int64_t)f * R + r] = utot;
    }
  }
}

// Second stage of the split finalize: the parts of each formula in order.
__global__ __launch_bounds__(64) void k_finalize_parts(FinalizeArgs a) {
  const int fl = blockIdx.x, f = a.f_base + fl;
  const int r = blockIdx.y * 64 + threadIdx.x;
  const int R = a.R;
  if (r >= R) return;
  double tot = 0.0;
  int utot = 0;
  for (int p = 0; p < a.split; ++p) {
    tot += a.part_l[((int64_t)fl * a.split + p) * R + r];
    utot += a.part_u[((int64_t)fl * a.split + p) * R + r];
  }
  if (a.loss_out) a.loss_out[(int64_t)f * R + r] = (float)(tot + (double)a.n_empty[f]);
  if (a.unsat_out) a.unsat_out[(int64_t)f * R + r] = utot + a.n_empty[f];
}

// ---------------------------------------------------------- init / copy

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

// ------------------------------------------------------- round & count
//
// bits[w][v]: bit l = [x[v][64w + l] > 0.5] packed by wavefront ballots.
// P lanes per variable (P = 64, or 32 / 16 when all restarts fit one word
// and R <= P), so one ballot packs 64/P variables; a wave takes kPackU
// ballots' worth of consecutive variables per trip, all loads first.
constexpr int kPackU = 8;

template <int P>
__global__ __launch_bounds__(256) void k_pack_bits(const float* x, int32_t ldx, int32_t n,
                                                   int32_t R, uint64_t* bits) {
  constexpr int VPB = 64 / P;  // variables per ballot
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int word = blockIdx.y;
  const int sub = lane / P, r = word * 64 + lane % P;
  for (int64_t v0 = ((int64_t)blockIdx.x * 4 + wv) * kPackU * VPB; v0 < n;
       v0 += (int64_t)gridDim.x * 4 * kPackU * VPB) {
    float val[kPackU];
#pragma unroll
    for (int u = 0; u < kPackU; ++u) {
      const int64_t v = v0 + u * VPB + sub;
      val[u] = (r < R && v < n) ? x[v * ldx + r] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kPackU; ++u) {
      const uint64_t m = __ballot(val[u] > 0.5f);
      const int64_t v = v0 + u * VPB + lane;  // lane k < VPB stores variable k's word
      if (lane < VPB && v < n) {
        uint64_t w = m;
        if constexpr (P < 64) w = (m >> (lane * P)) & ((1ULL << P) - 1ULL);
        bits[(int64_t)word * n + v] = w;
      }
    }
  }
}

// mask AND "literal false" over the literals [ps, pe) of one clause, W
// literals a trip: their codes, then their bit-plane words, all loads in
// flight (positions past the clause reread its last literal and are not
// used).
template <int W>
__device__ __forceinline__ uint64_t and_literals_false(const int32_t* clause_lits,
                                                       const uint64_t* bw, int ps, int pe,
                                                       uint64_t mask) {
  for (int p = ps; p < pe; p += W) {
    int code[W];
    uint64_t b[W];
#pragma unroll
    for (int u = 0; u < W; ++u) code[u] = clause_lits[min(p + u, pe - 1)];
#pragma unroll
    for (int u = 0; u < W; ++u) b[u] = bw[code[u] >> 1];
#pragma unroll
    for (int u = 0; u < W; ++u)
      if (p + u < pe) mask &= (code[u] & 1) ? b[u] : ~b[u];
  }
  return mask;
}

// Lanes take one clause each; for the 64 restarts of word w a clause's
// "unsatisfied" mask is the AND over its literals of "literal false"
// (eight literals a trip for clauses longer than 8, else four).  The
// per-restart count over the wave's 64 clauses is then one ballot and one
// popcount per restart, accumulated by the lane that owns the restart.
// order: block -> chunk (-1: nothing), or null.
__global__ __launch_bounds__(256) void k_count_unsat(const int32_t* clause_ptr,
                                                     const int32_t* clause_lits,
                                                     const int32_t* chunk_cbeg,
                                                     const int32_t* chunk_cend,
                                                     const int32_t* order,
                                                     const uint64_t* bits, int32_t n, int32_t R,
                                                     int32_t* unsat_part) {
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int chunk = order ? order[blockIdx.x] : (int)blockIdx.x, word = blockIdx.y;
  if (chunk < 0) return;  // padding of the XCD-aware order: the whole block leaves
  const int cb = chunk_cbeg[chunk], ce = chunk_cend[chunk];
  const int rem = R - word * 64;
  const uint64_t valid = rem >= 64 ? ~0ULL : ((1ULL << rem) - 1ULL);
  const int jmax = rem >= 64 ? 64 : rem;
  const uint64_t* bw = bits + (int64_t)word * n;
  int cnt = 0;
  for (int base = cb + wv * 64; base < ce; base += 256) {
    const int t = base + lane;
    uint64_t mask = 0;
    if (t < ce) {
      mask = valid;
      const int ps = clause_ptr[t], pe = clause_ptr[t + 1];
      if (pe - ps > 8)
        mask = and_literals_false<8>(clause_lits, bw, ps, pe, mask);
      else
        mask = and_literals_false<4>(clause_lits, bw, ps, pe, mask);
    }
    // restarts past R have no bits (valid masks them), so their ballots
    // are skipped: the loop runs over this word's restarts only
    for (int j = 0; j < jmax; ++j) {
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
}  // namespace

hipError_t launch_short_clause(const ClausePassArgs& a, Tile t, int ks, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  if (ks != 4 && ks != kShortClauseMax) return hipErrorInvalidValue;
  const int tiles = launch_tiles(a, t);
  dim3 grid(chunks, tiles), block(kBlock);
  switch (t.lpi * 8 + t.rpl) {
#define GALSAT_SHORT_CASE(L, P)                                                                 \
  case L * 8 + P:                                                                               \
    if (ks == 4)                                                                                \
      hipLaunchKernelGGL((k_short_clause<L, P, 4>), grid, block, 0, s, a);                      \
    else                                                                                        \
      hipLaunchKernelGGL((k_short_clause<L, P, kShortClauseMax>), grid, block, 0, s, a);        \
    break;
    GALSAT_SHORT_CASE(4, 1)
    GALSAT_SHORT_CASE(4, 2)
    GALSAT_SHORT_CASE(4, 4)
    GALSAT_SHORT_CASE(8, 1)
    GALSAT_SHORT_CASE(8, 2)
    GALSAT_SHORT_CASE(8, 4)
    GALSAT_SHORT_CASE(16, 1)
    GALSAT_SHORT_CASE(16, 2)
    GALSAT_SHORT_CASE(16, 4)
    GALSAT_SHORT_CASE(32, 1)
    GALSAT_SHORT_CASE(32, 2)
    GALSAT_SHORT_CASE(32, 4)
    GALSAT_SHORT_CASE(64, 1)
    GALSAT_SHORT_CASE(64, 2)
    GALSAT_SHORT_CASE(64, 4)
#undef GALSAT_SHORT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wave_clause(const ClausePassArgs& a, Tile t, int maxc, int chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  if (wave_clause_kmax(t) <= 0) return hipErrorInvalidValue;
  if (maxc != kWaveClauseSmallChunks && maxc != wave_clause_chunks(t.lpi)) return hipErrorInvalidValue;
  const int tiles = launch_tiles(a, t);
  dim3 grid(chunks, tiles), block(kBlock);
  switch (t.lpi * 8 + t.rpl) {
#define GALSAT_WAVE_CASE(L, P)                                                                  \
  case L * 8 + P:                                                                               \
    if (maxc == kWaveClauseSmallChunks)                                                         \
      hipLaunchKernelGGL((k_wave_clause<L, P, kWaveClauseSmallChunks>), grid, block, 0, s, a);  \
    else                                                                                        \
      hipLaunchKernelGGL((k_wave_clause<L, P, wave_clause_chunks(L)>), grid, block, 0, s, a);   \
    break;
    GALSAT_WAVE_CASE(4, 1)
    GALSAT_WAVE_CASE(4, 2)
    GALSAT_WAVE_CASE(4, 4)
    GALSAT_WAVE_CASE(8, 1)
    GALSAT_WAVE_CASE(8, 2)
    GALSAT_WAVE_CASE(8, 4)
    GALSAT_WAVE_CASE(16, 1)
    GALSAT_WAVE_CASE(16, 2)
    GALSAT_WAVE_CASE(16, 4)
#undef GALSAT_WAVE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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

hipError_t launch_finalize(const FinalizeArgs& a_in, int F, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  FinalizeArgs a = a_in;
  const int gy = (a.R + 63) / 64;
  // few formulas x restart groups: cut each formula's rows into parts
  // summed by separate workgroups (about 512 workgroups in all), when the
  // part sums fit the workspace
  a.split = 1;
  if ((int64_t)F * gy < 512 && a.part_l && a.part_u) {
    const int64_t want = (512 + (int64_t)F * gy - 1) / ((int64_t)F * gy);
    const int64_t fit = kFinalizeScratch / ((int64_t)F * a.R);
    const int64_t rows = std::max<int64_t>(1, a.max_rows / 256);  // >= 256 rows a part
    a.split = (int)std::max<int64_t>(1, std::min(std::min(want, fit), rows));
  }
  dim3 grid(F * a.split, gy);
  if (a.split > 1) {
    hipLaunchKernelGGL((k_finalize<4>), grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize_parts, dim3(F, gy), dim3(64), 0, s, a);
  } else if ((int64_t)F * gy < 256) {
    // few large formulas: more waves per formula; many small ones: fewer
    hipLaunchKernelGGL((k_finalize<16>), grid, dim3(1024), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_finalize<4>), grid, dim3(256), 0, s, a);
  }
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
  const int P = R <= 16 ? 16 : R <= 32 ? 32 : 64;
  const int64_t per_block = 4 * kPackU * (64 / P);
  dim3 grid(grid_x_for((n + per_block - 1) / per_block), (R + 63) / 64), block(256);
  if (P == 16)
    hipLaunchKernelGGL((k_pack_bits<16>), grid, block, 0, s, x, ldx, n, R, bits);
  else if (P == 32)
    hipLaunchKernelGGL((k_pack_bits<32>), grid, block, 0, s, x, ldx, n, R, bits);
  else
    hipLaunchKernelGGL((k_pack_bits<64>), grid, block, 0, s, x, ldx, n, R, bits);
  return hipGetLastError();
}

hipError_t launch_count_unsat(const int32_t* clause_ptr, const int32_t* clause_lits,
                              const int32_t* chunk_cbeg,
                              const int32_t* chunk_cend, const int32_t* order, int blocks,
                              const uint64_t* bits, int32_t n, int32_t R, int32_t* unsat_part,
                              hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  dim3 grid(blocks, (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_count_unsat, grid, block, 0, s, clause_ptr, clause_lits, chunk_cbeg,
                     chunk_cend, order, bits, n, R, unsat_part);
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
