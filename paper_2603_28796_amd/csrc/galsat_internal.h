// Internal declarations shared by the host runtime and the kernels of
// libgalsat.  Not part of the public ABI (include/galsat.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/galsat.h"

namespace galsat {

constexpr int kBlock = 256;  // threads per workgroup of the general passes

// Launch shape of a general pass: each variable (or clause) is handled by
// `lpi` lanes, each lane covering `rpl` consecutive restarts, so one item
// covers a restart tile of lpi*rpl restarts; grid.y walks the tiles.
struct Tile {
  int lpi = 64;
  int rpl = 1;
  int tile() const { return lpi * rpl; }
};

// Arguments of the variable-parallel pass (backward gather + fused update).
struct VarPassArgs {
  const int32_t* var_ptr;
  const int4* occ;              // [L] occurrence record of each variable-major slot
  const int4* occx;             // [L] second record word (5 to 8 literal clauses)
  const int32_t* clause_ptr;
  const int32_t* clause_lits;
  const int32_t* chunk_vbeg;    // [chunks] item range of each chunk (variables or segments)
  const int32_t* chunk_vend;
  const int32_t* chunk_row;     // [chunks] partial-sum row of each chunk
  const int32_t* chunk_order;   // [blocks] chunk of each workgroup (-1: none), or null
  const int32_t* seg_var;       // [segments] variable of each segment of a split variable
  const int32_t* seg_perm;      // [segments] run order: segment chunks cover runs of it
  const int32_t* seg_q0;        // [segments] occurrence range of the segment
  const int32_t* seg_q1;
  double* gseg;                 // [segments][R] partial gradients of the segments
  const int32_t* heavy_var;     // [heavy] split variables
  const int32_t* heavy_sbeg;    // [heavy+1] segment range of each split variable
  const int32_t* var_formula;   // [n] formula of each variable (upstream scaling)
  int32_t chunk_base;           // first chunk of this launch
  int32_t tile_base;            // first restart tile of this launch
  int32_t tile_count;           // restart tiles of this launch (0: all from tile_base)
  int32_t xcd_pin;              // 1: the single pass maps tiles to XCDs (see k_var_pass)
  int32_t stream_items;         // 1: walk each slot's variables as one occurrence list
  const int32_t* occ_own;       // [L] own variable of each slot (two-phase plan)
  const int32_t* var_perm;      // [n] variable processed as the i-th item of the variable
                                // chunks (cost-sorted within each chunk), or null: identity
  float* C;                     // [L][ldD] per-occurrence contributions (two-phase plan)
  const float* x;
  int32_t ldx;
  float* out;                   // next state (update modes) or gradient (grad mode)
  int32_t ldo;
  const float* D;               // stored partials [rows][ldD]
  int64_t ldD;
  float* mom;                   // Adam first moment [n][ldm]
  float* vel;                   // Adam second moment [n][ldm]
  int32_t ldm;
  const float* upstream;        // grad mode: [F*R] or null
  double* loss_part;            // [rows][R] partial sums (row = chunk id)
  int32_t* unsat_part;
  int32_t R;
  float lr;
  float b1, b2, eps;
  double inv_c1, inv_c2;        // Adam bias corrections 1/(1-b^t)
  // flat plan (galsat_flat.hip)
  const int2* pairs;            // [pairs] {other code 1 | own_neg << 31, other code 2}, codes
                                // relative to the first variable of the formula
  const int32_t* pair_first;    // [n] first pair of each variable (first-literal pairs first)
  const int32_t* pair_end;      // [n] end of each variable's pairs
  const int32_t* pair_mid;      // [n] first pair of each variable whose own literal is not first
  const uint32_t* lrec;         // [row records] clause row within the formula
  const int32_t* lrec_ptr;      // [n] first row record: positive own literals first, then negated
  const int32_t* lrec_mid;      // [n] first row record of a negated own literal
  const int32_t* lrec_end;      // [n] end of each variable's row records
  const uint32_t* qrow;         // [clause rows][ldq] packed per-clause products
  int64_t ldq;
  const int32_t* chunk_fvb;     // [chunks] first variable of each variable chunk's formula
  const int32_t* chunk_rbase;   // [chunks] first clause row of each variable chunk's formula
  const int32_t* f_vbeg;        // [F+1]
  const int32_t* f_rbeg;        // [F+1] first clause row of each formula
  int32_t prefetch;             // 1: records of the next batch load during this batch's gathers
};

// Arguments of the clause-parallel pass (forward, and prefix/suffix
// partials for stored clauses).
struct ClausePassArgs {
  const int32_t* clause_ptr;
  const int32_t* clause_lits;
  const int32_t* lit_dslot;     // [L] stored row of each literal position
  const int32_t* clause_ids;    // [list] clause ids, or null for identity
  const int32_t* packed;        // short-clause classes: [list][2][KS] literal codes, then
                                // their D rows (-1 past the clause's end), or null
  const int32_t* chunk_cbeg;    // [chunks] range in the clause list
  const int32_t* chunk_cend;
  const int32_t* chunk_row;     // [chunks] partial-sum row, or null for row = chunk
  const int32_t* chunk_order;   // block -> chunk (-1: the block does nothing), or null
  int32_t chunk_base;
  int32_t tile_base;            // first restart tile of this launch
  int32_t tile_count;           // restart tiles of this launch (0: all from tile_base)
  const float* x;
  int32_t ldx;
  float* D;
  int64_t ldD;
  double* loss_part;
  int32_t* unsat_part;
  int32_t R;
  uint32_t* qrow;               // row pass of the flat plan: [list][ldq] packed clause values
  int64_t ldq;
  const int32_t* rlit_ptr;      // row pass: [list + 1] literals of each listed clause in rlits
  const int32_t* rlits;         // row pass: literal codes relative to the formula (code - 2 vbeg)
  const int32_t* chunk_fvb;     // row pass: [chunks] first variable of the chunk's formula
};

struct FinalizeArgs {
  const int32_t* a_beg;         // [F] partial rows [a_beg, a_end) of each formula
  const int32_t* a_end;
  const int32_t* n_empty;       // [F] empty clauses (U = 1, always unsatisfied)
  const double* loss_part;
  const int32_t* unsat_part;
  float* loss_out;              // [F*R] or null
  int32_t* unsat_out;           // [F*R] or null
  int32_t R;
  int32_t f_base;
  // split > 1: each formula's rows are cut into `split` contiguous parts
  // summed by separate workgroups into part_l / part_u ([F*split][R]), then
  // added in part order by a second kernel (launch_finalize sets these)
  double* part_l;
  int32_t* part_u;
  int32_t split;
  int32_t max_rows;             // most partial rows of one formula (host value; caps split)
};

// Persistent LDS schedule: one workgroup per (formula, restart group) runs
// every step with the group's state in LDS (galsat_persist.hip).
constexpr int kPersistBlock = 512;
struct PersistArgs {
  const int32_t* var_ptr;
  const int4* occ;              // occurrence records (every clause recomputed)
  const int4* occx;
  const int32_t* clause_ptr;
  const int32_t* clause_lits;
  const int32_t* f_vbeg;        // [F+1]
  const int32_t* f_order;       // [F] formula of each workgroup row (LPT order)
  const int32_t* n_empty;       // [F]
  float* x;                     // caller's state [n][ldx], read at the start, written at the end
  int32_t ldx;
  int32_t R;
  int32_t F;
  int32_t steps;
  int32_t nf_max;               // most variables of one formula
  int32_t nocc_max;             // most occurrences of one formula
  int32_t stage_occ;            // 1: records and var_ptr slice copied to LDS per launch
  float lr;
  float* loss_trace;            // [steps][F][R] or null
  int32_t* unsat_trace;
};
size_t persist_lds_bytes(int rg, int nf_max, int nocc_stage);
hipError_t launch_persistent(const PersistArgs& a, int rg, hipStream_t s);

// Workspace of the split finalize: entries of part_l and part_u.
constexpr int64_t kFinalizeScratch = 1024 * 64;

enum VarMode { kModeSGD = 0, kModeAdam = 1, kModeGrad = 2 };

// Short-clause pass: stored clauses of at most this many literals, one
// item per clause with its partials formed in registers.
constexpr int kShortClauseMax = 8;

// Wave-per-clause pass: chunks of G = 64 / lpi literals held in registers,
// and the longest clause it takes for a tile (0: the tile does not use it).
constexpr int wave_clause_chunks(int lpi) { return lpi == 4 ? 13 : 16; }
constexpr int kWaveClauseSmallChunks = 8;  // a second, lighter instance for shorter clauses
inline int wave_clause_kmax(Tile t) {
  return (t.lpi == 4 || t.lpi == 8 || t.lpi == 16) ? (64 / t.lpi) * wave_clause_chunks(t.lpi) : 0;
}

// Plan cache of the autotuner (galsat_tune.hip).
std::string plan_key(const galsat_problem* prob);
bool plan_cache_lookup(const std::string& key, std::string* plan);

// Launchers (galsat_varpass.hip, galsat_twophase.hip, galsat_clause.hip,
// galsat_modes.hip).  All return the launch's hipError_t.
hipError_t launch_var_pass(const VarPassArgs& a, int mode, Tile t, int chunks, hipStream_t s);
hipError_t launch_var_seg(const VarPassArgs& a, Tile t, int chunks, hipStream_t s);
// Two-phase plan: per-occurrence contributions, then per-variable sums.
hipError_t launch_occ_pass(const VarPassArgs& a, Tile t, int chunks, hipStream_t s);
hipError_t launch_var_sum(const VarPassArgs& a, int mode, Tile t, int chunks, hipStream_t s);
hipError_t launch_seg_sum(const VarPassArgs& a, Tile t, int chunks, hipStream_t s);
hipError_t launch_heavy_finish(const VarPassArgs& a, int mode, Tile t, int h0, int h1,
                               hipStream_t s);
// ks: 4 or kShortClauseMax literals; maxc: kWaveClauseSmallChunks or
// wave_clause_chunks(t.lpi) chunks of G literals.
hipError_t launch_wave_clause(const ClausePassArgs& a, Tile t, int maxc, int chunks, hipStream_t s);
hipError_t launch_short_clause(const ClausePassArgs& a, Tile t, int ks, int chunks, hipStream_t s);
hipError_t launch_clause_pass(const ClausePassArgs& a, bool write_d, Tile t, int chunks,
                              hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, int F, hipStream_t s);
// Flat plan (galsat_flat.hip): per-clause rows of every clause that is not
// 3 literals long, then the variable pass (pairs + clause rows) and the
// segments of split variables.
hipError_t launch_row_clause(const ClausePassArgs& a, Tile t, int chunks, hipStream_t s);
hipError_t launch_flat_var(const VarPassArgs& a, int mode, Tile t, int chunks, hipStream_t s);
hipError_t launch_flat_seg(const VarPassArgs& a, Tile t, int chunks, hipStream_t s);
hipError_t launch_init_state(float* x, int32_t ldx, int32_t n, int32_t R, uint64_t seed,
                             hipStream_t s);
hipError_t launch_copy_state(const float* src, int32_t lds, float* dst, int32_t ldd, int32_t n,
                             int32_t R, hipStream_t s);
hipError_t launch_pack_bits(const float* x, int32_t ldx, int32_t n, int32_t R, uint64_t* bits,
                            hipStream_t s);
hipError_t launch_count_unsat(const int32_t* clause_ptr, const int32_t* clause_lits,
                              const int32_t* chunk_cbeg,
                              const int32_t* chunk_cend, const int32_t* order, int blocks,
                              const uint64_t* bits, int32_t n, int32_t R, int32_t* unsat_part,
                              hipStream_t s);
hipError_t launch_best(const int32_t* unsat, int32_t F, int32_t R, int32_t* best, hipStream_t s);
hipError_t launch_best_assign(const uint64_t* bits, int32_t n, const int32_t* var_formula,
                              const int32_t* best, uint8_t* out, hipStream_t s);

hipError_t launch_gumbel_noise(float* out, int32_t ldo, int32_t n, int32_t R, uint64_t seed,
                               int32_t t, hipStream_t s);
hipError_t launch_gumbel_prep(const float* d, int32_t ldd, const float* noise, int32_t ldn,
                              uint64_t seed, int32_t t, int32_t n, int32_t R, float* xh, float* nb,
                              int32_t ld, hipStream_t s);
hipError_t launch_gumbel_update(float* d, int32_t ldd, const float* nb, const float* G, int32_t ld,
                                float* mom, float* vel, int32_t ldm, int32_t n, int32_t R, float tau,
                                float lr, float b1, float b2, float eps, double inv_c1,
                                double inv_c2, int32_t adam, hipStream_t s);
hipError_t launch_candidates(const float* d, int32_t ldd, const int32_t* var_formula,
                             const int32_t* best, int32_t n, int32_t num, uint64_t seed, float tau,
                             uint8_t* assign, float* conf, hipStream_t s);
hipError_t launch_confidence(const float* d, int32_t ldd, const int32_t* var_formula,
                             const int32_t* best, int32_t n, float tau, float* conf, hipStream_t s);
hipError_t launch_select(const float* conf, int32_t n, int32_t F, const int32_t* f_vbeg,
                         const int32_t* sel_off, int32_t stot, int32_t num, bool highest,
                         int32_t* out, hipStream_t s);
hipError_t launch_zero_i32(int32_t* p, int64_t count, hipStream_t s);

}  // namespace galsat
