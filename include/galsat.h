/*
 * galsat.h -- C ABI of libgalsat: gradient descent on the relaxed algebraic
 * encoding of CNF formulas, on one AMD Instinct MI355X (gfx950).
 *
 * Method (GaloisSAT, Section 3.2 "Differentiable SAT Formulation"):
 *   Eq. (1) NOT x = 1 - x, x AND y = x*y, x OR y = x + y - x*y;
 *   Eq. (2) a clause of literals with truth values s_i evaluates to
 *           C = 1 - prod_i (1 - s_i), exactly its satisfaction at 0/1 points;
 *   Eq. (5) the loss is L = -sum_t C_t.
 * The library evaluates, for a batch of R relaxed assignments ("restarts",
 * the paper's batch dimension B of independent random initialisations)
 * per formula:
 *   loss'[f][r] = sum_{t in f} U_t,  U_t = prod_i (1 - s_i) = 1 - C_t,
 * which is m_f + L (zero exactly on satisfying 0/1 points; same gradient),
 * its gradient with respect to every x[v][r], a fused projected-gradient
 * (or Adam, as in the paper's appendix "Experiment Setup") update, and the
 * exact number of unsatisfied clauses of the rounded assignment
 * x_hat = [x > 0.5] (a tie at 0.5 rounds to 0, the first maximal index of
 * the argmax of Eq. (4) over the pair (1 - x, x)).
 *
 * Conventions shared by every call
 *   - Literal code: code = 2*v + neg (neg = 1 for a negated literal), v a
 *     0-based global variable id.  A negated literal's clause factor is
 *     x_v, a positive literal's is 1 - x_v.
 *   - State x: FP32, variable-major [n][ldx] with the R restarts of a
 *     variable contiguous; ldx >= R.  Values outside [0,1] are accepted by
 *     galsat_loss_grad; galsat_step keeps x inside [0,1].
 *   - Per-(formula, restart) outputs are laid out [F][R] (index f*R + r).
 *   - Every pointer to state, gradient and output arrays is a DEVICE pointer
 *     owned by the caller (for example a torch tensor's data_ptr()); the
 *     library never frees it.
 *   - Calls are asynchronous and ordered on the HIP stream passed in
 *     (hipStream_t as void*; NULL = the default stream).  Outputs are valid
 *     once that stream has been synchronised.
 *   - Results are deterministic: for a given handle and inputs every output
 *     is bitwise reproducible (no floating-point atomics anywhere).
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Errors: every call returns galsat_status.  Argument and CSR
 *     validation errors are reported synchronously and leave the handle
 *     usable.  A device error (a failed launch or allocation) is sticky: the
 *     handle then fails every later call with GALSAT_EDEVICE.
 *     galsat_last_error() gives a message for the most recent failure.
 */
#ifndef GALSAT_H
#define GALSAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GALSAT_OK = 0,
  GALSAT_EINVAL = -1,       /* bad argument or malformed CSR */
  GALSAT_ENOMEM = -2,       /* device allocation failed or workspace budget too small */
  GALSAT_EDEVICE = -3,      /* HIP runtime error (sticky on the handle) */
  GALSAT_EOVERFLOW = -4,    /* a size does not fit the int32 CSR or the index range */
  GALSAT_EUNSUPPORTED = -5  /* valid request the library does not implement */
} galsat_status;

typedef struct galsat_ctx* galsat_handle;

/* A batch of F independent CNF formulas in both CSR orientations.
 * Formula f owns the contiguous variable ids [formula_var_begin[f],
 * formula_var_begin[f+1]) and clauses [formula_clause_begin[f],
 * formula_clause_begin[f+1]); every literal of a clause must name a
 * variable of the clause's formula.
 *
 *   clause_ptr [m+1]  clause-major offsets: clause t owns literal positions
 *                     [clause_ptr[t], clause_ptr[t+1]) of clause_lits;
 *                     clause_ptr[0] = 0, non-decreasing, clause_ptr[m] = L.
 *                     Empty clauses (U = 1, always unsatisfied, no
 *                     gradient), repeated variables and complementary
 *                     literals inside one clause are all accepted.
 *   clause_lits [L]   literal codes.
 *   var_ptr [n+1]     variable-major offsets into var_occ.
 *   var_occ [L]       for variable v, the positions p of clause_lits with
 *                     clause_lits[p] >> 1 == v: exactly the transpose of the
 *                     clause-major CSR, every position exactly once.  The
 *                     order inside a variable is the order in which the
 *                     single-pass and two-phase plans sum its gradient
 *                     contributions; the flat plan sums them in its own
 *                     fixed order (first-literal pairs, the other pairs,
 *                     then clause rows).
 * All arrays are int32; L < 2^31.  With inputs_on_device = 0 they are host
 * pointers, with 1 device pointers.  galsat_create copies them: the caller
 * may free or reuse them as soon as it returns.
 */
typedef struct {
  int32_t num_formulas;                 /* F >= 1 */
  const int32_t* formula_var_begin;     /* [F+1]; may be NULL when F == 1 */
  const int32_t* formula_clause_begin;  /* [F+1]; may be NULL when F == 1 */
  int32_t n_vars;                       /* n >= 0 (total over formulas) */
  int32_t n_clauses;                    /* m >= 0 */
  int32_t n_lits;                       /* L >= 0 */
  const int32_t* clause_ptr;
  const int32_t* clause_lits;
  const int32_t* var_ptr;
  const int32_t* var_occ;
  int32_t restarts;                     /* R >= 1, the same for every formula */
  int32_t inputs_on_device;
} galsat_problem;

enum { GALSAT_OPT_SGD_CLAMP = 0, GALSAT_OPT_ADAM = 1 };

/* How the backward obtains each literal's partial derivative
 * prod_{i != j} (1 - s_i):
 *   STORE      clause-parallel passes form them from prefix and suffix
 *              products and store them; a variable-parallel pass sums
 *              them in var_occ order.
 *   RECOMPUTE  the variable-parallel side recomputes them from x, so no
 *              per-literal or per-clause values are kept between passes.
 *   AUTO       the plan's choice, within workspace_budget_bytes: with at
 *              most 64 restarts the flat gradient (3-literal clauses
 *              recompute from x; every other clause is reduced once per
 *              step to a per-clause row holding the product of its nonzero
 *              factors and its count of zero factors, from which each
 *              occurrence's partial follows by one division); with more
 *              restarts the single-pass gradient, where clauses up to
 *              recompute_max_len literals (default 8) recompute and longer
 *              ones store; with an explicit two-phase gradient (plan key
 *              two=1), every clause stores, unless recompute_max_len is set.
 *              Sums run in a fixed order in every plan. */
enum { GALSAT_PARTIALS_AUTO = 0, GALSAT_PARTIALS_STORE = 1, GALSAT_PARTIALS_RECOMPUTE = 2 };

/* Execution schedule of galsat_step:
 *   GENERAL  multi-kernel passes per step over all formulas at once (the
 *            formulas' work items share every launch);
 *   LDS      one persistent launch runs every step: one workgroup per
 *            (formula, restart group) with that group's state double-
 *            buffered in LDS, and the formula's occurrence records too when
 *            they fit.  For small formulas (12 bytes per variable of the
 *            largest formula within 64 KB of LDS: up to about 5,400
 *            variables); projected SGD only, every clause recomputed.
 *            galsat_create returns GALSAT_EUNSUPPORTED otherwise.  States and
 *            unsat counts equal GENERAL's with every clause recomputed and
 *            the single-pass gradient bitwise (no variable split); the loss
 *            trace is summed in another fixed order.  The other entry points
 *            run the general passes;
 *   PLAIN    one formula at a time, kernels launched per pass per step
 *            (the reference point for batching, not a fast path);
 *   AUTO     GENERAL. */
enum { GALSAT_SCHED_AUTO = 0, GALSAT_SCHED_GENERAL = 1, GALSAT_SCHED_LDS = 2,
       GALSAT_SCHED_PLAIN = 3 };

typedef struct {
  int32_t optimizer;         /* GALSAT_OPT_*; default SGD_CLAMP */
  float lr;                  /* default 0.1 */
  float beta1, beta2, eps;   /* Adam only; defaults 0.9, 0.999, 1e-8 */
  int32_t partials;          /* GALSAT_PARTIALS_*; default AUTO */
  int32_t recompute_max_len; /* AUTO threshold in literals; 0 = library default */
  size_t workspace_budget_bytes; /* cap on stored partials; 0 = no cap */
  int32_t validate;          /* 1 (default): also check that var_occ is a permutation */
  int32_t schedule;          /* GALSAT_SCHED_*; default AUTO */
  int32_t use_graph;         /* 1: galsat_step replays a captured hipGraph (GENERAL) */
  const char* plan_override; /* NULL, or comma-separated key=value pairs:
                              lpi lanes per item (4..64), rpl restarts per lane (1, 2,
                              4), krec recompute threshold, tg restart tiles per launch,
                              xcdc chunks per formula of the XCD-aware order (0: off),
                              stream (1: streaming variable pass), two (1: two-phase
                              gradient, 0: single pass), dsort / csort (cost-sorted
                              variable items / length-sorted stored clauses, 0 or 1),
                              wave / short (0: no wave-per-clause / short-clause pass),
                              xseq (one formula: chunks of the XCD-contiguous order,
                              0: off), segdiv (heavy-variable split divisor), ldsrg
                              (LDS schedule: restarts per workgroup, 1, 2, 4, 8, 16 or
                              32), ldsstage (0: the LDS schedule reads the records from
                              global memory), ldslpt (0: the LDS schedule issues
                              formulas in index order, not LPT order), xpin (1: the
                              single pass maps restart tiles to XCDs by linear block
                              id, 0: off; on by default for one formula with at least
                              1,024 restarts), flat (1: the flat gradient, 0: not; on by
                              default for at most 64 restarts with AUTO partials and no
                              two= or krec= key), and for the flat plan pf (1/0: records
                              of the next batch loaded during the current one's
                              gathers; on by default from 24 occurrences per variable),
                              rsort (1/0: a variable's clause-row records in row order,
                              default 1), sord (1/0: split-variable segments run in
                              the order of the first clause row they read, default 1)
                              and psort (1/0: a variable's pair records in the order
                              of their nearer partner variable, default 1).
                              Keys left out take the plan's own choice. */
} galsat_options;

/* Fills *opt with the defaults listed above. */
void galsat_default_options(galsat_options* opt);

/* Validates and copies the problem to the device, derives the occurrence
 * tables the kernels use, chooses a plan and allocates its workspace.
 * The input is a CNF formula as the paper's SAT background subsection
 * defines it (a conjunction of clauses, each a disjunction of literals) in
 * both CSR orientations,
 * and the restart count is the batch dimension B of Section 3.2 (independent
 * random initialisations optimised together).
 * stream: used for the uploads (synchronised before returning).
 * On success *out holds a new handle; on failure *out is NULL and the
 * message is available from galsat_last_error(NULL). */
galsat_status galsat_create(const galsat_problem* prob, const galsat_options* opt, void* stream,
                            galsat_handle* out);

/* Frees all device memory, graphs and the handle.  NULL is accepted. */
galsat_status galsat_destroy(galsat_handle h);

/* Relaxed initial state (the paper initialises each batch element
 * independently at random, Section 3.2): x[v][r] = (hash >> 40) * 2^-24 with
 * hash = SplitMix64mix(seed XOR SplitMix64mix(v * 2^32 + r + 0x9e3779b97f4a7c15)),
 * uniform on a 2^-24 grid in [0, 1).  Writes x[n][ldx] for r < R. */
galsat_status galsat_init_state(galsat_handle h, float* x, int32_t ldx, uint64_t seed,
                                void* stream);

/* Forward and (optionally) backward at x (Eq. 2 and Eq. 5).
 *   x        device FP32 [n][ldx], read only.
 *   loss     device FP32 [F*R]: loss'[f][r] (required).
 *   grad     device FP32 [n][ldx] or NULL (loss only).  When given:
 *            grad[v][r] = w[f(v)][r] * d loss'[f(v)][r] / d x[v][r] with
 *            w = upstream, or 1 when upstream is NULL (autograd backward).
 *   upstream device FP32 [F*R] or NULL.
 * Entries grad[v][r] for r >= R are not written. */
galsat_status galsat_loss_grad(galsat_handle h, const float* x, int32_t ldx, const float* upstream,
                               float* loss, float* grad, void* stream);

/* `steps` iterations of gradient descent on the relaxed loss (Section 3.2:
 * clause value of Eq. (2) with the negation of Eq. (1), the clause-sum loss
 * of Eq. (5) shifted by the clause count, and its gradient by
 * backpropagation through the clause products).  Each iteration is
 * evaluated at the current x_k with every variable updated from the same
 * gradient (Jacobi):
 *   SGD_CLAMP  x_{k+1} = min(1, max(0, x_k - lr * g_k))
 *   ADAM       the optimizer of the appendix "Experiment Setup" (there
 *              with lr 0.5): m, v moments and bias correction at the
 *              handle's step counter t (starting at 1, advanced once per
 *              step), then the same clamp.  opt_state: device FP32 [2][n][ldx] (m then v),
 *              zero before the first step; NULL for SGD.
 * x is updated in place.  loss_trace ([steps][F*R] FP32) and unsat_trace
 * ([steps][F*R] int32), each optional, receive loss'(x_k) and the exact
 * unsatisfied-clause count of round(x_k) for every step k. */
galsat_status galsat_step(galsat_handle h, float* x, int32_t ldx, float* opt_state, int32_t steps,
                          float* loss_trace, int32_t* unsat_trace, void* stream);

/* For a handle created with use_graph: captures and instantiates the graph
 * of galsat_step with exactly these arguments without running it, so the
 * next galsat_step call with the same arguments only replays it.  Returns
 * GALSAT_EUNSUPPORTED when the call would run eagerly (no use_graph, Adam,
 * or profiling enabled); with the LDS schedule (a single launch already)
 * it does nothing. */
galsat_status galsat_step_prepare(galsat_handle h, float* x, int32_t ldx, float* opt_state,
                                  int32_t steps, float* loss_trace, int32_t* unsat_trace);

/* Straight-through Gumbel-softmax training, the paper's own optimizer loop
 * (Section 3.2, Eq. 3-5; appendix "Experiment Setup": Adam, lr 0.5,
 * tau 1.0).  Each (variable, restart) has two logits theta0, theta1; with
 * two states the softmax of Eq. (3) depends only on d = theta1 - theta0 and
 * on the noise difference l = g1 - g0 (g_j i.i.d. Gumbel(0,1)):
 *   y1 = sigma((d + l) / tau),   forward at x_hat = [d + l > 0]   (Eq. 4,
 *   a tie goes to state 0, taken in FP32),
 * loss' and the unsat count are evaluated at x_hat (both equal the number
 * of unsatisfied clauses there), and the straight-through backward sends
 * g1 = G * y1 (1 - y1) / tau to theta1 and -g1 to theta0, G being the
 * polynomial gradient at x_hat.  The handle's optimizer updates theta1 and
 * theta0 with these gradients; the state kept is d, which moves by twice
 * theta1's step (SGD: d -= 2 lr g1; Adam: theta0's moments are the exact
 * negatives of theta1's, so opt_state [2][n][ldd] holds theta1's m and v).
 * No clamp.  The noise difference for global step t (= step0 + k) is drawn
 * from a counter-based generator; g1 - g0 of independent Gumbel(0,1) draws
 * is standard logistic, so l is drawn directly from one uniform:
 *   l = log(u / (1 - u)), u = ((h >> 40) + 0.5) * 2^-24,
 *   h = M(seed ^ M(c ^ M(t + 0x632be59bd9b4e019))), c = v * 2^32 + r,
 * M the SplitMix64 output mix, evaluated in FP64 and rounded to FP32 once;
 * or, when `noise` is not NULL, read from it ([steps][n][ldd] FP32 l values).
 *   d            device FP32 [n][ldd], updated in place
 *   loss_trace   device FP32 [steps][F*R] or NULL; unsat_trace int32, same */
galsat_status galsat_gumbel_step(galsat_handle h, float* d, int32_t ldd, float* opt_state,
                                 uint64_t seed, int32_t step0, int32_t steps, float tau,
                                 const float* noise, float* loss_trace, int32_t* unsat_trace,
                                 void* stream);

/* The noise differences l of global step `step` that galsat_gumbel_step
 * draws: device FP32 [n][ldn], r < R written. */
galsat_status galsat_gumbel_noise(galsat_handle h, uint64_t seed, int32_t step, float* noise,
                                  int32_t ldn, void* stream);

/* Hand-off to the CPU stage (Section 3.3).  Candidate pool, Eq. (8): for
 * candidate k = 0 .. num-1 and every variable v of formula f, with
 * r = best_restart[f] and l the noise difference of step k, restart 0 of
 * the generator described at galsat_gumbel_step,
 *   assign[k][v] = [d[v][r] + l > 0]            (FP32, tie -> 0)
 *   conf[k][v]   = probability of that value under sigma((d + l) / tau).
 *   d            device FP32 [n][ldd] (logit differences, or any score whose
 *                sigmoid is the probability of the value 1)
 *   best_restart device int32 [F]
 *   assign       device uint8 [num][n];  conf  device FP32 [num][n] */
galsat_status galsat_candidates(galsat_handle h, const float* d, int32_t ldd,
                                const int32_t* best_restart, int32_t num, uint64_t seed, float tau,
                                uint8_t* assign, float* conf, void* stream);

/* Unperturbed confidence of the selected restart, for choosing branching
 * variables (Section 3.3.2): conf[v] = max(p, 1 - p), p = sigma(d[v][r] / tau),
 * r = best_restart[f(v)].  conf: device FP32 [n]. */
galsat_status galsat_confidence(galsat_handle h, const float* d, int32_t ldd,
                                const int32_t* best_restart, float tau, float* conf, void* stream);

/* Per formula f and row k of conf ([num][n], device FP32), selects the
 * S_f = min(n_f, max(min_count, ceil(frac * n_f))) most confident
 * (highest = 1: the unit clauses of Eq. 9-10, frac 0.0005 in the appendix)
 * or least confident (highest = 0, frac 0, min_count = d: the branching
 * variables of Lemma 1, d = 7 in the appendix) variables, ties to the lower
 * variable id, and writes their global ids in increasing order to
 * out[k][offsets[f] .. offsets[f+1]).  offsets: HOST int32 [F+1], always
 * filled (synchronously); out: device int32 [num][offsets[F]], or NULL to
 * query the sizes only.  The call synchronises `stream` once (it uploads the
 * offsets table). */
galsat_status galsat_select_vars(galsat_handle h, const float* conf, int32_t num, int32_t highest,
                                 float frac, int32_t min_count, int32_t* offsets, int32_t* out,
                                 void* stream);

/* Rounds x (x > 0.5 -> 1; an x that is already 0/1 is used as given; the
 * argmax of Eq. (4) over the pair (1 - x, x) with a tie to 0), counts
 * unsatisfied clauses exactly per (formula, restart) with wavefront ballot
 * and popcount (a clause is unsatisfied when every literal is false, the
 * 0/1 reading of Eq. (2)), and picks per formula the restart with the
 * fewest (ties to the lowest restart index): the hand-off of the GPU stage
 * to the CPU stage (architecture overview, Section 3.1, and Section 3.3:
 * the batch of minimal clause loss is the one passed on).
 *   unsat        device int32 [F*R]
 *   best_restart device int32 [F] or NULL
 *   best_assign  device uint8 [n] or NULL: the rounded assignment of each
 *                variable in its formula's best restart. */
galsat_status galsat_round_check(galsat_handle h, const float* x, int32_t ldx, int32_t* unsat,
                                 int32_t* best_restart, uint8_t* best_assign, void* stream);

/* Allocation-free variant of galsat_round_check, for callers that cannot
 * allocate device memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and kernels as galsat_round_check; its scratch (the rounding
 * bit-planes, the per-chunk unsat rows, the finalize part sums and, when
 * best_restart is NULL, the best restart) lives in a fixed 64 MiB device
 * array of the library instead of the handle's workspace, so the call
 * makes no hipMalloc, hipFree or other allocating call.  The array is
 * per GPU and held until the process ends; its address is looked up once
 * per device on the first call there.
 *   Limit: 8*n*ceil(R/64) + 4*R*(clause chunks) + 786,432 + 4*F bytes
 *   (each part rounded up to 256) must fit 64 MiB, else GALSAT_EOVERFLOW
 *   with a message giving the size needed.
 *   Must be called with the handle's device current (else GALSAT_EINVAL).
 *   Every call on one GPU shares that GPU's array: calls that overlap in
 *   time on one GPU (other streams, other threads, other handles) race and
 *   must be serialised by the caller.  Nothing in the array needs to carry
 *   over between calls (each call overwrites what it reads). */
galsat_status galsat_round_check_static(galsat_handle h, const float* x, int32_t ldx,
                                        int32_t* unsat, int32_t* best_restart,
                                        uint8_t* best_assign, void* stream);

/* Sets the Adam step counter (the next step uses t + 1); 0 restarts the bias
 * correction.  For checkpoint and resume. */
galsat_status galsat_set_adam_step(galsat_handle h, int32_t t);

/* Plan autotuner.  With at most 64 restarts and AUTO partials (no
 * recompute_max_len) the candidates are the flat gradient with and without
 * record prefetch, with 20 and 80 chunks per formula for batches, and the
 * two-phase gradient.  Otherwise it derives candidate plans from the
 * restart count (lanes per item and restarts per lane), the clause-length
 * histogram (recompute threshold when clauses longer than 8 literals
 * exist), the formula count (chunks per formula of the XCD-aware order)
 * and, for at most 64 restarts, single pass against two-phase gradient;
 * with the LDS schedule
 * instead its restarts per workgroup (1 to 32, up to the restarts rounded
 * to a power of two), records staged or not; creates a handle for
 * each, times `steps` steps of galsat_step from a copy of x0 with HIP
 * events on `stream`, and writes the fastest plan as a plan_override string
 * to plan_out (host, plan_cap >= 64 bytes) and its time per step to
 * *best_ms (may be NULL).  x0: device FP32 [n][ldx], not modified.  When the
 * environment variable GALSAT_PLAN_CACHE names a file, the result is
 * appended to it ("<shape key> | <plan>"), and galsat_create called without
 * plan_override uses the plan recorded for the problem's shape. */
galsat_status galsat_autotune(const galsat_problem* prob, const galsat_options* opt,
                              const float* x0, int32_t ldx, int32_t steps, void* stream,
                              char* plan_out, int32_t plan_cap, double* best_ms);

/* Plan and size information (host values). */
typedef struct {
  int32_t num_formulas, n_vars, n_clauses, n_lits, restarts;
  int32_t max_clause_len;
  int32_t recompute_max_len;    /* clauses up to this length recompute partials */
  int64_t stored_lits;          /* literal occurrences whose partials are stored */
  int32_t schedule;             /* schedule galsat_step uses (GALSAT_SCHED_*) */
  int32_t lanes_per_item;       /* restarts lanes of one variable or clause */
  int32_t restarts_per_lane;
  int32_t var_chunks, clause_chunks;
  int32_t two_phase;            /* 1: two-phase gradient (clause passes + variable sums) */
  int32_t xseq_chunks;          /* chunks of the XCD-contiguous order of one formula, 0: off */
  size_t device_bytes;          /* device memory held by the handle */
  int32_t adam_step;
  int32_t lds_restarts_per_group; /* LDS schedule: restarts per workgroup, 0: not used */
  int32_t lds_staged;           /* LDS schedule: 1 when the records are copied to LDS */
  int32_t flat;                 /* 1: flat gradient (3-literal clauses recomputed from pair
                                   records, every other clause through a per-clause row) */
  int32_t clause_rows;          /* flat gradient: clauses reduced to a per-clause row */
} galsat_info;

galsat_status galsat_get_info(galsat_handle h, galsat_info* info);

/* Per-kernel timing.  While profiling is enabled on a handle, every kernel
 * launch of the handle is bracketed by a pair of HIP events recorded on the
 * stream of the call, so each duration is that kernel's own time on its
 * stream.  galsat_profile(h, 1) clears the record and starts it;
 * galsat_profile(h, 0) stops it.  galsat_kernel_times synchronises the
 * recorded events and returns, per kernel kind, the number of launches and
 * their summed duration in milliseconds. */
enum {
  GALSAT_K_VAR_PASS = 0,     /* variable-parallel gather + fused update / gradient */
  GALSAT_K_CLAUSE_PASS = 1,  /* clause-parallel forward and stored partials (flat plan: the
                                clause-row pass) */
  GALSAT_K_FINALIZE = 2,     /* fixed-order reduction of per-chunk partial sums */
  GALSAT_K_COPY = 3,         /* state copy between the caller's and internal layouts */
  GALSAT_K_PACK = 4,         /* rounding bit-pack (ballot) */
  GALSAT_K_COUNT = 5,        /* unsat count (ballot + popcount) */
  GALSAT_K_SELECT = 6,       /* best restart and its assignment */
  GALSAT_K_OCC_PASS = 7,     /* two-phase plan: occurrence-parallel contributions */
  GALSAT_K_VAR_SUM = 8,      /* two-phase plan: per-variable sums + fused update */
  GALSAT_K_SEG_PASS = 9,     /* partial gradients of the segments of split variables */
  GALSAT_K_HEAVY = 10,       /* split variables: fixed-order sum of their segments + update */
  GALSAT_K_KINDS = 11
};

typedef struct {
  int32_t launches[GALSAT_K_KINDS];
  double total_ms[GALSAT_K_KINDS];
} galsat_kernel_stats;

galsat_status galsat_profile(galsat_handle h, int32_t enable);
galsat_status galsat_kernel_times(galsat_handle h, galsat_kernel_stats* out);

/* Clause normalization to a fixed width (Section 3.2, "Clause Normalization
 * for Vectorization", Eq. 6-7), host code, no device involved.
 * A clause longer than `width` (>= 3) becomes a chain of width-literal
 * clauses linked by fresh auxiliary variables: the first link holds the
 * first width-1 literals and f1, each middle link ~f_i, width-2 literals and
 * f_{i+1}, the last link ~f_last and the remaining literals; for width 3
 * this is Eq. (6).  Shorter clauses (and a short last link) are padded by
 * repeating their last literal; empty clauses stay empty.  Auxiliary
 * variables get ids n_vars, n_vars+1, ... in order of creation, so original
 * variables keep theirs.  Inputs: host int32 clause-major CSR
 * (clause_ptr [n_clauses+1], clause_lits, codes 2*v+neg).  Call once with
 * out_clause_ptr / out_clause_lits NULL to get the output sizes, then again
 * with host buffers of [out_n_clauses+1] and [out_n_lits] entries. */
galsat_status galsat_tseitin(int32_t width, int32_t n_vars, int32_t n_clauses,
                             const int32_t* clause_ptr, const int32_t* clause_lits,
                             int32_t* out_n_vars, int32_t* out_n_clauses, int32_t* out_n_lits,
                             int32_t* out_clause_ptr, int32_t* out_clause_lits);

/* Static description of a status code. */
const char* galsat_status_string(galsat_status s);

/* Message for the most recent failure on h (or of galsat_create when h is
 * NULL); "" if none.  Valid until the next call on the same handle. */
const char* galsat_last_error(galsat_handle h);

#ifdef __cplusplus
}
#endif

#endif /* GALSAT_H */
