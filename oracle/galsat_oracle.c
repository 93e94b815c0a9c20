/*
 * galsat_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what the relaxed-CNF gradient
 * descent computes.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code with the HIP library: it reads the clause-major CSR
 * only, keeps the state restart-major (x[r][v]) and parallelises over
 * restarts only.
 *
 * Paper: GaloisSAT, Section 3.2 "Differentiable SAT Formulation".
 *   Eq. (1)  Boolean operations as polynomials: NOT x = 1 - x, x AND y = x*y,
 *            x OR y = x + y - x*y.
 *   Eq. (2)  a clause of u literals with truth values s_i evaluates to
 *            C = 1 - prod_i (1 - s_i); at 0/1 points C is exactly the clause's
 *            satisfaction.
 *   Eq. (5)  loss L = -sum_t C_t (MaxSAT objective: no product over clauses).
 *
 * Readings taken where the paper is silent or leaves a choice open:
 *   - the state is the relaxed point x in [0,1] (literal truth s = x for a
 *     positive literal, 1 - x for a negated one) and the forward is evaluated
 *     at x itself;
 *   - the reported loss is loss' = sum_t U_t with U_t = prod_i (1 - s_i)
 *     = 1 - C_t, i.e. loss' = m + L: zero exactly on satisfying 0/1 points,
 *     same gradient as L;
 *   - an empty clause has U = 1 (empty product): always unsatisfied;
 *   - repeated variables inside a clause are kept as written (factor powers);
 *   - rounding x_hat = [x > 0.5] (a tie at 0.5 goes to 0, the first maximal
 *     index of the argmax of Eq. (4) over the state pair (1-x, x));
 *   - projected gradient descent x <- clamp(x - lr*g, 0, 1) is the default
 *     update; Adam (appendix "Experiment Setup": Adam, learning rate 0.5)
 *     with bias correction and PyTorch's default beta1, beta2, eps is the
 *     option, followed by the same clamp;
 *   - the hand-off restart of a formula is the one with the fewest
 *     unsatisfied clauses after rounding, ties to the lowest restart index.
 *
 * Literal code: code = 2*v + neg (neg = 1 for a negated literal).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Clause factor (1 - s) of Eq. (2) for one literal, s its truth value.
 * Positive literal: s = x, factor 1 - x.  Negated literal: s = 1 - x by the
 * negation rule of Eq. (1), factor 1 - (1 - x) = x, written out exactly. */
static double factor(int32_t code, const double* xr) {
  double xv = xr[code >> 1];
  return (code & 1) ? xv : 1.0 - xv;
}

/* d(factor)/dx_v: -1 for a positive literal, +1 for a negated one. */
static double factor_slope(int32_t code) { return (code & 1) ? 1.0 : -1.0; }

/* U_t = prod over the clause's literals of (1 - s_i)  (Eq. 2: C_t = 1 - U_t). */
double oracle_clause_U(int32_t k, const int32_t* codes, const double* xr) {
  double u = 1.0;
  for (int32_t i = 0; i < k; ++i) u *= factor(codes[i], xr);
  return u;
}

/* loss'[f*R + r] = sum over the clauses t of formula f of U_t at x[r]
 * (Eq. 5 shifted by the clause count: loss' = m_f + L).  Summed in clause
 * order in FP64. */
void oracle_loss(int32_t n, int32_t F, const int32_t* fcb, const int32_t* cptr,
                 const int32_t* lits, int32_t R, const double* x, double* loss) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t r = 0; r < R; ++r) {
    const double* xr = x + (int64_t)r * n;
    for (int32_t f = 0; f < F; ++f) {
      double s = 0.0;
      for (int64_t t = fcb[f]; t < fcb[f + 1]; ++t)
        s += oracle_clause_U(cptr[t + 1] - cptr[t], lits + cptr[t], xr);
      loss[(int64_t)f * R + r] = s;
    }
  }
}

/* Gradient of loss' with respect to every x[r][v] (backpropagation through
 * Eq. 2): for literal j of clause t, dU_t/dx_v = slope_j * prod_{i != j} a_i.
 * The per-occurrence products come from left and right running products of
 * the clause's factors (O(k) per clause; no division, so exact zero factors
 * are handled as they come).  Contributions are added in clause order.
 * absg[r][v] (optional) receives sum |dU_t/dx_v|, the conditioning scale of
 * the gradient's signed sum.  loss (optional) as in oracle_loss. */
void oracle_grad(int32_t n, int32_t F, const int32_t* fcb, const int32_t* cptr,
                 const int32_t* lits, int32_t R, const double* x, double* loss, double* grad,
                 double* absg) {
  int32_t kmax = 0;
  for (int64_t t = 0; t < fcb[F]; ++t)
    if (cptr[t + 1] - cptr[t] > kmax) kmax = cptr[t + 1] - cptr[t];
#pragma omp parallel
  {
    double* left = (double*)malloc(sizeof(double) * (size_t)(kmax + 1));
    double* a = (double*)malloc(sizeof(double) * (size_t)(kmax + 1));
#pragma omp for schedule(dynamic, 1)
    for (int32_t r = 0; r < R; ++r) {
      const double* xr = x + (int64_t)r * n;
      double* gr = grad + (int64_t)r * n;
      double* ar = absg ? absg + (int64_t)r * n : NULL;
      memset(gr, 0, sizeof(double) * (size_t)n);
      if (ar) memset(ar, 0, sizeof(double) * (size_t)n);
      for (int32_t f = 0; f < F; ++f) {
        double s = 0.0;
        for (int64_t t = fcb[f]; t < fcb[f + 1]; ++t) {
          const int32_t k = cptr[t + 1] - cptr[t];
          const int32_t* c = lits + cptr[t];
          /* left[j] = prod_{i<j} a_i */
          left[0] = 1.0;
          for (int32_t j = 0; j < k; ++j) {
            a[j] = factor(c[j], xr);
            left[j + 1] = left[j] * a[j];
          }
          s += left[k];
          /* right running product prod_{i>j} a_i, walked from the end */
          double right = 1.0;
          for (int32_t j = k - 1; j >= 0; --j) {
            const double others = left[j] * right;
            gr[c[j] >> 1] += factor_slope(c[j]) * others;
            if (ar) ar[c[j] >> 1] += fabs(others);
            right *= a[j];
          }
        }
        if (loss) loss[(int64_t)f * R + r] = s;
      }
    }
    free(left);
    free(a);
  }
}

/* The same gradient from the definition: for every occurrence (t, j) the
 * product over i != j is formed by its own loop (O(k^2) per clause). */
void oracle_grad_def(int32_t n, int32_t F, const int32_t* fcb, const int32_t* cptr,
                     const int32_t* lits, int32_t R, const double* x, double* grad) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t r = 0; r < R; ++r) {
    const double* xr = x + (int64_t)r * n;
    double* gr = grad + (int64_t)r * n;
    memset(gr, 0, sizeof(double) * (size_t)n);
    for (int64_t t = 0; t < fcb[F]; ++t) {
      const int32_t k = cptr[t + 1] - cptr[t];
      const int32_t* c = lits + cptr[t];
      for (int32_t j = 0; j < k; ++j) {
        double others = 1.0;
        for (int32_t i = 0; i < k; ++i)
          if (i != j) others *= factor(c[i], xr);
        gr[c[j] >> 1] += factor_slope(c[j]) * others;
      }
    }
  }
}

/* Central finite difference of loss' in x[r][v] for the listed variables,
 * restricted to the clauses that contain v (all other clauses cancel
 * exactly): (sum_{t ni v} U_t(x + h e_v) - U_t(x - h e_v)) / (2h).
 * out[r*nv + i] for variable vars[i].  The clauses containing each listed
 * variable are found by one scan of the clause-major CSR. */
void oracle_fd_grad(int32_t n, int32_t m, const int32_t* cptr, const int32_t* lits, int32_t R,
                    const double* x, int32_t nv, const int32_t* vars, double h, double* out) {
#pragma omp parallel
  {
    double* xp = (double*)malloc(sizeof(double) * (size_t)n);
    int64_t cap = 64;
    int64_t* tl = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(dynamic, 1)
    for (int32_t i = 0; i < nv; ++i) {
      const int32_t v = vars[i];
      int64_t cnt = 0;
      for (int64_t t = 0; t < m; ++t) {
        int has = 0;
        for (int32_t p = cptr[t]; p < cptr[t + 1]; ++p)
          if ((lits[p] >> 1) == v) has = 1;
        if (!has) continue;
        if (cnt == cap) {
          cap *= 2;
          tl = (int64_t*)realloc(tl, sizeof(int64_t) * (size_t)cap);
        }
        tl[cnt++] = t;
      }
      for (int32_t r = 0; r < R; ++r) {
        memcpy(xp, x + (int64_t)r * n, sizeof(double) * (size_t)n);
        const double x0 = xp[v];
        double up = 0.0, dn = 0.0;
        for (int64_t c = 0; c < cnt; ++c) {
          const int64_t t = tl[c];
          const int32_t k = cptr[t + 1] - cptr[t];
          xp[v] = x0 + h;
          up += oracle_clause_U(k, lits + cptr[t], xp);
          xp[v] = x0 - h;
          dn += oracle_clause_U(k, lits + cptr[t], xp);
        }
        xp[v] = x0;
        out[(int64_t)r * nv + i] = (up - dn) / (2.0 * h);
      }
    }
    free(tl);
    free(xp);
  }
}

/* Projected gradient descent: x <- min(1, max(0, x - lr*g)) for every
 * (r, v) simultaneously from the same g. */
void oracle_step_sgd(int64_t count, double lr, double* x, const double* g) {
  for (int64_t i = 0; i < count; ++i) {
    double y = x[i] - lr * g[i];
    if (y < 0.0) y = 0.0;
    if (y > 1.0) y = 1.0;
    x[i] = y;
  }
}

/* Adam (Kingma & Ba) with bias correction at step t (1-based), then the same
 * projection onto [0,1]:
 *   m <- b1*m + (1-b1)*g ;  v <- b2*v + (1-b2)*g^2
 *   x <- clamp(x - lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps), 0, 1) */
void oracle_step_adam(int64_t count, double lr, double b1, double b2, double eps, int32_t t,
                      double* x, double* mom, double* vel, const double* g) {
  const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < count; ++i) {
    mom[i] = b1 * mom[i] + (1.0 - b1) * g[i];
    vel[i] = b2 * vel[i] + (1.0 - b2) * g[i] * g[i];
    double y = x[i] - lr * (mom[i] / c1) / (sqrt(vel[i] / c2) + eps);
    if (y < 0.0) y = 0.0;
    if (y > 1.0) y = 1.0;
    x[i] = y;
  }
}

/* Exact unsatisfied-clause count per (formula, restart) of the rounded
 * assignment x_hat = [x > 0.5], by Boolean evaluation: a clause is
 * unsatisfied when none of its literals is true (no polynomial involved). */
void oracle_unsat(int32_t n, int32_t F, const int32_t* fcb, const int32_t* cptr,
                  const int32_t* lits, int32_t R, const double* x, int32_t* unsat) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t r = 0; r < R; ++r) {
    const double* xr = x + (int64_t)r * n;
    for (int32_t f = 0; f < F; ++f) {
      int32_t cnt = 0;
      for (int64_t t = fcb[f]; t < fcb[f + 1]; ++t) {
        int any_true = 0;
        for (int32_t p = cptr[t]; p < cptr[t + 1]; ++p) {
          const int32_t code = lits[p];
          const int value = xr[code >> 1] > 0.5;   /* rounded variable */
          const int lit_true = (code & 1) ? !value : value;
          if (lit_true) { any_true = 1; break; }
        }
        if (!any_true) ++cnt;
      }
      unsat[(int64_t)f * R + r] = cnt;
    }
  }
}

/* best[f] = the restart with the fewest unsatisfied clauses, ties to the
 * lowest restart index. */
void oracle_best(int32_t F, int32_t R, const int32_t* unsat, int32_t* best) {
  for (int32_t f = 0; f < F; ++f) {
    int32_t b = 0;
    for (int32_t r = 1; r < R; ++r)
      if (unsat[(int64_t)f * R + r] < unsat[(int64_t)f * R + b]) b = r;
    best[f] = b;
  }
}

/* One full iteration at x (restart-major, FP64): loss', unsat of round(x),
 * gradient, then the projected update of x in place.  This is the workload
 * that the CPU baseline times. */
void oracle_full_step(int32_t n, int32_t F, const int32_t* fcb, const int32_t* cptr,
                      const int32_t* lits, int32_t R, double lr, double* x, double* grad,
                      double* loss, int32_t* unsat) {
  oracle_unsat(n, F, fcb, cptr, lits, R, x, unsat);
  oracle_grad(n, F, fcb, cptr, lits, R, x, loss, grad, NULL);
  oracle_step_sgd((int64_t)R * n, lr, x, grad);
}

/* Initial state from a counter-based generator: the SplitMix64 output mix
 * (Steele, Lea & Flood 2014) applied twice,
 *   h = mix(seed XOR mix(v * 2^32 + r + 0x9e3779b97f4a7c15)),
 *   x[r][v] = (h >> 40) * 2^-24  in [0, 1),
 * a multiple of 2^-24, so the value is exact in FP32 and FP64. */
static uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* The SplitMix64 generator itself: state += golden gamma, output mix(state).
 * Exposed so its published reference outputs can be checked. */
void oracle_splitmix64(uint64_t state, int32_t count, uint64_t* out) {
  for (int32_t i = 0; i < count; ++i) {
    state += 0x9e3779b97f4a7c15ULL;
    out[i] = splitmix_mix(state);
  }
}

void oracle_init_state(uint64_t seed, int32_t n, int32_t R, double* x) {
  for (int32_t r = 0; r < R; ++r)
    for (int32_t v = 0; v < n; ++v) {
      uint64_t key = ((uint64_t)(uint32_t)v << 32) + (uint64_t)(uint32_t)r + 0x9e3779b97f4a7c15ULL;
      uint64_t h = splitmix_mix(seed ^ splitmix_mix(key));
      x[(int64_t)r * n + v] = (double)(h >> 40) * (1.0 / 16777216.0);
    }
}

/* ---- Straight-through Gumbel-softmax mode (Section 3.2, Eq. 3-5) ----
 *
 * Two logits per (variable, restart) enter a temperature softmax after
 * i.i.d. Gumbel(0,1) noise (Eq. 3); the forward uses the hard argmax
 * (Eq. 4) and the backward substitutes the soft probabilities' gradient.
 * With two states the softmax depends only on the logit difference
 * d = theta1 - theta0 and the noise difference l = g1 - g0:
 *   y1 = sigma((d + l) / tau),   x_hat = [d + l > 0]   (tie -> state 0).
 * The gradient reaching theta1 is G * y1 * (1 - y1) / tau, with G the
 * gradient of loss' at x_hat, and theta0 receives its negative. */

/* Gumbel noise difference for step t.  Only l = g1 - g0 of the two
 * independent Gumbel(0,1) draws enters (Eq. 3-4 with two states), and
 * that difference is standard logistic, so l is drawn directly by the
 * logistic quantile function from one uniform:
 *   l = log(u / (1 - u)),  u = ((h >> 40) + 0.5) * 2^-24,
 *   h = mix(seed ^ mix(c ^ mix(t + 0x632be59bd9b4e019))),  c = v * 2^32 + r,
 * mix being the SplitMix64 output mix, evaluated in FP64.  out is [R][n]. */
void oracle_gumbel_noise(uint64_t seed, int32_t t, int32_t n, int32_t R, double* out) {
  const uint64_t ts = splitmix_mix((uint64_t)(uint32_t)t + 0x632be59bd9b4e019ULL);
  for (int32_t r = 0; r < R; ++r)
    for (int32_t v = 0; v < n; ++v) {
      const uint64_t c = ((uint64_t)(uint32_t)v << 32) + (uint64_t)(uint32_t)r;
      const uint64_t h = splitmix_mix(seed ^ splitmix_mix(c ^ ts));
      const double u = ((double)(h >> 40) + 0.5) * (1.0 / 16777216.0);
      out[(int64_t)r * n + v] = log(u / (1.0 - u));
    }
}

/* One straight-through Gumbel step on the logit differences d ([R][n]),
 * given the noise differences l ([R][n], FP32 values).  The hard decision
 * d + l > 0 is taken in FP32, as the kernels take it.  Writes loss' and the
 * unsat count of x_hat ([F][R]; both equal the number of unsatisfied
 * clauses), then updates d:
 *   adam = 0:  theta1 -= lr * g1, theta0 += lr * g1, so d -= 2 lr g1;
 *   adam = 1:  Adam on theta1 with gradient g1 (theta0's moments are the
 *              exact negatives, its step the negative), so d moves by twice
 *              theta1's Adam step; t is the 1-based Adam step.
 * mom/vel are theta1's moments ([R][n]); x_hat is returned in xh. */
void oracle_gumbel_step(int32_t n, int32_t F, const int32_t* fcb, const int32_t* cptr,
                        const int32_t* lits, int32_t R, double* d, const float* l, double tau,
                        double lr, double b1, double b2, double eps, int32_t t, int32_t adam,
                        double* mom, double* vel, double* xh, double* loss, int32_t* unsat) {
  const int64_t cnt = (int64_t)R * n;
  double* G = (double*)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
  for (int64_t i = 0; i < cnt; ++i) {
    const float s = (float)d[i] + l[i];
    xh[i] = s > 0.0f ? 1.0 : 0.0;
  }
  oracle_grad(n, F, fcb, cptr, lits, R, xh, loss, G, NULL);
  oracle_unsat(n, F, fcb, cptr, lits, R, xh, unsat);
  const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < cnt; ++i) {
    const double y1 = 1.0 / (1.0 + exp(-(d[i] + (double)l[i]) / tau));
    const double g1 = G[i] * y1 * (1.0 - y1) / tau;
    if (adam) {
      mom[i] = b1 * mom[i] + (1.0 - b1) * g1;
      vel[i] = b2 * vel[i] + (1.0 - b2) * g1 * g1;
      d[i] -= 2.0 * lr * (mom[i] / c1) / (sqrt(vel[i] / c2) + eps);
    } else {
      d[i] -= 2.0 * lr * g1;
    }
  }
  free(G);
}
