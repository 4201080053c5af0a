/*
 * oracle.c -- plain, slow, FP64 CPU reference of the gradient MaxSAT solve loop
 * of "torchmSAT: A GPU-Accelerated Approximation To The Maximum Satisfiability
 * Problem" (Hosny & Reda, arXiv 2402.03640).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header or table with the HIP library; it reads the same DIMACS-style literal
 * array and builds everything it needs itself.
 *
 * Every function follows the definition as written, with no blocking or
 * reordering:
 *   - W (Section 4, "The Neural Network Architecture"): W[i][j] = +1 if x_i is
 *     a literal of c_j, -1 if its negation is, 0 otherwise.  A clause that
 *     holds both x_i and its negation gets W[i][j] = +1 - 1 = 0 (the dense
 *     matrix cannot hold both).  Repeated literals are kept once.
 *   - scores f(x) = tanh(x) . W (Section 4, display equation for f).
 *   - de-relaxation a_i = [x_i > 0] (Section 4; the "> 1" of the unsat-core
 *     paragraph and of Algorithm 1 is read as "> 0").
 *   - unsatisfied clauses (Section 4, "Unsatisfiable Cores"): a clause is
 *     unsatisfied iff every one of its literals is false under a.  The paper's
 *     s = -len(c) test is equivalent once a is mapped to {-1,+1}; a clause with
 *     a complementary pair is always satisfied, an empty clause never is.
 *   - loss (Section 4 example and Algorithm 1): mean squared error of f
 *     against zero, masked to the unsatisfied clauses, divided by m (all
 *     clauses).  Mode ALL uses every clause (mask = 1).
 *   - gradient by the chain rule through tanh (sech^2 written as
 *     4 e^{-2|x|} / (1 + e^{-2|x|})^2, which does not cancel).
 *   - optimizer (Section 5 Setup): Adam with PyTorch 1.10 semantics, or plain
 *     gradient descent as in the worked example.
 *   - Algorithm 1 loop: best_cost starts at m (the total weight) with the
 *     rounded start as its assignment and step -1; at every evaluation step
 *     (t a multiple of K, and the last iterate) the rounded iterate is
 *     counted before the step and kept when strictly better; then one step.
 *     The loop's state (x, moments, step, best so far) can be taken out and
 *     the loop continued from it.
 *   - brute force (n <= 24): Gray-code enumeration of all assignments.
 *   - clause weights (weighted partial CNF, defined in Section 2 and left to
 *     future work in Section 6): with positive integer weights w_j the
 *     cost is the total weight of the unsatisfied clauses, the loss is
 *     (1/m) sum_j mu_j w_j f_j^2 and the best cost starts at the total weight.
 *     Without weights every w_j is 1 and every formula above is unchanged.
 *   - SplitMix64 (Steele, Lea, Flood 2014) for the U(-1,1) initial values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_PARSE (-2)
#define OR_ERR_RANGE (-3)
#define OR_ERR_NOMEM (-5)

typedef struct {
    int32_t n, m;
    int64_t *loff;   /* m+1 offsets into lit                                   */
    int32_t *lit;    /* distinct literals of each clause, first-occurrence order */
    int64_t *woff;   /* m+1 offsets into wvar / wcoef                           */
    int32_t *wvar;   /* 0-based variable with a nonzero W entry                 */
    int8_t *wcoef;   /* that entry: +1 or -1                                    */
    uint8_t *taut;   /* 1 if the clause holds a variable and its negation       */
    int64_t *w;      /* clause weights (m), or NULL: every clause weighs 1      */
    int64_t wtot;    /* total weight (m without weights)                        */
} ocnf;

void oracle_free(ocnf *c) {
    if (!c) return;
    free(c->loff); free(c->lit); free(c->woff); free(c->wvar); free(c->wcoef); free(c->taut); free(c->w);
    free(c);
}

int32_t oracle_n(const ocnf *c) { return c->n; }
int32_t oracle_m(const ocnf *c) { return c->m; }

/* Parse and canonicalize.  lits: clauses of signed 1-based literals, each
 * ended by 0. */
int oracle_build(int32_t n, const int32_t *lits, int64_t nlits, ocnf **out) {
    *out = NULL;
    if (n < 0 || nlits < 0 || (nlits > 0 && !lits)) return OR_ERR_ARG;
    if (nlits > 0 && lits[nlits - 1] != 0) return OR_ERR_PARSE;
    int64_t m = 0;
    for (int64_t p = 0; p < nlits; ++p) {
        int32_t l = lits[p];
        if (l == 0) { ++m; continue; }
        if (l == INT32_MIN || (l < 0 ? -l : l) > n) return OR_ERR_RANGE;
    }
    ocnf *c = (ocnf *)calloc(1, sizeof(ocnf));
    if (!c) return OR_ERR_NOMEM;
    c->n = n; c->m = (int32_t)m; c->wtot = m;
    c->loff = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    c->woff = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    c->lit = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nlits + 1));
    c->wvar = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nlits + 1));
    c->wcoef = (int8_t *)malloc((size_t)(nlits + 1));
    c->taut = (uint8_t *)calloc((size_t)m + 1, 1);
    if (!c->loff || !c->woff || !c->lit || !c->wvar || !c->wcoef || !c->taut) {
        oracle_free(c);
        return OR_ERR_NOMEM;
    }
    int64_t nl = 0, nw = 0, start = 0;
    int32_t j = 0;
    for (int64_t p = 0; p < nlits; ++p) {
        if (lits[p] != 0) continue;
        /* clause j is lits[start .. p) */
        int64_t cl0 = nl;
        for (int64_t q = start; q < p; ++q) {
            int dup = 0;
            for (int64_t r = cl0; r < nl; ++r)
                if (c->lit[r] == lits[q]) { dup = 1; break; }
            if (!dup) c->lit[nl++] = lits[q];
        }
        /* W column: one entry per variable, in order of first appearance */
        for (int64_t r = cl0; r < nl; ++r) {
            int32_t v = abs(c->lit[r]) - 1;
            int seen = 0;
            for (int64_t s = cl0; s < r; ++s)
                if (abs(c->lit[s]) - 1 == v) { seen = 1; break; }
            if (seen) continue;
            int coef = 0;
            for (int64_t s = r; s < nl; ++s)
                if (abs(c->lit[s]) - 1 == v) coef += c->lit[s] > 0 ? 1 : -1;
            if (coef == 0) { c->taut[j] = 1; continue; }
            c->wvar[nw] = v; c->wcoef[nw] = (int8_t)coef; ++nw;
        }
        c->loff[j + 1] = nl;
        c->woff[j + 1] = nw;
        ++j;
        start = p + 1;
    }
    *out = c;
    return OR_OK;
}

/* Give every clause a weight (m positive integers); NULL restores weight 1. */
int oracle_set_weights(ocnf *c, const int64_t *w) {
    free(c->w);
    c->w = NULL;
    c->wtot = c->m;
    if (!w) return OR_OK;
    int64_t tot = 0;
    for (int32_t j = 0; j < c->m; ++j) {
        if (w[j] <= 0 || w[j] > ((int64_t)1 << 53) || tot > INT64_MAX - w[j]) return OR_ERR_ARG;
        tot += w[j];
    }
    c->w = (int64_t *)malloc(sizeof(int64_t) * ((size_t)c->m + 1));
    if (!c->w) return OR_ERR_NOMEM;
    memcpy(c->w, w, sizeof(int64_t) * (size_t)c->m);
    c->wtot = tot;
    return OR_OK;
}

int64_t oracle_total_weight(const ocnf *c) { return c->wtot; }

static int64_t weight(const ocnf *c, int32_t j) { return c->w ? c->w[j] : 1; }

static int lit_false(int32_t l, const uint8_t *a) {
    int32_t v = abs(l) - 1;
    return l > 0 ? (a[v] == 0) : (a[v] == 1);
}

/* 1 iff clause j is unsatisfied under the Boolean assignment a. */
static int clause_unsat(const ocnf *c, int32_t j, const uint8_t *a) {
    if (c->taut[j]) return 0;
    for (int64_t r = c->loff[j]; r < c->loff[j + 1]; ++r)
        if (!lit_false(c->lit[r], a)) return 0;
    return 1; /* includes the empty clause */
}

/* Cost of assignment a (n bytes, 0/1): the number of unsatisfied clauses,
 * or their total weight. */
int64_t oracle_count(const ocnf *c, const uint8_t *a) {
    int64_t u = 0;
    for (int32_t j = 0; j < c->m; ++j) u += weight(c, j) * clause_unsat(c, j, a);
    return u;
}

/* Per-clause unsat flags (m bytes). */
void oracle_unsat_mask(const ocnf *c, const uint8_t *a, uint8_t *mask) {
    for (int32_t j = 0; j < c->m; ++j) mask[j] = (uint8_t)clause_unsat(c, j, a);
}

static double sech2(double x) {
    double e = exp(-2.0 * fabs(x));
    return 4.0 * e / ((1.0 + e) * (1.0 + e));
}

/* Loss, scores and gradient at one relaxed point x (n doubles).
 * mode 0 = UNSAT (mask from the rounded x), 1 = ALL (mask = 1).
 * Returns the loss; f (m), mu (m), grad (n), unsat may be NULL. */
double oracle_loss_grad_d(const ocnf *c, const double *x, int mode, double *f_out,
                          uint8_t *mu_out, double *grad, int64_t *unsat) {
    int32_t n = c->n, m = c->m;
    uint8_t *a = (uint8_t *)malloc((size_t)n + 1);
    double *t = (double *)malloc(sizeof(double) * ((size_t)n + 1));
    double *G = (double *)calloc((size_t)n + 1, sizeof(double));
    for (int32_t i = 0; i < n; ++i) {
        a[i] = (uint8_t)(x[i] > 0.0); /* NaN, +0 and -0 round to false */
        t[i] = tanh(x[i]);
    }
    double loss = 0.0;
    int64_t u = 0;
    for (int32_t j = 0; j < m; ++j) {
        double fj = 0.0;
        for (int64_t r = c->woff[j]; r < c->woff[j + 1]; ++r)
            fj += (double)c->wcoef[r] * t[c->wvar[r]];
        int un = clause_unsat(c, j, a);
        double wj = (double)weight(c, j);
        u += weight(c, j) * un;
        /* the loss is a sum over the clauses in the mask (all of them in mode
         * ALL); a clause outside it is not in the sum, whatever its score */
        int in_loss = mode == 1 || un;
        if (f_out) f_out[j] = fj;
        if (mu_out) mu_out[j] = (uint8_t)in_loss;
        if (!in_loss) continue;
        loss += wj * fj * fj;
        double aj = m > 0 ? 2.0 / (double)m * wj * fj : 0.0;
        for (int64_t r = c->woff[j]; r < c->woff[j + 1]; ++r)
            G[c->wvar[r]] += (double)c->wcoef[r] * aj;
    }
    if (m > 0) loss /= (double)m;
    if (grad)
        for (int32_t i = 0; i < n; ++i) grad[i] = sech2(x[i]) * G[i];
    if (unsat) *unsat = u;
    free(a); free(t); free(G);
    return loss;
}

/* Same at an FP32 point: x holds float values, widened exactly. */
double oracle_loss_grad_f(const ocnf *c, const float *x, int mode, double *f_out,
                          uint8_t *mu_out, double *grad, int64_t *unsat) {
    double *xd = (double *)malloc(sizeof(double) * ((size_t)c->n + 1));
    for (int32_t i = 0; i < c->n; ++i) xd[i] = (double)x[i];
    double l = oracle_loss_grad_d(c, xd, mode, f_out, mu_out, grad, unsat);
    free(xd);
    return l;
}

/* One Adam step (PyTorch 1.10: no weight decay, no amsgrad, step counted
 * from 1). */
void oracle_adam_step(int32_t n, double *x, double *mm, double *vv, const double *g,
                      int32_t step, double lr, double b1, double b2, double eps) {
    double bc1 = 1.0 - pow(b1, (double)step);
    double bc2 = 1.0 - pow(b2, (double)step);
    for (int32_t i = 0; i < n; ++i) {
        mm[i] = b1 * mm[i] + (1.0 - b1) * g[i];
        vv[i] = b2 * vv[i] + (1.0 - b2) * g[i] * g[i];
        double denom = sqrt(vv[i]) / sqrt(bc2) + eps;
        x[i] = x[i] - (lr / bc1) * mm[i] / denom;
    }
}

void oracle_sgd_step(int32_t n, double *x, const double *g, double lr) {
    for (int32_t i = 0; i < n; ++i) x[i] = x[i] - lr * g[i];
}

/* SplitMix64: output number k (k >= 1) of the stream whose state starts at
 * `seed`; the state advances by the golden-ratio increment before mixing. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Initial relaxed values [n][R]: restart r draws from the stream seeded with
 * seed + r, variable i takes its output number i + 1; the top 24 bits give
 * u in [0,1) and x = 2u - 1, exact in FP32. */
void oracle_init_x(int32_t n, int32_t R, uint64_t seed, float *x) {
    for (int32_t i = 0; i < n; ++i)
        for (int32_t r = 0; r < R; ++r) {
            uint64_t z = oracle_splitmix64(seed + (uint64_t)r, (uint64_t)i + 1);
            double u = (double)(z >> 40) * (1.0 / 16777216.0);
            x[(int64_t)i * R + r] = (float)(2.0 * u - 1.0);
        }
}

/* Algorithm 1 (Section 4, "The Solving Process") for R independent restarts,
 * continued from a given state for T more steps.  The state is what the loop
 * carries from one iteration to the next:
 *   x, mm, vv   [n][R] doubles: relaxed values and Adam moments (in/out);
 *   *step       iterations already taken (in), plus T (out);
 *   best[R], best_step[R]: fewest unsatisfied clauses seen and the step of
 *               that iterate, -1 for "not beaten since the start" (in/out);
 *   best_a      [R][n] bytes: the rounded iterate that reached best (in/out).
 * With t the global iteration index: whenever t % K == 0, and at the last
 * iterate, the rounded iterate is counted and kept if strictly better; then
 * the loss gradient at x_t (mask from the same rounding) takes Adam step
 * number t + 1, or an SGD step.  final_loss[R] (may be NULL) receives the loss
 * at the last iterate.  A solve of T1 + T2 steps equals this call with T1
 * then with T2 on the state it left, bit for bit, when T1 is a multiple of K
 * (otherwise the extra count of the T1-th iterate may only lower best).
 *   opt: 0 = Adam, 1 = SGD.  mode: 0 = UNSAT, 1 = ALL.  threads > 1 runs the
 *   restarts in parallel (OpenMP), each restart unchanged. */
int oracle_run(const ocnf *c, int32_t T, int32_t R, int32_t K, int32_t opt, double lr, double b1,
               double b2, double eps, int32_t mode, int32_t threads, double *x_s, double *m_s,
               double *v_s, int32_t *step, int64_t *best_s, int32_t *best_step_s, uint8_t *best_a_s,
               double *final_loss) {
    int32_t n = c->n;
    if (R <= 0 || T < 0 || K <= 0 || !step || *step < 0 || *step > INT32_MAX - T) return OR_ERR_ARG;
    const int32_t t0 = *step, t1 = *step + T;
#ifdef _OPENMP
    int nt = threads > 0 ? threads : 1;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
#endif
    for (int32_t r = 0; r < R; ++r) {
        double *x = (double *)malloc(sizeof(double) * ((size_t)n + 1));
        double *mm = (double *)malloc(sizeof(double) * ((size_t)n + 1));
        double *vv = (double *)malloc(sizeof(double) * ((size_t)n + 1));
        double *g = (double *)malloc(sizeof(double) * ((size_t)n + 1));
        uint8_t *a = (uint8_t *)malloc((size_t)n + 1);
        uint8_t *best_a = best_a_s + (size_t)r * n;
        for (int32_t i = 0; i < n; ++i) {
            x[i] = x_s[(int64_t)i * R + r];
            mm[i] = m_s[(int64_t)i * R + r];
            vv[i] = v_s[(int64_t)i * R + r];
        }
        int64_t best = best_s[r];
        int32_t best_step = best_step_s[r];
        for (int32_t t = t0; t <= t1; ++t) {
            if (t % K == 0 || t == t1) {
                for (int32_t i = 0; i < n; ++i) a[i] = (uint8_t)(x[i] > 0.0);
                int64_t cnt = oracle_count(c, a);
                if (cnt < best) {
                    best = cnt; best_step = t;
                    memcpy(best_a, a, (size_t)n);
                }
            }
            if (t == t1) {
                if (final_loss) final_loss[r] = oracle_loss_grad_d(c, x, mode, NULL, NULL, NULL, NULL);
                break;
            }
            oracle_loss_grad_d(c, x, mode, NULL, NULL, g, NULL);
            if (opt == 0) oracle_adam_step(n, x, mm, vv, g, t + 1, lr, b1, b2, eps);
            else oracle_sgd_step(n, x, g, lr);
        }
        best_s[r] = best; best_step_s[r] = best_step;
        for (int32_t i = 0; i < n; ++i) {
            x_s[(int64_t)i * R + r] = x[i];
            m_s[(int64_t)i * R + r] = mm[i];
            v_s[(int64_t)i * R + r] = vv[i];
        }
        free(x); free(mm); free(vv); free(g); free(a);
    }
    *step = t1;
    return OR_OK;
}

/* The state of Algorithm 1 before its first iteration: x^0 from x0 ([n][R]
 * floats) or SplitMix64 with `seed`, zero moments, step 0, best = the total
 * weight (every clause unsatisfied), best_step = -1, best_a = round(x^0). */
void oracle_init_state(const ocnf *c, int32_t R, uint64_t seed, const float *x0, double *x_s, double *m_s,
                       double *v_s, int32_t *step, int64_t *best_s, int32_t *best_step_s, uint8_t *best_a_s) {
    int32_t n = c->n;
    float *xi = (float *)malloc(sizeof(float) * ((size_t)n * R + 1));
    if (x0) memcpy(xi, x0, sizeof(float) * (size_t)n * R);
    else oracle_init_x(n, R, seed, xi);
    for (int64_t e = 0; e < (int64_t)n * R; ++e) {
        x_s[e] = (double)xi[e];
        m_s[e] = 0.0;
        v_s[e] = 0.0;
    }
    for (int32_t r = 0; r < R; ++r) {
        best_s[r] = c->wtot;
        best_step_s[r] = -1;
        for (int32_t i = 0; i < n; ++i) best_a_s[(size_t)r * n + i] = (uint8_t)(x_s[(int64_t)i * R + r] > 0.0);
    }
    *step = 0;
    free(xi);
}

/* Algorithm 1 for R independent restarts from the start.
 *   opt: 0 = Adam, 1 = SGD.  mode: 0 = UNSAT, 1 = ALL.
 *   x0: [n][R] floats or NULL (SplitMix64 with `seed`).
 *   Outputs (any may be NULL): restart_best[R], restart_step[R],
 *   final_loss[R] (loss at x_T), best_assign[n] (of the best restart; ties
 *   go to the lowest restart), x_out [n][R] doubles (x_T).  Returns the
 *   instance best cost (negative on an argument error). */
int64_t oracle_solve(const ocnf *c, int32_t T, int32_t R, int32_t K, uint64_t seed,
                     int32_t opt, double lr, double b1, double b2, double eps, int32_t mode,
                     const float *x0, int32_t threads, int64_t *restart_best,
                     int32_t *restart_step, double *final_loss, uint8_t *best_assign,
                     int32_t *best_restart, double *x_out) {
    int32_t n = c->n;
    if (R <= 0 || T < 0 || K <= 0) return -1;
    size_t nR = (size_t)n * R + 1;
    double *xs = (double *)malloc(sizeof(double) * nR);
    double *ms = (double *)malloc(sizeof(double) * nR);
    double *vs = (double *)malloc(sizeof(double) * nR);
    int64_t *rb = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    int32_t *rs = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    uint8_t *ra = (uint8_t *)malloc(nR);
    int32_t step = 0;
    oracle_init_state(c, R, seed, x0, xs, ms, vs, &step, rb, rs, ra);
    int rc = oracle_run(c, T, R, K, opt, lr, b1, b2, eps, mode, threads, xs, ms, vs, &step, rb, rs, ra,
                        final_loss);
    int64_t best = -1;
    if (rc == OR_OK) {
        int32_t br = 0;
        for (int32_t r = 1; r < R; ++r)
            if (rb[r] < rb[br]) br = r;
        if (restart_best) memcpy(restart_best, rb, sizeof(int64_t) * (size_t)R);
        if (restart_step) memcpy(restart_step, rs, sizeof(int32_t) * (size_t)R);
        if (best_assign) memcpy(best_assign, ra + (size_t)br * n, (size_t)n);
        if (best_restart) *best_restart = br;
        if (x_out) memcpy(x_out, xs, sizeof(double) * (size_t)n * R);
        best = rb[br];
    }
    free(xs); free(ms); free(vs); free(rb); free(rs); free(ra);
    return best;
}

/* Exact optimum by enumerating all 2^n assignments in Gray-code order.
 * Returns 0 on success; opt = minimum unsat count, n_opt = how many
 * assignments reach it, arg = the first one met (n bytes, may be NULL). */
int oracle_bruteforce(const ocnf *c, int64_t *opt, int64_t *n_opt, uint8_t *arg) {
    int32_t n = c->n, m = c->m;
    if (n > 26) return OR_ERR_ARG;
    /* occurrence lists over the distinct literals */
    int64_t L = c->loff[m];
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t r = 0; r < L; ++r) cnt[abs(c->lit[r]) - 1]++;
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    int32_t *ocl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L + 1));
    int8_t *osg = (int8_t *)malloc((size_t)(L + 1));
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t j = 0; j < m; ++j)
        for (int64_t r = c->loff[j]; r < c->loff[j + 1]; ++r) {
            int32_t v = abs(c->lit[r]) - 1;
            int64_t p = off[v] + fill[v]++;
            ocl[p] = j; osg[p] = (int8_t)(c->lit[r] > 0 ? 1 : -1);
        }
    uint8_t *a = (uint8_t *)calloc((size_t)n + 1, 1);
    int32_t *ntrue = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    int64_t u = 0;
    for (int32_t j = 0; j < m; ++j) {
        for (int64_t r = c->loff[j]; r < c->loff[j + 1]; ++r)
            if (!lit_false(c->lit[r], a)) ntrue[j]++;
        if (!c->taut[j] && ntrue[j] == 0) u += weight(c, j);
    }
    int64_t best = u, nb = 1;
    if (arg) memcpy(arg, a, (size_t)n);
    uint64_t total = (uint64_t)1 << n;
    for (uint64_t k = 1; k < total; ++k) {
        int32_t i = __builtin_ctzll(k);
        a[i] ^= 1;
        for (int64_t p = off[i]; p < off[i + 1]; ++p) {
            int32_t j = ocl[p];
            /* literal became true iff its sign matches the new value */
            int now_true = osg[p] > 0 ? a[i] == 1 : a[i] == 0;
            int before = ntrue[j];
            ntrue[j] += now_true ? 1 : -1;
            if (c->taut[j]) continue;
            if (before == 0 && ntrue[j] > 0) u -= weight(c, j);
            else if (before > 0 && ntrue[j] == 0) u += weight(c, j);
        }
        if (u < best) {
            best = u; nb = 1;
            if (arg) memcpy(arg, a, (size_t)n);
        } else if (u == best) {
            nb++;
        }
    }
    *opt = best; *n_opt = nb;
    free(cnt); free(off); free(ocl); free(osg); free(fill); free(a); free(ntrue);
    return OR_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
