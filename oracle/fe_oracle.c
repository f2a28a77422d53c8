/*
 * FP64 reference evaluation of the Walsh-Fourier relaxed objective.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP path.  Single-threaded, plain
 * loops, no blocking or fusion beyond what each definition states.
 *
 * Conventions (Background, "Walsh-Fourier Transformation"): True -> -1,
 * False -> +1.  A literal with sign s over variable x has value y = s * x, so a
 * positive literal is true at x = -1.  A symmetric constraint over k literals
 * is given by its spectrum sp[t] (t = 0..k): -1 where it holds with exactly t
 * true literals, +1 where it does not (eq. wfcoef).
 *
 * Two evaluation routes, equal in exact arithmetic:
 *   ESP route  - FE = sum_j a_j e_j(y) (eq. wft grouped by |S|, eq. 2), with
 *                the elementary symmetric polynomials built by the O(k^2)
 *                recurrence e_j <- e_j + y_i e_{j-1}.  The gradient uses the
 *                multilinear identity e_j(y) = e_j(y_-i) + y_i e_{j-1}(y_-i),
 *                so dFE/dy_i = sum_{j>=1} a_j e_{j-1}(y_-i), recomputed per i.
 *   PMF route  - the multilinear extension as an expectation: with independent
 *                literals of mean y_i, literal i is true with probability
 *                p_i = (1 - y_i)/2 and FE = sum_t sp_t Pr[T = t], T the number
 *                of true literals.  Pr[T = t] comes from the Poisson-binomial
 *                dynamic programme; dFE/dy_i = sum_u d_u Pr[T_-i = u] with
 *                d_u = (sp_u - sp_{u+1})/2 (eq. wfcoef) from forward prefix
 *                distributions and a backward recurrence.  Every intermediate
 *                is a convex combination, so this route stays accurate where
 *                the ESP route cancels catastrophically (long cardinality
 *                constraints near a corner).
 *
 * Objective (Background, "Satisfaction as Optimisation"): F = sum_c w_c FE_c on
 * [-1,1]^n; projected gradient step x <- clip(x - lr * grad F, -1, 1);
 * a corner satisfies the formula iff sum_c FE_c(sign x) = -m.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ESP 0
#define ORC_PMF 1
#define ORC_AUTO 2

/* ---------------------------------------------------------------- ESP route */

/* e_0..e_k of the literals y[0..k-1], leaving out index `skip` (-1 = none). */
static void esp_build(int k, const double *y, int skip, double *e)
{
    e[0] = 1.0;
    for (int j = 1; j <= k; ++j) e[j] = 0.0;
    int used = 0;
    for (int i = 0; i < k; ++i) {
        if (i == skip) continue;
        ++used;
        for (int j = used; j >= 1; --j) e[j] += y[i] * e[j - 1];
    }
}

double orc_fe_esp(int k, const double *a, const double *y, double *cond)
{
    double *e = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    esp_build(k, y, -1, e);
    double fe = 0.0;
    for (int j = 0; j <= k; ++j) fe += a[j] * e[j];
    if (cond) {
        /* condition estimate: sum_j |a_j| e_j(|y|) */
        double *ya = (double *)calloc((size_t)(k + 1), sizeof(double));
        for (int i = 0; i < k; ++i) ya[i] = fabs(y[i]);
        esp_build(k, ya, -1, e);
        double c = 0.0;
        for (int j = 0; j <= k; ++j) c += fabs(a[j]) * e[j];
        *cond = c;
        free(ya);
    }
    free(e);
    return fe;
}

void orc_grad_esp(int k, const double *a, const double *y, double *g)
{
    double *e = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    for (int i = 0; i < k; ++i) {
        esp_build(k, y, i, e);
        double s = 0.0;
        for (int j = 1; j <= k; ++j) s += a[j] * e[j - 1];
        g[i] = s;
    }
    free(e);
}

/* ---------------------------------------------------------------- PMF route */

double orc_fe_pmf(int k, const double *sp, const double *y)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    q[0] = 1.0;
    for (int t = 1; t <= k; ++t) q[t] = 0.0;
    for (int i = 0; i < k; ++i) {
        double p = 0.5 * (1.0 - y[i]);
        for (int t = i + 1; t >= 1; --t) q[t] = (1.0 - p) * q[t] + p * q[t - 1];
        q[0] = (1.0 - p) * q[0];
    }
    double fe = 0.0;
    for (int t = 0; t <= k; ++t) fe += sp[t] * q[t];
    free(q);
    return fe;
}

void orc_grad_pmf(int k, const double *sp, const double *y, double *g)
{
    /* F[i][a]: distribution of the number of true literals among y[0..i-1]. */
    size_t w = (size_t)(k + 1);
    double *F = (double *)calloc(w * w, sizeof(double));
    double *D = (double *)malloc(sizeof(double) * (w + 1));
    F[0] = 1.0;
    for (int i = 0; i < k - 1; ++i) {
        double p = 0.5 * (1.0 - y[i]);
        const double *cur = F + (size_t)i * w;
        double *nxt = F + (size_t)(i + 1) * w;
        for (int a = 0; a <= i + 1; ++a) {
            double stay = (a <= i) ? cur[a] : 0.0;
            double up = (a >= 1) ? cur[a - 1] : 0.0;
            nxt[a] = (1.0 - p) * stay + p * up;
        }
    }
    /* D(a) = E[d_{a + T_later}], starting from no later literals: D(a) = d_a. */
    for (int a = 0; a <= k; ++a) D[a] = (a < k) ? 0.5 * (sp[a] - sp[a + 1]) : 0.0;
    D[k + 1] = 0.0;
    for (int i = k - 1; i >= 0; --i) {
        const double *pre = F + (size_t)i * w;
        double s = 0.0;
        for (int a = 0; a <= i; ++a) s += pre[a] * D[a];
        g[i] = s;
        double p = 0.5 * (1.0 - y[i]);
        for (int a = 0; a <= k; ++a) D[a] = (1.0 - p) * D[a] + p * D[a + 1];
    }
    free(F);
    free(D);
}

/* One constraint: FE, per-literal gradient (may be NULL) and ESP condition. */
int orc_eval_constraint(int k, const double *sp, const double *a, const double *y, int method,
                        double *fe, double *g, double *cond)
{
    double c = 0.0;
    int use_pmf = (method == ORC_PMF);
    if (method != ORC_PMF) {
        if (!a) return -1;
        double v = orc_fe_esp(k, a, y, &c);
        if (method == ORC_AUTO && ldexp((double)k * c, -52) > 1e-12) use_pmf = 1;
        if (!use_pmf) {
            *fe = v;
            if (g) orc_grad_esp(k, a, y, g);
        }
    }
    if (use_pmf) {
        *fe = orc_fe_pmf(k, sp, y);
        if (g) orc_grad_pmf(k, sp, y, g);
    }
    if (cond) *cond = c;
    return use_pmf;
}

/* ------------------------------------------------------------ whole problem */

/*
 * Objective and gradient for R restarts.  x and grad are [R][n] (one full
 * assignment per row).  Constraint c has literals lit[row_ptr[c] .. row_ptr[c+1])
 * encoded +v / -v (1-based variable, negative = negated literal); its spectrum
 * and coefficients sit at offset row_ptr[c] + c of sp_all / coef_all.
 * sig_obj[r] = sum_c |w_c FE_c| and sig_grad[r][v] = sum |w_c dFE_c/dy_i| are
 * the magnitudes a computed sum's rounding error scales with.
 * Returns the number of constraint evaluations that took the PMF route.
 */
long orc_eval_problem(int n, int m, const int32_t *row_ptr, const int32_t *lit, const double *sp_all,
                      const double *coef_all, const double *weight, int R, const double *x,
                      double *obj, double *grad, double *sig_obj, double *sig_grad, int method)
{
    int kmax = 0;
    for (int c = 0; c < m; ++c) {
        int k = row_ptr[c + 1] - row_ptr[c];
        if (k > kmax) kmax = k;
    }
    double *y = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *gc = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    long n_pmf = 0;
    for (int r = 0; r < R; ++r) {
        const double *xr = x + (size_t)r * n;
        double F = 0.0, sF = 0.0;
        if (grad) memset(grad + (size_t)r * n, 0, sizeof(double) * (size_t)n);
        if (sig_grad) memset(sig_grad + (size_t)r * n, 0, sizeof(double) * (size_t)n);
        for (int c = 0; c < m; ++c) {
            int b = row_ptr[c], k = row_ptr[c + 1] - b;
            for (int i = 0; i < k; ++i) {
                int l = lit[b + i];
                int v = (l > 0 ? l : -l) - 1;
                y[i] = (l > 0 ? 1.0 : -1.0) * xr[v];
            }
            double wc = weight ? weight[c] : 1.0;
            double fe;
            const double *sp = sp_all + b + c;
            const double *a = coef_all ? coef_all + b + c : NULL;
            n_pmf += orc_eval_constraint(k, sp, a, y, coef_all ? method : ORC_PMF, &fe,
                                         grad ? gc : NULL, NULL);
            F += wc * fe;
            sF += fabs(wc * fe);
            if (grad) {
                for (int i = 0; i < k; ++i) {
                    int l = lit[b + i];
                    int v = (l > 0 ? l : -l) - 1;
                    double s = (l > 0 ? 1.0 : -1.0);
                    grad[(size_t)r * n + v] += wc * s * gc[i];
                    if (sig_grad) sig_grad[(size_t)r * n + v] += fabs(wc * gc[i]);
                }
            }
        }
        obj[r] = F;
        if (sig_obj) sig_obj[r] = sF;
    }
    free(y);
    free(gc);
    return n_pmf;
}

/*
 * Per-constraint gradient statistic behind adaptive weighting (Case Studies,
 * "Redundant Constraint Effect": weights informed by per-constraint gradient
 * magnitudes): out[c] = sum over the R restarts of sum_i (dFE_c/dy_i)^2, the
 * unweighted squared gradient of constraint c with respect to its literal
 * values.  PMF route (stable at every length).
 */
void orc_constraint_grad_sq(int n, int m, const int32_t *row_ptr, const int32_t *lit, const double *sp_all,
                            int R, const double *x, double *out)
{
    int kmax = 0;
    for (int c = 0; c < m; ++c) {
        int k = row_ptr[c + 1] - row_ptr[c];
        if (k > kmax) kmax = k;
    }
    double *y = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *gc = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    for (int c = 0; c < m; ++c) out[c] = 0.0;
    for (int r = 0; r < R; ++r) {
        const double *xr = x + (size_t)r * n;
        for (int c = 0; c < m; ++c) {
            int b = row_ptr[c], k = row_ptr[c + 1] - b;
            for (int i = 0; i < k; ++i) {
                int l = lit[b + i];
                int v = (l > 0 ? l : -l) - 1;
                y[i] = (l > 0 ? 1.0 : -1.0) * xr[v];
            }
            double fe;
            orc_eval_constraint(k, sp_all + b + c, NULL, y, ORC_PMF, &fe, gc, NULL);
            for (int i = 0; i < k; ++i) out[c] += gc[i] * gc[i];
        }
    }
    free(y);
    free(gc);
}

/* Projected gradient step (Background, "Satisfaction as Optimisation"). */
void orc_step(long count, const double *x, const double *grad, double lr, double *x_out)
{
    for (long i = 0; i < count; ++i) {
        double v = x[i] - lr * grad[i];
        x_out[i] = v < -1.0 ? -1.0 : (v > 1.0 ? 1.0 : v);
    }
}

/*
 * Rounding of x to a corner and exact violation count.  assign[r][v] = -1
 * (True) when x < 0, else +1 (False; -0.0 also maps here).  A literal is true
 * when s * assign = -1.  Constraint c is violated when sp[#true] = +1.
 * best = lowest unsat count, ties to the lowest restart index.
 */
void orc_extract(int n, int m, const int32_t *row_ptr, const int32_t *lit, const double *sp_all, int R,
                 const double *x, int8_t *assign, int32_t *unsat, int32_t *best)
{
    int b_idx = -1;
    int32_t b_val = 0;
    for (int r = 0; r < R; ++r) {
        const double *xr = x + (size_t)r * n;
        int8_t *ar = assign + (size_t)r * n;
        for (int v = 0; v < n; ++v) ar[v] = (xr[v] < 0.0) ? -1 : 1;
        int32_t u = 0;
        for (int c = 0; c < m; ++c) {
            int b = row_ptr[c], k = row_ptr[c + 1] - b, t = 0;
            for (int i = 0; i < k; ++i) {
                int l = lit[b + i];
                int v = (l > 0 ? l : -l) - 1;
                int s = l > 0 ? 1 : -1;
                if (s * ar[v] == -1) ++t;
            }
            if (sp_all[b + c + t] > 0.0) ++u;
        }
        unsat[r] = u;
        if (b_idx < 0 || u < b_val) {
            b_idx = r;
            b_val = u;
        }
    }
    if (best) *best = b_idx;
}

/* ------------------------------------------------------- Philox4x32-10 RNG */
/*
 * Counter-based generator of Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplies
 * with Weyl-sequence key increments between rounds.
 */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/*
 * Uniform restart initialisation: x[r][v] from counter (r, v, 0, 0) and key
 * (seed low word, seed high word); the top 24 bits i of the first output word
 * give x = (i - 2^23) / 2^23, a dyadic value in [-1, 1).
 */
void orc_init_uniform(int R, int n, uint64_t seed, double *x)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int r = 0; r < R; ++r) {
        for (int v = 0; v < n; ++v) {
            uint32_t ctr[4] = {(uint32_t)r, (uint32_t)v, 0u, 0u}, o[4];
            orc_philox4x32_10(ctr, key, o);
            x[(size_t)r * n + v] = ldexp((double)((int32_t)(o[0] >> 8) - 8388608), -23);
        }
    }
}
