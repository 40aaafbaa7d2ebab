/*
 * Reference oracle for restarted PDHG on discrete optimal transport.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 statement of
 * what the GPU path computes.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never does,
 * and the two share no code, header, table or helper.
 *
 * Source: H. Lu, J. Yang, "PDOT: a Practical Primal-Dual Algorithm and a
 * GPU-Based Solver for Optimal Transport" (arXiv 2407.19689).
 *   - problem (ot):      min <C,X>  s.t.  X 1 = f,  X^T 1 = g,  X >= 0   (Section 1, eq. ot)
 *   - matrix-free A:     A vec(X) = [X 1; X^T 1],  A^T [p;q] = p 1^T + 1 q^T (Section 3.1, eq. ot-lp-data)
 *   - PDHG iteration:    Algorithm 2 (alg:rpd)
 *   - KKT error:         Section 3.1, display after Algorithm 2 (stacked 2-norm of primal
 *                        residual, positive part of A^T y - c, scaled duality gap)
 *   - restart candidate, adaptive restart (i)-(iii), step size, primal weight:
 *                        Section 5, "Adaptive restart" and "Adaptive step-size and primal weight"
 *   - termination:       Section 5.1, "Termination criteria"
 *   - rounding:          Algorithm 3 (alg:round) and Lemma lem:round
 *   - duality gap:       Section 5.1, "Optimality gap"
 *
 * Readings taken where the paper is silent or garbled (each is a parameter):
 *   R1 relative KKT (the paper uses it but defines only the absolute form with an
 *      unknown radius R): kkt_mode 0 divides each block by its own scale,
 *        rel_P = ||[X1-f; X^T1-g]|| / ||[f;g]||,  rel_D = ||[p1^T+1q^T-C]^+||_F / ||C||_F,
 *        rel_G = |<C,X> - f^T p - g^T q| / (|<C,X>| + |f^T p + g^T q|),
 *        relKKT = sqrt(rel_P^2 + rel_D^2 + rel_G^2);
 *      kkt_mode 1 uses the denominators 1+||[f;g]||, 1+||C||_F, 1+|pobj|+|dobj|.
 *   R2 start point X=0, p=q=0; eta0 = 1/sqrt(m+n) = 1/||A||_2 (Proposition prop:norm-sharp).
 *   R3 step-size bound uses the squared omega-weighted norm over 2|dy^T A dx| (the printed
 *      square root makes the bound scale-dependent), +inf when the denominator is 0; a
 *      rejected trial is retried from the same point with the PDLP update
 *      eta' = min((1-(T+1)^-0.3) eta_bar, (1+(T+1)^-0.6) eta), T = accepted iterations.
 *   R4 averages weighted by the step eta used (uniform 1/(k+1) when eta is constant).
 *   R5 restart checks after every accepted iteration; candidate ties go to the average;
 *      KKT of the previous candidate right after a restart is the restart KKT;
 *      total_iteration counts accepted iterations of the whole solve.
 *   R6 restart moves to the candidate (PDOT) -- restart_rule 1 is Algorithm 2's literal
 *      rule (average, beta decay), restart_rule 2 never restarts.
 *   R7 primal weight updated at every restart after moving, eps_zero = 1e-10.
 *   R8 the returned plan is the candidate that met the tolerance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double tol;
    int64_t max_iters;       /* accepted-iteration cap                    */
    int64_t max_passes;      /* trial cap (accepted + rejected)           */
    double time_limit_s;     /* <= 0: none                                 */
    int32_t kkt_mode;        /* R1                                         */
    int32_t step_rule;       /* 0 adaptive (R3), 1 constant eta            */
    int32_t restart_rule;    /* 0 PDOT adaptive, 1 Algorithm 2 basic, 2 none */
    int32_t avg_weighting;   /* 0 eta-weighted, 1 uniform                  */
    int32_t primal_weight_update; /* 1: on                                 */
    int32_t output;          /* 0 candidate, 1 current iterate             */
    double beta_sufficient, beta_necessary, beta_artificial, beta_basic;
    double theta, omega0, eta0, eps_zero;
    double step_reduction_exp, step_growth_exp;
} orc_params;

typedef struct {
    int32_t status;          /* 0 converged, 4 iteration/time limit        */
    int32_t returned_average;
    int64_t iterations, passes, restarts;
    double objective, dual_objective;
    double rel_primal, rel_dual, rel_gap, rel_kkt;
    double eta, omega, seconds;
} orc_result;

typedef struct {
    int64_t pass, iter;
    int32_t accepted, restart, cand_avg, pad;
    double eta_used, eta_bar, k_cur, k_avg, omega;
} orc_trace;

void orc_params_default(orc_params *p)
{
    memset(p, 0, sizeof(*p));
    p->tol = 1e-4;                 /* Section 5.1 termination tolerance */
    p->max_iters = 1000000;
    p->max_passes = 4000000;
    p->time_limit_s = 0.0;
    p->beta_sufficient = 0.1;      /* Section 5, adaptive restart */
    p->beta_necessary = 0.9;
    p->beta_artificial = 0.36;
    p->beta_basic = 0.2;
    p->theta = 0.5;                /* Section 5, primal weight */
    p->omega0 = 1.0;
    p->eta0 = 0.0;                 /* 0: 1/sqrt(m+n) */
    p->eps_zero = 1e-10;
    p->step_reduction_exp = 0.3;
    p->step_growth_exp = 0.6;
    p->primal_weight_update = 1;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ---- the two matrix-free products of Section 3.1 --------------------------------- */

/* rows = X 1_n, cols = X^T 1_m.  Every sum runs in index order, so the result does not
 * depend on the number of threads. */
void orc_apply_A(int64_t m, int64_t n, const double *X, double *rows, double *cols)
{
    int64_t i, j;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double s = 0.0;
        for (j = 0; j < n; ++j) s += X[i * n + j];
        rows[i] = s;
    }
    const int64_t B = 64;
    int64_t nb = (n + B - 1) / B, b;
#pragma omp parallel for schedule(static)
    for (b = 0; b < nb; ++b) {
        int64_t j0 = b * B, j1 = j0 + B < n ? j0 + B : n, jj, ii;
        for (jj = j0; jj < j1; ++jj) cols[jj] = 0.0;
        for (ii = 0; ii < m; ++ii)
            for (jj = j0; jj < j1; ++jj) cols[jj] += X[ii * n + jj];
    }
}

/* out = p 1_n^T + 1_m q^T */
void orc_apply_AT(int64_t m, int64_t n, const double *p, const double *q, double *out)
{
    int64_t i, j;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j) out[i * n + j] = p[i] + q[j];
}

/* Sum of a per-row array in index order. */
static double ordered_sum(const double *a, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += a[i];
    return s;
}

static double dot(const double *a, const double *b, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += a[i] * b[i];
    return s;
}

/* ---- KKT error (Section 3.1) and its relative form (reading R1) ---------------- */

typedef struct {
    double pres2;   /* ||X1-f||^2 + ||X^T1-g||^2           */
    double dres2;   /* ||[p1^T + 1q^T - C]^+||_F^2         */
    double pobj;    /* <C,X>                                */
    double dobj;    /* f^T p + g^T q                        */
} kkt_raw;

typedef struct {
    int64_t m, n;
    const double *C, *f, *g;
    double norm_b, norm_c;   /* ||[f;g]||_2, ||C||_F */
    double *rows, *cols, *rowacc, *rowacc2;
} problem;

static kkt_raw kkt_evaluate(const problem *P, const double *X, const double *p, const double *q)
{
    int64_t m = P->m, n = P->n, i, j;
    kkt_raw r;
    orc_apply_A(m, n, X, P->rows, P->cols);
    double s = 0.0;
    for (i = 0; i < m; ++i) s += (P->rows[i] - P->f[i]) * (P->rows[i] - P->f[i]);
    for (j = 0; j < n; ++j) s += (P->cols[j] - P->g[j]) * (P->cols[j] - P->g[j]);
    r.pres2 = s;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double d = 0.0, o = 0.0;
        for (j = 0; j < n; ++j) {
            double c = P->C[i * n + j];
            double v = p[i] + q[j] - c;
            if (v > 0.0) d += v * v;
            o += c * X[i * n + j];
        }
        P->rowacc[i] = d;
        P->rowacc2[i] = o;
    }
    r.dres2 = ordered_sum(P->rowacc, m);
    r.pobj = ordered_sum(P->rowacc2, m);
    r.dobj = dot(P->f, p, m) + dot(P->g, q, n);
    return r;
}

static void kkt_relative(const problem *P, int32_t mode, kkt_raw r, double out[4])
{
    double rp, rd, rg;
    double ap = sqrt(r.pres2), ad = sqrt(r.dres2), gap = fabs(r.pobj - r.dobj);
    if (mode == 1) {
        rp = ap / (1.0 + P->norm_b);
        rd = ad / (1.0 + P->norm_c);
        rg = gap / (1.0 + fabs(r.pobj) + fabs(r.dobj));
    } else {
        rp = P->norm_b > 0.0 ? ap / P->norm_b : ap;
        rd = P->norm_c > 0.0 ? ad / P->norm_c : ad;
        double den = fabs(r.pobj) + fabs(r.dobj);
        rg = den > 0.0 ? gap / den : 0.0;
    }
    out[0] = rp;
    out[1] = rd;
    out[2] = rg;
    out[3] = sqrt(rp * rp + rd * rd + rg * rg);
}

static void problem_init(problem *P, int64_t m, int64_t n, const double *C, const double *f,
                         const double *g)
{
    P->m = m;
    P->n = n;
    P->C = C;
    P->f = f;
    P->g = g;
    P->norm_b = sqrt(dot(f, f, m) + dot(g, g, n));
    P->rows = (double *)malloc(sizeof(double) * (size_t)m);
    P->cols = (double *)malloc(sizeof(double) * (size_t)n);
    P->rowacc = (double *)malloc(sizeof(double) * (size_t)m);
    P->rowacc2 = (double *)malloc(sizeof(double) * (size_t)m);
    int64_t i, j;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double s = 0.0;
        for (j = 0; j < n; ++j) s += C[i * n + j] * C[i * n + j];
        P->rowacc[i] = s;
    }
    P->norm_c = sqrt(ordered_sum(P->rowacc, m));
}

static void problem_free(problem *P)
{
    free(P->rows);
    free(P->cols);
    free(P->rowacc);
    free(P->rowacc2);
}

/* Relative KKT of a given triple (used by tests on any plan, e.g. one the GPU returned).
 * out = {rel_P, rel_D, rel_G, relKKT, pobj, dobj, ||X1-f;X^T1-g||, ||[.]^+||}. */
void orc_kkt(int64_t m, int64_t n, const double *C, const double *f, const double *g,
             const double *X, const double *p, const double *q, int32_t kkt_mode, double out[8])
{
    problem P;
    problem_init(&P, m, n, C, f, g);
    kkt_raw r = kkt_evaluate(&P, X, p, q);
    kkt_relative(&P, kkt_mode, r, out);
    out[4] = r.pobj;
    out[5] = r.dobj;
    out[6] = sqrt(r.pres2);
    out[7] = sqrt(r.dres2);
    problem_free(&P);
}

/* ---- restarted PDHG: Algorithm 2 with the Section 5 enhancements ----------------- */

int orc_solve(int64_t m, int64_t n, const double *C, const double *f, const double *g,
              const orc_params *prm, double *X_out, double *p_out, double *q_out,
              double *Xavg_out, orc_result *res, orc_trace *trace, int64_t trace_cap,
              int32_t nthreads)
{
#ifdef _OPENMP
    const int threads_before = omp_get_max_threads();
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double t0 = now_s();
    const int64_t mn = m * n;
    const size_t MB = sizeof(double) * (size_t)mn;
    problem P;
    problem_init(&P, m, n, C, f, g);

    /* iterates (Algorithm 2): current, trial, average, restart anchor, scratch */
    double *X = (double *)calloc((size_t)mn, sizeof(double));
    double *Xn = (double *)calloc((size_t)mn, sizeof(double));
    double *Xb = (double *)calloc((size_t)mn, sizeof(double));
    double *Xa = (double *)calloc((size_t)mn, sizeof(double));
    double *E = (double *)malloc(MB);
    double *p = (double *)calloc((size_t)m, sizeof(double));
    double *q = (double *)calloc((size_t)n, sizeof(double));
    double *pn = (double *)malloc(sizeof(double) * (size_t)m);
    double *qn = (double *)malloc(sizeof(double) * (size_t)n);
    double *pb = (double *)calloc((size_t)m, sizeof(double));
    double *qb = (double *)calloc((size_t)n, sizeof(double));
    double *pa = (double *)calloc((size_t)m, sizeof(double));
    double *qa = (double *)calloc((size_t)n, sizeof(double));
    double *er = (double *)malloc(sizeof(double) * (size_t)m);
    double *ec = (double *)malloc(sizeof(double) * (size_t)n);
    double *dr = (double *)malloc(sizeof(double) * (size_t)m);
    double *dc = (double *)malloc(sizeof(double) * (size_t)n);

    double omega = prm->omega0 > 0.0 ? prm->omega0 : 1.0;
    double eta = prm->eta0 > 0.0 ? prm->eta0 : 1.0 / sqrt((double)(m + n));
    int64_t T = 0, k = 0, passes = 0, restarts = 0, ntrace = 0;
    double wsum = 0.0;
    int status = 4;
    int cand_is_avg = 0;
    double kk[4];

    /* KKT of the start point: the first restart reference */
    kkt_relative(&P, prm->kkt_mode, kkt_evaluate(&P, X, p, q), kk);
    double K_start = kk[3], K_prev = kk[3], K_cand = kk[3];
    if (K_cand <= prm->tol) status = 0;

    int64_t i, j;
    while (status != 0) {
        if (T >= prm->max_iters || passes >= prm->max_passes) break;
        if (prm->time_limit_s > 0.0 && now_s() - t0 >= prm->time_limit_s) break;

        /* ---- one PDHG step, retried with a smaller eta until the bound holds ---- */
        double eta_used = eta, eta_bar = INFINITY;
        int accepted = 0;
        while (!accepted) {
            if (passes >= prm->max_passes) break;
            ++passes;
            const double tau = eta / omega, sigma = eta * omega;
            /* X+ = Proj_{>=0}(X - tau (C - p 1^T - 1 q^T)) */
#pragma omp parallel for schedule(static)
            for (i = 0; i < m; ++i)
                for (j = 0; j < n; ++j) {
                    double v = X[i * n + j] - tau * (C[i * n + j] - p[i] - q[j]);
                    Xn[i * n + j] = v > 0.0 ? v : 0.0;
                }
            /* extrapolated plan 2X+ - X and its marginals */
#pragma omp parallel for schedule(static)
            for (i = 0; i < mn; ++i) E[i] = 2.0 * Xn[i] - X[i];
            orc_apply_A(m, n, E, er, ec);
            for (i = 0; i < m; ++i) pn[i] = p[i] + sigma * (f[i] - er[i]);
            for (j = 0; j < n; ++j) qn[j] = q[j] + sigma * (g[j] - ec[j]);

            eta_used = eta;
            if (prm->step_rule == 1) {
                accepted = 1;
                eta_bar = INFINITY;
            } else {
                /* ||dX||^2 and A dX from the difference matrix itself */
#pragma omp parallel for schedule(static)
                for (i = 0; i < mn; ++i) E[i] = Xn[i] - X[i];
#pragma omp parallel for schedule(static)
                for (i = 0; i < m; ++i) {
                    double s = 0.0;
                    for (j = 0; j < n; ++j) s += E[i * n + j] * E[i * n + j];
                    P.rowacc[i] = s;
                }
                double dx2 = ordered_sum(P.rowacc, m);
                orc_apply_A(m, n, E, dr, dc);
                double dy2 = 0.0, inter = 0.0;
                for (i = 0; i < m; ++i) {
                    double d = pn[i] - p[i];
                    dy2 += d * d;
                    inter += d * dr[i];
                }
                for (j = 0; j < n; ++j) {
                    double d = qn[j] - q[j];
                    dy2 += d * d;
                    inter += d * dc[j];
                }
                double num = omega * dx2 + dy2 / omega;
                double den = 2.0 * fabs(inter);
                eta_bar = den > 0.0 ? num / den : INFINITY;
                accepted = eta <= eta_bar;
                double tt = (double)(T + 1);
                double shrink = (1.0 - pow(tt, -prm->step_reduction_exp)) * eta_bar;
                double grow = (1.0 + pow(tt, -prm->step_growth_exp)) * eta;
                eta = shrink < grow ? shrink : grow;
            }
            if (trace && ntrace < trace_cap && !accepted) {
                orc_trace *t = &trace[ntrace++];
                memset(t, 0, sizeof(*t));
                t->pass = passes;
                t->iter = T;
                t->eta_used = eta_used;
                t->eta_bar = eta_bar;
                t->omega = omega;
            }
        }
        if (!accepted) break;

        /* accept */
        { double *t = X; X = Xn; Xn = t; }
        { double *t = p; p = pn; pn = t; }
        { double *t = q; q = qn; qn = t; }
        ++T;
        ++k;

        /* running average (Algorithm 2, last update of the inner loop) */
        double w = prm->avg_weighting == 1 ? 1.0 : eta_used;
        wsum += w;
        double a = w / wsum;
        if (k == 1) {
            memcpy(Xb, X, MB);
            memcpy(pb, p, sizeof(double) * (size_t)m);
            memcpy(qb, q, sizeof(double) * (size_t)n);
        } else {
#pragma omp parallel for schedule(static)
            for (i = 0; i < mn; ++i) Xb[i] = (1.0 - a) * Xb[i] + a * X[i];
            for (i = 0; i < m; ++i) pb[i] = (1.0 - a) * pb[i] + a * p[i];
            for (j = 0; j < n; ++j) qb[j] = (1.0 - a) * qb[j] + a * q[j];
        }

        /* KKT of the current iterate and of the average; restart candidate */
        double kc[4], ka[4];
        kkt_relative(&P, prm->kkt_mode, kkt_evaluate(&P, X, p, q), kc);
        kkt_relative(&P, prm->kkt_mode, kkt_evaluate(&P, Xb, pb, qb), ka);
        cand_is_avg = !(kc[3] < ka[3]);
        K_cand = cand_is_avg ? ka[3] : kc[3];

        int restart = 0;
        if (K_cand <= prm->tol) {
            status = 0;
        } else if (prm->restart_rule == 0) {
            if (K_cand <= prm->beta_sufficient * K_start) restart = 1;
            else if (K_cand <= prm->beta_necessary * K_start && K_cand > K_prev) restart = 2;
            else if ((double)k >= prm->beta_artificial * (double)T) restart = 3;
        } else if (prm->restart_rule == 1) {
            /* Algorithm 2 / eq. restart-condition: decay of the average's KKT */
            if (ka[3] <= prm->beta_basic * K_start) { restart = 1; cand_is_avg = 1; K_cand = ka[3]; }
        }

        if (trace && ntrace < trace_cap) {
            orc_trace *t = &trace[ntrace++];
            memset(t, 0, sizeof(*t));
            t->pass = passes;
            t->iter = T;
            t->accepted = 1;
            t->restart = restart;
            t->cand_avg = cand_is_avg;
            t->eta_used = eta_used;
            t->eta_bar = eta_bar;
            t->k_cur = kc[3];
            t->k_avg = ka[3];
            t->omega = omega;
        }

        if (restart) {
            if (cand_is_avg) {
                memcpy(X, Xb, MB);
                memcpy(p, pb, sizeof(double) * (size_t)m);
                memcpy(q, qb, sizeof(double) * (size_t)n);
            }
            /* primal weight (Section 5): distances from the previous restart point */
#pragma omp parallel for schedule(static)
            for (i = 0; i < m; ++i) {
                double s = 0.0;
                for (j = 0; j < n; ++j) {
                    double d = X[i * n + j] - Xa[i * n + j];
                    s += d * d;
                }
                P.rowacc[i] = s;
            }
            double dX = sqrt(ordered_sum(P.rowacc, m));
            double s = 0.0;
            for (i = 0; i < m; ++i) s += (p[i] - pa[i]) * (p[i] - pa[i]);
            for (j = 0; j < n; ++j) s += (q[j] - qa[j]) * (q[j] - qa[j]);
            double dY = sqrt(s);
            if (prm->primal_weight_update && dX > prm->eps_zero && dY > prm->eps_zero)
                omega = exp(prm->theta * log(dY / dX) + (1.0 - prm->theta) * log(omega));
            memcpy(Xa, X, MB);
            memcpy(pa, p, sizeof(double) * (size_t)m);
            memcpy(qa, q, sizeof(double) * (size_t)n);
            wsum = 0.0;
            k = 0;
            ++restarts;
            K_start = K_cand;
            K_prev = K_cand;
            cand_is_avg = 0;   /* the current iterate now is the candidate */
        } else {
            K_prev = K_cand;
        }
    }

    /* returned plan: the candidate (reading R8) or the current iterate */
    const double *Xr = X, *pr = p, *qr = q;
    int ret_avg = 0;
    if (prm->output == 0 && cand_is_avg && T > 0 && k > 0) {
        Xr = Xb;
        pr = pb;
        qr = qb;
        ret_avg = 1;
    }
    if (X_out) memcpy(X_out, Xr, MB);
    if (p_out) memcpy(p_out, pr, sizeof(double) * (size_t)m);
    if (q_out) memcpy(q_out, qr, sizeof(double) * (size_t)n);
    if (Xavg_out) memcpy(Xavg_out, Xb, MB);
    if (res) {
        kkt_raw r = kkt_evaluate(&P, Xr, pr, qr);
        double rel[4];
        kkt_relative(&P, prm->kkt_mode, r, rel);
        memset(res, 0, sizeof(*res));
        res->status = status;
        res->returned_average = ret_avg;
        res->iterations = T;
        res->passes = passes;
        res->restarts = restarts;
        res->objective = r.pobj;
        res->dual_objective = r.dobj;
        res->rel_primal = rel[0];
        res->rel_dual = rel[1];
        res->rel_gap = rel[2];
        res->rel_kkt = rel[3];
        res->eta = eta;
        res->omega = omega;
        res->seconds = now_s() - t0;
    }

    free(X); free(Xn); free(Xb); free(Xa); free(E);
    free(p); free(q); free(pn); free(qn); free(pb); free(qb); free(pa); free(qa);
    free(er); free(ec); free(dr); free(dc);
    problem_free(&P);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(threads_before);   /* the caller's setting again */
#endif
    return (int)ntrace;
}

/* ---- Algorithm 3: rounding to an exactly feasible plan ---------------------------- */

void orc_round(int64_t m, int64_t n, const double *f, const double *g, const double *X,
               double *Xf)
{
    int64_t i, j;
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *err_r = (double *)malloc(sizeof(double) * (size_t)m);
    double *err_c = (double *)malloc(sizeof(double) * (size_t)n);
    /* D_x = Diag(min(f_i / (X1)_i, 1)) */
    orc_apply_A(m, n, X, r, c);
    for (i = 0; i < m; ++i) {
        double x = r[i] > 0.0 ? f[i] / r[i] : 1.0;
        if (x > 1.0) x = 1.0;
        for (j = 0; j < n; ++j) Xf[i * n + j] = x * X[i * n + j];
    }
    /* D_y = Diag(min(g_j / (X_tmp^T 1)_j, 1)) */
    orc_apply_A(m, n, Xf, r, c);
    for (j = 0; j < n; ++j) {
        double y = c[j] > 0.0 ? g[j] / c[j] : 1.0;
        if (y > 1.0) y = 1.0;
        c[j] = y;
    }
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j) Xf[i * n + j] *= c[j];
    /* rank-one correction err_r err_c^T / ||err_r||_1 */
    orc_apply_A(m, n, Xf, r, c);
    double l1 = 0.0;
    for (i = 0; i < m; ++i) {
        err_r[i] = f[i] - r[i];
        l1 += fabs(err_r[i]);
    }
    for (j = 0; j < n; ++j) err_c[j] = g[j] - c[j];
    if (l1 > 0.0)
        for (i = 0; i < m; ++i)
            for (j = 0; j < n; ++j) Xf[i * n + j] += err_r[i] * err_c[j] / l1;
    free(r); free(c); free(err_r); free(err_c);
}

/* Weak-duality lower bound from any p: q_j = min_i (C_ij - p_i) makes (p,q) dual feasible,
 * so f^T p + g^T q <= OPT. */
double orc_dual_lower_bound(int64_t m, int64_t n, const double *C, const double *f,
                            const double *g, const double *p)
{
    double lb = dot(f, p, m);
    for (int64_t j = 0; j < n; ++j) {
        double qmin = INFINITY;
        for (int64_t i = 0; i < m; ++i) {
            double v = C[i * n + j] - p[i];
            if (v < qmin) qmin = v;
        }
        lb += g[j] * qmin;
    }
    return lb;
}
