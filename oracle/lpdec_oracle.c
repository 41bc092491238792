/*
 * lpdec_oracle.c -- plain FP64 reference for ADMM-based LP decoding.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP library is
 * measured against; it shares no code, header, table or helper with the HIP
 * path and must never be linked into it.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it.
 *
 * Paper: Barman, Liu, Draper, Recht, "Decomposition Methods for Large Scale LP
 * Decoding" (arXiv 1204.0556).
 *
 * Contents
 *   lpo_project      Euclidean projection onto the parity polytope PP_d,
 *                    following Algorithm 2 (Sec. 4.4): sort, clip to the box,
 *                    constituent parity r (Lemma const_parity), the two early
 *                    returns, beta_max, and the root of f_r^T z(beta) = r on
 *                    [0, beta_max] (Lemma optimality, eq. find-beta).  The root
 *                    is located by evaluating f_r^T z(beta) at every candidate
 *                    breakpoint (the sets E1, L1, E2, L2 of Sec. 4.4, plus 0 and
 *                    beta_max) and interpolating linearly on the bracketing gap,
 *                    instead of the printed incremental march.
 *   lpo_max_linear   Algorithm 3 (Appendix A): maximise c^T z over PP_d.
 *   lpo_decode_batch Algorithm 1 (Sec. 3.3) with the over-relaxation of Sec. 5.2
 *                    (Boyd et al., Sec. 3.4.3), one frame per worker thread.
 *   lpo_dual_decode_batch  the dual subgradient ascent of Appendix A: x by the
 *                    Heaviside rule, z_j by Algorithm 3, lambda_j += mu (P_j x - z_j).
 *   lpo_evaluate     the per-frame bookkeeping behind the ML lower bound of
 *                    Sec. 5.1: word error, codeword test of the rounded estimate,
 *                    and whether its cost beats the transmitted codeword's.
 *
 * Readings of the paper taken here (each listed in the design notes):
 *   - Over-relaxation: q_j = rho P_j x + (1 - rho) z_j replaces P_j x in both the
 *     z-input and the dual update; rho = 1 is Algorithm 1 verbatim.
 *   - The dual is carried scaled, u = lambda / mu (Sec. 3.4's lambda').
 *   - gamma_i / mu sits inside the 1/|N_v(i)| average (Sec. 3.2 and Alg. 1).
 *   - Stopping: sum ||P_j x^k - z_j^k||^2 < eps^2 E and sum ||z_j^k - z_j^{k-1}||^2
 *     < eps^2 E with E = nnz(H) (= Md for a regular code); the primal residual
 *     uses the unrelaxed x.  Returned x is the x of the last iteration run.
 *   - Flags: converged; integral (max_i min(x_i, 1 - x_i) <= 1e-3); codeword
 *     (H xhat = 0 mod 2, xhat_i = [x_i >= 1/2]); ML-certified = all three
 *     (Sec. 1: an integral LP solution is the ML codeword); invalid input
 *     (a non-finite gamma; the frame is not decoded).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LPO_MAXD 64

#define LPO_FLAG_CONVERGED 0x01
#define LPO_FLAG_INTEGRAL 0x02
#define LPO_FLAG_CODEWORD 0x04
#define LPO_FLAG_CERTIFIED 0x08
#define LPO_FLAG_INVALID 0x80

/* which return of Algorithm 2 was taken */
#define LPO_BRANCH_ALL_ONE 0   /* r = d: the clipped vector is the all-ones vertex  */
#define LPO_BRANCH_BOX 1       /* f_r^T zhat <= r: the clipped vector lies in PP_d  */
#define LPO_BRANCH_SEARCH 2    /* beta_opt > 0 found on [0, beta_max]              */

static double clip01(double a) { return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a); }

/* f_r^T z(beta) for a vector already sorted in descending order, with
 * z(beta) = Pi_[0,1](v - beta f_r) and f_r = (+1 x (r+1), -1 x (d-r-1)). */
static double g_of_beta(int d, int r, const double *v, double beta) {
    double g = 0.0;
    for (int k = 0; k < d; ++k) {
        double f = (k <= r) ? 1.0 : -1.0;
        g += f * clip01(v[k] - beta * f);
    }
    return g;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Pi_PPd(u) -> z.  r_out / beta_out / branch_out may be NULL.  Returns 0, or -1 on
 * a bad degree.  Sorting is stable by index (ties keep their input order). */
int lpo_project(int d, const double *u, double *z, int *r_out, double *beta_out, int *branch_out) {
    if (d < 1 || d > LPO_MAXD) return -1;
    int Q[LPO_MAXD];
    double v[LPO_MAXD], zh[LPO_MAXD];

    /* Alg. 2, first step: permute u into v sorted in decreasing order (v = Q u). */
    for (int k = 0; k < d; ++k) Q[k] = k;
    for (int k = 1; k < d; ++k) { /* stable insertion sort, descending */
        int q = Q[k], p = k;
        while (p > 0 && u[Q[p - 1]] < u[q]) { Q[p] = Q[p - 1]; --p; }
        Q[p] = q;
    }
    for (int k = 0; k < d; ++k) v[k] = u[Q[k]];

    /* zhat = Pi_[0,1]^d(v); r = even floor of ||zhat||_1 (Lemma const_parity). */
    double s = 0.0;
    for (int k = 0; k < d; ++k) { zh[k] = clip01(v[k]); s += zh[k]; }
    int r = 2 * (int)floor(s / 2.0);
    if (r > d) r = d; /* s <= d always; guards rounding only */
    if (r_out) *r_out = r;

    double beta = 0.0;
    int branch;
    if (r == d) {
        branch = LPO_BRANCH_ALL_ONE;
    } else {
        /* 0-based: v_{r+1} is v[r], v_{r+2} is v[r+1]. */
        double beta_max = (r <= d - 2) ? 0.5 * (v[r] - v[r + 1]) : v[r];
        double g0 = g_of_beta(d, r, v, 0.0);
        if (g0 <= (double)r) {
            branch = LPO_BRANCH_BOX;
        } else {
            /* Root of f_r^T z(beta) = r on [0, beta_max].  Between consecutive
             * members of B = (E1 u L1 u E2 u L2) n [0, beta_max] u {0, beta_max}
             * the function is linear (eq. find-beta), so locate the first
             * candidate where it is <= r and interpolate on that gap. */
            double cand[4 * LPO_MAXD + 2];
            int nc = 0;
            cand[nc++] = 0.0;
            cand[nc++] = beta_max;
            for (int k = 0; k < d; ++k) {
                double a, b;
                if (k <= r) { a = v[k] - 1.0; b = v[k]; }   /* E1, L1 */
                else        { a = -v[k];      b = 1.0 - v[k]; } /* E2, L2 */
                if (a > 0.0 && a < beta_max) cand[nc++] = a;
                if (b > 0.0 && b < beta_max) cand[nc++] = b;
            }
            qsort(cand, (size_t)nc, sizeof(double), cmp_double);
            beta = beta_max;
            double c_prev = cand[0], g_prev = g0;
            for (int i = 1; i < nc; ++i) {
                if (cand[i] == c_prev) continue;
                double gi = g_of_beta(d, r, v, cand[i]);
                if (gi <= (double)r) {
                    beta = c_prev + (g_prev - (double)r) * (cand[i] - c_prev) / (g_prev - gi);
                    break;
                }
                c_prev = cand[i];
                g_prev = gi;
            }
            branch = LPO_BRANCH_SEARCH;
        }
    }
    if (beta_out) *beta_out = beta;
    if (branch_out) *branch_out = branch;

    /* z* = Q^T Pi_[0,1](v - beta_opt f_r) */
    for (int k = 0; k < d; ++k) {
        double f = (k <= r) ? 1.0 : -1.0;
        z[Q[k]] = (branch == LPO_BRANCH_SEARCH) ? clip01(v[k] - beta * f) : zh[k];
    }
    return 0;
}

/* Algorithm 3 (Appendix A): a maximiser of c^T z over PP_d (a vertex).  The
 * printed comparison "c_ip > c_in" holds trivially for a positive c_ip and a
 * non-positive c_in; the two candidate vertices differ by adding i_n (gain c_in)
 * or dropping i_p (loss c_ip), so the larger objective is chosen: add i_n iff
 * c_ip + c_in > 0. */
int lpo_max_linear(int d, const double *c, double *z) {
    if (d < 1) return -1;
    int npos = 0, ip = -1, in = -1;
    for (int i = 0; i < d; ++i) {
        z[i] = c[i] > 0.0 ? 1.0 : 0.0;
        if (c[i] > 0.0) {
            ++npos;
            if (ip < 0 || c[i] < c[ip]) ip = i;
        } else if (in < 0 || c[i] > c[in]) {
            in = i;
        }
    }
    if (npos % 2 == 0) return 0;
    if (in >= 0 && c[ip] + c[in] > 0.0) z[in] = 1.0;
    else z[ip] = 0.0;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 (with over-relaxation), one frame.                             */

typedef struct {
    int m, n, nnz;
    const int *row_ptr, *col_idx; /* CSR over checks */
    int *var_ptr, *var_edge;       /* for each variable, its edges (ascending edge id) */
    int maxd;
} lpo_graph;

typedef struct {
    double mu, rho, tol;
    int max_iter;
} lpo_params;

typedef struct {
    long long n_proj[3]; /* projection branch counts */
} lpo_stats;

static int graph_build(lpo_graph *g, int m, int n, const int *row_ptr, const int *col_idx) {
    g->m = m; g->n = n; g->nnz = row_ptr[m];
    g->row_ptr = row_ptr; g->col_idx = col_idx;
    g->var_ptr = (int *)calloc((size_t)n + 1, sizeof(int));
    g->var_edge = (int *)malloc(sizeof(int) * (size_t)(g->nnz > 0 ? g->nnz : 1));
    if (!g->var_ptr || !g->var_edge) return -1;
    g->maxd = 0;
    for (int j = 0; j < m; ++j) {
        int d = row_ptr[j + 1] - row_ptr[j];
        if (d > g->maxd) g->maxd = d;
        for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) g->var_ptr[col_idx[e] + 1]++;
    }
    for (int i = 0; i < n; ++i) g->var_ptr[i + 1] += g->var_ptr[i];
    int *fill = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!fill) return -1;
    memcpy(fill, g->var_ptr, sizeof(int) * (size_t)n);
    for (int e = 0; e < g->nnz; ++e) g->var_edge[fill[col_idx[e]]++] = e; /* ascending e */
    free(fill);
    return 0;
}

static void graph_free(lpo_graph *g) {
    free(g->var_ptr);
    free(g->var_edge);
}

/* Decode one frame.  z,u are the edge-indexed replicas and scaled duals (length
 * nnz, CSR edge order); they hold the initial state on entry (zero for a cold
 * start) and the final state on exit. */
static void decode_frame(const lpo_graph *g, const lpo_params *p, const double *gamma,
                         double *x, double *z, double *u, int *iters, unsigned char *flags,
                         lpo_stats *st) {
    const int n = g->n, m = g->m, E = g->nnz;
    for (int i = 0; i < n; ++i) {
        if (!isfinite(gamma[i])) {
            for (int k = 0; k < n; ++k) x[k] = 0.5;
            *iters = 0;
            *flags = LPO_FLAG_INVALID;
            return;
        }
    }
    double v[LPO_MAXD], zn[LPO_MAXD];
    const double thresh = p->tol * p->tol * (double)E;
    int converged = 0, k = 0;
    for (k = 1; k <= p->max_iter; ++k) {
        /* x-update (Sec. 3.2): average of (z - lambda/mu) over the variable's
         * checks, minus gamma_i/mu, divided by |N_v(i)|, projected onto [0,1]. */
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int t = g->var_ptr[i]; t < g->var_ptr[i + 1]; ++t) {
                int e = g->var_edge[t];
                acc += z[e] - u[e];
            }
            double deg = (double)(g->var_ptr[i + 1] - g->var_ptr[i]);
            x[i] = clip01((acc - gamma[i] / p->mu) / deg);
        }
        /* z- and lambda-updates, check by check. */
        double rp = 0.0, rd = 0.0;
        for (int j = 0; j < m; ++j) {
            int e0 = g->row_ptr[j], d = g->row_ptr[j + 1] - e0;
            for (int t = 0; t < d; ++t) {
                int e = e0 + t;
                double q = p->rho * x[g->col_idx[e]] + (1.0 - p->rho) * z[e];
                v[t] = q + u[e];
            }
            int br = 0;
            lpo_project(d, v, zn, NULL, NULL, &br);
            if (st) st->n_proj[br]++;
            for (int t = 0; t < d; ++t) {
                int e = e0 + t;
                double xe = x[g->col_idx[e]];
                u[e] = v[t] - zn[t]; /* u + q - z' */
                rp += (xe - zn[t]) * (xe - zn[t]);
                rd += (zn[t] - z[e]) * (zn[t] - z[e]);
                z[e] = zn[t];
            }
        }
        if (rp < thresh && rd < thresh) { converged = 1; break; }
    }
    *iters = converged ? k : p->max_iter;

    unsigned char fl = converged ? LPO_FLAG_CONVERGED : 0;
    double frac = 0.0;
    for (int i = 0; i < n; ++i) {
        double a = x[i] < 1.0 - x[i] ? x[i] : 1.0 - x[i];
        if (a > frac) frac = a;
    }
    if (frac <= 1e-3) fl |= LPO_FLAG_INTEGRAL;
    int ok = 1;
    for (int j = 0; j < m && ok; ++j) {
        int par = 0;
        for (int e = g->row_ptr[j]; e < g->row_ptr[j + 1]; ++e) par ^= (x[g->col_idx[e]] >= 0.5);
        if (par) ok = 0;
    }
    if (ok) fl |= LPO_FLAG_CODEWORD;
    if ((fl & 0x07) == 0x07) fl |= LPO_FLAG_CERTIFIED;
    *flags = fl;
}

typedef struct {
    const lpo_graph *g;
    const lpo_params *p;
    int batch;
    const float *llr;
    double *x_out, *z_io, *u_io;
    int *iters_out;
    unsigned char *flags_out;
    int warm;
    int next; /* shared frame counter */
    long long n_proj[3];
    pthread_mutex_t mu;
    int error;
} lpo_job;

static void *worker(void *arg) {
    lpo_job *J = (lpo_job *)arg;
    const int n = J->g->n, E = J->g->nnz;
    double *gamma = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double *u = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    lpo_stats st = {{0, 0, 0}};
    if (!gamma || !z || !u) {
        __atomic_store_n(&J->error, 1, __ATOMIC_SEQ_CST);
    } else {
        for (;;) {
            int f = __atomic_fetch_add(&J->next, 1, __ATOMIC_SEQ_CST);
            if (f >= J->batch) break;
            for (int i = 0; i < n; ++i) gamma[i] = (double)J->llr[(size_t)f * n + i];
            if (J->warm && J->z_io && J->u_io) {
                memcpy(z, J->z_io + (size_t)f * E, sizeof(double) * (size_t)E);
                memcpy(u, J->u_io + (size_t)f * E, sizeof(double) * (size_t)E);
            } else {
                memset(z, 0, sizeof(double) * (size_t)E);
                memset(u, 0, sizeof(double) * (size_t)E);
            }
            decode_frame(J->g, J->p, gamma, J->x_out + (size_t)f * n, z, u, &J->iters_out[f],
                         &J->flags_out[f], &st);
            if (J->z_io) memcpy(J->z_io + (size_t)f * E, z, sizeof(double) * (size_t)E);
            if (J->u_io) memcpy(J->u_io + (size_t)f * E, u, sizeof(double) * (size_t)E);
        }
    }
    pthread_mutex_lock(&J->mu);
    for (int b = 0; b < 3; ++b) J->n_proj[b] += st.n_proj[b];
    pthread_mutex_unlock(&J->mu);
    free(gamma); free(z); free(u);
    return NULL;
}

/* Decode `batch` frames of one code.  llr is [batch][n] float (promoted to FP64).
 * x_out [batch][n]; iters_out, flags_out [batch].  z_io / u_io ([batch][nnz], CSR
 * edge order) may be NULL; when given they receive the final state, and with
 * warm != 0 they also supply the initial state.  proj_counts (3 entries) may be
 * NULL.  Returns 0 on success, -1 on bad input, -2 on allocation failure. */
int lpo_decode_batch(int m, int n, const int *row_ptr, const int *col_idx, int batch,
                     const float *llr, double mu, double rho, int max_iter, double tol,
                     double *x_out, int *iters_out, unsigned char *flags_out, double *z_io,
                     double *u_io, int warm, int nthreads, long long *proj_counts) {
    if (m < 1 || n < 1 || batch < 0 || max_iter < 1 || !(mu > 0.0)) return -1;
    for (int j = 0; j < m; ++j) {
        int d = row_ptr[j + 1] - row_ptr[j];
        if (d < 1 || d > LPO_MAXD) return -1;
        for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e)
            if (col_idx[e] < 0 || col_idx[e] >= n) return -1;
    }
    lpo_graph g;
    if (graph_build(&g, m, n, row_ptr, col_idx)) { graph_free(&g); return -2; }
    for (int i = 0; i < n; ++i)
        if (g.var_ptr[i + 1] == g.var_ptr[i]) { graph_free(&g); return -1; }
    lpo_params p = {mu, rho, tol, max_iter};
    lpo_job J;
    memset(&J, 0, sizeof J);
    J.g = &g; J.p = &p; J.batch = batch; J.llr = llr; J.x_out = x_out; J.z_io = z_io;
    J.u_io = u_io; J.iters_out = iters_out; J.flags_out = flags_out; J.warm = warm;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > batch) nthreads = batch > 0 ? batch : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    if (th) {
        for (int t = 0; t < nthreads; ++t)
            if (pthread_create(&th[t], NULL, worker, &J) == 0) ++started;
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        free(th);
    }
    if (started == 0) worker(&J);
    pthread_mutex_destroy(&J.mu);
    if (proj_counts)
        for (int b = 0; b < 3; ++b) proj_counts[b] = J.n_proj[b];
    graph_free(&g);
    return J.error ? -2 : 0;
}

/* ------------------------------------------------------------------------- */
/* Dual subgradient ascent (Appendix A), one frame.                           */
/*
 * With the un-augmented Lagrangian L0 = gamma^T x + sum_j lambda_j^T (P_j x - z_j):
 *   x^{k+1}_i = theta(-gamma_i - sum_{j in N_v(i)} lambda_{j,i})   theta(t) = [t > 0]
 *   z_j^{k+1} = argmax_{z in PP_d} lambda_j^T z                    (Algorithm 3)
 *   lambda_j^{k+1} = lambda_j + mu (P_j x^{k+1} - z_j^{k+1})
 * x and z both use lambda^k.  Each update adds mu times an integer in {-1,0,1}
 * to an edge's multiplier, so lambda_e = mu K_e with an integer count K_e; the
 * counts are carried exactly and lambda is formed from them (reading: this is
 * the same iteration without accumulated rounding).  The decision for x_i is
 * taken in FP64 as (-gamma_i) - mu S_i with S_i the integer sum of its counts.
 * Stopping (reading; the appendix gives none): when P_j x = z_j for every
 * check, lambda no longer moves and (x, z) minimises L0 while being feasible,
 * so x is an LP optimum and a codeword: the frame is converged and certified.
 * Otherwise the iteration stops after max_iter passes and returns the last x.
 */
static void dual_frame(const lpo_graph *g, double mu, int max_iter, const double *gamma, long long *K,
                       double *x, int *iters, unsigned char *flags) {
    const int n = g->n, m = g->m;
    for (int i = 0; i < n; ++i) {
        if (!isfinite(gamma[i])) {
            for (int k = 0; k < n; ++k) x[k] = 0.5;
            *iters = 0;
            *flags = LPO_FLAG_INVALID;
            return;
        }
    }
    double c[LPO_MAXD], zv[LPO_MAXD];
    int converged = 0, k;
    for (k = 1; k <= max_iter; ++k) {
        for (int i = 0; i < n; ++i) {
            long long S = 0;
            for (int t = g->var_ptr[i]; t < g->var_ptr[i + 1]; ++t) S += K[g->var_edge[t]];
            const double t_i = (-gamma[i]) - mu * (double)S;
            x[i] = t_i > 0.0 ? 1.0 : 0.0;
        }
        int moved = 0;
        for (int j = 0; j < m; ++j) {
            const int e0 = g->row_ptr[j], d = g->row_ptr[j + 1] - e0;
            for (int t = 0; t < d; ++t) c[t] = mu * (double)K[e0 + t];
            lpo_max_linear(d, c, zv);
            for (int t = 0; t < d; ++t) {
                const long long delta = (long long)x[g->col_idx[e0 + t]] - (long long)zv[t];
                if (delta != 0) moved = 1;
                K[e0 + t] += delta;
            }
        }
        if (!moved) { converged = 1; break; }
    }
    *iters = converged ? k : max_iter;
    unsigned char fl = LPO_FLAG_INTEGRAL | (converged ? LPO_FLAG_CONVERGED : 0);
    int ok = 1;
    for (int j = 0; j < m && ok; ++j) {
        int par = 0;
        for (int e = g->row_ptr[j]; e < g->row_ptr[j + 1]; ++e) par ^= (x[g->col_idx[e]] >= 0.5);
        if (par) ok = 0;
    }
    if (ok) fl |= LPO_FLAG_CODEWORD;
    if ((fl & 0x07) == 0x07) fl |= LPO_FLAG_CERTIFIED;
    *flags = fl;
}

/* Decode `batch` frames of one code by dual subgradient ascent (Appendix A).
 * llr [batch][n] float; mu > 0 is the step size; x_out [batch][n] receives the
 * final x (0 or 1); iters_out, flags_out [batch].  Frames run one after another.
 * Returns 0, -1 on bad input, -2 on allocation failure. */
int lpo_dual_decode_batch(int m, int n, const int *row_ptr, const int *col_idx, int batch, const float *llr,
                          double mu, int max_iter, double *x_out, int *iters_out, unsigned char *flags_out) {
    if (m < 1 || n < 1 || batch < 0 || max_iter < 1 || !(mu > 0.0)) return -1;
    for (int j = 0; j < m; ++j) {
        int d = row_ptr[j + 1] - row_ptr[j];
        if (d < 1 || d > LPO_MAXD) return -1;
        for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e)
            if (col_idx[e] < 0 || col_idx[e] >= n) return -1;
    }
    lpo_graph g;
    if (graph_build(&g, m, n, row_ptr, col_idx)) { graph_free(&g); return -2; }
    for (int i = 0; i < n; ++i)
        if (g.var_ptr[i + 1] == g.var_ptr[i]) { graph_free(&g); return -1; }
    double *gamma = (double *)malloc(sizeof(double) * (size_t)n);
    long long *K = (long long *)malloc(sizeof(long long) * (size_t)g.nnz);
    if (!gamma || !K) { free(gamma); free(K); graph_free(&g); return -2; }
    for (int f = 0; f < batch; ++f) {
        for (int i = 0; i < n; ++i) gamma[i] = (double)llr[(size_t)f * n + i];
        memset(K, 0, sizeof(long long) * (size_t)g.nnz);
        dual_frame(&g, mu, max_iter, gamma, K, x_out + (size_t)f * n, &iters_out[f], &flags_out[f]);
    }
    free(gamma); free(K);
    graph_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* ML lower-bound bookkeeping (Sec. 5.1, the MacKay-code experiment).          */
/*
 * The decoder's x is rounded to xhat_i = [x_i >= 1/2].  A frame is a word error
 * when xhat differs from the transmitted word.  If xhat is nevertheless a
 * codeword (H xhat = 0) and it is more likely than the transmitted word given
 * the channel output -- cost gamma^T xhat < gamma^T sent, since gamma is the
 * negative log-likelihood ratio (Sec. 2) -- an ML decoder would have erred as
 * well.  Counting only those frames gives a lower bound on the ML word-error
 * rate.  Costs are summed in FP64; a tie counts as an ML success.
 *   sent   [batch][n] bits, or NULL for the all-zero codeword
 *   outcome bit0 word error, bit1 xhat is a codeword, bit2 ML error witnessed
 */
int lpo_evaluate(int m, int n, const int *row_ptr, const int *col_idx, int batch, const float *llr,
                 const double *x, const unsigned char *sent, int *bit_errors, double *cost_hat,
                 double *cost_sent, unsigned char *outcome) {
    if (m < 1 || n < 1 || batch < 0) return -1;
    for (int f = 0; f < batch; ++f) {
        const float *g = llr + (size_t)f * n;
        const double *xf = x + (size_t)f * n;
        const unsigned char *sf = sent ? sent + (size_t)f * n : NULL;
        int be = 0;
        double ch = 0.0, cs = 0.0;
        for (int i = 0; i < n; ++i) {
            const int xh = xf[i] >= 0.5;
            const int si = sf ? (sf[i] != 0) : 0;
            be += xh != si;
            if (xh) ch += (double)g[i];
            if (si) cs += (double)g[i];
        }
        int cw = 1;
        for (int j = 0; j < m && cw; ++j) {
            int par = 0;
            for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) par ^= (xf[col_idx[e]] >= 0.5);
            if (par) cw = 0;
        }
        unsigned char o = 0;
        if (be) o |= 0x01;
        if (cw) o |= 0x02;
        if (be && cw && ch < cs) o |= 0x04;
        bit_errors[f] = be;
        cost_hat[f] = ch;
        cost_sent[f] = cs;
        outcome[f] = o;
    }
    return 0;
}
