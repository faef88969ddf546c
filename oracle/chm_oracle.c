/*
 * CPU oracle for the ternary Cahn-Hilliard time step -- TEST INFRASTRUCTURE.
 *
 * Plain FP64 C, one loop per definition, no blocking or fusion.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg load it; the
 * GPU library never does, and the two share no source.
 *
 * Citations name the paper's sections, equations and Algorithm 1.  Where the
 * paper leaves a choice open, the comment states the reading taken here.
 */
#include "chm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Host threads.  The row loops of the solve (sparse products, smoothing,    */
/* vector updates) may be split over threads by OpenMP with a static        */
/* schedule: each row is still computed by one thread with the same          */
/* operations in the same order, and every sum over rows (dot products,      */
/* norms) stays a serial loop, so the results are bitwise the same for any   */
/* thread count.                                                              */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

#define MAXLEV 32

typedef struct {
    int n, m;        /* rows, columns */
    int *rp, *ci;    /* row pointers, column indices (ascending per row) */
    double *v;
} csr_t;

typedef struct {
    int n;
    int degree;      /* smoother degree (Chebyshev) or sweeps (Jacobi) on this level */
    csr_t A;
    double *invdiag;
    double rho;      /* Gershgorin bound of the spectrum of D^-1 A */
    int nc;
    int *agg;        /* aggregate of each row (not on the coarsest level) */
    csr_t P, R;
    double *chol;    /* coarsest level: dense Cholesky factor, row-major lower */
} level_t;

typedef struct {
    int nlev;
    double ratio; /* Chebyshev interval [rho/ratio, rho] */
    level_t lev[MAXLEV];
} hier_t;

struct orc_solver {
    orc_params_t prm;
    int dim, nv, ncell;
    double *coords;
    int *cells;
    csr_t M, K, As[2];
    hier_t hM, hA[2];
    int nq;
    double qb[64 * 4], qw[64];
    int64_t step_count;
    double vc_rho; /* measured V-cycle contraction (schur_pcg = -1), else 0 */
};

/* ------------------------------------------------------------------ */
/* small helpers                                                       */

static void csr_free(csr_t *a)
{
    free(a->rp);
    free(a->ci);
    free(a->v);
    memset(a, 0, sizeof(*a));
}

static void csr_mv(const csr_t *a, const double *x, double *y)
{
    #pragma omp parallel for schedule(static) if (a->n >= 4096)
    for (int i = 0; i < a->n; ++i) {
        double s = 0.0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k)
            s += a->v[k] * x[a->ci[k]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static int find_col(const csr_t *a, int row, int col)
{
    int lo = a->rp[row], hi = a->rp[row + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (a->ci[mid] == col)
            return mid;
        if (a->ci[mid] < col)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i)
        f *= i;
    return f;
}

/* ------------------------------------------------------------------ */
/* P1 element matrices (Section 3: "standard mass and stiffness        */
/* matrices").  Lambda_0..d are the barycentric coordinates; their     */
/* gradients come from the inverse of J = [x1-x0, ..., xd-x0].         */
/*   K_T[a][b] = |T| grad(lambda_a) . grad(lambda_b)                   */
/*   M_T[a][b] = |T| (1 + delta_ab) / ((d+1)(d+2))                     */

int orc_element_matrices(int dim, const double *xv, double *MT, double *KT, double *vol)
{
    if (dim != 2 && dim != 3)
        return ORC_EINVAL;
    double J[3][3], Ji[3][3], det;
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            J[r][c] = xv[(c + 1) * dim + r] - xv[r]; /* column c = x_{c+1} - x_0 */
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (det == 0.0)
            return ORC_EINVAL;
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        if (det == 0.0)
            return ORC_EINVAL;
        /* inverse = adjugate / det; adj[r][c] = cofactor[c][r] */
        Ji[0][0] = c00 / det;
        Ji[1][0] = c01 / det;
        Ji[2][0] = c02 / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    double T = fabs(det) / factorial(dim);
    /* grad lambda_{a} for a = 1..d is row a-1 of J^-1; grad lambda_0 = -sum */
    double g[4][3];
    for (int c = 0; c < dim; ++c) {
        g[0][c] = 0.0;
        for (int a = 1; a <= dim; ++a) {
            g[a][c] = Ji[a - 1][c];
            g[0][c] -= Ji[a - 1][c];
        }
    }
    int nl = dim + 1;
    for (int a = 0; a < nl; ++a)
        for (int b = 0; b < nl; ++b) {
            double s = 0.0;
            for (int c = 0; c < dim; ++c)
                s += g[a][c] * g[b][c];
            KT[a * nl + b] = T * s;
            MT[a * nl + b] = T * (a == b ? 2.0 : 1.0) / ((dim + 1) * (dim + 2));
        }
    if (vol)
        *vol = T;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Quadrature for f_j = integral over T of f'(phi_h) lambda_j.          */
/* The paper assembles this term with UFL and does not state a rule.   */
/* Reading: the collapsed-coordinate (conical product) Gauss rule with  */
/* three points per direction, exact for polynomials of degree 5.       */
/* Direction k of a d-simplex carries the Jacobi weight (1-u)^(d-1-k);  */
/* its nodes are the zeros of the Jacobi polynomial P_3^(alpha,0),      */
/* found by Newton's method on the three-term recurrence, and its       */
/* weights are 2^(alpha+1) / ((1-t^2) P_3'(t)^2) on [-1,1].             */

/* P_n^(a,b)(x) by the standard three-term recurrence */
static double jacobi_p(int n, double a, double b, double x)
{
    if (n == 0)
        return 1.0;
    double p0 = 1.0, p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
    for (int k = 2; k <= n; ++k) {
        double c = 2.0 * k + a + b;
        double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
        double a2 = (c - 1.0) * (a * a - b * b);
        double a3 = (c - 2.0) * (c - 1.0) * c;
        double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* d/dx P_n^(a,b) = (n+a+b+1)/2 * P_{n-1}^(a+1,b+1) */
static double jacobi_dp(int n, double a, double b, double x)
{
    if (n == 0)
        return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x);
}

/* nodes u in [0,1] and weights for integral_0^1 (1-u)^alpha g(u) du, 3 points */
static void gauss_jacobi3(double alpha, double *u, double *w)
{
    const int n = 3;
    double t[3];
    for (int k = 0; k < n; ++k) {
        /* Chebyshev-like start, then Newton with deflation of found roots */
        double x = -cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
        for (int it = 0; it < 100; ++it) {
            double p = jacobi_p(n, alpha, 0.0, x);
            double dp = jacobi_dp(n, alpha, 0.0, x);
            double s = 0.0;
            for (int j = 0; j < k; ++j)
                s += 1.0 / (x - t[j]);
            double dx = p / (dp - s * p);
            x -= dx;
            if (fabs(dx) < 1e-16)
                break;
        }
        t[k] = x;
    }
    for (int k = 0; k < n; ++k) {
        double dp = jacobi_dp(n, alpha, 0.0, t[k]);
        double wk = pow(2.0, alpha + 1.0) / ((1.0 - t[k] * t[k]) * dp * dp);
        u[k] = 0.5 * (1.0 + t[k]);
        w[k] = wk * pow(0.5, alpha + 1.0); /* du = dt/2 and (1-u) = (1-t)/2 */
    }
}

int orc_quadrature(int dim, int *npts, double *bary, double *w)
{
    double u[3][3], wu[3][3];
    if (dim < 1 || dim > 3)
        return ORC_EINVAL;
    for (int k = 0; k < dim; ++k)
        gauss_jacobi3((double)(dim - 1 - k), u[k], wu[k]);
    int q = 0;
    double vol = 1.0 / factorial(dim);
    if (dim == 1) {   /* Gauss-Legendre on an edge (weight (1-u)^0) */
        for (int a = 0; a < 3; ++a) {
            bary[q * 2 + 1] = u[0][a];
            bary[q * 2 + 0] = 1.0 - u[0][a];
            w[q] = wu[0][a];
            ++q;
        }
    } else if (dim == 2) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double x = u[0][a];
                double y = u[1][b] * (1.0 - u[0][a]);
                bary[q * 3 + 1] = x;
                bary[q * 3 + 2] = y;
                bary[q * 3 + 0] = 1.0 - x - y;
                w[q] = wu[0][a] * wu[1][b] / vol;
                ++q;
            }
    } else {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    double x = u[0][a];
                    double y = u[1][b] * (1.0 - u[0][a]);
                    double z = u[2][c] * (1.0 - u[1][b]) * (1.0 - u[0][a]);
                    bary[q * 4 + 1] = x;
                    bary[q * 4 + 2] = y;
                    bary[q * 4 + 3] = z;
                    bary[q * 4 + 0] = 1.0 - x - y - z;
                    w[q] = wu[0][a] * wu[1][b] * wu[2][c] / vol;
                    ++q;
                }
    }
    *npts = q;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Bulk potential (Section 2, eq. logarithmicpotential; Section 4,      */
/* eq. polynomial_potential).  phi_s = 1 - phi_p - phi_n (only phi_p    */
/* and phi_n are unknowns), so the derivatives are total derivatives    */
/* with d(phi_s)/d(phi_p) = d(phi_s)/d(phi_n) = -1.                     */

static double clamp_log(double x, double floor_, int *clamped)
{
    if (x < floor_) {
        if (clamped)
            ++*clamped;
        x = floor_;
    }
    return log(x);
}

static void potential_eval(const orc_params_t *p, double php, double phn, double *f,
                           double *fp, double *fn, int *clamped)
{
    double phs = 1.0 - php - phn;
    if (p->potential == ORC_POT_FLORY_HUGGINS) {
        double lp = clamp_log(php, p->log_floor, clamped);
        double ln_ = clamp_log(phn, p->log_floor, clamped);
        double ls = clamp_log(phs, p->log_floor, clamped);
        if (f)
            *f = php * lp / p->Np + phn * ln_ / p->Nn + phs * ls / p->Ns + p->chi_pn * php * phn
                 + p->chi_ps * php * phs + p->chi_ns * phn * phs;
        /* d/dphi_p of (phi ln phi)/N is (ln phi + 1)/N; the solvent term enters with -1 */
        if (fp)
            *fp = (lp + 1.0) / p->Np - (ls + 1.0) / p->Ns + p->chi_pn * phn
                  + p->chi_ps * (phs - php) - p->chi_ns * phn;
        if (fn)
            *fn = (ln_ + 1.0) / p->Nn - (ls + 1.0) / p->Ns + p->chi_pn * php - p->chi_ps * php
                  + p->chi_ns * (phs - phn);
    } else if (p->potential == ORC_POT_POLYNOMIAL) {
        /* f = 3.5 phi_p^2 phi_n^2 + 0.1 phi_s^2 */
        if (f)
            *f = 3.5 * php * php * phn * phn + 0.1 * phs * phs;
        if (fp)
            *fp = 7.0 * php * phn * phn - 0.2 * phs;
        if (fn)
            *fn = 7.0 * php * php * phn - 0.2 * phs;
    } else {
        if (f)
            *f = 0.0;
        if (fp)
            *fp = 0.0;
        if (fn)
            *fn = 0.0;
    }
}

int orc_potential(const orc_params_t *p, double php, double phn, double *f, double *fp, double *fn)
{
    if (!p)
        return ORC_EINVAL;
    potential_eval(p, php, phn, f, fp, fn, NULL);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Assembly.  Pattern = vertex adjacency through cells plus the         */
/* diagonal, columns ascending; M and K share it (K keeps the entries   */
/* that cancel to zero).  Values are summed over cells in index order.  */

static int assemble(orc_solver_t *s)
{
    int nv = s->nv, nl = s->dim + 1;
    int *cnt = calloc((size_t)nv + 1, sizeof(int));
    if (!cnt)
        return ORC_ENOMEM;
    for (int c = 0; c < s->ncell; ++c)
        for (int a = 0; a < nl; ++a)
            cnt[s->cells[c * nl + a] + 1] += nl;
    for (int i = 0; i < nv; ++i)
        cnt[i + 1] += cnt[i];
    int *lst = malloc(sizeof(int) * (size_t)(cnt[nv] > 0 ? cnt[nv] : 1));
    int *fill = calloc((size_t)nv, sizeof(int));
    if (!lst || !fill) {
        free(cnt);
        free(lst);
        free(fill);
        return ORC_ENOMEM;
    }
    for (int c = 0; c < s->ncell; ++c)
        for (int a = 0; a < nl; ++a) {
            int i = s->cells[c * nl + a];
            for (int b = 0; b < nl; ++b)
                lst[cnt[i] + fill[i]++] = s->cells[c * nl + b];
        }
    s->M.n = s->M.m = nv;
    s->M.rp = calloc((size_t)nv + 1, sizeof(int));
    int total = 0;
    for (int i = 0; i < nv; ++i) {
        int *seg = lst + cnt[i];
        int len = cnt[i + 1] - cnt[i];
        qsort(seg, (size_t)len, sizeof(int), cmp_int);
        int u = 0;
        for (int k = 0; k < len; ++k)
            if (u == 0 || seg[k] != seg[u - 1])
                seg[u++] = seg[k];
        fill[i] = u;
        total += u;
        s->M.rp[i + 1] = total;
    }
    s->M.ci = malloc(sizeof(int) * (size_t)(total ? total : 1));
    s->M.v = calloc((size_t)(total ? total : 1), sizeof(double));
    for (int i = 0; i < nv; ++i)
        memcpy(s->M.ci + s->M.rp[i], lst + cnt[i], sizeof(int) * (size_t)fill[i]);
    free(lst);
    free(fill);
    free(cnt);
    s->K = s->M;
    s->K.rp = malloc(sizeof(int) * ((size_t)nv + 1));
    s->K.ci = malloc(sizeof(int) * (size_t)(total ? total : 1));
    s->K.v = calloc((size_t)(total ? total : 1), sizeof(double));
    memcpy(s->K.rp, s->M.rp, sizeof(int) * ((size_t)nv + 1));
    memcpy(s->K.ci, s->M.ci, sizeof(int) * (size_t)total);

    double xv[4 * 3], MT[16], KT[16];
    for (int c = 0; c < s->ncell; ++c) {
        for (int a = 0; a < nl; ++a)
            for (int d = 0; d < s->dim; ++d)
                xv[a * s->dim + d] = s->coords[(size_t)s->cells[c * nl + a] * s->dim + d];
        int rc = orc_element_matrices(s->dim, xv, MT, KT, NULL);
        if (rc)
            return rc;
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nl; ++b) {
                int k = find_col(&s->M, s->cells[c * nl + a], s->cells[c * nl + b]);
                s->M.v[k] += MT[a * nl + b];
                s->K.v[k] += KT[a * nl + b];
            }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Smoothed-aggregation AMG (the paper's AMG, Section 4, is replaced    */
/* by smoothed aggregation: Vanek, Mandel and Brezina 1996).            */
/*                                                                      */
/* Strength: every stored off-diagonal entry (structural graph), so the */
/* hierarchy's shape depends only on the sparsity pattern.              */
/* Aggregation roots: a distance-2 maximal independent set built in     */
/* synchronous rounds (Bell, Dalton and Olson 2012): every node holds    */
/* the tuple (state, hash, index) with state IN > UNDECIDED > OUT;      */
/* two rounds of "max over self and neighbours" give each node the      */
/* largest tuple within distance 2; an undecided node that finds its     */
/* own tuple becomes IN, one that finds an IN tuple becomes OUT.        */
/* hash(i) is the SplitMix64 output for counter i of stream 0.           */

static uint64_t mix64(uint64_t i)
{
    uint64_t z = (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    int state; /* 0 OUT, 1 UNDECIDED, 2 IN */
    uint64_t h;
    int idx;
} tup_t;

static int tup_gt(const tup_t *a, const tup_t *b)
{
    if (a->state != b->state)
        return a->state > b->state;
    if (a->h != b->h)
        return a->h > b->h;
    return a->idx > b->idx;
}

static int mis2_roots(const csr_t *A, int *state)
{
    int n = A->n;
    tup_t *t0 = malloc(sizeof(tup_t) * (size_t)n);
    tup_t *t1 = malloc(sizeof(tup_t) * (size_t)n);
    if (!t0 || !t1) {
        free(t0);
        free(t1);
        return ORC_ENOMEM;
    }
    for (int i = 0; i < n; ++i)
        state[i] = 1;
    for (;;) {
        int undecided = 0;
        for (int i = 0; i < n; ++i)
            undecided += (state[i] == 1);
        if (!undecided)
            break;
        for (int i = 0; i < n; ++i) {
            t0[i].state = state[i];
            t0[i].h = mix64((uint64_t)i);
            t0[i].idx = i;
        }
        for (int sweep = 0; sweep < 2; ++sweep) {
            for (int i = 0; i < n; ++i) {
                tup_t best = t0[i];
                for (int k = A->rp[i]; k < A->rp[i + 1]; ++k)
                    if (tup_gt(&t0[A->ci[k]], &best))
                        best = t0[A->ci[k]];
                t1[i] = best;
            }
            tup_t *tmp = t0;
            t0 = t1;
            t1 = tmp;
        }
        for (int i = 0; i < n; ++i) {
            if (state[i] != 1)
                continue;
            if (t0[i].idx == i)
                state[i] = 2;
            else if (t0[i].state == 2)
                state[i] = 0;
        }
    }
    free(t0);
    free(t1);
    return ORC_OK;
}

/* Aggregates: roots numbered by increasing node index; every node next */
/* to a root joins it (at most one root is adjacent, roots being at      */
/* distance >= 3); every other node joins, among its neighbours placed  */
/* in that first pass, the one with the smallest aggregate number.       */
static int aggregate(const csr_t *A, int *agg, int *nagg)
{
    int n = A->n;
    int *state = malloc(sizeof(int) * (size_t)(n ? n : 1));
    int *first = malloc(sizeof(int) * (size_t)(n ? n : 1));
    if (!state || !first) {
        free(state);
        free(first);
        return ORC_ENOMEM;
    }
    int rc = mis2_roots(A, state);
    if (rc) {
        free(state);
        free(first);
        return rc;
    }
    int na = 0;
    for (int i = 0; i < n; ++i)
        agg[i] = (state[i] == 2) ? na++ : -1;
    for (int i = 0; i < n; ++i) {
        first[i] = agg[i];
        if (first[i] >= 0)
            continue;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k)
            if (state[A->ci[k]] == 2)
                first[i] = agg[A->ci[k]];
    }
    for (int i = 0; i < n; ++i) {
        if (first[i] >= 0) {
            agg[i] = first[i];
            continue;
        }
        int best = -1;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int a = first[A->ci[k]];
            if (a >= 0 && (best < 0 || a < best))
                best = a;
        }
        agg[i] = best; /* >= 0 whenever the root set is distance-2 maximal */
    }
    free(state);
    free(first);
    *nagg = na;
    for (int i = 0; i < n; ++i)
        if (agg[i] < 0)
            return ORC_EINVAL;
    return ORC_OK;
}

/* C = A * B by rows with a dense accumulator; the pattern is symbolic   */
/* (an entry exists when some product touches it, even if it sums to 0).*/
static int spgemm(const csr_t *A, const csr_t *B, csr_t *C)
{
    int n = A->n, m = B->m;
    double *acc = calloc((size_t)(m ? m : 1), sizeof(double));
    int *mark = malloc(sizeof(int) * (size_t)(m ? m : 1));
    int *touched = malloc(sizeof(int) * (size_t)(m ? m : 1));
    C->n = n;
    C->m = m;
    C->rp = calloc((size_t)n + 1, sizeof(int));
    if (!acc || !mark || !touched || !C->rp)
        return ORC_ENOMEM;
    for (int j = 0; j < m; ++j)
        mark[j] = -1;
    /* symbolic pass */
    for (int i = 0; i < n; ++i) {
        int cnt = 0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int j = A->ci[k];
            for (int l = B->rp[j]; l < B->rp[j + 1]; ++l)
                if (mark[B->ci[l]] != i) {
                    mark[B->ci[l]] = i;
                    ++cnt;
                }
        }
        C->rp[i + 1] = C->rp[i] + cnt;
    }
    int nnz = C->rp[n];
    C->ci = malloc(sizeof(int) * (size_t)(nnz ? nnz : 1));
    C->v = malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
    if (!C->ci || !C->v)
        return ORC_ENOMEM;
    for (int j = 0; j < m; ++j)
        mark[j] = -1;
    for (int i = 0; i < n; ++i) {
        int nt = 0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int j = A->ci[k];
            double a = A->v[k];
            for (int l = B->rp[j]; l < B->rp[j + 1]; ++l) {
                int c = B->ci[l];
                if (mark[c] != i) {
                    mark[c] = i;
                    acc[c] = 0.0;
                    touched[nt++] = c;
                }
                acc[c] += a * B->v[l];
            }
        }
        qsort(touched, (size_t)nt, sizeof(int), cmp_int);
        for (int t = 0; t < nt; ++t) {
            C->ci[C->rp[i] + t] = touched[t];
            C->v[C->rp[i] + t] = acc[touched[t]];
        }
    }
    free(acc);
    free(mark);
    free(touched);
    return ORC_OK;
}

static int transpose(const csr_t *A, csr_t *T)
{
    int n = A->n, m = A->m, nnz = A->rp[n];
    T->n = m;
    T->m = n;
    T->rp = calloc((size_t)m + 1, sizeof(int));
    T->ci = malloc(sizeof(int) * (size_t)(nnz ? nnz : 1));
    T->v = malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
    int *pos = malloc(sizeof(int) * (size_t)(m ? m : 1));
    if (!T->rp || !T->ci || !T->v || !pos)
        return ORC_ENOMEM;
    for (int k = 0; k < nnz; ++k)
        T->rp[A->ci[k] + 1]++;
    for (int j = 0; j < m; ++j)
        T->rp[j + 1] += T->rp[j];
    for (int j = 0; j < m; ++j)
        pos[j] = T->rp[j];
    for (int i = 0; i < n; ++i) /* rows in order, so each column of T stays ascending */
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int p = pos[A->ci[k]]++;
            T->ci[p] = i;
            T->v[p] = A->v[k];
        }
    free(pos);
    return ORC_OK;
}

static int csr_copy(const csr_t *A, csr_t *B)
{
    int nnz = A->rp[A->n];
    B->n = A->n;
    B->m = A->m;
    B->rp = malloc(sizeof(int) * ((size_t)A->n + 1));
    B->ci = malloc(sizeof(int) * (size_t)(nnz ? nnz : 1));
    B->v = malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
    if (!B->rp || !B->ci || !B->v)
        return ORC_ENOMEM;
    memcpy(B->rp, A->rp, sizeof(int) * ((size_t)A->n + 1));
    memcpy(B->ci, A->ci, sizeof(int) * (size_t)nnz);
    memcpy(B->v, A->v, sizeof(double) * (size_t)nnz);
    return ORC_OK;
}

static int level_diag(level_t *L)
{
    const csr_t *A = &L->A;
    L->invdiag = malloc(sizeof(double) * (size_t)(A->n ? A->n : 1));
    if (!L->invdiag)
        return ORC_ENOMEM;
    L->rho = 0.0;
    for (int i = 0; i < A->n; ++i) {
        double d = 0.0, row = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            if (A->ci[k] == i)
                d = A->v[k];
            row += fabs(A->v[k]);
        }
        if (!(d > 0.0))
            return ORC_EINVAL; /* the operators here are SPD */
        L->invdiag[i] = 1.0 / d;
        if (row / d > L->rho)
            L->rho = row / d;
    }
    return ORC_OK;
}

static int dense_cholesky(level_t *L)
{
    int n = L->n;
    double *a = calloc((size_t)n * (size_t)n, sizeof(double));
    if (!a)
        return ORC_ENOMEM;
    for (int i = 0; i < n; ++i)
        for (int k = L->A.rp[i]; k < L->A.rp[i + 1]; ++k)
            a[(size_t)i * n + L->A.ci[k]] = L->A.v[k];
    for (int j = 0; j < n; ++j) {
        double d = a[(size_t)j * n + j];
        for (int k = 0; k < j; ++k)
            d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(d > 0.0)) {
            free(a);
            return ORC_EINVAL;
        }
        d = sqrt(d);
        a[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = a[(size_t)i * n + j];
            for (int k = 0; k < j; ++k)
                v -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = v / d;
        }
    }
    L->chol = a;
    return ORC_OK;
}

static void hier_free(hier_t *h)
{
    for (int l = 0; l < h->nlev; ++l) {
        level_t *L = &h->lev[l];
        csr_free(&L->A);
        csr_free(&L->P);
        csr_free(&L->R);
        free(L->invdiag);
        free(L->agg);
        free(L->chol);
    }
    memset(h, 0, sizeof(*h));
}

/* degree: the smoother degree of the finest level; degree_coarse: of the  */
/* levels below it (0: degree)                                            */
static int hier_build(const orc_params_t *prm, const csr_t *A0, double ratio, int degree,
                      int degree_coarse, hier_t *h)
{
    int rc;
    memset(h, 0, sizeof(*h));
    h->ratio = ratio;
    int maxlev = prm->max_levels < MAXLEV ? prm->max_levels : MAXLEV;
    if (maxlev < 1)
        maxlev = 1;
    double *B = malloc(sizeof(double) * (size_t)(A0->n ? A0->n : 1));
    if (!B)
        return ORC_ENOMEM;
    for (int i = 0; i < A0->n; ++i)
        B[i] = 1.0; /* constants: the near-null space of the stiffness part */
    if ((rc = csr_copy(A0, &h->lev[0].A)))
        return rc;
    h->lev[0].n = A0->n;
    h->nlev = 1;
    for (int l = 0;; ++l) {
        level_t *L = &h->lev[l];
        L->degree = (l > 0 && degree_coarse > 0) ? degree_coarse : degree;
        if ((rc = level_diag(L)))
            return rc;
        if (L->n <= prm->coarse_max || l + 1 >= maxlev)
            break;
        L->agg = malloc(sizeof(int) * (size_t)L->n);
        if (!L->agg)
            return ORC_ENOMEM;
        if ((rc = aggregate(&L->A, L->agg, &L->nc)))
            return rc;
        if (L->nc >= L->n || L->nc == 0) { /* no coarsening possible: stop here */
            free(L->agg);
            L->agg = NULL;
            break;
        }
        /* tentative prolongator: T[i, agg(i)] = B_i / ||B restricted to agg(i)|| */
        double *Bn = calloc((size_t)L->nc, sizeof(double));
        if (!Bn)
            return ORC_ENOMEM;
        for (int i = 0; i < L->n; ++i)
            Bn[L->agg[i]] += B[i] * B[i];
        for (int a = 0; a < L->nc; ++a)
            Bn[a] = sqrt(Bn[a]);
        /* P = (I - omega D^-1 A) T, omega = 4 / (3 rho) */
        double omega = 4.0 / (3.0 * L->rho);
        csr_t T = {0};
        T.n = L->n;
        T.m = L->nc;
        T.rp = malloc(sizeof(int) * ((size_t)L->n + 1));
        T.ci = malloc(sizeof(int) * (size_t)L->n);
        T.v = malloc(sizeof(double) * (size_t)L->n);
        if (!T.rp || !T.ci || !T.v)
            return ORC_ENOMEM;
        for (int i = 0; i <= L->n; ++i)
            T.rp[i] = i;
        for (int i = 0; i < L->n; ++i) {
            T.ci[i] = L->agg[i];
            T.v[i] = B[i] / Bn[L->agg[i]];
        }
        csr_t S = {0}; /* S = I - omega D^-1 A, same pattern as A */
        if ((rc = csr_copy(&L->A, &S)))
            return rc;
        for (int i = 0; i < S.n; ++i)
            for (int k = S.rp[i]; k < S.rp[i + 1]; ++k)
                S.v[k] = (S.ci[k] == i ? 1.0 : 0.0) - omega * L->invdiag[i] * L->A.v[k];
        if ((rc = spgemm(&S, &T, &L->P)))
            return rc;
        csr_free(&S);
        csr_free(&T);
        if ((rc = transpose(&L->P, &L->R)))
            return rc;
        csr_t AP = {0};
        if ((rc = spgemm(&L->A, &L->P, &AP)))
            return rc;
        level_t *C = &h->lev[l + 1];
        if ((rc = spgemm(&L->R, &AP, &C->A)))
            return rc;
        csr_free(&AP);
        C->n = L->nc;
        h->nlev = l + 2;
        free(B);
        B = Bn;
    }
    free(B);
    return dense_cholesky(&h->lev[h->nlev - 1]);
}

/* ------------------------------------------------------------------ */
/* V-cycle.  Smoothing: Chebyshev polynomial of the given degree in     */
/* D^-1 A over [rho/ratio, rho] (three-term recurrence of Chebyshev     */
/* acceleration, Saad, Iterative Methods, Algorithm 12.1) or that many   */
/* damped-Jacobi sweeps with weight 4/(3 rho); one application before   */
/* and one after the coarse correction.  Coarsest level: dense          */
/* Cholesky solve.                                                      */

static void smooth(const orc_params_t *prm, const hier_t *h, const level_t *L, const double *b,
                   double *x, double *r, double *d)
{
    int n = L->n;
    if (prm->smoother == ORC_SMOOTH_JACOBI) {
        double omega = 4.0 / (3.0 * L->rho);
        for (int it = 0; it < L->degree; ++it) {
            csr_mv(&L->A, x, r);
            #pragma omp parallel for schedule(static) if (n >= 4096)
            for (int i = 0; i < n; ++i)
                x[i] += omega * L->invdiag[i] * (b[i] - r[i]);
        }
        return;
    }
    double lmax = L->rho, lmin = L->rho / h->ratio;
    double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    double sigma = theta / delta, rho_old = 1.0 / sigma;
    csr_mv(&L->A, x, r);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i)
        d[i] = L->invdiag[i] * (b[i] - r[i]) / theta;
    for (int k = 1; k <= L->degree; ++k) {
        #pragma omp parallel for schedule(static) if (n >= 4096)
        for (int i = 0; i < n; ++i)
            x[i] += d[i];
        if (k == L->degree)
            break;
        csr_mv(&L->A, x, r);
        double rho = 1.0 / (2.0 * sigma - rho_old);
        #pragma omp parallel for schedule(static) if (n >= 4096)
        for (int i = 0; i < n; ++i)
            d[i] = rho * rho_old * d[i] + (2.0 * rho / delta) * L->invdiag[i] * (b[i] - r[i]);
        rho_old = rho;
    }
}

static void coarse_solve(const level_t *L, const double *b, double *x)
{
    int n = L->n;
    const double *a = L->chol;
    for (int i = 0; i < n; ++i) { /* L y = b */
        double v = b[i];
        for (int k = 0; k < i; ++k)
            v -= a[(size_t)i * n + k] * x[k];
        x[i] = v / a[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) { /* L^T x = y */
        double v = x[i];
        for (int k = i + 1; k < n; ++k)
            v -= a[(size_t)k * n + i] * x[k];
        x[i] = v / a[(size_t)i * n + i];
    }
}

/* x = V-cycle(b) starting from x = 0 */
static void vcycle(const orc_params_t *prm, const hier_t *h, int l, const double *b, double *x)
{
    const level_t *L = &h->lev[l];
    int n = L->n;
    if (l == h->nlev - 1) {
        coarse_solve(L, b, x);
        return;
    }
    double *r = malloc(sizeof(double) * (size_t)n);
    double *d = malloc(sizeof(double) * (size_t)n);
    double *bc = malloc(sizeof(double) * (size_t)L->nc);
    double *xc = malloc(sizeof(double) * (size_t)L->nc);
    double *e = malloc(sizeof(double) * (size_t)n);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i)
        x[i] = 0.0;
    smooth(prm, h, L, b, x, r, d);
    csr_mv(&L->A, x, r);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i)
        r[i] = b[i] - r[i];
    csr_mv(&L->R, r, bc);
    vcycle(prm, h, l + 1, bc, xc);
    csr_mv(&L->P, xc, e);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i)
        x[i] += e[i];
    smooth(prm, h, L, b, x, r, d);
    free(r);
    free(d);
    free(bc);
    free(xc);
    free(e);
}

/* Stationary AMG solve: V-cycles from a zero guess, x <- x + V(b - A x): */
/* amg_cycles of them, or with amg_tol > 0 until the residual norm is at  */
/* most amg_tol ||b|| (at least one cycle, at most amg_cycles).           */
static void amg_stationary(const orc_params_t *prm, const hier_t *h, const double *b, double *x)
{
    int n = h->lev[0].n;
    vcycle(prm, h, 0, b, x);
    if (prm->amg_cycles <= 1)
        return;
    double *r = malloc(sizeof(double) * (size_t)n);
    double *e = malloc(sizeof(double) * (size_t)n);
    const double bnorm = prm->amg_tol > 0.0 ? sqrt(dot(n, b, b)) : 0.0;
    for (int c = 1; c < prm->amg_cycles; ++c) {
        csr_mv(&h->lev[0].A, x, r);
        #pragma omp parallel for schedule(static) if (n >= 4096)
        for (int i = 0; i < n; ++i)
            r[i] = b[i] - r[i];
        if (prm->amg_tol > 0.0 && sqrt(dot(n, r, r)) <= prm->amg_tol * bnorm)
            break;
        vcycle(prm, h, 0, r, e);
        #pragma omp parallel for schedule(static) if (n >= 4096)
        for (int i = 0; i < n; ++i)
            x[i] += e[i];
    }
    free(r);
    free(e);
}

/* Krylov-accelerated AMG solve: k steps of conjugate gradients from a   */
/* zero guess with one V-cycle as preconditioner (Hestenes-Stiefel      */
/* recurrences).  A step whose curvature d.Ad or r.z vanishes takes a   */
/* zero step length (this happens only for b = 0).                      */
static void amg_pcg(const orc_params_t *prm, const hier_t *h, int k, const double *b, double *x)
{
    int n = h->lev[0].n;
    const csr_t *A = &h->lev[0].A;
    double *r = calloc((size_t)n + 1, sizeof(double)), *z = malloc(sizeof(double) * (size_t)n);
    double *d = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
    }
    vcycle(prm, h, 0, r, z);
    memcpy(d, z, sizeof(double) * (size_t)n);
    double rz = dot(n, r, z);
    for (int it = 1; it <= k; ++it) {
        csr_mv(A, d, q);
        double dq = dot(n, d, q);
        double alpha = dq != 0.0 ? rz / dq : 0.0;
        #pragma omp parallel for schedule(static) if (n >= 4096)
        for (int i = 0; i < n; ++i) {
            x[i] += alpha * d[i];
            r[i] -= alpha * q[i];
        }
        if (it == k)
            break;
        vcycle(prm, h, 0, r, z);
        double rz_new = dot(n, r, z);
        double beta = rz != 0.0 ? rz_new / rz : 0.0;
        #pragma omp parallel for schedule(static) if (n >= 4096)
        for (int i = 0; i < n; ++i)
            d[i] = z[i] + beta * d[i];
        rz = rz_new;
    }
    free(r);
    free(z);
    free(d);
    free(q);
}

/* Contraction of one V-cycle V of an As hierarchy in the As-norm, for     */
/* choosing the number of inner CG steps (schur_pcg = -1): the power       */
/* iteration e <- (I - V As) e, six steps, from the start e_i = 2u - 1     */
/* with u the top 53 bits of SplitMix64 counter 2^32 + 2 i + species       */
/* divided by 2^53; the result is ||e_6||_As / ||e_5||_As.  The V-cycle is */
/* symmetric, so I - V As is self-adjoint in the As inner product and the  */
/* ratio approaches its spectral radius from below.  Returns -1 when out  */
/* of memory.                                                             */
static double vcycle_contraction(const orc_params_t *prm, const hier_t *h, int species)
{
    const csr_t *A = &h->lev[0].A;
    int n = A->n;
    double *e = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    if (!e || !q || !z) {
        free(e);
        free(q);
        free(z);
        return -1.0;
    }
    for (int i = 0; i < n; ++i) {
        uint64_t c = (1ull << 32) + 2ull * (uint64_t)i + (uint64_t)species;
        e[i] = 2.0 * ((double)(mix64(c) >> 11) / 9007199254740992.0) - 1.0;
    }
    double prev = 0.0, rho = 0.0;
    for (int it = 0; it <= 6; ++it) {
        csr_mv(A, e, q);
        double a = dot(n, e, q);
        if (it > 0)
            rho = prev > 0.0 ? sqrt((a > 0.0 ? a : 0.0) / prev) : 0.0;
        prev = a;
        if (it == 6)
            break;
        vcycle(prm, h, 0, q, z);
        for (int i = 0; i < n; ++i)
            e[i] -= z[i];
    }
    free(e);
    free(q);
    free(z);
    return rho;
}

/* the AMG solve used for the As systems of Algorithm 1 */
static void amg_schur(const orc_params_t *prm, const hier_t *h, const double *b, double *x)
{
    if (prm->schur_pcg > 0)
        amg_pcg(prm, h, prm->schur_pcg, b, x);
    else
        amg_stationary(prm, h, b, x);
}

/* ------------------------------------------------------------------ */
/* Saddle-point operator of species s (eq. saddle_point_system):        */
/*   [ M        tau' K        ] [phi]                                    */
/*   [ tau' K   -(tau'/eps) M ] [mu ]   with tau' = tau * mobility.      */

static double tau_s(const orc_params_t *p, int sp) { return p->tau * p->mobility[sp]; }

static void saddle(const orc_solver_t *s, int sp, const double *x, double *y)
{
    int n = s->nv;
    double t = tau_s(&s->prm, sp), te = t / s->prm.eps[sp];
    double *a = malloc(sizeof(double) * (size_t)n), *b = malloc(sizeof(double) * (size_t)n);
    csr_mv(&s->M, x, a);
    csr_mv(&s->K, x + n, b);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i)
        y[i] = a[i] + t * b[i];
    csr_mv(&s->K, x, a);
    csr_mv(&s->M, x + n, b);
    #pragma omp parallel for schedule(static) if (n >= 4096)
    for (int i = 0; i < n; ++i)
        y[n + i] = t * a[i] - te * b[i];
    free(a);
    free(b);
}

/* Algorithm 1: w1 ~ M^-1 v1; w2 ~ As^-1 M As^-1 v2 with                */
/* As = tau' K + sqrt(tau'/eps) M, i.e. the inverse of the matching      */
/* Schur approximation S~ = As M^-1 As.                                 */
static void prec(const orc_solver_t *s, int sp, const double *v, double *w)
{
    int n = s->nv;
    double *t = malloc(sizeof(double) * (size_t)n), *u = malloc(sizeof(double) * (size_t)n);
    if (s->prm.mass_solver == ORC_MASS_CHEBYSHEV) {
        /* w1 = the Chebyshev semi-iteration on M from zero (t, u as work) */
        memset(w, 0, sizeof(double) * (size_t)n);
        smooth(&s->prm, &s->hM, &s->hM.lev[0], v, w, t, u);
    } else {
        amg_stationary(&s->prm, &s->hM, v, w);
    }
    amg_schur(&s->prm, &s->hA[sp], v + n, t);
    csr_mv(&s->M, t, u);
    amg_schur(&s->prm, &s->hA[sp], u, w + n);
    free(t);
    free(u);
}

/* ------------------------------------------------------------------ */
/* Flexible GMRES(m), right preconditioned (Saad 1993), modified        */
/* Gram-Schmidt, Givens rotations.  Stops when the Arnoldi residual     */
/* estimate is at most rtol * ||b||_2; the true residual is then        */
/* checked and the method restarts if that check fails.                 */

static int fgmres(const orc_solver_t *s, int sp, const double *b, double *x, int32_t *iters,
                  double *relres)
{
    const orc_params_t *p = &s->prm;
    int n2 = 2 * s->nv, m = p->restart;
    if (m < 1)
        return ORC_EINVAL;
    double *V = malloc(sizeof(double) * (size_t)n2 * (m + 1));
    double *Z = malloc(sizeof(double) * (size_t)n2 * m);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *g = malloc(sizeof(double) * (m + 1)), *y = malloc(sizeof(double) * m);
    double *r = malloc(sizeof(double) * (size_t)n2);
    int rc = ORC_OK, total = 0;
    double bnorm = sqrt(dot(n2, b, b));
    double tol = p->rtol * bnorm;
    double res = 0.0;
    for (;;) {
        saddle(s, sp, x, r);
        #pragma omp parallel for schedule(static) if (n2 >= 4096)
        for (int i = 0; i < n2; ++i)
            r[i] = b[i] - r[i];
        double beta = sqrt(dot(n2, r, r));
        res = beta;
        if (!isfinite(beta)) {
            rc = ORC_ENAN;
            break;
        }
        if (beta <= tol)
            break;
        if (total >= p->max_iters) {
            rc = ORC_ENOCONV;
            break;
        }
        #pragma omp parallel for schedule(static) if (n2 >= 4096)
        for (int i = 0; i < n2; ++i)
            V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i)
            g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && total < p->max_iters; ++j) {
            double *vj = V + (size_t)j * n2, *zj = Z + (size_t)j * n2, *w = V + (size_t)(j + 1) * n2;
            prec(s, sp, vj, zj);
            saddle(s, sp, zj, w);
            for (int i = 0; i <= j; ++i) {
                double hij = dot(n2, w, V + (size_t)i * n2);
                H[i * m + j] = hij;
                #pragma omp parallel for schedule(static) if (n2 >= 4096)
                for (int t = 0; t < n2; ++t)
                    w[t] -= hij * V[(size_t)i * n2 + t];
            }
            double hn = sqrt(dot(n2, w, w));
            H[(j + 1) * m + j] = hn;
            if (hn > 0.0) {
                #pragma omp parallel for schedule(static) if (n2 >= 4096)
                for (int t = 0; t < n2; ++t)
                    w[t] /= hn;
            }
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double rr = sqrt(a * a + c * c);
            if (rr == 0.0) {
                cs[j] = 1.0;
                sn[j] = 0.0;
            } else {
                cs[j] = a / rr;
                sn[j] = c / rr;
            }
            H[j * m + j] = rr;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            k = j + 1;
            if (!isfinite(g[j + 1])) {
                rc = ORC_ENAN;
                break;
            }
            if (fabs(g[j + 1]) <= tol || hn == 0.0)
                break;
        }
        if (rc)
            break;
        for (int i = k - 1; i >= 0; --i) {
            double v = g[i];
            for (int t = i + 1; t < k; ++t)
                v -= H[i * m + t] * y[t];
            y[i] = v / H[i * m + i];
        }
        for (int i = 0; i < k; ++i) {
            #pragma omp parallel for schedule(static) if (n2 >= 4096)
            for (int t = 0; t < n2; ++t)
                x[t] += y[i] * Z[(size_t)i * n2 + t];
        }
    }
    *iters = total;
    *relres = bnorm > 0.0 ? res / bnorm : res;
    free(V);
    free(Z);
    free(H);
    free(cs);
    free(sn);
    free(g);
    free(y);
    free(r);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Boundary terms of eq. chternary:2 (Section 2; the coefficients of     */
/* Section 4).  A facet of a cell (the cell without one of its           */
/* vertices) lies on the top boundary when all its vertices have the     */
/* largest second coordinate of the mesh, on the bottom when all have    */
/* the smallest.  On the top, solvent evaporation enters as an inflow of */
/* polymer and acceptor, g_i = k phi_i phi_s; on the bottom, the         */
/* substrate flux g_i = p_i(x) (g_i + 2 h_i phi_i) with p_p = 1 on the   */
/* first, third and fifth sixth of the bottom and p_n = 1 on the others  */
/* (or p = 1 without patterning).  G_j = integral of g_i lambda_j over   */
/* the boundary facets, by the degree-5 rule of the facet's dimension.   */

static double facet_measure(int d, const double *xv, int dim)
{
    /* d = number of facet vertices (2: edge, 3: triangle); xv: d points */
    double e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        e1[k] = xv[dim + k] - xv[k];
        if (d == 3)
            e2[k] = xv[2 * dim + k] - xv[k];
    }
    if (d == 2)
        return sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    double c0 = e1[1] * e2[2] - e1[2] * e2[1], c1 = e1[2] * e2[0] - e1[0] * e2[2],
           c2 = e1[0] * e2[1] - e1[1] * e2[0];
    return 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
}

int orc_boundary(orc_solver_t *s, const double *php, const double *phn, double *gp, double *gn)
{
    if (!s || !php || !phn || !gp || !gn)
        return ORC_EINVAL;
    const int n = s->nv, dim = s->dim, nl = dim + 1, d = dim;
    const orc_params_t *p = &s->prm;
    for (int i = 0; i < n; ++i)
        gp[i] = gn[i] = 0.0;
    if (!p->boundary)
        return ORC_OK;
    double ymin = INFINITY, ymax = -INFINITY, xmin = INFINITY, xmax = -INFINITY;
    for (int i = 0; i < n; ++i) {
        ymin = fmin(ymin, s->coords[(size_t)i * dim + 1]);
        ymax = fmax(ymax, s->coords[(size_t)i * dim + 1]);
        xmin = fmin(xmin, s->coords[(size_t)i * dim]);
        xmax = fmax(xmax, s->coords[(size_t)i * dim]);
    }
    const double tol = 1e-12 * (ymax - ymin);
    int nq;
    double qb[64 * 4], qw[64];
    orc_quadrature(d - 1, &nq, qb, qw);
    for (int c = 0; c < s->ncell; ++c) {
        const int *v = s->cells + (size_t)c * nl;
        for (int omit = 0; omit < nl; ++omit) {
            int fv[3], k = 0;
            for (int a = 0; a < nl; ++a)
                if (a != omit)
                    fv[k++] = v[a];
            int top = 1, bot = 1;
            for (int a = 0; a < d; ++a) {
                const double y = s->coords[(size_t)fv[a] * dim + 1];
                top = top && fabs(y - ymax) <= tol;
                bot = bot && fabs(y - ymin) <= tol;
            }
            if (!top && !bot)
                continue;
            double xv[9];
            for (int a = 0; a < d; ++a)
                for (int k2 = 0; k2 < dim; ++k2)
                    xv[a * dim + k2] = s->coords[(size_t)fv[a] * dim + k2];
            const double meas = facet_measure(d, xv, dim);
            for (int q = 0; q < nq; ++q) {
                const double *lam = qb + q * d;
                double pp = 0.0, pn = 0.0, x = 0.0;
                for (int a = 0; a < d; ++a) {
                    pp += lam[a] * php[fv[a]];
                    pn += lam[a] * phn[fv[a]];
                    x += lam[a] * xv[a * dim];
                }
                double fp_, fn_;
                if (top) {
                    const double ps = 1.0 - pp - pn;
                    fp_ = p->bc_k * pp * ps;
                    fn_ = p->bc_k * pn * ps;
                } else {
                    double wp = 1.0, wn = 1.0;
                    if (p->bc_pattern) {
                        int six = (int)floor(6.0 * (x - xmin) / (xmax - xmin));
                        six = six < 0 ? 0 : (six > 5 ? 5 : six);
                        wp = (six % 2 == 0) ? 1.0 : 0.0;
                        wn = 1.0 - wp;
                    }
                    fp_ = wp * (p->bc_g[0] + 2.0 * p->bc_h[0] * pp);
                    fn_ = wn * (p->bc_g[1] + 2.0 * p->bc_h[1] * pn);
                }
                for (int a = 0; a < d; ++a) {
                    gp[fv[a]] += meas * qw[q] * fp_ * lam[a];
                    gn[fv[a]] += meas * qw[q] * fn_ * lam[a];
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Right-hand side (eq. saddle_point_system): b1 = M phi^k (+ tau G,    */
/* the boundary vector, when the boundary terms are on),                */
/* b2 = -(tau'/eps) f^k, f^k_j = sum over cells of the quadrature of     */
/* f'(phi_h^k) lambda_j.                                                */

static int rhs_both(orc_solver_t *s, const double *php, const double *phn, double *bp, double *bn,
                    int *clamped)
{
    int n = s->nv, nl = s->dim + 1;
    double *fp = calloc((size_t)n, sizeof(double)), *fn = calloc((size_t)n, sizeof(double));
    double xv[12], MT[16], KT[16], vol;
    if (!fp || !fn)
        return ORC_ENOMEM;
    for (int c = 0; c < s->ncell; ++c) {
        const int *v = s->cells + (size_t)c * nl;
        for (int a = 0; a < nl; ++a)
            for (int d = 0; d < s->dim; ++d)
                xv[a * s->dim + d] = s->coords[(size_t)v[a] * s->dim + d];
        orc_element_matrices(s->dim, xv, MT, KT, &vol);
        for (int q = 0; q < s->nq; ++q) {
            const double *lam = s->qb + q * nl;
            double pp = 0.0, pn = 0.0;
            for (int a = 0; a < nl; ++a) {
                pp += lam[a] * php[v[a]];
                pn += lam[a] * phn[v[a]];
            }
            double dfp, dfn;
            potential_eval(&s->prm, pp, pn, NULL, &dfp, &dfn, clamped);
            for (int a = 0; a < nl; ++a) {
                fp[v[a]] += vol * s->qw[q] * dfp * lam[a];
                fn[v[a]] += vol * s->qw[q] * dfn * lam[a];
            }
        }
    }
    csr_mv(&s->M, php, bp);
    csr_mv(&s->M, phn, bn);
    if (s->prm.boundary) {
        /* the boundary flux enters the first block row times tau (the flux
         * value already contains the mobility) */
        double *gp = malloc(sizeof(double) * n), *gn = malloc(sizeof(double) * n);
        if (!gp || !gn) {
            free(gp);
            free(gn);
            free(fp);
            free(fn);
            return ORC_ENOMEM;
        }
        orc_boundary(s, php, phn, gp, gn);
        for (int i = 0; i < n; ++i) {
            bp[i] += s->prm.tau * gp[i];
            bn[i] += s->prm.tau * gn[i];
        }
        free(gp);
        free(gn);
    }
    double cp = tau_s(&s->prm, 0) / s->prm.eps[0], cn = tau_s(&s->prm, 1) / s->prm.eps[1];
    for (int i = 0; i < n; ++i) {
        bp[n + i] = -cp * fp[i];
        bn[n + i] = -cn * fn[i];
    }
    free(fp);
    free(fn);
    return ORC_OK;
}

int orc_rhs(orc_solver_t *s, const double *php, const double *phn, double *bp, double *bn)
{
    if (!s || !php || !phn || !bp || !bn)
        return ORC_EINVAL;
    return rhs_both(s, php, phn, bp, bn, NULL);
}

/* ------------------------------------------------------------------ */

int orc_create(int dim, int64_t nv, const double *coords, int64_t nc, const int32_t *cells,
               const orc_params_t *prm, orc_solver_t **out)
{
    if (!out || !prm || !coords || !cells || (dim != 2 && dim != 3) || nv < 1 || nc < 1
        || nv > 0x3fffffff || nc > 0x3fffffff)
        return ORC_EINVAL;
    if (!(prm->tau > 0.0) || !(prm->eps[0] > 0.0) || !(prm->eps[1] > 0.0)
        || !(prm->mobility[0] > 0.0) || !(prm->mobility[1] > 0.0) || prm->restart < 1
        || !(prm->cheb_ratio > 1.0) || !(prm->cheb_ratio_mass > 1.0) || prm->cheb_degree < 1
        || prm->cheb_degree_mass < 1 || prm->cheb_degree_coarse < 0 || prm->amg_cycles < 1
        || prm->schur_pcg < -1 || (prm->schur_pcg < 0 && prm->krylov != ORC_KRYLOV_FGMRES)
        || (prm->krylov != ORC_KRYLOV_FGMRES && prm->krylov != ORC_KRYLOV_MINRES)
        || (prm->krylov == ORC_KRYLOV_MINRES && prm->schur_pcg != 0)
        || !(prm->amg_tol >= 0.0) || !isfinite(prm->amg_tol)
        || (prm->mass_solver != ORC_MASS_AMG && prm->mass_solver != ORC_MASS_CHEBYSHEV)
        || (prm->range_check != 0 && prm->range_check != 1))
        return ORC_EINVAL;
    for (int64_t i = 0; i < nc * (dim + 1); ++i)
        if (cells[i] < 0 || cells[i] >= nv)
            return ORC_EINVAL;
    orc_solver_t *s = calloc(1, sizeof(*s));
    if (!s)
        return ORC_ENOMEM;
    s->prm = *prm;
    s->dim = dim;
    s->nv = (int)nv;
    s->ncell = (int)nc;
    s->coords = malloc(sizeof(double) * (size_t)nv * dim);
    s->cells = malloc(sizeof(int) * (size_t)nc * (dim + 1));
    memcpy(s->coords, coords, sizeof(double) * (size_t)nv * dim);
    memcpy(s->cells, cells, sizeof(int) * (size_t)nc * (dim + 1));
    int rc = assemble(s);
    if (!rc)
        rc = orc_quadrature(dim, &s->nq, s->qb, s->qw);
    for (int sp = 0; sp < 2 && !rc; ++sp) {
        double t = tau_s(prm, sp), sq = sqrt(t / prm->eps[sp]);
        rc = csr_copy(&s->K, &s->As[sp]);
        if (!rc)
            for (int k = 0; k < s->K.rp[s->nv]; ++k)
                s->As[sp].v[k] = t * s->K.v[k] + sq * s->M.v[k];
    }
    if (!rc)
        rc = hier_build(prm, &s->M, prm->cheb_ratio_mass, prm->cheb_degree_mass, 0, &s->hM);
    for (int sp = 0; sp < 2 && !rc; ++sp)
        rc = hier_build(prm, &s->As[sp], prm->cheb_ratio, prm->cheb_degree,
                        prm->cheb_degree_coarse, &s->hA[sp]);
    if (!rc && prm->schur_pcg < 0) {
        /* automatic inner CG steps from the measured V-cycle contraction */
        double r0 = vcycle_contraction(prm, &s->hA[0], 0), r1 = vcycle_contraction(prm, &s->hA[1], 1);
        if (r0 < 0.0 || r1 < 0.0)
            rc = ORC_ENOMEM;
        s->vc_rho = r0 > r1 ? r0 : r1;
        s->prm.schur_pcg = s->vc_rho <= 0.3 ? 2 : (s->vc_rho <= 0.6 ? 4 : 6);
    }
    if (rc) {
        orc_destroy(s);
        return rc;
    }
    *out = s;
    return ORC_OK;
}

int orc_schur_info(const orc_solver_t *s, int32_t *schur_pcg, double *contraction)
{
    if (!s)
        return ORC_EINVAL;
    if (schur_pcg)
        *schur_pcg = s->prm.schur_pcg;
    if (contraction)
        *contraction = s->vc_rho;
    return ORC_OK;
}

void orc_destroy(orc_solver_t *s)
{
    if (!s)
        return;
    csr_free(&s->M);
    csr_free(&s->K);
    csr_free(&s->As[0]);
    csr_free(&s->As[1]);
    hier_free(&s->hM);
    hier_free(&s->hA[0]);
    hier_free(&s->hA[1]);
    free(s->coords);
    free(s->cells);
    free(s);
}

int64_t orc_nnz(const orc_solver_t *s) { return s ? s->M.rp[s->nv] : -1; }

int orc_get_matrix(const orc_solver_t *s, int which, int32_t *rowptr, int32_t *col, double *val)
{
    if (!s || which < 0 || which > 3)
        return ORC_EINVAL;
    const csr_t *A = which == 0 ? &s->M : which == 1 ? &s->K : &s->As[which - 2];
    if (rowptr)
        memcpy(rowptr, A->rp, sizeof(int) * ((size_t)A->n + 1));
    if (col)
        memcpy(col, A->ci, sizeof(int) * (size_t)A->rp[A->n]);
    if (val)
        memcpy(val, A->v, sizeof(double) * (size_t)A->rp[A->n]);
    return ORC_OK;
}

static const hier_t *get_hier(const orc_solver_t *s, int hier)
{
    if (!s || hier < 0 || hier > 2)
        return NULL;
    return hier == 0 ? &s->hM : &s->hA[hier - 1];
}

int orc_num_levels(const orc_solver_t *s, int hier)
{
    const hier_t *h = get_hier(s, hier);
    return h ? h->nlev : ORC_EINVAL;
}

int orc_level_info(const orc_solver_t *s, int hier, int lev, int64_t *n, int64_t *nnzA,
                   int64_t *nnzP, double *rho)
{
    const hier_t *h = get_hier(s, hier);
    if (!h || lev < 0 || lev >= h->nlev)
        return ORC_EINVAL;
    const level_t *L = &h->lev[lev];
    if (n)
        *n = L->n;
    if (nnzA)
        *nnzA = L->A.rp[L->n];
    if (nnzP)
        *nnzP = L->P.rp ? L->P.rp[L->n] : 0;
    if (rho)
        *rho = L->rho;
    return ORC_OK;
}

int orc_level_get(const orc_solver_t *s, int hier, int lev, int32_t *Arp, int32_t *Aci, double *Av,
                  int32_t *agg, int32_t *Prp, int32_t *Pci, double *Pv)
{
    const hier_t *h = get_hier(s, hier);
    if (!h || lev < 0 || lev >= h->nlev)
        return ORC_EINVAL;
    const level_t *L = &h->lev[lev];
    int nnz = L->A.rp[L->n];
    if (Arp)
        memcpy(Arp, L->A.rp, sizeof(int) * ((size_t)L->n + 1));
    if (Aci)
        memcpy(Aci, L->A.ci, sizeof(int) * (size_t)nnz);
    if (Av)
        memcpy(Av, L->A.v, sizeof(double) * (size_t)nnz);
    if (L->agg) {
        int pn = L->P.rp[L->n];
        if (agg)
            memcpy(agg, L->agg, sizeof(int) * (size_t)L->n);
        if (Prp)
            memcpy(Prp, L->P.rp, sizeof(int) * ((size_t)L->n + 1));
        if (Pci)
            memcpy(Pci, L->P.ci, sizeof(int) * (size_t)pn);
        if (Pv)
            memcpy(Pv, L->P.v, sizeof(double) * (size_t)pn);
    }
    return ORC_OK;
}

int orc_amg_solve(const orc_solver_t *s, int hier, const double *b, double *x)
{
    const hier_t *h = get_hier(s, hier);
    if (!h || !b || !x)
        return ORC_EINVAL;
    amg_stationary(&s->prm, h, b, x);
    return ORC_OK;
}

int orc_vcycle(const orc_solver_t *s, int hier, const double *b, double *x)
{
    const hier_t *h = get_hier(s, hier);
    if (!h || !b || !x)
        return ORC_EINVAL;
    vcycle(&s->prm, h, 0, b, x);
    return ORC_OK;
}

int orc_smooth(const orc_solver_t *s, int hier, int lev, const double *b, double *x)
{
    const hier_t *h = get_hier(s, hier);
    if (!h || lev < 0 || lev >= h->nlev || !b || !x)
        return ORC_EINVAL;
    const level_t *L = &h->lev[lev];
    double *r = malloc(sizeof(double) * (size_t)(L->n + 1));
    double *d = malloc(sizeof(double) * (size_t)(L->n + 1));
    if (!r || !d) {
        free(r);
        free(d);
        return ORC_ENOMEM;
    }
    smooth(&s->prm, h, L, b, x, r, d);
    free(r);
    free(d);
    return ORC_OK;
}

int orc_schur_solve(const orc_solver_t *s, int species, const double *b, double *x)
{
    if (!s || species < 0 || species > 1 || !b || !x)
        return ORC_EINVAL;
    amg_schur(&s->prm, &s->hA[species], b, x);
    return ORC_OK;
}

int orc_apply_saddle(const orc_solver_t *s, int species, const double *x, double *y)
{
    if (!s || species < 0 || species > 1 || !x || !y)
        return ORC_EINVAL;
    saddle(s, species, x, y);
    return ORC_OK;
}

int orc_apply_prec(const orc_solver_t *s, int species, const double *v, double *w)
{
    if (!s || species < 0 || species > 1 || !v || !w)
        return ORC_EINVAL;
    prec(s, species, v, w);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Preconditioned MINRES (Paige and Saunders 1975) for the symmetric     */
/* saddle-point matrix with the symmetric positive definite Algorithm 1  */
/* of stationary V-cycles: the Lanczos process on P^-1 A in the P inner  */
/* product (three-term recurrence with the vectors r1, r2 and their      */
/* preconditioned images), the QR factorisation of its tridiagonal       */
/* matrix by Givens rotations, and the iterate updated along the         */
/* directions w.  phibar, the residual in the P^-1 norm, comes from the  */
/* rotations; the method stops when it is at most rtol times the P^-1    */
/* norm of b.  relres reports the true 2-norm residual relative to b.    */

static int minres(const orc_solver_t *s, int sp, const double *b, double *x, int32_t *iters,
                  double *relres)
{
    const orc_params_t *p = &s->prm;
    const int n2 = 2 * s->nv;
    double *r1 = malloc(sizeof(double) * n2), *r2 = malloc(sizeof(double) * n2);
    double *y = malloc(sizeof(double) * n2), *v = malloc(sizeof(double) * n2);
    double *w1 = calloc((size_t)n2, sizeof(double)), *w2 = calloc((size_t)n2, sizeof(double));
    double *pb = malloc(sizeof(double) * n2);
    int rc = ORC_OK, k = 0;
    if (!r1 || !r2 || !y || !v || !w1 || !w2 || !pb) {
        rc = ORC_ENOMEM;
        goto out;
    }
    prec(s, sp, b, pb);
    const double bnp2 = dot(n2, b, pb);
    if (!(bnp2 >= 0.0)) {
        rc = ORC_ENAN;   /* an indefinite (or non-finite) preconditioner */
        goto out;
    }
    const double tol = p->rtol * sqrt(bnp2);
    saddle(s, sp, x, r1);
    for (int i = 0; i < n2; ++i)
        r1[i] = b[i] - r1[i];
    prec(s, sp, r1, y);
    double beta = dot(n2, r1, y);
    if (!(beta >= 0.0)) {
        rc = ORC_ENAN;
        goto out;
    }
    beta = sqrt(beta);
    memcpy(r2, r1, sizeof(double) * n2);
    double oldb = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta, cs = -1.0, sn = 0.0;
    while (phibar > tol) {
        if (k >= p->max_iters) {
            rc = ORC_ENOCONV;
            break;
        }
        ++k;
        for (int i = 0; i < n2; ++i)
            v[i] = y[i] / beta;
        saddle(s, sp, v, y);
        if (k >= 2)
            for (int i = 0; i < n2; ++i)
                y[i] -= (beta / oldb) * r1[i];
        const double alfa = dot(n2, v, y);
        for (int i = 0; i < n2; ++i)
            y[i] -= (alfa / beta) * r2[i];
        memcpy(r1, r2, sizeof(double) * n2);
        memcpy(r2, y, sizeof(double) * n2);
        prec(s, sp, r2, y);
        oldb = beta;
        beta = dot(n2, r2, y);
        if (!(beta >= 0.0)) {
            rc = ORC_ENAN;
            break;
        }
        beta = sqrt(beta);
        const double oldeps = epsln;
        const double delta = cs * dbar + sn * alfa;
        const double gbar = sn * dbar - cs * alfa;
        epsln = sn * beta;
        dbar = -cs * beta;
        double gamma = sqrt(gbar * gbar + beta * beta);
        if (gamma == 0.0)
            gamma = 1e-300;
        cs = gbar / gamma;
        sn = beta / gamma;
        const double phi = cs * phibar;
        phibar = sn * phibar;
        for (int i = 0; i < n2; ++i) {
            const double wn = (v[i] - oldeps * w1[i] - delta * w2[i]) / gamma;
            w1[i] = w2[i];
            w2[i] = wn;
            x[i] += phi * wn;
        }
        if (!isfinite(phibar)) {
            rc = ORC_ENAN;
            break;
        }
    }
    saddle(s, sp, x, r1);
    for (int i = 0; i < n2; ++i)
        r1[i] = b[i] - r1[i];
    {
        const double bn = sqrt(dot(n2, b, b)), rn = sqrt(dot(n2, r1, r1));
        *relres = bn > 0.0 ? rn / bn : rn;
    }
out:
    *iters = k;
    free(r1);
    free(r2);
    free(y);
    free(v);
    free(w1);
    free(w2);
    free(pb);
    return rc;
}

int orc_minres(const orc_solver_t *s, int species, const double *b, double *x, int32_t *iters,
               double *relres)
{
    if (!s || species < 0 || species > 1 || !b || !x || !iters || !relres)
        return ORC_EINVAL;
    return minres(s, species, b, x, iters, relres);
}

/* the Krylov method of the parameters */
static int krylov(const orc_solver_t *s, int sp, const double *b, double *x, int32_t *iters,
                  double *relres)
{
    if (s->prm.krylov == ORC_KRYLOV_MINRES)
        return minres(s, sp, b, x, iters, relres);
    return fgmres(s, sp, b, x, iters, relres);
}

int orc_fgmres(const orc_solver_t *s, int species, const double *b, double *x, int32_t *iters,
               double *relres)
{
    if (!s || species < 0 || species > 1 || !b || !x || !iters || !relres)
        return ORC_EINVAL;
    return fgmres(s, species, b, x, iters, relres);
}

/* One time step of eq. FE_systems for both species, then phi_s =       */
/* 1 - phi_p - phi_n (Section 2) and, while evaporation is on, removal  */
/* of evap_ds solvent per node, given to phi_p and phi_n in proportion  */
/* to their fractions (equal halves where both vanish).  On failure the */
/* state is left unchanged.                                             */
int orc_step(orc_solver_t *s, double *php, double *phn, double *mup, double *mun, orc_stats_t *st)
{
    if (!s || !php || !phn || !mup || !mun)
        return ORC_EINVAL;
    int n = s->nv, clamped = 0, rc;
    double *bp = malloc(sizeof(double) * 2 * (size_t)n), *bn = malloc(sizeof(double) * 2 * (size_t)n);
    double *xp = malloc(sizeof(double) * 2 * (size_t)n), *xn = malloc(sizeof(double) * 2 * (size_t)n);
    orc_stats_t loc = {{0, 0}, {0.0, 0.0}, 0, 0, 0};
    double *np_ = NULL, *nn_ = NULL;
    if ((rc = rhs_both(s, php, phn, bp, bn, &clamped)))
        goto done;
    memcpy(xp, php, sizeof(double) * n);
    memcpy(xp + n, mup, sizeof(double) * n);
    memcpy(xn, phn, sizeof(double) * n);
    memcpy(xn + n, mun, sizeof(double) * n);
    loc.clamped = clamped;
    rc = krylov(s, 0, bp, xp, &loc.iters[0], &loc.relres[0]);
    if (!rc)
        rc = krylov(s, 1, bn, xn, &loc.iters[1], &loc.relres[1]);
    else {
        int32_t it;
        double rr;
        krylov(s, 1, bn, xn, &it, &rr);
        loc.iters[1] = it;
        loc.relres[1] = rr;
    }
    if (rc)
        goto done;
    for (int i = 0; i < 2 * n; ++i)
        if (!isfinite(xp[i]) || !isfinite(xn[i])) {
            rc = ORC_ENAN;
            goto done;
        }
    /* the new volume fractions: the solve's, then the solvent removal */
    np_ = malloc(sizeof(double) * (size_t)n);
    nn_ = malloc(sizeof(double) * (size_t)n);
    if (!np_ || !nn_) {
        rc = ORC_ENOMEM;
        goto done;
    }
    memcpy(np_, xp, sizeof(double) * n);
    memcpy(nn_, xn, sizeof(double) * n);
    if (s->prm.evap_ds > 0.0 && s->step_count < s->prm.evap_steps) {
        double ds = s->prm.evap_ds;
        for (int i = 0; i < n; ++i) {
            double sum = np_[i] + nn_[i];
            if (sum > 0.0) {
                double gp = ds * np_[i] / sum, gn = ds * nn_[i] / sum;
                np_[i] += gp;
                nn_[i] += gn;
            } else {
                np_[i] += 0.5 * ds;
                nn_[i] += 0.5 * ds;
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        double a = np_[i], b = nn_[i], c = 1.0 - np_[i] - nn_[i];
        if (a < 0.0 || a > 1.0 || b < 0.0 || b > 1.0 || c < 0.0 || c > 1.0)
            loc.outside++;
    }
    if (s->prm.range_check && loc.outside > 0) {
        rc = ORC_EDOMAIN;
        goto done;
    }
    memcpy(php, np_, sizeof(double) * n);
    memcpy(mup, xp + n, sizeof(double) * n);
    memcpy(phn, nn_, sizeof(double) * n);
    memcpy(mun, xn + n, sizeof(double) * n);
    s->step_count++;
done:
    loc.status = rc;
    if (st)
        *st = loc;
    free(bp);
    free(bn);
    free(xp);
    free(xn);
    free(np_);
    free(nn_);
    return rc;
}

/* discrete Ginzburg-Landau energy (eq. ginzburglandau without the      */
/* substrate term): integral of f(phi_h) + (eps/2) phi^T K phi per      */
/* species                                                               */
double orc_energy(const orc_solver_t *s, const double *php, const double *phn)
{
    int n = s->nv, nl = s->dim + 1;
    double e = 0.0, xv[12], MT[16], KT[16], vol;
    for (int c = 0; c < s->ncell; ++c) {
        const int *v = s->cells + (size_t)c * nl;
        for (int a = 0; a < nl; ++a)
            for (int d = 0; d < s->dim; ++d)
                xv[a * s->dim + d] = s->coords[(size_t)v[a] * s->dim + d];
        orc_element_matrices(s->dim, xv, MT, KT, &vol);
        for (int q = 0; q < s->nq; ++q) {
            const double *lam = s->qb + q * nl;
            double pp = 0.0, pn = 0.0, f;
            for (int a = 0; a < nl; ++a) {
                pp += lam[a] * php[v[a]];
                pn += lam[a] * phn[v[a]];
            }
            potential_eval(&s->prm, pp, pn, &f, NULL, NULL, NULL);
            e += vol * s->qw[q] * f;
        }
    }
    double *t = malloc(sizeof(double) * (size_t)n);
    csr_mv(&s->K, php, t);
    e += 0.5 * s->prm.eps[0] * dot(n, php, t);
    csr_mv(&s->K, phn, t);
    e += 0.5 * s->prm.eps[1] * dot(n, phn, t);
    free(t);
    return e;
}
