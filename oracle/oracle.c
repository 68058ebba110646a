/*
 * oracle.c -- plain, slow, obviously-correct FP64 reference for the
 * rational-program hot path.  TEST INFRASTRUCTURE ONLY: this file is built
 * and called by the tests, by the smoke check and by the benchmark's CPU
 * baseline leg; the product library never links, loads or calls it, and it
 * shares no code, header or table with the product.
 *
 * What it computes, with the passage each function follows:
 *   or_monomials      monomial exponent sets of a rational model (Section 4.2,
 *                     the display defining f_b = p_b / q_b), total-degree form,
 *                     graded order; plain definition + sort.
 *   or_monomials_box  the same order over a per-variable degree box (the
 *                     display's bounds on each variable's degree).
 *   or_candidates_2d  the finite set F of 2-D thread-block formats
 *                     (Section 3.3 assumptions; Section 4: threads per block
 *                     bounded, product a multiple of the wave size).
 *   or_fit            linearised least squares for N/Q with q0 = 1
 *                     (Section 4.2: linear in the fitting parameters, Ax = b,
 *                     min ||b - Ax||); Householder QR with the numerical rank
 *                     decided column by column in the natural order, and the
 *                     minimum-norm solution through a complete orthogonal
 *                     decomposition when A is rank deficient (the result the
 *                     paper's SVD solver returns, Section 4.2); with fewer
 *                     samples than unknowns, the minimum-norm interpolant by
 *                     Householder QR of A^T.
 *   or_eval_rational  direct evaluation of N/Q (Section 2, Definition 1:
 *                     only +, -, x and one division per rational).
 *   or_mwpcwp         the MWP-CWP-style template (Section 2, Examples 1-2;
 *                     equation (occupancy) with the wave size as a parameter).
 *                     PARITY UNPINNED against the paper: the paper does not
 *                     print the model's equations; the template is this
 *                     project's restatement of the cited MWP-CWP model and is
 *                     pinned only by hand-worked examples and special cases.
 *   or_occupancy      hardware occupancy W_active / W_max of a block format
 *                     (Section 2, Example 1, equation (occupancy)); the
 *                     resident-block count that the paper gives as a flow
 *                     chart is taken as the smallest of the per-unit limits
 *                     on blocks, waves, registers and LDS bytes.
 *   or_argmin         exhaustive evaluation and selection (Section 3.3,
 *                     steps 4-5), lowest index wins exact ties.
 *   or_select         the same with a sense (minimise a time, maximise an
 *                     occupancy) and an optional second program that breaks
 *                     exact ties of the first (Section 3.3 step 5: a second
 *                     performance metric refines the choice), then the
 *                     lowest index.
 *   or_loss_grad      true rational loss sum (N/Q - y)^2 and its closed-form
 *                     gradient (refinement of the linearised fit).
 *   or_refine         Levenberg-Marquardt / Gauss-Newton on that loss, each
 *                     step solved by the same QR least-squares routine.
 *   or_regret         the "Error" percentage of Section 5.
 *   or_split_fit      one decision node of a rational program fitted from the
 *                     samples (Section 3.2, third consequence: decision nodes
 *                     are rational and could be fitted too): a threshold on
 *                     one variable found by exhaustive search over the
 *                     breakpoints between sorted samples, each side fitted
 *                     by or_fit, the sum of the sides' squared residuals
 *                     minimised.
 *
 * Conventions shared with the product only as documented interfaces:
 * coefficient layout [alpha_0..alpha_{a-1} | beta_1..beta_b] in graded
 * monomial order; status codes 0 OK, 1 rank deficient, 2 underdetermined,
 * 3 non-finite input, 4 Q non-positive at a sample, 5 not converged.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXV 8

enum { OR_OK = 0, OR_RANK_DEFICIENT = 1, OR_UNDERDETERMINED = 2,
       OR_NONFINITE = 3, OR_Q_NONPOSITIVE = 4, OR_NOT_CONVERGED = 5 };

/* ------------------------------------------------------------------ */
/* Monomial exponent sets                                              */
/* ------------------------------------------------------------------ */

static int g_sort_nvars;

/* Graded order: total degree ascending; within a degree, the exponent of
 * x1 descending, then x2 descending, and so on. */
static int cmp_exps(const void* pa, const void* pb) {
    const unsigned char* a = (const unsigned char*)pa;
    const unsigned char* b = (const unsigned char*)pb;
    int da = 0, db = 0;
    for (int k = 0; k < g_sort_nvars; k++) { da += a[k]; db += b[k]; }
    if (da != db) return da < db ? -1 : 1;
    for (int k = 0; k < g_sort_nvars; k++)
        if (a[k] != b[k]) return a[k] > b[k] ? -1 : 1;
    return 0;
}

static pthread_mutex_t g_sort_lock = PTHREAD_MUTEX_INITIALIZER;

/* All e in N^v with sum(e) <= degree, graded order.  Returns 0, or -1 on bad
 * arguments.  exps may be NULL to query the count. */
int or_monomials(int nvars, int degree, unsigned char* exps, int* count) {
    if (nvars < 1 || nvars > OR_MAXV || degree < 0 || degree > 15 || !count) return -1;
    /* odometer over the box [0, degree]^v, keeping total degree <= degree */
    int e[OR_MAXV] = {0};
    int n = 0;
    unsigned char* buf = NULL;
    long box = 1;
    for (int k = 0; k < nvars; k++) box *= (degree + 1);
    buf = (unsigned char*)malloc((size_t)box * nvars);
    if (!buf) return -1;
    for (long t = 0; t < box; t++) {
        long r = t; int s = 0;
        for (int k = 0; k < nvars; k++) { e[k] = (int)(r % (degree + 1)); r /= (degree + 1); s += e[k]; }
        if (s <= degree) {
            for (int k = 0; k < nvars; k++) buf[n * nvars + k] = (unsigned char)e[k];
            n++;
        }
    }
    pthread_mutex_lock(&g_sort_lock);
    g_sort_nvars = nvars;
    qsort(buf, (size_t)n, (size_t)nvars, cmp_exps);
    pthread_mutex_unlock(&g_sort_lock);
    if (exps) memcpy(exps, buf, (size_t)n * nvars);
    *count = n;
    free(buf);
    return 0;
}

/* The per-variable degree box of the Section 4.2 model display: every e
 * with 0 <= e_k <= maxdeg[k], in the same graded order.  Returns 0, or -1 on
 * bad arguments (1 <= nvars <= 8, 0 <= maxdeg[k] <= 15).  exps may be NULL
 * to query the count. */
int or_monomials_box(int nvars, const int* maxdeg, unsigned char* exps, int* count) {
    if (nvars < 1 || nvars > OR_MAXV || !maxdeg || !count) return -1;
    long box = 1;
    for (int k = 0; k < nvars; k++) {
        if (maxdeg[k] < 0 || maxdeg[k] > 15) return -1;
        box *= (maxdeg[k] + 1);
    }
    unsigned char* buf = (unsigned char*)malloc((size_t)box * nvars);
    if (!buf) return -1;
    /* odometer over the box */
    for (long t = 0; t < box; t++) {
        long r = t;
        for (int k = 0; k < nvars; k++) {
            buf[t * nvars + k] = (unsigned char)(r % (maxdeg[k] + 1));
            r /= (maxdeg[k] + 1);
        }
    }
    pthread_mutex_lock(&g_sort_lock);
    g_sort_nvars = nvars;
    qsort(buf, (size_t)box, (size_t)nvars, cmp_exps);
    pthread_mutex_unlock(&g_sort_lock);
    if (exps) memcpy(exps, buf, (size_t)box * nvars);
    *count = (int)box;
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Candidate set F of 2-D block formats                                */
/* ------------------------------------------------------------------ */

/* All integer (bx, by) >= 1 with bx*by <= max_prod and multiple | bx*by,
 * ordered by bx then by. */
int or_candidates_2d(int max_prod, int multiple, int* bxby, int* count) {
    if (max_prod < 1 || multiple < 1 || !count) return -1;
    int n = 0;
    for (int bx = 1; bx <= max_prod; bx++)
        for (int by = 1; by <= max_prod; by++) {
            long p = (long)bx * by;
            if (p <= max_prod && p % multiple == 0) {
                if (bxby) { bxby[2 * n] = bx; bxby[2 * n + 1] = by; }
                n++;
            }
        }
    *count = n;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Monomials and rational evaluation                                   */
/* ------------------------------------------------------------------ */

static double monomial(const unsigned char* e, const double* u, int nvars) {
    double m = 1.0;
    for (int k = 0; k < nvars; k++)
        for (int t = 0; t < e[k]; t++) m *= u[k];
    return m;
}

typedef struct {
    int nvars, a, b;          /* a numerator terms, b denominator terms (no constant) */
    unsigned char* ne;        /* [a * nvars] */
    unsigned char* de;        /* [(b+1) * nvars], entry 0 is the constant */
} model_t;

static int model_init(model_t* M, int nvars, int dn, int dq) {
    int a, b1;
    if (or_monomials(nvars, dn, NULL, &a) || or_monomials(nvars, dq, NULL, &b1)) return -1;
    M->nvars = nvars; M->a = a; M->b = b1 - 1;
    M->ne = (unsigned char*)malloc((size_t)a * nvars);
    M->de = (unsigned char*)malloc((size_t)b1 * nvars);
    or_monomials(nvars, dn, M->ne, &a);
    or_monomials(nvars, dq, M->de, &b1);
    return 0;
}

static void model_free(model_t* M) { free(M->ne); free(M->de); }

static void model_nq(const model_t* M, const double* coef, const double* u,
                     double* N, double* Q) {
    double n = 0.0, q = 1.0;
    for (int j = 0; j < M->a; j++) n += coef[j] * monomial(M->ne + j * M->nvars, u, M->nvars);
    for (int j = 1; j <= M->b; j++) q += coef[M->a + j - 1] * monomial(M->de + j * M->nvars, u, M->nvars);
    *N = n; *Q = q;
}

/* f(u) = N(u)/Q(u) at m points u[k*ldu + i]. */
int or_eval_rational(int nvars, int dn, int dq, const double* coef,
                     const double* u, long ldu, long m, double* out) {
    model_t M;
    if (model_init(&M, nvars, dn, dq)) return -1;
    double ui[OR_MAXV];
    for (long i = 0; i < m; i++) {
        for (int k = 0; k < nvars; k++) ui[k] = u[k * ldu + i];
        double N, Q;
        model_nq(&M, coef, ui, &N, &Q);
        out[i] = N / Q;
    }
    model_free(&M);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Least squares: Householder QR with column pivoting + COD             */
/* ------------------------------------------------------------------ */

/* Back-substitution of a triangularised least-squares problem.  On entry the
 * first r columns of A (column-major, leading dimension m; column j holds
 * original unknown perm[j]) are upper triangular with a nonsingular leading
 * r x r block, the remaining n - r columns hold Q^T times the columns set
 * aside, and b holds Q^T b.  With r == n this is the unique solution; with
 * r < n the set-aside columns are replaced by their projections onto the
 * first r (their rows r.. are ignored) and x gets the minimum-norm minimiser
 * of that problem through a complete orthogonal decomposition. */
static void finish_lls(int m, int n, double* A, const double* b, const int* perm, int r,
                       double* x) {
    double* z = (double*)calloc((size_t)n, sizeof(double));
#define R(i, j) A[(i) + (long)(j) * m]
    if (r == n) {
        for (int i = n - 1; i >= 0; i--) {
            double s = b[i];
            for (int j = i + 1; j < n; j++) s -= R(i, j) * z[j];
            z[i] = s / R(i, i);
        }
    } else if (r > 0) {
        /* complete orthogonal decomposition: [R11 R12] H_0 ... H_{r-1} = [T 0],
         * built from the last row upwards; each H_i acts on coordinates
         * {i} U {r..n-1}. */
        int nt = n - r;
        double* W = (double*)malloc(sizeof(double) * (size_t)r * (nt + 1));
        double* wtw = (double*)malloc(sizeof(double) * (size_t)r);
        for (int i = r - 1; i >= 0; i--) {
            double* w = W + (long)i * (nt + 1);
            double s2 = R(i, i) * R(i, i);
            for (int t = 0; t < nt; t++) s2 += R(i, r + t) * R(i, r + t);
            double nrm = sqrt(s2);
            double alpha = R(i, i) >= 0.0 ? -nrm : nrm;
            w[0] = R(i, i) - alpha;
            for (int t = 0; t < nt; t++) w[1 + t] = R(i, r + t);
            double ww = 0.0;
            for (int t = 0; t <= nt; t++) ww += w[t] * w[t];
            wtw[i] = ww;
            if (ww == 0.0) continue;
            for (int ip = 0; ip <= i; ip++) {
                double s = R(ip, i) * w[0];
                for (int t = 0; t < nt; t++) s += R(ip, r + t) * w[1 + t];
                double f = 2.0 * s / ww;
                R(ip, i) -= f * w[0];
                for (int t = 0; t < nt; t++) R(ip, r + t) -= f * w[1 + t];
            }
        }
        for (int i = r - 1; i >= 0; i--) {
            double s = b[i];
            for (int j = i + 1; j < r; j++) s -= R(i, j) * z[j];
            z[i] = s / R(i, i);
        }
        for (int i = 0; i < r; i++) {          /* z <- H_{r-1} ... H_0 [w; 0] */
            if (wtw[i] == 0.0) continue;
            const double* w = W + (long)i * (nt + 1);
            double s = z[i] * w[0];
            for (int t = 0; t < nt; t++) s += z[r + t] * w[1 + t];
            double f = 2.0 * s / wtw[i];
            z[i] -= f * w[0];
            for (int t = 0; t < nt; t++) z[r + t] -= f * w[1 + t];
        }
        free(W); free(wtw);
    }
#undef R
    for (int j = 0; j < n; j++) x[perm[j]] = z[j];
    free(z);
}

/* Householder reflection of rows k..m-1 of column k of A (column-major,
 * leading dimension m) with the column's remaining norm nrm > 0; applied to
 * the columns k+1..n-1 and to b.  Column k becomes (.., alpha, 0, .., 0). */
static void reflect(int m, int n, double* A, double* b, int k, double nrm) {
    double* col = A + (long)k * m;
    double alpha = col[k] >= 0.0 ? -nrm : nrm;
    col[k] -= alpha;                       /* v = x - alpha e1, stored in place */
    double vtv = 0.0;
    for (int i = k; i < m; i++) vtv += col[i] * col[i];
    for (int j = k + 1; j < n; j++) {
        double* cj = A + (long)j * m;
        double s = 0.0;
        for (int i = k; i < m; i++) s += col[i] * cj[i];
        double f = 2.0 * s / vtv;
        for (int i = k; i < m; i++) cj[i] -= f * col[i];
    }
    if (b) {
        double s = 0.0;
        for (int i = k; i < m; i++) s += col[i] * b[i];
        double f = 2.0 * s / vtv;
        for (int i = k; i < m; i++) b[i] -= f * col[i];
    }
    col[k] = alpha;
    for (int i = k + 1; i < m; i++) col[i] = 0.0;
}

/* Solve min ||b - A x|| for A (m x n, column-major, leading dimension m).
 * A and b are overwritten.  Householder QR with column pivoting (largest
 * remaining norm first); columns whose remaining norm is at most
 * max(m, n) 2^-53 |R_00| are set aside.  Returns the numerical rank; x gets
 * the minimum-norm minimiser when the rank is below n.  (A general-purpose
 * least-squares routine: the tests' own pins and the Levenberg-Marquardt
 * steps use it; the linearised fit decides its rank by lls_natural.) */
static int lls_qrcp(int m, int n, double* A, double* b, double* x) {
    int* perm = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; j++) perm[j] = j;
    int kmax = m < n ? m : n;
    double tol = (double)(m > n ? m : n) * ldexp(1.0, -53);
    double r00 = 0.0;
    int rank = kmax;
    for (int k = 0; k < kmax; k++) {
        /* pivot: the remaining column of largest norm (first on ties) */
        int p = k; double best = -1.0;
        for (int j = k; j < n; j++) {
            double s = 0.0;
            for (int i = k; i < m; i++) s += A[i + (long)j * m] * A[i + (long)j * m];
            if (s > best) { best = s; p = j; }
        }
        if (p != k) {
            for (int i = 0; i < m; i++) {
                double t = A[i + (long)k * m]; A[i + (long)k * m] = A[i + (long)p * m]; A[i + (long)p * m] = t;
            }
            int t = perm[k]; perm[k] = perm[p]; perm[p] = t;
        }
        double nrm = sqrt(best);
        if (k == 0) r00 = nrm;
        if (nrm == 0.0 || nrm <= tol * r00) { rank = k; break; }
        reflect(m, n, A, b, k, nrm);
    }
    finish_lls(m, n, A, b, perm, rank, x);
    free(perm);
    return rank;
}

/* Solve min ||b - A x|| with the numerical rank decided column by column in
 * the natural order: column j is dependent when its distance from the span of
 * the columns kept before it is at most tau times its own norm.  Kept columns
 * are triangularised by Householder reflections in their order; a dependent
 * column is moved behind every other column (its coefficient then comes from
 * the minimum-norm completion of finish_lls).  A and b are overwritten;
 * returns the number of kept columns.  Column norms of zero count as
 * dependent. */
static int lls_natural(int m, int n, double* A, double* b, double* x, double tau) {
    int* perm = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double* cn = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* tmp = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int j = 0; j < n; j++) {
        perm[j] = j;
        double s = 0.0;
        for (int i = 0; i < m; i++) s += A[i + (long)j * m] * A[i + (long)j * m];
        cn[j] = sqrt(s);
    }
    int r = 0, undecided = n;
    while (undecided > 0) {
        /* the next column in natural order sits at position r */
        double s = 0.0;
        for (int i = r; i < m; i++) s += A[i + (long)r * m] * A[i + (long)r * m];
        double dist = sqrt(s);
        if (dist <= tau * cn[perm[r]]) {
            /* dependent: rotate columns r..n-1 left by one, this one last */
            int pj = perm[r];
            memcpy(tmp, A + (long)r * m, sizeof(double) * (size_t)m);
            memmove(A + (long)r * m, A + (long)(r + 1) * m, sizeof(double) * (size_t)m * (n - r - 1));
            memcpy(A + (long)(n - 1) * m, tmp, sizeof(double) * (size_t)m);
            memmove(perm + r, perm + r + 1, sizeof(int) * (size_t)(n - r - 1));
            perm[n - 1] = pj;
        } else {
            reflect(m, n, A, b, r, dist);
            r++;
        }
        undecided--;
    }
    finish_lls(m, n, A, b, perm, r, x);
    free(perm); free(cn); free(tmp);
    return r;
}

/* Minimum-norm solution of an underdetermined system A x = b (m < n, A m x n
 * column-major) when its rows are independent by the sample rule: in sample
 * order, row i is dependent when its distance from the span of the rows
 * before it is at most tau times its own norm.  Householder QR of A^T
 * (A^T = H_0 .. H_{m-1} [R; 0], R m x m upper triangular), then
 * x = H_0 .. H_{m-1} [R^-T b; 0].  Returns 1 with x set, or 0 (x untouched)
 * when some row is dependent. */
static int min_norm_rows(int m, int n, const double* A, const double* b, double* x, double tau) {
    double* V = (double*)malloc(sizeof(double) * (size_t)n * (m > 0 ? m : 1));  /* A^T, n x m */
    double* vtv = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* Rm = (double*)calloc((size_t)m * (m > 0 ? m : 1), sizeof(double));  /* R[i + j m] */
    double* w = (double*)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) V[j + (long)i * n] = A[i + (long)j * m];
    int ok = 1;
    for (int k = 0; k < m; k++) {
        double* col = V + (long)k * n;
        double s0 = 0.0, s = 0.0;
        /* the row's own norm (taken from A: the reflections applied to this
         * column so far are orthogonal) and its distance from the rows before */
        for (int j = 0; j < n; j++) s0 += A[k + (long)j * m] * A[k + (long)j * m];
        for (int j = k; j < n; j++) s += col[j] * col[j];
        double nrm = sqrt(s);
        if (!(nrm > tau * sqrt(s0))) { ok = 0; break; }
        for (int i = 0; i < k; i++) Rm[i + (long)k * m] = col[i];
        double alpha = col[k] >= 0.0 ? -nrm : nrm;
        col[k] -= alpha;
        double vv = 0.0;
        for (int j = k; j < n; j++) vv += col[j] * col[j];
        vtv[k] = vv;
        Rm[k + (long)k * m] = alpha;
        for (int c = k + 1; c < m; c++) {
            double* cc = V + (long)c * n;
            double t = 0.0;
            for (int j = k; j < n; j++) t += col[j] * cc[j];
            double f = 2.0 * t / vv;
            for (int j = k; j < n; j++) cc[j] -= f * col[j];
        }
    }
    if (ok) {
        for (int i = 0; i < m; i++) {          /* R^T w = b */
            double s = b[i];
            for (int k = 0; k < i; k++) s -= Rm[k + (long)i * m] * w[k];
            w[i] = s / Rm[i + (long)i * m];
        }
        for (int k = m - 1; k >= 0; k--) {     /* w <- H_k w, k descending */
            const double* col = V + (long)k * n;
            double t = 0.0;
            for (int j = k; j < n; j++) t += col[j] * w[j];
            double f = 2.0 * t / vtv[k];
            for (int j = k; j < n; j++) w[j] -= f * col[j];
        }
        for (int j = 0; j < n; j++) x[j] = w[j];
    }
    free(V); free(vtv); free(Rm); free(w);
    return ok;
}

/* Public wrapper of the least-squares routine (for the tests' own pins). */
int or_lstsq(int m, int n, const double* A_colmajor, const double* b, double* x) {
    double* A = (double*)malloc(sizeof(double) * (size_t)m * n);
    double* bb = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    memcpy(A, A_colmajor, sizeof(double) * (size_t)m * n);
    memcpy(bb, b, sizeof(double) * (size_t)m);
    int r = lls_qrcp(m, n, A, bb, x);
    free(A); free(bb);
    return r;
}

/* Linearised design: row i = [m_j(u_i)]_{j<a} ++ [-y_i m'_j(u_i)]_{1<=j<=b}, rhs y_i. */
static void build_design(const model_t* M, long m, const double* x, long ldx,
                         const double* y, double* A /* col-major m x n */) {
    int n = M->a + M->b;
    double ui[OR_MAXV];
    for (long i = 0; i < m; i++) {
        for (int k = 0; k < M->nvars; k++) ui[k] = x[k * ldx + i];
        for (int j = 0; j < M->a; j++)
            A[i + (long)j * m] = monomial(M->ne + j * M->nvars, ui, M->nvars);
        for (int j = 1; j <= M->b; j++)
            A[i + (long)(M->a + j - 1) * m] = -y[i] * monomial(M->de + j * M->nvars, ui, M->nvars);
    }
    (void)n;
}

/* Materialised design matrix, row-major [m][n], and rhs (for the tests). */
int or_design(long m, int nvars, int dn, int dq, const double* x, long ldx,
              const double* y, double* A_rowmajor, double* rhs) {
    model_t M;
    if (model_init(&M, nvars, dn, dq)) return -1;
    int n = M.a + M.b;
    double* A = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * n);
    build_design(&M, m, x, ldx, y, A);
    for (long i = 0; i < m; i++) {
        for (int j = 0; j < n; j++) A_rowmajor[i * n + j] = A[i + (long)j * m];
        rhs[i] = y[i];
    }
    free(A); model_free(&M);
    return 0;
}

/* Numerical-rank thresholds of the linearised fit (the paper's SVD solver
 * needs one; it names none): a column whose distance from the span of the
 * columns kept before it is at most OR_TAU_COL of its norm is dependent; with
 * fewer samples than unknowns, a sample whose design row lies within
 * OR_TAU_ROW of its norm from the span of the rows before it is dependent. */
#define OR_TAU_COL 1e-5
#define OR_TAU_ROW 3.1622776601683794e-07   /* sqrt(1e-13) */

/* The linearised fit's least-squares solve with its rank rule: with fewer
 * samples than unknowns and independent samples, the unique minimum-norm
 * interpolant; otherwise the natural-order column rule (the minimum-norm
 * minimiser of the problem whose dependent columns are replaced by their
 * projections).  A (column-major) and b are overwritten; returns the rank. */
static int fit_lls(int m, int n, double* A, double* b, double* x) {
    if (m < n && min_norm_rows(m, n, A, b, x, OR_TAU_ROW)) return m;
    return lls_natural(m, n, A, b, x, OR_TAU_COL);
}

/* Public wrapper of fit_lls (for the tests' pins of the rank rule). */
int or_lstsq_fit(int m, int n, const double* A_colmajor, const double* b, double* x) {
    double* A = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (n > 0 ? n : 1));
    double* bb = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    memcpy(A, A_colmajor, sizeof(double) * (size_t)m * n);
    memcpy(bb, b, sizeof(double) * (size_t)m);
    int r = fit_lls(m, n, A, bb, x);
    free(A); free(bb);
    return r;
}

/* One linearised fit.  x[k*ldx + i], y[i] for i < m.  coef has a + b entries.
 * status per the codes above; rank = numerical rank; resid = ||y - A c||. */
int or_fit(long m, int nvars, int dn, int dq, const double* x, long ldx,
           const double* y, double* coef, int* status, int* rank, double* resid) {
    model_t M;
    if (model_init(&M, nvars, dn, dq)) return -1;
    int n = M.a + M.b;
    for (long i = 0; i < m; i++) {
        int bad = !isfinite(y[i]);
        for (int k = 0; k < nvars; k++) bad |= !isfinite(x[k * ldx + i]);
        if (bad) {
            for (int j = 0; j < n; j++) coef[j] = NAN;
            *status = OR_NONFINITE; *rank = 0; *resid = NAN;
            model_free(&M);
            return 0;
        }
    }
    double* A = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * n);
    double* b = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    build_design(&M, m, x, ldx, y, A);
    memcpy(b, y, sizeof(double) * (size_t)m);
    /* numerical rank: with fewer samples than unknowns and independent
     * samples, the unique minimum-norm interpolant; otherwise the natural-
     * order column rule (the minimum-norm minimiser of the problem whose
     * dependent columns are replaced by their projections) */
    int r = fit_lls((int)m, n, A, b, coef);
    /* residual of the linear problem, from the original data */
    build_design(&M, m, x, ldx, y, A);
    double rr = 0.0;
    for (long i = 0; i < m; i++) {
        double s = y[i];
        for (int j = 0; j < n; j++) s -= A[i + (long)j * m] * coef[j];
        rr += s * s;
    }
    *resid = sqrt(rr);
    *rank = r;
    if (m < n) *status = OR_UNDERDETERMINED;
    else if (r < n) *status = OR_RANK_DEFICIENT;
    else {
        *status = OR_OK;
        double ui[OR_MAXV];
        for (long i = 0; i < m; i++) {
            for (int k = 0; k < nvars; k++) ui[k] = x[k * ldx + i];
            double N, Q;
            model_nq(&M, coef, ui, &N, &Q);
            if (!(Q > 0.0)) { *status = OR_Q_NONPOSITIVE; break; }
        }
    }
    free(A); free(b); model_free(&M);
    return 0;
}

/* Batch driver over host threads (one fit per task). */
typedef struct {
    int F; const int64_t* off; const int32_t* nv; const int32_t* dn; const int32_t* dq;
    const double* x; long ldx; const double* y; const int64_t* coff;
    double* coef; int32_t* status; double* resid;
    volatile long next; pthread_mutex_t lock;
} batch_t;

static void* batch_worker(void* p) {
    batch_t* B = (batch_t*)p;
    for (;;) {
        pthread_mutex_lock(&B->lock);
        long f = B->next++;
        pthread_mutex_unlock(&B->lock);
        if (f >= B->F) break;
        int st, rk; double rs;
        long a = B->off[f];
        or_fit(B->off[f + 1] - a, B->nv[f], B->dn[f], B->dq[f], B->x + a, B->ldx,
               B->y + a, B->coef + B->coff[f], &st, &rk, &rs);
        B->status[f] = st; B->resid[f] = rs;
    }
    return NULL;
}

int or_fit_batch(int F, const int64_t* sample_off, const int32_t* nvars,
                 const int32_t* dn, const int32_t* dq, const double* x, long ldx,
                 const double* y, const int64_t* coef_off, double* coef,
                 int32_t* status, double* resid, int nthreads) {
    batch_t B = {F, sample_off, nvars, dn, dq, x, ldx, y, coef_off, coef, status, resid, 0,
                 PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1) nthreads = 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, batch_worker, &B);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    return 0;
}

/* ------------------------------------------------------------------ */
/* True loss, gradient, Levenberg-Marquardt                            */
/* ------------------------------------------------------------------ */

/* loss = sum_i (N_i/Q_i - y_i)^2; grad wrt [alpha | beta]. */
int or_loss_grad(long m, int nvars, int dn, int dq, const double* x, long ldx,
                 const double* y, const double* coef, double* loss, double* grad) {
    model_t M;
    if (model_init(&M, nvars, dn, dq)) return -1;
    int n = M.a + M.b;
    if (grad) for (int j = 0; j < n; j++) grad[j] = 0.0;
    double L = 0.0, ui[OR_MAXV];
    for (long i = 0; i < m; i++) {
        for (int k = 0; k < nvars; k++) ui[k] = x[k * ldx + i];
        double N, Q;
        model_nq(&M, coef, ui, &N, &Q);
        double f = N / Q, r = f - y[i];
        L += r * r;
        if (grad) {
            for (int j = 0; j < M.a; j++)
                grad[j] += 2.0 * r * monomial(M.ne + j * nvars, ui, nvars) / Q;
            for (int j = 1; j <= M.b; j++)
                grad[M.a + j - 1] -= 2.0 * r * (N / (Q * Q)) * monomial(M.de + j * nvars, ui, nvars);
        }
    }
    *loss = L;
    model_free(&M);
    return 0;
}

/* Levenberg-Marquardt from coef (in/out): each step solves
 * min || [J; sqrt(lambda) D] d - [r; 0] || with J_i = (1/Q_i)[m(u_i), -f_i m'(u_i)],
 * r_i = y_i - f_i and D = diag(column norms of J).  lambda starts at 0 (a pure
 * Gauss-Newton step).  Stops when a step changes the loss by less than
 * rtol * loss, or after max_iter steps. */
int or_refine(long m, int nvars, int dn, int dq, const double* x, long ldx,
              const double* y, double* coef, int max_iter, double rtol,
              double* loss_out, int* iters_out) {
    model_t M;
    if (model_init(&M, nvars, dn, dq)) return -1;
    int n = M.a + M.b;
    long rows = m + n;
    double* A = (double*)malloc(sizeof(double) * (size_t)rows * n);
    double* b = (double*)malloc(sizeof(double) * (size_t)rows);
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    double* cn = (double*)malloc(sizeof(double) * (size_t)n);
    double loss, lossn, lambda = 0.0, ui[OR_MAXV];
    or_loss_grad(m, nvars, dn, dq, x, ldx, y, coef, &loss, NULL);
    int it = 0, rejects = 0;
    for (it = 0; it < max_iter; it++) {
        for (long i = 0; i < m; i++) {
            for (int k = 0; k < nvars; k++) ui[k] = x[k * ldx + i];
            double N, Q;
            model_nq(&M, coef, ui, &N, &Q);
            double f = N / Q;
            for (int j = 0; j < M.a; j++)
                A[i + (long)j * rows] = monomial(M.ne + j * nvars, ui, nvars) / Q;
            for (int j = 1; j <= M.b; j++)
                A[i + (long)(M.a + j - 1) * rows] = -f * monomial(M.de + j * nvars, ui, nvars) / Q;
            b[i] = y[i] - f;
        }
        for (int j = 0; j < n; j++) {
            double s = 0.0;
            for (long i = 0; i < m; i++) s += A[i + (long)j * rows] * A[i + (long)j * rows];
            double dj = sqrt(lambda) * sqrt(s);
            for (int jj = 0; jj < n; jj++) A[m + jj + (long)j * rows] = (jj == j) ? dj : 0.0;
            b[m + j] = 0.0;
        }
        lls_qrcp((int)rows, n, A, b, d);
        for (int j = 0; j < n; j++) cn[j] = coef[j] + d[j];
        or_loss_grad(m, nvars, dn, dq, x, ldx, y, cn, &lossn, NULL);
        if (lossn <= loss) {
            double change = loss - lossn;
            memcpy(coef, cn, sizeof(double) * (size_t)n);
            loss = lossn;
            lambda = lambda * 0.1;
            if (lambda < 1e-12) lambda = 0.0;
            rejects = 0;
            if (change <= rtol * loss) { it++; break; }
        } else {
            lambda = lambda == 0.0 ? 1e-6 : lambda * 10.0;
            if (++rejects > 30) { it++; break; }
        }
    }
    *loss_out = loss;
    *iters_out = it;
    free(A); free(b); free(d); free(cn); model_free(&M);
    return 0;
}

/* ------------------------------------------------------------------ */
/* MWP-CWP-style template                                              */
/* ------------------------------------------------------------------ */

/* Metric slots (16) and hardware-vector entries (17); see the design notes. */
enum { G_COMP, G_COAL, G_UNCOAL, G_SYNCH, G_COAL_PER_MW, G_UNCOAL_PER_MW,
       G_LOAD_BYTES, G_REGS, G_LDS_BYTES, G_BLOCKS, G_SFU, G_LDS_INSTS,
       G_LDS_CONFLICT, G_BRANCH, G_L2_HIT, G_DIVERGENCE, G_COUNT };
enum { H_WAVE, H_NUM_CU, H_SIMD, H_TMAX, H_BMAX, H_WMAX, H_REGS_CU, H_LDS_CU,
       H_MEM_LAT, H_L2_LAT, H_DEP_COAL, H_DEP_UNCOAL, H_ISSUE, H_SFU_ISSUE,
       H_LDS_ISSUE, H_CLOCK, H_BW, H_COUNT };

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* Estimated cycles Ec for a block of T = bx*by threads given the 16 raw metric
 * values g and hardware vector h.  Returns +INFINITY for an infeasible block
 * (too many threads, or no block fits on a compute unit).  parts (optional,
 * 8 entries) receives B_active, N, MWP, CWP, Rep, Comp_cycles, Mem_cycles and
 * the case taken (1, 2 or 3). */
double or_mwpcwp(const double* g, const double* h, double bx, double by, double* parts) {
    double T = bx * by;
    double W = h[H_WAVE];
    if (!(T >= 1.0) || T > h[H_TMAX]) return INFINITY;
    /* guards: counts are nonnegative, rates lie in [0, 1], transactions >= 1 */
    double comp = dmax(g[G_COMP], 0.0), coal = dmax(g[G_COAL], 0.0);
    double uncoal = dmax(g[G_UNCOAL], 0.0), synch = dmax(g[G_SYNCH], 0.0);
    double coal_mw = dmax(g[G_COAL_PER_MW], 1.0), uncoal_mw = dmax(g[G_UNCOAL_PER_MW], 1.0);
    double load_bytes = dmax(g[G_LOAD_BYTES], 0.0);
    double regs = ceil(dmax(g[G_REGS], 1.0));
    double lds = ceil(dmax(g[G_LDS_BYTES], 0.0));
    double blocks = ceil(dmax(g[G_BLOCKS], 1.0));
    double sfu = dmax(g[G_SFU], 0.0), lds_insts = dmax(g[G_LDS_INSTS], 0.0);
    double conflict = dmax(g[G_LDS_CONFLICT], 0.0), branch = dmax(g[G_BRANCH], 0.0);
    double hit = dmin(dmax(g[G_L2_HIT], 0.0), 1.0);
    double diverge = dmin(dmax(g[G_DIVERGENCE], 0.0), 1.0);

    /* occupancy: blocks resident per compute unit, then equation (occupancy) */
    double wpb = ceil(T / W);
    double b_waves = floor(h[H_WMAX] / wpb);
    double b_regs = floor(h[H_REGS_CU] / (regs * W * wpb));
    double b_lds = lds > 0.0 ? floor(h[H_LDS_CU] / lds) : h[H_BMAX];
    double b_active = dmin(dmin(h[H_BMAX], b_waves), dmin(b_regs, b_lds));
    if (!(b_active >= 1.0)) return INFINITY;
    double N = dmin(floor(b_active * T / W), h[H_WMAX]);
    double active_cu = dmin(h[H_NUM_CU], blocks);
    double rep = ceil(blocks / (b_active * active_cu));

    /* memory warp parallelism */
    double mem = coal + uncoal;
    double w_u = mem > 0.0 ? uncoal / mem : 0.0;
    double w_c = 1.0 - w_u;
    double mem_eff = dmax(mem, 1.0);
    double lat = (1.0 - hit) * h[H_MEM_LAT] + hit * h[H_L2_LAT];
    double mem_l_uncoal = lat + (uncoal_mw - 1.0) * h[H_DEP_UNCOAL];
    double mem_l_coal = lat + (coal_mw - 1.0) * h[H_DEP_COAL];
    double mem_l = mem_l_uncoal * w_u + mem_l_coal * w_c;
    double dep = h[H_DEP_UNCOAL] * uncoal_mw * w_u + h[H_DEP_COAL] * coal_mw * w_c;
    double mwp_nobw = mem_l / dep;
    double mwp_bw = INFINITY;
    if (load_bytes > 0.0) {
        double bw_per_warp = h[H_CLOCK] * load_bytes / mem_l;
        mwp_bw = h[H_BW] / (bw_per_warp * active_cu);
    }
    double mwp = dmax(dmin(dmin(mwp_nobw, mwp_bw), N), 1.0);

    /* computation warp parallelism */
    double comp_cycles = h[H_ISSUE] * (comp + mem + branch * (1.0 + diverge))
                       + h[H_SFU_ISSUE] * sfu + h[H_LDS_ISSUE] * lds_insts * (1.0 + conflict);
    comp_cycles = dmax(comp_cycles, h[H_ISSUE]);
    double mem_cycles = mem_l_uncoal * uncoal + mem_l_coal * coal;
    double cwp_full = (mem_cycles + comp_cycles) / comp_cycles;
    double cwp = dmin(cwp_full, N);

    double e; int cas;
    if (mwp == N && cwp == N) {
        e = (mem_cycles + comp_cycles + comp_cycles / mem_eff * (mwp - 1.0)) * rep; cas = 1;
    } else if (cwp >= mwp || comp_cycles > mem_cycles) {
        e = (mem_cycles * N / mwp + comp_cycles / mem_eff * (mwp - 1.0)) * rep; cas = 2;
    } else {
        e = (lat + comp_cycles * N) * rep; cas = 3;
    }
    double synch_cost = dep * (mwp - 1.0) * synch * b_active * rep;
    if (parts) {
        parts[0] = b_active; parts[1] = N; parts[2] = mwp; parts[3] = cwp;
        parts[4] = rep; parts[5] = comp_cycles; parts[6] = mem_cycles; parts[7] = cas;
    }
    return e + synch_cost;
}

/* Hardware occupancy of a block of T = bx*by threads that uses regs
 * registers per thread and lds bytes of LDS per block: the number of active
 * waves per compute unit over the maximum, W_active / W_max, with W_active =
 * min(floor(B_active T / W), W_max) (equation (occupancy), wave size W as a
 * parameter) and B_active the number of blocks that fit on one unit at once:
 * at most max_blocks, at most max_waves / ceil(T / W) by waves, at most
 * regs_per_cu / (regs W ceil(T / W)) by registers (a partial wave holds a
 * whole wave's registers) and at most lds_per_cu / lds by LDS, each rounded
 * down.  Counts are rounded up and kept >= 1 (registers) or >= 0 (LDS) as in
 * or_mwpcwp.  -INFINITY when the block cannot run (T > max_threads or no
 * block fits). */
double or_occupancy(double regs_in, double lds_in, const double* h, double bx, double by) {
    double T = bx * by;
    double W = h[H_WAVE];
    if (!(T >= 1.0) || T > h[H_TMAX]) return -INFINITY;
    double regs = ceil(dmax(regs_in, 1.0));
    double lds = ceil(dmax(lds_in, 0.0));
    double waves_per_block = ceil(T / W);
    double by_blocks = h[H_BMAX];
    double by_waves = floor(h[H_WMAX] / waves_per_block);
    double by_regs = floor(h[H_REGS_CU] / (regs * W * waves_per_block));
    double by_lds = lds > 0.0 ? floor(h[H_LDS_CU] / lds) : h[H_BMAX];
    double b_active = dmin(dmin(by_blocks, by_waves), dmin(by_regs, by_lds));
    if (!(b_active >= 1.0)) return -INFINITY;
    double w_active = dmin(floor(b_active * T / W), h[H_WMAX]);
    return w_active / h[H_WMAX];
}

/* ------------------------------------------------------------------ */
/* Program evaluation and exhaustive argmin                            */
/* ------------------------------------------------------------------ */

enum { OR_TEMPLATE_SINGLE = 0, OR_TEMPLATE_MWPCWP = 1, OR_TEMPLATE_OCCUPANCY = 2 };

/* Value of a program whose L metric models are already built.  The metric
 * rationals take u = (n / scale[0], c_0 / scale[1], ...). */
static double program_value_m(int template_id, int L, const model_t* M,
                              const int64_t* coef_off, const double* coef,
                              const double* hw, const double* scale, double n,
                              const int32_t* c, int cdim) {
    double u[OR_MAXV], g[32];
    int nvars = M[0].nvars;
    if (nvars != 1 + cdim || L > 32) return NAN;
    u[0] = n / scale[0];
    for (int k = 0; k < cdim; k++) u[1 + k] = (double)c[k] / scale[1 + k];
    for (int l = 0; l < L; l++) {
        double N, Q;
        model_nq(&M[l], coef + coef_off[l], u, &N, &Q);
        if (template_id == OR_TEMPLATE_SINGLE && !(Q > 0.0)) return INFINITY;
        g[l] = N / Q;
    }
    if (template_id == OR_TEMPLATE_SINGLE) return g[0];
    if (template_id == OR_TEMPLATE_OCCUPANCY) {
        /* metrics: registers per thread, LDS bytes per block */
        if (L != 2 || cdim != 2) return NAN;
        return or_occupancy(g[0], g[1], hw, (double)c[0], (double)c[1]);
    }
    if (L != G_COUNT || cdim != 2) return NAN;
    return or_mwpcwp(g, hw, (double)c[0], (double)c[1], NULL);
}

static int build_models(model_t* M, int L, int nvars, const int32_t* dn, const int32_t* dq) {
    for (int l = 0; l < L; l++)
        if (model_init(&M[l], nvars, dn[l], dq[l])) {
            for (int t = 0; t < l; t++) model_free(&M[t]);
            return -1;
        }
    return 0;
}

/* Evaluate one program at data size n and candidate c[0..cdim-1]. */
double or_program_value(int template_id, int L, int nvars, const int32_t* dn,
                        const int32_t* dq, const int64_t* coef_off, const double* coef,
                        const double* hw, const double* scale, double n,
                        const int32_t* c, int cdim) {
    model_t M[32];
    if (L < 1 || L > 32 || build_models(M, L, nvars, dn, dq)) return NAN;
    double v = program_value_m(template_id, L, M, coef_off, coef, hw, scale, n, c, cdim);
    for (int l = 0; l < L; l++) model_free(&M[l]);
    return v;
}

/* For each program p and data size n_j: the candidate minimising the value
 * (lowest index on exact ties, non-finite values skipped; -1 when none is
 * finite), the best value and the best value among the other candidates.
 * Program p uses metric models p*L .. p*L+L-1 and hardware vector
 * hw + p*hw_stride (hw may be NULL for the single-rational template). */
int or_argmin(int template_id, int num_programs, int L, int nvars,
              const int32_t* dn, const int32_t* dq, const int64_t* coef_off,
              const double* coef, const double* hw, int hw_stride,
              const double* scale, const double* n_grid, int num_n,
              const int32_t* cand, int num_cand, int cdim,
              int32_t* argmin, double* best, double* second) {
    model_t M[32];
    if (L < 1 || L > 32) return -1;
    for (int p = 0; p < num_programs; p++) {
        if (build_models(M, L, nvars, dn + (long)p * L, dq + (long)p * L)) return -1;
        const double* hp = hw ? hw + (long)p * hw_stride : NULL;
        for (int j = 0; j < num_n; j++) {
            int bi = -1; double bv = INFINITY, sv = INFINITY;
            for (int c = 0; c < num_cand; c++) {
                double v = program_value_m(template_id, L, M, coef_off + (long)p * L, coef,
                                           hp, scale, n_grid[j], cand + (long)c * cdim, cdim);
                if (!isfinite(v)) continue;
                if (bi < 0 || v < bv) { sv = bv; bv = v; bi = c; }
                else if (v < sv) sv = v;
            }
            argmin[(long)p * num_n + j] = bi;
            best[(long)p * num_n + j] = bv;
            second[(long)p * num_n + j] = sv;
        }
        for (int l = 0; l < L; l++) model_free(&M[l]);
    }
    return 0;
}

/* Selection with a sense and an optional tie-breaking program.  For program
 * p and data size n_j, every candidate's value E (non-finite values skipped)
 * is compared by sense * E (sense = +1: smallest E wins, -1: largest); among
 * candidates whose E equals the winner's exactly, the tie program (if given,
 * with its own sense; a non-finite tie value ranks last) decides, then the
 * lowest index.  choice = -1 when no E is finite; best = the winner's E;
 * second = the winning-most E among the other candidates (sense * second =
 * +INFINITY when there is none).  Both programs take the same (n, candidate). */
int or_select(int template_id, int num_programs, int L, int nvars,
              const int32_t* dn, const int32_t* dq, const int64_t* coef_off,
              const double* coef, const double* hw, int hw_stride, double sense,
              int tie_template, int tie_L, const int32_t* tie_dn, const int32_t* tie_dq,
              const int64_t* tie_coef_off, const double* tie_coef, const double* tie_hw,
              int tie_hw_stride, double tie_sense,
              const double* scale, const double* n_grid, int num_n,
              const int32_t* cand, int num_cand, int cdim,
              int32_t* choice, double* best, double* second) {
    model_t M[32], MT[32];
    int use_tie = tie_L > 0;
    if (L < 1 || L > 32 || tie_L > 32) return -1;
    if (!(sense == 1.0 || sense == -1.0) || (use_tie && !(tie_sense == 1.0 || tie_sense == -1.0)))
        return -1;
    double* val = (double*)malloc(sizeof(double) * (size_t)(num_cand > 0 ? num_cand : 1));
    for (int p = 0; p < num_programs; p++) {
        if (build_models(M, L, nvars, dn + (long)p * L, dq + (long)p * L)) { free(val); return -1; }
        if (use_tie && build_models(MT, tie_L, nvars, tie_dn + (long)p * tie_L, tie_dq + (long)p * tie_L)) {
            for (int l = 0; l < L; l++) model_free(&M[l]);
            free(val);
            return -1;
        }
        const double* hp = hw ? hw + (long)p * hw_stride : NULL;
        const double* thp = tie_hw ? tie_hw + (long)p * tie_hw_stride : NULL;
        for (int j = 0; j < num_n; j++) {
            /* first key: sense * E over every candidate */
            for (int c = 0; c < num_cand; c++)
                val[c] = sense * program_value_m(template_id, L, M, coef_off + (long)p * L, coef,
                                                 hp, scale, n_grid[j], cand + (long)c * cdim, cdim);
            double kbest = INFINITY;
            for (int c = 0; c < num_cand; c++)
                if (isfinite(val[c]) && val[c] < kbest) kbest = val[c];
            int bi = -1;
            double tbest = INFINITY;
            if (isfinite(kbest)) {
                /* every candidate reaching kbest, the tie key deciding */
                for (int c = 0; c < num_cand; c++) {
                    if (!(val[c] == kbest)) continue;
                    double t = 0.0;
                    if (use_tie) {
                        t = tie_sense * program_value_m(tie_template, tie_L, MT,
                                                        tie_coef_off + (long)p * tie_L, tie_coef,
                                                        thp, scale, n_grid[j],
                                                        cand + (long)c * cdim, cdim);
                        if (!isfinite(t)) t = INFINITY;
                    }
                    if (bi < 0 || t < tbest) { bi = c; tbest = t; }
                }
            }
            double ksecond = INFINITY;
            for (int c = 0; c < num_cand; c++)
                if (c != bi && isfinite(val[c]) && val[c] < ksecond) ksecond = val[c];
            choice[(long)p * num_n + j] = bi;
            best[(long)p * num_n + j] = sense * kbest;
            second[(long)p * num_n + j] = sense * ksecond;
        }
        for (int l = 0; l < L; l++) model_free(&M[l]);
        if (use_tie) for (int l = 0; l < tie_L; l++) model_free(&MT[l]);
    }
    free(val);
    return 0;
}

/* "Error" of Section 5: (C_rt - Best_t) / (Worst_t - Best_t) * 100. */
double or_regret(double crt, double best_t, double worst_t) {
    return (crt - best_t) / (worst_t - best_t) * 100.0;
}

/* ------------------------------------------------------------------ */
/* One decision node fitted from the samples (Section 3.2, the third   */
/* consequence: the branch conditions of a rational program are         */
/* themselves rational and could be fitted like its process nodes)      */
/* ------------------------------------------------------------------ */

/* A piecewise rational function with one decision node on variable s:
 * y = f_L(u) where u_s <= theta, f_R(u) where u_s > theta, f_L and f_R of
 * total degree d over d.  Fitted by exhaustive search over the breakpoint:
 * with the samples in ascending order of u_s (equal values by sample index),
 * every split k -- the first k samples on the left -- that leaves at least
 * n_min samples on each side and does not separate two equal values of u_s
 * is a candidate; each side is fitted by the linearised least squares of
 * or_fit and the candidate's objective is the sum of the two sides' squared
 * residual norms.  The smallest objective wins, the smallest k on exact
 * ties.  theta = (u_s of sample k-1 + u_s of sample k) / 2 in the sorted
 * order.  Outputs: *k_out (-1 when there is no candidate, then theta and
 * the coefficients are NaN and *obj_out is +inf), *theta, coef_l, coef_r
 * (num_coefs(nvars, d, d) each), the sides' statuses, *obj_out, and
 * obj_all[k] for k = 0..m (+inf where k is no candidate; may be NULL).  A
 * node with a non-finite sample has no candidate and both statuses
 * non-finite. */
static const double* g_split_key;
static int split_cmp(const void* pa, const void* pb) {
    long a = *(const long*)pa, b = *(const long*)pb;
    double ka = g_split_key[a], kb = g_split_key[b];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (a > b) - (a < b);
}

int or_split_fit(long m, int nvars, int d, int split_var, long n_min, const double* x, long ldx,
                 const double* y, long* k_out, double* theta, double* coef_l, double* coef_r,
                 int* status_l, int* status_r, double* obj_out, double* obj_all) {
    model_t M;
    if (split_var < 0 || split_var >= nvars || n_min < 1) return -1;
    if (model_init(&M, nvars, d, d)) return -1;
    int n = M.a + M.b;
    model_free(&M);
    /* a non-finite sample: no candidate, both sides non-finite */
    for (long i = 0; i < m; i++) {
        int bad = !isfinite(y[i]);
        for (int k = 0; k < nvars; k++) bad |= !isfinite(x[k * ldx + i]);
        if (bad) {
            *k_out = -1; *theta = NAN; *obj_out = INFINITY;
            for (int j = 0; j < n; j++) { coef_l[j] = NAN; coef_r[j] = NAN; }
            *status_l = *status_r = OR_NONFINITE;
            if (obj_all) for (long k = 0; k <= m; k++) obj_all[k] = INFINITY;
            return 0;
        }
    }
    long* perm = (long*)malloc(sizeof(long) * (size_t)(m > 0 ? m : 1));
    for (long i = 0; i < m; i++) perm[i] = i;
    /* sort by u_s (qsort with the index as the second key: a total order) */
    static pthread_mutex_t sort_lock = PTHREAD_MUTEX_INITIALIZER;
    pthread_mutex_lock(&sort_lock);
    g_split_key = x + (long)split_var * ldx;
    qsort(perm, (size_t)m, sizeof(long), split_cmp);
    pthread_mutex_unlock(&sort_lock);
    double* xs = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * nvars);
    double* ys = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* xl = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * nvars);
    double* cl = (double*)malloc(sizeof(double) * (size_t)n);
    double* cr = (double*)malloc(sizeof(double) * (size_t)n);
    for (long i = 0; i < m; i++) {
        for (int k = 0; k < nvars; k++) xs[k * m + i] = x[k * ldx + perm[i]];
        ys[i] = y[perm[i]];
    }
    long best_k = -1;
    double best = INFINITY;
    if (obj_all) for (long k = 0; k <= m; k++) obj_all[k] = INFINITY;
    const double* us = xs + (long)split_var * m;
    for (long k = n_min; k <= m - n_min; k++) {
        if (!(us[k - 1] < us[k])) continue;     /* equal values stay together */
        int stl, str, rk;
        double rl, rr;
        /* the left samples [0, k) as a fit of their own (leading dimension k) */
        for (int j = 0; j < nvars; j++)
            for (long i = 0; i < k; i++) xl[j * k + i] = xs[j * m + i];
        or_fit(k, nvars, d, d, xl, k, ys, cl, &stl, &rk, &rl);
        or_fit(m - k, nvars, d, d, xs + k, m, ys + k, cr, &str, &rk, &rr);
        double obj = rl * rl + rr * rr;
        if (obj_all) obj_all[k] = obj;
        if (obj < best) {
            best = obj; best_k = k;
            memcpy(coef_l, cl, sizeof(double) * (size_t)n);
            memcpy(coef_r, cr, sizeof(double) * (size_t)n);
            *status_l = stl; *status_r = str;
        }
    }
    *k_out = best_k;
    *obj_out = best;
    if (best_k < 0) {
        *theta = NAN;
        for (int j = 0; j < n; j++) { coef_l[j] = NAN; coef_r[j] = NAN; }
        *status_l = *status_r = OR_UNDERDETERMINED;
    } else {
        *theta = 0.5 * (us[best_k - 1] + us[best_k]);
    }
    free(perm); free(xs); free(ys); free(xl); free(cl); free(cr);
    return 0;
}
