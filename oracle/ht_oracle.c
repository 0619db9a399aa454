/*
 * ht_oracle.c -- CPU FP64 oracle for Hessenberg-triangular (HT) reduction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py use it.  It shares no code with the HIP implementation.
 *
 * Problem (Bujanovic, Karlsson, Kressner, "A Householder-based algorithm for
 * Hessenberg-triangular reduction", Sec. 1 and Sec. 3 opening): given A and an
 * upper triangular B, find orthogonal Q, Z (initialised to I) such that
 * H = Q^T A Z is upper Hessenberg and T = Q^T B Z is upper triangular.
 *
 * Two independent constructions are provided:
 *
 *   orc_basic_ht  -- Algorithm 2 (BasicHouseHT, Appendix A): per column j a
 *                    conventional Householder reflector from the left reduces
 *                    A(j+1:n, j), a dense solve B(j+1:n, j+1:n) x = e1 gives
 *                    an opposite reflector (Sec. 2.2) applied from the right,
 *                    which reduces column j+1 of B.  Theta(n^4).
 *   orc_ms_ht     -- the Givens-rotation HT reduction of Moler and Stewart
 *                    (the paper's comparison baseline, Sec. 1): rotations from
 *                    the left annihilate A(i, j) bottom-up, each fill-in
 *                    B(i, i-1) is removed by a rotation from the right.
 *                    Theta(n^3), needs no solves.
 *
 * Both leave Q e1 = e1 and Z e1 = e1 exactly, so by the implicit-Q theorem
 * their outputs agree up to +-1 diagonal scalings when the pencil is regular
 * and H T^{-1} is unreduced.
 *
 * Conventions (readings where the paper is silent):
 *   - house(x) follows Golub & Van Loan, Matrix Computations, Alg. 5.1.1,
 *     as cited in Lemma 2.1: P x = +||x||_2 e1, v(1) = 1; with x(2:m) = 0
 *     and x(1) < 0 we use beta = 2 (P = diag(-1, 1, ..)), with x(1) >= 0
 *     beta = 0.  Norms are computed on a scaled copy so entries near
 *     1e+-300 do not overflow or underflow.
 *   - zero pivots are replaced by 2 u rho ||B||_F, rho ~ N(0,1) (Sec. 3.2.1,
 *     Remark 2.2); rho is drawn from splitmix64 (Steele, Lea, Flood 2014)
 *     keyed by (seed, draw counter) and mapped by Box-Muller.
 *   - the back substitution rescales its partial solution whenever the next
 *     entry would exceed 2^600, returning a vector parallel to the solution;
 *     only the direction of x enters the opposite reflector (Lemma 2.1).
 *
 * All matrices are column-major FP64 with leading dimension n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(j) * (size_t)(ld) + (size_t)(i))

/* ------------------------------------------------------------------------ */
/* Random numbers for the zero-diagonal perturbation (Sec. 3.2.1).          */
/* ------------------------------------------------------------------------ */

static uint64_t orc_splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Standard normal number number `counter` of stream `seed` (Box-Muller on
 * two 53-bit uniforms in (0, 1]). */
double orc_normal(uint64_t seed, uint64_t counter)
{
    uint64_t a = orc_splitmix64(seed ^ orc_splitmix64(2 * counter));
    uint64_t b = orc_splitmix64(seed ^ orc_splitmix64(2 * counter + 1));
    double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;
    double u2 = ((double)(b >> 11)) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ------------------------------------------------------------------------ */
/* Householder reflector, Golub & Van Loan Alg. 5.1.1 (Sec. 2.1).          */
/* ------------------------------------------------------------------------ */

/* Computes v (v[0] = 1) and beta with (I - beta v v^T) x = alpha e1,
 * alpha = ||x||_2 >= 0.  Returns alpha. */
double orc_house(int m, const double *x, double *v, double *beta)
{
    double scale = 0.0;
    for (int i = 0; i < m; i++)
        if (fabs(x[i]) > scale) scale = fabs(x[i]);
    v[0] = 1.0;
    for (int i = 1; i < m; i++) v[i] = 0.0;
    if (scale == 0.0) { *beta = 0.0; return 0.0; }

    double y1 = x[0] / scale;
    double sigma = 0.0;
    for (int i = 1; i < m; i++) { double t = x[i] / scale; sigma += t * t; }
    if (sigma == 0.0) {
        if (y1 >= 0.0) { *beta = 0.0; return x[0]; }
        *beta = 2.0;            /* P = diag(-1, 1, ...): P x = |x1| e1 */
        return -x[0];
    }
    double mu = sqrt(y1 * y1 + sigma);
    double v1 = (y1 <= 0.0) ? (y1 - mu) : (-sigma / (y1 + mu));
    *beta = 2.0 * v1 * v1 / (sigma + v1 * v1);
    for (int i = 1; i < m; i++) v[i] = (x[i] / scale) / v1;
    return mu * scale;
}

/* X(0:m, 0:nc) <- (I - beta v v^T) X */
static void orc_apply_left(int m, int nc, const double *v, double beta,
                           double *X, int ldx)
{
    if (beta == 0.0) return;
    for (int c = 0; c < nc; c++) {
        double *col = X + IDX(0, c, ldx);
        double d = 0.0;
        for (int i = 0; i < m; i++) d += v[i] * col[i];
        d *= beta;
        for (int i = 0; i < m; i++) col[i] -= d * v[i];
    }
}

/* X(0:nr, 0:m) <- X (I - beta v v^T) */
static void orc_apply_right(int nr, int m, const double *v, double beta,
                            double *X, int ldx)
{
    if (beta == 0.0) return;
    double *w = (double *)calloc((size_t)nr, sizeof(double));
    for (int c = 0; c < m; c++) {
        const double *col = X + IDX(0, c, ldx);
        for (int r = 0; r < nr; r++) w[r] += col[r] * v[c];
    }
    for (int c = 0; c < m; c++) {
        double *col = X + IDX(0, c, ldx);
        double f = beta * v[c];
        for (int r = 0; r < nr; r++) col[r] -= w[r] * f;
    }
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Dense solve M x = b by LU with partial pivoting (Algorithm 2's linear    */
/* system step), zero-pivot rule and overflow-safe back substitution.       */
/* ------------------------------------------------------------------------ */

/* M (m x m, ld m) is overwritten.  On return x is parallel to M^{-1} b
 * (x = sigma M^{-1} b with 0 < sigma <= 1).  *perturbed counts replaced
 * pivots; *draws is the running counter of normal numbers used. */
static void orc_solve_dense(int m, double *M, const double *b, double *x,
                            double normB, uint64_t seed, uint64_t *draws,
                            int *perturbed)
{
    const double u = 0x1.0p-53;
    int *piv = (int *)malloc((size_t)m * sizeof(int));
    for (int k = 0; k < m; k++) {
        int p = k;
        double best = fabs(M[IDX(k, k, m)]);
        for (int i = k + 1; i < m; i++)
            if (fabs(M[IDX(i, k, m)]) > best) { best = fabs(M[IDX(i, k, m)]); p = i; }
        piv[k] = p;
        if (p != k)
            for (int c = 0; c < m; c++) {
                double t = M[IDX(k, c, m)];
                M[IDX(k, c, m)] = M[IDX(p, c, m)];
                M[IDX(p, c, m)] = t;
            }
        if (M[IDX(k, k, m)] == 0.0) {
            M[IDX(k, k, m)] = 2.0 * u * orc_normal(seed, (*draws)++) * normB;
            (*perturbed)++;
        }
        double d = M[IDX(k, k, m)];
        for (int i = k + 1; i < m; i++) M[IDX(i, k, m)] /= d;
        for (int c = k + 1; c < m; c++) {
            double f = M[IDX(k, c, m)];
            if (f == 0.0) continue;
            for (int i = k + 1; i < m; i++) M[IDX(i, c, m)] -= M[IDX(i, k, m)] * f;
        }
    }
    /* forward substitution with the unit lower factor on the permuted rhs */
    for (int i = 0; i < m; i++) x[i] = b[i];
    for (int k = 0; k < m; k++)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int k = 0; k < m; k++)
        for (int i = k + 1; i < m; i++) x[i] -= M[IDX(i, k, m)] * x[k];
    /* back substitution with the upper factor, rescaling to stay finite */
    const double big = 0x1.0p600, shrink = 0x1.0p-600;
    for (int i = m - 1; i >= 0; i--) {
        double s = x[i];
        for (int c = i + 1; c < m; c++) s -= M[IDX(i, c, m)] * x[c];
        double d = M[IDX(i, i, m)];
        while (fabs(s) > big * fabs(d) || fabs(s) > big) {
            for (int t = 0; t < m; t++) x[t] *= shrink;
            s *= shrink;
        }
        x[i] = s / d;
    }
    free(piv);
}

static double orc_frob(int n, const double *X)
{
    double scale = 0.0, ssq = 1.0;
    for (size_t i = 0; i < (size_t)n * n; i++) {
        double a = fabs(X[i]);
        if (a == 0.0) continue;
        if (a > scale) { ssq = 1.0 + ssq * (scale / a) * (scale / a); scale = a; }
        else ssq += (a / scale) * (a / scale);
    }
    return scale * sqrt(ssq);
}

static void orc_identity(int n, double *X)
{
    memset(X, 0, (size_t)n * n * sizeof(double));
    for (int i = 0; i < n; i++) X[IDX(i, i, n)] = 1.0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (BasicHouseHT), Appendix A.                                   */
/* ------------------------------------------------------------------------ */

/* Reduces the first `ncols` columns (ncols <= n-2; pass n-2 for the full
 * reduction).  A, B are overwritten by H, T; Q, Z are set.  B must be upper
 * triangular on entry.  Returns the number of perturbed pivots. */
int orc_basic_ht(int n, double *A, double *B, double *Q, double *Z,
                 int ncols, uint64_t seed)
{
    orc_identity(n, Q);
    orc_identity(n, Z);
    if (ncols > n - 2) ncols = n - 2;
    const double normB = orc_frob(n, B);
    uint64_t draws = 0;
    int perturbed = 0;
    double *v = (double *)malloc((size_t)n * sizeof(double));
    double *x = (double *)malloc((size_t)n * sizeof(double));
    double *rhs = (double *)malloc((size_t)n * sizeof(double));
    double *M = (double *)malloc((size_t)n * n * sizeof(double));

    for (int j = 0; j < ncols; j++) {
        const int m = n - j - 1;            /* rows/cols j+1 .. n-1 */
        double beta;
        /* F_j = I_j (+) House(A(j+1:n, j)) */
        double alpha = orc_house(m, A + IDX(j + 1, j, n), v, &beta);
        /* A <- F_j A, B <- F_j B, Q <- Q F_j */
        orc_apply_left(m, n, v, beta, A + IDX(j + 1, 0, n), n);
        orc_apply_left(m, n, v, beta, B + IDX(j + 1, 0, n), n);
        orc_apply_right(n, m, v, beta, Q + IDX(0, j + 1, n), n);
        /* A(j+2:n, j) <- 0 */
        A[IDX(j + 1, j, n)] = alpha;
        for (int i = j + 2; i < n; i++) A[IDX(i, j, n)] = 0.0;

        /* solve B(j+1:n, j+1:n) x = e1 */
        for (int c = 0; c < m; c++)
            memcpy(M + IDX(0, c, m), B + IDX(j + 1, j + 1 + c, n),
                   (size_t)m * sizeof(double));
        for (int i = 0; i < m; i++) rhs[i] = (i == 0) ? 1.0 : 0.0;
        orc_solve_dense(m, M, rhs, x, normB, seed, &draws, &perturbed);

        /* G_j = I_j (+) House(x): A <- A G_j, B <- B G_j, Z <- Z G_j */
        double gamma;
        orc_house(m, x, v, &gamma);
        orc_apply_right(n, m, v, gamma, A + IDX(0, j + 1, n), n);
        orc_apply_right(n, m, v, gamma, B + IDX(0, j + 1, n), n);
        orc_apply_right(n, m, v, gamma, Z + IDX(0, j + 1, n), n);
        /* B(j+2:n, j+1) <- 0 */
        for (int i = j + 2; i < n; i++) B[IDX(i, j + 1, n)] = 0.0;
    }
    free(v); free(x); free(rhs); free(M);
    return perturbed;
}

/* ------------------------------------------------------------------------ */
/* Moler-Stewart Givens HT reduction (the comparison algorithm of Sec. 1).  */
/* ------------------------------------------------------------------------ */

/* Rotation (c, s) with [c s; -s c] [a; b] = [r; 0]. */
static void orc_givens(double a, double b, double *c, double *s)
{
    if (b == 0.0) { *c = 1.0; *s = 0.0; return; }
    double r = hypot(a, b);
    *c = a / r;
    *s = b / r;
}

/* rows p, p+1 of X (all nc columns) <- [c s; -s c] rows */
static void orc_rot_rows(int nc, double c, double s, double *X, int ldx, int p)
{
    for (int col = 0; col < nc; col++) {
        double a = X[IDX(p, col, ldx)], b = X[IDX(p + 1, col, ldx)];
        X[IDX(p, col, ldx)] = c * a + s * b;
        X[IDX(p + 1, col, ldx)] = -s * a + c * b;
    }
}

/* columns p, p+1 of X (all nr rows) <- [col_p, col_p+1] [c s; -s c] */
static void orc_rot_cols(int nr, double c, double s, double *X, int ldx, int p)
{
    double *x0 = X + IDX(0, p, ldx), *x1 = X + IDX(0, p + 1, ldx);
    for (int r = 0; r < nr; r++) {
        double a = x0[r], b = x1[r];
        x0[r] = c * a - s * b;
        x1[r] = s * a + c * b;
    }
}

/* Reduces the first `ncols` columns of A (ncols <= n-2).  Q, Z are set. */
void orc_ms_ht(int n, double *A, double *B, double *Q, double *Z, int ncols)
{
    orc_identity(n, Q);
    orc_identity(n, Z);
    if (ncols > n - 2) ncols = n - 2;
    for (int j = 0; j < ncols; j++) {
        for (int i = n - 1; i >= j + 2; i--) {
            double c, s;
            /* left rotation on rows (i-1, i) annihilates A(i, j) */
            orc_givens(A[IDX(i - 1, j, n)], A[IDX(i, j, n)], &c, &s);
            orc_rot_rows(n, c, s, A, n, i - 1);
            orc_rot_rows(n, c, s, B, n, i - 1);
            /* Q <- Q G^T: columns (i-1, i) get [c -s; s c] */
            orc_rot_cols(n, c, -s, Q, n, i - 1);
            A[IDX(i, j, n)] = 0.0;
            /* right rotation on columns (i-1, i) annihilates B(i, i-1):
             * with b1 = B(i,i-1), b2 = B(i,i): [b1 b2][c s; -s c] has first
             * entry c b1 - s b2 = 0 for c = b2/r, s = b1/r. */
            double b1 = B[IDX(i, i - 1, n)], b2 = B[IDX(i, i, n)];
            if (b1 != 0.0) {
                double r = hypot(b1, b2);
                c = b2 / r;
                s = b1 / r;
                orc_rot_cols(n, c, s, B, n, i - 1);
                orc_rot_cols(n, c, s, A, n, i - 1);
                orc_rot_cols(n, c, s, Z, n, i - 1);
            }
            B[IDX(i, i - 1, n)] = 0.0;
        }
    }
}

/* Frobenius norm exported for the Python side's tolerance computations. */
double orc_frobenius(int n, const double *X) { return orc_frob(n, X); }
