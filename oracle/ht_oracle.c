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
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

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

/* ------------------------------------------------------------------------ */
/* O-fast: Algorithm 2's reflector pair per column, with the trailing block */
/* of B kept upper triangular, so every solve is a triangular one.          */
/* ------------------------------------------------------------------------ */
/*
 * Per column j (m = n-j-1 trailing rows/columns, R = B(j+1:n, j+1:n) upper
 * triangular on entry):
 *   1. F = I - tau v v^T = House(A(j+1:n, j)) is applied to A(j+1:n, j:n)
 *      and accumulated in Q(:, j+1:n), exactly as in Algorithm 2.
 *   2. x solves (F R) x = e1, i.e. R x = F e1 = e1 - tau v v(1): the
 *      right-hand side of the first-column formula of Sec. 2.2 / 3.2.2,
 *      by scaled back substitution.
 *   3. G = I - gamma w w^T = House(x) is applied to A(:, j+1:n),
 *      Z(:, j+1:n) and the rows 0..j of B(:, j+1:n).
 *   4. F R G = R - tau v t^T - gamma p w^T with t = R^T v and
 *      p = R w - tau v (t^T w).  Its first column is a multiple of e1 up to
 *      rounding (Lemma 2.1) and is set to that; its first row is formed
 *      directly; its trailing block is R22 + a1 b1^T + a2 b2^T with
 *      a1 = -tau v(2:m), b1 = t(2:m), a2 = -gamma p(2:m), b2 = w(2:m).
 *   5. The trailing block is made triangular again by two rank-one QR
 *      updates with Givens rotations (Golub & Van Loan, Matrix
 *      Computations, Sec. 6.5): rotations bottom-up turn a into ||a|| e1
 *      (R22 becomes upper Hessenberg), the rank-one term then only changes
 *      the first row, and rotations top-down restore the triangle.  a2 is
 *      rotated along with the first update.  These rotations act on rows
 *      j+2..n-1 only; they are further left transformations, applied to
 *      A(j+2:n, j+1:n) and accumulated in Q(:, j+2:n).  They leave the
 *      reduced columns of A and column j+1 of B untouched, and Q e1 = e1.
 * The result satisfies the same problem statement as Algorithm 2 (Q e1 =
 * e1, H Hessenberg, T triangular), so by the implicit-Q theorem it equals
 * Algorithm 2's up to the signs of the columns of Q and Z.  Cost
 * Theta(n^3) (about 33 n^3 flops) instead of Theta(n^4).
 *
 * OpenMP parallelises only loops whose iterations are independent
 * (columns of A and R, row chunks of Q and Z); every sum is formed in the
 * same order whatever the thread count, so results are bitwise independent
 * of it.
 */

typedef struct { int p; double c, s; } orc_rot;  /* rows (p, p+1): [c s; -s c] */

/* ORC_PLANT (compile-time, default 0) plants one deliberate mistake in the
 * O(n^3) form so that the tests can show their pins catch it; the library
 * the tests and benchmarks use is always built with 0.
 *   1: a2 is not rotated along with the first rank-one update;
 *   2: p = R w, dropping the -tau v (t^T w) term of F R G;
 *   3: the rotations are not accumulated in Q;
 *   4: the solve uses e1 instead of F e1 as its right-hand side;
 *   5: Q accumulates Omega instead of Omega^T (a transposed rotation). */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

static int orc_nthreads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* x(p), x(p+1) <- [c s; -s c] (x(p), x(p+1)) for rotations r[0..nr) in
 * order, skipping those with p > pmax (they meet only zeros of x). */
static void orc_rot_vec(const orc_rot *r, int nr, double *x, int pmax)
{
    for (int k = 0; k < nr; k++) {
        const int p = r[k].p;
        if (p > pmax) continue;
        const double a = x[p], b = x[p + 1];
        x[p] = r[k].c * a + r[k].s * b;
        x[p + 1] = -r[k].s * a + r[k].c * b;
    }
}

/* X(:, p), X(:, p+1) <- same rotation on columns, rows 0..nr-1: this is
 * X <- X Omega^T for the left rotation Omega, i.e. the accumulation of Q. */
static void orc_rot_cols_list(int nrows, double *X, int ld, const orc_rot *r, int nrot, int nt)
{
    const int CH = 64;
    const int nch = (nrows + CH - 1) / CH;
    #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && nrot > 16)
    for (int ch = 0; ch < nch; ch++) {
        const int r0 = ch * CH, r1 = r0 + CH < nrows ? r0 + CH : nrows;
        for (int k = 0; k < nrot; k++) {
            double *x0 = X + IDX(0, r[k].p, ld), *x1 = X + IDX(0, r[k].p + 1, ld);
            const double c = r[k].c, s = ORC_PLANT == 5 ? -r[k].s : r[k].s;
            for (int i = r0; i < r1; i++) {
                const double a = x0[i], b = x1[i];
                x0[i] = c * a + s * b;
                x1[i] = -s * a + c * b;
            }
        }
    }
}

/* Rotations r[0..nr) in order to the columns c0..c1-1 (at most four) of X,
 * interleaved so that the columns' independent dependency chains overlap.
 * Each column gets exactly the arithmetic of orc_rot_vec. */
static void orc_rot_group(const orc_rot *r, int nr, double *X, int ld, int c0, int c1)
{
    if (c1 - c0 < 4) {
        for (int c = c0; c < c1; c++) orc_rot_vec(r, nr, X + IDX(0, c, ld), 1 << 30);
        return;
    }
    double *x0 = X + IDX(0, c0, ld), *x1 = x0 + ld, *x2 = x1 + ld, *x3 = x2 + ld;
    for (int k = 0; k < nr; k++) {
        const int p = r[k].p;
        const double c = r[k].c, s = r[k].s;
        const double a0 = x0[p], b0 = x0[p + 1], a1 = x1[p], b1 = x1[p + 1];
        const double a2 = x2[p], b2 = x2[p + 1], a3 = x3[p], b3 = x3[p + 1];
        x0[p] = c * a0 + s * b0; x0[p + 1] = -s * a0 + c * b0;
        x1[p] = c * a1 + s * b1; x1[p + 1] = -s * a1 + c * b1;
        x2[p] = c * a2 + s * b2; x2[p + 1] = -s * a2 + c * b2;
        x3[p] = c * a3 + s * b3; x3[p + 1] = -s * a3 + c * b3;
    }
}

/* Columns c0..c1-1 of X (rows in the rotations' frame) <- rotations in
 * order, in groups of four columns. */
static void orc_rot_rows_list(int c0, int c1, double *X, int ld, const orc_rot *r, int nrot,
                              int nt)
{
    const int ng = (c1 - c0 + 3) / 4;
    #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && ng > 8)
    for (int g = 0; g < ng; g++) {
        const int a = c0 + 4 * g, b = a + 4 < c1 ? a + 4 : c1;
        orc_rot_group(r, nrot, X, ld, a, b);
    }
}

/* Rank-one QR update of the upper triangular R (m x m, ld): R + a b^T is
 * brought back to upper triangular form by left rotations, which are
 * appended to rot[] (first the bottom-up ones, then the top-down ones) and
 * also applied to the vector `carry` (may be NULL).  a is destroyed.
 * Returns the number of rotations written (2 (m-1) at most). */
static int orc_qr_rank1(int m, double *R, int ld, double *a, const double *b, double *carry,
                        orc_rot *rot, int nt)
{
    int nr = 0;
    if (m <= 0) return 0;
    /* bottom-up: rotations on (p, p+1), p = m-2..0, turn a into +-||a|| e1 */
    for (int p = m - 2; p >= 0; p--) {
        double c, s;
        orc_givens(a[p], a[p + 1], &c, &s);
        const double ap = a[p], aq = a[p + 1];
        a[p] = c * ap + s * aq;
        a[p + 1] = 0.0;
        rot[nr].p = p; rot[nr].c = c; rot[nr].s = s;
        nr++;
    }
    const int nb = nr;
    /* R <- (rotations) R: column col meets rotations with p <= col; it
     * gains one subdiagonal entry (upper Hessenberg) */
    {
        const int ng = (m + 3) / 4;
        #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && m > 64)
        for (int g = 0; g < ng; g++) {
            /* rotations with p > col come first and meet only the zeros of
             * column col below its diagonal, so a group of columns may
             * start at the first rotation its last column needs */
            const int a = 4 * g, b = a + 4 < m ? a + 4 : m;
            const int k0 = (m - 2) - (b - 1) > 0 ? (m - 2) - (b - 1) : 0;
            orc_rot_group(rot + k0, nb - k0, R, ld, a, b);
        }
    }
    if (carry) orc_rot_vec(rot, nb, carry, 1 << 30);
    /* the rank-one term now lives in the first row */
    for (int col = 0; col < m; col++) R[IDX(0, col, ld)] += a[0] * b[col];
    /* top-down: rotation p zeroes the subdiagonal entry (p+1, p).  Columns
     * are processed in blocks: inside a block serially (each rotation needs
     * its column updated by the previous ones), then the block's rotations
     * go to all later columns at once. */
    const int NBK = 64;
    orc_rot *td = rot + nr;
    for (int c0 = 0; c0 < m - 1; c0 += NBK) {
        const int c1 = c0 + NBK < m - 1 ? c0 + NBK : m - 1;
        for (int col = c0; col < c1; col++) {
            double *x = R + IDX(0, col, ld);
            orc_rot_vec(td + c0, col - c0, x, 1 << 30);
            double c, s;
            orc_givens(x[col], x[col + 1], &c, &s);
            const double xp = x[col], xq = x[col + 1];
            x[col] = c * xp + s * xq;
            x[col + 1] = 0.0;
            td[col].p = col; td[col].c = c; td[col].s = s;
        }
        orc_rot_rows_list(c1, m, R, ld, td + c0, c1 - c0, nt);
    }
    nr += m - 1;
    if (carry) orc_rot_vec(td, m - 1, carry, 1 << 30);
    return nr;
}

/* Upper triangular R (m x m, ld): x = sigma R^{-1} y with 0 < sigma <= 1,
 * column-oriented back substitution that shrinks the partial solution and
 * the remaining right-hand side by 2^-600 whenever the next entry would
 * exceed 2^600 (only the direction of x is used, Lemma 2.1).  y is
 * overwritten. */
static void orc_trsv_scaled(int m, const double *R, int ld, double *y, double *x)
{
    const double big = 0x1.0p600, shrink = 0x1.0p-600;
    for (int i = m - 1; i >= 0; i--) {
        const double d = R[IDX(i, i, ld)];
        while (fabs(y[i]) > big * fabs(d) || fabs(y[i]) > big) {
            for (int t = 0; t <= i; t++) y[t] *= shrink;
            for (int t = i + 1; t < m; t++) x[t] *= shrink;
        }
        x[i] = y[i] / d;
        const double *col = R + IDX(0, i, ld);
        for (int r = 0; r < i; r++) y[r] -= col[r] * x[i];
    }
}

/* Modelled flops of column j of orc_fast_ht (the loops below counted as
 * 2 per multiply-add, 6 per rotation and entry). */
static double orc_fast_col_flops(int n, int j)
{
    const double m = n - j - 1, m2 = m - 1, N = n;
    return 4 * m * m + 4 * N * m          /* F to A, Q */
         + m * m + m * m                  /* t = R^T v, solve */
         + 8 * N * m + 4 * (j + 1.0) * m  /* G to A, Z, B rows 0..j */
         + m * m                          /* p = R w */
         + 12 * m2 * m2                   /* two rank-one QR updates of R22 */
         + 24 * m2 * m + 24 * m2 * N;     /* their rotations to A and Q */
}

double orc_fast_flops(int n, int ncols)
{
    double f = 0.0;
    if (ncols > n - 2) ncols = n - 2;
    for (int j = 0; j < ncols; j++) f += orc_fast_col_flops(n, j);
    return f;
}

/* X(0:nr, 0:m) <- X (I - beta v v^T), rows in parallel chunks (each row's
 * sum in the same order as orc_apply_right). */
static void orc_apply_right_par(int nr, int m, const double *v, double beta, double *X, int ldx,
                                int nt)
{
    if (beta == 0.0 || nr <= 0 || m <= 0) return;
    const int CH = 64;
    const int nch = (nr + CH - 1) / CH;
    #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && nch > 1)
    for (int ch = 0; ch < nch; ch++) {
        const int r0 = ch * CH, r1 = r0 + CH < nr ? r0 + CH : nr;
        double acc[64];
        for (int r = r0; r < r1; r++) acc[r - r0] = 0.0;
        for (int c = 0; c < m; c++) {
            const double *col = X + IDX(0, c, ldx);
            for (int r = r0; r < r1; r++) acc[r - r0] += col[r] * v[c];
        }
        for (int c = 0; c < m; c++) {
            double *col = X + IDX(0, c, ldx);
            const double f = beta * v[c];
            for (int r = r0; r < r1; r++) col[r] -= acc[r - r0] * f;
        }
    }
}

/* Reduces the first `ncols` columns (pass n-2 for the full reduction) with
 * `nthreads` OpenMP threads (0: the runtime's default).  A, B are
 * overwritten by H, T; Q, Z are set.  B must be upper triangular on entry
 * (its strictly lower triangle is ignored and set to zero).  Returns the
 * number of zero pivots replaced by 2 u rho ||B||_F.  `timing` may be
 * NULL, or point to 2 doubles: on entry timing[0] > 0 limits the column
 * loop to that many seconds (it stops after the first column that reaches
 * the limit); on exit timing[0] is the wall time of the column loop alone
 * (without the set-up of Q, Z and ||B||_F) and timing[1] the number of
 * columns reduced. */
int orc_fast_ht(int n, double *A, double *B, double *Q, double *Z, int ncols, uint64_t seed,
                int nthreads, double *timing)
{
    const double u = 0x1.0p-53;
    const int nt = orc_nthreads(nthreads);
    orc_identity(n, Q);
    orc_identity(n, Z);
    for (int c = 0; c < n; c++)
        for (int i = c + 1; i < n; i++) B[IDX(i, c, n)] = 0.0;
    if (ncols > n - 2) ncols = n - 2;
    const double normB = orc_frob(n, B);
    uint64_t draws = 0;
    int perturbed = 0;
    const size_t N = n > 0 ? (size_t)n : 1;
    double *v = (double *)malloc(N * sizeof(double));
    double *w = (double *)malloc(N * sizeof(double));
    double *t = (double *)malloc(N * sizeof(double));
    double *p = (double *)malloc(N * sizeof(double));
    double *y = (double *)malloc(N * sizeof(double));
    double *x = (double *)malloc(N * sizeof(double));
    double *a1 = (double *)malloc(N * sizeof(double));
    double *a2 = (double *)malloc(N * sizeof(double));
    orc_rot *rot = (orc_rot *)malloc(4 * N * sizeof(orc_rot));

    const double limit = timing && timing[0] > 0.0 ? timing[0] : 0.0;
    /* optional progress lines on stderr (long runs): every 512 columns */
    const int progress = getenv("HT_ORACLE_PROGRESS") != NULL;
    struct timespec ts0, ts1;
    clock_gettime(CLOCK_MONOTONIC, &ts0);
    int done = 0;
    for (int j = 0; j < ncols; j++) {
        const int o = j + 1, m = n - j - 1;
        if (progress && j % 512 == 0 && j > 0) {
            clock_gettime(CLOCK_MONOTONIC, &ts1);
            fprintf(stderr, "O-fast n=%d: column %d of %d, %.1f s\n", n, j, ncols,
                    (double)(ts1.tv_sec - ts0.tv_sec) + 1e-9 * (double)(ts1.tv_nsec - ts0.tv_nsec));
            fflush(stderr);
        }
        double *R = B + IDX(o, o, n);
        /* 1. left reflector F on A(j+1:n, j:n), accumulated in Q */
        double tau;
        const double alpha = orc_house(m, A + IDX(o, j, n), v, &tau);
        if (tau != 0.0) {
            #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && m > 64)
            for (int c = j + 1; c < n; c++) {
                double *col = A + IDX(o, c, n);
                double d = 0.0;
                for (int i = 0; i < m; i++) d += v[i] * col[i];
                d *= tau;
                for (int i = 0; i < m; i++) col[i] -= d * v[i];
            }
        }
        A[IDX(o, j, n)] = alpha;
        for (int i = o + 1; i < n; i++) A[IDX(i, j, n)] = 0.0;
        orc_apply_right_par(n, m, v, tau, Q + IDX(0, o, n), n, nt);
        /* t = R^T v */
        #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && m > 64)
        for (int c = 0; c < m; c++) {
            const double *col = R + IDX(0, c, n);
            double d = 0.0;
            for (int i = 0; i <= c; i++) d += col[i] * v[i];
            t[c] = d;
        }
        /* 2. x = sigma R^{-1} (e1 - tau v v(1)); zero pivots first */
        for (int i = 0; i < m; i++)
            if (R[IDX(i, i, n)] == 0.0) {
                R[IDX(i, i, n)] = 2.0 * u * orc_normal(seed, draws++) * normB;
                perturbed++;
            }
        for (int i = 0; i < m; i++) y[i] = ORC_PLANT == 4 ? 0.0 : -tau * v[i] * v[0];
        y[0] += 1.0;
        orc_trsv_scaled(m, R, n, y, x);
        /* 3. right reflector G = House(x) on A(:, j+1:n), Z, B(0:j+1, j+1:n) */
        double gamma;
        orc_house(m, x, w, &gamma);
        orc_apply_right_par(n, m, w, gamma, A + IDX(0, o, n), n, nt);
        orc_apply_right_par(n, m, w, gamma, Z + IDX(0, o, n), n, nt);
        orc_apply_right_par(o, m, w, gamma, B + IDX(0, o, n), n, nt);
        /* 4. F R G = R - tau v t^T - gamma p w^T, p = R w - tau v (t^T w) */
        double tw = 0.0;
        for (int i = 0; i < m; i++) tw += t[i] * w[i];
        {
            const int CH = 64, nch = (m + CH - 1) / CH;
            #pragma omp parallel for num_threads(nt) schedule(static) if (nt > 1 && m > 256)
            for (int ch = 0; ch < nch; ch++) {
                const int r0 = ch * CH, r1 = r0 + CH < m ? r0 + CH : m;
                for (int i = r0; i < r1; i++) p[i] = 0.0;
                for (int c = r0; c < m; c++) {
                    const double *col = R + IDX(0, c, n);
                    const int re = c + 1 < r1 ? c + 1 : r1;
                    for (int i = r0; i < re; i++) p[i] += col[i] * w[c];
                }
                if (ORC_PLANT != 2)
                    for (int i = r0; i < r1; i++) p[i] -= tau * v[i] * tw;
            }
        }
        for (int c = 0; c < m; c++)
            R[IDX(0, c, n)] += -tau * v[0] * t[c] - gamma * p[0] * w[c];
        for (int i = 1; i < m; i++) R[IDX(i, 0, n)] = 0.0;
        /* 5. trailing block R22 + a1 t(2:m)^T + a2 w(2:m)^T back to triangular */
        const int m2 = m - 1;
        if (m2 >= 1) {
            double *R22 = R + IDX(1, 1, n);
            for (int i = 0; i < m2; i++) {
                a1[i] = -tau * v[i + 1];
                a2[i] = -gamma * p[i + 1];
            }
            int nr = orc_qr_rank1(m2, R22, n, a1, t + 1, ORC_PLANT == 1 ? NULL : a2, rot, nt);
            nr += orc_qr_rank1(m2, R22, n, a2, w + 1, NULL, rot + nr, nt);
            /* the rotations (rows j+2..n-1) on A(j+2:n, j+1:n) and Q(:, j+2:n) */
            orc_rot_rows_list(0, m, A + IDX(o + 1, o, n), n, rot, nr, nt);
            if (ORC_PLANT != 3) orc_rot_cols_list(n, Q + IDX(0, o + 1, n), n, rot, nr, nt);
        }
        done = j + 1;
        if (limit > 0.0) {
            clock_gettime(CLOCK_MONOTONIC, &ts1);
            if ((double)(ts1.tv_sec - ts0.tv_sec) + 1e-9 * (double)(ts1.tv_nsec - ts0.tv_nsec) >= limit)
                break;
        }
    }
    clock_gettime(CLOCK_MONOTONIC, &ts1);
    if (timing) {
        timing[0] = (double)(ts1.tv_sec - ts0.tv_sec) + 1e-9 * (double)(ts1.tv_nsec - ts0.tv_nsec);
        timing[1] = (double)done;
    }
    free(v); free(w); free(t); free(p); free(y); free(x);
    free(a1); free(a2); free(rot);
    return perturbed;
}
