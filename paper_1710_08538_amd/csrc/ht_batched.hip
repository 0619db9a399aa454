// ht_batched.hip -- many independent HT reductions of small pencils in one
// persistent launch (the batched form; small pencils of uneven order arise
// e.g. as deflation windows of the QZ algorithm, Sec. 1).
//
// Each pencil (order n <= 512) is reduced by one 256-thread workgroup with
// Algorithm 1: the panel reduction of Sec. 3.2 (column update a, left
// reflector b, factored solve with iterative refinement c, opposite
// reflector and Y column d) over panels of nb columns (nb = 0: one panel over
// all columns), each followed by an absorption in which the accumulated
// block reflectors
//   Q = I - U S U^T,  Z = I - V T V^T  (Sec. 2.4)
// are applied to B, Q, Z and the not yet reduced part of A as dense
// products.  Within one panel B is never modified (Sec. 3.2), so its solves
// use the triangular B the panel started from; after the panel the two-sided
// product (I - U S^T U^T) B (I - V T V^T) is triangular up to rounding in the
// panel's columns (Lemma 2.1), whose strict lower parts are set to zero as
// in Algorithm 2, and full in its trailing block.  That block is brought
// back to triangular form by a blocked Householder QR whose transformations
// also go to A (rows j+1..n-1) and Q; the next panel starts at the next
// column.  When iterative refinement fails for column j (Algorithm 1), the
// column is restored and the panel ends there in the same way.  The banded
// chains of Sec. 3.3 are not used: for n <= 512 and nb = 64 the trailing
// block is a few panels wide, where a dense QR costs about as much.
//
// Dense products run on FP64 matrix cores (v_mfma_f64_16x16x4f64), one
// 32 x 32 output tile per wavefront at a time; matrix-vector products and
// the triangular solve use the vector units with LDS staging.
//
// Scheduling: a one-workgroup kernel sorts the pencils by decreasing order
// (counting sort on n) and resets the work counter; the persistent kernel's
// workgroups then take pencils in that order from an atomic ticket, so the
// largest pencils start first.  Nothing is read back by the host: the two
// launches can be captured in a hipGraph.  Solves are scaled as in the
// single-pencil path (a power-of-two exponent; rescaling by 2^-600 before
// any entry of x exceeds 2^600 times its pivot).
#include "../../include/htred.h"
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l = 16 g + c supplies a = A(c, g) and
// b = B(g, c) and holds D(g + 4 e, c) in register e
__device__ __forceinline__ v4d mfma4(double a, double b, v4d acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

namespace {

constexpr int kBT = 256;  // threads per pencil workgroup
constexpr int kBNW = kBT / 64;
constexpr int kBMax = 512;
constexpr int kStatWords = 8;

struct BatchArgs {
  int batch, nmax, max_ir;
  int nb;               // panel width; 0: one panel over the whole pencil
  int rblock;           // reflectors per block of B's re-triangularisation
  const int32_t* n;
  double* const* A;
  double* const* B;
  double* const* Q;
  double* const* Z;
  const int32_t* ld;
  int32_t* info;
  int* counter;
  int* order;
  int64_t* stats;       // per pencil: kStatWords words (see k_batched)
  double* scratch;      // per workgroup: scratch_stride doubles
  size_t scratch_stride;
  double tol_factor;
  uint64_t seed;
};

// Per-pencil scratch (global memory, leading dimension nmax).
struct BWork {
  double *U, *V, *Y, *S, *T, *P, *P2;
  double *ctil, *ysol, *dsol, *wv, *w2, *rv, *acol, *tk, *tk2;
  int ld;
};

__device__ BWork bwork(double* base, int nmax) {
  BWork w;
  const size_t sq = (size_t)nmax * nmax;
  w.ld = nmax;
  w.U = base;
  w.V = w.U + sq;
  w.Y = w.V + sq;
  w.S = w.Y + sq;
  w.T = w.S + sq;
  w.P = w.T + sq;
  w.P2 = w.P + sq;
  double* v = w.P2 + sq;
  w.ctil = v; v += nmax;
  w.ysol = v; v += nmax;
  w.dsol = v; v += nmax;
  w.wv = v; v += nmax;
  w.w2 = v; v += nmax;
  w.rv = v; v += nmax;
  w.acol = v; v += nmax;
  w.tk = v; v += nmax;
  w.tk2 = v; v += nmax;
  return w;
}

// ---------------------------------------------------------------------------
// Workgroup-level building blocks.  Every one ends with a barrier, so its
// global-memory results are visible to the whole workgroup.
// ---------------------------------------------------------------------------

__device__ __noinline__ void wg_fill(double* x, int m, double v) {
  for (int i = threadIdx.x; i < m; i += kBT) x[i] = v;
  __syncthreads();
}
__device__ __noinline__ void wg_copy(double* y, const double* x, int m) {
  for (int i = threadIdx.x; i < m; i += kBT) y[i] = x[i];
  __syncthreads();
}
__device__ __noinline__ void wg_zero_mat(double* X, int m, int n, int ld) {
  for (int c = 0; c < n; ++c)
    for (int i = threadIdx.x; i < m; i += kBT) X[i + (size_t)c * ld] = 0.0;
  __syncthreads();
}

// LDS staging area of the pencil workgroup: a vector of up to kBMax entries
// and a block that holds either 4 columns of an operand (kBMax x 4) or the
// 64 x 64 diagonal tile of a triangular solve (leading dimension 65).
constexpr int kTileLd = 65;
struct Lds {
  double xs[kBMax];
  double bs[64 * kTileLd];
};

__device__ void stage_vec(double* xs, const double* x, int k, int incx) {
  for (int c = threadIdx.x; c < k; c += kBT) xs[c] = x[(size_t)c * incx];
  __syncthreads();
}

// Dot product of a strided global row segment with an LDS vector, NA
// independent accumulators so that NA loads are in flight at a time (the
// pencil workgroups are latency-bound, not bandwidth-bound).
template <int NA = 16>
__device__ __forceinline__ double row_dot(const double* X, size_t ldx, const double* xs, int c0,
                                          int c1) {
  double s[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) s[u] = 0.0;
  int c = c0;
  for (; c + NA <= c1; c += NA) {
#pragma unroll
    for (int u = 0; u < NA; ++u) s[u] = fma(X[(size_t)(c + u) * ldx], xs[c + u], s[u]);
  }
#pragma unroll
  for (int u = 0; u < NA - 1; ++u)
    if (c + u < c1) s[u] = fma(X[(size_t)(c + u) * ldx], xs[c + u], s[u]);
#pragma unroll
  for (int h = NA / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int u = 0; u < h; ++u) s[u] += s[u + h];
  return s[0];
}

// Sums eight per-lane values over the wavefront in ten exchanges (a
// butterfly that halves the number of values per lane at each of the first
// three stages); lane l receives the total of value (l >> 3) & 7.
__device__ __forceinline__ double wave_sum8(const double (&v)[8]) {
  const int lane = threadIdx.x & 63;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  double a[4], b[2];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    a[j] = (h5 ? v[j + 4] : v[j]) + __shfl_xor(h5 ? v[j] : v[j + 4], 32, 64);
#pragma unroll
  for (int j = 0; j < 2; ++j)
    b[j] = (h4 ? a[j + 2] : a[j]) + __shfl_xor(h4 ? a[j] : a[j + 2], 16, 64);
  double c = (h3 ? b[1] : b[0]) + __shfl_xor(h3 ? b[0] : b[1], 8, 64);
  c += __shfl_xor(c, 4, 64);
  c += __shfl_xor(c, 2, 64);
  c += __shfl_xor(c, 1, 64);
  return c;
}

// y(0:m) = alpha X(0:m, 0:k) x + beta y   (x with stride incx; y distinct
// from X and x)
__device__ __noinline__ void wg_gemv_n(int m, int k, double alpha, const double* X, int ldx, const double* x,
                          int incx, double beta, double* y, Lds& ls) {
  stage_vec(ls.xs, x, k, incx);
  for (int i = threadIdx.x; i < m; i += kBT) {
    const double s = row_dot(X + i, ldx, ls.xs, 0, k);
    y[i] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * y[i]);
  }
  __syncthreads();
}

// z(0:k) = alpha X(0:m, 0:k)^T x + beta z: each wavefront takes eight
// columns at a time (lanes split the rows, two rows per lane in flight) and
// reduces them together with wave_sum8.  upper: X is upper triangular with
// zeros below the diagonal, so column c needs rows 0..c only.
__device__ __noinline__ void wg_gemv_t_core(int m, int k, double alpha, const double* X, int ldx,
                                            double beta, double* z, bool upper, Lds& ls) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c0 = 8 * wv; c0 < k; c0 += 8 * kBNW) {
    const int nc = min(8, k - c0);
    const int mr = upper ? min(m, c0 + 8) : m;
    // columns past the last one repeat it; their sums are not stored
    const double* colq[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) colq[q] = X + (size_t)(c0 + min(q, nc - 1)) * ldx;
    double v[8], u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = u[q] = 0.0;
    int i = lane;
    for (; i + 64 < mr; i += 128) {
      const double x0 = ls.xs[i], x1 = ls.xs[i + 64];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        v[q] = fma(colq[q][i], x0, v[q]);
        u[q] = fma(colq[q][i + 64], x1, u[q]);
      }
    }
    if (i < mr) {
      const double x0 = ls.xs[i];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = fma(colq[q][i], x0, v[q]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] += u[q];
    const double s = wave_sum8(v);
    const int c = c0 + ((lane >> 3) & 7);
    if ((lane & 7) == 0 && c < k) z[c] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * z[c]);
  }
  __syncthreads();
}

__device__ void wg_gemv_t(int m, int k, double alpha, const double* X, int ldx, const double* x,
                          double beta, double* z, Lds& ls) {
  stage_vec(ls.xs, x, m, 1);
  wg_gemv_t_core(m, k, alpha, X, ldx, beta, z, false, ls);
}

// Upper triangular products of the workgroup.  The strictly lower triangles
// of B (zeroed on entry and kept zero), S and T (zeroed at each panel start)
// are exact zeros, so every wavefront starts its rows at the column of its
// first row: all lanes then read the same columns (coalesced), and the few
// zeros below the diagonal add nothing.

// y = alpha op(T) x for upper triangular T (k x k); y distinct from x
__device__ void wg_trmv_small(bool trans, int k, const double* T, int ldt, const double* x,
                              double alpha, double* y, Lds& ls) {
  stage_vec(ls.xs, x, k, 1);
  if (trans) {
    wg_gemv_t_core(k, k, alpha, T, ldt, 0.0, y, true, ls);
    return;
  }
  const int lane = threadIdx.x & 63;
  for (int t = threadIdx.x; t < k; t += kBT) y[t] = alpha * row_dot(T + t, ldt, ls.xs, t - lane, k);
  __syncthreads();
}

// Compact-WY append (Sec. 2.4): T(0:kk, kk) = -tau T(0:kk, 0:kk) z, T(kk, kk) = tau
__device__ __noinline__ void wg_wy_append(double* T, int ldt, int kk, const double* z, double tau, Lds& ls) {
  stage_vec(ls.xs, z, kk, 1);
  const int lane = threadIdx.x & 63;
  for (int t = threadIdx.x; t < kk; t += kBT)
    T[t + (size_t)kk * ldt] = -tau * row_dot(T + t, ldt, ls.xs, t - lane, kk);
  if (threadIdx.x == 0) T[kk + (size_t)kk * ldt] = tau;
  __syncthreads();
}

// Householder reflector of x (length m), LAPACK convention: v[0] = 1,
// (I - tau v v^T) x = beta e1; x overwritten with (beta, 0, ...) if asked.
__device__ __noinline__ void wg_house(int m, double* x, double* v, double& tau, double& beta, bool overwrite,
                         double* sh) {
  const double alpha = x[0];
  double amax = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += kBT) amax = fmax(amax, fabs(x[i]));
  amax = block_max(amax, sh);
  const double sc = safe_scale(fmax(amax, fabs(alpha)));
  double ss = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += kBT) {
    const double t = x[i] * sc;
    ss = fma(t, t, ss);
  }
  ss = block_sum(ss, sh);
  const Refl r = make_refl_ss(alpha * sc, ss);
  const double f = sc * r.scal;
  tau = r.tau;
  beta = r.beta / sc;
  __syncthreads();  // alpha read everywhere before x is overwritten
  for (int i = 1 + threadIdx.x; i < m; i += kBT) {
    v[i] = x[i] * f;
    if (overwrite) x[i] = 0.0;
  }
  if (threadIdx.x == 0) {
    v[0] = 1.0;
    if (overwrite) x[0] = beta;
  }
  __syncthreads();
}

// C(0:m, 0:n) = alpha op(A) op(B) + beta C (C distinct from A, B).
//   op(A): m x k (A or A^T),  op(B): k x n (B or B^T).
// FP64 matrix cores, fragments loaded straight from global memory: each
// wavefront owns 32 x 32 tiles of C and forms their transposes,
//   C^T tile (16 x 16) += op(B)^T fragment (16 x 4) . op(A)^T fragment (4 x 16),
// so that in the accumulator lane 16 g + c holds C(i0 + c, j0 + g + 4 q) in
// register q: the epilogue writes 16 consecutive rows of a column per lane
// group.  Lane (g, c) loads op(A)(i0 + c, l) and op(B)(l, j0 + c) for
// l = l0 + 4 u + g; entries past m, n or k count as zero (their loads are
// clamped to row / column 0 and index k - 1, all in bounds).
__device__ __noinline__ void wg_gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A,
                        int lda, const double* B, int ldb, double beta, double* C, int ldc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int tm = (m + 31) / 32, tn = (n + 31) / 32;
  // op(A)(i, l) = A[i * sai + l * sal],  op(B)(l, j) = B[l * sbl + j * sbj]
  const size_t sai = ta ? (size_t)lda : 1, sal = ta ? 1 : (size_t)lda;
  const size_t sbl = tb ? (size_t)ldb : 1, sbj = tb ? 1 : (size_t)ldb;
  for (int t = wv; t < tm * tn; t += kBT / 64) {
    const int i0 = 32 * (t % tm), j0 = 32 * (t / tm);
    bool ra[2], rb[2];
    const double* pa[2];
    const double* pb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = i0 + 16 * h + c, j = j0 + 16 * h + c;
      ra[h] = i < m;
      rb[h] = j < n;
      pa[h] = A + (ra[h] ? (size_t)i * sai : 0);
      pb[h] = B + (rb[h] ? (size_t)j * sbj : 0);
    }
    v4d acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[r][q] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < k; l0 += 16) {
      double av[4][2], bv[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // loads from a clamped (in-bounds) index, then a select: no branches
        const int l = l0 + 4 * u + g;
        const bool lk = l < k;
        const size_t lc = (size_t)min(l, k - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double x = pa[h][lc * sal], y = pb[h][lc * sbl];
          av[u][h] = (lk && ra[h]) ? x : 0.0;
          bv[u][h] = (lk && rb[h]) ? y : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int q = 0; q < 2; ++q) acc[r][q] = mfma4(bv[u][q], av[u][r], acc[r][q]);
    }
    // acc[r][q] register e: C(i0 + 16 r + c, j0 + 16 q + g + 4 e)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = i0 + 16 * r + c;
      if (i >= m) continue;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = j0 + 16 * q + g + 4 * e;
          if (j < n) {
            double* p = C + i + (size_t)j * ldc;
            *p = (beta == 0.0) ? alpha * acc[r][q][e] : fma(alpha, acc[r][q][e], beta * *p);
          }
        }
    }
  }
  __syncthreads();
}

// y = B(0:m, 0:m) x for upper triangular B (zeros below the diagonal, read
// as in wg_trmv_small); y distinct from x
__device__ __noinline__ void wg_trmv_upper(int m, const double* B, int ldb, const double* x, double* y, Lds& ls) {
  stage_vec(ls.xs, x, m, 1);
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < m; i += kBT) y[i] = row_dot(B + i, ldb, ls.xs, i - lane, m);
  __syncthreads();
}

// Scaled back substitution: B(0:m, 0:m) x = 2^{-E} c, returns E >= 0.
// r (LDS, m doubles) carries the right-hand side and then x; dg (LDS) holds
// one 64 x 64 diagonal tile (leading dimension kTileLd).  Wavefront 0 substitutes a 64-row block; any
// rescaling it needs is then applied to all other entries by everyone.
__device__ __noinline__ int wg_trsv(int m, const double* B, int ldb, const double* c, double* x, double* r,
                       double* dg, int* shi) {
  for (int i = threadIdx.x; i < m; i += kBT) r[i] = c[i];
  int E = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  for (int b = (m + 63) / 64 - 1; b >= 0; --b) {
    const int r0 = 64 * b, nr = min(64, m - r0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // eight loads of a thread in flight before their LDS stores
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int idx = threadIdx.x + (8 * h + q) * kBT, rr = idx & 63, cc = idx >> 6;
        t[q] = (rr < nr && cc < nr && rr <= cc) ? B[(size_t)(r0 + rr) + (size_t)(r0 + cc) * ldb]
                                                 : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int idx = threadIdx.x + (8 * h + q) * kBT;
        dg[(idx & 63) + (idx >> 6) * kTileLd] = t[q];
      }
    }
    __syncthreads();
    if (wv == 0) {
      const bool live = lane < nr;
      double rhs = live ? r[r0 + lane] : 0.0;
      const double d_own = live ? dg[lane * kTileLd + lane] : 1.0;
      const double dp = (d_own != 0.0) ? d_own : 1.0;  // zero pivots only when B = 0
      const double dinv = 1.0 / dp;
      int shr = 0;
#pragma unroll 2
      for (int rr = nr - 1; rr >= 0; --rr) {
        double t = readlane_d(rhs, rr);
        const double dr = readlane_d(dp, rr);
        int g = 0;
        while (!(fabs(t) <= kBig * fabs(dr)) && g < 8) {
          rhs *= kShrink;
          ++shr;
          t = readlane_d(rhs, rr);
          ++g;
        }
        const double xr = t * readlane_d(dinv, rr);
        if (lane == rr) rhs = xr;
        if (lane < rr) rhs = fma(-dg[rr * kTileLd + lane], xr, rhs);
      }
      if (live) r[r0 + lane] = rhs;
      if (lane == 0) shi[0] = shr;
    }
    __syncthreads();
    const int shr = shi[0];
    E += kShrinkExp * shr;
    // rows below the block (already x) take the rescaling; rows above take it
    // and the block's products
    for (int i = r0 + 64 + threadIdx.x; i < m; i += kBT)
      if (shr) r[i] = ldexp(r[i], -kShrinkExp * shr);
    for (int i = threadIdx.x; i < r0; i += kBT) {
      const double acc = shr ? ldexp(r[i], -kShrinkExp * shr) : r[i];
      r[i] = acc - row_dot<8>(B + i + (size_t)r0 * ldb, ldb, r + r0, 0, nr);
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < m; i += kBT) x[i] = r[i];
  __syncthreads();
  return E;
}

// X(rows, cols) -= (X V) T V^T on the column range of the panel's local
// frame: X is rows x L (leading dimension ldx), V L x k, T k x k.
__device__ __noinline__ void wg_right_wy(int rows, int L, int k, double* X, int ldx, const double* V,
                            const double* T, const BWork& w, Lds& ls) {
  if (rows <= 0 || k <= 0) return;
  wg_gemm(false, false, rows, k, L, 1.0, X, ldx, V, w.ld, 0.0, w.P, w.ld);
  wg_gemm(false, false, rows, k, k, 1.0, w.P, w.ld, T, w.ld, 0.0, w.P2, w.ld);
  wg_gemm(false, true, rows, L, k, -1.0, w.P2, w.ld, V, w.ld, 1.0, X, ldx);
}
// X(0:L, cols) -= U S^T (U^T X): X is L x ncols
__device__ __noinline__ void wg_left_wy(int L, int ncols, int k, double* X, int ldx, const double* U,
                           const double* S, const BWork& w, Lds& ls) {
  if (ncols <= 0 || k <= 0) return;
  wg_gemm(true, false, k, ncols, L, 1.0, U, w.ld, X, ldx, 0.0, w.P, w.ld);
  wg_gemm(true, false, k, ncols, k, 1.0, S, w.ld, w.P, w.ld, 0.0, w.P2, w.ld);
  wg_gemm(false, false, L, ncols, k, -1.0, U, w.ld, w.P2, w.ld, 1.0, X, ldx);
}

struct Pencil {
  int n, ld;
  double *A, *B, *Q, *Z;
};

// Factored solve (Sec. 3.2.2 c): ctil <- (I - U S U^T) ctil (nu reflectors),
// B(s+1:n, s+1:n) ysol = 2^{-E} ctil, ysol <- (I - V T^T V^T) ysol (kk).
__device__ __noinline__ int factored_solve(const Pencil& P, const BWork& w, int s, int kk, int nu, double* ctil,
                              double* ysol, double* r, double* dg, int* shi, Lds& ls) {
  const int L = P.n - s - 1;
  wg_gemv_t(L, nu, 1.0, w.U, w.ld, ctil, 0.0, w.tk, ls);
  wg_trmv_small(false, nu, w.S, w.ld, w.tk, 1.0, w.tk2, ls);
  wg_gemv_n(L, nu, -1.0, w.U, w.ld, w.tk2, 1, 1.0, ctil, ls);
  const double* Bp = P.B + (size_t)(s + 1) + (size_t)(s + 1) * P.ld;
  const int E = wg_trsv(L, Bp, P.ld, ctil, ysol, r, dg, shi);
  if (kk > 0) {
    wg_gemv_t(L, kk, 1.0, w.V, w.ld, ysol, 0.0, w.tk, ls);
    wg_trmv_small(true, kk, w.T, w.ld, w.tk, 1.0, w.tk2, ls);
    wg_gemv_n(L, kk, -1.0, w.V, w.ld, w.tk2, 1, 1.0, ysol, ls);
  }
  return E;
}

// Residual of the refined solve (Sec. 3.2.2 c): w = (I - V T V^T)[0; x],
// w = B w, w = (I - U S^T U^T) w, r = 2^{-E} e1 - w(kk:); returns whether
// ||r|| <= tol_factor u ||B||_F ||x||.
__device__ __noinline__ bool residual(const Pencil& P, const BWork& w, int s, int kk, const double* x, int E,
                         double normB, double tol_factor, double* sh, Lds& ls) {
  const int L = P.n - s - 1, m = L - kk;
  for (int i = threadIdx.x; i < L; i += kBT) w.wv[i] = (i < kk) ? 0.0 : x[i - kk];
  __syncthreads();
  wg_gemv_t(m, kk, 1.0, w.V + kk, w.ld, x, 0.0, w.tk, ls);
  wg_trmv_small(false, kk, w.T, w.ld, w.tk, 1.0, w.tk2, ls);
  wg_gemv_n(L, kk, -1.0, w.V, w.ld, w.tk2, 1, 1.0, w.wv, ls);
  const double* Bp = P.B + (size_t)(s + 1) + (size_t)(s + 1) * P.ld;
  wg_trmv_upper(L, Bp, P.ld, w.wv, w.w2, ls);
  wg_gemv_t(L, kk + 1, 1.0, w.U, w.ld, w.w2, 0.0, w.tk, ls);
  wg_trmv_small(true, kk + 1, w.S, w.ld, w.tk, 1.0, w.tk2, ls);
  wg_gemv_n(L, kk + 1, -1.0, w.U, w.ld, w.tk2, 1, 1.0, w.w2, ls);
  double rmax = 0.0, xmax = 0.0;
  for (int i = threadIdx.x; i < m; i += kBT) {
    const double ri = ldexp(i == 0 ? 1.0 : 0.0, -E) - w.w2[kk + i];
    w.rv[i] = ri;
    rmax = fmax(rmax, fabs(ri));
    xmax = fmax(xmax, fabs(x[i]));
  }
  rmax = block_max(rmax, sh);
  xmax = block_max(xmax, sh);
  const double ir = safe_scale(rmax), ix = safe_scale(xmax);
  double rs = 0.0, xs = 0.0;
  for (int i = threadIdx.x; i < m; i += kBT) {
    const double a = w.rv[i] * ir, b = x[i] * ix;
    rs = fma(a, a, rs);
    xs = fma(b, b, xs);
  }
  rs = block_sum(rs, sh);
  xs = block_sum(xs, sh);
  const double rn = sqrt(rs) / ir, xn = sqrt(xs) / ix;
  return rn <= tol_factor * kUnitRoundoff * normB * xn;
}

// Householder QR of B(c0:n, c0:n) (restores a triangular trailing block);
// the reflectors are applied to B(c:n, c+1:n), A(c:n, a0:n) and Q(:, c:n).
// Blocked: rb (1..64) reflectors at a time are formed on their own columns
// and kept in compact WY form I - U S U^T (Sec. 2.4; U, S reuse the panel's
// storage), then applied to the rest of B, to A and to Q as workgroup
// products.
__device__ __noinline__ void retriangularise(const Pencil& P, const BWork& w, int c0, int a0, int rb,
                                             double* sh, Lds& ls) {
  const int n = P.n, ld = P.ld;
  for (int cb = c0; cb < n - 1; cb += rb) {
    const int nbr = min(rb, n - 1 - cb);
    const int m0 = n - cb;  // rows cb..n-1, local row index = global - cb
    wg_zero_mat(w.U, m0, nbr, w.ld);
    wg_zero_mat(w.S, nbr, nbr, w.ld);
    for (int t = 0; t < nbr; ++t) {
      const int col = cb + t, m = n - col;
      double* u = w.U + t + (size_t)t * w.ld;
      double tau, beta;
      wg_house(m, P.B + (size_t)col + (size_t)col * ld, u, tau, beta, true, sh);
      if (t > 0) wg_gemv_t(m, t, 1.0, w.U + t, w.ld, u, 0.0, w.tk, ls);
      wg_wy_append(w.S, w.ld, t, w.tk, tau, ls);
      // the reflector on the block's remaining columns: X -= tau u (X^T u)
      const int nrest = cb + nbr - col - 1;
      if (nrest > 0 && tau != 0.0) {
        double* X = P.B + (size_t)col + (size_t)(col + 1) * ld;
        wg_gemv_t(m, nrest, 1.0, X, ld, u, 0.0, w.tk2, ls);
        for (int cc = 0; cc < nrest; ++cc) {
          const double f = -tau * w.tk2[cc];
          for (int i = threadIdx.x; i < m; i += kBT)
            X[i + (size_t)cc * ld] = fma(f, u[i], X[i + (size_t)cc * ld]);
        }
        __syncthreads();
      }
    }
    // (I - U S U^T)^T on the rest of B and on A's rows, (I - U S U^T) on Q's columns
    if (n - (cb + nbr) > 0)
      wg_left_wy(m0, n - (cb + nbr), nbr, P.B + (size_t)cb + (size_t)(cb + nbr) * ld, ld, w.U,
                 w.S, w, ls);
    wg_left_wy(m0, n - a0, nbr, P.A + (size_t)cb + (size_t)a0 * ld, ld, w.U, w.S, w, ls);
    wg_right_wy(n, m0, nbr, P.Q + (size_t)cb * ld, ld, w.U, w.S, w, ls);
  }
}

// Absorb the k reflector pairs of the panel starting at column s; columns
// s..j-1 (j = s+k) are reduced, columns j..n-1 still carry the pending
// updates.  failed: the panel ended at column j by a refinement failure.
__device__ __noinline__ void absorb_dense(const Pencil& P, const BWork& w, int s, int k, bool failed,
                             Lds& ls) {
  const int n = P.n, ld = P.ld, L = n - s - 1, j = s + k;
  if (k > 0) {
    // A: rows 0..s take the right transformation on columns s+1..n-1; rows
    // s+1.. of the unreduced columns j..n-1 take the column update (a)
    wg_right_wy(s + 1, L, k, P.A + (size_t)(s + 1) * ld, ld, w.V, w.T, w, ls);
    double* Aj = P.A + (size_t)(s + 1) + (size_t)j * ld;
    wg_gemm(false, true, L, n - j, k, -1.0, w.Y, w.ld, w.V + (j - s - 1), w.ld, 1.0, Aj, ld);
    wg_left_wy(L, n - j, k, Aj, ld, w.U, w.S, w, ls);
    // B: (I - U S^T U^T) B (I - V T V^T) on rows/columns s+1..n-1 (rows
    // 0..s only from the right)
    wg_right_wy(n, L, k, P.B + (size_t)(s + 1) * ld, ld, w.V, w.T, w, ls);
    wg_left_wy(L, L, k, P.B + (size_t)(s + 1) + (size_t)(s + 1) * ld, ld, w.U, w.S, w, ls);
    // Q <- Q (I - U S U^T), Z <- Z (I - V T V^T) on columns s+1..n-1
    {
      double* X = P.Q + (size_t)(s + 1) * ld;
      wg_gemm(false, false, n, k, L, 1.0, X, ld, w.U, w.ld, 0.0, w.P, w.ld);
      wg_gemm(false, false, n, k, k, 1.0, w.P, w.ld, w.S, w.ld, 0.0, w.P2, w.ld);
      wg_gemm(false, true, n, L, k, -1.0, w.P2, w.ld, w.U, w.ld, 1.0, X, ld);
    }
    wg_right_wy(n, L, k, P.Z + (size_t)(s + 1) * ld, ld, w.V, w.T, w, ls);
  }
  // reduced columns of B: the entries below the diagonal are rounding noise
  // of the opposite reflectors (Lemma 2.1)
  const int clast = failed ? j : n - 1;
  for (int c = s + 1; c <= clast && c < n; ++c)
    for (int i = c + 1 + threadIdx.x; i < n; i += kBT) P.B[i + (size_t)c * ld] = 0.0;
  __syncthreads();
}

// Counters of one pencil's reduction: panels (absorptions), refinement
// steps, and device-clock ticks spent in the solves, the residuals, the
// absorptions and the re-triangularisations of B (read by thread 0 between
// the helpers' closing barriers).
struct PencilCount {
  int panels, ir;
  int64_t t_solve, t_resid, t_absorb, t_retri;
};

__device__ PencilCount reduce_pencil(const BatchArgs& a, const Pencil& P, const BWork& w, uint64_t seed,
                              double* r, double* dg, int* shi, double* sh, Lds& ls) {
  const int n = P.n, ld = P.ld;
  // Q = Z = I; B's strict lower triangle ignored on entry
  for (int c = 0; c < n; ++c)
    for (int i = threadIdx.x; i < n; i += kBT) {
      P.Q[i + (size_t)c * ld] = (i == c) ? 1.0 : 0.0;
      P.Z[i + (size_t)c * ld] = (i == c) ? 1.0 : 0.0;
      if (i > c) P.B[i + (size_t)c * ld] = 0.0;
    }
  __syncthreads();
  // ||B||_F with a power-of-two scaling
  double bmax = 0.0;
  for (int c = 0; c < n; ++c)
    for (int i = threadIdx.x; i <= c; i += kBT) bmax = fmax(bmax, fabs(P.B[i + (size_t)c * ld]));
  bmax = block_max(bmax, sh);
  const double bsc = safe_scale(bmax);
  double bss = 0.0;
  for (int c = 0; c < n; ++c)
    for (int i = threadIdx.x; i <= c; i += kBT) {
      const double t = P.B[i + (size_t)c * ld] * bsc;
      bss = fma(t, t, bss);
    }
  bss = block_sum(bss, sh);
  const double normB = sqrt(bss) / bsc;
  PencilCount cnt = {0, 0, 0, 0, 0, 0};
  if (n <= 2) return cnt;
  int64_t tc = 0;
  auto tick = [&](int64_t& acc) {
    const int64_t now = (int64_t)wall_clock64();
    acc += now - tc;
    tc = now;
  };

  int s = 0;
  uint64_t panel = 0;
  while (s <= n - 3) {
    const int L = n - s - 1;
    const int kmax = (a.nb > 0) ? min(a.nb, n - 2 - s) : n - 2 - s;
    // zero-diagonal rule (Remark 2.2) for the trailing diagonal
    if (normB > 0.0) {
      for (int i = s + 1 + threadIdx.x; i < n; i += kBT) {
        double* p = P.B + (size_t)i + (size_t)i * ld;
        if (fabs(*p) < 2.2250738585072014e-308) {
          double rho = normal_draw(seed, (panel + 1) * (uint64_t)n + (uint64_t)i);
          if (rho == 0.0) rho = 1.0;
          *p = 2.0 * kUnitRoundoff * rho * normB;
        }
      }
    }
    wg_zero_mat(w.U, L, kmax + 1, w.ld);
    wg_zero_mat(w.V, L, kmax, w.ld);
    wg_zero_mat(w.S, kmax + 1, kmax + 1, w.ld);
    wg_zero_mat(w.T, kmax, kmax, w.ld);
    int k = 0;
    bool failed = false;
    for (int kk = 0; kk < kmax; ++kk) {
      const int j = s + kk;
      double* acol = P.A + (size_t)(s + 1) + (size_t)j * ld;
      wg_copy(w.acol, acol, L);
      // (a) column update with the kk pending pairs
      if (kk > 0) {
        wg_gemv_n(L, kk, -1.0, w.Y, w.ld, w.V + (kk - 1), w.ld, 1.0, acol, ls);
        wg_gemv_t(L, kk, 1.0, w.U, w.ld, acol, 0.0, w.tk, ls);
        wg_trmv_small(true, kk, w.S, w.ld, w.tk, 1.0, w.tk2, ls);
        wg_gemv_n(L, kk, -1.0, w.U, w.ld, w.tk2, 1, 1.0, acol, ls);
      }
      // (b) left reflector, S
      const int m = L - kk;
      double* ucol = w.U + kk + (size_t)kk * w.ld;
      double tau_u, beta_u;
      wg_house(m, acol + kk, ucol, tau_u, beta_u, true, sh);
      if (kk > 0) wg_gemv_t(m, kk, 1.0, w.U + kk, w.ld, ucol, 0.0, w.tk, ls);
      wg_wy_append(w.S, w.ld, kk, w.tk, tau_u, ls);
      // (c) solve, with refinement from the second column on
      wg_fill(w.ctil, L, 0.0);
      if (threadIdx.x == 0) w.ctil[kk] = 1.0;
      __syncthreads();
      tc = (int64_t)wall_clock64();
      int E = factored_solve(P, w, s, kk, kk + 1, w.ctil, w.ysol, r, dg, shi, ls);
      tick(cnt.t_solve);
      double* x = w.ysol + kk;
      bool ok = true;
      if (kk > 0) {
        bool st = residual(P, w, s, kk, x, E, normB, a.tol_factor, sh, ls);
        tick(cnt.t_resid);
        for (int it = 0; !st && it < a.max_ir; ++it) {
          for (int i = threadIdx.x; i < L; i += kBT) w.ctil[i] = (i < kk) ? 0.0 : w.rv[i - kk];
          __syncthreads();
          tc = (int64_t)wall_clock64();
          const int E2 = factored_solve(P, w, s, kk, kk + 1, w.ctil, w.dsol, r, dg, shi, ls);
          tick(cnt.t_solve);
          for (int i = threadIdx.x; i < m; i += kBT) x[i] = ldexp(x[i], -E2) + w.dsol[kk + i];
          __syncthreads();
          E += E2;
          tc = (int64_t)wall_clock64();
          st = residual(P, w, s, kk, x, E, normB, a.tol_factor, sh, ls);
          tick(cnt.t_resid);
          ++cnt.ir;
        }
        ok = st;
      }
      if (!ok) {
        wg_copy(acol, w.acol, L);  // undo (a) and (b) on column j
        failed = true;
        break;
      }
      // (d) opposite reflector, T, Y column
      double* vcol = w.V + kk + (size_t)kk * w.ld;
      double tau_v, beta_v;
      wg_house(m, x, vcol, tau_v, beta_v, false, sh);
      if (kk > 0) wg_gemv_t(m, kk, 1.0, w.V + kk, w.ld, vcol, 0.0, w.tk, ls);
      wg_wy_append(w.T, w.ld, kk, w.tk, tau_v, ls);
      double* ycol = w.Y + (size_t)kk * w.ld;
      wg_gemv_n(L, m, 1.0, P.A + (size_t)(s + 1) + (size_t)(j + 1) * ld, ld, vcol, 1, 0.0, ycol, ls);
      if (kk > 0) wg_gemv_n(L, kk, -1.0, w.Y, w.ld, w.tk, 1, 1.0, ycol, ls);
      for (int i = threadIdx.x; i < L; i += kBT) ycol[i] *= tau_v;
      __syncthreads();
      k = kk + 1;
    }
    tc = (int64_t)wall_clock64();
    // a panel that ends before the last column (refinement failure or the
    // panel width) leaves B's trailing block to be re-triangularised
    const bool retri = failed || s + k < n - 2;
    absorb_dense(P, w, s, k, retri, ls);
    tick(cnt.t_absorb);
    if (retri) {
      retriangularise(P, w, s + k + 1, s + k, a.rblock, sh, ls);
      tick(cnt.t_retri);
    }
    s += k;
    ++panel;
  }
  cnt.panels = (int)panel;
  return cnt;
}

// Counting sort of the pencils by decreasing order; resets the ticket.
__global__ __launch_bounds__(1024) void k_batched_order(BatchArgs a) {
  __shared__ int cnt[kBMax + 2];
  for (int i = threadIdx.x; i < kBMax + 2; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  auto bin = [&](int i) {
    const int nn = min(max(a.n[i], 0), kBMax + 1);
    return kBMax + 1 - nn;
  };
  for (int i = threadIdx.x; i < a.batch; i += blockDim.x) atomicAdd(&cnt[bin(i)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int b = 0; b < kBMax + 2; ++b) {
      const int c = cnt[b];
      cnt[b] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.batch; i += blockDim.x) a.order[atomicAdd(&cnt[bin(i)], 1)] = i;
  if (threadIdx.x == 0) a.counter[0] = 0;
}

// Three workgroups per CU: the helpers above are kept out of line so that
// each is register-allocated on its own (no spills inside their loops).
__global__ __launch_bounds__(kBT, 3) void k_batched(BatchArgs a) {
  __shared__ double r[kBMax];
  __shared__ double sh[kBNW];
  __shared__ int shi[2];
  __shared__ Lds ls;
  double* dg = ls.bs;  // the solve's diagonal tile shares the operand block
  const BWork w = bwork(a.scratch + (size_t)blockIdx.x * a.scratch_stride, a.nmax);
  for (;;) {
    if (threadIdx.x == 0) shi[1] = atomicAdd(a.counter, 1);
    __syncthreads();
    const int t = shi[1];
    __syncthreads();
    if (t >= a.batch) break;
    const int pi = a.order[t];
    Pencil P;
    P.n = a.n[pi];
    P.ld = a.ld[pi];
    P.A = a.A[pi];
    P.B = a.B[pi];
    P.Q = a.Q[pi];
    P.Z = a.Z[pi];
    const int64_t t0 = (int64_t)wall_clock64();
    int info = 0;
    PencilCount cnt = {0, 0, 0, 0, 0, 0};
    if (P.n < 0 || P.n > a.nmax || P.ld < max(1, P.n) ||
        (P.n > 0 && (!P.A || !P.B || !P.Q || !P.Z)))
      info = -1;
    else
      cnt = reduce_pencil(a, P, w, a.seed ^ splitmix64((uint64_t)pi + 1), r, dg, shi, sh, ls);
    __syncthreads();
    if (threadIdx.x == 0) {
      a.info[pi] = info;
      int64_t* st = a.stats + kStatWords * (size_t)pi;
      st[0] = t0;
      st[1] = (int64_t)wall_clock64();
      st[2] = cnt.panels;
      st[3] = cnt.ir;
      st[4] = cnt.t_solve;
      st[5] = cnt.t_resid;
      st[6] = cnt.t_absorb;
      st[7] = cnt.t_retri;
    }
    __syncthreads();
  }
}

// resident workgroups: wg_per_cu (<= 3, the occupancy k_batched is built
// for) per compute unit, no more than there are pencils
size_t batch_grid(int batch, int wg_per_cu) {
  return (size_t)std::max(1, std::min(batch, wg_per_cu * num_cus()));
}
size_t batch_stride(int nmax) {
  const size_t d = 7 * (size_t)nmax * nmax + 9 * (size_t)nmax;
  return (d * 8 + 255) / 256 * 32;  // doubles, rounded to 256 bytes
}

size_t order_bytes(int batch) { return ((size_t)batch * 4 + 255) / 256 * 256; }
size_t stats_bytes(int batch) { return ((size_t)batch * kStatWords * 8 + 255) / 256 * 256; }

}  // namespace

size_t batched_workspace_bytes(int batch, int nmax, int wg_per_cu) {
  if (batch <= 0) return 256;
  return 256 + order_bytes(batch) + stats_bytes(batch) +
         batch_grid(batch, wg_per_cu) * batch_stride(nmax) * 8;
}

const int64_t* batched_stats_ptr(const void* workspace, int batch) {
  return (const int64_t*)((const char*)workspace + 256 + order_bytes(batch));
}

int batched_reduce(hipStream_t st, int batch, const int32_t* n_dev, double* const* A_dev,
                   double* const* B_dev, double* const* Q_dev, double* const* Z_dev,
                   const int32_t* ld_dev, int32_t* info_dev, int nmax, int nb, int rblock,
                   int wg_per_cu, int max_ir, double tol_factor, uint64_t seed, void* workspace) {
  if (batch <= 0) return 0;
  char* base = (char*)workspace;
  BatchArgs a;
  a.batch = batch;
  a.nmax = std::max(nmax, 1);
  a.max_ir = max_ir;
  a.nb = nb;
  a.rblock = std::min(std::max(rblock, 1), 64);
  a.n = n_dev;
  a.A = A_dev;
  a.B = B_dev;
  a.Q = Q_dev;
  a.Z = Z_dev;
  a.ld = ld_dev;
  a.info = info_dev;
  a.counter = (int*)base;
  a.order = (int*)(base + 256);
  a.stats = (int64_t*)(base + 256 + order_bytes(batch));
  a.scratch = (double*)(base + 256 + order_bytes(batch) + stats_bytes(batch));
  a.scratch_stride = batch_stride(a.nmax);
  a.tol_factor = tol_factor;
  a.seed = seed;
  hipLaunchKernelGGL(k_batched_order, dim3(1), dim3(1024), 0, st, a);
  const int wpc = std::min(std::max(wg_per_cu, 1), 3);
  hipLaunchKernelGGL(k_batched, dim3((unsigned)batch_grid(batch, wpc)), dim3(kBT), 0, st, a);
  return 0;
}

}  // namespace htk
