// ht_blas.hip -- dense FP64 building blocks (GEMM, GEMV, TRMV, norms, copies)
// used by the HouseHT driver.  All kernels are deterministic (fixed
// reduction order, no floating-point atomics).
#include <algorithm>

#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// GEMM on the FP64 matrix cores: C = alpha op(A) op(B) + beta C.
// A 256-thread workgroup computes a 64 x 64 tile of C; wavefront w owns the
// 32 x 32 quarter (rows 32 (w & 1), columns 32 (w >> 1)) as 2 x 2 tiles of
// v_mfma_f64_16x16x4f64.  The kernel forms the transposed tile
// C^T = op(B)^T op(A)^T, whose accumulator layout (lane 16 g + c, register
// i <-> row g + 4 i, column c of the 16 x 16 result) puts 16 consecutive
// rows of one column of C in each lane group, so the stores are 128-byte
// runs of the column-major C.  The contraction runs in chunks of 16: the
// next chunk's op(A) (64 x 16) and op(B) (16 x 64) are loaded into
// registers while the current chunk's MFMAs run from LDS, then stored to the
// other LDS buffer (one barrier per chunk).  Out-of-range rows, columns and
// contraction indices are staged as zeros.
//
// Split contraction: with gridDim.z = S > 1, slice z covers contraction
// indices [z kc, min(k, (z + 1) kc)) and writes its raw sums to
// part[z m n + j m + i]; k_gemm_reduce then adds the S slices in order and
// applies alpha and beta, so results do not depend on timing.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_mgemm(int m, int n, int k, int kc, double alpha,
                                               const double* __restrict__ A, int lda,
                                               const double* __restrict__ B, int ldb,
                                               double beta, double* __restrict__ C, int ldc,
                                               double* __restrict__ part) {
  __shared__ double As[2][16][65];  // As[buf][kk][i] = op(A)(i0 + i, k0 + kk); padded rows
  __shared__ double Bs[2][16][65];  // Bs[buf][kk][j] = op(B)(k0 + kk, j0 + j)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int kb = blockIdx.z * kc, ke = min(k, kb + kc);
  const int wm = 32 * (wave & 1), wn = 32 * (wave >> 1);

  // staging assignment: 1024 elements of each operand chunk, 4 per thread;
  // the fast index follows the operand's contiguous dimension
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int i, kk;
      if (!TA) { i = e & 63; kk = e >> 6; } else { kk = e & 15; i = e >> 4; }
      const int gi = i0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < ke)
        v = TA ? A[(size_t)gk + (size_t)gi * lda] : A[(size_t)gi + (size_t)gk * lda];
      ra[r] = v;
      int j;
      if (!TB) { kk = e & 15; j = e >> 4; } else { j = e & 63; kk = e >> 6; }
      const int gj = j0 + j, gk2 = k0 + kk;
      v = 0.0;
      if (gj < n && gk2 < ke)
        v = TB ? B[(size_t)gj + (size_t)gk2 * ldb] : B[(size_t)gk2 + (size_t)gj * ldb];
      rb[r] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      if (!TA) As[buf][e >> 6][e & 63] = ra[r];
      else As[buf][e & 15][e >> 4] = ra[r];
      if (!TB) Bs[buf][e & 15][e >> 4] = rb[r];
      else Bs[buf][e >> 6][e & 63] = rb[r];
    }
  };

  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

  if (kb < ke) {
    load(kb);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += 16) {
      const bool more = k0 + 16 < ke;
      if (more) load(k0 + 16);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 4 * q + g;
        // MFMA A operand: op(B)^T rows (columns of C), B operand: op(A)^T
        const double b0 = Bs[buf][kk][wn + c], b1 = Bs[buf][kk][wn + 16 + c];
        const double a0 = As[buf][kk][wm + c], a1 = As[buf][kk][wm + 16 + c];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc[1][1], 0, 0, 0);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // acc[y][x][r]: C(i0 + wm + 16 x + c, j0 + wn + 16 y + g + 4 r)
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int i = i0 + wm + 16 * x + c;
    if (i >= m) continue;
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + wn + 16 * y + g + 4 * r;
        if (j >= n) continue;
        if (part) {
          part[(size_t)blockIdx.z * m * n + (size_t)j * m + i] = acc[y][x][r];
        } else {
          double* p = C + (size_t)i + (size_t)j * ldc;
          *p = (beta == 0.0) ? alpha * acc[y][x][r] : fma(alpha, acc[y][x][r], beta * *p);
        }
      }
  }
}

__global__ void k_gemm_reduce(int m, int n, int S, double alpha, const double* __restrict__ part,
                              double beta, double* __restrict__ C, int ldc) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  double s = 0.0;
  for (int z = 0; z < S; ++z) s += part[(size_t)z * m * n + e];
  double* p = C + (size_t)i + (size_t)j * ldc;
  *p = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * *p);
}

template <bool TA, bool TB>
static void launch_mgemm(hipStream_t st, dim3 grid, int m, int n, int k, int kc, double alpha,
                         const double* A, int lda, const double* B, int ldb, double beta,
                         double* C, int ldc, double* part) {
  hipLaunchKernelGGL((k_mgemm<TA, TB>), grid, dim3(256), 0, st, m, n, k, kc, alpha, A, lda, B,
                     ldb, beta, C, ldc, part);
}

void gemm_ws(hipStream_t st, bool transA, bool transB, int m, int n, int k, double alpha,
             const double* A, int lda, const double* B, int ldb, double beta, double* C,
             int ldc, double* part, size_t part_doubles) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0 && beta == 1.0) return;
  const int kk = std::max(k, 0);
  const int tiles = (int)(cdiv(m, 64) * cdiv(n, 64));
  // split a long contraction over few output tiles (at least 512 indices
  // per slice, at most what the partial-sum area holds)
  int S = 1, kc = std::max(kk, 1);
  if (part && tiles < 128 && kk >= 1024) {
    const size_t cap = part_doubles / ((size_t)m * n);
    S = (int)std::min<size_t>(cap, (size_t)std::min(256 / tiles, kk / 512));
    if (S > 1) {
      kc = (int)((cdiv(kk, S) + 15) / 16 * 16);
      S = (int)cdiv(kk, kc);
    }
    if (S < 2) { S = 1; kc = std::max(kk, 1); }
  }
  dim3 grid(cdiv(m, 64), cdiv(n, 64), S);
  double* pp = S > 1 ? part : nullptr;
  if (!transA && !transB) launch_mgemm<false, false>(st, grid, m, n, kk, kc, alpha, A, lda, B, ldb, beta, C, ldc, pp);
  else if (transA && !transB) launch_mgemm<true, false>(st, grid, m, n, kk, kc, alpha, A, lda, B, ldb, beta, C, ldc, pp);
  else if (!transA && transB) launch_mgemm<false, true>(st, grid, m, n, kk, kc, alpha, A, lda, B, ldb, beta, C, ldc, pp);
  else launch_mgemm<true, true>(st, grid, m, n, kk, kc, alpha, A, lda, B, ldb, beta, C, ldc, pp);
  if (S > 1)
    hipLaunchKernelGGL(k_gemm_reduce, dim3(cdiv((long)m * n, 256)), dim3(256), 0, st, m, n, S,
                       alpha, part, beta, C, ldc);
}

void gemm(hipStream_t st, bool transA, bool transB, int m, int n, int k, double alpha,
          const double* A, int lda, const double* B, int ldb, double beta, double* C,
          int ldc) {
  gemm_ws(st, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, 0);
}

// ---------------------------------------------------------------------------
// GEMV y = alpha X x + beta y and TRMV y = B x (B upper triangular).
// Small k: one thread per row, one launch.  Large k: 64-row x KC-column
// blocks (each wave a quarter of the columns, lanes = consecutive rows, so a
// wave reads 512 contiguous bytes per column); partial sums per column chunk
// are added in chunk order by a second kernel (deterministic).
// ---------------------------------------------------------------------------
constexpr int KC = 512;
constexpr int kSmallK = 256;

__global__ __launch_bounds__(256) void k_gemv_n_small(int m, int k, double alpha,
                                                      const double* __restrict__ X, int ldx,
                                                      const double* __restrict__ x, int incx,
                                                      double beta, double* y,
                                                      const double* __restrict__ post) {
  __shared__ double xs[kSmallK];
  for (int t = threadIdx.x; t < k; t += 256) xs[t] = x[(size_t)t * incx];
  __syncthreads();
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= m) return;
  const double* p = X + row;
  // sixteen loads in flight per lane, four partial sums
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = 0;
  for (; c + 16 <= k; c += 16) {
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = p[(size_t)(c + u) * ldx];
#pragma unroll
    for (int u = 0; u < 16; u += 4) {
      s0 = fma(a[u], xs[c + u], s0);
      s1 = fma(a[u + 1], xs[c + u + 1], s1);
      s2 = fma(a[u + 2], xs[c + u + 2], s2);
      s3 = fma(a[u + 3], xs[c + u + 3], s3);
    }
  }
  for (; c < k; ++c) s0 = fma(p[(size_t)c * ldx], xs[c], s0);
  const double s = (s0 + s1) + (s2 + s3);
  const double v = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * y[row]);
  y[row] = post ? v * post[0] : v;
}

template <bool TRI>
__global__ __launch_bounds__(256) void k_gemv_part(int m, int k, const double* __restrict__ X,
                                                   int ldx, const double* __restrict__ x, int incx,
                                                   double* __restrict__ part) {
  __shared__ double xs[KC];
  __shared__ double red[4][64];
  const int row0 = blockIdx.x * 64;
  const int c0 = blockIdx.y * KC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = row0 + lane;
  if (TRI && c0 + KC <= row0) {  // chunk entirely below the diagonal
    if (wave == 0 && row < m) part[(size_t)blockIdx.y * m + row] = 0.0;
    return;
  }
  const int kc = min(KC, k - c0);
  for (int t = threadIdx.x; t < kc; t += 256) xs[t] = x[(size_t)(c0 + t) * incx];
  __syncthreads();
  constexpr int CW = KC / 4;
  int cs = wave * CW, ce = min(kc, cs + CW);
  if (TRI) cs = max(cs, row - c0);
  // sixteen loads in flight per lane (four partial sums), so that a wave
  // keeps enough bytes outstanding to stream X at the HBM rate
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (row < m) {
    const double* p = X + (size_t)row + (size_t)c0 * ldx;
    int c = cs;
    for (; c + 16 <= ce; c += 16) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = p[(size_t)(c + u) * ldx];
#pragma unroll
      for (int u = 0; u < 16; u += 4) {
        s0 = fma(a[u], xs[c + u], s0);
        s1 = fma(a[u + 1], xs[c + u + 1], s1);
        s2 = fma(a[u + 2], xs[c + u + 2], s2);
        s3 = fma(a[u + 3], xs[c + u + 3], s3);
      }
    }
    for (; c < ce; ++c) s0 = fma(p[(size_t)c * ldx], xs[c], s0);
  }
  red[wave][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (wave == 0 && row < m)
    part[(size_t)blockIdx.y * m + row] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ __launch_bounds__(256) void k_gemv_n_fin(int m, int nch, const double* __restrict__ part,
                                                    double alpha, double beta, double* y) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= m) return;
  // chunk order as a plain loop, eight loads in flight
  double s = 0.0;
  int c = 0;
  for (; c + 8 <= nch; c += 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = part[(size_t)(c + u) * m + row];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += a[u];
  }
  for (; c < nch; ++c) s += part[(size_t)c * m + row];
  y[row] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * y[row]);
}

void gemv_n(hipStream_t st, int m, int k, double alpha, const double* X, int ldx,
            const double* x, int incx, double beta, double* y, double* partials) {
  if (m <= 0) return;
  if (k <= kSmallK) {
    hipLaunchKernelGGL(k_gemv_n_small, dim3(cdiv(m, 256)), dim3(256), 0, st, m, k, alpha, X, ldx,
                       x, incx, beta, y, (const double*)nullptr);
    return;
  }
  const int nch = cdiv(k, KC);
  hipLaunchKernelGGL(k_gemv_part<false>, dim3(cdiv(m, 64), nch), dim3(256), 0, st, m, k, X, ldx,
                     x, incx, partials);
  hipLaunchKernelGGL(k_gemv_n_fin, dim3(cdiv(m, 256)), dim3(256), 0, st, m, nch, partials, alpha,
                     beta, y);
}

void gemv_n_small_scaled(hipStream_t st, int m, int k, double alpha, const double* X, int ldx,
                         const double* x, double beta, double* y, const double* post) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_gemv_n_small, dim3(cdiv(m, 256)), dim3(256), 0, st, m, k, alpha, X, ldx,
                     x, 1, beta, y, post);
}

void trmv_upper(hipStream_t st, int m, const double* B, int ldb, const double* x, double* y,
                double* partials) {
  if (m <= 0) return;
  const int nch = cdiv(m, KC);
  hipLaunchKernelGGL(k_gemv_part<true>, dim3(cdiv(m, 64), nch), dim3(256), 0, st, m, m, B, ldb,
                     x, 1, partials);
  hipLaunchKernelGGL(k_gemv_n_fin, dim3(cdiv(m, 256)), dim3(256), 0, st, m, nch, partials, 1.0,
                     0.0, y);
}

// ---------------------------------------------------------------------------
// GEMV^T z = alpha X^T x + beta z: workgroup (column c, row chunk); with one
// chunk the result is written directly.
// ---------------------------------------------------------------------------
constexpr int RC = 4096;

__global__ __launch_bounds__(256) void k_gemv_t_part(int m, int k, const double* __restrict__ X,
                                                     int ldx, const double* __restrict__ x,
                                                     double* __restrict__ part, int direct,
                                                     double alpha, double beta, double* z) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int r1 = min(m, r0 + RC);
  const double* p = X + (size_t)c * ldx;
  // four rows per thread in flight, four partial sums
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int r = r0 + threadIdx.x;
  for (; r + 768 < r1; r += 1024) {
    const double a0 = p[r], a1 = p[r + 256], a2 = p[r + 512], a3 = p[r + 768];
    const double b0 = x[r], b1 = x[r + 256], b2 = x[r + 512], b3 = x[r + 768];
    s0 = fma(a0, b0, s0);
    s1 = fma(a1, b1, s1);
    s2 = fma(a2, b2, s2);
    s3 = fma(a3, b3, s3);
  }
  for (; r < r1; r += 256) s0 = fma(p[r], x[r], s0);
  double s = block_sum((s0 + s1) + (s2 + s3), sh);
  if (threadIdx.x == 0) {
    if (direct) z[c] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * z[c]);
    else part[(size_t)blockIdx.y * k + c] = s;
  }
}

__global__ void k_gemv_t_fin(int k, int nch, const double* __restrict__ part, double alpha,
                             double beta, double* z) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int i = 0; i < nch; ++i) s += part[(size_t)i * k + c];
  z[c] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * z[c]);
}

void gemv_t(hipStream_t st, int m, int k, double alpha, const double* X, int ldx,
            const double* x, double beta, double* z, double* partials) {
  if (k <= 0) return;
  const int nch = m > 0 ? cdiv(m, RC) : 0;
  if (nch == 1) {
    hipLaunchKernelGGL(k_gemv_t_part, dim3(k, 1), dim3(256), 0, st, m, k, X, ldx, x, partials, 1,
                       alpha, beta, z);
    return;
  }
  if (nch > 0)
    hipLaunchKernelGGL(k_gemv_t_part, dim3(k, nch), dim3(256), 0, st, m, k, X, ldx, x, partials,
                       0, alpha, beta, z);
  hipLaunchKernelGGL(k_gemv_t_fin, dim3(cdiv(k, 128)), dim3(128), 0, st, k, nch, partials, alpha,
                     beta, z);
}

// ---------------------------------------------------------------------------
// Block-reflector application to one vector, the step that the panel of
// Sec. 3.2.2 repeats for every column (the column update, the factored
// solve's two factors and the residual's two factors):
//   xu(0:mu) += alpha U(0:mu, 0:k) op(S) (U(d0:d0+md, 0:k)^T xd)
// in two launches: the column sums U^T xd (k_gemv_t_part, partial sums per
// chunk of rows), then k_wy_apply, whose every workgroup adds the partial
// sums in chunk order, multiplies by the k x k triangular op(S) and updates
// its 256 rows of xu.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wy_apply(int mu, int k, int nch,
                                                  const double* __restrict__ part,
                                                  const double* __restrict__ zrow, int ldz,
                                                  const double* __restrict__ S, int lds,
                                                  int transS, double alpha,
                                                  const double* __restrict__ U, int ldu,
                                                  const double* __restrict__ xin, int xoff,
                                                  int unit, double* __restrict__ xu) {
  __shared__ double zs[128], ys[128];
  const int t = threadIdx.x;
  if (t < k) {
    double s = 0.0;
    if (zrow) {
      s = zrow[(size_t)t * ldz];  // U^T e_unit: row `unit` of U
    } else {
      for (int c = 0; c < nch; ++c) s += part[(size_t)c * k + t];
    }
    zs[t] = s;
  }
  __syncthreads();
  if (t < k)
    ys[t] = transS ? dot_in_order(S + (size_t)t * lds, 1, zs, 0, t + 1)
                   : dot_in_order(S + t, (size_t)lds, zs, t, k);
  __syncthreads();
  const int row = blockIdx.x * 256 + t;
  if (row >= mu) return;
  const double* p = U + row;
  // sixteen loads in flight per lane, four partial sums
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = 0;
  for (; c + 16 <= k; c += 16) {
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = p[(size_t)(c + u) * ldu];
#pragma unroll
    for (int u = 0; u < 16; u += 4) {
      s0 = fma(a[u], ys[c + u], s0);
      s1 = fma(a[u + 1], ys[c + u + 1], s1);
      s2 = fma(a[u + 2], ys[c + u + 2], s2);
      s3 = fma(a[u + 3], ys[c + u + 3], s3);
    }
  }
  for (; c < k; ++c) s0 = fma(p[(size_t)c * ldu], ys[c], s0);
  // the vector being updated: in place, the unit vector e_unit, or [0; xin]
  const double base = (unit >= 0) ? (row == unit ? 1.0 : 0.0)
                      : (xin ? (row < xoff ? 0.0 : xin[row - xoff]) : xu[row]);
  xu[row] = fma(alpha, (s0 + s1) + (s2 + s3), base);
}

static void wy_apply_impl(hipStream_t st, int mu, int md, int d0, int k, double alpha,
                          const double* U, int ldu, const double* S, int lds, bool transS,
                          const double* xd, double* xu, double* z, double* partials,
                          const double* xin, int xoff) {
  if (k <= 0 || mu <= 0) return;
  const int nch = md > 0 ? cdiv(md, RC) : 0;
  const double* src = partials;
  if (nch == 1) {
    hipLaunchKernelGGL(k_gemv_t_part, dim3(k, 1), dim3(256), 0, st, md, k, U + d0, ldu, xd,
                       partials, 1, 1.0, 0.0, z);
    src = z;
  } else if (nch > 1) {
    hipLaunchKernelGGL(k_gemv_t_part, dim3(k, nch), dim3(256), 0, st, md, k, U + d0, ldu, xd,
                       partials, 0, 1.0, 0.0, z);
  }
  hipLaunchKernelGGL(k_wy_apply, dim3(cdiv(mu, 256)), dim3(256), 0, st, mu, k, nch, src,
                     (const double*)nullptr, 0, S, lds, transS ? 1 : 0, alpha, U, ldu, xin, xoff,
                     -1, xu);
}

void wy_apply(hipStream_t st, int mu, int md, int d0, int k, double alpha, const double* U,
              int ldu, const double* S, int lds, bool transS, const double* xd, double* xu,
              double* z, double* partials) {
  wy_apply_impl(st, mu, md, d0, k, alpha, U, ldu, S, lds, transS, xd, xu, z, partials, nullptr,
                0);
}

void wy_apply_padded(hipStream_t st, int mu, int md, int d0, int k, double alpha,
                     const double* U, int ldu, const double* S, int lds, bool transS,
                     const double* xd, double* xu, double* z, double* partials) {
  if (k <= 0) {
    pad_copy(st, xu, d0, xd, mu - d0);
    return;
  }
  wy_apply_impl(st, mu, md, d0, k, alpha, U, ldu, S, lds, transS, xd, xu, z, partials, xd, d0);
}

void wy_apply_unit(hipStream_t st, int mu, int idx, int k, double alpha, const double* U,
                   int ldu, const double* S, int lds, bool transS, double* xu) {
  if (mu <= 0) return;
  if (k <= 0) {
    unit_vec(st, xu, mu, idx);
    return;
  }
  hipLaunchKernelGGL(k_wy_apply, dim3(cdiv(mu, 256)), dim3(256), 0, st, mu, k, 0,
                     (const double*)nullptr, U + idx, ldu, S, lds, transS ? 1 : 0, alpha, U, ldu,
                     (const double*)nullptr, 0, idx, xu);
}

// ---------------------------------------------------------------------------
// Elementwise helpers.
// ---------------------------------------------------------------------------
__global__ void k_fill(double* x, int m, double v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = v;
}
void fill(hipStream_t st, double* x, int m, double v) {
  if (m > 0) hipLaunchKernelGGL(k_fill, dim3(cdiv(m, 256)), dim3(256), 0, st, x, m, v);
}

// x(0:m) = e_idx (idx in 0..m-1)
__global__ void k_unit(double* x, int m, int idx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = (i == idx) ? 1.0 : 0.0;
}
void unit_vec(hipStream_t st, double* x, int m, int idx) {
  if (m > 0) hipLaunchKernelGGL(k_unit, dim3(cdiv(m, 256)), dim3(256), 0, st, x, m, idx);
}

// x(0:z) = 0, x(z:z+m) = src(0:m)
__global__ void k_pad_copy(double* x, int z, const double* src, int m) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < z) x[i] = 0.0;
  else if (i < z + m) x[i] = src[i - z];
}
void pad_copy(hipStream_t st, double* x, int z, const double* src, int m) {
  if (z + m > 0)
    hipLaunchKernelGGL(k_pad_copy, dim3(cdiv(z + m, 256)), dim3(256), 0, st, x, z, src, m);
}

__global__ void k_copy(double* d, const double* s, int m) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) d[i] = s[i];
}
void copy(hipStream_t st, double* dst, const double* src, int m) {
  if (m > 0) hipLaunchKernelGGL(k_copy, dim3(cdiv(m, 256)), dim3(256), 0, st, dst, src, m);
}

__global__ void k_copy_mat(int m, int n, const double* s, int lds, double* d, int ldd) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < m && j < n) d[(size_t)i + (size_t)j * ldd] = s[(size_t)i + (size_t)j * lds];
}
void copy_mat(hipStream_t st, int m, int n, const double* src, int lds, double* dst, int ldd) {
  if (m > 0 && n > 0)
    hipLaunchKernelGGL(k_copy_mat, dim3(cdiv(m, 256), n), dim3(256), 0, st, m, n, src, lds, dst, ldd);
}

__global__ void k_set_identity(double* X, int n, int ld) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < n) X[(size_t)i + (size_t)j * ld] = (i == j) ? 1.0 : 0.0;
}
void set_identity(hipStream_t st, double* X, int n, int ld) {
  if (n > 0) hipLaunchKernelGGL(k_set_identity, dim3(cdiv(n, 256), n), dim3(256), 0, st, X, n, ld);
}

// zero entries with row > col + offset (offset 0: strictly lower; 1: below
// the first subdiagonal)
__global__ void k_zero_lower(double* X, int n, int ld, int offset) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < n && i > j + offset) X[(size_t)i + (size_t)j * ld] = 0.0;
}
void zero_lower(hipStream_t st, double* X, int n, int ld, int offset) {
  if (n > 0) hipLaunchKernelGGL(k_zero_lower, dim3(cdiv(n, 256), n), dim3(256), 0, st, X, n, ld, offset);
}

__global__ void k_zero_mat(double* X, int m, int n, int ld) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i < m && j < n) X[(size_t)i + (size_t)j * ld] = 0.0;
}
void zero_mat(hipStream_t st, double* X, int m, int n, int ld) {
  if (m > 0 && n > 0) hipLaunchKernelGGL(k_zero_mat, dim3(cdiv(m, 256), n), dim3(256), 0, st, X, m, n, ld);
}

__global__ void k_scale_pow2(double* x, int m, const int* e, int sign) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = ldexp(x[i], sign * e[0]);
}
void scale_pow2(hipStream_t st, double* x, int m, const int* e_dev, int sign) {
  if (m > 0) hipLaunchKernelGGL(k_scale_pow2, dim3(cdiv(m, 256)), dim3(256), 0, st, x, m, e_dev, sign);
}

// Frobenius norm: per column, the sum of squares of the entries scaled by
// an exact power of two that brings the column's largest magnitude into
// [2^-450, 2^450] (no underflow of tiny columns, no overflow of huge ones);
// the final pass brings the columns to the scale of the largest one.
__global__ __launch_bounds__(256) void k_fro_part(int m, int n, const double* X, int ld,
                                                  double* part) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double mx = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) mx = fmax(mx, fabs(X[(size_t)i + (size_t)j * ld]));
  mx = block_max(mx, sh);
  const double sc = safe_scale(mx);
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double v = X[(size_t)i + (size_t)j * ld] * sc;
    s = fma(v, v, s);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    part[j] = s;
    part[n + j] = sc;
  }
}
__global__ __launch_bounds__(256) void k_fro_fin(int n, const double* part, double* out) {
  __shared__ double sh[4];
  // the smallest column scale belongs to the largest column (scales are
  // powers of two, so their reciprocals are exact)
  double imax = 0.0;
  for (int j = threadIdx.x; j < n; j += 256)
    if (part[j] > 0.0) imax = fmax(imax, 1.0 / part[n + j]);
  imax = block_max(imax, sh);
  const double smin = (imax > 0.0) ? 1.0 / imax : 1.0;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double r = smin / part[n + j];  // power of two <= 1
    s = fma(part[j] * r, r, s);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = (s > 0.0) ? sqrt(s) / smin : 0.0;
}
void fro_norm(hipStream_t st, int m, int n, const double* X, int ld, double* out,
              double* partials) {
  if (m <= 0 || n <= 0) { fill(st, out, 1, 0.0); return; }
  hipLaunchKernelGGL(k_fro_part, dim3(n), dim3(256), 0, st, m, n, X, ld, partials);
  hipLaunchKernelGGL(k_fro_fin, dim3(1), dim3(256), 0, st, n, partials, out);
}

int num_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

}  // namespace htk
