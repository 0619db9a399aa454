// ht_lu.hip -- block back substitution with a block upper triangular B
// (Sec. 3.5, impact of the l-block absorption on Algorithm 1): the LU
// decomposition with partial pivoting of every diagonal block, once per
// panel, and the solve with one block's factors.
//
// The diagonal blocks of the trailing L x L matrix have order S and are
// aligned at its bottom: block i (from the bottom) is [max(0, L - (i+1) S),
// L - i S).  Factors live in an L x S area `lu` (column q of block [a, e) at
// lu + a + q ld) with the pivots, 0-based within the block, at piv + a.
#include <algorithm>

#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

constexpr int kLuNT = 256;

// One workgroup per diagonal block (order <= 128 < kLuNT): copy the block,
// then right-looking elimination in global memory.  Ties in the pivot
// search go to the smallest row; an exactly zero pivot column is given the
// pivot eps * ||B||_F (the solves then carry an error that refinement sees).
__global__ __launch_bounds__(kLuNT) void k_lu_blocks(int L, int S, const double* __restrict__ B,
                                                     int ldb, double* __restrict__ lu, int ldlu,
                                                     int* __restrict__ piv,
                                                     const double* __restrict__ normB) {
  __shared__ double sval[kLuNT];
  __shared__ int sidx[kLuNT];
  const int e = L - (int)blockIdx.x * S;
  if (e <= 0) return;
  const int a = max(0, e - S), z = e - a, tid = threadIdx.x;
  double* F = lu + a;
  for (int q = 0; q < z; ++q)
    for (int r = tid; r < z; r += kLuNT)
      F[r + (size_t)q * ldlu] = B[(size_t)(a + r) + (size_t)(a + q) * ldb];
  __syncthreads();
  for (int c = 0; c < z; ++c) {
    const int r = c + tid;
    sval[tid] = r < z ? fabs(F[r + (size_t)c * ldlu]) : -1.0;
    sidx[tid] = r;
    __syncthreads();
    for (int h = kLuNT / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const double v2 = sval[tid + h];
        const int i2 = sidx[tid + h];
        if (v2 > sval[tid] || (v2 == sval[tid] && i2 < sidx[tid])) {
          sval[tid] = v2;
          sidx[tid] = i2;
        }
      }
      __syncthreads();
    }
    const int pr = sidx[0];
    if (tid == 0) piv[a + c] = pr;
    if (pr != c)
      for (int q = tid; q < z; q += kLuNT) {
        const double t = F[c + (size_t)q * ldlu];
        F[c + (size_t)q * ldlu] = F[pr + (size_t)q * ldlu];
        F[pr + (size_t)q * ldlu] = t;
      }
    __syncthreads();
    double d = F[c + (size_t)c * ldlu];
    if (d == 0.0) d = 0x1.0p-52 * normB[0];
    __syncthreads();
    if (tid == 0) F[c + (size_t)c * ldlu] = d;
    for (int rr = c + 1 + tid; rr < z; rr += kLuNT) F[rr + (size_t)c * ldlu] /= d;
    __syncthreads();
    const int t = z - c - 1;
    for (int idx = tid; idx < t * t; idx += kLuNT) {
      const int rr = c + 1 + idx % t, q = c + 1 + idx / t;
      F[rr + (size_t)q * ldlu] -= F[rr + (size_t)c * ldlu] * F[c + (size_t)q * ldlu];
    }
    __syncthreads();
  }
}

// x(a:a+z) <- U^{-1} L^{-1} P x(a:a+z) with the factors of one block.
__global__ __launch_bounds__(kLuNT) void k_lu_solve(const double* __restrict__ lu, int ldlu,
                                                    const int* __restrict__ piv, int a, int z,
                                                    double* __restrict__ x) {
  __shared__ double xs[128];
  const int tid = threadIdx.x;
  const double* F = lu + a;
  if (tid < z) xs[tid] = x[a + tid];
  __syncthreads();
  if (tid == 0)
    for (int c = 0; c < z; ++c) {
      const int p = piv[a + c];
      const double t = xs[c];
      xs[c] = xs[p];
      xs[p] = t;
    }
  __syncthreads();
  for (int c = 0; c < z; ++c) {
    const double xc = xs[c];
    if (tid > c && tid < z) xs[tid] -= F[tid + (size_t)c * ldlu] * xc;
    __syncthreads();
  }
  for (int c = z - 1; c >= 0; --c) {
    const double xc = xs[c] / F[c + (size_t)c * ldlu];
    __syncthreads();
    if (tid < c) xs[tid] -= F[tid + (size_t)c * ldlu] * xc;
    if (tid == c) xs[c] = xc;
    __syncthreads();
  }
  if (tid < z) x[a + tid] = xs[tid];
}

void lu_blocks(hipStream_t st, int L, int S, const double* B, int ldb, double* lu, int ldlu,
               int* piv, const double* normB) {
  if (L <= 0 || S <= 0 || S > 128) return;
  const int nblk = (L + S - 1) / S;
  hipLaunchKernelGGL(k_lu_blocks, dim3(nblk), dim3(kLuNT), 0, st, L, S, B, ldb, lu, ldlu, piv,
                     normB);
}

void block_solve(hipStream_t st, int L, int S, const double* B, int ldb, const double* lu,
                 int ldlu, const int* piv, const double* c, double* x, double* partials) {
  if (L <= 0 || S <= 0 || S > 128) return;
  copy(st, x, c, L);
  for (int e = L; e > 0; e -= S) {
    const int a = std::max(0, e - S), z = e - a;
    if (e < L)
      gemv_n(st, z, L - e, -1.0, B + (size_t)a + (size_t)e * ldb, ldb, x + e, 1, 1.0, x + a,
             partials);
    hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(kLuNT), 0, st, lu, ldlu, piv, a, z, x);
  }
}

}  // namespace htk
