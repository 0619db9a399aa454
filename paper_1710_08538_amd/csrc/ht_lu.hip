// ht_lu.hip -- block back substitution with a block upper triangular B
// (Sec. 3.5, impact of the l-block absorption on Algorithm 1): the LU
// decomposition with partial pivoting of every diagonal block, once per
// panel, and the solve with one block's factors.
//
// The diagonal blocks of the trailing L x L matrix have order S and are
// aligned at its bottom: block i (from the bottom) is [max(0, L - (i+1) S),
// L - i S).  Factors live in an L x S area `lu` (column q of block [a, e) at
// lu + a + q ld); the row permutation of the pivoting, 0-based within the
// block (row r of P x is x[perm[r]]), at perm + a.
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
                                                     int* __restrict__ perm,
                                                     const double* __restrict__ normB) {
  __shared__ double sval[kLuNT];
  __shared__ int sidx[kLuNT];
  __shared__ int spiv[128];
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
    if (tid == 0) spiv[c] = pr;
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
  // the interchanges, applied in order to the identity, as one permutation
  if (tid == 0) {
    for (int r = 0; r < z; ++r) sidx[r] = r;
    for (int c = 0; c < z; ++c) {
      const int t = sidx[c];
      sidx[c] = sidx[spiv[c]];
      sidx[spiv[c]] = t;
    }
  }
  __syncthreads();
  if (tid < z) perm[a + tid] = sidx[tid];
}

// x(a:a+z) <- U^{-1} L^{-1} P x(a:a+z) with the factors of one block: one
// wavefront, lane l holding rows l and l + 64; each substitution step
// broadcasts the finished entry from its lane.  The factor columns are read
// in chunks of kCh, the next chunk's loads issued before the current chunk
// is used, so that the serial steps do not wait on memory; the row indexes
// of the loads are clamped into the block (unused rows are masked).
constexpr int kCh = 16;

__device__ __forceinline__ void lu_load_cols(const double* __restrict__ F, int ldlu, int q0,
                                             int q1, int cfirst, int z, double f0[kCh],
                                             double f1[kCh]) {
#pragma unroll
  for (int u = 0; u < kCh; ++u) {
    const int c = min(max(cfirst + u, 0), z - 1);
    f0[u] = F[q0 + (size_t)c * ldlu];
    f1[u] = F[q1 + (size_t)c * ldlu];
  }
}

__global__ __launch_bounds__(64) void k_lu_solve(const double* __restrict__ lu, int ldlu,
                                                 const int* __restrict__ perm, int a, int z,
                                                 double* __restrict__ x) {
  const int r0 = threadIdx.x, r1 = threadIdx.x + 64;
  const int q0 = min(r0, z - 1), q1 = min(r1, z - 1);
  const double* F = lu + a;
  double v0 = r0 < z ? x[a + perm[a + r0]] : 0.0;
  double v1 = r1 < z ? x[a + perm[a + r1]] : 0.0;
  const double rd0 = 1.0 / F[q0 + (size_t)q0 * ldlu], rd1 = 1.0 / F[q1 + (size_t)q1 * ldlu];
  double f0[kCh], f1[kCh], g0[kCh], g1[kCh];
  // forward substitution with the unit lower factor, columns ascending
  lu_load_cols(F, ldlu, q0, q1, 0, z, f0, f1);
  for (int c0 = 0; c0 < z; c0 += kCh) {
    if (c0 + kCh < z) lu_load_cols(F, ldlu, q0, q1, c0 + kCh, z, g0, g1);
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      const int c = c0 + u;
      if (c < z) {
        const double xc = c < 64 ? __shfl(v0, c) : __shfl(v1, c - 64);
        if (r0 > c && r0 < z) v0 -= f0[u] * xc;
        if (r1 > c && r1 < z) v1 -= f1[u] * xc;
      }
    }
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      f0[u] = g0[u];
      f1[u] = g1[u];
    }
  }
  // back substitution with the upper factor, columns descending: chunk
  // [c0 - kCh + 1, c0], entry u at column c0 - u
  auto load_desc = [&](int chi, double h0[kCh], double h1[kCh]) {
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      const int c = min(max(chi - u, 0), z - 1);
      h0[u] = F[q0 + (size_t)c * ldlu];
      h1[u] = F[q1 + (size_t)c * ldlu];
    }
  };
  load_desc(z - 1, f0, f1);
  for (int c0 = z - 1; c0 >= 0; c0 -= kCh) {
    if (c0 - kCh >= 0) load_desc(c0 - kCh, g0, g1);
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      const int c = c0 - u;
      if (c >= 0) {
        const double xc = c < 64 ? __shfl(v0 * rd0, c) : __shfl(v1 * rd1, c - 64);
        if (r0 < c) v0 -= f0[u] * xc;
        if (r1 < c) v1 -= f1[u] * xc;
        if (r0 == c) v0 = xc;
        if (r1 == c) v1 = xc;
      }
    }
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      f0[u] = g0[u];
      f1[u] = g1[u];
    }
  }
  if (r0 < z) x[a + r0] = v0;
  if (r1 < z) x[a + r1] = v1;
}

void lu_blocks(hipStream_t st, int L, int S, const double* B, int ldb, double* lu, int ldlu,
               int* perm, const double* normB) {
  if (L <= 0 || S <= 0 || S > 128) return;
  const int nblk = (L + S - 1) / S;
  hipLaunchKernelGGL(k_lu_blocks, dim3(nblk), dim3(kLuNT), 0, st, L, S, B, ldb, lu, ldlu, perm,
                     normB);
}

void block_solve(hipStream_t st, int L, int S, const double* B, int ldb, const double* lu,
                 int ldlu, const int* perm, const double* c, double* x, double* partials) {
  if (L <= 0 || S <= 0 || S > 128) return;
  copy(st, x, c, L);
  for (int e = L; e > 0; e -= S) {
    const int a = std::max(0, e - S), z = e - a;
    if (e < L)
      gemv_n(st, z, L - e, -1.0, B + (size_t)a + (size_t)e * ldb, ldb, x + e, 1, 1.0, x + a,
             partials);
    hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(64), 0, st, lu, ldlu, perm, a, z, x);
  }
}

}  // namespace htk
