// ht_panel.hip -- kernels of the panel reduction (Sec. 3.2): reflector
// generation, the overflow-safe triangular solve behind the opposite
// reflectors, iterative-refinement bookkeeping, compact-WY factor updates.
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Householder reflector of a device vector (one 1024-thread workgroup).
// Reflector of Sec. 2.1 in the LAPACK sign convention: H x = beta e1 with
// beta = -sign(x0) ||x||_2; the norm is accumulated on x / max|x| so that
// entries near the FP64 range limits neither overflow nor underflow.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_house(int m, double* x, double* v, double* tau_out,
                                                double* beta_out, int overwrite) {
  __shared__ double sh[16];
  const double alpha = x[0];
  double ss = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += 1024) ss = fma(x[i], x[i], ss);
  ss = block_sum(ss, sh);
  // When ss >= m 2^-900, ss <= 2^880 and |alpha| <= 2^440, the largest
  // magnitude lies in [2^-450, 2^450] and no scaling is needed (the sum is
  // the one the scaled pass below would give with factor 1).  Otherwise scale
  // exactly by a power of two into the safe range (tiny or huge columns).
  double sc = 1.0;
  if (!(ss >= (double)m * 0x1.0p-900 && ss <= 0x1.0p880 && fabs(alpha) <= 0x1.0p440)) {
    double amax = 0.0;
    for (int i = 1 + threadIdx.x; i < m; i += 1024) amax = fmax(amax, fabs(x[i]));
    amax = block_max(amax, sh);
    sc = safe_scale(fmax(amax, fabs(alpha)));
    ss = 0.0;
    if (amax > 0.0) {
      for (int i = 1 + threadIdx.x; i < m; i += 1024) {
        const double t = x[i] * sc;
        ss = fma(t, t, ss);
      }
    }
    ss = block_sum(ss, sh);
  }
  const Refl r = make_refl_ss(alpha * sc, ss);
  const double f = sc * r.scal;
  for (int i = 1 + threadIdx.x; i < m; i += 1024) {
    double xi = x[i];
    v[i] = xi * f;
    if (overwrite) x[i] = 0.0;
  }
  if (threadIdx.x == 0) {
    const double beta = r.beta / sc;
    v[0] = 1.0;
    if (overwrite) x[0] = beta;
    tau_out[0] = r.tau;
    beta_out[0] = beta;
  }
}

void house(hipStream_t st, int m, double* x, double* v, double* tau, double* beta,
           bool overwrite) {
  hipLaunchKernelGGL(k_house, dim3(1), dim3(1024), 0, st, m, x, v, tau, beta,
                     overwrite ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Compact-WY append (Sec. 2.4, used for S in step b and T in step d):
// T(0:kk, kk) = -tau T(0:kk, 0:kk) z,  T(kk, kk) = tau.
// ---------------------------------------------------------------------------
__global__ void k_wy_append(double* T, int ldt, int kk, const double* z, const double* tau) {
  __shared__ double zs[128];
  const int t = threadIdx.x;
  if (t < kk) zs[t] = z[t];
  __syncthreads();
  const double ta = tau[0];
  if (t < kk) T[t + (size_t)kk * ldt] = -ta * dot_in_order(T + t, (size_t)ldt, zs, t, kk);
  if (t == 0) T[kk + (size_t)kk * ldt] = ta;
}
void wy_append(hipStream_t st, double* T, int ldt, int kk, const double* z, const double* tau) {
  hipLaunchKernelGGL(k_wy_append, dim3(1), dim3(128), 0, st, T, ldt, kk, z, tau);
}

// ---------------------------------------------------------------------------
// Iterative refinement (Sec. 2.3, step c of Sec. 3.2.2).
// r = 2^{-Erhs} c - w (c = e1 when c == NULL); status = 1 when
// ||r||_2 <= tol_factor * u * ||B||_F * ||x||_2.  norms[0..1] = ||r||, ||x||.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_ir_residual(int m, const double* w, const double* c,
                                                      const int* Erhs, double* r, const double* x,
                                                      const double* normB, double tol_factor,
                                                      int* status, double* norms) {
  __shared__ double sh[32];
  const int E = Erhs[0];
  double rmax = 0.0, xmax = 0.0;
  for (int i = threadIdx.x; i < m; i += 1024) {
    double ci = c ? c[i] : (i == 0 ? 1.0 : 0.0);
    double ri = ldexp(ci, -E) - w[i];
    r[i] = ri;
    rmax = fmax(rmax, fabs(ri));
    xmax = fmax(xmax, fabs(x[i]));
  }
  block_max2(rmax, xmax, sh);
  double rs = 0.0, xs = 0.0;
  // exact power-of-two scalings (subnormal or huge entries are safe)
  const double ir = safe_scale(rmax), ix = safe_scale(xmax);
  for (int i = threadIdx.x; i < m; i += 1024) {
    double a = r[i] * ir, b = x[i] * ix;
    rs = fma(a, a, rs);
    xs = fma(b, b, xs);
  }
  block_sum2(rs, xs, sh);
  if (threadIdx.x == 0) {
    const double rn = sqrt(rs) / ir, xn = sqrt(xs) / ix;
    norms[0] = rn;
    norms[1] = xn;
    const double tol = tol_factor * kUnitRoundoff * normB[0];
    status[0] = (rn <= tol * xn) ? 1 : 0;
  }
}
void ir_residual(hipStream_t st, int m, const double* w, const double* c, const int* Erhs,
                 double* r, const double* x, const double* normB, double tol_factor, int* status,
                 double* norms) {
  hipLaunchKernelGGL(k_ir_residual, dim3(1), dim3(1024), 0, st, m, w, c, Erhs, r, x, normB,
                     tol_factor, status, norms);
}

__global__ void k_ir_update(int m, double* x, const double* d, const int* E2, int* Erhs,
                            int last_block) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = E2[0];
  if (i < m) x[i] = ldexp(x[i], -e) + d[i];
  if (last_block && i == 0) Erhs[0] += e;
}
void ir_update(hipStream_t st, int m, double* x, const double* d, const int* E2, int* Erhs) {
  // the exponent is bumped by a separate one-thread launch after all blocks
  // have read E2 (E2 and Erhs may be distinct words; order kept by the stream)
  hipLaunchKernelGGL(k_ir_update, dim3(cdiv(m, 256)), dim3(256), 0, st, m, x, d, E2, Erhs, 0);
  hipLaunchKernelGGL(k_ir_update, dim3(1), dim3(1), 0, st, 0, x, d, E2, Erhs, 1);
}

// ---------------------------------------------------------------------------
// Zero-diagonal rule (Sec. 3.2.1, Remark 2.2): a zero (or subnormal) diagonal
// entry of B(s:n, s:n) becomes 2 u rho ||B||_F with rho ~ N(0,1).
// ---------------------------------------------------------------------------
__global__ void k_fix_diag(double* B, int ldb, int s, int n, const double* normB, uint64_t seed,
                           uint64_t salt, int* count) {
  const int i = s + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* p = B + (size_t)i + (size_t)i * ldb;
  const double d = *p;
  if (normB[0] > 0.0 && fabs(d) < 2.2250738585072014e-308) {
    double rho = normal_draw(seed, salt * (uint64_t)n + (uint64_t)i);
    if (rho == 0.0) rho = 1.0;
    *p = 2.0 * kUnitRoundoff * rho * normB[0];
    atomicAdd(count, 1);
  }
}
void fix_diagonal(hipStream_t st, double* B, int ldb, int s, int n, const double* normB,
                  uint64_t seed, uint64_t salt, int* count_dev) {
  if (n - s <= 0) return;
  hipLaunchKernelGGL(k_fix_diag, dim3(cdiv(n - s, 256)), dim3(256), 0, st, B, ldb, s, n, normB,
                     seed, salt, count_dev);
}

}  // namespace htk
