// ht_device.h -- device-side helpers shared by the HIP kernels of libhtred.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace htk {

constexpr double kUnitRoundoff = 0x1.0p-53;
constexpr double kBig = 0x1.0p600;      // rescale threshold for solves
constexpr double kShrink = 0x1.0p-600;  // 1 / kBig
constexpr int kShrinkExp = 600;

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide sum over blockDim.x threads (multiple of 64, <= 1024); every
// thread receives the result.  `sh` must hold blockDim.x/64 doubles; the
// summation order is fixed, so results are deterministic.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s = fmax(s, sh[i]);
  return s;
}

// s = sum over c in [c0, c1) of M[c * step] * z[c], accumulated in order of c
// (the same rounding as the plain loop) with sixteen loads in flight, so that
// a long strided sum is not one load latency per term.
__device__ __forceinline__ double dot_in_order(const double* __restrict__ M, size_t step,
                                               const double* z, int c0, int c1) {
  double s = 0.0;
  int c = c0;
  for (; c + 16 <= c1; c += 16) {
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = M[(size_t)(c + u) * step];
#pragma unroll
    for (int u = 0; u < 16; ++u) s = fma(a[u], z[c + u], s);
  }
  for (; c < c1; ++c) s = fma(M[(size_t)c * step], z[c], s);
  return s;
}

// block_sum / block_max of two values at once (two barriers instead of
// four; each value is reduced exactly as by the single-value version).
// `sh` must hold 2 * blockDim.x/64 doubles.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    sh[wv] = a;
    sh[nw + wv] = b;
  }
  __syncthreads();
  double s = 0.0, t = 0.0;
  for (int i = 0; i < nw; ++i) {
    s += sh[i];
    t += sh[nw + i];
  }
  a = s;
  b = t;
}
__device__ __forceinline__ void block_max2(double& a, double& b, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = wave_max(a);
  b = wave_max(b);
  __syncthreads();
  if (lane == 0) {
    sh[wv] = a;
    sh[nw + wv] = b;
  }
  __syncthreads();
  double s = 0.0, t = 0.0;
  for (int i = 0; i < nw; ++i) {
    s = fmax(s, sh[i]);
    t = fmax(t, sh[nw + i]);
  }
  a = s;
  b = t;
}

// Counter-based N(0,1) numbers: splitmix64 (Steele, Lea, Flood 2014) feeding
// Box-Muller; used for the zero-diagonal perturbation rho.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double normal_draw(uint64_t seed, uint64_t counter) {
  uint64_t a = splitmix64(seed ^ splitmix64(2 * counter));
  uint64_t b = splitmix64(seed ^ splitmix64(2 * counter + 1));
  double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;
  double u2 = ((double)(b >> 11)) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Reflector coefficients from alpha (pivot) and the scaled norm of the
// remaining entries (LAPACK dlarfg convention): (I - tau v v^T) x = beta e1,
// beta = -sign(alpha) ||x||, v = x / (alpha - beta) below the pivot.
struct Refl { double tau, beta, scal; };

// Power-of-two factor that brings a vector whose largest magnitude is amx
// into [2^-450, 2^450] (1 when it is there already, or zero).  Squares and
// reciprocals of the scaled entries then neither overflow nor underflow to
// zero (subnormal entries included), and the scaling itself is exact.
__device__ __forceinline__ double safe_scale(double amx) {
  if (amx > 0.0 && amx < 0x1.0p-450) return 0x1.0p600;
  if (amx > 0x1.0p450) return 0x1.0p-600;
  return 1.0;
}

// Householder reflector (LAPACK sign convention, beta = -sign(alpha) ||.||)
// from the pivot alpha and ss = ||x||^2 of the rest, both of a vector that
// safe_scale has brought into range: v = [1; x * scal], H = I - tau v v^T.
__device__ __forceinline__ Refl make_refl_ss(double alpha, double ss) {
  Refl r;
  if (ss == 0.0) { r.tau = 0.0; r.beta = alpha; r.scal = 0.0; return r; }
  const double nrm = sqrt(fma(alpha, alpha, ss));
  r.beta = (alpha >= 0.0) ? -nrm : nrm;
  r.tau = (r.beta - alpha) / r.beta;
  r.scal = 1.0 / (alpha - r.beta);
  return r;
}

}  // namespace htk
