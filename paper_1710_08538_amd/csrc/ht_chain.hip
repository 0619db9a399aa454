// ht_chain.hip -- small Householder factorisations for the absorption chains
// of Sec. 3.3: QL of the blocks of V2 (step b of Sec. 3.3.1), QR of the
// blocks of U2 (step b of Sec. 3.3.2), RQ of the subdiagonal blocks of B when
// restoring it from the right (step e), QR when restoring it from the left
// (step f).  RQ is done as QL of the transposed block.
//
// One workgroup factors one w x k tile (w <= 2*128, k <= 128) and returns the
// orthogonal factor in regular WY form Qf = I - V W^T (Sec. 2.4, W = V T^T),
// with the reflectors taken in the order they were computed so that
//   QR:  tile = Qf [R; 0],   QL:  tile = Qf [0; L].
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

// Logical tile element (r, c) of a w x k tile stored at p with leading
// dimension ld, optionally transposed in memory.
__device__ __forceinline__ size_t tidx(int r, int c, int ld, int trans) {
  return trans ? ((size_t)c + (size_t)r * ld) : ((size_t)r + (size_t)c * ld);
}

// Shared-memory layout when the tile is staged (w+1 leading dimension keeps
// column-per-lane accesses free of bank conflicts).
constexpr int kChainThreads = 256;

__global__ __launch_bounds__(kChainThreads) void k_chain_factor(
    int mode, int w, int k, double* __restrict__ X, int ldx, int trans, double* __restrict__ Vout,
    double* __restrict__ Wout, double* __restrict__ Gws, int staged) {
  extern __shared__ double dyn[];
  __shared__ double taus[128];
  __shared__ double vsh[256];
  __shared__ double red[4];
  __shared__ double pdot[4][128];

  const int tid = threadIdx.x;
  // Working copies: M (w x k) and V (w x k).
  double* M;
  int ldm;
  double* V;
  int ldv;
  if (staged) {
    ldm = w + 1;
    M = dyn;
    V = dyn + (size_t)ldm * k;
    ldv = ldm;
    for (int e = tid; e < w * k; e += kChainThreads) {
      int r, c;
      if (trans) { c = e % k; r = e / k; } else { r = e % w; c = e / w; }
      M[r + (size_t)c * ldm] = X[tidx(r, c, ldx, trans)];
    }
  } else {
    M = nullptr;  // work in place (global)
    ldm = 0;
    V = Vout;
    ldv = w;
  }
  __syncthreads();
  auto Mref = [&](int r, int c) -> double& {
    return staged ? M[r + (size_t)c * ldm] : X[tidx(r, c, ldx, trans)];
  };

  const int ncg = (k <= 64) ? 64 : 128;  // columns per pass
  const int tpc = kChainThreads / ncg;   // threads per column (4 or 2)
  const int mycol = tid % ncg;
  const int part = tid / ncg;

  for (int step = 0; step < k; ++step) {
    const int i = (mode == 0) ? step : (k - 1 - step);
    const int p = (mode == 0) ? i : (w - k + i);
    // x-part of column i: QR rows p+1..w-1, QL rows 0..p-1
    const int x0 = (mode == 0) ? p + 1 : 0;
    const int x1 = (mode == 0) ? w : p;
    double amax = 0.0;
    for (int r = x0 + tid; r < x1; r += kChainThreads) amax = fmax(amax, fabs(Mref(r, i)));
    amax = block_max(amax, red);
    double ss = 0.0;
    if (amax > 0.0) {
      const double inv = 1.0 / amax;
      for (int r = x0 + tid; r < x1; r += kChainThreads) {
        double t = Mref(r, i) * inv;
        ss = fma(t, t, ss);
      }
    }
    ss = block_sum(ss, red);
    const double alpha = Mref(p, i);
    const Refl rf = make_refl(alpha, amax * sqrt(ss));
    for (int r = tid; r < w; r += kChainThreads) {
      double v;
      if (r == p) v = 1.0;
      else if (r >= x0 && r < x1) v = Mref(r, i) * rf.scal;
      else v = 0.0;
      vsh[r] = v;
      V[r + (size_t)step * ldv] = v;
      if (r == p) Mref(r, i) = rf.beta;
      else if (r >= x0 && r < x1) Mref(r, i) = 0.0;
    }
    if (tid == 0) taus[step] = rf.tau;
    __syncthreads();
    // apply (I - tau v v^T) to the columns still to be reduced
    const int s0 = (mode == 0) ? p : 0;       // support rows [s0, s1)
    const int s1 = (mode == 0) ? w : p + 1;
    for (int cb = 0; cb < k; cb += ncg) {
      const int c = cb + mycol;
      const bool act = (c < k) && ((mode == 0) ? (c > i) : (c < i));
      double d = 0.0;
      if (act)
        for (int r = s0 + part; r < s1; r += tpc) d = fma(vsh[r], Mref(r, c), d);
      pdot[part][mycol] = d;
      __syncthreads();
      if (act) {
        double dd = 0.0;
        for (int q = 0; q < tpc; ++q) dd += pdot[q][mycol];
        const double f = rf.tau * dd;
        if (f != 0.0)
          for (int r = s0 + part; r < s1; r += tpc) Mref(r, c) = fma(-f, vsh[r], Mref(r, c));
      }
      __syncthreads();
    }
  }

  // write the factor back (staged case) -- R or L with exact zeros
  if (staged) {
    for (int e = tid; e < w * k; e += kChainThreads) {
      int r, c;
      if (trans) { c = e % k; r = e / k; } else { r = e % w; c = e / w; }
      X[tidx(r, c, ldx, trans)] = M[r + (size_t)c * ldm];
    }
  }
  __syncthreads();

  // Compact-WY T (upper triangular, forward order of computation):
  // T(s,s) = tau_s, T(0:s, s) = -tau_s T(0:s, 0:s) (V(:,0:s)^T v_s).
  // G = V^T V (strictly upper part), then W = V T^T.
  double* G;
  double* T;
  if (staged) {
    G = dyn;                    // reuse the M area (k*k <= (w+1)*k)
    T = dyn + (size_t)k * k;    // fits: 2k^2 <= (w+1)k for w >= 2k-1 ... else use Gws
    if ((size_t)2 * k * k > (size_t)(w + 1) * k) { G = Gws; T = Gws + (size_t)k * k; }
  } else {
    G = Gws;
    T = Gws + (size_t)k * k;
  }
  for (int e = tid; e < k * k; e += kChainThreads) {
    const int a = e % k, b = e / k;
    double s = 0.0;
    if (a < b)
      for (int r = 0; r < w; ++r) s = fma(V[r + (size_t)a * ldv], V[r + (size_t)b * ldv], s);
    G[a + (size_t)b * k] = s;
    T[a + (size_t)b * k] = (a == b) ? taus[a] : 0.0;
  }
  __syncthreads();
  for (int b = 1; b < k; ++b) {
    if (tid < b) {
      double s = 0.0;
      for (int c = tid; c < b; ++c) s = fma(T[tid + (size_t)c * k], G[c + (size_t)b * k], s);
      T[tid + (size_t)b * k] = -taus[b] * s;
    }
    __syncthreads();
  }
  // W(r, b) = sum_{c >= b} V(r, c) T(b, c)
  for (int e = tid; e < w * k; e += kChainThreads) {
    const int r = e % w, b = e / w;
    double s = 0.0;
    for (int c = b; c < k; ++c) s = fma(V[r + (size_t)c * ldv], T[b + (size_t)c * k], s);
    Wout[r + (size_t)b * w] = s;
  }
  if (staged) {
    __syncthreads();
    for (int e = tid; e < w * k; e += kChainThreads) {
      const int r = e % w, c = e / w;
      Vout[r + (size_t)c * w] = V[r + (size_t)c * ldv];
    }
  }
}

static void launch_chain(hipStream_t st, int mode, int w, int k, double* tile, int ldt, int trans,
                         double* Vout, double* Wout, double* Gws) {
  if (w <= 0 || k <= 0) return;
  const size_t stage_bytes = (size_t)2 * (w + 1) * k * sizeof(double);
  const int staged = stage_bytes <= 150 * 1024 ? 1 : 0;
  hipLaunchKernelGGL(k_chain_factor, dim3(1), dim3(kChainThreads), staged ? stage_bytes : 0, st,
                     mode, w, k, tile, ldt, trans, Vout, Wout, Gws, staged);
}

void chain_factor(hipStream_t st, int mode, int w, int k, double* tile, int ldt, double* Vout,
                  double* Wout, double* Tscratch) {
  launch_chain(st, mode, w, k, tile, ldt, 0, Vout, Wout, Tscratch);
}

void chain_factor_t(hipStream_t st, int mode, int w, int k, double* tile, int ldt, double* Vout,
                    double* Wout, double* Tscratch) {
  launch_chain(st, mode, w, k, tile, ldt, 1, Vout, Wout, Tscratch);
}

}  // namespace htk
