// ht_chain.hip -- small Householder factorisations for the absorption chains
// of Sec. 3.3: QL of the blocks of V2 (step b of Sec. 3.3.1), QR of the
// blocks of U2 (step b of Sec. 3.3.2), RQ of the subdiagonal blocks of B when
// restoring it from the right (step e), QR when restoring it from the left
// (step f).  RQ is done as QL of the transposed block.
//
// One workgroup (1024 threads for k <= 64, 512 for k <= 128) factors one
// w x k tile (w <= 2*KMAX, k <= KMAX)
// held in registers: thread (c, g) owns column c, rows g*RPG .. g*RPG+RPG-1.
// The orthogonal factor is returned in regular WY form Qf = I - V W^T
// (Sec. 2.4), reflectors in the order they are computed, so that
//   QR:  tile = Qf [R; 0],   QL:  tile = Qf [0; L].
// W is accumulated alongside the factorisation:  with Qf_i = I - V_i W_i^T,
//   Qf_i (I - tau v v^T) = I - [V_i v] [(I - tau v v^T) W_i, tau v]^T,
// so after column c has produced its reflector the registers that held
// column c of the tile hold column c of W and receive the later reflectors
// exactly like the columns still to be reduced.  Each reflector costs three
// workgroup barriers; one wavefront forms the reflector, everyone applies it.
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

__device__ __forceinline__ size_t tidx(int r, int c, int ld, int trans) {
  return trans ? ((size_t)c + (size_t)r * ld) : ((size_t)r + (size_t)c * ld);
}

template <int KMAX, int NT>
__global__ __launch_bounds__(NT) void k_chain_reg(int mode, int w, int k, double* __restrict__ X,
                                                    int ldx, int trans, double* __restrict__ Vout,
                                                    double* __restrict__ Wout) {
  constexpr int G = NT / KMAX;          // row groups
  constexpr int RPG = 2 * KMAX / G;     // rows per group
  constexpr int WR = 2 * KMAX / 64;     // rows per lane when one wave scans a column
  static_assert(RPG <= 64, "a group's rows must fit one wavefront");
  __shared__ double vraw[2 * KMAX];
  __shared__ double vfin[2 * KMAX];
  __shared__ double sref[1];            // tau
  __shared__ double pdot[G][KMAX];

  const int tid = threadIdx.x;
  const int c = tid % KMAX;
  const int g = tid / KMAX;
  const int lane = tid & 63;
  const int r0 = g * RPG;
  (void)lane;
  const bool colok = c < k;

  double reg[RPG];
#pragma unroll
  for (int q = 0; q < RPG; ++q) {
    const int r = r0 + q;
    reg[q] = (colok && r < w) ? X[tidx(r, c, ldx, trans)] : 0.0;
  }

  for (int step = 0; step < k; ++step) {
    const int i = (mode == 0) ? step : (k - 1 - step);
    const int p = (mode == 0) ? i : (w - k + i);
    const int x0 = (mode == 0) ? p + 1 : 0;  // x-part rows [x0, x1)
    const int x1 = (mode == 0) ? w : p;
    // phase A: the owners of column i publish it
    if (c == i) {
#pragma unroll
      for (int q = 0; q < RPG; ++q) vraw[r0 + q] = reg[q];
    }
    __syncthreads();
    // phase A2: wave 0 forms the reflector and the final v
    if (tid < 64) {
      double xv[WR];
      double amax = 0.0, ss = 0.0;
#pragma unroll
      for (int q = 0; q < WR; ++q) {
        const int r = lane + 64 * q;
        xv[q] = (r >= x0 && r < x1) ? vraw[r] : 0.0;
        amax = fmax(amax, fabs(xv[q]));
        ss = fma(xv[q], xv[q], ss);
      }
      amax = wave_max(amax);
      ss = wave_sum(ss);
      double xnorm;
      if (amax == 0.0) {
        xnorm = 0.0;
      } else if (amax > 0x1.0p-450 && amax < 0x1.0p450) {
        xnorm = sqrt(ss);
      } else {  // rescaled second pass near the ends of the FP64 range
        const double inv = 1.0 / amax;
        double s2 = 0.0;
#pragma unroll
        for (int q = 0; q < WR; ++q) { const double t = xv[q] * inv; s2 = fma(t, t, s2); }
        xnorm = amax * sqrt(wave_sum(s2));
      }
      const Refl rf = make_refl(vraw[p], xnorm);
#pragma unroll
      for (int q = 0; q < WR; ++q) {
        const int r = lane + 64 * q;
        const double v = (r == p) ? 1.0 : xv[q] * rf.scal;
        vfin[r] = v;
        if (r < w) {
          // column i of the factor (R or L) and reflector `step`
          double out = vraw[r];
          if (r == p) out = rf.beta;
          else if (r >= x0 && r < x1) out = 0.0;
          X[tidx(r, i, ldx, trans)] = out;
          Vout[(size_t)r + (size_t)step * w] = v;
        }
      }
      if (lane == 0) sref[0] = rf.tau;
    }
    __syncthreads();
    const double tau = sref[0];
    // v of this group's rows, read from LDS (the same address in every lane)
    const double* vg = vfin + r0;
    if (c == i) {
#pragma unroll
      for (int q = 0; q < RPG; ++q) reg[q] = tau * vg[q];  // column `step` of W
      pdot[g][c] = 0.0;
    } else {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < RPG; ++q) {
        d = fma(vg[q], reg[q], d);
        if ((q & 7) == 7) __asm__ volatile("" ::: "memory");  // keep LDS reads in chunks
      }
      pdot[g][c] = d;
    }
    __syncthreads();
    // phase C: rank-1 update of every other column (tile or W)
    if (c != i && colok) {
      double d = 0.0;
#pragma unroll
      for (int h = 0; h < G; ++h) d += pdot[h][c];
      const double f = tau * d;
      if (f != 0.0) {
#pragma unroll
        for (int q = 0; q < RPG; ++q) {
          reg[q] = fma(-f, vg[q], reg[q]);
          if ((q & 7) == 7) __asm__ volatile("" ::: "memory");
        }
      }
    }
  }
  // registers now hold W; column c was produced at step s(c)
  if (colok) {
    const int sc = (mode == 0) ? c : (k - 1 - c);
#pragma unroll
    for (int q = 0; q < RPG; ++q) {
      const int r = r0 + q;
      if (r < w) Wout[(size_t)r + (size_t)sc * w] = reg[q];
    }
  }
}

static void launch_chain(hipStream_t st, int mode, int w, int k, double* tile, int ldt, int trans,
                         double* Vout, double* Wout) {
  if (w <= 0 || k <= 0) return;
  if (k <= 64 && w <= 128)
    hipLaunchKernelGGL((k_chain_reg<64, 1024>), dim3(1), dim3(1024), 0, st, mode, w, k, tile,
                       ldt, trans, Vout, Wout);
  else
    hipLaunchKernelGGL((k_chain_reg<128, 1024>), dim3(1), dim3(1024), 0, st, mode, w, k, tile,
                       ldt, trans, Vout, Wout);
}

void chain_factor(hipStream_t st, int mode, int w, int k, double* tile, int ldt, double* Vout,
                  double* Wout, double* Tscratch) {
  (void)Tscratch;
  launch_chain(st, mode, w, k, tile, ldt, 0, Vout, Wout);
}

void chain_factor_t(hipStream_t st, int mode, int w, int k, double* tile, int ldt, double* Vout,
                    double* Wout, double* Tscratch) {
  (void)Tscratch;
  launch_chain(st, mode, w, k, tile, ldt, 1, Vout, Wout);
}

}  // namespace htk
