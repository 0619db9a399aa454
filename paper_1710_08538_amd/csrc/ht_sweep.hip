// ht_sweep.hip -- fused FP64-MFMA sweeps of block reflectors over row slabs.
//
// The absorption of Sec. 3.3 applies long sequences of overlapping 2k x 2k
// orthogonal transformations to A, B, Q and Z: the QL factors Q^_1..Q^_r of
// V2 (step c/d/e of Sec. 3.3.1, eq. (commuteQ)), the RQ factors that restore
// B from the right, and (as right multiplications of Q) the QR factors of U2
// and of the left restoration.  Each factor is held in regular WY form
// I - V W^T (V, W: 2k x k, column-major), and consecutive windows overlap by
// k columns and move by k columns.
//
// This kernel applies a whole run of such windows to a slab of 64 rows of a
// column-major matrix X:  X(:, win_t) <- X(:, win_t) - (X(:, win_t) V_t) W_t^T
// for t = 0 .. nwin-1, window t starting at column c0 + dir t k.  The slab's
// 2k window columns stay in registers; per window only the k columns that
// enter are loaded and the k that leave are stored, so a window costs
// 8 * 64 * k^2 flops for 16 * 64 * k bytes of HBM traffic (k/2 flop/byte).
//
// Arithmetic runs on v_mfma_f64_16x16x4f64.  Its accumulator layout is: lane
// l = 16 g + c holds rows g, g+4, g+8, g+12 of column c of the 16 x 16 tile
// in registers 0..3, which is exactly the B-operand layout of the k-chunks
// 0..3 of the next product, so results feed the next MFMA in place:
//   step 1   P^T (k x 64)  = V^T (k x 2k) . X^T (2k x 64)
//   step 2   X^T (2k x 64) -= W (2k x k) . P^T (k x 64)
// Each wavefront owns 16 slab rows (the MFMA N dimension); V and -W are
// staged through LDS in 16-wide chunks (double-buffered) and shared by the
// four wavefronts.  For an upper triangular X (B), windows that lie entirely
// left of the slab's first row are structurally zero there and are skipped.
#include "ht_device.h"
#include "ht_internal.h"
#include "ht_sweep.h"

namespace htk {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// V chunk t: rows [16 t, 16 t + 16) x columns [0, K) of V (column-major,
// ld 2K), staged as Vs[(4 kc + g) * K + 16 p + c] = V[16 t + 4 kc + g][16 p + c].
// -W chunk p: columns [16 p, 16 p + 16), all 2K rows, staged as
// Ws[(4 kc + g) * 2K + 16 t + c] = -W[16 t + c][16 p + 4 kc + g].
// The global loads go to registers first and are written to LDS after the
// MFMAs of the previous chunk, hiding their latency.
template <int K>
struct VReg {
  double v[K / 16];
  __device__ __forceinline__ void load(const double* __restrict__ V, int t, int tid) {
#pragma unroll
    for (int j = 0; j < K / 16; ++j) {
      const int e = tid + 256 * j;
      v[j] = V[(size_t)(16 * t + (e & 15)) + (size_t)(e >> 4) * 2 * K];
    }
  }
  __device__ __forceinline__ void store(double* Vs, int tid) const {
#pragma unroll
    for (int j = 0; j < K / 16; ++j) {
      const int e = tid + 256 * j;
      Vs[(e & 15) * K + (e >> 4)] = v[j];
    }
  }
};

template <int K>
struct WReg {
  double v[K / 8];
  __device__ __forceinline__ void load(const double* __restrict__ W, int p, int tid) {
#pragma unroll
    for (int j = 0; j < K / 8; ++j) {
      const int e = tid + 256 * j;
      v[j] = W[(size_t)(e % (2 * K)) + (size_t)(16 * p + e / (2 * K)) * 2 * K];
    }
  }
  __device__ __forceinline__ void store(double* Ws, int tid) const {
#pragma unroll
    for (int j = 0; j < K / 8; ++j) {
      const int e = tid + 256 * j;
      Ws[(e / (2 * K)) * 2 * K + (e % (2 * K))] = -v[j];
    }
  }
};

// TR = 1: the sweep of X^T, i.e. the left application
//   X(win, :) <- (I - V W^T)^T X(win, :) = X(win, :) - W (V^T X(win, :))
// on slabs of 64 columns of X: "rows" are columns of X (relative to the
// job's first column) and window "columns" are absolute rows of X.
template <int K, int DIR, int TR>
__global__ __launch_bounds__(256) void k_sweep_rows(SweepArgs a) {
  constexpr int NT = 2 * K / 16;  // window tiles of 16 columns
  constexpr int NP = K / 16;      // tiles of P^T
  constexpr int NH = NP;          // tiles entering / leaving per window
  __shared__ double stage[2][16 * 2 * K];

  // locate the job and the slab
  int jb = 0;
  while (jb + 1 < a.njobs && (int)blockIdx.x >= a.job[jb + 1].wg0) ++jb;
  const SweepJob job = a.job[jb];
  const int ra = ((int)blockIdx.x - job.wg0) * 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int row = ra + 16 * wave + c;
  const bool rok = row < job.nrows;
  double* __restrict__ X = job.X;
  const size_t ld = (size_t)job.ld;
  const size_t rowc = (size_t)min(row, job.nrows - 1);

  // Windows that are structurally zero on this slab of an upper triangular
  // X are skipped (applying a transform to zeros leaves zeros).
  int t0 = 0, tend = a.nwin;
  if (job.tri && !TR && DIR > 0) {
    // right sweep: X(r, win) = 0 when the window ends left of row r
    const int need = ra + job.tri_off;  // global row of the slab's first row
    const int q = need - a.c0 - 2 * K;
    if (q >= 0) t0 = q / K + 1;
  }
  if (job.tri && TR) {
    // left sweep: X(win, c) = 0 when the window starts below row c, i.e.
    // below the slab's last column
    const int last = ra + job.tri_off + 63;
    if (DIR > 0) {
      tend = (a.c0 > last) ? 0 : min(a.nwin, (last - a.c0) / K + 1);
    } else {
      const int q = a.c0 - last;
      if (q > 0) t0 = (q + K - 1) / K;
    }
  }
  if (t0 >= tend) return;

  v4d xt[NT];
  v4d pre[NH];
  int cs = a.c0 + DIR * t0 * K;  // first column of the current window

  auto at = [&](size_t r, int col) -> size_t {
    return TR ? (size_t)col + r * ld : r + (size_t)col * ld;
  };
  auto load_tile = [&](int col0) -> v4d {
    v4d v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double x = X[at(rowc, col0 + g + 4 * i)];
      v[i] = rok ? x : 0.0;
    }
    return v;
  };
  auto store_tile = [&](int col0, const v4d& v) {
    if (rok) {
#pragma unroll
      for (int i = 0; i < 4; ++i) X[at((size_t)row, col0 + g + 4 * i)] = v[i];
    }
  };

#pragma unroll
  for (int t = 0; t < NT; ++t) xt[t] = load_tile(cs + 16 * t);

  for (int w = t0; w < tend; ++w) {
    const double* V = a.Vp + (size_t)(a.slot0 + w * a.slot_step) * (2 * K * K);
    const double* W = a.Wp + (size_t)(a.slot0 + w * a.slot_step) * (2 * K * K);
    // ---- step 1: P^T = V^T X^T
    v4d pt[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) pt[p] = v4d{0.0, 0.0, 0.0, 0.0};
    // only the run's nonzero tiles of V (rows tlo..thi-1, reflectors < phi)
    const int tlo = a.tlo, thi = a.thi, phi = a.phi;
    VReg<K> vr;
    vr.load(V, tlo, tid);
    __syncthreads();  // the stage buffers are free
    vr.store(stage[tlo & 1], tid);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < tlo || t >= thi) continue;
      if (t + 1 < thi) vr.load(V, t + 1, tid);
      const double* Vs = stage[t & 1];
      // per accumulator the order is still t, then kc
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (p >= phi) break;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          pt[p] = mfma4(Vs[(4 * kc + g) * K + 16 * p + c], xt[t][kc], pt[p]);
      }
      if (t + 1 < thi) vr.store(stage[(t + 1) & 1], tid);
      __syncthreads();
    }
    // prefetch the columns entering the next window
    const int ncs = cs + DIR * K;
    if (w + 1 < tend) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
        pre[h] = load_tile((DIR > 0 ? ncs + K : ncs) + 16 * h);
    }
    // ---- step 2: X^T -= W P^T
    WReg<K> wr;
    wr.load(W, 0, tid);
    wr.store(stage[0], tid);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (p >= phi) continue;
      if (p + 1 < phi) wr.load(W, p + 1, tid);
      const double* Ws = stage[p & 1];
      // per accumulator the order is still p, then kc
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t < tlo || t >= thi) continue;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          xt[t] = mfma4(Ws[(4 * kc + g) * 2 * K + 16 * t + c], pt[p][kc], xt[t]);
      }
      if (p + 1 < phi) wr.store(stage[(p + 1) & 1], tid);
      __syncthreads();
    }
    // ---- advance: store the leaving half, shift the carry, take the entering half
    if (w + 1 < tend) {
      if (DIR > 0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) store_tile(cs + 16 * h, xt[h]);
#pragma unroll
        for (int h = 0; h < NH; ++h) { xt[h] = xt[h + NH]; xt[h + NH] = pre[h]; }
      } else {
#pragma unroll
        for (int h = 0; h < NH; ++h) store_tile(cs + K + 16 * h, xt[h + NH]);
#pragma unroll
        for (int h = 0; h < NH; ++h) { xt[h + NH] = xt[h]; xt[h] = pre[h]; }
      }
      cs = ncs;
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t) store_tile(cs + 16 * t, xt[t]);
    }
  }
}

bool sweep_supported(int k) { return k == 64 || k == 128; }

template <int K>
void launch_sweep(hipStream_t st, const SweepArgs& args, int grid, int dir, bool trans) {
  if (trans) {
    if (dir > 0) hipLaunchKernelGGL((k_sweep_rows<K, 1, 1>), dim3(grid), dim3(256), 0, st, args);
    else hipLaunchKernelGGL((k_sweep_rows<K, -1, 1>), dim3(grid), dim3(256), 0, st, args);
  } else {
    if (dir > 0) hipLaunchKernelGGL((k_sweep_rows<K, 1, 0>), dim3(grid), dim3(256), 0, st, args);
    else hipLaunchKernelGGL((k_sweep_rows<K, -1, 0>), dim3(grid), dim3(256), 0, st, args);
  }
}

void sweep_rows(hipStream_t st, const SweepArgs& args, int k, int dir, bool trans) {
  if (args.nwin <= 0 || args.njobs <= 0) return;
  const int grid = args.job[args.njobs - 1].wg0 +
                   (args.job[args.njobs - 1].nrows + 63) / 64;
  if (grid <= 0) return;
  if (k == 128) launch_sweep<128>(st, args, grid, dir, trans);
  else launch_sweep<64>(st, args, grid, dir, trans);
}

}  // namespace htk
