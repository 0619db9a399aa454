// ht_chain.hip -- small Householder factorisations for the absorption chains
// of Sec. 3.3: QL of the blocks of V2 (step b of Sec. 3.3.1), QR of the
// blocks of U2 (step b of Sec. 3.3.2), RQ of the subdiagonal blocks of B when
// restoring it from the right (step e), QR when restoring it from the left
// (step f).  RQ is done as QL of the transposed block.
//
// k_chain_reg: one workgroup factors one w x k tile (w <= 2 KMAX,
// k <= KMAX) held in registers, one workgroup barrier per reflector;
// k_chain_blk (further down) factors the larger tiles in panels of 16 columns
// with FP64 MFMA block updates.  The orthogonal factor is returned in regular WY form
// Qf = I - V W^T (Sec. 2.4), reflectors in the order they are computed, so
//   QR:  tile = Qf [R; 0],   QL:  tile = Qf [0; L].
// W is accumulated alongside the factorisation:  with Qf_i = I - V_i W_i^T,
//   Qf_i (I - tau v v^T) = I - [V_i v] [(I - tau v v^T) W_i, tau v]^T,
// so once column c has produced its reflector, the registers that held it
// hold column c of W and take the later reflectors like the columns still
// to be reduced.
//
// Register layout.  KMAX/8 wavefronts; in each, lane l = 32 h + r_l works on
// rows r_l RQ .. r_l RQ + RQ-1 (RQ = 2 KMAX / 32) of the four columns
// 8 wave + 4 h + (0..3).  A wavefront thus spans all rows, and the column
// sums of a reflector step are reduced inside each 32-lane half with DPP row
// operations and v_permlane16_swap, without LDS.  Per reflector:
//   1. the wavefront owning column i reduces its norm, forms the reflector
//      (sign convention of LAPACK's dlarfg: beta = -sign(alpha) ||x||;
//      columns outside [2^-450, 2^450] are scaled by an exact power of two
//      first) and writes v and the finished column of the factor (R or L)
//      to one of two pairs of LDS buffers;
//   2. one workgroup barrier;
//   3. every wavefront reads v for its rows, forms the four column dots,
//      reduces them and applies the rank-1 update; each wavefront also
//      stores 16 rows of v and of the factor column to global memory, so
//      the owner's next reflector does not wait behind those stores.
// The owner of column i+1 proceeds to step 1 of the next reflector as soon as
// its own update is done; the double buffers make the single barrier enough.
// v sits in LDS with lane rl's RQ rows strided by 32 (entry q of lane rl at
// q * 32 + rl), so the reads of a wavefront hit consecutive banks.
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

namespace {

__device__ __forceinline__ size_t tidx(int r, int c, int ld, int trans) {
  return trans ? ((size_t)c + (size_t)r * ld) : ((size_t)r + (size_t)c * ld);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// DPP controls: quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1]
// (lane ^ 2), row_half_mirror (lane i of 8 <- 7 - i), row_mirror (lane i of
// 16 <- 15 - i).  Applied in this order, each step combines disjoint groups,
// so after the four steps every lane of a 16-lane row holds the row's result.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

__device__ __forceinline__ double row_sum16(double x) {
  x += dpp_d<kDppXor1>(x);
  x += dpp_d<kDppXor2>(x);
  x += dpp_d<kDppHalfMirror>(x);
  x += dpp_d<kDppMirror>(x);
  return x;
}
__device__ __forceinline__ double row_max16(double x) {
  x = fmax(x, dpp_d<kDppXor1>(x));
  x = fmax(x, dpp_d<kDppXor2>(x));
  x = fmax(x, dpp_d<kDppHalfMirror>(x));
  x = fmax(x, dpp_d<kDppMirror>(x));
  return x;
}

// v_permlane16_swap on a pair of doubles: for each pair of 16-lane rows
// (0,1) and (2,3), row 1 of x and row 0 of y trade places.  Afterwards
//   x = {row e: x_e,  row o: y_e},   y = {row e: x_o,  row o: y_o}.
__device__ __forceinline__ void swap16(double& x, double& y) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false,
                                                   false);
  x = __hiloint2double((int)hi[0], (int)lo[0]);
  y = __hiloint2double((int)hi[1], (int)lo[1]);
}

// Sum / max over each 32-lane half, result in every lane of the half.
__device__ __forceinline__ double half_sum(double x) {
  x = row_sum16(x);
  double y = x;
  swap16(x, y);
  return x + y;
}
__device__ __forceinline__ double half_max(double x) {
  x = row_max16(x);
  double y = x;
  swap16(x, y);
  return fmax(x, y);
}

}  // namespace

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KMAX>
__global__ __launch_bounds__(KMAX * 8) void k_chain_reg(ChainJobs jobs) {
  // one tile per workgroup
  const ChainJob& jb = jobs.job[blockIdx.x];
  const int mode = jb.mode, w = jb.w, k = jb.k, ldx = jb.ldx, trans = jb.trans, ldo = jb.ldo;
  double* __restrict__ X = jb.X;
  double* __restrict__ Vout = jb.V;
  double* __restrict__ Wout = jb.W;
  constexpr int RQ = 2 * KMAX / 32;  // rows per lane
  constexpr int CJ = 4;              // columns per lane
  __shared__ double vbuf[2][2 * KMAX];  // v, strided layout (vslot)
  __shared__ double rbuf[2][2 * KMAX];  // the factor column, by row
  __shared__ double tbuf[2];
  auto vslot = [](int r) { return (r % RQ) * 32 + r / RQ; };

  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int h = lane >> 5, rl = lane & 31;
  const int rbase = rl * RQ;
  const int cbase = 8 * wv + 4 * h;

  // reg[q][j]: row rbase + q, column cbase + j (a 4-vector per row, so that
  // the owner can pick column i's entries by a vector element select)
  v4d reg[RQ];
#pragma unroll
  for (int q = 0; q < RQ; ++q)
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int r = rbase + q, c = cbase + j;
      reg[q][j] = (r < w && c < k) ? X[tidx(r, c, ldx, trans)] : 0.0;
    }

  // Step 1 for the reflector of `step`, run by the owning wavefront only.
  auto form = [&](int step) __attribute__((always_inline)) {
    const int i = (mode == 0) ? step : (k - 1 - step);
    const int p = (mode == 0) ? i : (w - k + i);
    const int x0 = (mode == 0) ? p + 1 : 0;  // x-part rows [x0, x1)
    const int x1 = (mode == 0) ? w : p;
    const int ji = i & 3, hi = (i >> 2) & 1;
    double x[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) {  // select tree (no indexed register access)
      const double a = (ji & 1) ? reg[q][1] : reg[q][0];
      const double b = (ji & 1) ? reg[q][3] : reg[q][2];
      x[q] = (ji & 2) ? b : a;
    }
    double ss = 0.0, am = 0.0, ap = 0.0;
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int r = rbase + q;
      const double xv = (r >= x0 && r < x1) ? x[q] : 0.0;
      am = fmax(am, fabs(xv));
      ss = fma(xv, xv, ss);
      if (q == p % RQ) ap = x[q];
    }
    ss = readlane_d(half_sum(ss), 32 * hi);
    am = readlane_d(half_max(am), 32 * hi);
    const double alpha = readlane_d(ap, 32 * hi + p / RQ);
    // tiny or huge columns: redo the sum of squares with an exact
    // power-of-two scaling into the safe range
    const double sc = safe_scale(fmax(am, fabs(alpha)));
    if (sc != 1.0) {
      double s2 = 0.0;
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int r = rbase + q;
        const double t = (r >= x0 && r < x1) ? x[q] * sc : 0.0;
        s2 = fma(t, t, s2);
      }
      ss = readlane_d(half_sum(s2), 32 * hi);
    }
    const Refl rf0 = make_refl_ss(alpha * sc, ss);
    Refl rf = rf0;
    rf.scal = rf0.scal * sc;   // v = x * scal for the unscaled x
    rf.beta = rf0.beta / sc;
    if (h == hi) {
      double* vb = vbuf[step & 1];
      double* rb = rbuf[step & 1];
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int r = rbase + q;
        const bool inx = r >= x0 && r < x1;
        vb[vslot(r)] = (r == p) ? 1.0 : (inx ? x[q] * rf.scal : 0.0);
        // column i of the factor (R or L)
        rb[r] = (r == p) ? rf.beta : (inx ? 0.0 : x[q]);
      }
      if (rl == 0) tbuf[step & 1] = rf.tau;
    }
  };

  if (wv == (((mode == 0) ? 0 : (k - 1)) >> 3)) form(0);

  for (int step = 0; step < k; ++step) {
    const int i = (mode == 0) ? step : (k - 1 - step);
    __syncthreads();
    const double tau = tbuf[step & 1];
    double v[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) v[q] = vbuf[step & 1][vslot(rbase + q)];
    {
      // reflector `step` and column i of the factor: 16 rows per wavefront
      const int r = 16 * wv + (lane & 15);
      if (lane < 32 && r < w) {
        if (lane < 16) Vout[(size_t)r + (size_t)step * ldo] = vbuf[step & 1][vslot(r)];
        else X[tidx(r, i, ldx, trans)] = rbuf[step & 1][r];
      }
    }
    double d[CJ];
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < RQ; ++q) s = fma(v[q], reg[q][j], s);
      d[j] = s;
    }
    // reduce the four column dots over the 32 lanes of each half:
    // pairwise across the two rows (scattering d0/d1 and d2/d3 to the even
    // and odd rows), across each row, then gathered back into every lane
    swap16(d[0], d[1]);
    swap16(d[2], d[3]);
    double e0 = row_sum16(d[0] + d[1]);
    double e1 = row_sum16(d[2] + d[3]);
    double f0 = e0, f1 = e1;
    swap16(e0, f0);  // e0 = sum of column 0 everywhere, f0 = column 1
    swap16(e1, f1);
    const double dd[CJ] = {e0, f0, e1, f1};
    if (wv == (i >> 3)) {
      // the owner wavefront: column i becomes column `step` of W
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        const bool isi = (cbase + j) == i;
        const double f = tau * dd[j];
#pragma unroll
        for (int q = 0; q < RQ; ++q) reg[q][j] = isi ? tau * v[q] : fma(-f, v[q], reg[q][j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        const double f = tau * dd[j];
#pragma unroll
        for (int q = 0; q < RQ; ++q) reg[q][j] = fma(-f, v[q], reg[q][j]);
      }
    }
    if (step + 1 < k) {
      const int in = (mode == 0) ? step + 1 : (k - 2 - step);
      if (wv == (in >> 3)) form(step + 1);
    }
  }

  // registers now hold W; column c was produced at step s(c)
#pragma unroll
  for (int j = 0; j < CJ; ++j) {
    const int c = cbase + j;
    if (c < k) {
      const int sc = (mode == 0) ? c : (k - 1 - c);
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int r = rbase + q;
        if (r < w) Wout[(size_t)r + (size_t)sc * ldo] = reg[q][j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Blocked factorisation: panels of 16 columns, FP64 MFMA block updates.
//
// The tile is taken in its QR orientation: for QL the rows and columns are
// reversed (logical row r = physical row w-1-r, logical column c = physical
// column k-1-c), which turns the QL factorisation into a QR factorisation
// with the same reflectors in the same order.  With Qf = I - V W^T after the
// reflectors of panels 0..p-1, panel p (columns 16p..16p+15) is factored by
// the wavefront that holds it, one reflector after the other as above (its
// finished columns becoming columns of W and taking the panel's later
// reflectors); the panel's factor is then Qp = I - Vp Wp^T, and every other
// column, still to be reduced or already a column of W, takes Qp^T at once:
//   C <- C - Wp (Vp^T C),
// two 16-deep products on v_mfma_f64_16x16x4f64.  The result equals the
// reflector-by-reflector scheme up to rounding (the same reflectors, the
// same W).
//
// Layouts.  Eight wavefronts; wavefront wv holds logical columns 16wv ..
// 16wv+15 in MFMA accumulator layout: lane l = 16g + c, register xt[t][i] =
// row 16t + g + 4i of column 16wv + c, which is also the B-operand layout of
// the k-chunks of a product over rows.  While it factors its panel, the
// owning wavefront holds the panel in row layout instead, in the same
// registers: xt[j][q] = row l + 64q of a panel column.  The reflectors run
// four to a loop pass with pivot columns xt[0..3], after which the columns
// rotate by four registers (four rotations restore the order): four
// unrolled reflector steps instead of sixteen keep the loop inside the
// instruction cache.  Reflector sums over rows are reductions over the 64
// lanes; the 16 column sums of a reflector step are reduce-scattered
// (v_permlane32/16_swap, then DPP mirrors) so that lane 4j ends with the
// sum of column j.
// ---------------------------------------------------------------------------
namespace {

constexpr int kBlkNT = 512;  // threads: eight wavefronts of 16 columns
constexpr int kLP = 258;     // leading dimension of the panel and Vp in LDS
constexpr int kLW = 272;     // leading dimension of -Wp in LDS

__device__ __forceinline__ v4d mfma4(double a, double b, v4d acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ void swap32(double& x, double& y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false,
                                                   false);
  x = __hiloint2double((int)hi[0], (int)lo[0]);
  y = __hiloint2double((int)hi[1], (int)lo[1]);
}

// DPP move without an old value (every lane has a source under the
// controls used here).
template <int CTRL>
__device__ __forceinline__ double dpp_m(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_total16(double x) {
  x += dpp_m<kDppXor1>(x);
  x += dpp_m<kDppXor2>(x);
  x += dpp_m<kDppHalfMirror>(x);
  x += dpp_m<kDppMirror>(x);
  return x;
}

// Sum over all 64 lanes, in every lane.
__device__ __forceinline__ double wave_total(double x) {
  x = row_total16(x);
  double y = x;
  swap16(x, y);
  x += y;
  y = x;
  swap32(x, y);
  return x + y;
}
__device__ __forceinline__ double wave_maxall(double x) {
  x = row_max16(x);
  double y = x;
  swap16(x, y);
  x = fmax(x, y);
  y = x;
  swap32(x, y);
  return fmax(x, y);
}

// One reduce-scatter step inside 16-lane rows: lanes with `upper` set keep
// b's sum, the others a's; the partner lane is given by the DPP control.
template <int CTRL>
__device__ __forceinline__ double rs_pair(double a, double b, bool upper) {
  const double send = upper ? a : b;
  const double keep = upper ? b : a;
  return keep + dpp_m<CTRL>(send);
}

// d[0..15]: per-lane partial sums of 16 quantities.  Returns, in lane l, the
// total over all lanes of quantity (l >> 2) & 15.
__device__ __forceinline__ double reduce_scatter16(double (&d)[16], int lane) {
  double u[8], w4[4], y2[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double a = d[i], b = d[i + 8];
    swap32(a, b);
    u[i] = a + b;  // lanes 0-31: quantity i, lanes 32-63: i + 8
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double a = u[i], b = u[i + 4];
    swap16(a, b);
    w4[i] = a + b;  // even rows: u[i], odd rows: u[i + 4]
  }
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) y2[i] = rs_pair<kDppMirror>(w4[i], w4[i + 2], b3);
  double z = rs_pair<kDppHalfMirror>(y2[0], y2[1], b2);
  z += dpp_m<kDppXor2>(z);
  z += dpp_m<kDppXor1>(z);
  return z;
}

struct BlkLds {
  double pw[16 * kLW];  // the panel (ld kLP) while it is factored, then -Wp (ld kLW)
  double vs[16 * kLP];  // Vp, column-major
  double rs[16 * 128];  // the panel's factor columns, rows 0..pivot
};

}  // namespace

__global__ __launch_bounds__(kBlkNT) void k_chain_blk(ChainJobs jobs) {
  const ChainJob& jb = jobs.job[blockIdx.x];
  const int mode = jb.mode, w = jb.w, k = jb.k, ldx = jb.ldx, trans = jb.trans, ldo = jb.ldo;
  double* __restrict__ X = jb.X;
  double* __restrict__ Vout = jb.V;
  double* __restrict__ Wout = jb.W;
  __shared__ BlkLds S;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int mycol = 16 * wv + c;
  auto prow = [&](int r) { return mode == 0 ? r : (w - 1 - r); };
  auto pcol = [&](int cl) { return mode == 0 ? cl : (k - 1 - cl); };

  // loads from clamped addresses, then masked (no divergent branches)
  v4d xt[16];
  {
    const int cc = pcol(min(mycol, k - 1));
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * t + g + 4 * i;
        const double x = X[tidx(prow(min(r, w - 1)), cc, ldx, trans)];
        xt[t][i] = (r < w && mycol < k) ? x : 0.0;
      }
  }

  const int np = (k + 15) >> 4;
  for (int p = 0; p < np; ++p) {
    // the owner hands its columns over in LDS (panel column-major, ld kLP)
    if (wv == p) {
#pragma unroll
      for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) S.pw[c * kLP + 16 * t + g + 4 * i] = xt[t][i];
    }
    __syncthreads();
    if (wv == p) {
      // row layout: xt[j][q] = row lane + 64 q of panel column j
#pragma unroll
      for (int j = 0; j < 16; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) xt[j][q] = S.pw[j * kLP + lane + 64 * q];
      // One reflector: panel column j (logical column 16p + j) is xt[ji].
      auto reflect = [&](const int j, const int ji) __attribute__((always_inline)) {
        const int pr = 16 * p + j;  // pivot row = logical column
        if (pr >= k) {
#pragma unroll
          for (int q = 0; q < 4; ++q) S.vs[j * kLP + lane + 64 * q] = 0.0;
          return;
        }
        double ss = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double xv = (lane + 64 * q > pr) ? xt[ji][q] : 0.0;
          ss = fma(xv, xv, ss);
        }
        ss = wave_total(ss);
        const double xa = (pr >= 64) ? xt[ji][1] : xt[ji][0];
        const double alpha = readlane_d(xa, pr & 63);
        // a sum of squares in [2^-900, 2^900] with a pivot below 2^450 needs
        // no scaling (the largest entry is then within [2^-454, 2^450] and
        // alpha^2 + ss cannot overflow); otherwise bring the column into
        // range by an exact power of two first
        double sc = 1.0, isc = 1.0;
        if (!(ss >= 0x1.0p-900 && ss <= 0x1.0p900 && fabs(alpha) <= 0x1.0p450)) {
          double am = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            am = fmax(am, (lane + 64 * q > pr) ? fabs(xt[ji][q]) : 0.0);
          am = wave_maxall(am);
          sc = safe_scale(fmax(am, fabs(alpha)));
          if (sc != 1.0) {
            isc = (sc > 1.0) ? 0x1.0p-600 : 0x1.0p600;
            double s2 = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const double xv = (lane + 64 * q > pr) ? xt[ji][q] * sc : 0.0;
              s2 = fma(xv, xv, s2);
            }
            ss = wave_total(s2);
          }
        }
        const Refl rf = make_refl_ss(alpha * sc, ss);
        const double scal = rf.scal * sc, beta = rf.beta * isc, tau = rf.tau;
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = lane + 64 * q;
          v[q] = (r == pr) ? 1.0 : ((r > pr) ? xt[ji][q] * scal : 0.0);
          S.vs[j * kLP + r] = v[q];
        }
        // factor column: rows 0..pr (pr < 128)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int r = lane + 64 * q;
          if (r <= pr) S.rs[j * 128 + r] = (r == pr) ? beta : xt[ji][q];
        }
        // the other 15 columns take the reflector; the pivot column becomes tau v
        double d[16];
#pragma unroll
        for (int jc = 0; jc < 16; ++jc) {
          double sd = 0.0;
          if (jc != ji) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sd = fma(v[q], xt[jc][q], sd);
          }
          d[jc] = sd;
        }
        const double td = tau * reduce_scatter16(d, lane);
#pragma unroll
        for (int jc = 0; jc < 16; ++jc) {
          if (jc == ji) continue;
          const double f = readlane_d(td, 4 * jc);
#pragma unroll
          for (int q = 0; q < 4; ++q) xt[jc][q] = fma(-f, v[q], xt[jc][q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) xt[ji][q] = tau * v[q];
      };
      // four reflectors per pass; then the columns rotate by four registers
      // so that the next four pivot columns are xt[0..3]
#pragma unroll 1
      for (int j0 = 0; j0 < 16; j0 += 4) {
#pragma unroll
        for (int ji = 0; ji < 4; ++ji) reflect(j0 + ji, ji);
        const v4d t0 = xt[0], t1 = xt[1], t2 = xt[2], t3 = xt[3];
#pragma unroll
        for (int i = 0; i < 12; ++i) xt[i] = xt[i + 4];
        xt[12] = t0;
        xt[13] = t1;
        xt[14] = t2;
        xt[15] = t3;
      }
      // -Wp for the products of the other wavefronts
#pragma unroll
      for (int j = 0; j < 16; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) S.pw[j * kLW + lane + 64 * q] = -xt[j][q];
    }
    __syncthreads();
    if (wv == p) {
      // back to the MFMA layout: the panel's columns are now Wp
#pragma unroll
      for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) xt[t][i] = -S.pw[c * kLW + 16 * t + g + 4 * i];
    } else if (16 * wv < k) {
      // C <- C - Wp (Vp^T C); Vp and Wp vanish above row 16p
      v4d z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 64; ++s4)
        if (s4 >= 4 * p) z = mfma4(S.vs[c * kLP + 4 * s4 + g], xt[s4 >> 2][s4 & 3], z);
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (t >= p) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc)
            xt[t] = mfma4(S.pw[(4 * kc + g) * kLW + 16 * t + c], z[kc], xt[t]);
        }
    }
    // V and factor columns of the panel to global memory
    for (int e = tid; e < 16 * 256; e += kBlkNT) {
      const int j = e >> 8, r = e & 255, cl = 16 * p + j;
      if (cl < k && r < w) {
        Vout[(size_t)prow(r) + (size_t)cl * ldo] = S.vs[j * kLP + r];
        X[tidx(prow(r), pcol(cl), ldx, trans)] = (r <= cl) ? S.rs[j * 128 + r] : 0.0;
      }
    }
    __syncthreads();
  }
  // W (the sizes pass through an empty asm statement so that the row masks
  // of the loads are recomputed here rather than kept in registers)
  int w2 = w, k2 = k;
  __asm__ volatile("" : "+s"(w2), "+s"(k2));
  if (16 * wv < k2 && mycol < k2) {
    double* __restrict__ wcol = Wout + (size_t)mycol * ldo;
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * t + g + 4 * i;
        if (r < w2) wcol[mode == 0 ? r : (w2 - 1 - r)] = xt[t][i];
      }
  }
}

void chain_factor_jobs(hipStream_t st, const ChainJobs& jobs) {
  if (jobs.njobs <= 0) return;
  bool small = true;
  for (int i = 0; i < jobs.njobs; ++i)
    small = small && jobs.job[i].k <= 64 && jobs.job[i].w <= 128;
  // Tiles of at most 128 x 64: the register kernel (128 x 64: 92 vs 97 us).
  // Larger ones: the blocked kernel (256 x 128: 221 vs 295 us for the
  // register kernel with 128 columns; 160 x 37: 69 vs 79 us).
  if (small)
    hipLaunchKernelGGL((k_chain_reg<64>), dim3(jobs.njobs), dim3(512), 0, st, jobs);
  else
    hipLaunchKernelGGL(k_chain_blk, dim3(jobs.njobs), dim3(kBlkNT), 0, st, jobs);
}

static void launch_chain(hipStream_t st, int mode, int w, int k, double* tile, int ldt, int trans,
                         double* Vout, double* Wout, int ldo) {
  if (w <= 0 || k <= 0) return;
  ChainJobs jobs;
  jobs.njobs = 1;
  jobs.job[0] = ChainJob{mode, w, k, tile, ldt, trans, Vout, Wout, ldo};
  chain_factor_jobs(st, jobs);
}

void chain_factor(hipStream_t st, int mode, int w, int k, double* tile, int ldt, double* Vout,
                  double* Wout, int ldo) {
  launch_chain(st, mode, w, k, tile, ldt, 0, Vout, Wout, ldo);
}

void chain_factor_t(hipStream_t st, int mode, int w, int k, double* tile, int ldt, double* Vout,
                    double* Wout, int ldo) {
  launch_chain(st, mode, w, k, tile, ldt, 1, Vout, Wout, ldo);
}

}  // namespace htk
