// ht_trsv.hip -- overflow-safe upper triangular solve B x = 2^{-E} c behind
// the opposite reflectors (Sec. 2.2, step c of Sec. 3.2.2).
//
// Rows are split into 64-row blocks.  One "solver" workgroup walks the blocks
// bottom-up and performs the substitution: for block i it adds the products
// of the kLA block columns right of the diagonal (tiles prefetched one step
// ahead and staged in LDS, x of those blocks kept in LDS), takes the sum over
// all farther block columns from a helper, and runs the 64-row back
// substitution of the diagonal block on one wavefront.  Every other
// workgroup is a helper that owns block rows and streams their far tiles
// B(i, c), c >= i+kLA+1, as the solver publishes x_c, then publishes the far
// sum of block i ahead of the solver's arrival.  The launch is cooperative,
// so every workgroup is resident and the spin-waits terminate.
//
// Workgroups have 1024 threads (16 wavefronts); a 64 x 64 tile is read with
// lanes on consecutive rows (512 contiguous bytes per column) and 4 columns
// per wavefront, so a thread has only 4 loads in flight per tile.
//
// Publication uses 64-bit words that carry the call's epoch in the upper
// half and 32 data bits in the lower half (a double takes two words).  A
// 64-bit store is single-copy atomic, so a reader that sees the current epoch
// in every word of a block has the whole block: one round trip, no fences.
//
// Scaling: the solution of a triangular system with a small diagonal grows
// geometrically and overflows FP64 (the ill-conditioned test pencils reach
// 1e+300 within a few hundred rows).  Every block carries its own
// power-of-two exponent e_i (true value = x_i 2^{e_i}); sums align exponents
// to their largest term, and the substitution inside a block rescales by
// 2^-600 whenever an entry would exceed 2^600 times its pivot.  The final
// pass shifts all blocks to the largest exponent E (entries smaller by more
// than the FP64 range become zero) and reports E: only the direction of x
// enters an opposite reflector (Lemma 2.1).
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

constexpr int kLA = 3;       // near block columns handled by the solver
constexpr int kRing = 4;     // x blocks kept in LDS (>= kLA + 1)
constexpr int kWords = 130;  // per block: 128 words for 64 doubles + exponent + pad
constexpr int kNT = 1024;    // threads per workgroup
constexpr int kNW = kNT / 64;
constexpr int kCPW = 64 / kNW;  // tile columns per wavefront
constexpr int kTLD = 65;     // LDS leading dimension of a staged tile

struct TrsvArgs {
  int m;
  const double* B;
  int ldb;
  const double* c;
  double* x;        // plain copy of the solution blocks (for later kernels)
  int* exps;        // plain copy of the block exponents
  uint64_t* xll;    // published x blocks (epoch-tagged words)
  uint64_t* all;    // published far sums
  uint32_t epoch;
};

__device__ __forceinline__ uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_word(uint64_t* p, uint32_t epoch, uint32_t v) {
  __hip_atomic_store(p, ((uint64_t)epoch << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool word_ok(uint64_t w, uint32_t epoch) {
  return (uint32_t)(w >> 32) == epoch;
}
__device__ __forceinline__ double join_words(uint64_t lo, uint64_t hi) {
  return __hiloint2double((int)(uint32_t)hi, (int)(uint32_t)lo);
}

// Publish a 64-double block (lane l holds entry l) and an exponent.
__device__ __forceinline__ void publish_block(uint64_t* blk, uint32_t epoch, double v, int e,
                                              int lane) {
  st_word(blk + 2 * lane, epoch, (uint32_t)__double2loint(v));
  st_word(blk + 2 * lane + 1, epoch, (uint32_t)__double2hiint(v));
  if (lane == 0) st_word(blk + 128, epoch, (uint32_t)e);
}

// This thread's part of tile B(block row ib, block column cb):
// t[q] = B(64 ib + lane, 64 cb + kCPW wave + q); zero outside the matrix and,
// for the diagonal block, below the diagonal.  Addresses are clamped so every
// load is in bounds and no load sits behind a branch.
__device__ __forceinline__ void load_tile(const TrsvArgs& a, int ib, int cb, bool diag, int lane,
                                          int wave, double t[kCPW]) {
  const int row = ib * 64 + lane;
  const int rowc = min(row, a.m - 1);
  const int cbase = cb * 64 + wave * kCPW;
#pragma unroll
  for (int q = 0; q < kCPW; ++q) {
    const int col = cbase + q;
    const bool ok = row < a.m && col < a.m && cb >= 0 && (!diag || col >= row);
    const int colc = min(max(col, 0), a.m - 1);
    const double v = a.B[(size_t)rowc + (size_t)colc * a.ldb];
    t[q] = ok ? v : 0.0;
  }
}

// Back substitution of one 64-row diagonal block on one wavefront: lane l
// holds row l of the right-hand side; dg is the block (column-major, leading
// dimension kTLD) in LDS.  Returns the lane's entry of x and updates the
// block exponent e.  The fast pass assumes no entry exceeds 2^600 times its
// pivot; if any entry of the result is that large or not finite, the block is
// redone with a per-row rescaling by 2^-600.
__device__ __forceinline__ double diag_solve(double rhs0, const double* dg, int nr, int lane,
                                             int& e) {
  const bool live = lane < nr;
  const double d_own = live ? dg[lane * kTLD + lane] : 1.0;
  // a zero pivot survives only when ||B||_F = 0; any direction then works
  const double dinv = (d_own != 0.0) ? 1.0 / d_own : 1.0;
  double rhs = rhs0, xo = 0.0;
#pragma unroll
  for (int r = 63; r >= 0; --r) {
    if (r < nr) {
      const double xr = readlane_d(rhs, r) * readlane_d(dinv, r);
      if (lane == r) xo = xr;
      rhs = fma(-dg[r * kTLD + lane], xr, rhs);
    }
  }
  const bool bad = live && !(fabs(xo) <= kBig);
  if (!__any(bad)) return live ? xo : 0.0;
  // careful pass
  rhs = rhs0;
  xo = 0.0;
  for (int r = nr - 1; r >= 0; --r) {
    double t = readlane_d(rhs, r);
    const double dr0 = readlane_d(d_own, r);
    const double dr = (dr0 != 0.0) ? dr0 : 1.0;
    int guard = 0;
    while (!(fabs(t) <= kBig * fabs(dr)) && guard < 8) {
      rhs *= kShrink;
      xo *= kShrink;
      e += kShrinkExp;
      t = readlane_d(rhs, r);
      ++guard;
    }
    const double xr = t * readlane_d(dinv, r);
    if (lane == r) xo = xr;
    rhs = fma(-dg[r * kTLD + lane], xr, rhs);
  }
  return live ? xo : 0.0;
}

__global__ __launch_bounds__(kNT) void k_trsv_la(TrsvArgs a) {
  const int nb = (a.m + 63) >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nfar = nb - 1 - kLA;  // block rows 0..nfar-1 take far sums from helpers
  __shared__ double red[kNW][64];

  if (blockIdx.x == 0) {
    // ----------------------------- solver -----------------------------
    __shared__ double ring[kRing][64];
    __shared__ int ringe[kRing];
    __shared__ double tl[kLA][64 * kTLD];  // near tiles of the current block
    __shared__ double dg[64 * kTLD];       // its diagonal block
    __shared__ int sfE;
    double tn[kLA][kCPW], dn[kCPW];
    double facc = 0.0;
    int fE = 0;
    uint64_t wlo = 0, whi = 0, wex = 0;  // pending far-sum words (wave 0)
    // stage the first block's tiles
#pragma unroll
    for (int t = 0; t < kLA; ++t) load_tile(a, nb - 1, nb + t, false, lane, wave, tn[t]);
    load_tile(a, nb - 1, nb - 1, true, lane, wave, dn);
#pragma unroll
    for (int t = 0; t < kLA; ++t)
#pragma unroll
      for (int q = 0; q < kCPW; ++q) tl[t][(wave * kCPW + q) * kTLD + lane] = tn[t][q];
#pragma unroll
    for (int q = 0; q < kCPW; ++q) dg[(wave * kCPW + q) * kTLD + lane] = dn[q];
    __syncthreads();
    for (int ib = nb - 1; ib >= 0; --ib) {
      const int r0 = ib * 64;
      const int nr = min(64, a.m - r0);
      const int row = r0 + lane;
      const bool want_far = (ib - 1 >= 0) && (ib - 1 < nfar);
      // issue the loads of the next block's far sum and tiles (used next step)
      if (wave == 0 && want_far) {
        const uint64_t* blk = a.all + (size_t)(ib - 1) * kWords;
        wlo = ld_word(blk + 2 * lane);
        whi = ld_word(blk + 2 * lane + 1);
        wex = ld_word(blk + 128);
      }
      const double crow = a.c[min(row, a.m - 1)];
      if (ib > 0) {
#pragma unroll
        for (int t = 0; t < kLA; ++t) load_tile(a, ib - 1, ib + t, false, lane, wave, tn[t]);
        load_tile(a, ib - 1, ib - 1, true, lane, wave, dn);
      }
      // near products: block columns ib+1 .. ib+kLA (tiles and x in LDS)
      int E = fE;
#pragma unroll
      for (int t = 0; t < kLA; ++t)
        if (ib + 1 + t < nb) E = max(E, ringe[(ib + 1 + t) % kRing]);
      double part = 0.0;
#pragma unroll
      for (int t = 0; t < kLA; ++t) {
        const int cb = ib + 1 + t;
        if (cb < nb) {
          const double* xr = ring[cb % kRing] + wave * kCPW;
          const double* tp = tl[t] + wave * kCPW * kTLD + lane;
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < kCPW; ++q) s = fma(tp[q * kTLD], xr[q], s);
          part = fma(s, ldexp(1.0, ringe[cb % kRing] - E), part);
        }
      }
      red[wave][lane] = part;
      __syncthreads();
      if (wave == 0) {
        const bool live = lane < nr;
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < kNW; ++w) tot += red[w][lane];
        const double rhs = live ? (ldexp(crow, -E) - tot - ldexp(facc, fE - E)) : 0.0;
        int e = E;
        const double xo = diag_solve(rhs, dg, nr, lane, e);
        ring[ib % kRing][lane] = xo;
        if (lane == 0) ringe[ib % kRing] = e;
        if (live) a.x[row] = xo;
        if (lane == 0) a.exps[ib] = e;
        publish_block(a.xll + (size_t)ib * kWords, a.epoch, xo, e, lane);
        // the far sum of the next block: complete the loads issued above
        if (want_far) {
          while (!__all(word_ok(wlo, a.epoch) && word_ok(whi, a.epoch) &&
                        word_ok(wex, a.epoch))) {
            __builtin_amdgcn_s_sleep(1);
            const uint64_t* blk = a.all + (size_t)(ib - 1) * kWords;
            wlo = ld_word(blk + 2 * lane);
            whi = ld_word(blk + 2 * lane + 1);
            wex = ld_word(blk + 128);
          }
          facc = join_words(wlo, whi);
          fE = (int)(uint32_t)wex;
        } else {
          facc = 0.0;
          fE = 0;
        }
        if (lane == 0) sfE = fE;
      }
      __syncthreads();
      fE = sfE;  // every wave needs the far exponent; facc stays in wave 0
      // stage the next block's tiles
      if (ib > 0) {
#pragma unroll
        for (int t = 0; t < kLA; ++t)
#pragma unroll
          for (int q = 0; q < kCPW; ++q) tl[t][(wave * kCPW + q) * kTLD + lane] = tn[t][q];
#pragma unroll
        for (int q = 0; q < kCPW; ++q) dg[(wave * kCPW + q) * kTLD + lane] = dn[q];
      }
      __syncthreads();
    }
    return;
  }

  // ------------------------------ helpers ------------------------------
  // Tiles and x words are double-buffered (A, B) so every load has two tile
  // steps to arrive.  Each wavefront owns kCPW columns of every tile and reads
  // their 2 kCPW words (lanes 0..2kCPW-1) and the exponent word (other lanes).
  const int H = gridDim.x - 1;
  const int h = blockIdx.x - 1;
  const int widx = (lane < 2 * kCPW) ? (wave * 2 * kCPW + lane) : 128;
  for (int r = nfar - 1 - h; r >= 0; r -= H) {
    double acc = 0.0;
    int E = 0;
    const int cend = r + 1 + kLA;  // last block column of the far part
    double tA[kCPW], tB[kCPW];
    uint64_t wA, wB = 0;
    load_tile(a, r, nb - 1, false, lane, wave, tA);
    wA = ld_word(a.xll + (size_t)(nb - 1) * kWords + widx);
    if (nb - 2 >= cend) {
      load_tile(a, r, nb - 2, false, lane, wave, tB);
      wB = ld_word(a.xll + (size_t)(nb - 2) * kWords + widx);
    }
    auto consume = [&](const double* t, uint64_t w, int cb) {
      while (!__all(lane > 2 * kCPW || word_ok(w, a.epoch))) {
        __builtin_amdgcn_s_sleep(1);
        w = ld_word(a.xll + (size_t)cb * kWords + widx);
      }
      const int ec = (int)(uint32_t)__shfl(w, 2 * kCPW, 64);
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kCPW; ++q) {
        const uint64_t lo = __shfl(w, 2 * q, 64);
        const uint64_t hi = __shfl(w, 2 * q + 1, 64);
        s = fma(t[q], join_words(lo, hi), s);
      }
      if (ec > E) { acc = ldexp(acc, E - ec); E = ec; }
      acc = fma(s, ldexp(1.0, ec - E), acc);
    };
    for (int cb = nb - 1; cb >= cend; cb -= 2) {
      consume(tA, wA, cb);
      if (cb - 2 >= cend) {
        load_tile(a, r, cb - 2, false, lane, wave, tA);
        wA = ld_word(a.xll + (size_t)(cb - 2) * kWords + widx);
      }
      if (cb - 1 >= cend) {
        consume(tB, wB, cb - 1);
        if (cb - 3 >= cend) {
          load_tile(a, r, cb - 3, false, lane, wave, tB);
          wB = ld_word(a.xll + (size_t)(cb - 3) * kWords + widx);
        }
      }
    }
    // every wave saw the same exponents, so the partial sums share E
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < kNW; ++w) tot += red[w][lane];
      publish_block(a.all + (size_t)r * kWords, a.epoch, tot, E, lane);
    }
    __syncthreads();
  }
}

// Shift blocks to the largest exponent; E_dev = that exponent.
__global__ __launch_bounds__(1024) void k_trsv_fin(int m, double* x, const int* exps, int* E_dev) {
  __shared__ int smax[16];
  const int nb = (m + 63) >> 6;
  int e = 0;
  for (int i = threadIdx.x; i < nb; i += 1024) e = max(e, exps[i]);
  e = wave_max_i(e);
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = e;
  __syncthreads();
  int E = 0;
  for (int i = 0; i < 16; ++i) E = max(E, smax[i]);
  for (int i = threadIdx.x; i < m; i += 1024) {
    const int d = exps[i >> 6] - E;
    if (d != 0) x[i] = ldexp(x[i], d);
  }
  if (threadIdx.x == 0) E_dev[0] = E;
}

static int trsv_grid_cap() {
  static int cap = 0;
  if (cap == 0) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_trsv_la, kNT, 0) != hipSuccess ||
        per < 1)
      per = 1;
    cap = per * num_cus();
  }
  return cap;
}

// flags area layout: exps[nb] ints, then (256-aligned) xll[(nb+1) * kWords]
// and all[(nb+1) * kWords] 64-bit words.
size_t trsv_flag_bytes(int m) {
  const size_t nb = (size_t)(m + 63) / 64 + 1;
  return 256 + nb * sizeof(int) + 256 + 2 * nb * kWords * sizeof(uint64_t) + 256;
}

void trsv_upper_scaled(hipStream_t st, int m, const double* B, int ldb, const double* c,
                       double* x, int* flags, int epoch, int* E_dev) {
  if (m <= 0) return;
  const int nb = (m + 63) / 64;
  int* exps = flags;
  uint64_t* xll = (uint64_t*)(((uintptr_t)(flags + nb + 1) + 255) & ~(uintptr_t)255);
  uint64_t* all = xll + (size_t)(nb + 1) * kWords;
  const int nfar = nb - 1 - kLA;
  const int helpers = nfar > 0 ? std::min(nfar, trsv_grid_cap() - 1) : 0;
  TrsvArgs args{m, B, ldb, c, x, exps, xll, all, (uint32_t)epoch};
  void* kargs[] = {(void*)&args};
  (void)hipLaunchCooperativeKernel((const void*)k_trsv_la, dim3(1 + helpers), dim3(kNT), kargs,
                                   0, st);
  hipLaunchKernelGGL(k_trsv_fin, dim3(1), dim3(1024), 0, st, m, x, exps, E_dev);
}

}  // namespace htk
