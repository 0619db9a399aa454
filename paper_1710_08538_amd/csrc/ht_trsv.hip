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
  double* x;        // solution (plain stores; rescaled to one exponent at the end)
  int* exps;        // block exponents (plain stores)
  uint64_t* xll;    // published x blocks (epoch-tagged words)
  uint64_t* all;    // published far sums
  int* ctl;         // role and row tickets, two sets used by alternate epochs
  int* E_dev;       // exponent of the result
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
// t[q] = B(64 ib + lane, 64 cb + kCPW wave + q).  Addresses are clamped into
// the matrix and the loads carry no condition, so they all issue back to
// back; the entries outside the matrix (and below the diagonal of a diagonal
// tile) are zeroed by mask_tile when the values are used.
__device__ __forceinline__ void load_tile(const TrsvArgs& a, int ib, int cb, int lane, int wave,
                                          double t[kCPW]) {
  const int rowc = min(ib * 64 + lane, a.m - 1);
  const int cbase = cb * 64 + wave * kCPW;
#pragma unroll
  for (int q = 0; q < kCPW; ++q) {
    const int colc = min(max(cbase + q, 0), a.m - 1);
    t[q] = a.B[(size_t)rowc + (size_t)colc * a.ldb];
  }
}
__device__ __forceinline__ void mask_tile(const TrsvArgs& a, int ib, int cb, bool diag, int lane,
                                          int wave, double t[kCPW]) {
  const int row = ib * 64 + lane;
  const int cbase = cb * 64 + wave * kCPW;
#pragma unroll
  for (int q = 0; q < kCPW; ++q) {
    const int col = cbase + q;
    const bool ok = row < a.m && col < a.m && cb >= 0 && (!diag || col >= row);
    t[q] = ok ? t[q] : 0.0;
  }
}

// Stage a masked diagonal tile in LDS twice: dgu as is, dgs with column c
// divided by its pivot and the pivot itself replaced by 0, so that the fast
// substitution needs one FMA per row.  Rows beyond the matrix get pivot 1
// and no coupling.  A zero pivot survives only when ||B||_F = 0; any
// direction then works, and it is treated as 1.
__device__ __forceinline__ void stage_diag(const double t[kCPW], int lane, int wave, double* dgu,
                                           double* dgs) {
  // the wavefront's kCPW pivots, gathered into lanes 0..kCPW-1 so that one
  // division serves them all
  double piv = 1.0;
#pragma unroll
  for (int q = 0; q < kCPW; ++q) {
    const double d = readlane_d(t[q], wave * kCPW + q);
    if (lane == q) piv = d;
  }
  const double inv = (piv != 0.0) ? 1.0 / piv : 1.0;
#pragma unroll
  for (int q = 0; q < kCPW; ++q) {
    const int c = wave * kCPW + q;
    const double dinv = readlane_d(inv, q);
    dgu[c * kTLD + lane] = t[q];
    dgs[c * kTLD + lane] = (lane < c) ? t[q] * dinv : 0.0;
  }
}

// Back substitution of one 64-row diagonal block on one wavefront: lane l
// holds row l of the right-hand side (rows >= nr hold zeros).  Returns the
// lane's entry of x and updates the block exponent e.  The fast pass runs
// rhs_i -= (B_ir / B_rr) rhs_r down the rows and divides at the end; if any
// entry of the result exceeds 2^600 or is not finite, the block is redone
// from the unscaled tile with a per-row rescaling by 2^-600.
__device__ __forceinline__ double diag_solve(double rhs0, const double* dgu, const double* dgs,
                                             int nr, int lane, int& e) {
  const bool live = lane < nr;
  const double d_own = live ? dgu[lane * kTLD + lane] : 1.0;
  const double dinv = (d_own != 0.0) ? 1.0 / d_own : 1.0;
  // The scaled couplings are read from LDS 8 rows at a time, one chunk
  // ahead of the substitution (the empty asm statements keep the compiler
  // from sinking the reads next to their uses), so the dependency chain per
  // row is a readlane and an FMA.  Row 0 has no coupling (its column is 0).
  double rhs = rhs0;
  double ca[8], cb[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) ca[i] = dgs[(63 - i) * kTLD + lane];
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    const int rtop = 63 - 8 * ch;
    __asm__ volatile("" ::: "memory");
    if (ch + 1 < 8) {
#pragma unroll
      for (int i = 0; i < 8; ++i) cb[i] = dgs[(rtop - 8 - i) * kTLD + lane];
    }
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (rtop - i >= 1) rhs = fma(-ca[i], readlane_d(rhs, rtop - i), rhs);
#pragma unroll
    for (int i = 0; i < 8; ++i) ca[i] = cb[i];
  }
  const double xf = rhs * dinv;
  const bool bad = live && !(fabs(xf) <= kBig);
  if (!__any(bad)) return live ? xf : 0.0;
  // careful pass
  rhs = rhs0;
  double xo = 0.0;
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
    rhs = fma(-dgu[r * kTLD + lane], xr, rhs);
  }
  return live ? xo : 0.0;
}

// Far sum of block row r, sum over block columns cb >= r+kLA+1 of
// B(r, cb) x_cb, computed by one wavefront from the published x words.  The
// solver falls back to this when no helper has taken the row (for instance
// when no other workgroup of the launch is resident).
__device__ double far_sum_wave(const TrsvArgs& a, int r, int nb, int lane, int& E) {
  double acc = 0.0;
  E = 0;
  const int row = r * 64 + lane;  // r < nb - 1: a full block row
  for (int cb = nb - 1; cb >= r + 1 + kLA; --cb) {
    const uint64_t* blk = a.xll + (size_t)cb * kWords;
    const int ec = (int)(uint32_t)ld_word(blk + 128);
    double s = 0.0;
    for (int j = 0; j < 64; ++j) {
      const int col = cb * 64 + j;
      if (col < a.m) {
        const double xv = join_words(ld_word(blk + 2 * j), ld_word(blk + 2 * j + 1));
        s = fma(a.B[(size_t)row + (size_t)col * a.ldb], xv, s);
      }
    }
    if (ec > E) { acc = ldexp(acc, E - ec); E = ec; }
    acc = fma(s, ldexp(1.0, ec - E), acc);
  }
  return acc;
}

// One launch solves the system.  The first workgroup to start takes the
// solver role (a ticket from ctl), the others are helpers that take block
// rows from a second ticket.  Nothing waits on a workgroup that has not
// started: a helper only waits for x blocks of the solver, which runs, and
// the solver computes a far sum itself when no helper has taken that row.
__global__ __launch_bounds__(kNT) void k_trsv(TrsvArgs a) {
  const int nb = (a.m + 63) >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nfar = nb - 1 - kLA;  // block rows 0..nfar-1 take far sums from helpers
  int* tick = a.ctl + 4 * (a.epoch & 1);
  __shared__ double red[kNW][64];
  __shared__ int sticket;
  if (threadIdx.x == 0) sticket = atomicAdd(tick, 1);
  __syncthreads();
  const int role = sticket;
  __syncthreads();

  if (role == 0) {
    // ----------------------------- solver -----------------------------
    // Near tiles of the current block row live in registers (tc, masked);
    // those of the next block row and its diagonal tile are in flight (tx,
    // dx) while the current block is solved, and are masked and staged after.
    __shared__ double ring[kRing][64];
    __shared__ int ringe[kRing];
    __shared__ double dgu[64 * kTLD];  // diagonal tile of the current block
    __shared__ double dgs[64 * kTLD];  // the same with scaled columns
    __shared__ int sfE, sEmax;
    // the other ticket set belongs to the previous launch, which has ended;
    // clear it for the next one
    if (threadIdx.x < 4) a.ctl[4 * ((a.epoch + 1) & 1) + threadIdx.x] = 0;
    double tc[kLA][kCPW], tx[kLA][kCPW], dx[kCPW];
    double facc = 0.0;
    int fE = 0, emax = 0;
    uint64_t wlo = 0, whi = 0, wex = 0;  // pending far-sum words (wave 0)
#pragma unroll
    for (int t = 0; t < kLA; ++t) {
      load_tile(a, nb - 1, nb + t, lane, wave, tc[t]);
      mask_tile(a, nb - 1, nb + t, false, lane, wave, tc[t]);
    }
    load_tile(a, nb - 1, nb - 1, lane, wave, dx);
    mask_tile(a, nb - 1, nb - 1, true, lane, wave, dx);
    stage_diag(dx, lane, wave, dgu, dgs);
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
        for (int t = 0; t < kLA; ++t) load_tile(a, ib - 1, ib + t, lane, wave, tx[t]);
        load_tile(a, ib - 1, ib - 1, lane, wave, dx);
      }
      // near products: block columns ib+1 .. ib+kLA (x in LDS)
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
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < kCPW; ++q) s = fma(tc[t][q], xr[q], s);
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
        const double xo = diag_solve(rhs, dgu, dgs, nr, lane, e);
        emax = max(emax, e);
        ring[ib % kRing][lane] = xo;
        if (lane == 0) ringe[ib % kRing] = e;
        if (live) a.x[row] = xo;
        if (lane == 0) a.exps[ib] = e;
        publish_block(a.xll + (size_t)ib * kWords, a.epoch, xo, e, lane);
        // the far sum of the next block: complete the loads issued above
        if (want_far) {
          const int rr = ib - 1;
          const uint64_t* blk = a.all + (size_t)rr * kWords;
          bool own = false;
          while (!__all(word_ok(wlo, a.epoch) && word_ok(whi, a.epoch) &&
                        word_ok(wex, a.epoch))) {
            // not published yet: take the row if no helper has
            const int handed = __hip_atomic_load(tick + 1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (handed <= nfar - 1 - rr) {
              int got = 0;
              if (lane == 0)
                got = atomicCAS(tick + 1, nfar - 1 - rr, nfar - rr) == nfar - 1 - rr;
              if (__shfl(got, 0, 64)) { own = true; break; }
            }
            __builtin_amdgcn_s_sleep(1);
            wlo = ld_word(blk + 2 * lane);
            whi = ld_word(blk + 2 * lane + 1);
            wex = ld_word(blk + 128);
          }
          if (own) {
            facc = far_sum_wave(a, rr, nb, lane, fE);
          } else {
            facc = join_words(wlo, whi);
            fE = (int)(uint32_t)wex;
          }
        } else {
          facc = 0.0;
          fE = 0;
        }
        if (lane == 0) sfE = fE;
        if (lane == 0) sEmax = emax;
      }
      __syncthreads();
      fE = sfE;  // every wave needs the far exponent; facc stays in wave 0
      // the next block's tiles: mask, keep the near ones, stage the diagonal
      // (wave 0 read dgu/dgs before the barrier above; the barrier after the
      // next near products orders these writes before its reads)
      if (ib > 0) {
#pragma unroll
        for (int t = 0; t < kLA; ++t) {
          mask_tile(a, ib - 1, ib + t, false, lane, wave, tx[t]);
#pragma unroll
          for (int q = 0; q < kCPW; ++q) tc[t][q] = tx[t][q];
        }
        mask_tile(a, ib - 1, ib - 1, true, lane, wave, dx);
        stage_diag(dx, lane, wave, dgu, dgs);
      }
    }
    // bring every block to the largest exponent (entries smaller by more than
    // the FP64 range become zero) and report it
    __syncthreads();
    const int Em = sEmax;
    for (int i = threadIdx.x; i < a.m; i += kNT) {
      const int d = a.exps[i >> 6] - Em;
      if (d != 0) a.x[i] = ldexp(a.x[i], d);
    }
    if (threadIdx.x == 0) a.E_dev[0] = Em;
    return;
  }

  // ------------------------------ helpers ------------------------------
  // A helper takes block rows r in decreasing order from the row ticket and,
  // for each, streams the far tiles B(r, cb), cb = nb-1 down to r+kLA+1, as
  // the solver publishes x_cb.  Tiles are double-buffered in registers (A, B).
  // Wavefront 0 alone polls the published words of x_cb and copies the block
  // into LDS; one barrier per tile hands it to the other wavefronts.
  __shared__ double xs[2][64];
  __shared__ int xe[2];
  __shared__ int srow;
  for (;;) {
    if (threadIdx.x == 0) srow = atomicAdd(tick + 1, 1);
    __syncthreads();
    const int r = nfar - 1 - srow;
    __syncthreads();
    if (r < 0) break;
    double acc = 0.0;
    int E = 0;
    const int cend = r + 1 + kLA;  // last block column of the far part
    double tA[kCPW], tB[kCPW];
    load_tile(a, r, nb - 1, lane, wave, tA);
    if (nb - 2 >= cend) load_tile(a, r, nb - 2, lane, wave, tB);
    auto consume = [&](double* t, int cb) {
      if (wave == 0) {
        const uint64_t* blk = a.xll + (size_t)cb * kWords;
        uint64_t lo = ld_word(blk + 2 * lane), hi = ld_word(blk + 2 * lane + 1);
        uint64_t ex = ld_word(blk + 128);
        while (!__all(word_ok(lo, a.epoch) && word_ok(hi, a.epoch) && word_ok(ex, a.epoch))) {
          __builtin_amdgcn_s_sleep(2);
          lo = ld_word(blk + 2 * lane);
          hi = ld_word(blk + 2 * lane + 1);
          ex = ld_word(blk + 128);
        }
        xs[cb & 1][lane] = join_words(lo, hi);
        if (lane == 0) xe[cb & 1] = (int)(uint32_t)ex;
      }
      __syncthreads();
      mask_tile(a, r, cb, false, lane, wave, t);
      const int ec = xe[cb & 1];
      const double* xv = xs[cb & 1] + wave * kCPW;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kCPW; ++q) s = fma(t[q], xv[q], s);
      if (ec > E) { acc = ldexp(acc, E - ec); E = ec; }
      acc = fma(s, ldexp(1.0, ec - E), acc);
    };
    for (int cb = nb - 1; cb >= cend; cb -= 2) {
      consume(tA, cb);
      if (cb - 2 >= cend) load_tile(a, r, cb - 2, lane, wave, tA);
      if (cb - 1 >= cend) {
        consume(tB, cb - 1);
        if (cb - 3 >= cend) load_tile(a, r, cb - 3, lane, wave, tB);
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

// flags area layout: ctl[8] ints and exps[nb] ints, then (256-aligned)
// xll[(nb+1) * kWords] and all[(nb+1) * kWords] 64-bit words.
size_t trsv_flag_bytes(int m) {
  const size_t nb = (size_t)(m + 63) / 64 + 1;
  return 256 + (8 + nb) * sizeof(int) + 256 + 2 * nb * kWords * sizeof(uint64_t) + 256;
}

void trsv_upper_scaled(hipStream_t st, int m, const double* B, int ldb, const double* c,
                       double* x, int* flags, int epoch, int* E_dev, bool solo) {
  if (m <= 0) return;
  const int nb = (m + 63) / 64;
  int* ctl = flags;
  int* exps = flags + 8;
  uint64_t* xll = (uint64_t*)(((uintptr_t)(exps + nb + 1) + 255) & ~(uintptr_t)255);
  uint64_t* all = xll + (size_t)(nb + 1) * kWords;
  const int nfar = nb - 1 - kLA;
  const int helpers = (nfar > 0 && !solo) ? std::min(nfar, num_cus() - 1) : 0;
  TrsvArgs args{m, B, ldb, c, x, exps, xll, all, ctl, E_dev, (uint32_t)epoch};
  hipLaunchKernelGGL(k_trsv, dim3(1 + helpers), dim3(kNT), 0, st, args);
}

}  // namespace htk
