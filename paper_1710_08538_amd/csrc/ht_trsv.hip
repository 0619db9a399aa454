// ht_trsv.hip -- overflow-safe upper triangular solve B x = 2^{-E} c behind
// the opposite reflectors (Sec. 2.2, step c of Sec. 3.2.2).
//
// Rows are split into 64-row blocks, solved bottom-up.  For block b,
//   x_b = B_bb^{-1} (c_b - B_{b,b+1} x_{b+1} - [B_{b,b+2} x_{b+2} + B_{b,b+3} x_{b+3}]
//                       - sum_{c >= b+4} B_{b,c} x_c),
// and the four parts are produced by different hands, so that the serial
// substitution is the only work on the critical path:
//   * the substitution of block b+1 (one wavefront) also accumulates
//     B_{b,b+1} x_{b+1}, one extra FMA per row off its dependency chain;
//   * the other fifteen wavefronts of the solver workgroup ("staff") compute
//     B_{b,b+2} x_{b+2} + B_{b,b+3} x_{b+3} and stage the next diagonal and
//     coupling tiles in LDS while that substitution runs;
//   * helper workgroups stream the far tiles of a block row as the x blocks
//     are published and publish its far sum long before it is needed.
// The solver workgroup synchronises once per block.
//
// Publication uses 64-bit words that carry the call's epoch in the upper
// half and 32 data bits in the lower half (a double takes two words).  A
// 64-bit store is single-copy atomic, so a reader that sees the current epoch
// in every word of a block has the whole block: one round trip, no fences.
//
// Scaling: the solution of a triangular system with a small diagonal grows
// geometrically and overflows FP64 (ill-conditioned pencils reach 1e+300
// within a few hundred rows).  Every block carries its own power-of-two
// exponent e_b (true value = x_b 2^{e_b}); sums align exponents to their
// largest term.  The substitution works in 8-row chunks: after a chunk, if
// an entry of x exceeds 2^300 everything is scaled by 2^-600, and if one
// exceeds 2^600 (or is not finite) the chunk is redone row by row, scaling
// by 2^-600 before any entry would exceed 2^600 times its pivot.  The final
// pass shifts all blocks to the largest exponent E (entries smaller by more
// than the FP64 range become zero) and reports E: only the direction of x
// enters an opposite reflector (Lemma 2.1).
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

constexpr int kLA = 3;       // near block columns handled inside the solver workgroup
constexpr int kRing = 4;     // x blocks kept in LDS (>= kLA + 1)
constexpr int kWords = 130;  // per block: 128 words for 64 doubles + exponent + pad
constexpr int kNT = 1024;    // threads per workgroup
constexpr int kNW = kNT / 64;
constexpr int kCPW = 64 / kNW;  // helper tile columns per wavefront
constexpr int kSW = kNW - 1;    // staff wavefronts of the solver workgroup
constexpr int kSC = 5;          // staff tile columns per wavefront: (wave - 1) + 15 k
constexpr double kWarn = 0x1.0p300;

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

// Helper tiles: t[q] = B(64 ib + lane, 64 cb + kCPW wave + q).  Addresses are
// clamped into the matrix and the loads carry no condition, so they all issue
// back to back; entries outside the matrix are zeroed by mask_tile when the
// values are used.
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
__device__ __forceinline__ void mask_tile(const TrsvArgs& a, int ib, int cb, int lane, int wave,
                                          double t[kCPW]) {
  const int row = ib * 64 + lane;
  const int cbase = cb * 64 + wave * kCPW;
#pragma unroll
  for (int q = 0; q < kCPW; ++q) {
    const bool ok = row < a.m && cbase + q < a.m && cb >= 0;
    t[q] = ok ? t[q] : 0.0;
  }
}

// Staff tiles: t[k] = B(64 rb + lane, 64 cb + (wv-1) + 15 k) for the columns
// that exist (zero otherwise; rows beyond the matrix hold a clamped copy and
// are masked by the user).  The column address is uniform (scalar), the row
// offset is the lane.
__device__ __forceinline__ void staff_load(const TrsvArgs& a, int nb, int rb, int cb, int wv,
                                           int lane, double t[kSC]) {
  if (rb < 0 || rb >= nb || cb < 0 || cb >= nb) {
#pragma unroll
    for (int k = 0; k < kSC; ++k) t[k] = 0.0;
    return;
  }
  const int roff = min(lane, a.m - 1 - 64 * rb);
#pragma unroll
  for (int k = 0; k < kSC; ++k) {
    const int cc = (wv - 1) + 15 * k;
    const int col = 64 * cb + cc;
    if (cc < 64 && col < a.m)
      t[k] = a.B[(size_t)col * a.ldb + (size_t)(64 * rb) + roff];
    else
      t[k] = 0.0;
  }
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

// LDS of the solver workgroup.  Staged tiles are column-major with leading
// dimension 64: gs = diagonal tile with column c divided by its pivot and
// zero on and below the diagonal, ts = coupling tile B(b-1, b) divided the
// same way; pv = pivots (1 where zero or beyond the matrix), iv = 1 / pv.
struct SolverLds {
  double gs[2][64 * 64];
  double ts[2][64 * 64];
  double pv[2][64];
  double iv[2][64];
  double part[2][kSW][64];  // staff partial products for the next block
  double ring[kRing][64];   // recent x blocks
  int ringe[kRing];
  int bad[2][kSW];          // a staged scaled entry is not finite
  int emax;
};

// Stage block blk's tiles into buffer `buf` (staff wavefront wv, columns
// (wv-1) + 15 k): dg holds rows of block blk, dt rows of block blk-1.
__device__ __forceinline__ void staff_stage(const TrsvArgs& a, SolverLds& L, int buf, int blk,
                                            const double dg[kSC], const double dt[kSC], int wv,
                                            int lane) {
  // the wavefront's pivots gathered into lanes 0..kSC-1: one division
  double psel = 0.0;
#pragma unroll
  for (int k = 0; k < kSC; ++k) {
    const int cc = (wv - 1) + 15 * k;
    if (cc < 64) {
      const double d = readlane_d(dg[k], cc);
      if (lane == k) psel = d;
    }
  }
  const double inv = (psel != 0.0) ? 1.0 / psel : 1.0;
  const bool rowok = 64 * blk + lane < a.m;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < kSC; ++k) {
    const int cc = (wv - 1) + 15 * k;
    if (cc < 64) {
      const double ik = readlane_d(inv, k);
      const double pk = readlane_d(psel, k);
      const double g = (rowok && lane < cc) ? dg[k] * ik : 0.0;
      const double t = (blk >= 1) ? dt[k] * ik : 0.0;
      L.gs[buf][cc * 64 + lane] = g;
      L.ts[buf][cc * 64 + lane] = t;
      if (lane == 0) {
        L.iv[buf][cc] = ik;
        L.pv[buf][cc] = (pk != 0.0) ? pk : 1.0;
      }
      bad = bad || !(fabs(g) <= __DBL_MAX__) || !(fabs(t) <= __DBL_MAX__);
    }
  }
  const bool anybad = __any(bad);
  if (lane == 0) L.bad[buf][wv - 1] = anybad ? 1 : 0;
}

// Substitution of block b on wavefront 0.  In: rhs (lane l = row l, zero
// beyond the matrix) at exponent e.  Out: rhs holds the substituted values y
// (x = y / pivot), r2 the coupling sum B(b-1, b) x_b, both at the returned
// exponent e.
__device__ __forceinline__ void wave0_substitute(const SolverLds& L, int buf, int lane,
                                                 double& rhs, double& r2, int& e) {
  const double* gs = L.gs[buf];
  const double* ts = L.ts[buf];
  const double dinv = L.iv[buf][lane];
  const double dp = L.pv[buf][lane];
  double ga[8], ta[8], gb[8], tb[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ga[i] = gs[(63 - i) * 64 + lane];
    ta[i] = ts[(63 - i) * 64 + lane];
  }
  r2 = 0.0;
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    const int rtop = 63 - 8 * ch;
    __asm__ volatile("" ::: "memory");
    if (ch + 1 < 8) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        gb[i] = gs[(rtop - 8 - i) * 64 + lane];
        tb[i] = ts[(rtop - 8 - i) * 64 + lane];
      }
    }
    __asm__ volatile("" ::: "memory");
    const double rs = rhs, rs2 = r2;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double y = readlane_d(rhs, rtop - i);
      rhs = fma(-ga[i], y, rhs);
      r2 = fma(ta[i], y, r2);
    }
    const double xv = fabs(rhs * dinv);
    const bool inch = lane <= rtop && lane > rtop - 8;
    if (__any(inch && !(xv <= kBig))) {
      // redo the chunk row by row with scaling before each division
      rhs = rs;
      r2 = rs2;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = rtop - i;
        double t = readlane_d(rhs, r);
        const double dr = readlane_d(dp, r);
        int guard = 0;
        while (!(fabs(t) <= kBig * fabs(dr)) && guard < 8) {
          rhs *= kShrink;
          r2 *= kShrink;
          e += kShrinkExp;
          t = readlane_d(rhs, r);
          ++guard;
        }
        rhs = fma(-ga[i], t, rhs);
        r2 = fma(ta[i], t, r2);
      }
    } else if (__any(inch && xv > kWarn)) {
      rhs *= kShrink;
      r2 *= kShrink;
      e += kShrinkExp;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ga[i] = gb[i];
      ta[i] = tb[i];
    }
  }
}

// The same from the unscaled matrix in global memory, row by row; used when
// a scaled entry of the staged tiles is not finite (a pivot tiny relative to
// its column).
__device__ void wave0_substitute_slow(const TrsvArgs& a, const SolverLds& L, int buf, int b,
                                      int nr, int lane, double& rhs, double& r2, int& e) {
  const double dinv = L.iv[buf][lane];
  const double dp = L.pv[buf][lane];
  r2 = 0.0;
  for (int r = nr - 1; r >= 0; --r) {
    double t = readlane_d(rhs, r);
    const double dr = readlane_d(dp, r);
    int guard = 0;
    while (!(fabs(t) <= kBig * fabs(dr)) && guard < 8) {
      rhs *= kShrink;
      r2 *= kShrink;
      e += kShrinkExp;
      t = readlane_d(rhs, r);
      ++guard;
    }
    const double xr = t * readlane_d(dinv, r);
    const double* col = a.B + (size_t)(64 * b + r) * a.ldb;
    const double own = (lane < r) ? col[64 * b + lane] : 0.0;
    const double up = (b >= 1) ? col[64 * (b - 1) + lane] : 0.0;
    rhs = fma(-own, xr, rhs);
    r2 = fma(up, xr, r2);
  }
}

// One launch solves the system.  The first workgroup to start takes the
// solver role (a ticket from ctl), the others are helpers that take block
// rows from a second ticket.  Nothing waits on a workgroup that has not
// started: a helper only waits for x blocks of the solver, which runs, and
// the solver computes a far sum itself when no helper has taken that row.
__global__ __launch_bounds__(kNT) void k_trsv(TrsvArgs a) {
  const int nb = (a.m + 63) >> 6;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
    __shared__ SolverLds L;
    // the other ticket set belongs to the previous launch, which has ended;
    // clear it for the next one
    if (threadIdx.x < 4) a.ctl[4 * ((a.epoch + 1) & 1) + threadIdx.x] = 0;
    if (wave == 0) {
      // ---- substitution wavefront ----
      double rhs2 = 0.0, facc = 0.0;
      int e2 = 0, fE = 0, emax = 0;
      // right-hand sides are read two blocks ahead, off the critical path
      double crow = a.c[min(64 * (nb - 1) + lane, a.m - 1)];
      double crow_next = (nb >= 2) ? a.c[64 * (nb - 2) + lane] : 0.0;
      __syncthreads();  // staged tiles of block nb-1
      for (int b = nb - 1; b >= 0; --b) {
        const double crow_nn = (b >= 2) ? a.c[64 * (b - 2) + lane] : 0.0;
        const int buf = b & 1;
        const int nr = min(64, a.m - 64 * b);
        const bool live = lane < nr;
        const bool want_far = (b - 1 >= 0) && (b - 1 < nfar);
        uint64_t wlo = 0, whi = 0, wex = 0;
        if (want_far) {
          const uint64_t* blk = a.all + (size_t)(b - 1) * kWords;
          wlo = ld_word(blk + 2 * lane);
          whi = ld_word(blk + 2 * lane + 1);
          wex = ld_word(blk + 128);
        }
        // right-hand side at a common exponent
        int eP = 0;
        double sumP = 0.0;
        if (b + 2 < nb) {
          eP = L.ringe[(b + 2) % kRing];
          if (b + 3 < nb) eP = max(eP, L.ringe[(b + 3) % kRing]);
#pragma unroll
          for (int w = 0; w < kSW; ++w) sumP += L.part[buf][w][lane];
        }
        const int E = max(max(e2, eP), fE);
        double rhs = live ? (ldexp(crow, -E) - ldexp(rhs2, e2 - E) - ldexp(sumP, eP - E) -
                             ldexp(facc, fE - E))
                          : 0.0;
        int bad = 0;
#pragma unroll
        for (int w = 0; w < kSW; ++w) bad |= L.bad[buf][w];
        int e = E;
        double r2;
        if (!bad) wave0_substitute(L, buf, lane, rhs, r2, e);
        else wave0_substitute_slow(a, L, buf, b, nr, lane, rhs, r2, e);
        const double xo = live ? rhs * L.iv[buf][lane] : 0.0;
        emax = max(emax, e);
        L.ring[b % kRing][lane] = xo;
        if (lane == 0) L.ringe[b % kRing] = e;
        if (live) a.x[64 * b + lane] = xo;
        if (lane == 0) a.exps[b] = e;
        publish_block(a.xll + (size_t)b * kWords, a.epoch, xo, e, lane);
        rhs2 = r2;
        e2 = e;
        crow = crow_next;
        crow_next = crow_nn;
        // the far sum of the next block: complete the loads issued above
        if (want_far) {
          const int rr = b - 1;
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
            wex = ld_word(blk + 128);
            if (__all(word_ok(wex, a.epoch))) {  // then the data words
              wlo = ld_word(blk + 2 * lane);
              whi = ld_word(blk + 2 * lane + 1);
            }
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
        __syncthreads();
      }
      if (lane == 0) L.emax = emax;
    } else {
      // ---- staff wavefronts ----
      // Tile sets: for the step that solves block s they hold
      // p1 = B(s-1, s+1), p2 = B(s-1, s+2), dg = B(s-1, s-1), dt = B(s-2, s-1),
      // loaded two steps ahead (set X for blocks nb-1, nb-3, ..., Y for the others).
      double xp1[kSC], xp2[kSC], xdg[kSC], xdt[kSC];
      double yp1[kSC], yp2[kSC], ydg[kSC], ydt[kSC];
      {
        double dg0[kSC], dt0[kSC];
        staff_load(a, nb, nb - 1, nb - 1, wave, lane, dg0);
        staff_load(a, nb, nb - 2, nb - 1, wave, lane, dt0);
        const int s = nb - 1;
        staff_load(a, nb, s - 1, s + 1, wave, lane, xp1);
        staff_load(a, nb, s - 1, s + 2, wave, lane, xp2);
        staff_load(a, nb, s - 1, s - 1, wave, lane, xdg);
        staff_load(a, nb, s - 2, s - 1, wave, lane, xdt);
        const int s2 = nb - 2;
        staff_load(a, nb, s2 - 1, s2 + 1, wave, lane, yp1);
        staff_load(a, nb, s2 - 1, s2 + 2, wave, lane, yp2);
        staff_load(a, nb, s2 - 1, s2 - 1, wave, lane, ydg);
        staff_load(a, nb, s2 - 2, s2 - 1, wave, lane, ydt);
        staff_stage(a, L, (nb - 1) & 1, nb - 1, dg0, dt0, wave, lane);
      }
      __syncthreads();
      auto step = [&](int b, double* p1, double* p2, double* dg, double* dt)
                      __attribute__((always_inline)) {
        if (b - 1 >= 0) {
          // partial products of block b-1 with x_{b+1}, x_{b+2}
          int e1 = 0, ex2 = 0;
          if (b + 1 < nb) e1 = L.ringe[(b + 1) % kRing];
          if (b + 2 < nb) ex2 = L.ringe[(b + 2) % kRing];
          const int eP = (b + 2 < nb) ? max(e1, ex2) : e1;
          double s1 = 0.0, s2 = 0.0;
#pragma unroll
          for (int k = 0; k < kSC; ++k) {
            const int cc = (wave - 1) + 15 * k;
            if (cc < 64) {
              if (b + 1 < nb) s1 = fma(p1[k], L.ring[(b + 1) % kRing][cc], s1);
              if (b + 2 < nb) s2 = fma(p2[k], L.ring[(b + 2) % kRing][cc], s2);
            }
          }
          double part = 0.0;
          if (b + 1 < nb) part += ldexp(s1, e1 - eP);
          if (b + 2 < nb) part += ldexp(s2, ex2 - eP);
          L.part[(b - 1) & 1][wave - 1][lane] = part;
          staff_stage(a, L, (b - 1) & 1, b - 1, dg, dt, wave, lane);
        }
        // tiles for the step that solves block b-2
        const int s = b - 2;
        if (s >= 0) {
          staff_load(a, nb, s - 1, s + 1, wave, lane, p1);
          staff_load(a, nb, s - 1, s + 2, wave, lane, p2);
          staff_load(a, nb, s - 1, s - 1, wave, lane, dg);
          staff_load(a, nb, s - 2, s - 1, wave, lane, dt);
        }
        __syncthreads();
      };
      for (int b = nb - 1; b >= 0; b -= 2) {
        step(b, xp1, xp2, xdg, xdt);
        if (b - 1 >= 0) step(b - 1, yp1, yp2, ydg, ydt);
      }
    }
    // bring every block to the largest exponent (entries smaller by more than
    // the FP64 range become zero) and report it
    __syncthreads();
    const int Em = L.emax;
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
        // poll the exponent word alone (one address for the whole wavefront)
        // until it carries this call's epoch, then read the data words, which
        // were stored before it (re-read until every word is current)
        const uint64_t* blk = a.xll + (size_t)cb * kWords;
        uint64_t ex = ld_word(blk + 128);
        while (!__all(word_ok(ex, a.epoch))) {
          __builtin_amdgcn_s_sleep(2);
          ex = ld_word(blk + 128);
        }
        uint64_t lo = ld_word(blk + 2 * lane), hi = ld_word(blk + 2 * lane + 1);
        while (!__all(word_ok(lo, a.epoch) && word_ok(hi, a.epoch))) {
          lo = ld_word(blk + 2 * lane);
          hi = ld_word(blk + 2 * lane + 1);
        }
        xs[cb & 1][lane] = join_words(lo, hi);
        if (lane == 0) xe[cb & 1] = (int)(uint32_t)ex;
      }
      __syncthreads();
      mask_tile(a, r, cb, lane, wave, t);
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
