// ht_driver.hip -- host driver of the HouseHT reduction and the C ABI.
//
// Algorithm 1 (HouseHT) with the panel reduction of Sec. 3.2 and the
// absorption of Sec. 3.3, on one GPU.  Indices are 0-based: a panel starts
// at column s, its reflectors have support rows/columns >= s+1, and the
// "local" frame of a panel is rows/columns s+1 .. n-1 (L = n-s-1 of them).
// U, V, Y are stored in that local frame (local row r <-> global row s+1+r).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <mutex>
#include <vector>

#include "../../include/htred.h"
#include "ht_internal.h"
#include "ht_sweep.h"

using namespace htk;

namespace {

hipError_t g_last_hip = hipSuccess;

// Block structure of the trailing m' = n-j-1 rows/columns for an absorption
// of k reflectors with block stride s >= k (s = nb).  Blocks b_0 = [0, p) and
// b_t = [p+(t-1)s, p+ts), t = 1..T; right window t spans the last k rows of
// b_{t-1} and all of b_t (s+k rows; the first window has p+s, Remark 3.3).
// The left side mirrors this from the bottom: d_0 = [m'-p, m'),
// d_t = [m'-p-ts, m'-p-(t-1)s), left window t = d_t and the first k rows of
// d_{t-1}.  With s = k this is the basic scheme of Sec. 3.3 (2k x k
// windows).  After an early absorption (k < nb) the stride stays nb, so the
// chains of V2 and U2 have (m'/nb) windows of k reflectors each, and the
// restoring chains factor nb x (nb+k) blocks (B's fill band is nb+k wide).
// When m' <= s there is a single block b_1 = [0, m') and p = 0.
struct Blocks {
  int p, T, m, k, s;
  int rbs(int t) const { return t == 0 ? 0 : p + (t - 1) * s; }  // b_t
  int rbe(int t) const { return t == 0 ? p : std::min(p + t * s, m); }
  int rws(int t) const { return t == 1 ? 0 : rbs(t) - k; }       // right window t
  int rwe(int t) const { return rbe(t); }
  int ds(int t) const { return t == 0 ? m - p : std::max(m - p - t * s, 0); }  // d_t
  int de(int t) const { return t == 0 ? m : m - p - (t - 1) * s; }
  int lws(int t) const { return ds(t); }                           // left window t
  int lwe(int t) const { return t == 1 ? m : de(t) + k; }
};

Blocks make_blocks(int mprime, int k, int stride) {
  Blocks b;
  b.m = mprime;
  b.k = k;
  b.s = std::max(stride, k);
  if (mprime <= b.s) { b.p = 0; b.T = 1; return b; }
  const int q = mprime % b.s;
  b.p = q ? q : b.s;
  b.T = (mprime - b.p) / b.s;
  return b;
}

struct Work {
  int n = 0, nb = 0;
  double *U, *V, *Y, *S, *T, *Ucp;
  double *acol_save, *ctil, *ysol, *dsol, *wv, *w2, *rv;
  double *acol_save2, *ysol2, *rv2;  // the same for odd columns (speculation)
  double *tk, *tk2, *gk, *Ucat, *Kt, *Kt2, *P, *Wk;
  double* partials;
  double* kpart;       // split-contraction sums of the WY products
  double* pool[4][2];  // chain transform pools: [chain][V or W]
  double* Gws;
  double* dscal;       // [0] tau_u, [1] beta_u, [2] normB, [3..4] IR norms, [5] tau_v, [6] beta_v
  // ints: [1] E_rhs, [2] E_corr, [3] status, [4] fixes, [5] scaled; [9], [11]
  // E_rhs and status of odd columns
  int *flags, *ints;
  double* lu;  // l-block scheme: LU factors of B's diagonal blocks (N x S)
  int* perm;   // and their row permutations
  int epoch = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// slices of k x k partial sums for split-contraction WY products
constexpr size_t kKpartSlices = 32;

// S > 0: room for the diagonal-block LU factors of the l-block scheme.
size_t layout(Work* w, int n, int nb, char* base, int S = 0) {
  size_t off = 0;
  auto take = [&](size_t doubles) -> double* {
    double* p = base ? (double*)(base + off) : nullptr;
    off += align256(doubles * 8);
    return p;
  };
  const size_t N = (size_t)std::max(n, 1), K = (size_t)nb;
  w->n = n;
  w->nb = nb;
  w->U = take(N * K);
  w->V = take(N * K);
  w->Y = take(N * K);
  w->Ucp = take(N * K);
  w->S = take(K * K);
  w->T = take(K * K);
  w->acol_save = take(N);
  w->acol_save2 = take(N);
  w->ysol2 = take(N);
  w->rv2 = take(N);
  w->ctil = take(N);
  w->ysol = take(N);
  w->dsol = take(N);
  w->wv = take(N);
  w->w2 = take(N);
  w->rv = take(N);
  w->tk = take(4 * K);
  w->tk2 = take(4 * K);
  w->gk = take(4 * K);
  w->Ucat = take(2 * K * K);
  w->Kt = take(N * K);
  w->Kt2 = take(N * K);
  w->P = take(N * 2 * K);
  w->Wk = take(N * K);
  w->partials = take(std::max<size_t>(((N + 511) / 512 + 1) * N, 64 * K));
  w->kpart = take(kKpartSlices * K * K);
  size_t poolsz = 2 * N * K + 4 * K * K;
  if (S > 0) poolsz = std::max(poolsz, (size_t)(S + K) * (S + K));  // l-block windows
  for (int c = 0; c < 4; ++c)
    for (int v = 0; v < 2; ++v) w->pool[c][v] = take(poolsz);
  w->Gws = take(2 * K * K + 8);
  w->dscal = take(64);
  w->flags = (int*)take(trsv_flag_bytes((int)N) / 8 + 1);
  w->ints = (int*)take(32);
  w->lu = S > 0 ? take(N * (size_t)S) : nullptr;
  w->perm = S > 0 ? (int*)take(N / 2 + 1) : nullptr;
  return off;
}

// The refinement state of a panel column lives in one of two sets, by the
// parity of the column, so that the next column can be started before this
// one's verdict is known (see run()).
struct ColBufs {
  double *save, *ysol, *rv;
  int *Erhs, *status;
};
ColBufs colbufs(Work& w, int kk) {
  const int p = kk & 1;
  return ColBufs{p ? w.acol_save2 : w.acol_save, p ? w.ysol2 : w.ysol, p ? w.rv2 : w.rv,
                 w.ints + 1 + 8 * p, w.ints + 3 + 8 * p};
}

// Window list of a chain: (start, width, nrefl, slot, roff) in application
// order.  The transform of a window is kept in slot `slot` of its chain's
// pool as V, W of 2s x s (column-major, leading dimension 2s) with the real
// wdt x nrefl factors at row offset roff; the rest is zero.  Right windows
// are bottom-aligned in the slot (roff = 2s - wdt), left windows top-aligned,
// so that every full window is a 2s-wide window moving by s.
struct Win { int a, wdt, k, slot, roff; };

double* tV(Work& w, int ch, const Win& wn, int s) {
  return w.pool[ch][0] + (size_t)wn.slot * 2 * s * s + wn.roff;
}
double* tW(Work& w, int ch, const Win& wn, int s) {
  return w.pool[ch][1] + (size_t)wn.slot * 2 * s * s + wn.roff;
}

__global__ void k_scale_by(double* x, int m, const double* s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] *= s[0];
}
__global__ void k_count_scaled(const int* E, int* counter) {
  if (E[0] > 0) atomicAdd(counter, 1);
}
__global__ void k_set_int(int* p, int v) { p[0] = v; }
__global__ void k_init_ints(int* p) {
  if (threadIdx.x < 32) p[threadIdx.x] = 0;
}
__global__ void k_check_finite(int m, int n, const double* X, int ld, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < m && j < n) {
    const double v = X[(size_t)i + (size_t)j * ld];
    if (!isfinite(v)) atomicOr(bad, 1);
  }
}

inline double* at(double* X, int ld, int r, int c) { return X + (size_t)r + (size_t)c * ld; }

// zero[j] = 1 when column j of the upper triangle of B is zero; *offdiag
// becomes 1 when any strictly upper entry is nonzero (B not diagonal).
__global__ void k_zero_columns(int n, const double* B, int ld, int* zero, int* offdiag) {
  __shared__ int nz;
  const int j = blockIdx.x;
  if (threadIdx.x == 0) nz = 0;
  __syncthreads();
  int any = 0, off = 0;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    const bool z = B[(size_t)i + (size_t)j * ld] == 0.0;
    any |= !z;
    off |= (!z && i < j);
  }
  if (any) atomicOr(&nz, 1);
  if (off) atomicOr(offdiag, 1);
  __syncthreads();
  if (threadIdx.x == 0) zero[j] = nz ? 0 : 1;
}

// dst(i, j) = src(rp[i], cp[j]) (identity where rp / cp is NULL); with a
// NULL src, src is the identity matrix.
__global__ void k_gather(int n, const double* src, int lds, double* dst, int ldd, const int* rp,
                         const int* cp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const int si = rp ? rp[i] : i, sj = cp ? cp[j] : j;
  dst[(size_t)i + (size_t)j * ldd] = src ? src[(size_t)si + (size_t)sj * lds] : (si == sj ? 1.0 : 0.0);
}

// Per-kernel-class device timing with HIP events (HT_FLAG_PROFILE).  The
// events belong to the call: created on demand, destroyed by release() once
// their times are read, so the library holds no HIP object between calls.
struct Prof {
  bool on = false;
  struct Rec { int cls; hipEvent_t a, b; double work; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  bool failed = false;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) {
        failed = true;
        return nullptr;
      }
      pool.push_back(e);
    }
    return pool[used++];
  }
  int begin(hipStream_t st, int cls) {
    if (!on || failed) return -1;
    Rec r{cls, get(), get(), 0.0};
    if (!r.a || !r.b) return -1;
    (void)hipEventRecord(r.a, st);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(hipStream_t st, int idx, double work) {
    if (idx < 0) return;
    recs[idx].work = work;
    (void)hipEventRecord(recs[idx].b, st);
  }
  void collect(ht_stats* s) {
    for (auto& r : recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) s->prof_ms[r.cls] += ms;
      s->prof_work[r.cls] += r.work;
      s->prof_launches[r.cls] += 1;
    }
  }
  void release() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
    recs.clear();
    used = 0;
  }
};

struct Ctx {
  hipStream_t st;
  Work* w;
  int n, nb;
  int S = 0;  // l-block scheme: diagonal block order (l - 1) nb of B; 0: basic scheme
  double *A, *B, *Q, *Z;
  int lda, ldb, ldq, ldz;
  bool wantQ, wantZ;
  ht_options opt;
  int* host_ints;  // pinned mirror of w->ints
  Prof prof;
  hipEvent_t status_ev[2] = {nullptr, nullptr};  // see post_status

  double flops = 0.0;
  int64_t cols_extra_ir = 0, ir_steps = 0, ir_failures = 0, absorptions = 0, columns = 0;
};

// A product of the WY updates (the absorption's window applications and
// rank-k corrections): FP64 MFMA, or the emulated-FP64 split product of the
// precision form.  Panels, solves, chains and the T/S factors never come
// here.
void wy(Ctx& c, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
        const double* B, int ldb, double beta, double* C, int ldc) {
  if (c.opt.prec == HT_PREC_FP64)
    gemm_ws(c.st, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, c.w->kpart,
            kKpartSlices * (size_t)c.nb * c.nb);
  else
    split_gemm(c.st, c.opt.prec == HT_PREC_SPLIT_BF16 ? 0 : 1, c.opt.n_slices, ta, tb, m, n, k,
               alpha, A, lda, B, ldb, beta, C, ldc);
}

// X(0:rows, window) <- X (I - V W^T), window width wdt, k reflectors (V, W
// with leading dimension ldv).
void right_apply(Ctx& c, double* X, int ld, int rows, int wdt, int k, const double* Vf,
                 const double* Wf, int ldv) {
  if (rows <= 0 || wdt <= 0 || k <= 0) return;
  const int pi = c.prof.begin(c.st, HT_PROF_WY);
  wy(c, false, false, rows, k, wdt, 1.0, X, ld, Vf, ldv, 0.0, c.w->P, c.n);
  wy(c, false, true, rows, wdt, k, -1.0, c.w->P, c.n, Wf, ldv, 1.0, X, ld);
  c.prof.end(c.st, pi, 4.0 * rows * (double)wdt * k);
  c.flops += 4.0 * rows * (double)wdt * k;
}

// X(window, 0:ncols) <- (I - V W^T)^T X = X - W (V^T X).
void left_apply(Ctx& c, double* X, int ld, int ncols, int wdt, int k, const double* Vf,
                const double* Wf, int ldv) {
  if (ncols <= 0 || wdt <= 0 || k <= 0) return;
  const int pi = c.prof.begin(c.st, HT_PROF_WY);
  wy(c, true, false, k, ncols, wdt, 1.0, Vf, ldv, X, ld, 0.0, c.w->P, k);
  wy(c, false, false, wdt, ncols, k, -1.0, Wf, ldv, c.w->P, k, 1.0, X, ld);
  c.prof.end(c.st, pi, 4.0 * ncols * (double)wdt * k);
  c.flops += 4.0 * ncols * (double)wdt * k;
}

std::vector<Win> right_windows(const Blocks& bl, int chain) {
  std::vector<Win> v;
  auto win = [&](int a, int e, int nr, int t) {
    v.push_back({a, e - a, nr, t, 2 * bl.s - (e - a)});
  };
  if (chain == 0) {  // Q^_1 .. Q^_T (QL of V2), applied first to last
    for (int t = 1; t <= bl.T; ++t) win(bl.rws(t), bl.rwe(t), bl.k, t);
  } else {           // RQ restore G_T .. G_1, G_0 (nrefl = rows of b_t)
    for (int t = bl.T; t >= 1; --t) win(bl.rws(t), bl.rwe(t), bl.rbe(t) - bl.rbs(t), t);
    if (bl.p > 0) win(0, bl.p, bl.p, 0);
  }
  return v;
}

std::vector<Win> left_windows(const Blocks& bl, int chain) {
  std::vector<Win> v;
  auto win = [&](int a, int e, int nr, int t) { v.push_back({a, e - a, nr, t, 0}); };
  if (chain == 2) {  // Q~_1 .. Q~_T (QR of U2, bottom to top)
    for (int t = 1; t <= bl.T; ++t) win(bl.lws(t), bl.lwe(t), bl.k, t);
  } else {           // QR restore H_T .. H_1, H_0 (nrefl = columns of d_t)
    for (int t = bl.T; t >= 1; --t) win(bl.lws(t), bl.lwe(t), bl.de(t) - bl.ds(t), t);
    if (bl.p > 0) win(bl.ds(0), bl.m, bl.p, 0);
  }
  return v;
}

// A matrix (or row range) receiving a right sweep: rows 0..rows-1 of X,
// absolute column indices; `tri` marks an upper triangular X (B), whose rows
// below a window's last column are zero there.
struct RJob { double* X; int ld; int rows; bool tri; int tri_off; };

// Apply the windows of a chain, in order, as right multiplications
// X(:, j+1+win) <- X(:, j+1+win) (I - V W^T) to every job, or with `left`
// as left multiplications X(j+1+win, :) <- (I - V W^T)^T X(j+1+win, :) to
// the columns of every job (job.X at its first column, rows = its number of
// columns, tri_off = that column's index).  Runs of consecutive full windows
// (width 2k, moving by k) go to the fused MFMA sweep kernel in one launch
// for all jobs; the odd windows at the ends of a chain (first window p+k
// wide, last one p x p) use the generic product.
void sweep_jobs(Ctx& c, const std::vector<RJob>& jobs, int j, const Blocks& bl, int chain,
                const std::vector<Win>& wins, bool left = false) {
  const int s = bl.s, K = bl.s;
  // a full window: its 2s-wide slot window (the real window plus zero
  // padding) lies inside the trailing part; consecutive full windows move by s
  auto slot_start = [&](const Win& w) { return w.a - w.roff; };
  auto full_win = [&](const Win& w) {
    const int a0 = slot_start(w);
    return a0 >= 0 && a0 + 2 * s <= bl.m;
  };
  size_t i = 0;
  while (i < wins.size()) {
    const Win& w0 = wins[i];
    // the fused sweep is FP64 only; the precision form applies windows one
    // at a time through split products
    const bool full = c.opt.prec == HT_PREC_FP64 && sweep_supported(K) && jobs.size() <= 4 &&
                      full_win(w0);
    size_t e = i + 1;
    int dir = 0;
    if (full) {
      while (e < wins.size() && full_win(wins[e])) {
        const int d = slot_start(wins[e]) - slot_start(wins[e - 1]);
        if (!((d == s || d == -s) && (dir == 0 || d == dir * s))) break;
        dir = d > 0 ? 1 : -1;
        ++e;
      }
    }
    if (full && e - i >= 2) {
      SweepArgs sa;
      memset(&sa, 0, sizeof(sa));
      int wg = 0;
      for (const RJob& jb : jobs) {
        if (jb.rows <= 0) continue;
        SweepJob& sj = sa.job[sa.njobs++];
        sj.X = jb.X;
        sj.ld = jb.ld;
        sj.nrows = jb.rows;
        sj.tri = jb.tri ? 1 : 0;
        sj.tri_off = jb.tri_off;
        sj.wg0 = wg;
        wg += (jb.rows + 63) / 64;
      }
      sa.nwin = (int)(e - i);
      sa.c0 = j + 1 + slot_start(w0);
      sa.Vp = c.w->pool[chain][0];
      sa.Wp = c.w->pool[chain][1];
      sa.slot0 = w0.slot;
      sa.slot_step = wins[i + 1].slot - w0.slot;
      {
        // tiles of the slots that can hold nonzeros (narrow windows of early
        // absorptions and of the Remark 3.3 blocks are zero-padded)
        int r0 = 2 * s, r1 = 0, kx = 0;
        for (size_t t = i; t < e; ++t) {
          r0 = std::min(r0, wins[t].roff);
          r1 = std::max(r1, wins[t].roff + wins[t].wdt);
          kx = std::max(kx, wins[t].k);
        }
        sa.tlo = r0 / 16;
        sa.thi = std::min(2 * s / 16, (r1 + 15) / 16);
        sa.phi = std::min(s / 16, (kx + 15) / 16);
      }
      double fl = 0.0;  // algorithmic: 4 rows wdt nrefl per window
      for (const RJob& jb : jobs) {
        if (jb.rows <= 0) continue;
        for (size_t t = i; t < e; ++t) {
          // B: right, rows below a window's end are zero; left, columns
          // left of a window's start
          const int ws = j + 1 + wins[t].a;
          const int r = !jb.tri ? jb.rows
                        : left ? jb.rows - std::min(jb.rows, std::max(0, ws - jb.tri_off))
                               : std::max(0, std::min(jb.rows, ws + wins[t].wdt - jb.tri_off));
          fl += 4.0 * r * (double)wins[t].wdt * wins[t].k;
        }
      }
      const int pi = c.prof.begin(c.st, HT_PROF_SWEEP);
      sweep_rows(c.st, sa, K, dir, left);
      c.prof.end(c.st, pi, fl);
      c.flops += fl;
      i = e;
      continue;
    }
    for (const RJob& jb : jobs) {
      if (jb.rows <= 0) continue;
      if (left) {
        const int cs = jb.tri ? std::min(jb.rows, std::max(0, j + 1 + w0.a - jb.tri_off)) : 0;
        left_apply(c, at(jb.X, jb.ld, j + 1 + w0.a, cs), jb.ld, jb.rows - cs, w0.wdt, w0.k,
                   tV(*c.w, chain, w0, s), tW(*c.w, chain, w0, s), 2 * s);
        continue;
      }
      const int r = jb.tri ? std::min(jb.rows, j + 1 + w0.a + w0.wdt - jb.tri_off) : jb.rows;
      right_apply(c, at(jb.X, jb.ld, 0, j + 1 + w0.a), jb.ld, r, w0.wdt, w0.k,
                  tV(*c.w, chain, w0, s), tW(*c.w, chain, w0, s), 2 * s);
    }
    ++i;
  }
}

// Right sweep of a chain over X(0:rows, j+1 : n).
void sweep_right(Ctx& c, double* X, int ld, int rows, bool tri, int j, const Blocks& bl,
                 int chain) {
  sweep_jobs(c, {RJob{X, ld, rows, tri, 0}}, j, bl, chain, right_windows(bl, chain));
}

// Left sweep of a chain over rows j+1.. of X, columns [c0, n).  With
// `tri`, columns left of a window's first row are zero and skipped.
void sweep_left(Ctx& c, double* X, int ld, int c0, bool tri, int j, const Blocks& bl, int chain) {
  sweep_jobs(c, {RJob{at(X, ld, 0, c0), ld, c.n - c0, tri, c0}}, j, bl, chain,
             left_windows(bl, chain), true);
}

// Q(:, j+1 : n) <- Q * (chain transforms in order).
void sweep_cols_right(Ctx& c, double* X, int ld, int rows, int j, const Blocks& bl, int chain) {
  sweep_jobs(c, {RJob{X, ld, rows, false, 0}}, j, bl, chain, left_windows(bl, chain));
}

// One chain factorisation, timed as HT_PROF_CHAIN (flops of a Householder
// QR/QL of a wdt x k tile plus the W build: about 4 wdt k^2).  V and W are
// written with leading dimension ldo.
void chain(Ctx& c, int mode, bool trans, int wdt, int k, double* tile, int ld, double* Vf,
           double* Wf, int ldo) {
  const int pi = c.prof.begin(c.st, HT_PROF_CHAIN);
  if (trans) chain_factor_t(c.st, mode, wdt, k, tile, ld, Vf, Wf, ldo);
  else chain_factor(c.st, mode, wdt, k, tile, ld, Vf, Wf, ldo);
  c.prof.end(c.st, pi, 4.0 * wdt * (double)k * k);
  c.flops += 4.0 * wdt * (double)k * k;
}

// The refinement verdict of a column: copied to host memory behind the
// work enqueued so far (post_status), read when needed (read_status).  With
// an event per parity the host waits only for that copy, so the work
// enqueued after it keeps the GPU busy meanwhile.
void post_status(Ctx& c, const ColBufs& cb, int kk) {
  const int p = kk & 1;
  (void)hipMemcpyAsync(c.host_ints + 16 + p, cb.status, sizeof(int), hipMemcpyDeviceToHost, c.st);
  if (c.status_ev[p]) (void)hipEventRecord(c.status_ev[p], c.st);
}
int read_status(Ctx& c, int kk) {
  const int p = kk & 1;
  if (c.status_ev[p]) (void)hipEventSynchronize(c.status_ev[p]);
  else (void)hipStreamSynchronize(c.st);
  return c.host_ints[16 + p];
}
int sync_status(Ctx& c, const ColBufs& cb, int kk) {
  post_status(c, cb, kk);
  return read_status(c, kk);
}

// ---------------------------------------------------------------------------
// Factored solve (Sec. 3.2.2 c, steps 1-3): ctil <- (I - U S U^T) ctil;
// B ytil = 2^{-E} ctil; y <- (I - V T V^T)^T ytil.  nu = reflectors in U.
// ---------------------------------------------------------------------------
// unit >= 0: ctil is taken to be e_unit (not read) and formed here.
void factored_solve(Ctx& c, int s, int kk, int nu, double* ctil, double* ysol, int* Eout,
                    int unit = -1) {
  Work& w = *c.w;
  const int L = c.n - s - 1, n = c.n;
  if (unit >= 0)
    wy_apply_unit(c.st, L, unit, nu, -1.0, w.U, n, w.S, c.nb, false, ctil);
  else
    wy_apply(c.st, L, L, 0, nu, -1.0, w.U, n, w.S, c.nb, false, ctil, ctil, w.tk, w.partials);
  const double* Bp = at(c.B, c.ldb, s + 1, s + 1);
  const int pi = c.prof.begin(c.st, HT_PROF_TRSV);
  if (c.S > 0) {
    // block upper triangular B (l-block scheme, Sec. 3.5): block back
    // substitution with the panel's LU factors, no scaling (E = 0)
    block_solve(c.st, L, c.S, Bp, c.ldb, w.lu, n, w.perm, ctil, ysol, w.partials);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, c.st, Eout, 0);
    c.prof.end(c.st, pi, 8.0 * L * (double)(L + c.S) / 2.0);
  } else {
    trsv_upper_scaled(c.st, L, Bp, c.ldb, ctil, ysol, w.flags, ++w.epoch, Eout,
                      (c.opt.flags & HT_FLAG_SOLVE_SOLO) != 0);
    c.prof.end(c.st, pi, 8.0 * L * (double)(L + 1) / 2.0);
    hipLaunchKernelGGL(k_count_scaled, dim3(1), dim3(1), 0, c.st, Eout, w.ints + 5);
  }
  if (kk > 0) {
    wy_apply(c.st, L, L, 0, kk, -1.0, w.V, n, w.T, c.nb, true, ysol, ysol, w.tk, w.partials);
  }
  c.flops += 1.0 * L * (double)L + 4.0 * L * (double)(nu + kk);
}

// Residual (Sec. 3.2.2 c): w = (I - V T V^T)[0; x]; w = B w;
// w = (I - U S^T U^T) w; r = 2^{-E} rhs - w(kk:), rhs = e1 if NULL.
void residual(Ctx& c, int s, int kk, const double* x, const double* rhs, const ColBufs& cb) {
  Work& w = *c.w;
  const int L = c.n - s - 1, n = c.n, m = L - kk;
  wy_apply_padded(c.st, L, m, kk, kk, -1.0, w.V, n, w.T, c.nb, false, x, w.wv, w.tk,
                  w.partials);
  const double* Bp = at(c.B, c.ldb, s + 1, s + 1);
  const int pi = c.prof.begin(c.st, HT_PROF_TRMV);
  if (c.S > 0) {
    // block upper triangular B: a full product (the entries below the
    // diagonal blocks are exact zeros)
    gemv_n(c.st, L, L, 1.0, Bp, c.ldb, w.wv, 1, 0.0, w.w2, w.partials);
    c.prof.end(c.st, pi, 8.0 * L * (double)L);
  } else {
    trmv_upper(c.st, L, Bp, c.ldb, w.wv, w.w2, w.partials);
    c.prof.end(c.st, pi, 8.0 * L * (double)(L + 1) / 2.0);
  }
  wy_apply(c.st, L, L, 0, kk + 1, -1.0, w.U, n, w.S, c.nb, true, w.w2, w.w2, w.tk, w.partials);
  ir_residual(c.st, m, w.w2 + kk, rhs, cb.Erhs, cb.rv, x, w.dscal + 2, c.opt.ir_tol_factor,
              cb.status, w.dscal + 3);
  c.flops += 1.0 * L * (double)L + 4.0 * L * (double)(2 * kk + 1);
}


// ---------------------------------------------------------------------------
// Parts of an absorption common to the basic and the l-block schemes.
// ---------------------------------------------------------------------------
// (3.3.1 c, d, e) rank-k part of the right absorption, once V2 = [0; L1] and
// the windows' transforms are applied.  B, Z and rows 0..s of A:
//   W = X(:, s+1:j+1) V1 + X(:, n-k:n) L1;  X(:, s+1:j+1) -= W T V1^T;
//   X(:, n-k:n) -= W T L1^T;
// rows s+1..n-1 of A through Y = A V T (Sec. 3.3.1 e):
//   A(:, j) -= Y V1(k-1,:)^T;  A(:, n-k:n) -= Y L1^T.
void right_rank_k(Ctx& c, int s, int k) {
  Work& w = *c.w;
  const int n = c.n, j = s + k, L = n - s - 1;
  double* A = c.A;
  const int lda = c.lda;
  struct RT { double* X; int ld; int rows; };
  const RT rts[3] = {{c.B, c.ldb, n}, {c.wantZ ? c.Z : nullptr, c.ldz, n}, {A, lda, s + 1}};
  const double* L1 = w.V + (L - k);
  const double* V1 = w.V;
  for (const RT& rt : rts) {
    if (!rt.X || rt.rows <= 0) continue;
    double* Xs = at(rt.X, rt.ld, 0, s + 1);
    double* Xe = at(rt.X, rt.ld, 0, n - k);
    wy(c, false, false, rt.rows, k, k, 1.0, Xs, rt.ld, V1, n, 0.0, w.Wk, n);
    wy(c, false, false, rt.rows, k, k, 1.0, Xe, rt.ld, L1, n, 1.0, w.Wk, n);
    wy(c, false, false, rt.rows, k, k, 1.0, w.Wk, n, w.T, c.nb, 0.0, w.P, n);
    wy(c, false, true, rt.rows, k, k, -1.0, w.P, n, V1, n, 1.0, Xs, rt.ld);
    wy(c, false, true, rt.rows, k, k, -1.0, w.P, n, L1, n, 1.0, Xe, rt.ld);
    c.flops += 10.0 * rt.rows * (double)k * k;
  }
  gemv_n(c.st, L, k, -1.0, w.Y, n, w.V + (k - 1), n, 1.0, at(A, lda, s + 1, j), w.partials);
  wy(c, false, true, L, k, k, -1.0, w.Y, n, L1, n, 1.0, at(A, lda, s + 1, n - k), lda);
  c.flops += 4.0 * L * (double)k * k;
}

// (3.3.2 c) spike columns s+1..j of B:
//   B(s+1:j+1, s+1:j+1) -= U1 S^T (U^T B(s+1:n, s+1:j+1));  B(j+1:n, s+1:j+1) = 0.
void spike(Ctx& c, int s, int k) {
  Work& w = *c.w;
  const int n = c.n, j = s + k, L = n - s - 1, mp = n - j - 1;
  double* B = c.B;
  const int ldb = c.ldb;
  wy(c, true, false, k, k, L, 1.0, w.U, n, at(B, ldb, s + 1, s + 1), ldb, 0.0, w.Kt, k);
  wy(c, true, false, k, k, k, 1.0, w.S, c.nb, w.Kt, k, 0.0, w.Kt2, k);
  wy(c, false, false, k, k, k, -1.0, w.U, n, w.Kt2, k, 1.0, at(B, ldb, s + 1, s + 1), ldb);
  zero_mat(c.st, at(B, ldb, j + 1, s + 1), mp, k, ldb);
  // Fact 3: columns s+1..j are now triangular; their entries below the
  // diagonal are rounding noise of the opposite reflectors (Lemma 2.1) and are
  // set to exact zeros, as Algorithm 2 does.
  zero_lower(c.st, at(B, ldb, s + 1, s + 1), k, ldb, 0);
  c.flops += 2.0 * k * (double)k * (L + 2 * k);
}

// (3.3.2 c, e) corrections with Ucat = [U1; R1] on rows s+1..j+k of B
// (columns j+1..n-1) and A (columns j..n-1):  X -= Ucat S^T (Ucat^T X).
void left_rank_k(Ctx& c, int s, int k) {
  Work& w = *c.w;
  const int n = c.n, j = s + k;
  const int ncb = n - j - 1, nca = n - j;
  double* Bs = at(c.B, c.ldb, s + 1, j + 1);
  wy(c, true, false, k, ncb, 2 * k, 1.0, w.Ucat, 2 * k, Bs, c.ldb, 0.0, w.Kt, k);
  wy(c, true, false, k, ncb, k, 1.0, w.S, c.nb, w.Kt, k, 0.0, w.Kt2, k);
  wy(c, false, false, 2 * k, ncb, k, -1.0, w.Ucat, 2 * k, w.Kt2, k, 1.0, Bs, c.ldb);
  double* As = at(c.A, c.lda, s + 1, j);
  wy(c, true, false, k, nca, 2 * k, 1.0, w.Ucat, 2 * k, As, c.lda, 0.0, w.Kt, k);
  wy(c, true, false, k, nca, k, 1.0, w.S, c.nb, w.Kt, k, 0.0, w.Kt2, k);
  wy(c, false, false, 2 * k, nca, k, -1.0, w.Ucat, 2 * k, w.Kt2, k, 1.0, As, c.lda);
  c.flops += 10.0 * (double)k * k * (nca + ncb);
}

// (3.3.2 d) after Q(:, j+1:n) <- Q Q~:  W = Q(:, s+1:j+k+1) Ucat;
// Q(:, s+1:..) -= W S Ucat^T.
void q_rank_k(Ctx& c, int s, int k) {
  Work& w = *c.w;
  const int n = c.n;
  double* Qs = at(c.Q, c.ldq, 0, s + 1);
  wy(c, false, false, n, k, 2 * k, 1.0, Qs, c.ldq, w.Ucat, 2 * k, 0.0, w.Wk, n);
  wy(c, false, false, n, k, k, 1.0, w.Wk, n, w.S, c.nb, 0.0, w.P, n);
  wy(c, false, true, n, 2 * k, k, -1.0, w.P, n, w.Ucat, 2 * k, 1.0, Qs, c.ldq);
  c.flops += 10.0 * (double)n * k * k;
}

// ---------------------------------------------------------------------------
// Absorption of k left and right reflectors (Sec. 3.3).
// ---------------------------------------------------------------------------
void absorb(Ctx& c, int s, int k) {
  Work& w = *c.w;
  const int n = c.n, j = s + k, L = n - s - 1, mp = n - j - 1;
  const Blocks bl = make_blocks(mp, k, c.nb);
  const int sb = bl.s, ldo = 2 * bl.s;
  double *A = c.A, *B = c.B;
  const int lda = c.lda, ldb = c.ldb;
  c.absorptions++;
  // windows narrower than their 2s slot: clear the slots' padding
  if (k < sb) {
    const size_t slots = (size_t)(bl.T + 1) * 2 * sb * sb;
    for (int ch = 0; ch < 4; ++ch)
      for (int v = 0; v < 2; ++v) zero_mat(c.st, w.pool[ch][v], (int)slots, 1, (int)slots);
  }

  // (3.3.1 b) V2 = Q^_1 ... Q^_T [0; L1]: QL chain, top to bottom, in place;
  // (3.3.2 b) U2 = Q~_1 ... Q~_T [R1; 0]: QR chain, bottom to top, on a copy
  // (the spike update below needs the original U2).  The two chains are
  // independent and have the same windows count: window t of both is
  // factored in one launch on two workgroups.
  double* V2 = w.V + k;
  copy_mat(c.st, mp, k, w.U + k, n, w.Ucp, n);

  // (3.3.1 c, d, e) right absorption.  B, Z and rows 0..s of A:
  //   X(:, j+1:n) <- X Q^;  W = X(:, s+1:j+1) V1 + X(:, n-k:n) L1;
  //   X(:, s+1:j+1) -= W T V1^T;  X(:, n-k:n) -= W T L1^T.
  struct RT { double* X; int ld; int rows; bool tri; };
  std::vector<RT> rts;
  rts.push_back({B, ldb, n, true});
  if (c.wantZ) rts.push_back({c.Z, c.ldz, n, false});
  rts.push_back({A, lda, s + 1, false});
  std::vector<RJob> rjobs;
  for (auto& rt : rts) rjobs.push_back(RJob{rt.X, rt.ld, rt.rows, rt.tri, 0});
  rjobs.push_back(RJob{at(A, lda, s + 1, 0), lda, L, false, s + 1});
  {
    const std::vector<Win> r0 = right_windows(bl, 0), l2 = left_windows(bl, 2);
    for (size_t t = 0; t < r0.size(); ++t) {
      const Win &a = r0[t], &b = l2[t];
      ChainJobs jobs;
      jobs.njobs = 2;
      jobs.job[0] = ChainJob{1, a.wdt, k, V2 + a.a, n, 0, tV(w, 0, a, sb), tW(w, 0, a, sb), ldo};
      jobs.job[1] = ChainJob{0, b.wdt, k, w.Ucp + b.a, n, 0, tV(w, 2, b, sb), tW(w, 2, b, sb), ldo};
      const int pi = c.prof.begin(c.st, HT_PROF_CHAIN);
      chain_factor_jobs(c.st, jobs);
      const double fl = 4.0 * (a.wdt + b.wdt) * (double)k * k;
      c.prof.end(c.st, pi, fl);
      c.flops += fl;
    }
    sweep_jobs(c, rjobs, j, bl, 0, r0);
  }
  copy_mat(c.st, k, k, w.U, n, w.Ucat, 2 * k);
  copy_mat(c.st, k, k, w.Ucp, n, w.Ucat + k, 2 * k);
  right_rank_k(c, s, k);

  // (3.3.1 e) restore B by RQ decompositions, bottom to top: the k x (w)
  // block of row block b_t is factored as [0 R] G_t; G_t^T is applied to
  // the rows above it at once (the next step needs row block b_{t-1}).
  for (const Win& wn : right_windows(bl, 1)) {
    const int r0 = bl.rbs(wn.slot);
    const int kr = wn.k;  // rows of the block
    double* C = at(B, ldb, j + 1 + r0, j + 1 + wn.a);
    chain(c, 1, true, wn.wdt, kr, C, ldb, tV(w, 1, wn, sb), tW(w, 1, wn, sb), ldo);
    right_apply(c, at(B, ldb, 0, j + 1 + wn.a), ldb, j + 1 + r0, wn.wdt, kr, tV(w, 1, wn, sb),
                tW(w, 1, wn, sb), ldo);
  }
  {
    std::vector<RJob> jobs{RJob{A, lda, n, false, 0}};
    if (c.wantZ) jobs.push_back(RJob{c.Z, c.ldz, n, false, 0});
    sweep_jobs(c, jobs, j, bl, 1, right_windows(bl, 1));
  }

  spike(c, s, k);

  // (3.3.2 c, e) rows j+1..n-1: B(:, j+1:n) and A(:, j:n) <- Q~^T (.)
  sweep_jobs(c, {RJob{at(B, ldb, 0, j + 1), ldb, n - j - 1, true, j + 1},
                 RJob{at(A, lda, 0, j), lda, n - j, false, j}},
             j, bl, 2, left_windows(bl, 2), true);
  left_rank_k(c, s, k);
  // (3.3.2 d) Q(:, j+1:n) <- Q Q~, then the Ucat correction
  if (c.wantQ) {
    sweep_cols_right(c, c.Q, c.ldq, n, j, bl, 2);
    q_rank_k(c, s, k);
  }

  // (3.3.2 f) restore B by QR decompositions, top to bottom; each H_t^T is
  // applied at once to the columns right of its block (the next step needs
  // them), then to A(j+1:n, j:n) and Q(:, j+1:n).
  for (const Win& wn : left_windows(bl, 3)) {
    const int t = wn.slot;
    const int cs = bl.ds(t), ce = bl.de(t);  // columns d_t
    double* M = at(B, ldb, j + 1 + wn.a, j + 1 + cs);
    chain(c, 0, false, wn.wdt, ce - cs, M, ldb, tV(w, 3, wn, sb), tW(w, 3, wn, sb), ldo);
    left_apply(c, at(B, ldb, j + 1 + wn.a, j + 1 + ce), ldb, mp - ce, wn.wdt, ce - cs,
               tV(w, 3, wn, sb), tW(w, 3, wn, sb), ldo);
  }
  sweep_left(c, A, lda, j, false, j, bl, 3);
  if (c.wantQ) sweep_cols_right(c, c.Q, c.ldq, n, j, bl, 3);
}

// ---------------------------------------------------------------------------
// Absorption with l >= 3 blocks (Sec. 3.5, accelerated reduction of V2 and
// U2).  B's trailing part is kept block upper triangular with diagonal
// blocks of order S = (l - 1) nb aligned at its bottom (ell_bounds; the top
// block holds the remainder), so the chains have one window per diagonal
// block (S + k rows) instead of one per nb rows, and each restoring step
// clears only the k-wide fill next to a block with k reflectors:
//   right: the first k rows of the orthogonal factor of the RQ decomposition
//     of the block's rows over the window's columns, reduced by an LQ
//     decomposition (the 2nb x 3nb construction for l = 3, k = nb);
//   left: the last k columns of the orthogonal factor of the QR
//     decomposition of the block's columns over its rows and the k rows
//     below, reduced by a QL decomposition.
// Every window's transform is applied at once, by general products, to B, A
// and Z (right) or B, A and Q (left).  The entries that a restoring step
// clears are set to exact zeros, so that the solves and residuals of the
// next panel see B's block structure exactly.
// ---------------------------------------------------------------------------
std::vector<int> ell_bounds(int m, int S) {
  std::vector<int> b{0};
  if (m <= 0) return b;
  if (m <= S) {
    b.push_back(m);
    return b;
  }
  const int p = m % S ? m % S : S;
  for (int e = p; e <= m; e += S) b.push_back(e);
  return b;
}

void absorb_ell(Ctx& c, int s, int k) {
  Work& w = *c.w;
  const int n = c.n, j = s + k, mp = n - j - 1, S = c.S;
  double *A = c.A, *B = c.B;
  const int lda = c.lda, ldb = c.ldb;
  c.absorptions++;
  const std::vector<int> bd = ell_bounds(mp, S);
  const int nblk = (int)bd.size() - 1;
  const int ldo = S + c.nb;  // rows of every window and restoring block
  double *Vw = w.pool[0][0], *Ww = w.pool[0][1];    // chain window (k reflectors)
  double *V1 = w.pool[1][0], *W1 = w.pool[1][1];    // restoring RQ / QR (block order)
  double *V2r = w.pool[2][0], *W2r = w.pool[2][1];  // its k-reflector reduction
  double *Ct = w.pool[3][0], *Mt = w.pool[3][1];    // copies and the factor's block
  double* V2 = w.V + k;
  copy_mat(c.st, mp, k, w.U + k, n, w.Ucp, n);

  // (3.3.1 b, c) V2 -> [0; L1] by QL windows from the top, one per diagonal
  // block with the rows carried from the window above; each window's
  // transform goes at once to B (rows above the window's end), A and Z.
  std::vector<int> carry_r(nblk, 0);
  {
    int carry = 0;
    for (int i = 0; i < nblk; ++i) {
      const int ws = bd[i] - carry, we = bd[i + 1], rows = we - ws;
      carry_r[i] = carry;
      carry = std::min(k, rows);
      if (i == 0 && nblk > 1 && rows <= k) continue;  // a small top block is carried whole
      chain(c, 1, false, rows, k, V2 + ws, n, Vw, Ww, ldo);
      right_apply(c, at(B, ldb, 0, j + 1 + ws), ldb, j + 1 + we, rows, k, Vw, Ww, ldo);
      right_apply(c, at(A, lda, 0, j + 1 + ws), lda, n, rows, k, Vw, Ww, ldo);
      if (c.wantZ) right_apply(c, at(c.Z, c.ldz, 0, j + 1 + ws), c.ldz, n, rows, k, Vw, Ww, ldo);
    }
  }
  right_rank_k(c, s, k);

  // (3.3.1 e) back to block upper triangular form, bottom block first: for
  // block i, C = B(block rows, window columns) = R Q (RQ through the QL
  // decomposition of C^T = Qf [0; L], Q = Qf^T); the first `cr` columns of
  // Qf, E1 - V1 W1(0:cr, :)^T, are reduced by a QR decomposition Qf2 [R2; 0],
  // and C Qf2 has zero first cr columns.
  for (int i = nblk - 1; i >= 1; --i) {
    const int cr = carry_r[i];
    if (cr <= 0) continue;
    const int a = bd[i], e = bd[i + 1], z = e - a, ws = a - cr, wdt = z + cr;
    double* C = at(B, ldb, j + 1 + a, j + 1 + ws);
    copy_mat(c.st, z, wdt, C, ldb, Ct, ldo);
    chain(c, 1, true, wdt, z, Ct, ldo, V1, W1, ldo);
    zero_mat(c.st, Mt, wdt, cr, ldo);
    set_identity(c.st, Mt, cr, ldo);
    gemm(c.st, false, true, wdt, cr, z, -1.0, V1, ldo, W1, ldo, 1.0, Mt, ldo);
    chain(c, 0, false, wdt, cr, Mt, ldo, V2r, W2r, ldo);
    right_apply(c, at(B, ldb, 0, j + 1 + ws), ldb, j + 1 + e, wdt, cr, V2r, W2r, ldo);
    right_apply(c, at(A, lda, 0, j + 1 + ws), lda, n, wdt, cr, V2r, W2r, ldo);
    if (c.wantZ) right_apply(c, at(c.Z, c.ldz, 0, j + 1 + ws), c.ldz, n, wdt, cr, V2r, W2r, ldo);
    zero_mat(c.st, C, z, cr, ldb);
  }

  spike(c, s, k);

  // (3.3.2 b, c, d) U2 -> [R1; 0] by QR windows from the bottom, aligned with
  // the tops of the diagonal blocks; each goes at once to B (columns j+1..),
  // A (columns j..) and Q.
  {
    int carry = 0;
    for (int i = nblk - 1; i >= 0; --i) {
      const int ws = bd[i], we = bd[i + 1] + carry, rows = we - ws;
      carry = std::min(k, rows);
      chain(c, 0, false, rows, k, w.Ucp + ws, n, Vw, Ww, ldo);
      left_apply(c, at(B, ldb, j + 1 + ws, j + 1), ldb, mp, rows, k, Vw, Ww, ldo);
      left_apply(c, at(A, lda, j + 1 + ws, j), lda, n - j, rows, k, Vw, Ww, ldo);
      if (c.wantQ) right_apply(c, at(c.Q, c.ldq, 0, j + 1 + ws), c.ldq, n, rows, k, Vw, Ww, ldo);
    }
  }
  copy_mat(c.st, k, k, w.U, n, w.Ucat, 2 * k);
  copy_mat(c.st, k, k, w.Ucp, n, w.Ucat + k, 2 * k);
  left_rank_k(c, s, k);
  if (c.wantQ) q_rank_k(c, s, k);

  // (3.3.2 f) back to block upper triangular form, top block first: for
  // block i and the k rows below it, C = B(rows, block columns) = Qf [R; 0];
  // the last k columns of Qf, E_last - V1 W1(z:z+k, :)^T, are reduced by a QL
  // decomposition Qf3 [0; L3], and Qf3^T C has zero last k rows.
  for (int i = 0; i + 1 < nblk; ++i) {
    const int a = bd[i], e = bd[i + 1], z = e - a, cr = std::min(k, mp - e), wdt = z + cr;
    if (cr <= 0) continue;
    double* C = at(B, ldb, j + 1 + a, j + 1 + a);
    copy_mat(c.st, wdt, z, C, ldb, Ct, ldo);
    chain(c, 0, false, wdt, z, Ct, ldo, V1, W1, ldo);
    zero_mat(c.st, Mt, wdt, cr, ldo);
    set_identity(c.st, Mt + z, cr, ldo);
    gemm(c.st, false, true, wdt, cr, z, -1.0, V1, ldo, W1 + z, ldo, 1.0, Mt, ldo);
    chain(c, 1, false, wdt, cr, Mt, ldo, V2r, W2r, ldo);
    left_apply(c, C, ldb, mp - a, wdt, cr, V2r, W2r, ldo);
    left_apply(c, at(A, lda, j + 1 + a, j), lda, n - j, wdt, cr, V2r, W2r, ldo);
    if (c.wantQ) right_apply(c, at(c.Q, c.ldq, 0, j + 1 + a), c.ldq, n, wdt, cr, V2r, W2r, ldo);
    zero_mat(c.st, at(B, ldb, j + 1 + e, j + 1 + a), cr, z, ldb);
  }
}

// ---------------------------------------------------------------------------
// Householder QR of the columns [c0, c0 + ncols) of M, rows [r0, n), for the
// steps before the reduction (the QR front end of the QZ algorithm, Sec. 1,
// and the zero-column preprocessing of Sec. 3.5).  Panels of nb columns;
// each panel is factored by a chain of window QRs from the bottom up, as U2
// in Sec. 3.3.2 b (windows of 2 nb rows moving by nb, the R factor of one
// window becoming the bottom of the next), so that its transformation is
// the window sequence the absorption already applies: from the left to the
// column ranges `lefts` (window rows only) and to the panel's own trailing
// columns, and from the right to the columns r..n-1 of Q.
// ---------------------------------------------------------------------------
struct LRange { double* X; int ld; int cs; int ce; };  // columns [cs, ce) of X

void qr_panels(Ctx& c, double* M, int ldm, int r0, int c0, int ncols,
               const std::vector<LRange>& lefts) {
  Work& w = *c.w;
  const int n = c.n, nb = c.nb;
  for (int p = 0; p < ncols; p += nb) {
    const int r = r0 + p, col = c0 + p;
    const int mp = n - r;
    if (mp <= 1) break;
    const int k = std::min(std::min(nb, ncols - p), mp);
    const Blocks bl = make_blocks(mp, k, nb);
    const int sb = bl.s, ldo = 2 * bl.s;
    if (k < sb) {
      const size_t slots = (size_t)(bl.T + 1) * 2 * sb * sb;
      for (int v = 0; v < 2; ++v) zero_mat(c.st, w.pool[2][v], (int)slots, 1, (int)slots);
    }
    const std::vector<Win> wins = left_windows(bl, 2);
    for (const Win& wn : wins)
      chain(c, 0, false, wn.wdt, k, at(M, ldm, r + wn.a, col), ldm, tV(w, 2, wn, sb),
            tW(w, 2, wn, sb), ldo);
    std::vector<RJob> jobs;
    if (col + k < c0 + ncols)
      jobs.push_back(RJob{at(M, ldm, 0, col + k), ldm, c0 + ncols - col - k, false, col + k});
    for (const LRange& lr : lefts)
      if (lr.ce > lr.cs) jobs.push_back(RJob{at(lr.X, lr.ld, 0, lr.cs), lr.ld, lr.ce - lr.cs, false, lr.cs});
    for (size_t i = 0; i < jobs.size(); i += 4) {
      std::vector<RJob> part(jobs.begin() + i, jobs.begin() + std::min(jobs.size(), i + 4));
      sweep_jobs(c, part, r - 1, bl, 2, wins, true);
    }
    if (c.wantQ) sweep_cols_right(c, c.Q, c.ldq, n, r - 1, bl, 2);
  }
}

// ---------------------------------------------------------------------------
// Algorithm 1.
// ---------------------------------------------------------------------------
int run(Ctx& c) {
  Work& w = *c.w;
  const int n = c.n, nb = c.nb;
  hipStream_t st = c.st;
  hipLaunchKernelGGL(k_init_ints, dim3(1), dim3(64), 0, st, w.ints);
  zero_lower(st, c.B, n, c.ldb, 0);
  fro_norm(st, n, n, c.B, c.ldb, w.dscal + 2, w.partials);
  if (n <= 2) return 0;

  // columns before ilo are already in final form (ht_preprocess)
  int s = c.opt.ilo;
  int64_t panel = 0;
  while (s <= n - 3) {
    const int L = n - s - 1;
    const int kmax = std::min(std::min(nb, n - 2 - s), L / 2);
    if (c.S > 0)  // block upper triangular B: LU of its diagonal blocks, once per panel
      lu_blocks(st, L, c.S, at(c.B, c.ldb, s + 1, s + 1), c.ldb, w.lu, n, w.perm, w.dscal + 2);
    else
      fix_diagonal(st, c.B, c.ldb, s + 1, n, w.dscal + 2, c.opt.seed, (uint64_t)panel + 1,
                   w.ints + 4);
    zero_mat(st, w.U, L, nb, n);
    zero_mat(st, w.V, L, nb, n);
    zero_mat(st, w.S, nb, nb, nb);
    zero_mat(st, w.T, nb, nb, nb);
    // (d) of column kk: right reflector on x; extend T and Y
    auto step_d = [&](int kk) {
      const ColBufs cb = colbufs(w, kk);
      const int j = s + kk, m = L - kk;
      double* x = cb.ysol + kk;
      double* vcol = at(w.V, n, kk, kk);
      house(st, m, x, vcol, w.dscal + 5, w.dscal + 6, false);
      if (kk > 0) gemv_t(st, m, kk, 1.0, w.V + kk, n, vcol, 0.0, w.tk, w.partials);
      wy_append(st, w.T, nb, kk, w.tk, w.dscal + 5);
      double* ycol = at(w.Y, n, 0, kk);
      const int pi = c.prof.begin(st, HT_PROF_YGEMV);
      gemv_n(st, L, m, 1.0, at(c.A, c.lda, s + 1, j + 1), c.lda, vcol, 1, 0.0, ycol, w.partials);
      c.prof.end(st, pi, 8.0 * L * (double)m);
      if (kk > 0)  // y = gamma (A v - Y (V^T v)), the scaling in the same launch
        gemv_n_small_scaled(st, L, kk, -1.0, w.Y, n, w.tk, 1.0, ycol, w.dscal + 5);
      else
        hipLaunchKernelGGL(k_scale_by, dim3((L + 255) / 256), dim3(256), 0, st, ycol, L,
                           w.dscal + 5);
      c.flops += 2.0 * L * (double)m + 4.0 * L * (double)kk;
    };
    // Column kk up to its first refinement verdict (posted, not read), then
    // (d) on the assumption that no refinement is needed.
    auto enqueue = [&](int kk) {
      const ColBufs cb = colbufs(w, kk);
      const int j = s + kk, m = L - kk;
      double* acol = at(c.A, c.lda, s + 1, j);
      copy(st, cb.save, acol, L);
      // (a) update column j with the kk pending reflector pairs
      if (kk > 0) {
        gemv_n(st, L, kk, -1.0, w.Y, n, w.V + (kk - 1), n, 1.0, acol, w.partials);
        wy_apply(st, L, L, 0, kk, -1.0, w.U, n, w.S, nb, true, acol, acol, w.tk, w.partials);
        c.flops += 6.0 * L * (double)kk;
      }
      // (b) left reflector on A(j+1:n, j); extend S
      double* ucol = at(w.U, n, kk, kk);
      house(st, m, acol + kk, ucol, w.dscal + 0, w.dscal + 1, true);
      if (kk > 0) gemv_t(st, m, kk, 1.0, w.U + kk, n, ucol, 0.0, w.tk, w.partials);
      wy_append(st, w.S, nb, kk, w.tk, w.dscal + 0);
      // (c) solve B~22 x = e1 via the enlarged system
      //   ctil = (I - U S U^T) e_kk, with U^T e_kk read as row kk of U
      factored_solve(c, s, kk, kk + 1, w.ctil, cb.ysol, cb.Erhs, kk);
      if (kk > 0) {  // the first column of a panel is not refined (Sec. 2.3)
        residual(c, s, kk, cb.ysol + kk, nullptr, cb);
        post_status(c, cb, kk);
      }
      step_d(kk);
    };
    // Refinement of column kk after a failed first verdict: correction
    // steps until the residual test passes or max_ir steps are spent.
    auto refine = [&](int kk) -> bool {
      const ColBufs cb = colbufs(w, kk);
      const int m = L - kk;
      double* x = cb.ysol + kk;
      int status = 0;
      for (int it = 0; !status && it < c.opt.max_ir; ++it) {
        // correction: solve B~22 d = r, x <- 2^{-E2} x + d
        pad_copy(st, w.ctil, kk, cb.rv, m);
        factored_solve(c, s, kk, kk + 1, w.ctil, w.dsol, w.ints + 2);
        ir_update(st, m, x, w.dsol + kk, w.ints + 2, cb.Erhs);
        residual(c, s, kk, x, nullptr, cb);
        status = sync_status(c, cb, kk);
        c.ir_steps++;
      }
      return status != 0;
    };

    // The columns run one ahead of their verdicts: column kk is enqueued
    // (including its (d)) before column kk-1's verdict is read, so the GPU
    // is not idle while the host waits.  When column kk-1 needs refinement,
    // column kk is rolled back (its column of A restored; everything else it
    // wrote is rewritten when it runs again), column kk-1 is refined and its
    // (d) redone, or, if refinement fails, undone as in Algorithm 1.  The
    // work that stands is the same, in the same order, as without the
    // speculation.
    int k = 0;
    int pending = -1;  // enqueued column whose verdict is not read yet
    int kk = 0;
    for (;;) {
      const bool enq = kk < kmax;
      if (enq) enqueue(kk);
      if (pending >= 0) {
        const int q = pending;
        pending = -1;
        if (q > 0 && !read_status(c, q)) {
          if (enq) copy(st, at(c.A, c.lda, s + 1, s + kk), colbufs(w, kk).save, L);
          c.cols_extra_ir++;
          if (!refine(q)) {
            // undo the left reflector: restore column s+q; U(:, q), S(:, q) are dropped
            copy(st, at(c.A, c.lda, s + 1, s + q), colbufs(w, q).save, L);
            c.ir_failures++;
            k = q;
            break;
          }
          step_d(q);
          c.columns++;
          if (enq) continue;  // column kk runs again
        } else {
          c.columns++;
        }
      }
      if (!enq) {
        k = kmax;
        break;
      }
      pending = kk++;
    }
    if (k == 0) return HT_ERR_HIP;  // cannot happen: the first column never refines
    if (c.S > 0) absorb_ell(c, s, k);
    else absorb(c, s, k);
    s += k;
    ++panel;
  }
  return 0;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int ht_default_options(ht_options* opt) {
  if (!opt) return -1;
  memset(opt, 0, sizeof(*opt));
  opt->struct_size = (int32_t)sizeof(ht_options);
  opt->nb = 64;
  opt->max_ir = 10;
  opt->qmode = HT_QZ_IDENTITY;
  opt->zmode = HT_QZ_IDENTITY;
  opt->prec = HT_PREC_FP64;
  opt->n_slices = 0;
  opt->flags = 0;
  opt->ir_tol_factor = 2.0;
  opt->seed = 0x5EEDull;
  opt->batch_block = 32;
  opt->batch_wg_per_cu = 3;
  opt->ell = 2;
  return 0;
}

// Diagonal block order of B in the l-block scheme (0: basic scheme).
static int ell_stride(const ht_options& o) { return o.ell > 2 ? (o.ell - 1) * o.nb : 0; }

static int resolve_opts(const ht_options* in, ht_options* out) {
  ht_default_options(out);
  if (!in) return 0;
  if (in->struct_size != (int32_t)sizeof(ht_options)) return -10;
  *out = *in;
  if (out->nb == 0) out->nb = 64;
  if (out->nb < 1 || out->nb > 128) return -10;
  if (out->max_ir < 0) return -10;
  if (out->qmode < 0 || out->qmode > 2 || out->zmode < 0 || out->zmode > 2) return -10;
  if (!(out->ir_tol_factor >= 0.0)) return -10;
  if (out->batch_block == 0) out->batch_block = 32;
  if (out->batch_wg_per_cu == 0) out->batch_wg_per_cu = 3;
  if (out->batch_block < 1 || out->batch_block > 64) return -10;
  if (out->batch_wg_per_cu < 1 || out->batch_wg_per_cu > 3) return -10;
  if (out->ilo < 0) return -10;
  if (out->ell == 0) out->ell = 2;
  if (out->ell < 2 || (out->ell > 2 && (out->ell - 1) * out->nb > 128)) return -10;
  if (out->prec < HT_PREC_FP64 || out->prec > HT_PREC_SPLIT_FP8) return -10;
  if (out->prec != HT_PREC_FP64) {
    const int fmt = out->prec == HT_PREC_SPLIT_BF16 ? 0 : 1;
    if (out->n_slices == 0) out->n_slices = split_default_slices(fmt);
    if (out->n_slices < 1 || out->n_slices > split_max_slices(fmt)) return -10;
  }
  return 0;
}

size_t ht_workspace_size(int64_t n, const ht_options* opt) {
  ht_options o;
  if (resolve_opts(opt, &o) != 0 || n < 0 || n > (1 << 30)) return 0;
  Work w;
  return layout(&w, (int)n, o.nb, nullptr, ell_stride(o)) + 256;
}

}  // extern "C"

namespace {

// Device memory of the allocation-free entry point ht_reduce_noalloc: one
// array per GPU, alive until the process ends.  Host code never passes the
// array's name to a kernel; it uses the device address that
// hipGetSymbolAddress returns for the current device (scratch_ptr).
constexpr size_t kScratchBytes = (size_t)HT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, resolved once per device.
int scratch_ptr(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HT_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HT_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = (char*)g_scratch_ptr[dev];
  return HT_OK;
}

// Bytes of the device workspace for order n, panel width nb, including the
// finite-scan flag at its end.
size_t workspace_need(int n, int nb, int S = 0) {
  Work w;
  return layout(&w, n, nb, nullptr, S) + 256;
}

// The common body of ht_reduce and ht_reduce_noalloc.  `ws` is the device
// workspace (caller's, the library's scratch, or NULL: allocate).  With
// `noalloc` nothing is allocated: the refinement verdict is read into
// pageable host memory of this call, and profiling is refused.
int reduce_impl(double* A, double* B, double* Q, double* Z, int64_t n, int64_t lda, int64_t ldb,
                int64_t ldq, int64_t ldz, const ht_options* opt, ht_stats* stats, char* ws,
                size_t ws_bytes, hipStream_t st, bool noalloc) {
  const auto t0 = std::chrono::steady_clock::now();
  ht_options o;
  int rc = resolve_opts(opt, &o);
  if (rc) return rc;
  if (n < 0 || n > (int64_t)1 << 30) return -5;
  const int64_t ldmin = std::max<int64_t>(1, n);
  // leading dimensions are carried as 32-bit integers by the kernels
  if (lda < ldmin || lda > INT32_MAX) return -6;
  if (ldb < ldmin || ldb > INT32_MAX) return -7;
  const bool wantQ = o.qmode != HT_QZ_NONE, wantZ = o.zmode != HT_QZ_NONE;
  if (wantQ && (ldq < ldmin || ldq > INT32_MAX)) return -8;
  if (wantZ && (ldz < ldmin || ldz > INT32_MAX)) return -9;
  if (n > 0 && (!A || !B)) return !A ? -1 : -2;
  if (n > 0 && wantQ && !Q) return -3;
  if (n > 0 && wantZ && !Z) return -4;
  if (o.ilo > std::max<int64_t>(n, 0)) return -10;
  if (noalloc && (o.flags & HT_FLAG_PROFILE)) return HT_ERR_UNSUPPORTED;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n == 0) return 0;

  const int ni = (int)n;
  const size_t need = workspace_need(ni, o.nb, ell_stride(o));
  char* base = ws;
  bool owned = false;
  if (base) {
    if (ws_bytes < need || ((uintptr_t)base & 255)) return HT_ERR_WORKSPACE;
  } else if (noalloc) {
    return HT_ERR_WORKSPACE;
  }

  // Q and Z start as I unless the caller's Q_in, Z_in are to be
  // accumulated: every update of Q and Z is a right multiplication over all
  // n rows (Sec. 3.3.1 d, 3.3.2 d), so Q_in Q and Z_in Z come out directly.
  if (wantQ && o.qmode == HT_QZ_IDENTITY) set_identity(st, Q, ni, (int)ldq);
  if (wantZ && o.zmode == HT_QZ_IDENTITY) set_identity(st, Z, ni, (int)ldz);

  // host memory for the refinement verdicts of this call: pinned (allocated
  // and freed here), or in the no-allocation form a pageable array
  int host_local[64] = {0};
  int* pinned = nullptr;
  if (!noalloc &&
      hipHostMalloc((void**)&pinned, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return HT_ERR_HIP;
  int* hints = pinned ? pinned : host_local;
  auto finish = [&](int code) {
    if (pinned) (void)hipHostFree(pinned);
    return code;
  };

  if (o.flags & HT_FLAG_CHECK_FINITE) {
    int* bad = nullptr;
    if (base) {
      bad = (int*)(base + need - 256);  // the flag word at the workspace's end
    } else if (hipMalloc(&bad, sizeof(int)) != hipSuccess) {
      return finish(HT_ERR_HIP);
    }
    (void)hipMemsetAsync(bad, 0, sizeof(int), st);
    hipLaunchKernelGGL(k_check_finite, dim3((ni + 255) / 256, ni), dim3(256), 0, st, ni, ni, A,
                       (int)lda, bad);
    hipLaunchKernelGGL(k_check_finite, dim3((ni + 255) / 256, ni), dim3(256), 0, st, ni, ni, B,
                       (int)ldb, bad);
    (void)hipMemcpyAsync(hints, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    if (!base) (void)hipFree(bad);
    if (hints[0]) return finish(HT_ERR_NONFINITE);
  }

  if (!base) {
    if (hipMalloc((void**)&base, need) != hipSuccess) return finish(HT_ERR_HIP);
    owned = true;
  }
  Work w;
  layout(&w, ni, o.nb, base, ell_stride(o));
  (void)hipMemsetAsync(w.flags, 0, trsv_flag_bytes(ni), st);

  Ctx c;
  c.st = st;
  c.w = &w;
  c.n = ni;
  c.nb = o.nb;
  c.S = ell_stride(o);
  c.A = A; c.B = B; c.Q = Q; c.Z = Z;
  c.lda = (int)lda; c.ldb = (int)ldb; c.ldq = (int)ldq; c.ldz = (int)ldz;
  c.wantQ = wantQ;
  c.wantZ = wantZ;
  c.opt = o;
  c.host_ints = hints;
  c.prof.on = (o.flags & HT_FLAG_PROFILE) != 0 && stats != nullptr;
  // events that let the host wait for a posted verdict alone (not in the
  // no-allocation form, which waits for the stream instead)
  if (!noalloc)
    for (int p = 0; p < 2; ++p)
      if (hipEventCreateWithFlags(&c.status_ev[p], hipEventDisableTiming) != hipSuccess)
        c.status_ev[p] = nullptr;
  rc = run(c);
  for (int p = 0; p < 2; ++p)
    if (c.status_ev[p]) (void)hipEventDestroy(c.status_ev[p]);
  const hipError_t le = hipGetLastError();
  if (rc == 0 && le != hipSuccess) { g_last_hip = le; rc = HT_ERR_HIP; }
  if (stats || owned) (void)hipStreamSynchronize(st);
  if (stats) {
    (void)hipMemcpyAsync(hints, w.ints, 8 * sizeof(int), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    stats->columns = c.columns;
    stats->cols_extra_ir = c.cols_extra_ir;
    stats->ir_steps = c.ir_steps;
    stats->ir_failures = c.ir_failures;
    stats->absorptions = c.absorptions;
    stats->scaled_solves = hints[5];
    stats->flops = c.flops;
    c.prof.collect(stats);
    stats->ms_total = std::chrono::duration<double, std::milli>(
        std::chrono::steady_clock::now() - t0).count();
  }
  c.prof.release();
  if (owned) (void)hipFree(base);
  return finish(rc);
}

// Workspace and context of the steps before the reduction (QR front end,
// preprocessing): the same workspace as ht_reduce.  Returns HT_OK or an
// error; on success the caller must call release().
struct StepCall {
  Work w;
  Ctx c;
  char* base = nullptr;
  bool owned = false;
  int host[64] = {0};
  int release(int rc) {
    if (owned) {
      (void)hipStreamSynchronize(c.st);
      (void)hipFree(base);
    }
    return rc;
  }
};

int step_setup(StepCall& sc, double* A, double* B, double* Q, double* Z, int n, int lda, int ldb,
               int ldq, int ldz, const ht_options& o, char* ws, size_t ws_bytes, hipStream_t st) {
  const size_t need = workspace_need(n, o.nb);
  sc.base = ws;
  if (ws) {
    if (ws_bytes < need || ((uintptr_t)ws & 255)) return HT_ERR_WORKSPACE;
  } else {
    if (hipMalloc((void**)&sc.base, need) != hipSuccess) return HT_ERR_HIP;
    sc.owned = true;
  }
  layout(&sc.w, n, o.nb, sc.base);
  Ctx& c = sc.c;
  c.st = st;
  c.w = &sc.w;
  c.n = n;
  c.nb = o.nb;
  c.A = A; c.B = B; c.Q = Q; c.Z = Z;
  c.lda = lda; c.ldb = ldb; c.ldq = ldq; c.ldz = ldz;
  c.wantQ = o.qmode != HT_QZ_NONE;
  c.wantZ = o.zmode != HT_QZ_NONE;
  c.opt = o;
  c.host_ints = sc.host;
  return HT_OK;
}

// Common argument checks (argument positions as in ht_preprocess).
int step_args(const ht_options* opt, ht_options* o, int64_t n, int64_t lda, int64_t ldb,
              int64_t ldq, int64_t ldz, const double* A, const double* B, const double* Q,
              const double* Z, bool useZ) {
  const int rc = resolve_opts(opt, o);
  if (rc) return rc;
  if (o->prec != HT_PREC_FP64) return HT_ERR_UNSUPPORTED;
  if (n < 0 || n > (int64_t)1 << 30) return -5;
  const int64_t ldmin = std::max<int64_t>(1, n);
  if (lda < ldmin || lda > INT32_MAX) return -6;
  if (ldb < ldmin || ldb > INT32_MAX) return -7;
  const bool wantQ = o->qmode != HT_QZ_NONE, wantZ = useZ && o->zmode != HT_QZ_NONE;
  if (wantQ && (ldq < ldmin || ldq > INT32_MAX)) return -8;
  if (wantZ && (ldz < ldmin || ldz > INT32_MAX)) return -9;
  if (n > 0 && (!A || !B)) return !A ? -1 : -2;
  if (n > 0 && wantQ && !Q) return -3;
  if (n > 0 && wantZ && !Z) return -4;
  return HT_OK;
}

}  // namespace

extern "C" {

int ht_reduce(double* A, double* B, double* Q, double* Z, int64_t n, int64_t lda, int64_t ldb,
              int64_t ldq, int64_t ldz, const ht_options* opt, ht_stats* stats, void* workspace,
              size_t ws_bytes, void* stream) {
  return reduce_impl(A, B, Q, Z, n, lda, ldb, ldq, ldz, opt, stats, (char*)workspace, ws_bytes,
                     (hipStream_t)stream, false);
}

int ht_reduce_noalloc(double* A, double* B, double* Q, double* Z, int64_t n, int64_t lda,
                      int64_t ldb, int64_t ldq, int64_t ldz, const ht_options* opt,
                      ht_stats* stats, void* stream) {
  ht_options o;
  const int orc = resolve_opts(opt, &o);
  if (orc) return orc;
  if (n < 0 || n > (int64_t)1 << 30) return -5;
  if (n > 0 && workspace_need((int)n, o.nb, ell_stride(o)) > kScratchBytes)
    return HT_ERR_TOO_LARGE;
  char* p = nullptr;
  if (n > 0) {
    const int src = scratch_ptr(&p);
    if (src != HT_OK) return src;
  }
  return reduce_impl(A, B, Q, Z, n, lda, ldb, ldq, ldz, opt, stats, p, kScratchBytes,
                     (hipStream_t)stream, true);
}

int ht_triangularize_b(double* A, double* B, double* Q, int64_t n, int64_t lda, int64_t ldb,
                       int64_t ldq, const ht_options* opt, void* workspace, size_t ws_bytes,
                       void* stream) {
  ht_options o;
  int rc = step_args(opt, &o, n, lda, ldb, ldq, 1, A, B, Q, nullptr, false);
  if (rc) return rc;
  if (n == 0) return HT_OK;
  hipStream_t st = (hipStream_t)stream;
  const int ni = (int)n;
  if (o.qmode == HT_QZ_IDENTITY) set_identity(st, Q, ni, (int)ldq);
  StepCall sc;
  o.zmode = HT_QZ_NONE;
  rc = step_setup(sc, A, B, Q, nullptr, ni, (int)lda, (int)ldb, (int)ldq, 1, o, (char*)workspace,
                  ws_bytes, st);
  if (rc) return rc;
  qr_panels(sc.c, B, (int)ldb, 0, 0, ni, {LRange{A, (int)lda, 0, ni}});
  zero_lower(st, B, ni, (int)ldb, 0);
  if (hipGetLastError() != hipSuccess) rc = HT_ERR_HIP;
  return sc.release(rc);
}

int ht_preprocess(double* A, double* B, double* Q, double* Z, int64_t n, int64_t lda,
                  int64_t ldb, int64_t ldq, int64_t ldz, const ht_options* opt, int32_t* ilo,
                  void* workspace, size_t ws_bytes, void* stream) {
  ht_options o;
  int rc = step_args(opt, &o, n, lda, ldb, ldq, ldz, A, B, Q, Z, true);
  if (rc) return rc;
  if (!ilo) return -11;
  *ilo = 0;
  if (n == 0) return HT_OK;
  hipStream_t st = (hipStream_t)stream;
  const int ni = (int)n;
  const bool wantQ = o.qmode != HT_QZ_NONE, wantZ = o.zmode != HT_QZ_NONE;

  // which columns of B are zero, and is B diagonal (its strictly lower
  // triangle is ignored, as by ht_reduce: cleared first)
  zero_lower(st, B, ni, (int)ldb, 0);
  int* dflags = nullptr;
  if (hipMalloc((void**)&dflags, (size_t)(ni + 1) * sizeof(int)) != hipSuccess) return HT_ERR_HIP;
  (void)hipMemsetAsync(dflags, 0, (size_t)(ni + 1) * sizeof(int), st);
  hipLaunchKernelGGL(k_zero_columns, dim3(ni), dim3(256), 0, st, ni, B, (int)ldb, dflags,
                     dflags + ni);
  std::vector<int> zf((size_t)ni + 1);
  if (hipMemcpyAsync(zf.data(), dflags, zf.size() * sizeof(int), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(dflags);
    return HT_ERR_HIP;
  }
  std::vector<int> perm;
  for (int j = 0; j < ni; ++j)
    if (zf[j]) perm.push_back(j);
  const int ell = (int)perm.size();
  const bool diagonal = zf[ni] == 0;
  if (ell <= 1) {  // the preprocessing needs more than one zero column
    (void)hipFree(dflags);
    if (wantQ && o.qmode == HT_QZ_IDENTITY) set_identity(st, Q, ni, (int)ldq);
    if (wantZ && o.zmode == HT_QZ_IDENTITY) set_identity(st, Z, ni, (int)ldz);
    return hipGetLastError() == hipSuccess ? HT_OK : HT_ERR_HIP;
  }
  for (int j = 0; j < ni; ++j)
    if (!zf[j]) perm.push_back(j);

  // Z0 moves the zero columns to the front; Q0 = Z0 when B is diagonal
  int* dperm = dflags;  // reuse: n ints
  double* tmp = nullptr;
  rc = HT_OK;
  if (hipMemcpyAsync(dperm, perm.data(), (size_t)ni * sizeof(int), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMalloc((void**)&tmp, (size_t)ni * ni * sizeof(double)) != hipSuccess)
    rc = HT_ERR_HIP;
  if (rc == HT_OK) {
    const dim3 grid((ni + 255) / 256, ni);
    const int* rp = diagonal ? dperm : nullptr;
    double* M[2] = {A, B};
    const int ldm[2] = {(int)lda, (int)ldb};
    for (int t = 0; t < 2; ++t) {
      copy_mat(st, ni, ni, M[t], ldm[t], tmp, ni);
      hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, st, ni, tmp, ni, M[t], ldm[t], rp, dperm);
    }
    if (wantZ) {
      const bool acc = o.zmode == HT_QZ_ACCUMULATE;
      if (acc) copy_mat(st, ni, ni, Z, (int)ldz, tmp, ni);
      hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, st, ni, acc ? tmp : nullptr, ni, Z,
                         (int)ldz, nullptr, dperm);
    }
    if (wantQ) {
      const bool acc = o.qmode == HT_QZ_ACCUMULATE;
      if (diagonal) {
        if (acc) copy_mat(st, ni, ni, Q, (int)ldq, tmp, ni);
        hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, st, ni, acc ? tmp : nullptr, ni, Q,
                           (int)ldq, nullptr, dperm);
      } else if (!acc) {
        set_identity(st, Q, ni, (int)ldq);
      }
    }
    StepCall sc;
    rc = step_setup(sc, A, B, Q, Z, ni, (int)lda, (int)ldb, (int)ldq, (int)ldz, o,
                    (char*)workspace, ws_bytes, st);
    if (rc == HT_OK) {
      // QR of the first l columns of A0: A1 = [A11 A12; 0 A22], B1 = [0 B12; 0 B22]
      qr_panels(sc.c, A, (int)lda, 0, 0, ell,
                {LRange{A, (int)lda, ell, ni}, LRange{B, (int)ldb, ell, ni}});
      // B22 made triangular again, its transformation applied to A22
      qr_panels(sc.c, B, (int)ldb, ell, ell, ni - ell, {LRange{A, (int)lda, ell, ni}});
      zero_lower(st, B, ni, (int)ldb, 0);
      if (hipGetLastError() != hipSuccess) rc = HT_ERR_HIP;
      rc = sc.release(rc);
    }
  }
  (void)hipStreamSynchronize(st);
  if (tmp) (void)hipFree(tmp);
  (void)hipFree(dflags);
  if (rc == HT_OK) *ilo = ell;
  return rc;
}

const char* ht_strerror(int code) {
  if (code < 0) return "invalid argument";
  switch (code) {
    case HT_OK: return "success";
    case HT_ERR_HIP: return "HIP runtime error";
    case HT_ERR_WORKSPACE: return "workspace too small or misaligned";
    case HT_ERR_NONFINITE: return "NaN or Inf in the input";
    case HT_ERR_UNSUPPORTED: return "unsupported option combination";
    case HT_ERR_NOLIB: return "device code missing for this GPU";
    case HT_ERR_TOO_LARGE:
      return "order too large for the library's fixed scratch (ht_reduce_noalloc)";
  }
  return "unknown error";
}

const char* ht_version(void) { return "htred 0.1 gfx950"; }

size_t ht_batched_workspace_size(int32_t batch, int32_t nmax, const ht_options* opt) {
  ht_options o;
  if (resolve_opts(opt, &o) != 0 || batch < 0 || nmax < 0 || nmax > 512) return 0;
  return batched_workspace_bytes(batch, std::max(nmax, 1), o.batch_wg_per_cu) + 256;
}

int ht_reduce_batched(int32_t batch, const int32_t* n_dev, double* const* A_dev,
                      double* const* B_dev, double* const* Q_dev, double* const* Z_dev,
                      const int32_t* ld_dev, int32_t* info_dev, int32_t nmax,
                      const ht_options* opt, void* workspace, size_t ws_bytes, void* stream) {
  if (batch < 0) return -1;
  if (batch == 0) return HT_OK;
  if (!n_dev) return -2;
  if (!A_dev || !B_dev) return -3;
  if (!Q_dev || !Z_dev) return -5;
  if (!ld_dev) return -7;
  if (!info_dev) return -8;
  if (nmax < 0 || nmax > 512) return -9;
  ht_options o;
  const int rc = resolve_opts(opt, &o);
  if (rc != 0) return rc;
  if (o.prec != HT_PREC_FP64) return HT_ERR_UNSUPPORTED;
  if (!workspace || ((uintptr_t)workspace & 255) ||
      ws_bytes < batched_workspace_bytes(batch, std::max(nmax, 1), o.batch_wg_per_cu))
    return HT_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  // the panel width of the batched form is the caller's nb as given (0: one
  // panel over each whole pencil); no options means the defaults
  const int nb = opt ? std::max(opt->nb, 0) : o.nb;
  batched_reduce(st, batch, n_dev, A_dev, B_dev, Q_dev, Z_dev, ld_dev, info_dev,
                 std::max(nmax, 1), nb, o.batch_block, o.batch_wg_per_cu, o.max_ir,
                 o.ir_tol_factor, o.seed, workspace);
  if (hipGetLastError() != hipSuccess) return HT_ERR_HIP;
  return HT_OK;
}

int ht_batched_pencil_stats(const void* workspace, int32_t batch, int64_t* out, void* stream) {
  constexpr int W = 8;  // words per pencil in the device record
  if (batch < 0) return -2;
  if (batch == 0) return HT_OK;
  if (!workspace) return -1;
  if (!out) return -3;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int64_t> raw((size_t)batch * W);
  if (hipMemcpyAsync(raw.data(), batched_stats_ptr(workspace, batch), raw.size() * 8,
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HT_ERR_HIP;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return HT_ERR_HIP;
  int64_t t0 = raw[0];
  for (int i = 1; i < batch; ++i) t0 = std::min(t0, raw[W * (size_t)i]);
  const double ns_per_tick = 1.0e6 / (double)khz;
  auto ns = [&](int64_t ticks) { return (int64_t)((double)ticks * ns_per_tick); };
  for (int i = 0; i < batch; ++i) {
    const int64_t* r = &raw[W * (size_t)i];
    int64_t* o = out + 8 * (size_t)i;
    o[0] = ns(r[0] - t0);
    o[1] = ns(r[1] - t0);
    o[2] = r[2];
    o[3] = r[3];
    o[4] = ns(r[4]);
    o[5] = ns(r[5]);
    o[6] = ns(r[6]);
    o[7] = ns(r[7]);
  }
  return HT_OK;
}

int ht_check(const double* A0, const double* B0, const double* H, const double* T,
             const double* Q, const double* Z, int64_t n, int64_t ld, double* out, void* stream) {
  if (n < 0 || n > INT32_MAX) return -7;
  if (ld < std::max<int64_t>(1, n)) return -8;
  if (!out) return -9;
  if (n == 0) {
    for (int i = 0; i < 4; ++i) out[i] = 0.0;
    return HT_OK;
  }
  const double* ptrs[6] = {A0, B0, H, T, Q, Z};
  for (int i = 0; i < 6; ++i)
    if (!ptrs[i]) return -(i + 1);
  hipStream_t st = (hipStream_t)stream;
  const int ni = (int)n, ldi = (int)ld;
  const size_t sq = (size_t)ni * ni;
  double *W1 = nullptr, *W2 = nullptr, *part = nullptr, *res = nullptr;
  if (hipMalloc((void**)&W1, sq * 8) != hipSuccess) return HT_ERR_HIP;
  if (hipMalloc((void**)&W2, sq * 8) != hipSuccess) { (void)hipFree(W1); return HT_ERR_HIP; }
  if (hipMalloc((void**)&part, (size_t)2 * ni * 8 + 64 * 8) != hipSuccess) {
    (void)hipFree(W1);
    (void)hipFree(W2);
    return HT_ERR_HIP;
  }
  res = part + 2 * (size_t)ni;
  // res[0] = ||Q H Z^T - A0||, res[1] = ||A0||, res[2], res[3] the same for
  // T and B0, res[4] = ||Q^T Q - I||, res[5] = ||Z^T Z - I|| (Frobenius)
  const double* X[2] = {H, T};
  const double* X0[2] = {A0, B0};
  for (int t = 0; t < 2; ++t) {
    htk::gemm(st, false, false, ni, ni, ni, 1.0, Q, ldi, X[t], ldi, 0.0, W1, ni);
    htk::copy_mat(st, ni, ni, X0[t], ldi, W2, ni);
    htk::gemm(st, false, true, ni, ni, ni, 1.0, W1, ni, Z, ldi, -1.0, W2, ni);
    htk::fro_norm(st, ni, ni, W2, ni, res + 2 * t, part);
    htk::fro_norm(st, ni, ni, X0[t], ldi, res + 2 * t + 1, part);
  }
  const double* O[2] = {Q, Z};
  for (int t = 0; t < 2; ++t) {
    htk::set_identity(st, W1, ni, ni);
    htk::gemm(st, true, false, ni, ni, ni, 1.0, O[t], ldi, O[t], ldi, -1.0, W1, ni);
    htk::fro_norm(st, ni, ni, W1, ni, res + 4 + t, part);
  }
  double h[6];
  int rc = HT_OK;
  if (hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    rc = HT_ERR_HIP;
  (void)hipFree(W1);
  (void)hipFree(W2);
  (void)hipFree(part);
  if (rc != HT_OK) return rc;
  out[0] = h[0] / (h[1] > 0.0 ? h[1] : 1.0);
  out[1] = h[2] / (h[3] > 0.0 ? h[3] : 1.0);
  out[2] = h[4];
  out[3] = h[5];
  return HT_OK;
}

int ht_wy_gemm(int32_t prec, int32_t n_slices, int32_t transA, int32_t transB, int64_t m,
               int64_t n, int64_t k, double alpha, const double* A, int64_t lda, const double* B,
               int64_t ldb, double beta, double* C, int64_t ldc, void* stream) {
  if (prec < HT_PREC_FP64 || prec > HT_PREC_SPLIT_FP8) return -1;
  const int fmt = prec == HT_PREC_SPLIT_BF16 ? 0 : 1;
  int ns = n_slices;
  if (prec != HT_PREC_FP64) {
    if (ns == 0) ns = split_default_slices(fmt);
    if (ns < 1 || ns > split_max_slices(fmt)) return -2;
  }
  if (m < 0 || m > INT32_MAX) return -5;
  if (n < 0 || n > INT32_MAX) return -6;
  if (k < 0 || k > INT32_MAX) return -7;
  const int64_t ra = transA ? k : m, rb = transB ? n : k;
  if (lda < std::max<int64_t>(1, ra)) return -10;
  if (ldb < std::max<int64_t>(1, rb)) return -12;
  if (ldc < std::max<int64_t>(1, m)) return -15;
  if (m == 0 || n == 0) return HT_OK;
  if (k > 0 && !A) return -9;
  if (k > 0 && !B) return -11;
  if (!C) return -14;
  hipStream_t st = (hipStream_t)stream;
  if (prec == HT_PREC_FP64)
    htk::gemm(st, transA != 0, transB != 0, (int)m, (int)n, (int)k, alpha, A, (int)lda, B,
              (int)ldb, beta, C, (int)ldc);
  else
    htk::split_gemm(st, fmt, ns, transA != 0, transB != 0, (int)m, (int)n, (int)k, alpha, A,
                    (int)lda, B, (int)ldb, beta, C, (int)ldc);
  return hipGetLastError() == hipSuccess ? HT_OK : HT_ERR_HIP;
}

}  // extern "C"
