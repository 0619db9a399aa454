// ht_sweep.h -- launch interface of the fused block-reflector sweeps.
#pragma once
#include <hip/hip_runtime.h>

namespace htk {

// One matrix (or row range of a matrix) swept by the same window sequence.
struct SweepJob {
  double* X;     // row 0 of the job (column indices are absolute)
  int ld;
  int nrows;     // rows 0 .. nrows-1 (columns, for a transposed sweep)
  int tri;       // 1: X is upper triangular in global indices (skip zero windows)
  int tri_off;   // global row (column, transposed) index of the job's row 0
  int wg0;       // first workgroup of this job in the launch
};

struct SweepArgs {
  SweepJob job[4];
  int njobs;
  int nwin;           // number of windows (width 2k, stride k)
  int c0;             // absolute column of window 0
  const double* Vp;   // pool of V factors (2k x k, column-major, ld 2k)
  const double* Wp;   // pool of W factors
  int slot0;          // window w uses slot slot0 + w * slot_step
  int slot_step;      // (slot stride 2 k^2 doubles)
  // Nonzero part of every slot of the run: rows [16 tlo, 16 thi) of V and W
  // (window positions) and columns [0, 16 phi) (reflectors); products with
  // the zero tiles outside are skipped.  0, 2k/16, k/16 for full windows.
  int tlo, thi, phi;
};

bool sweep_supported(int k);
// X(:, win) <- X(:, win) - (X(:, win) V) W^T for every window in order;
// dir = +1 (windows move right) or -1 (left).  trans: sweep X^T instead,
// i.e. X(win, :) <- X(win, :) - W (V^T X(win, :)) over slabs of columns
// (job.X at the job's first column, window indices = absolute rows).
void sweep_rows(hipStream_t st, const SweepArgs& args, int k, int dir, bool trans = false);

}  // namespace htk
