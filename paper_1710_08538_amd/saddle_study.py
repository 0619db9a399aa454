"""Saddle-point pencils with and without the zero-column preprocessing.

The pencils of the paper's Test Suite 4 (Sec. 4): A = [X Y; Y^T 0],
B = diag(I, 0) with X symmetric positive definite of order 3n/4 and Y of
full rank (inputs.saddle_pencil).  B has n/4 zero columns, so the pencil has
many infinite eigenvalues and the solves with B need iterative refinement,
which often fails and cuts panels short.  For each order the script reduces
the same pencil twice on the GPU -- ht_reduce directly, and ht_preprocess
followed by ht_reduce from column ilo -- and reports the statistics of the
paper's table for this test suite: the share of reduced columns whose
refinement failed, the share that needed extra refinement steps, and the
average number of refinement steps per column, beside the time and the
backward errors (ht_check).

Usage: python -m paper_1710_08538_amd.saddle_study [--n 1000 4000] [--nb 64]
Prints one JSON object per order.
"""
import argparse
import json
import time

import torch

from paper_1710_08538_amd import htred, inputs


def one(n, nb, pre, seed):
    A0, B0 = inputs.saddle_pencil(n, seed=seed)
    A0d, B0d = htred.to_device_colmajor(A0), htred.to_device_colmajor(B0)
    A, B = A0d.clone(), B0d.clone()
    Q, Z = htred.colmajor_empty(n), htred.colmajor_empty(n)
    ws = torch.empty(htred.workspace_size(n, nb=nb), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t = time.time()
    ilo = 0
    kw = {}
    if pre:
        _, _, ilo = htred.preprocess(A, B, Q, Z, nb=nb, workspace=ws)
        kw = dict(ilo=ilo, qmode=htred.HT_QZ_ACCUMULATE, zmode=htred.HT_QZ_ACCUMULATE)
    st = htred.reduce(A, B, Q, Z, nb=nb, stats=True, workspace=ws, **kw)[2]
    torch.cuda.synchronize()
    dt = time.time() - t
    err = htred.check(A0d, B0d, A, B, Q, Z)
    cols = max(st["columns"], 1)
    return {"preprocessing": pre, "ilo": ilo, "time_s": dt, "columns": st["columns"],
            "pct_columns_failed_ir": 100.0 * st["ir_failures"] / cols,
            "pct_columns_extra_ir": 100.0 * st["cols_extra_ir"] / cols,
            "avg_ir_steps_per_column": st["ir_steps"] / cols,
            "absorptions": st["absorptions"], "backward_error": err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[1000, 4000])
    ap.add_argument("--nb", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    for n in args.n:
        one(min(n, 256), args.nb, True, args.seed)  # warm-up of both paths
        res = {"n": n, "nb": args.nb, "seed": args.seed,
               "plain": one(n, args.nb, False, args.seed),
               "preprocessed": one(n, args.nb, True, args.seed)}
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
