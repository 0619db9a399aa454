"""Panel-width autotuner for ht_reduce and ht_reduce_batched.

The panel width nb (reflector pairs per absorption, Sec. 3.3) trades the
length of the absorption chains and the width of the WY products against
the number of panels.  This tool times ht_reduce on the GPU for every
candidate nb at a grid of orders (random pencils of the paper's first test
generator), keeps the fastest nb per order, and writes the table to
``nb_table.json`` beside this file.  ``htred.reduce(nb=0)`` then takes nb
from the table entry of the nearest order (log scale); without a table it
uses the library default.

With ``--batched`` it also times the batched form on the batched workload
(orders U{32..512}, child seeds of SeedSequence(4)) for panel widths 0 (one
panel per pencil), 32, 64 and 128, and stores the fastest; ``BatchedPlan``
uses it when no nb is given.

    python -m paper_1710_08538_amd.autotune [--orders 1024 2048 4096] [--nb 32 64 128] [--batched]
"""
import argparse
import json
import math
import os
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "nb_table.json")
CANDIDATES = (32, 64, 128)


def load_table(path=TABLE):
    """{order: nb} from the table file, or {} if there is none."""
    try:
        with open(path) as f:
            data = json.load(f)
        return {int(k): int(v["nb"]) for k, v in data["orders"].items()}
    except (OSError, ValueError, KeyError):
        return {}


BATCHED_DEFAULT = 64
BATCHED_CANDIDATES = (0, 32, 64, 128)


def load_batched(path=TABLE):
    """The tuned panel width of the batched form, or None."""
    try:
        with open(path) as f:
            return int(json.load(f)["batched"]["nb"])
    except (OSError, ValueError, KeyError, TypeError):
        return None


def pick_batched_nb(path=TABLE):
    nb = load_batched(path)
    return BATCHED_DEFAULT if nb is None else nb


def pick_nb(n, table=None):
    """nb for order n: the table entry of the nearest order (log scale), or
    0 (library default) without a table."""
    table = load_table() if table is None else table
    if not table or n <= 0:
        return 0
    best = min(table, key=lambda m: abs(math.log(m) - math.log(n)))
    return table[best]


def time_reduce(htred, inputs, torch, n, nb, reps):
    A0, B0 = inputs.random_pencil(n, seed=7000 + n)
    A0d, B0d = htred.to_device_colmajor(A0), htred.to_device_colmajor(B0)
    A, B = htred.colmajor_empty(n), htred.colmajor_empty(n)
    Q, Z = htred.colmajor_empty(n), htred.colmajor_empty(n)
    best = float("inf")
    for r in range(reps + 1):  # the first run warms up
        A.copy_(A0d)
        B.copy_(B0d)
        torch.cuda.synchronize()
        t = time.time()
        htred.reduce(A, B, Q, Z, nb=nb)
        torch.cuda.synchronize()
        if r > 0:
            best = min(best, time.time() - t)
    return best


def time_batched(htred, inputs, torch, nb, count=2048, seed=4, reps=1):
    pencils = inputs.batch_pencils(count, seed)
    A0s = [htred.to_device_colmajor(A) for A, _ in pencils]
    B0s = [htred.to_device_colmajor(B) for _, B in pencils]
    As = [A.clone() for A in A0s]
    Bs = [B.clone() for B in B0s]
    Qs = [htred.colmajor_empty(A.shape[0]) for A in As]
    Zs = [htred.colmajor_empty(A.shape[0]) for A in As]
    plan = htred.BatchedPlan(As, Bs, Qs, Zs, nb=nb)
    best = float("inf")
    for r in range(reps + 1):
        for i in range(count):
            As[i].copy_(A0s[i])
            Bs[i].copy_(B0s[i])
        torch.cuda.synchronize()
        t = time.time()
        plan.run()
        torch.cuda.synchronize()
        if r > 0:
            best = min(best, time.time() - t)
    if not bool((plan.info[:count].cpu() == 0).all()):
        raise RuntimeError("batched reduction reported errors at nb=%d" % nb)
    return best


def tune_batched(candidates=BATCHED_CANDIDATES, reps=1, path=TABLE):
    import torch
    from paper_1710_08538_amd import htred, inputs
    if not torch.cuda.is_available():
        raise RuntimeError("the autotuner times the GPU path and needs a GPU")
    times = {}
    for nb in candidates:
        times[nb] = time_batched(htred, inputs, torch, nb, reps=reps)
        print("autotune: batched nb=%d %.3f s" % (nb, times[nb]), flush=True)
    best = min(times, key=times.get)
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data["batched"] = {"nb": best, "workload": "2048 pencils, orders U{32..512}, seed 4",
                       "seconds": {str(k): v for k, v in times.items()}}
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    return data


def tune(orders, candidates=CANDIDATES, reps=1, path=TABLE):
    import torch
    from paper_1710_08538_amd import htred, inputs
    if not torch.cuda.is_available():
        raise RuntimeError("the autotuner times the GPU path and needs a GPU")
    result = {}
    for n in orders:
        times = {}
        for nb in candidates:
            if nb >= n:
                continue
            times[nb] = time_reduce(htred, inputs, torch, n, nb, reps)
            print("autotune: n=%d nb=%d %.3f s" % (n, nb, times[nb]), flush=True)
        nb_best = min(times, key=times.get)
        result[str(n)] = {"nb": nb_best, "seconds": {str(k): v for k, v in times.items()}}
    data = {"device": torch.cuda.get_device_name(0), "generator": "random_pencil",
            "orders": result}
    old = {}
    try:
        with open(path) as f:
            old = json.load(f)
    except (OSError, ValueError):
        pass
    if "batched" in old:
        data["batched"] = old["batched"]
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    return data


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--orders", type=int, nargs="+", default=[512, 1024, 2048, 4096, 8192])
    ap.add_argument("--nb", type=int, nargs="+", default=list(CANDIDATES))
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--batched", action="store_true", help="also tune the batched form")
    ap.add_argument("--only-batched", action="store_true")
    args = ap.parse_args()
    if not args.only_batched:
        tune(args.orders, tuple(args.nb), args.reps, args.out)
    if args.batched or args.only_batched:
        tune_batched(reps=args.reps, path=args.out)
    with open(args.out) as f:
        print(f.read())


if __name__ == "__main__":
    main()
