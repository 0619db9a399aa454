"""Panel-width autotuner for ht_reduce.

The panel width nb (reflector pairs per absorption, Sec. 3.3) trades the
length of the absorption chains and the width of the WY products against
the number of panels.  This tool times ht_reduce on the GPU for every
candidate nb at a grid of orders (random pencils of the paper's first test
generator), keeps the fastest nb per order, and writes the table to
``nb_table.json`` beside this file.  ``htred.reduce(nb=0)`` then takes nb
from the table entry of the nearest order (log scale); without a table it
uses the library default.

    python -m paper_1710_08538_amd.autotune [--orders 1024 2048 4096] [--nb 32 64 128]
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
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    return data


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--orders", type=int, nargs="+", default=[512, 1024, 2048, 4096, 8192])
    ap.add_argument("--nb", type=int, nargs="+", default=list(CANDIDATES))
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    data = tune(args.orders, tuple(args.nb), args.reps, args.out)
    print(json.dumps(data))


if __name__ == "__main__":
    main()
