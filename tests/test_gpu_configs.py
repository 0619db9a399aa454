"""Entry-by-entry parity of the binding workload configurations with the
O(n^3) CPU oracle (O-fast: Algorithm 2's reflector pair per column with B
kept triangular by Givens QR updates), plus the precision form on the
headline pencil.

* n = 4096 random pencil (Test Suite 1 generator, seed 1): every entry of
  the sign-normalised H, T, Q, Z at panel widths 32, 64 and 128 in FP64 and
  with BF16 / FP8 split WY products, against one O-fast reduction of the same
  pencil (tolerance 1e-10 relative to ||A||_F, ||B||_F, sqrt(n)).
* the batched workload (2048 pencils, orders U{32..512}, child seeds of
  SeedSequence(4)): one persistent launch at the tuned parameters, every
  pencil compared entry by entry with its own O-fast reduction (host
  threads, one oracle call each) and checked against the invariants.
* the n = 16384 ill-conditioned pencil with split WY products: the
  invariants of Theorem A.1 (B is numerically singular there, so T is not
  numerically unique and entries are not compared), and a backward error
  within a small factor of the native FP64 run's on the same pencil.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from oracle import checks
from paper_1710_08538_amd import htred, inputs

pytestmark = pytest.mark.gpu
TOL = 1e-10


def host_workers():
    """Worker threads for the host-side oracle: the CPUs this process may
    run on, at most 16."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return max(1, min(16, ncpu))


@pytest.fixture(scope="module")
def n4096_oracle():
    A0, B0 = inputs.workload("n4096")
    print("O-fast oracle n=4096 on %d threads" % host_workers(), flush=True)
    ref = oracle.fast_ht(A0, B0, threads=host_workers())[:4]
    return A0, B0, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("nb,prec", [(32, "fp64"), (64, "fp64"), (128, "fp64"),
                                     (128, "bf16"), (128, "fp8")])
def test_config_n4096_every_entry(n4096_oracle, nb, prec):
    A0, B0, ref = n4096_oracle
    n = A0.shape[0]
    p = {"fp64": htred.HT_PREC_FP64, "bf16": htred.HT_PREC_SPLIT_BF16,
         "fp8": htred.HT_PREC_SPLIT_FP8}[prec]
    print("ht_reduce n=4096 nb=%d prec=%s" % (nb, prec), flush=True)
    A = htred.to_device_colmajor(A0)
    B = htred.to_device_colmajor(B0)
    Q, Z = htred.reduce(A, B, nb=nb, prec=p)
    torch.cuda.synchronize()
    Ad, Bd = htred.to_device_colmajor(A0), htred.to_device_colmajor(B0)
    inv = checks.invariants(Ad, Bd, A, B, Q, Z)
    assert checks.invariants_ok(inv, n), inv
    del Ad, Bd
    got = tuple(M.cpu().numpy() for M in (A, B, Q, Z))
    d = checks.compare(ref, got, A0, B0)
    print("n=4096 nb=%d %s: %s" % (nb, prec, {k: "%.2e" % v for k, v in d.items()}), flush=True)
    for key in ("max_H", "max_T", "max_Q", "max_Z"):
        assert d[key] <= TOL, (key, d)


BATCH_COUNT, BATCH_SEED, BATCH_PARTS = 2048, 4, 8


@pytest.fixture(scope="module")
def batched_workload_outputs():
    """The batched workload reduced in one persistent launch at the tuned
    parameters; the invariants of every pencil checked with device products;
    the outputs returned on the host."""
    count, seed = BATCH_COUNT, BATCH_SEED
    sizes = inputs.batch_sizes(count, seed)
    print("ht_reduce_batched workload: %d pencils, orders %d..%d" % (count, min(sizes), max(sizes)),
          flush=True)
    pencils = inputs.batch_pencils(count, seed)
    As = [htred.to_device_colmajor(A) for A, _ in pencils]
    Bs = [htred.to_device_colmajor(B) for _, B in pencils]
    Qs = [htred.colmajor_empty(A.shape[0]) for A in As]
    Zs = [htred.colmajor_empty(A.shape[0]) for A in As]
    plan = htred.BatchedPlan(As, Bs, Qs, Zs)
    plan.run()
    torch.cuda.synchronize()
    info = plan.info[:count].cpu().numpy()
    bad = []
    for i in range(count):
        A0, B0 = pencils[i]
        inv = checks.invariants(htred.to_device_colmajor(A0), htred.to_device_colmajor(B0),
                                As[i], Bs[i], Qs[i], Zs[i])
        if not checks.invariants_ok(inv, int(sizes[i])):
            bad.append((i, int(sizes[i]), inv))
    outs = [tuple(M.cpu().numpy() for M in (As[i], Bs[i], Qs[i], Zs[i])) for i in range(count)]
    del As, Bs, Qs, Zs, plan
    torch.cuda.empty_cache()
    return sizes, info, bad, outs


def test_batched_workload_info_and_invariants(batched_workload_outputs):
    sizes, info, bad, _ = batched_workload_outputs
    assert (info == 0).all(), np.nonzero(info)
    assert not bad, bad[:3]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("part", range(BATCH_PARTS))
def test_batched_workload_every_pencil(batched_workload_outputs, part):
    """Every pencil of the workload (in eight parts) against its own O-fast
    reduction, sign-normalised, at 1e-10."""
    sizes, _, _, outs = batched_workload_outputs
    count, seed = BATCH_COUNT, BATCH_SEED
    idx = list(range(part, count, BATCH_PARTS))

    def one(i):
        A0, B0 = inputs.batch_pencil(i, sizes[i], count, seed)
        ref = oracle.fast_ht(A0, B0, threads=1)[:4]
        d = checks.compare(ref, outs[i], A0, B0)
        return i, max(d["max_H"], d["max_T"], d["max_Q"], d["max_Z"])

    print("O-fast oracle on %d pencils, %d host threads" % (len(idx), host_workers()), flush=True)
    order = sorted(idx, key=lambda i: -int(sizes[i]))  # largest first: the pool drains evenly
    with ThreadPoolExecutor(max_workers=host_workers()) as ex:
        res = list(ex.map(one, order))
    worst = max(res, key=lambda t: t[1])
    print("worst pencil %d (n=%d): %.2e" % (worst[0], sizes[worst[0]], worst[1]), flush=True)
    over = [(i, int(sizes[i]), e) for i, e in res if not e <= TOL]
    assert not over, over[:5]


@pytest.fixture(scope="module")
def headline_pencil():
    """The n = 16384 ill-conditioned pencil resident on the device, with
    buffers for one reduction and the invariants of each form run on it."""
    A0, B0 = inputs.workload("n16384", order="C")
    n = A0.shape[0]
    A0d = htred.colmajor_empty(n)
    A0d.copy_(torch.from_numpy(A0).to("cuda"))
    B0d = htred.colmajor_empty(n)
    B0d.copy_(torch.from_numpy(B0).to("cuda"))
    del A0, B0
    bufs = [htred.colmajor_empty(n) for _ in range(4)]
    ws = torch.empty(htred.workspace_size(n, nb=128), dtype=torch.uint8, device="cuda")
    yield {"n": n, "A0": A0d, "B0": B0d, "bufs": bufs, "ws": ws, "inv": {}}
    del bufs, ws, A0d, B0d
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("form", ["fp64", "bf16", "fp8"])
def test_precision_form_n16384_headline_pencil(headline_pencil, form):
    """The split-precision form on the n = 16384 ill-conditioned pencil at
    nb = 128, BF16 and FP8 digit slices, beside the native FP64 run: the
    invariants, and a backward error and loss of orthogonality no more than
    100 times those of the FP64 run on the same pencil (all far inside the
    1e-14 n bars)."""
    hp = headline_pencil
    n = hp["n"]
    A, B, Q, Z = hp["bufs"]
    p = {"fp64": htred.HT_PREC_FP64, "bf16": htred.HT_PREC_SPLIT_BF16,
         "fp8": htred.HT_PREC_SPLIT_FP8}[form]
    print("ht_reduce n=16384 illcond nb=128 prec=%s" % form, flush=True)
    A.copy_(hp["A0"])
    B.copy_(hp["B0"])
    htred.reduce(A, B, Q, Z, nb=128, prec=p, workspace=hp["ws"])
    torch.cuda.synchronize()
    inv = htred.check(hp["A0"], hp["B0"], A, B, Q, Z)
    zH, zT = checks.structure_violations(A, B)
    e1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    e1[0] = 1.0
    inv.update(zeros_H=zH, zeros_T=zT,
               e1_Q=bool((Q[:, 0] == e1).all() and (Q[0, :] == e1).all()),
               e1_Z=bool((Z[:, 0] == e1).all() and (Z[0, :] == e1).all()))
    print("n=16384 %s: %s" % (form, inv), flush=True)
    assert checks.invariants_ok(inv, n), (form, inv)
    hp["inv"][form] = inv
    if form != "fp64":
        ref = hp["inv"].get("fp64")
        assert ref is not None, "the FP64 run of the same pencil comes first"
        for key in ("bwd_A", "bwd_B", "orth_Q", "orth_Z"):
            assert inv[key] <= 100.0 * ref[key], (form, key, inv, ref)
