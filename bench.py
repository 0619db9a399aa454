#!/usr/bin/env python3
"""Benchmark: HouseHT reduction of one n x n pencil on one MI355X.

One step = one full HT reduction (Algorithm 1: panels + absorption) of the
synthetic pencil, restored from a pristine device copy at the start of the
step (a device-to-device copy of A and B, < 0.1% of the step).  The default
workload is the n = 16384 FP64 pencil with an ill-conditioned triangular B
(panel width nb = 128).  Prints ONE JSON line.

value = nominal GFLOP/s = 39 n^3 / time (the nominal count of the basic
two-block absorption scheme); the executed flop count, time per step,
backward errors and the IR statistics are reported beside it.

roofline: the kernel class with the largest device time in one extra step
run after the timed ones with every launch bracketed by HIP events on the
library's stream (the timed steps run without events); achieved =
algorithmic work of that class / its summed launch durations.

cpu_baseline: the O(n^3) CPU oracle (O-fast, plain C with OpenMP on every
host core) on the first columns of the same pencil for a bounded time,
extrapolated to the whole reduction by the oracle's modelled work per
column (labelled as extrapolated).

Budget: the whole run fits --budget-s seconds of wall time (default 450).
--steps and --warmup are upper bounds; after the first warm-up step the
number of timed steps is chosen so that the profiled step, the invariant
check, the CPU baseline and the forms still fit, dropping the forms (FP8,
then BF16, then batched) before timing fewer than two steps.  The JSON line
reports the steps actually timed.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HT reduction GFLOP/s + time at n=16384 FP64 (vs split-prec/batched), backward err"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0


def nominal_flops(n):
    return 39.0 * float(n) ** 3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A0, B0, target_s):
    """The O(n^3) CPU oracle (O-fast: Algorithm 2's reflector pair per column
    with B kept triangular by Givens QR updates; plain C, OpenMP on every host
    core) on the first columns of the same pencil, for about `target_s`
    seconds of its column loop, extrapolated to the whole reduction by the
    oracle's modelled flops per column.  The early columns are the largest,
    so the extrapolation is by work, not by column count."""
    import oracle
    n = A0.shape[0]
    threads = os.cpu_count() or 1
    tm = {"limit_s": float(target_s)}
    oracle.fast_ht(A0, B0, threads=threads, timing=tm)
    c = max(tm["columns"], 1)
    w_sample = oracle.fast_flops(n, c)
    w_full = oracle.fast_flops(n)
    t_full = tm["loop_s"] * w_full / w_sample
    return {"value": nominal_flops(n) / t_full / 1e9, "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": ("O-fast oracle (Algorithm 2's reflector pair per column, B kept "
                       "triangular by Givens QR updates; plain C, OpenMP, %d threads on %s) on "
                       "the first %d of %d columns of the same n=%d pencil: %.1f s; whole "
                       "reduction EXTRAPOLATED by the oracle's modelled flops per column to "
                       "%.0f s; value = 39 n^3 nominal flops / that time"
                       % (threads, cpu_model(), c, n - 2, n, tm["loop_s"], t_full)),
            "columns_sampled": c, "sample_s": tm["loop_s"], "time_s_extrapolated": t_full,
            "oracle_gflops_modelled": w_full / t_full / 1e9, "cpu_model": cpu_model()}


def batched_form(torch, htred, inputs, checks, count=2048, seed=4):
    """The batched workload: `count` pencils with orders U{32..512} (child seeds
    of SeedSequence(seed)), reduced in one persistent launch; timed eagerly and
    as a hipGraph replay, inputs restored from device copies before each run."""
    import numpy as np

    sizes = inputs.batch_sizes(count, seed)
    pencils = inputs.batch_pencils(count, seed)
    A0s = [htred.to_device_colmajor(A) for A, _ in pencils]
    B0s = [htred.to_device_colmajor(B) for _, B in pencils]
    As = [htred.to_device_colmajor(A) for A, _ in pencils]
    Bs = [htred.to_device_colmajor(B) for _, B in pencils]
    Qs = [htred.colmajor_empty(A.shape[0]) for A in As]
    Zs = [htred.colmajor_empty(A.shape[0]) for A in As]
    plan = htred.BatchedPlan(As, Bs, Qs, Zs)

    def restore():
        for i in range(count):
            As[i].copy_(A0s[i])
            Bs[i].copy_(B0s[i])

    restore()
    plan.run()
    torch.cuda.synchronize()
    restore()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t = time.time()
    ev0.record()
    plan.run()  # on the current stream, which the events bracket
    ev1.record()
    torch.cuda.synchronize()
    eager_s = time.time() - t
    launch_ms = ev0.elapsed_time(ev1)
    ps = plan.pencil_stats().numpy()
    lat_ms = (ps[:, 1] - ps[:, 0]) / 1e6
    big = np.asarray(sizes) >= 480
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    restore()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            plan.run(stream=st)
    torch.cuda.current_stream().wait_stream(st)
    restore()
    torch.cuda.synchronize()
    t = time.time()
    g.replay()
    torch.cuda.synchronize()
    graph_s = time.time() - t
    info = plan.info[:count].cpu().numpy()
    worst = {"bwd_A": 0.0, "bwd_B": 0.0, "orth_Q": 0.0, "orth_Z": 0.0}
    ok = bool((info == 0).all())
    for i in range(0, count, 32):
        inv = checks.invariants(A0s[i], B0s[i], As[i], Bs[i], Qs[i], Zs[i])
        ok = ok and bool(checks.invariants_ok(inv, int(sizes[i])))
        for k in worst:
            worst[k] = max(worst[k], float(inv[k]))
    fl = float(sum(39.0 * float(n) ** 3 for n in sizes))
    # roofline of the launch: the bytes every reduced column must move (A's
    # trailing block for Y = A v, 8 m^2, and B's triangle for the solve and
    # the residual, 8 m^2; m = n - j - 1) against the HBM peak
    alg = float(sum(16.0 * (n - 1) * n * (2 * n - 1) / 6.0 for n in sizes))
    ach = alg / (launch_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS,
            "traffic": measured_traffic("batched", {"nb": plan.nb, "block": plan.block,
                                                    "wg_per_cu": plan.wg_per_cu}),
            "kernel": "htk::k_batched", "launch_ms": launch_ms, "algorithmic_bytes": alg}
    return {"pencils": count, "orders": "U{32..512}", "seed": seed, "panel_width": plan.nb,
            "retriangularise_block": plan.block, "workgroups_per_cu": plan.wg_per_cu,
            "ms": 1000.0 * eager_s, "pencils_per_s": count / eager_s,
            "gflops_nominal": fl / eager_s / 1e9, "graph_replay_ms": 1000.0 * graph_s,
            "latency_ms_p50": float(np.percentile(lat_ms, 50)),
            "latency_ms_p99": float(np.percentile(lat_ms, 99)),
            "latency_ms_mean_n_ge_480": float(lat_ms[big].mean()) if big.any() else None,
            "device_span_ms": float(ps[:, 1].max() / 1e6),
            "panels_total": int(ps[:, 2].sum()), "ir_steps_total": int(ps[:, 3].sum()),
            "phase_share_n_ge_480": ({k: float(ps[big, c].sum() / (ps[big, 1] - ps[big, 0]).sum())
                                      for k, c in (("solve", 4), ("residual", 5), ("absorb", 6),
                                                   ("retriangularise", 7))}
                                     if big.any() else None),
            "checked_sample": len(range(0, count, 32)), "invariants_ok": ok,
            "backward_error_max": worst, "roofline": roof}


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "hbm_traffic.json")


def measured_traffic(cls, params=None):
    """HBM bytes per launch of the kernel class `cls` from the committed PMC
    counts (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a copy of
    known size), or None if there are none, the kernel's source changed
    since they were taken, or they were taken with other parameters."""
    try:
        with open(TRAFFIC_FILE) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    ent = table.get("classes", {}).get(cls)
    if not ent:
        return None
    if params is not None and ent.get("params") != params:
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), ent["source"])
    try:
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != ent["source_sha256"]:
                return None
    except OSError:
        return None
    return ent["bytes_per_launch"]


def precision_form(torch, htred, checks, A0d, B0d, A, B, Q, Z, ws, nb, name, t_fp64):
    """The precision form on the headline pencil: the WY products as
    emulated-FP64 split products (default slice count of the format), every
    other step native FP64; one run, timed, with its backward errors."""
    prec = {"bf16": htred.HT_PREC_SPLIT_BF16, "fp8": htred.HT_PREC_SPLIT_FP8}[name]
    n = A0d.shape[0]
    A.copy_(A0d)
    B.copy_(B0d)
    torch.cuda.synchronize()
    t = time.time()
    st = htred.reduce(A, B, Q, Z, nb=nb, prec=prec, stats=True, workspace=ws)[2]
    torch.cuda.synchronize()
    dt = time.time() - t
    inv = checks.invariants(A0d, B0d, A, B, Q, Z)
    return {"n": n, "nb": nb, "digits": name, "n_slices": {"bf16": 8, "fp8": 14}[name],
            "time_s": dt, "gflops_nominal": nominal_flops(n) / dt / 1e9,
            "time_vs_fp64": dt / t_fp64,
            "backward_error": {k: float(inv[k]) for k in ("bwd_A", "bwd_B", "orth_Q", "orth_Z")},
            "invariants_ok": bool(checks.invariants_ok(inv, n)),
            "absorptions": st["absorptions"]}


T_START = time.time()


class Budget:
    """Wall-clock budget of the whole run, from process start.  The timed
    steps are capped so that the run (inputs, warm-up, timed steps, the
    profiled step, the CPU baseline and the forms measured beside the
    headline) ends inside it; --steps and --warmup are upper bounds."""

    def __init__(self, total_s, clock=time.time, t0=None):
        self.total = float(total_s)
        self.clock = clock
        self.t0 = T_START if t0 is None else t0

    def left(self):
        return self.total - (self.clock() - self.t0)


def plan_steps(left_s, t_step, steps_cap, warm_cap, tail):
    """How many extra warm-up steps and timed steps fit in `left_s` seconds
    after the first warm-up step (which took `t_step`), keeping the time
    estimated for the optional parts `tail` (list of (name, seconds), most
    wanted first).  Optional parts are dropped from the end of the list
    until at least min(2, steps_cap) timed steps fit; at least one step is
    always timed.  Returns (extra_warmup, steps, kept_tail_names)."""
    tail = list(tail)
    want = min(2, steps_cap)
    while True:
        avail = left_s - sum(t for _, t in tail)
        k = int(avail // max(t_step, 1e-9))
        if k >= want or not tail:
            break
        tail.pop()
    k = max(1, min(steps_cap, k))
    spare = left_s - sum(t for _, t in tail) - k * t_step
    extra_w = max(0, min(warm_cap - 1, int(spare // max(t_step, 1e-9))))
    # extra warm-ups only when every requested timed step already fits
    if k < steps_cap:
        extra_w = 0
    return extra_w, k, [name for name, _ in tail]


def upload_colmajor(torch, htred, M):
    """Host matrix (any numpy layout) -> column-major device tensor; a
    row-major source is uploaded as is and transposed on the device."""
    t = torch.from_numpy(M).to("cuda") if M.flags.c_contiguous else torch.as_tensor(M)
    out = htred.colmajor_empty(M.shape[0], M.shape[1])
    out.copy_(t)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed steps (upper bound)")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up steps (upper bound, >= 1)")
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget of the whole run, from process start")
    ap.add_argument("--workload", default="n16384")
    ap.add_argument("--n", type=int, default=None, help="override the order (same generator)")
    ap.add_argument("--nb", type=int, default=128)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "bf16", "fp8"])
    ap.add_argument("--ell", type=int, default=2,
                    help="blocks per absorption window: 2 basic scheme, >= 3 the "
                         "accelerated absorption with block triangular B")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision and batched forms measured beside the headline run")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (the single-pencil reduction is not sharded "
              "across GPUs); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    from paper_1710_08538_amd import htred, inputs
    from oracle import checks

    budget = Budget(args.budget_s)

    def log(msg):
        print("bench [%5.1f s left]: %s" % (budget.left(), msg), file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = {"fp64": htred.HT_PREC_FP64, "bf16": htred.HT_PREC_SPLIT_BF16,
            "fp8": htred.HT_PREC_SPLIT_FP8}[args.prec]
    A0, B0 = inputs.workload(args.workload, n=args.n, order="C")
    n = A0.shape[0]
    log("workload %s n=%d nb=%d prec=%s generated" % (args.workload, n, args.nb, args.prec))
    A0d = upload_colmajor(torch, htred, A0)
    B0d = upload_colmajor(torch, htred, B0)
    A = htred.colmajor_empty(n)
    B = htred.colmajor_empty(n)
    Q = htred.colmajor_empty(n)
    Z = htred.colmajor_empty(n)
    ws = torch.empty(htred.workspace_size(n, nb=args.nb, ell=args.ell), dtype=torch.uint8,
                     device="cuda")
    torch.cuda.synchronize()
    log("inputs resident on the device")

    def step(profile):
        A.copy_(A0d)
        B.copy_(B0d)
        return htred.reduce(A, B, Q, Z, nb=args.nb, prec=prec, stats=True, workspace=ws,
                            profile=profile, ell=args.ell)[2]

    t = time.time()
    step(False)
    torch.cuda.synchronize()
    t_step = time.time() - t
    log("warm-up 0 done in %.2f s" % t_step)

    # what must still fit after the timed steps, most wanted first
    fp64 = prec == htred.HT_PREC_FP64
    tail = [("profiled_step", 1.1 * t_step + 3.0)]
    if not args.no_check:
        tail.append(("check", 8.0))
    if not args.no_cpu_baseline:
        tail.append(("cpu_baseline", args.cpu_seconds + 25.0))
    if not args.no_forms:
        tail.append(("batched", 40.0))
        if fp64:
            tail.append(("precision_bf16", 1.45 * t_step + 10.0))
            tail.append(("precision_fp8", 1.85 * t_step + 10.0))
    extra_w, K, kept = plan_steps(budget.left() - 10.0, t_step, max(args.steps, 1),
                                  max(args.warmup, 1), tail)
    log("plan: %d more warm-up step(s), %d timed step(s), then %s" % (extra_w, K, kept))
    for i in range(extra_w):
        step(False)
        torch.cuda.synchronize()
        log("warm-up %d done" % (i + 1))

    torch.cuda.synchronize()
    t0 = time.time()
    stats = []
    for i in range(K):
        stats.append(step(False))
        log("step %d done" % i)
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    ms_per_step = 1000.0 * elapsed / K

    # one more step, outside the timed region, with every launch bracketed by
    # HIP events on the library's stream: per-class device time and work
    t = time.time()
    pstats = [step(True)]
    torch.cuda.synchronize()
    log("profiled step done in %.2f s" % (time.time() - t))

    # roofline of the dominant kernel class over the profiled step
    ncls = len(htred.PROF_CLASSES)
    prof_ms = [sum(s["prof_ms"][c] for s in pstats) for c in range(ncls)]
    prof_work = [sum(s["prof_work"][c] for s in pstats) for c in range(ncls)]
    prof_l = [sum(s["prof_launches"][c] for s in pstats) for c in range(ncls)]
    dom = max(range(ncls), key=lambda c: prof_ms[c])

    def roofline_of(c):
        name = htred.PROF_CLASSES[c]
        if prof_ms[c] <= 0.0:
            return None
        if name in ("trsv", "trmv", "ygemv"):  # work = algorithmic bytes
            a = prof_work[c] / (prof_ms[c] * 1e-3) / 1e9
            r = {"bound": "hbm", "achieved": a, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
        elif name in ("sweep", "wy") and prec == htred.HT_PREC_FP64:  # FP64 MFMA
            a = prof_work[c] / (prof_ms[c] * 1e-3) / 1e12
            r = {"bound": "mfma", "achieved": a, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
        elif name == "wy":
            # split products: every FP64 flop costs ns(ns+1)/2 digit-pair
            # products on the BF16 / FP8 matrix cores
            ns = 8 if prec == htred.HT_PREC_SPLIT_BF16 else 14
            a = prof_work[c] * ns * (ns + 1) / 2 / (prof_ms[c] * 1e-3) / 1e12
            pk = PEAK_BF16_TFLOPS if prec == htred.HT_PREC_SPLIT_BF16 else PEAK_FP8_TFLOPS
            r = {"bound": "mfma", "achieved": a, "peak": pk, "unit": "TFLOP/s"}
        else:                                  # chains: FP64 vector ALU
            a = prof_work[c] / (prof_ms[c] * 1e-3) / 1e12
            r = {"bound": "alu", "achieved": a, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
        r["frac"] = r["achieved"] / r["peak"]
        r["traffic"] = measured_traffic(name)
        r["kernel_class"] = name
        r["launches_per_step"] = prof_l[c]
        r["avg_launch_us"] = 1000.0 * prof_ms[c] / max(prof_l[c], 1)
        return r

    roof = roofline_of(dom)
    by_class = {htred.PROF_CLASSES[c]: roofline_of(c) for c in range(ncls)}
    breakdown = {htred.PROF_CLASSES[c]: {"ms": prof_ms[c], "launches": prof_l[c],
                                         "work": prof_work[c]}
                 for c in range(ncls)}

    result = {
        "metric": METRIC,
        "value": nominal_flops(n) / (ms_per_step * 1e-3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": 1 + extra_w,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else ("f64-split-" + args.prec),
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "nb": args.nb, "ell": args.ell,
                   "generator": inputs.WORKLOADS[args.workload][0],
                   "flop_model": "39 n^3 nominal"},
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "budget_s": args.budget_s,
        "time_s": ms_per_step / 1000.0,
        "gflops_executed": stats[-1]["flops"] / (ms_per_step * 1e-3) / 1e9,
        "ir": {k: stats[-1][k] for k in ("cols_extra_ir", "ir_steps", "ir_failures",
                                         "absorptions", "scaled_solves")},
        "profiled_step": breakdown,
        "roofline": roof,
        "roofline_by_class": by_class,
        "skipped": [],
    }

    def fits(name, est):
        if name not in kept:
            result["skipped"].append(name)
            return False
        if budget.left() < est + 5.0:
            result["skipped"].append(name)
            log("skipping %s: %.0f s estimated, %.0f s left" % (name, est, budget.left()))
            return False
        return True

    est = dict(tail)
    if not args.no_check and fits("check", est["check"]):
        inv = checks.invariants(A0d, B0d, A, B, Q, Z)
        result["backward_error"] = {k: inv[k] for k in ("bwd_A", "bwd_B", "orth_Q", "orth_Z",
                                                       "zeros_H", "zeros_T")}
        result["invariants_ok"] = bool(checks.invariants_ok(inv, n))
        log("invariants checked")
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0 and \
            fits("cpu_baseline", est["cpu_baseline"]):
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(A0, B0, args.cpu_seconds)
        log("cpu baseline done")
    if not args.no_forms:
        result["forms"] = {}
        if fp64:
            for name in ("bf16", "fp8"):
                if not fits("precision_" + name, est["precision_" + name]):
                    continue
                log("precision form %s ..." % name)
                result["forms"]["precision_" + name] = precision_form(
                    torch, htred, checks, A0d, B0d, A, B, Q, Z, ws, args.nb, name,
                    ms_per_step / 1000.0)
    del A0d, B0d, A, B, Q, Z, ws
    torch.cuda.empty_cache()
    if not args.no_forms and fits("batched", est["batched"]):
        log("batched form ...")
        result["forms"]["batched"] = batched_form(torch, htred, inputs, checks)
        torch.cuda.empty_cache()
    result["wall_s"] = time.time() - T_START
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
