"""CPU checks of bench.py's contract: the one-GPU guard, the nominal flop
model, the wall-clock budget planner (with stubbed step times), the hash-
and parameter-keyed lookup of measured HBM traffic, and the shape of the
CPU-oracle baseline object."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1710_08538_amd import inputs  # noqa: E402


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_exits_with_a_message(args, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_nominal_flop_model():
    assert bench.nominal_flops(16384) == 39.0 * 16384 ** 3
    assert bench.nominal_flops(0) == 0.0


def _table(tmp_path, src_bytes, sha=None, params=None):
    src = tmp_path / "kernel.hip"
    src.write_bytes(src_bytes)
    ent = {"bytes_per_launch": 12345, "source": str(src),
           "source_sha256": sha or hashlib.sha256(src_bytes).hexdigest()}
    if params is not None:
        ent["params"] = params
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({"classes": {"k": ent}}))
    return str(path)


def test_measured_traffic_needs_the_measured_source_and_parameters(tmp_path, monkeypatch):
    # sources are resolved relative to the repository root; an absolute path
    # stays as it is under os.path.join
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _table(tmp_path, b"kernel v1"))
    assert bench.measured_traffic("k") == 12345
    assert bench.measured_traffic("missing") is None
    # the kernel source changed since the counters were taken
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _table(tmp_path, b"kernel v2", sha="0" * 64))
    assert bench.measured_traffic("k") is None
    # counters taken with other launch parameters
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        _table(tmp_path, b"kernel v3", params={"nb": 64, "block": 32}))
    assert bench.measured_traffic("k", {"nb": 64, "block": 32}) == 12345
    assert bench.measured_traffic("k", {"nb": 32, "block": 32}) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.measured_traffic("k") is None


def test_committed_traffic_matches_committed_sources():
    """Every class in the committed table was measured on the kernel source
    as it is now (a stale entry would make bench.py report null traffic)."""
    with open(bench.TRAFFIC_FILE) as f:
        table = json.load(f)
    for cls, ent in table["classes"].items():
        with open(os.path.join(ROOT, ent["source"]), "rb") as f:
            assert hashlib.sha256(f.read()).hexdigest() == ent["source_sha256"], cls
        assert bench.measured_traffic(cls, ent.get("params")) == ent["bytes_per_launch"]


def test_cpu_baseline_object():
    A0, B0 = inputs.random_pencil(48, seed=3)
    cb = bench.cpu_baseline(A0, B0, 0.5)
    assert set(cb) >= {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["cores"] == (os.cpu_count() or 1)
    assert cb["unit"] == "GFLOP/s"
    assert np.isfinite(cb["value"]) and cb["value"] > 0.0
    assert "O-fast" in cb["sample"] and "EXTRAPOLATED" in cb["sample"]
    assert 1 <= cb["columns_sampled"] <= 46


def test_cpu_baseline_sample_is_bounded():
    """A time limit far below the whole reduction stops the oracle early."""
    A0, B0 = inputs.random_pencil(600, seed=4)
    cb = bench.cpu_baseline(A0, B0, 1e-6)
    assert cb["columns_sampled"] == 1
    assert cb["time_s_extrapolated"] > cb["sample_s"]


# ------------------------------------------------------------- budget ---

TAIL = [("profiled_step", 40.0), ("check", 8.0), ("cpu_baseline", 45.0), ("batched", 40.0),
        ("precision_bf16", 60.0), ("precision_fp8", 75.0)]


def test_plan_fits_everything_when_there_is_room():
    w, k, kept = bench.plan_steps(2000.0, 10.0, 20, 5, TAIL)
    assert k == 20 and w == 4 and kept == [t for t, _ in TAIL]
    assert w * 10 + k * 10 + sum(t for _, t in TAIL) <= 2000.0


def test_plan_caps_steps_at_the_driver_command():
    """The driver's --steps 20 --warmup 5 with a 37 s step: timed steps are
    cut so that the tail still fits the budget; no extra warm-ups."""
    left = 450.0 - 25.0 - 37.0 - 10.0
    tail = [(n, t * (37.0 / 10.0) if n.startswith("precision") or n == "profiled_step" else t)
            for n, t in TAIL]
    w, k, kept = bench.plan_steps(left, 37.0, 20, 5, tail)
    assert w == 0 and 1 <= k < 20
    used = k * 37.0 + sum(t for n, t in tail if n in kept)
    assert used <= left
    assert kept[0] == "profiled_step"


def test_plan_drops_forms_before_timing_fewer_than_two_steps():
    w, k, kept = bench.plan_steps(200.0, 30.0, 20, 5, TAIL)
    assert k >= 2
    assert "precision_fp8" not in kept
    assert kept == [t for t, _ in TAIL][:len(kept)]  # dropped from the end
    assert k * 30.0 + sum(t for n, t in TAIL if n in kept) <= 200.0


def test_plan_always_times_one_step():
    w, k, kept = bench.plan_steps(5.0, 30.0, 20, 5, TAIL)
    assert k == 1 and w == 0 and kept == []
    w, k, kept = bench.plan_steps(1000.0, 1.0, 1, 1, TAIL)
    assert k == 1 and w == 0


def test_budget_counts_from_the_start():
    now = [100.0]
    b = bench.Budget(450.0, clock=lambda: now[0], t0=100.0)
    assert b.left() == 450.0
    now[0] = 400.0
    assert b.left() == 150.0
