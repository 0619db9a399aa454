"""Host logic of the panel-width autotuner (no GPU): table lookup by the
nearest order on a log scale, and the library default without a table."""
import json

from paper_1710_08538_amd import autotune


def test_pick_nb_nearest_order(tmp_path):
    path = tmp_path / "nb.json"
    path.write_text(json.dumps({"orders": {"512": {"nb": 32}, "4096": {"nb": 128},
                                           "1024": {"nb": 64}}}))
    table = autotune.load_table(str(path))
    assert table == {512: 32, 1024: 64, 4096: 128}
    assert autotune.pick_nb(100, table) == 32
    assert autotune.pick_nb(700, table) == 32     # log2 700 is nearer 512 than 1024
    assert autotune.pick_nb(800, table) == 64
    assert autotune.pick_nb(3000, table) == 128
    assert autotune.pick_nb(16384, table) == 128


def test_no_table_means_library_default(tmp_path):
    assert autotune.load_table(str(tmp_path / "missing.json")) == {}
    assert autotune.pick_nb(1000, {}) == 0


def test_batched_parameters_from_table(tmp_path):
    path = tmp_path / "nb.json"
    assert autotune.pick_batched(str(path)) == autotune.BATCHED_DEFAULT
    path.write_text(json.dumps({"orders": {}, "batched": {"nb": 32, "block": 16, "wg_per_cu": 2}}))
    assert autotune.pick_batched(str(path)) == {"nb": 32, "block": 16, "wg_per_cu": 2}
    path.write_text(json.dumps({"batched": {"nb": 0, "block": 64, "wg_per_cu": 3}}))
    assert autotune.pick_batched(str(path))["nb"] == 0
    # an entry without the shape parameters falls back to the defaults
    path.write_text(json.dumps({"batched": {"nb": 0}}))
    assert autotune.pick_batched(str(path)) == autotune.BATCHED_DEFAULT


def test_batched_candidates_cover_widths_and_shapes():
    c = autotune.BATCHED_CANDIDATES
    assert {nb for nb, _, _ in c} == {0, 32, 64, 128}
    assert {blk for _, blk, _ in c} == {16, 32, 64}
    assert {w for _, _, w in c} == {2, 3}
    assert len(set(c)) == len(c)


def test_committed_table_holds_the_batched_search():
    """The shipped table's batched entry is the fastest of its own recorded
    timings, over every candidate the tuner searches."""
    with open(autotune.TABLE) as f:
        data = json.load(f)
    ent = data["batched"]
    secs = ent["seconds"]
    assert set(secs) == {autotune.batched_key(*c) for c in autotune.BATCHED_CANDIDATES}
    best = min(secs, key=secs.get)
    assert best == autotune.batched_key(ent["nb"], ent["block"], ent["wg_per_cu"])
    assert autotune.pick_batched() == {k: ent[k] for k in ("nb", "block", "wg_per_cu")}
    # the single-pencil table: one width per order, from its own timings
    for n, e in data["orders"].items():
        assert int(e["nb"]) == int(min(e["seconds"], key=e["seconds"].get)), n
