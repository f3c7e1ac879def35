"""Host logic of the autotuner and its table (no GPU): classes, the text
format the library loads, and the shipped table."""
import paper_1012_0385_amd as A
from paper_1012_0385_amd import tune


def test_candidates_cover_whole_and_windows():
    c = tune.candidates(1 << 17, 64)
    assert {"windows": 1, "window_sweeps": 0, "rings_per_wg": 0} in c
    assert all(x["windows"] == 1 or (1 << 17) // 64 // x["windows"] >= 2 * (x["window_sweeps"] + 1)
               for x in c)
    assert dict(windows=4, window_sweeps=255, rings_per_wg=0) in c
    small = tune.candidates(1024, 8)
    assert any(x["rings_per_wg"] > 1 for x in small)
    assert all(x["windows"] == 1 for x in small)


def test_schedules_tried_only_where_left_open():
    assert tune.schedules_for(dict(L=1 << 17, p=1.0)) == [
        dict(cell_log2=6, subsweeps=4), dict(cell_log2=5, subsweeps=2)]
    assert tune.schedules_for(dict(L=1 << 17, p=1.0, subsweeps=4)) == [{}]
    assert tune.schedules_for(dict(L=1 << 16, model=1)) == [{}]
    assert len(tune.schedules_for(dict(L=1 << 16, slow_frac=0.1))) == 2
    assert tune.schedules_for(dict(L=1 << 16, schedule=1)) == [{}]


def test_table_roundtrip_and_library_agrees(tmp_path):
    path = str(tmp_path / "t.txt")
    kw = dict(L=4096, p=1.0, q=0.0)
    assert tune.lookup(kw, 8, path) == {}
    tune.store(kw, 8, dict(cell_log2=5, subsweeps=2, windows=2, window_sweeps=7, rings_per_wg=0,
                           rate=1.0), "gfx950", path)
    want = dict(cell_log2=5, subsweeps=2, windows=2, window_sweeps=7, rings_per_wg=0)
    assert tune.lookup(kw, 8, path) == want
    assert tune.lookup(kw, 16, path) == want      # the class spans 4 .. 16 samples
    assert tune.lookup(kw, 17, path) == {}
    assert tune.lookup(dict(kw, L=8192), 8, path) == {}
    # storing the same class again replaces the entry
    tune.store(kw, 8, dict(windows=1, rate=2.0), "gfx950", path)
    assert len(tune.load_entries(path)) == 1
    # the library reads the same file and fills the same values
    tune.store(kw, 8, dict(want, rate=1.0), "gfx950", path)
    try:
        A.load_tuning(path)
        got, plan = A.resolve(A.make_params(L=4096, samples=8, p=1.0))
        assert (got.cell_log2, got.subsweeps, got.windows, got.window_sweeps) == (5, 2, 2, 7)
        assert plan["windows"] == 2
    finally:
        A.load_tuning(None)


def test_stored_entry_goes_ahead_of_a_broader_one(tmp_path):
    # the first matching entry wins, so a class tuned later must not end up
    # behind a broad entry that also covers it
    path = str(tmp_path / "t.txt")
    with open(path, "w") as f:
        f.write("0 0 0 10 26 1 65536 5 2 0 0 0   # broad\n")
    kw = dict(L=4096, p=1.0, q=0.0)
    assert tune.lookup(kw, 8, path)["windows"] == 0
    tune.store(kw, 8, dict(windows=2, window_sweeps=7, rate=1.0), "gfx950", path)
    entries = tune.load_entries(path)
    assert [e["log2L_hi"] for e in entries] == [12, 26]
    assert tune.lookup(kw, 8, path)["windows"] == 2
    assert tune.lookup(dict(kw, L=1 << 20), 8, path)["cell_log2"] == 5


def test_shipped_table_loads_and_covers_the_benchmark_workload():
    entries = tune.load_entries()
    assert entries
    kw = dict(L=1 << 17, p=1.0, q=0.0, seed=1, stream=0)
    shape = tune.lookup(kw, 64)
    assert shape and shape["windows"] >= 1
    try:
        A.load_tuning(tune.DEFAULT_TABLE)
        got, _ = A.resolve(A.make_params(L=1 << 17, samples=64, p=1.0))
        assert got.windows == shape["windows"] and got.window_sweeps == shape["window_sweeps"]
        if shape["cell_log2"]:
            assert (got.cell_log2, got.subsweeps) == (shape["cell_log2"], shape["subsweeps"])
    finally:
        A.load_tuning(None)
