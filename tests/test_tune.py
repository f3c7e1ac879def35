"""Host logic of the launch-shape tuner (no GPU)."""
import json

from paper_1012_0385_amd import tune


def test_candidates_cover_whole_and_windows():
    c = tune.candidates(1 << 17, 64)
    assert {"windows": 1, "window_sweeps": 0, "rings_per_wg": 0} in c
    assert all(x["windows"] == 1 or (1 << 17) // 64 // x["windows"] >= 4 * (x["window_sweeps"] + 1)
               for x in c)
    small = tune.candidates(1024, 8)
    assert any(x["rings_per_wg"] > 1 for x in small)
    assert all(x["windows"] == 1 for x in small)


def test_table_roundtrip(tmp_path):
    path = str(tmp_path / "t.json")
    kw = dict(L=4096, p=1.0, q=0.0)
    assert tune.lookup(kw, 8, path) == {}
    tune.store(kw, 8, {"windows": 2, "window_sweeps": 7, "rings_per_wg": 0, "rate": 1.0}, "gfx950",
               path)
    assert tune.lookup(kw, 8, path) == {"windows": 2, "window_sweeps": 7, "rings_per_wg": 0}
    assert tune.lookup(kw, 9, path) == {}
    with open(path) as f:
        t = json.load(f)
    assert t["version"] == tune.TABLE_VERSION and t["device"] == "gfx950"


def test_shipped_table_has_the_benchmark_workload():
    kw = dict(L=1 << 17, p=1.0, q=0.0, seed=1, stream=0)
    shape = tune.lookup(kw, 64)
    assert shape and shape["windows"] >= 1
