"""The tile autotuner's host logic (paper_2311_03694_amd/tune.py) on the CPU: table keys,
the kernels a batch tunes, the JSON table round trip, the choice of the fastest variant
and apply() from a table.  The library calls are replaced by recording stubs."""
import json

from paper_2311_03694_amd import tune


class FakeRom:
    def __init__(self, N=40, dtype="fp32"):
        self.N, self.dtype, self.handle = N, dtype, 1234


def test_kinds_and_keys():
    assert tune.kinds_for(True, 1) == [0]
    assert tune.kinds_for(False, 1) == []           # one CP trajectory: resident runs, no tiles
    assert tune.kinds_for(True, 16) == [1]
    assert tune.kinds_for(False, 16) == [2, 3]
    assert tune.key(1, 400, 0, 256, "bf16") == "dense_batched:N400:R0:B256:bf16"
    assert tune.key(3, 1000, 2000, 64, "fp32") == "cp_scatter:N1000:R2000:B64:fp32"


def test_table_round_trip(tmp_path):
    path = str(tmp_path / "tiles.json")
    assert tune.load(path) == {}
    table = {"cp_proj:N40:R16:B16:fp32": 2, "dense1:N40:R0:B1:fp64": 0}
    tune.save(table, path)
    assert tune.load(path) == table
    with open(path) as f:
        assert json.load(f) == table                # plain JSON, sorted keys


def test_tune_picks_the_fastest_variant(monkeypatch):
    calls = []
    monkeypatch.setattr(tune.rb, "rom_set_tile", lambda h, kind, v: calls.append((h, kind, v)))
    monkeypatch.setattr(tune.rb, "rom_tile_count", lambda kind: 4)
    # the variant that was set last is the one a step is timed with
    times = {2: [3.0, 1.0, 2.0, 4.0], 3: [2.0, 2.5, 0.5, 1.0]}
    monkeypatch.setattr(tune, "_time_steps", lambda rom, u0, steps, reps: times[calls[-1][1]][calls[-1][2]])
    import numpy as np
    table = {}
    out = tune.tune(FakeRom(), np.zeros((16, 40)), dense=False, R=16, table=table)
    assert out["cp_proj:N40:R16:B16:fp32"]["best"] == 1
    assert out["cp_scatter:N40:R16:B16:fp32"]["best"] == 2
    assert table == {"cp_proj:N40:R16:B16:fp32": 1, "cp_scatter:N40:R16:B16:fp32": 2}
    # each kind ends on its best variant
    assert [c for c in calls if c[1] == 2][-1] == (1234, 2, 1)
    assert [c for c in calls if c[1] == 3][-1] == (1234, 3, 2)


def test_apply_sets_only_cached_kinds(monkeypatch):
    calls = []
    monkeypatch.setattr(tune.rb, "rom_set_tile", lambda h, kind, v: calls.append((kind, v)))
    table = {"cp_proj:N40:R16:B16:fp32": 3, "dense_batched:N40:R0:B16:fp32": 5}
    assert tune.apply(FakeRom(), 16, dense=False, R=16, table=table) == 1
    assert calls == [(2, 3)]
    calls.clear()
    assert tune.apply(FakeRom(), 16, dense=True, table=table) == 1
    assert calls == [(1, 5)]
    calls.clear()
    assert tune.apply(FakeRom(dtype="bf16"), 16, dense=True, table=table) == 0
    assert calls == []
