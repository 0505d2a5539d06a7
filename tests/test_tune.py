"""Host logic of the batched autotuner: candidate selection and the table
the binding applies (the timing itself runs on the GPU)."""
import json
import math

import pytest

from paper_2312_09376_amd import tune


def test_select_fastest_accepted():
    res = [dict(tile_cols2_min_n=tune.NEVER, wgs_per_cu=1, ms=10.0, ok=True),
           dict(tile_cols2_min_n=tune.NEVER, wgs_per_cu=2, ms=7.0, ok=True),
           dict(tile_cols2_min_n=0, wgs_per_cu=2, ms=5.0, ok=False),   # outputs differed
           dict(tile_cols2_min_n=0, wgs_per_cu=1, ms=math.nan, ok=True)]
    best = tune.select(res)
    assert (best["tile_cols2_min_n"], best["wgs_per_cu"]) == (tune.NEVER, 2)


def test_select_tie_prefers_fewer_tiles_then_more_workgroups():
    res = [dict(tile_cols2_min_n=0, wgs_per_cu=2, ms=5.0, ok=True),
           dict(tile_cols2_min_n=tune.NEVER, wgs_per_cu=1, ms=5.0, ok=True),
           dict(tile_cols2_min_n=tune.NEVER, wgs_per_cu=2, ms=5.0, ok=True)]
    best = tune.select(res)
    assert (best["tile_cols2_min_n"], best["wgs_per_cu"]) == (tune.NEVER, 2)


def test_select_none_accepted():
    with pytest.raises(ValueError):
        tune.select([dict(tile_cols2_min_n=tune.NEVER, wgs_per_cu=1, ms=1.0, ok=False)])


def test_candidates_cover_the_buckets():
    assert {(c["tile_cols2_min_n"], c["wgs_per_cu"]) for c in tune.CANDIDATES} == {
        (t, w) for t in tune.BUCKETS for w in (1, 2)}
    assert tune.BUCKETS[0] == 0 and tune.BUCKETS[-1] == tune.NEVER  # all-two and all-one included
    assert list(tune.BUCKETS) == sorted(tune.BUCKETS)


def test_committed_table_is_valid():
    table = tune.load_table()
    assert set(table) <= set(tune.PRECS)
    for e in table.values():
        assert 0 <= e["tile_cols2_min_n"] <= tune.NEVER and e["wgs_per_cu"] in (1, 2)


def test_load_table_rejects_invalid_entries(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"batched": {"fp32": {"tile_cols2_min_n": -1, "wgs_per_cu": 1}}}))
    with pytest.raises(ValueError):
        tune.load_table(str(p))
    assert tune.load_table(str(tmp_path / "missing.json")) == {}
