"""The driver's launch-choice cache file (host logic only; the GPU side is in
test_gpu_batching.py): round trip, replacement, incomplete records, atomic rewrite."""
import json
import os

import pytest

from paper_2511_17634_amd.driver import TUNING_FIELDS, load_tuning_cache, store_tuning_cache


def rec(pm=8, waves=4):
    return {"polish_m": pm, "waves": waves, "wg_per_cu": 1, "split": 0, "seed_waves": 4,
            "seed_wg_per_cu": 1, "seed_rows_per_thread": 1}


def test_missing_file_is_empty(tmp_path):
    assert load_tuning_cache(str(tmp_path / "none.json")) == {}


def test_round_trip_and_replace(tmp_path):
    p = str(tmp_path / "c.json")
    store_tuning_cache(p, "gfx950/cu256/64x1x63/m40", rec())
    store_tuning_cache(p, "gfx950/cu256/128x1x255/m60", rec(15, 8))
    got = load_tuning_cache(p)
    assert got == {"gfx950/cu256/64x1x63/m40": rec(), "gfx950/cu256/128x1x255/m60": rec(15, 8)}
    store_tuning_cache(p, "gfx950/cu256/64x1x63/m40", rec(6))
    assert load_tuning_cache(p)["gfx950/cu256/64x1x63/m40"]["polish_m"] == 6
    # only the record fields are kept; no temporary file is left behind
    store_tuning_cache(p, "k", {**rec(), "m": 30, "extra": 1})
    assert set(load_tuning_cache(p)["k"]) == set(TUNING_FIELDS)
    assert sorted(os.listdir(tmp_path)) == ["c.json"]


def test_incomplete_records_are_ignored_and_refused(tmp_path):
    p = str(tmp_path / "c.json")
    r = rec()
    del r["split"]
    with open(p, "w") as f:
        json.dump({"good": rec(), "bad": r, "junk": 3}, f)
    assert list(load_tuning_cache(p)) == ["good"]
    with pytest.raises(ValueError):
        store_tuning_cache(p, "bad", r)


def test_not_an_object(tmp_path):
    p = str(tmp_path / "c.json")
    with open(p, "w") as f:
        json.dump([1, 2], f)
    with pytest.raises(ValueError):
        load_tuning_cache(p)
    # a store replaces an unreadable file with a fresh object
    with open(p, "w") as f:
        f.write("{not json")
    store_tuning_cache(p, "k", rec())
    assert list(load_tuning_cache(p)) == ["k"]
