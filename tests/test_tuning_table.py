"""The autotune table's file handling (CPU): a missing file is an empty
table, a stored table reads back equal, the write is atomic (no temporary
file left behind), and a file that is not a table is refused."""
import json
import os

import pytest

from paper_2503_05408_amd import tuning


def test_missing_file_is_an_empty_table(tmp_path):
    assert tuning.load_table(str(tmp_path / "none.json")) == {}


def test_round_trip_and_no_temporary_left(tmp_path):
    path = str(tmp_path / "t.json")
    table = {"00ff/lower/S3-T9-K0/dev/gfx950": {"form": "async", "us": {"persistent": 9.0, "plain": 8.0,
                                                                         "async": 5.0}}}
    tuning.store_table(path, table)
    assert tuning.load_table(path) == table
    assert os.listdir(tmp_path) == ["t.json"]
    table["other"] = {"form": "plain", "us": {}}
    tuning.store_table(path, table)
    assert tuning.load_table(path) == table


def test_a_file_that_is_not_a_table_is_refused(tmp_path):
    path = str(tmp_path / "bad.json")
    with open(path, "w") as f:
        json.dump([1, 2, 3], f)
    with pytest.raises(ValueError):
        tuning.load_table(path)
