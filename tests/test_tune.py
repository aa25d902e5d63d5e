"""The autotune tile table (fram_set_tile_table / fram_auto_tile) and the
tuner's host logic: bucket boundaries, JSON round trip, validation, and the
FRAM_TUNE_CACHE hook.  No GPU: the table and the automatic choice are host
arithmetic.  The table is process-wide, so every test leaves it cleared."""
import json
import os
import pathlib
import subprocess
import sys

import pytest

from paper_2508_00887_amd import fram as F
from paper_2508_00887_amd import tune

ROOT = pathlib.Path(__file__).resolve().parents[1]


@pytest.fixture
def table():
    yield
    tune.clear()


def test_builtin_rule_without_a_table(table):
    tune.clear()
    # one tile up to 128, then the largest edge whose grid has at least 200 tiles, else 64
    assert [F.fram_auto_tile(n) for n in (1, 64, 65, 128, 129, 500, 1000, 1700, 1800, 3500, 3600,
                                          4000, 32768)] == \
        [64, 64, 128, 128, 64, 64, 64, 64, 128, 128, 256, 256, 256]
    assert F.fram_auto_tile(0) == 0 and F.fram_auto_tile(32769) == 0


def test_table_selects_per_bucket_then_falls_back(table):
    F.fram_set_tile_table([100, 1000, 3000], [256, 128, 64])
    got = {n: F.fram_auto_tile(n) for n in (1, 100, 101, 1000, 1001, 3000, 3001, 4000)}
    assert got == {1: 256, 100: 256, 101: 128, 1000: 128, 1001: 64, 3000: 64, 3001: 128,
                   4000: 256}
    # the workspace estimate follows the same choice
    for n in (100, 1000, 3000):
        t = F.fram_auto_tile(n)
        assert F.fram_workspace_bytes(n, F.FRAM_BF16, 0) == F.fram_workspace_bytes(n, F.FRAM_BF16, t)
    tune.clear()
    assert F.fram_auto_tile(100) == 128 and F.fram_auto_tile(200) == 64


@pytest.mark.parametrize("n_max,tile", [
    ([0], [64]),                 # n_max must be >= 1
    ([10, 10], [64, 128]),       # strictly increasing
    ([10, 5], [64, 128]),
    ([10], [96]),                # edge not in {64, 128, 256}
    (list(range(1, 66)), [64] * 65),  # more than 64 buckets
])
def test_invalid_tables_are_rejected_and_leave_the_table(table, n_max, tile):
    F.fram_set_tile_table([500], [256])
    with pytest.raises(F.FramError) as e:
        F.fram_set_tile_table(n_max, tile)
    assert e.value.status == F.FRAM_EINVAL
    assert F.fram_auto_tile(400) == 256


def test_null_arrays_with_a_count_are_rejected():
    lib = F.load_library()
    assert lib.fram_set_tile_table(None, None, 2) == F.FRAM_EINVAL
    assert lib.fram_set_tile_table(None, None, -1) == F.FRAM_EINVAL
    assert lib.fram_set_tile_table(None, None, 0) == F.FRAM_OK


def test_buckets_from_probes():
    probes = [{"n": 64, "tile": 64}, {"n": 256, "tile": 64}, {"n": 1000, "tile": 64},
              {"n": 2000, "tile": 128}, {"n": 4000, "tile": 256}, {"n": 8000, "tile": 256}]
    b = tune.buckets_from(probes)
    # boundaries at the geometric mean of neighbouring probes; equal edges merge
    assert b == [{"n_max": 1414, "tile": 64}, {"n_max": 2828, "tile": 128},
                 {"n_max": 8000, "tile": 256}]
    assert tune.buckets_from(list(reversed(probes))) == b


def test_save_load_apply_round_trip(tmp_path, table):
    t = {"version": 1, "probes": [], "buckets": [{"n_max": 300, "tile": 128},
                                                 {"n_max": 5000, "tile": 64}]}
    p = tmp_path / "t.json"
    tune.save(t, str(p))
    tune.apply(tune.load(str(p)))
    assert [F.fram_auto_tile(n) for n in (300, 301, 5000, 5001)] == [128, 64, 64, 256]


@pytest.mark.parametrize("bad", [
    {"version": 2, "buckets": []},
    {"version": 1},
    {"version": 1, "buckets": [{"n_max": 10, "tile": 32}]},
    {"version": 1, "buckets": [{"n_max": 10, "tile": 64}, {"n_max": 10, "tile": 128}]},
    {"version": 1, "buckets": [{"n_max": 1.5, "tile": 64}]},
])
def test_validate_rejects_malformed_tables(bad, tmp_path):
    with pytest.raises(ValueError):
        tune.validate(bad)
    p = tmp_path / "bad.json"
    p.write_text(json.dumps(bad))
    with pytest.raises(ValueError):
        tune.load(str(p))


def test_tune_cache_environment_variable_is_applied_on_load(tmp_path):
    p = tmp_path / "t.json"
    tune.save({"version": 1, "buckets": [{"n_max": 50000 // 2, "tile": 128}]}, str(p))
    code = ("from paper_2508_00887_amd import fram as F; F.load_library(); "
            "print(F.fram_auto_tile(4000), F.fram_auto_tile(30000))")
    env = dict(os.environ, FRAM_TUNE_CACHE=str(p))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["128", "256"]
