"""The autotuner on the GPU: it times the streaming SDSN pass per tile edge,
and a solve under the tuned table is bit for bit the solve with that edge
given explicitly (the table only replaces the automatic choice)."""
import math

import numpy as np
import pytest

import synth
from paper_2508_00887_amd import fram as F
from paper_2508_00887_amd import tune

pytestmark = pytest.mark.gpu


def test_tuned_table_equals_explicit_tile(ctx):
    try:
        table = tune.tune(ctx, sizes=(150, 700), passes=30, reps=1)
        assert [p["n"] for p in table["probes"]] == [150, 700]
        for p in table["probes"]:
            assert p["tile"] in (64, 128, 256)
            assert all(math.isfinite(v) and v > 0 for v in p["us_per_pass"].values())
        tune.apply(table)
        q = next(synth.config_pairs(0, [0]))  # n = 50: first bucket
        t = F.fram_auto_tile(q.n)
        assert t == table["buckets"][0]["tile"]
        p1, o1, s1 = ctx.solve(q.A, q.B, iters=20, tol=0.0, prec="fp32")
        p2, o2, s2 = ctx.solve(q.A, q.B, iters=20, tol=0.0, prec="fp32", tile=t)
        assert s1["gemm_tile"] == s2["gemm_tile"] == t
        np.testing.assert_array_equal(p1, p2)
        assert o1 == o2
    finally:
        tune.clear()
    assert F.fram_auto_tile(50) == 64
