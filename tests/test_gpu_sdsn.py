"""GPU parity of SDSN (Algorithm 2) through fram_sdsn_project (C ABI).

* Closed forms from Algorithm 2 (permutation inputs for theta <= 2 and
  theta > 2, constant and non-positive inputs) must hold to FP32 rounding.
* Random inputs: the GPU's pass count must match the FP64 oracle's (gamma is
  evaluated in FP64 on both sides), and after the same number of passes the
  matrices agree elementwise within an FP32 error budget that grows with the
  pass count (each pass is non-expansive; every pass adds at most a few FP32
  roundings of entries of size ~1/n).
* Output invariants: X >= 0 exactly, row/column sums within n*gamma.
"""
import numpy as np
import pytest

from oracle import fram64 as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("theta", [1.0, 2.0])
@pytest.mark.parametrize("n", [3, 64, 100])
def test_permutation_small_theta_one_pass(ctx, n, theta):
    Pi = np.eye(n, dtype=np.float32)[np.random.default_rng(n).permutation(n)]
    X, st = ctx.sdsn_project(Pi, theta)
    assert st["sdsn_passes"] == 1
    np.testing.assert_allclose(X, theta / 2 * Pi + (1 - theta / 2) / n, atol=2e-7, rtol=1e-6)


@pytest.mark.parametrize("n,theta", [(5, 4.0), (50, 3.0)])
def test_permutation_large_theta_closed_form(ctx, n, theta):
    Pi = np.eye(n, dtype=np.float32)[np.random.default_rng(n).permutation(n)]
    gth = 1e-4
    X, st = ctx.sdsn_project(Pi, theta, gamma_tol=gth, sdsn_max=100000)
    a0 = theta / 2
    k = next(k for k in range(1, 10**6) if (a0 - 1) * (1 - 1 / n) ** k <= gth)
    assert abs(st["sdsn_passes"] - k) <= 1
    a = 1 - (1 - a0) * (1 - 1 / n) ** st["sdsn_passes"]
    np.testing.assert_allclose(X, a * Pi, atol=1e-5)


@pytest.mark.parametrize("K", ["constant", "zero", "negative"])
def test_degenerate_inputs_give_uniform(ctx, K):
    n = 70
    M = {"constant": np.full((n, n), 3.5), "zero": np.zeros((n, n)),
         "negative": -np.random.default_rng(0).random((n, n))}[K].astype(np.float32)
    X, st = ctx.sdsn_project(M, 2.0)
    np.testing.assert_allclose(X, 1.0 / n, rtol=1e-6)
    # One pass is exact in real arithmetic; in FP32 the first pass cancels
    # terms of size theta/2 to produce entries 1/n, which can leave gamma a few
    # n*2^-24 above zero and cost one more (no-change) pass.
    assert st["sdsn_passes"] <= 2


def test_single_node(ctx):
    X, st = ctx.sdsn_project(np.array([[7.0]], dtype=np.float32), 2.0)
    assert X[0, 0] == 1.0


@pytest.mark.parametrize("theta", [2.0, 10.0])
@pytest.mark.parametrize("n", [2, 3, 17, 64, 65, 130, 255, 300, 777, 1000])
def test_sdsn_matches_oracle(ctx, n, theta):
    rng = np.random.default_rng(7 * n + int(theta))
    K = (rng.random((n, n)) ** 2).astype(np.float32)
    gth = 1e-6
    X, st = ctx.sdsn_project(K, theta, gamma_tol=gth, sdsn_max=20000)
    k = st["sdsn_passes"]
    _, info = O.sdsn(K.astype(np.float64), theta, gth, 20000)
    # Near gamma_tol gamma falls by ~1% per pass at theta = 10, and FP32
    # rounding of the pass output slows that tail: an FP32 model of the pass
    # needs up to ~11% more passes than FP64 on these inputs (1448 vs 1308 at
    # n = 1000; pinned on the CPU by tests/test_sdsn_fp32_rounding.py), so the
    # pass count is compared with that slack and the matrices are compared
    # element-wise after the GPU's own pass count.
    slack = 0.05 if theta <= 2.0 else 0.15
    assert abs(k - info.passes) <= max(3, int(slack * info.passes)), (k, info.passes)
    D, _ = O.sdsn(K.astype(np.float64), theta, 0.0, max_passes=k)
    err = np.abs(X.astype(np.float64) - D).max()
    assert err <= k * 2e-6 / n + 1e-7, err
    assert (X >= 0).all()
    tol = n * max(st["gamma"], 0.0) + 1e-4
    assert np.abs(X.astype(np.float64).sum(0) - 1).max() <= tol
    assert np.abs(X.astype(np.float64).sum(1) - 1).max() <= tol


def test_sdsn_deterministic(ctx):
    K = (np.random.default_rng(3).random((600, 600)) ** 3).astype(np.float32)
    X1, s1 = ctx.sdsn_project(K, 2.0)
    X2, s2 = ctx.sdsn_project(K, 2.0)
    np.testing.assert_array_equal(X1, X2)
    assert s1["sdsn_passes"] == s2["sdsn_passes"]


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_sdsn_tile_variants_agree(ctx, tile):
    K = (np.random.default_rng(5).random((300, 300)) ** 2).astype(np.float32)
    Xa, sa = ctx.sdsn_project(K, 2.0, tile=64)
    Xb, sb = ctx.sdsn_project(K, 2.0, tile=tile)
    assert abs(sa["sdsn_passes"] - sb["sdsn_passes"]) <= 1
    np.testing.assert_allclose(Xa, Xb, atol=1e-6)


@pytest.mark.parametrize("n,tile", [(1, 64), (37, 64), (64, 64), (100, 128), (200, 256)])
def test_single_tile_launch_equals_per_pass_launches(ctx, n, tile):
    # A matrix that is one tile runs the whole projection in one launch; with
    # profile = 1 every pass is its own launch.  Same passes, same arithmetic.
    K = (np.random.default_rng(90 + n).random((n, n)) ** 2).astype(np.float32)
    X1, s1 = ctx.sdsn_project(K, 2.0, tile=tile, sdsn_mode="stream")
    X2, s2 = ctx.sdsn_project(K, 2.0, tile=tile, sdsn_mode="stream", profile=True)
    assert s1["sdsn_passes"] == s2["sdsn_passes"] and s1["gamma"] == s2["gamma"]
    np.testing.assert_array_equal(X1, X2)
    # and a cap that stops the loop early is honoured exactly
    X3, s3 = ctx.sdsn_project(K, 2.0, tile=tile, sdsn_mode="stream", sdsn_max=3)
    X4, s4 = ctx.sdsn_project(K, 2.0, tile=tile, sdsn_mode="stream", sdsn_max=3, profile=True)
    assert s3["sdsn_passes"] == s4["sdsn_passes"] <= 3
    np.testing.assert_array_equal(X3, X4)


@pytest.mark.parametrize("n", [3, 65, 300, 1000, 2100, 4000])
def test_onchip_equals_streaming_bitwise(ctx, n):
    # Same formulas and the same fixed reduction order per tile: the on-chip
    # projection (one cooperative launch) must reproduce the per-pass launches.
    K = (np.random.default_rng(n).random((n, n)) ** 2).astype(np.float32)
    Xs, ss = ctx.sdsn_project(K, 2.0, sdsn_mode="stream")
    Xo, so = ctx.sdsn_project(K, 2.0, sdsn_mode="onchip")
    assert ss["sdsn_passes"] == so["sdsn_passes"]
    np.testing.assert_array_equal(Xs, Xo)


@pytest.mark.parametrize("n", [300, 4000])
def test_onchip_forced_fallbacks_equal_streaming(ctx, n):
    # A 1 us bound on the pass barriers (the roll call keeps its default)
    # makes the first barrier wait time out: the grid abandons the launch
    # without writing, and the projection streams from the untouched input.
    # A 1 us roll-call bound abandons it before any pass, or lets it run when
    # every workgroup checked in within the bound.  Every outcome must give
    # the streaming result bit for bit.
    K = (np.random.default_rng(7 + n).random((n, n)) ** 2).astype(np.float32)
    Xs, ss = ctx.sdsn_project(K, 2.0, sdsn_mode="stream")
    Xb, sb = ctx.sdsn_project(K, 2.0, sdsn_mode="onchip", onchip_barrier_us=1)
    Xr, sr = ctx.sdsn_project(K, 2.0, sdsn_mode="onchip", onchip_roll_us=1)
    for X, st in [(Xb, sb), (Xr, sr)]:
        assert st["sdsn_onchip"] + st["sdsn_fallbacks"] == 1
        assert st["sdsn_passes"] == ss["sdsn_passes"] and st["gamma"] == ss["gamma"]
        np.testing.assert_array_equal(X, Xs)
    if n == 4000:
        # 256 workgroups never all reach the first barrier within 1 us.
        assert sb["sdsn_fallbacks"] == 1
    # and a later projection on the same context runs on chip again
    Xo, so = ctx.sdsn_project(K, 2.0, sdsn_mode="onchip")
    assert so["sdsn_onchip"] == 1
    np.testing.assert_array_equal(Xo, Xs)


@pytest.mark.parametrize("mode", ["stream", "onchip"])
def test_modes_match_oracle_theta10(ctx, mode):
    n = 500
    K = (np.random.default_rng(42).random((n, n)) ** 2).astype(np.float32)
    X, st = ctx.sdsn_project(K, 10.0, sdsn_max=20000, sdsn_mode=mode)
    k = st["sdsn_passes"]
    D, _ = O.sdsn(K.astype(np.float64), 10.0, 0.0, max_passes=k)
    assert np.abs(X - D).max() <= k * 2e-6 / n + 1e-7


@pytest.mark.parametrize("n,tile", [(4000, 256), (4097, 256), (4097, 128)])
def test_sdsn_matches_oracle_at_full_size(ctx, n, tile):
    # The bench's layout (tile 256: a 16 x 16 grid at n = 4000) and ragged
    # grids past 16 tiles per side (n = 4097: 17 x 17 of 256, 33 x 33 of 128),
    # whose row/column partial chains take the general summation path.  A
    # fixed pass count on both sides (the FP64 oracle takes ~0.3 s per pass
    # at this size), then element-wise.  After only 24 passes the entries are
    # still of the size of the first pass's theta/2-scaled input, not ~1/n, so
    # the budget is relative to the largest entry: each pass rounds every
    # entry and its two FP32 corrections (<= 2 ulps), and the pass map is
    # non-expansive, so errors add at most linearly over the passes.
    rng = np.random.default_rng(n + tile)
    K = (rng.random((n, n)) ** 2).astype(np.float32)
    k = 24
    X, st = ctx.sdsn_project(K, 2.0, gamma_tol=1e-6, sdsn_max=k, tile=tile, sdsn_mode="stream")
    assert st["sdsn_passes"] == k and st["gemm_tile"] == tile
    D, info = O.sdsn(K.astype(np.float64), 2.0, 0.0, max_passes=k)
    assert info.passes == k
    err = np.abs(X.astype(np.float64) - D).max()
    assert err <= k * 2.0 ** -23 * max(D.max(), 1.0 / n) + 1e-7, err
    # gamma of the output, as the oracle defines it (Sec. 5.2), in FP64
    g_or = D.sum() / n - 1.0
    assert abs(st["gamma"] - g_or) <= 1e-4
