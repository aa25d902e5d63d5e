"""GPU parity of the whole FRAM solve (Algorithm 1 with SDSN, discretisation
and objective) through fram_solve_ex / fram_solve_dev / fram_solve_many.

* FP32 GEMMs must return the FP64 oracle's permutation exactly, with relative
  objective error <= 1e-5 (n = 50 workload: all 100 seeds; n = 1000 workload:
  all 10 seeds, stored oracle results; ragged and edge sizes computed here).
* BF16 / FP16 GEMMs: relative objective error <= 1e-3 and matching accuracy
  at most 0.5 points below the oracle's.
* Noiseless pairs: the hidden permutation and ||A||_F^2 (global optimum).
* The returned objective equals the FP64 gather of the returned permutation.
"""
import json
import pathlib

import numpy as np
import pytest

import synth
from oracle import fram64 as O

pytestmark = pytest.mark.gpu
GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"

# The batched kernel (one workgroup per pair, fram_solve_many for n <= 512)
# made a GPU memory access fault on its first test run on the device
# (8 pairs, FP32); a CPU emulation of the same launch finds no
# out-of-bounds access, so the cause is not shown and the kernel was
# removed.  These tests expect that kernel (gemm_tile 32) and stay skipped;
# fram_solve_many's lockstep group of small pairs has its own tests below
# (test_group_*).
BATCHED_OFF = pytest.mark.skip(
    reason="batched kernel switched off: it faulted the GPU on its first run and the cause "
           "is not found (a CPU emulation of the launch runs clean)")


def host_objective(A, B, perm):
    return float(np.sum(A * B[np.ix_(perm, perm)]))


def check_perm(perm, n):
    assert sorted(perm.tolist()) == list(range(n))


@pytest.mark.parametrize("seed", range(100))
def test_small_workload_fp32_equals_oracle(ctx, seed):
    pr = next(synth.config_pairs(0, [seed]))
    s_or, obj_or, _, _ = O.solve(pr.A, pr.B, theta=2.0, iters=100)
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=100, tol=0.0, prec="fp32")
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert st["outer_iters"] == 100


@pytest.mark.parametrize("n", [50, 300])
@pytest.mark.parametrize("tile", [64, 128, 256])
def test_fp32_solve_equals_oracle_for_every_tile_edge(ctx, n, tile):
    # Every tile edge on small grids: n = 300 at edge 256 is a 2 x 2 grid with
    # a ragged tail, without the XCD block mapping of the tile grid (the
    # eight-wave GEMM tile there is otherwise only reached at n = 4000).
    pr = synth.make_pair(n, 0.3, 0.03, 9500 + n, weights="half_open_top")
    s_or, obj_or, _, _ = O.solve(pr.A, pr.B, theta=2.0, iters=40)
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=40, tol=0.0, prec="fp32", tile=tile)
    assert st["gemm_tile"] == tile
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-9 * abs(obj_or)


@pytest.mark.parametrize("n", [2, 3, 5, 17, 63, 64, 65, 129, 200])
def test_edge_sizes_fp32_equals_oracle(ctx, n):
    pr = synth.make_pair(n, 0.5, 0.03, 9000 + n, weights="half_open_top")
    s_or, obj_or, _, _ = O.solve(pr.A, pr.B, theta=2.0, iters=60)
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=60, prec="fp32")
    check_perm(perm, n)
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("n", [100, 257])
def test_noiseless_pairs_reach_global_optimum(ctx, n, prec):
    pr = synth.make_pair(n, 0.4, 0.0, 7000 + n, weights="half_open_top")
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=60, prec=prec)
    np.testing.assert_array_equal(perm, pr.perm)
    ref = float((pr.A ** 2).sum())
    assert abs(obj - ref) <= 1e-12 * ref


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_precision_accuracy_gate(ctx, prec, seed):
    pr = synth.make_pair(300, 0.3, 0.05, 8000 + seed, outlier_frac=0.1)
    s_or, obj_or, _, _ = O.solve(pr.A, pr.B, theta=2.0, iters=100)
    acc_or = O.accuracy(s_or, pr.perm, pr.inlier)
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=100, prec=prec)
    check_perm(perm, 300)
    assert abs(obj - obj_or) <= 1e-3 * abs(obj_or)
    assert O.accuracy(perm, pr.perm, pr.inlier) >= acc_or - 0.005


def _golden(name):
    p = GOLDEN / name
    if not p.exists():
        pytest.skip(f"{name} not generated (tests/golden/make_golden.py)")
    return json.loads(p.read_text())


@pytest.mark.parametrize("seed", range(1000, 1010))
def test_n1000_workload_fp32_equals_oracle(ctx, seed):
    g = _golden(f"fram_c1_seed{seed}.json")
    pr = next(synth.config_pairs(1, [seed - 1000]))
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=g["theta"], iters=g["iters"], tol=g["tol"],
                              prec="fp32", gamma_tol=g["gamma_th"], sdsn_max=g["sdsn_max"])
    np.testing.assert_array_equal(perm, np.array(g["perm"]))
    assert abs(obj - g["objective"]) <= 1e-5 * abs(g["objective"])
    assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_n4000_workload_accuracy_gate(ctx, prec):
    g = _golden("fram_c2_seed2000.json")
    pr = next(synth.config_pairs(2, [0]))
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=g["theta"], iters=g["iters"], tol=g["tol"],
                              prec=prec, gamma_tol=g["gamma_th"], sdsn_max=g["sdsn_max"])
    check_perm(perm, pr.n)
    assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
    assert abs(obj - g["objective"]) <= 1e-3 * abs(g["objective"])
    assert O.accuracy(perm, pr.perm, pr.inlier) >= g["accuracy"] - 0.005


def test_n4000_full_size_properties(ctx):
    # Independent of the stored oracle run: a valid permutation, the FP64
    # objective of exactly that permutation, and recovery of most inliers.
    pr = next(synth.config_pairs(2, [0]))
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=100, tol=1e-6, prec="bf16")
    check_perm(perm, pr.n)
    assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
    assert O.accuracy(perm, pr.perm, pr.inlier) > 0.9
    assert st["gemm_tile"] == 256


@pytest.mark.parametrize("n", [4097, 6000])
def test_large_ragged_solve_properties(ctx, n):
    # Past the n = 4000 workload: a ragged tile grid (4097 = 16 tiles of 256
    # plus one row) and the assignment's global-memory mode (n > 4400).  No
    # stored oracle run: a valid permutation, the FP64 objective of exactly
    # that permutation, and the planted inliers recovered.
    pr = synth.make_pair(n, 0.3, 0.05, 9100 + n, outlier_frac=0.1)
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=100, tol=1e-6, prec="bf16",
                              stall_iters=3)
    check_perm(perm, n)
    assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
    assert O.accuracy(perm, pr.perm, pr.inlier) > 0.9
    assert st["converged"] == 1 and st["outer_iters"] < 100


def test_tolerance_stops_like_the_oracle(ctx):
    pr = synth.make_pair(120, 0.5, 0.05, 4242)
    _, full = O.fram(pr.A, pr.B, iters=80)
    tol = full.deltas[30] * 1.001
    _, info = O.fram(pr.A, pr.B, iters=80, tol=tol)
    perm, obj, st = ctx.solve(pr.A, pr.B, iters=80, tol=tol, prec="fp32")
    assert st["converged"] == 1
    assert abs(st["outer_iters"] - info.outer_iters) <= 1
    assert abs(st["delta"] - info.deltas[-1]) <= 1e-3 * info.deltas[-1] + 1e-9


def test_deterministic_and_device_entry_point(ctx):
    import torch
    pr = synth.make_pair(500, 0.4, 0.05, 4343)
    p1, o1, s1 = ctx.solve(pr.A, pr.B, iters=40, prec="bf16")
    p2, o2, s2 = ctx.solve(pr.A, pr.B, iters=40, prec="bf16")
    np.testing.assert_array_equal(p1, p2)
    assert o1 == o2 and s1["sdsn_passes"] == s2["sdsn_passes"]
    dA = torch.from_numpy(pr.A).cuda()
    dB = torch.from_numpy(pr.B).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    p3, o3, s3 = ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), 500, iters=40, prec="bf16",
                               stream=stream)
    np.testing.assert_array_equal(p1, p3)
    assert o1 == o3


def test_device_entry_point_rejects_invalid_device_input(ctx):
    import torch
    from paper_2508_00887_amd import FramError
    A = np.ones((50, 50)) - np.eye(50)
    B = A.copy()
    B[3, 4] = -1.0
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    with pytest.raises(FramError):
        ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), 50)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [33, 100, 257])
@pytest.mark.parametrize("defect", ["none", "asym_corner", "asym_tile_edge", "nan_diag",
                                    "inf_pair", "neg_pair_tail"])
def test_device_validation_over_tile_pairs(ctx, n, defect):
    # The device check compares 32 x 32 tiles with their mirror tiles: every
    # kind of defect, in the first, a straddling and the last (ragged) tile.
    import torch
    from paper_2508_00887_amd import FramError
    import paper_2508_00887_amd.fram as F
    rng = np.random.default_rng(n)
    A = np.triu(rng.random((n, n)), 1)
    A = A + A.T
    B = A.copy()
    if defect == "asym_corner":
        B[0, n - 1] += 1e-9
    elif defect == "asym_tile_edge":
        A[32, 31] += 1e-9
    elif defect == "nan_diag":
        B[n - 1, n - 1] = np.nan
    elif defect == "inf_pair":
        A[n - 1, 0] = A[0, n - 1] = np.inf
    elif defect == "neg_pair_tail":
        B[n - 2, n - 1] = B[n - 1, n - 2] = -0.5
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    if defect == "none":
        perm, _, _ = ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), n, iters=2, tol=0.0)
        assert sorted(perm.tolist()) == list(range(n))
    else:
        with pytest.raises(FramError) as e:
            ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), n, iters=2, tol=0.0)
        assert e.value.status == F.FRAM_EINVAL
    torch.cuda.synchronize()


def _small_batch(count, seed, n_hi=160):
    rng = np.random.default_rng(seed)
    return [synth.make_pair(int(rng.integers(20, n_hi + 1)), float(rng.uniform(0.1, 0.5)), 0.03,
                            seed * 1000 + i) for i in range(count)]


@BATCHED_OFF
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_pairs_match_oracle(ctx, prec):
    # The batched kernel (one workgroup per pair) against the FP64 oracle:
    # FP32 GEMMs give the oracle's permutation, BF16 the accuracy gate.
    pairs = _small_batch(8, 31)
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=60,
                                        prec=prec)
    for pr, perm, obj, st in zip(pairs, perms, objs, stats):
        s_or, obj_or, _, _ = O.solve(pr.A, pr.B, iters=60)
        check_perm(perm, pr.n)
        assert st["outer_iters"] == 60 and st["gemm_tile"] == 32
        assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
        if prec == "fp32":
            np.testing.assert_array_equal(perm, s_or)
            assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
        else:
            assert abs(obj - obj_or) <= 1e-3 * abs(obj_or)
            assert O.accuracy(perm, pr.perm) >= O.accuracy(s_or, pr.perm) - 0.005


@BATCHED_OFF
def test_batched_result_is_the_same_alone_and_in_the_mix(ctx):
    pairs = _small_batch(40, 32, n_hi=300)
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=40)
    for q in (0, 7, 39):
        p1, o1, s1 = ctx.solve_many([pairs[q].A], [pairs[q].B], iters=40)
        np.testing.assert_array_equal(p1[0], perms[q])
        assert o1[0] == objs[q]
        assert s1[0]["sdsn_passes"] == stats[q]["sdsn_passes"]


@BATCHED_OFF
def test_batched_mixed_sizes_and_tolerance(ctx):
    # n = 1 is answered on the host, n > 512 goes through the single-pair path.
    big = synth.make_pair(600, 0.3, 0.05, 6060)
    one = np.zeros((1, 1))
    small = synth.make_pair(40, 0.4, 0.02, 6061)
    perms, objs, stats = ctx.solve_many([one, small.A, big.A], [one, small.B, big.B], iters=100,
                                        tol=1e-4, prec="bf16")
    assert list(perms[0]) == [0] and objs[0] == 0.0
    for pr, perm, obj, st in zip([small, big], perms[1:], objs[1:], stats[1:]):
        check_perm(perm, pr.n)
        assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
        assert st["converged"] == 1 and st["delta"] <= 1e-4
    assert stats[2]["gemm_tile"] != 32


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [50, 700, 2100])
def test_onchip_and_streaming_solves_agree(ctx, n, prec):
    pr = synth.make_pair(n, 0.3, 0.05, 5100 + n)
    p1, o1, s1 = ctx.solve(pr.A, pr.B, iters=30, prec=prec, sdsn_mode="stream")
    p2, o2, s2 = ctx.solve(pr.A, pr.B, iters=30, prec=prec, sdsn_mode="onchip")
    np.testing.assert_array_equal(p1, p2)
    assert o1 == o2
    assert s1["sdsn_passes"] == s2["sdsn_passes"]
    assert abs(s1["delta"] - s2["delta"]) <= 1e-12 * max(s1["delta"], 1e-300)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_onchip_barrier_aborts_fall_back_inside_solves(ctx, prec):
    # Every on-chip launch of the solve gives up at its first pass barrier
    # (1 us bound); each iteration's projection and N update then stream from
    # the same X, so the solve equals the streaming one bit for bit.
    pr = synth.make_pair(4000, 0.3, 0.05, 5200)
    N1 = np.empty((pr.n, pr.n), dtype=np.float32)
    N2 = np.empty_like(N1)
    p1, o1, s1 = ctx.solve(pr.A, pr.B, iters=4, prec=prec, sdsn_mode="stream", N_out=N1)
    p2, o2, s2 = ctx.solve(pr.A, pr.B, iters=4, prec=prec, sdsn_mode="onchip",
                           onchip_barrier_us=1, N_out=N2)
    assert s2["outer_iters"] == 4 and s2["sdsn_fallbacks"] + s2["sdsn_onchip"] == 4
    assert s2["sdsn_fallbacks"] >= 1
    np.testing.assert_array_equal(N1, N2)
    np.testing.assert_array_equal(p1, p2)
    assert o1 == o2 and s1["sdsn_passes"] == s2["sdsn_passes"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_solve_many_group_equals_single_solves(ctx, prec):
    # Pairs whose matrix is one tile (n <= 256) run in the lockstep group;
    # each must equal solving it alone with its one-tile edge.  Larger pairs
    # run the single-pair path (default layout), concurrently with the group.
    sizes = [2, 17, 64, 65, 100, 128, 129, 200, 256, 257, 300]
    pairs = [synth.make_pair(m, 0.3, 0.05, 6100 + m) for m in sizes]
    perms, objs, sts = ctx.solve_many([q.A for q in pairs], [q.B for q in pairs], iters=60,
                                      tol=1e-6, prec=prec, stall_iters=3)
    for q, p, o, st in zip(pairs, perms, objs, sts):
        edge = 64 if q.n <= 64 else 128 if q.n <= 128 else 256
        kw = dict(tile=edge) if q.n <= 256 else {}
        p1, o1, s1 = ctx.solve(q.A, q.B, iters=60, tol=1e-6, prec=prec, stall_iters=3, **kw)
        np.testing.assert_array_equal(p, p1)
        assert o == o1, q.n
        for key in ("outer_iters", "sdsn_passes", "sdsn_passes_max", "converged", "stalled",
                    "lap_paths", "gemm_tile"):
            assert st[key] == s1[key], (q.n, key, st[key], s1[key])
        assert st["delta"] == s1["delta"] and st["gamma"] == s1["gamma"], q.n


@pytest.mark.parametrize("seed", range(6))
def test_stability_stop_matches_oracle(ctx, seed):
    pr = next(synth.config_pairs(0, [seed]))
    s_or, obj_or, _, info = O.solve(pr.A, pr.B, iters=100, stable_iters=3)
    perm, obj, st = ctx.solve(pr.A, pr.B, iters=100, prec="fp32", stable_iters=3)
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert abs(st["outer_iters"] - info.outer_iters) <= 2
    pb, ob, sb = ctx.solve_many([pr.A], [pr.B], iters=100, prec="fp32", stable_iters=3)
    np.testing.assert_array_equal(pb[0], s_or)
    assert abs(sb[0]["outer_iters"] - info.outer_iters) <= 2


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_n4000_stability_stop_accuracy_gate(ctx, prec):
    # The n = 4000 workload with delta <= 1e-6 or a 3-iteration stable argmax.
    # On this pair the row argmax of N is never a permutation (outlier rows of
    # B collide; the oracle's final row argmax is not one either), so the
    # stability rule cannot fire and a low-precision run ends at the cap or on
    # delta; either way the result must meet the accuracy gate against the
    # oracle's delta-converged solve.
    g = _golden("fram_c2_seed2000.json")
    assert not g["row_argmax_is_perm"]
    pr = next(synth.config_pairs(2, [0]))
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=100, tol=1e-6, prec=prec,
                              stable_iters=3)
    check_perm(perm, pr.n)
    assert st["outer_iters"] == 100 or st["delta"] <= 1e-6
    assert abs(obj - g["objective"]) <= 1e-3 * abs(g["objective"])
    assert O.accuracy(perm, pr.perm, pr.inlier) >= g["accuracy"] - 0.005


def test_solve_many_equals_single_solves(ctx):
    # fram_solve_many returns, pair by pair, what fram_solve returns for that
    # pair alone with the one-tile layout the lockstep group uses (n = 1
    # answered on the host).
    pairs = _small_batch(4, 33, n_hi=200)
    one = np.zeros((1, 1))
    As = [one] + [p.A for p in pairs]
    Bs = [one] + [p.B for p in pairs]
    perms, objs, stats = ctx.solve_many(As, Bs, iters=30, prec="bf16")
    assert list(perms[0]) == [0] and objs[0] == 0.0
    for pr, perm, obj, st in zip(pairs, perms[1:], objs[1:], stats[1:]):
        edge = 64 if pr.n <= 64 else 128 if pr.n <= 128 else 256
        p1, o1, s1 = ctx.solve(pr.A, pr.B, iters=30, prec="bf16", tile=edge)
        np.testing.assert_array_equal(perm, p1)
        assert obj == o1 and st["sdsn_passes"] == s1["sdsn_passes"]
    # Options the group does not take (here a fixed tile that is not the
    # pair's edge) send every pair down the single-pair path: the default
    # solve's result.
    perms, objs, stats = ctx.solve_many(As[1:], Bs[1:], iters=30, prec="bf16", tile=64)
    for pr, perm, obj, st in zip(pairs, perms, objs, stats):
        p1, o1, s1 = ctx.solve(pr.A, pr.B, iters=30, prec="bf16", tile=64)
        np.testing.assert_array_equal(perm, p1)
        assert obj == o1 and st["sdsn_passes"] == s1["sdsn_passes"]


def test_stall_stop_reaches_the_oracle_solution(ctx):
    # FP32 gradients: delta decreases like the oracle's down to the FP32
    # floor, where the stall rule stops the loop; the assignment is the
    # oracle's converged one.
    pr = next(synth.config_pairs(0, [0]))
    s_or, obj_or, _, info = O.solve(pr.A, pr.B, iters=400, tol=1e-9)
    perm, obj, st = ctx.solve(pr.A, pr.B, iters=400, tol=0.0, prec="fp32", stall_iters=3)
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert st["stalled"] == 1 and st["converged"] == 1 and st["outer_iters"] < 400


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_n4000_stall_stop_accuracy_gate(ctx, prec):
    # The n = 4000 workload with delta <= 1e-6 or the stall rule: the
    # low-precision paths level off above delta = 1e-6 and the stall rule
    # stops them well before the cap; the result must meet the accuracy gate
    # against the oracle's delta-converged solve.
    g = _golden("fram_c2_seed2000.json")
    pr = next(synth.config_pairs(2, [0]))
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=100, tol=1e-6, prec=prec,
                              stall_iters=3)
    check_perm(perm, pr.n)
    assert st["converged"] == 1 and st["outer_iters"] < 100
    assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
    assert abs(obj - g["objective"]) <= 1e-3 * abs(g["objective"])
    assert O.accuracy(perm, pr.perm, pr.inlier) >= g["accuracy"] - 0.005


# ---------------------------------------------------------------- DSPFP variant
from oracle import dspfp64 as P  # noqa: E402


@pytest.mark.parametrize("seed", range(4))
def test_dspfp_variant_equals_oracle(ctx, seed):
    # The baseline iteration (Sec. 4): FP32 GEMMs give the FP64 oracle's
    # permutation; the max-abs criterion trajectory is the oracle's, so the
    # stop iteration matches within one.
    pr = next(synth.config_pairs(0, [seed]))
    s_or, obj_or, _, info = P.solve(pr.A, pr.B, iters=60, tol=1e-4)
    perm, obj, st = ctx.solve(pr.A, pr.B, iters=60, tol=1e-4, prec="fp32", variant="dspfp")
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert abs(st["outer_iters"] - info.outer_iters) <= 1
    assert st["sdsn_passes"] == 30 * st["outer_iters"]


def test_dspfp_is_scale_sensitive_fram_is_not(ctx):
    # Sec. 5.1 on the device: scaling both graphs changes DSPFP's projected
    # iterates (here its criterion trajectory), never FRAM's.
    pr = synth.make_pair(120, 0.4, 0.05, 5151)
    s1 = ctx.solve(pr.A, pr.B, iters=8, prec="fp32", variant="dspfp")[2]
    s2 = ctx.solve(10 * pr.A, 10 * pr.B, iters=8, prec="fp32", variant="dspfp")[2]
    assert abs(s1["delta"] - s2["delta"]) > 1e-3 * max(s1["delta"], s2["delta"])
    f1 = ctx.solve(pr.A, pr.B, iters=8, prec="fp32")
    f2 = ctx.solve(10 * pr.A, 10 * pr.B, iters=8, prec="fp32")
    np.testing.assert_array_equal(f1[0], f2[0])
    assert f1[2]["sdsn_passes"] == f2[2]["sdsn_passes"]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("n", [50, 300])
def test_warm_start_resumes_bit_for_bit(ctx, n, prec):
    # Algorithm 1 step 1 with N^(0) = N0: a + b fixed iterations equal a
    # iterations followed by b iterations started from the first call's
    # final iterate, bit for bit (the iterate is the loop's whole state).
    pr = synth.make_pair(n, 0.3, 0.05, 8100 + n)
    a, b = 7, 5
    N_ab = np.empty((n, n), dtype=np.float32)
    p_ab, o_ab, s_ab = ctx.solve(pr.A, pr.B, iters=a + b, tol=0.0, prec=prec, N_out=N_ab)
    N_a = np.empty((n, n), dtype=np.float32)
    ctx.solve(pr.A, pr.B, iters=a, tol=0.0, prec=prec, N_out=N_a)
    N_b = np.empty((n, n), dtype=np.float32)
    p_b, o_b, s_b = ctx.solve(pr.A, pr.B, iters=b, tol=0.0, prec=prec, N0=N_a, N_out=N_b)
    np.testing.assert_array_equal(N_b, N_ab)
    np.testing.assert_array_equal(p_b, p_ab)
    assert o_b == o_ab and s_b["delta"] == s_ab["delta"]
    # The iterate is a convex combination of doubly stochastic matrices
    # started from 0: entries >= 0, row sums (1 - (1 - alpha)^t) within SDSN's
    # feasibility tolerance.
    assert N_ab.min() >= 0.0
    target = 1.0 - 0.05 ** (a + b)
    assert np.max(np.abs(N_ab.astype(np.float64).sum(axis=1) - target)) <= n * 1e-6 + 1e-5


def test_warm_start_on_device_memory(ctx):
    import torch
    n = 200
    pr = synth.make_pair(n, 0.3, 0.05, 8200)
    N_ab = np.empty((n, n), dtype=np.float32)
    p_ab, o_ab, _ = ctx.solve(pr.A, pr.B, iters=9, tol=0.0, prec="bf16", N_out=N_ab)
    dA = torch.from_numpy(pr.A).cuda()
    dB = torch.from_numpy(pr.B).cuda()
    dN = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), n, iters=4, tol=0.0, prec="bf16",
                  dN_out=dN.data_ptr())
    dN2 = torch.zeros_like(dN)
    p_b, o_b, _ = ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), n, iters=5, tol=0.0, prec="bf16",
                                dN0=dN.data_ptr(), dN_out=dN2.data_ptr())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dN2.cpu().numpy(), N_ab)
    np.testing.assert_array_equal(p_b, p_ab)
    assert o_b == o_ab


def test_concurrent_onchip_solves_equal_solving_alone(ctx):
    # Several contexts (fram_solve_many's workers, one stream and host thread
    # each) solving multi-tile pairs at once: their on-chip projections are
    # launched one after another across the streams, and every result equals
    # the streaming solve of that pair alone, bit for bit.
    sizes = [600, 900, 1300, 1700, 2100, 2500]
    pairs = [synth.make_pair(n, 0.3, 0.05, 5300 + n) for n in sizes]
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=20,
                                        prec="bf16", many_workers=6)
    for p, perm, obj, st in zip(pairs, perms, objs, stats):
        p1, o1, s1 = ctx.solve(p.A, p.B, iters=20, prec="bf16", sdsn_mode="stream")
        np.testing.assert_array_equal(perm, p1)
        assert obj == o1 and st["sdsn_passes"] == s1["sdsn_passes"]
        assert st["sdsn_onchip"] + st["sdsn_fallbacks"] == 20


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_group_pairs_match_oracle(ctx, prec):
    # The lockstep group (every pair here has n <= 160: one tile) against the
    # FP64 oracle: FP32 GEMMs give the oracle's permutation, BF16 the accuracy
    # gate.
    pairs = _small_batch(8, 31)
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=60,
                                        prec=prec)
    for pr, perm, obj, st in zip(pairs, perms, objs, stats):
        s_or, obj_or, _, _ = O.solve(pr.A, pr.B, iters=60)
        check_perm(perm, pr.n)
        assert st["outer_iters"] == 60 and st["gemm_tile"] >= pr.n
        assert abs(obj - host_objective(pr.A, pr.B, perm)) <= 1e-12 * abs(obj)
        if prec == "fp32":
            np.testing.assert_array_equal(perm, s_or)
            assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
        else:
            assert abs(obj - obj_or) <= 1e-3 * abs(obj_or)
            assert O.accuracy(perm, pr.perm) >= O.accuracy(s_or, pr.perm) - 0.005


def test_group_result_is_the_same_alone_and_in_the_mix(ctx):
    # 40 pairs up to n = 300: the grouped ones (n <= 256) and the single-pair
    # ones give the same result in the mix as in a call of their own.
    pairs = _small_batch(40, 32, n_hi=300)
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=40,
                                        tol=1e-6, stall_iters=3)
    for q in (0, 7, 39) + tuple(i for i, p in enumerate(pairs) if p.n > 256)[:2]:
        p1, o1, s1 = ctx.solve_many([pairs[q].A], [pairs[q].B], iters=40, tol=1e-6,
                                    stall_iters=3)
        np.testing.assert_array_equal(p1[0], perms[q])
        assert o1[0] == objs[q]
        assert s1[0]["sdsn_passes"] == stats[q]["sdsn_passes"]
        assert s1[0]["outer_iters"] == stats[q]["outer_iters"]


def test_group_honours_the_stall_rule(ctx):
    # BF16 delta levels off above tol = 1e-9: once it is below stall_delta
    # (1e-3) the delta-stall rule ends a grouped pair before the cap, each at
    # its own iteration; a pair whose delta stays above stall_delta runs to the
    # cap.  The results meet the accuracy gate against the FP64 oracle.
    pairs = _small_batch(6, 34, n_hi=250)
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=100,
                                        tol=1e-9, prec="bf16", stall_iters=3)
    assert any(st["stalled"] == 1 for st in stats)
    assert len({st["outer_iters"] for st in stats}) > 1
    for pr, perm, obj, st in zip(pairs, perms, objs, stats):
        if st["outer_iters"] < 100:
            assert st["converged"] == 1 and (st["stalled"] == 1 or st["delta"] <= 1e-9)
        else:
            assert st["delta"] > 1e-3, (pr.n, st["delta"])
        s_or, obj_or, _, _ = O.solve(pr.A, pr.B, iters=100, tol=1e-9)
        assert abs(obj - obj_or) <= 1e-3 * abs(obj_or)
        assert O.accuracy(perm, pr.perm) >= O.accuracy(s_or, pr.perm) - 0.005


@BATCHED_OFF
def test_batched_honours_the_stall_rule(ctx):
    # BF16 delta levels off near 1e-4, far above tol = 1e-9: the delta-stall
    # rule (the single-pair path's) ends every pair before the cap, and the
    # result still meets the accuracy gate against the FP64 oracle.
    pairs = _small_batch(6, 34, n_hi=250)
    perms, objs, stats = ctx.solve_many([p.A for p in pairs], [p.B for p in pairs], iters=100,
                                        tol=1e-9, prec="bf16", stall_iters=3)
    for pr, perm, obj, st in zip(pairs, perms, objs, stats):
        assert st["gemm_tile"] == 32 and st["stalled"] == 1 and st["outer_iters"] < 100
        s_or, obj_or, _, _ = O.solve(pr.A, pr.B, iters=100, tol=1e-9)
        assert abs(obj - obj_or) <= 1e-3 * abs(obj_or)
        assert O.accuracy(perm, pr.perm) >= O.accuracy(s_or, pr.perm) - 0.005
