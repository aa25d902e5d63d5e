"""GPU parity of the device linear assignment (Algorithm 1 step 10, eq. 2)
through fram_assign / fram_assign_dev, and of the solvers' use of it.

The oracle of the discretisation is an exact LAP (scipy's, called by
oracle.fram64.discretize) and, for tiny n, enumeration of all permutations.
Random continuous matrices have a unique optimum, so the permutation itself
must match; matrices with ties are compared on the optimal value and checked
to return a permutation.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import fram64 as O

pytestmark = pytest.mark.gpu


def value(W, p):
    Wd = np.asarray(W, dtype=np.float64)
    return float(Wd[np.arange(Wd.shape[0]), p].sum())


def check_perm(p, n):
    assert sorted(np.asarray(p).tolist()) == list(range(n))


def near_permutation(n, seed, collide_frac):
    """A matrix like FRAM's N near convergence: one dominant entry per row on a
    hidden permutation, small positive noise, and a fraction of rows whose
    maximum is moved onto another row's column (collisions)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    W = (0.01 * rng.random((n, n))).astype(np.float32)
    W[np.arange(n), perm] = 0.5 + 0.1 * rng.random(n).astype(np.float32)
    rows = rng.choice(n, size=int(round(collide_frac * n)), replace=False)
    for i in rows:
        k = rng.integers(n)
        W[i, perm[k]] = W[i, perm[i]] + np.float32(0.05 * rng.random())
    return W


@pytest.mark.parametrize("seed", range(8))
def test_assign_equals_enumeration(ctx, seed):
    rng = np.random.default_rng(seed)
    n = 7
    W = rng.random((n, n)).astype(np.float32)
    if seed % 2:
        W[:] = W[0]  # every row has the same maximiser: all rows collide
    p = ctx.assign(W)
    check_perm(p, n)
    best = max(itertools.permutations(range(n)), key=lambda q: value(W, list(q)))
    assert abs(value(W, p) - value(W, list(best))) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 50, 300, 1000])
def test_assign_random_matches_oracle(ctx, n):
    rng = np.random.default_rng(n)
    W = (rng.random((n, n)) ** 4).astype(np.float32)
    p = ctx.assign(W)
    ref = O.discretize(W.astype(np.float64))
    np.testing.assert_array_equal(p, ref)
    assert value(W, p) == value(W, ref)


# n <= 4096 runs the register solver (64 and 777 with sequential bids, 2048 to 4001
# after parallel bidding rounds; 777, 3998 and 4001 read rows column by column, the
# others as whole float4 groups); 4500 keeps the arrays of the other solver in LDS,
# 6000 and 10000 in the workspace.
@pytest.mark.parametrize("n", [64, 777, 2048, 3998, 4000, 4001, 4500, 6000, 10000])
def test_assign_near_permutation_matches_oracle(ctx, n):
    W = near_permutation(n, seed=n, collide_frac=0.05)
    p = ctx.assign(W)
    paths = ctx.last_stats()["lap_paths"]
    ref = O.discretize(W.astype(np.float64))
    np.testing.assert_array_equal(p, ref)
    assert paths > 0


def test_assign_argmax_permutation_needs_no_path(ctx):
    W = near_permutation(500, seed=3, collide_frac=0.0)
    W[np.arange(500), np.argmax(W, 1)] += 1.0  # argmax rows are a permutation
    assert len(set(np.argmax(W, 1).tolist())) == 500
    p = ctx.assign(W)
    np.testing.assert_array_equal(p, np.argmax(W, 1))
    assert ctx.last_stats()["lap_paths"] == 0


@pytest.mark.parametrize("n,levels", [(60, 3), (257, 2), (1000, 5), (1100, 4)])
def test_assign_with_ties_is_optimal(ctx, n, levels):
    rng = np.random.default_rng(n + levels)
    W = rng.integers(0, levels, size=(n, n)).astype(np.float32)
    p = ctx.assign(W)
    check_perm(p, n)
    ref = O.discretize(W.astype(np.float64))
    assert value(W, p) == value(W, ref)


def test_assign_constant_matrix_is_a_permutation(ctx):
    # Every permutation is optimal; all rows but the first collide on column 0
    # and must still end up matched, deterministically.
    W = np.full((333, 333), 0.25, dtype=np.float32)
    p = ctx.assign(W)
    check_perm(p, 333)
    assert ctx.last_stats()["lap_paths"] == 332
    np.testing.assert_array_equal(ctx.assign(W), p)


def test_assign_constant_matrix_with_parallel_bids(ctx):
    # n >= 1024: the parallel rounds cannot place any row (every drop is 0 and
    # every column is wanted by all), stop on the stall rule, and the paths
    # finish the job.
    W = np.full((1030, 1030), 0.5, dtype=np.float32)
    p = ctx.assign(W)
    check_perm(p, 1030)
    assert ctx.last_stats()["lap_paths"] == 1029
    np.testing.assert_array_equal(ctx.assign(W), p)


def test_assign_dev_wide_leading_dimension_and_stream(ctx):
    import torch
    n, ld = 1500, 1536
    W = near_permutation(n, seed=11, collide_frac=0.1)
    dW = torch.zeros((n, ld), dtype=torch.float32, device="cuda")
    dW[:, :n] = torch.from_numpy(W).cuda()
    dW[:, n:] = 10.0  # outside the n x n block: must never be read as an entry
    dp = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    ctx.assign_dev(dW.data_ptr(), ld, n, dp.data_ptr(), stream)
    p = dp.cpu().numpy()
    np.testing.assert_array_equal(p, O.discretize(W.astype(np.float64)))


@pytest.mark.parametrize("n", [40, 1100])
def test_assign_dev_non_finite_row_is_reported(ctx, n):
    import torch
    from paper_2508_00887_amd import fram as F
    W = torch.rand((n, n), dtype=torch.float32, device="cuda")
    W[5, :] = float("nan")
    dp = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(F.FramError) as e:
        ctx.assign_dev(W.data_ptr(), n, n, dp.data_ptr())
    assert e.value.status == F.FRAM_ENUMERIC
    assert (dp.cpu().numpy() == -1).all()
    # The context stays usable.
    Wh = np.eye(4, dtype=np.float32)[::-1].copy()
    np.testing.assert_array_equal(ctx.assign(Wh), [3, 2, 1, 0])


def test_solve_after_one_iteration_assigns_a_constant_matrix(ctx):
    # After one outer iteration N = alpha 11^T / n exactly (all rows collide):
    # the discretisation is the assignment of a constant matrix.
    pr = next(synth.config_pairs(0, [4]))
    perm, obj, st = ctx.solve(pr.A, pr.B, theta=2.0, iters=1, tol=0.0, prec="fp32")
    check_perm(perm, pr.n)
    assert st["lap_paths"] == pr.n - 1  # every row but the first collides
    host = float(np.sum(pr.A * pr.B[np.ix_(perm, perm)]))
    assert obj == pytest.approx(host, rel=1e-12)
    perms, objs, sts = ctx.solve_many([pr.A, pr.A], [pr.B, pr.B], theta=2.0, iters=1, tol=0.0,
                                      prec="fp32")
    for p, o, s in zip(perms, objs, sts):
        np.testing.assert_array_equal(p, perm)
        assert s["lap_paths"] == pr.n - 1
        assert o == obj
