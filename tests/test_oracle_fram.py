"""Pins of the oracle's FRAM (Algorithm 1), discretisation (eq. 2) and scoring.

Expected values come from closed forms of the first iterations, the
Cauchy-Schwarz optimality certificate of noiseless isomorphic pairs,
brute-force enumeration over all permutations, exact invariances (power-of-two
scaling, relabelling, swapping the graphs) and the matrix form of the
objective -- never from the oracle itself.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import fram64 as O


def _pair(n, p, sigma, seed, **kw):
    return synth.make_pair(n, p, sigma, seed, **kw)


def test_first_iterations_closed_form():
    # N^(0) = 0 => X^(1) = 0 => D^(1) = 11^T/n, N^(1) = alpha 11^T/n, delta^(1) = 1;
    # then X^(2) = (alpha/n) (A1)(B1)^T is rank one.
    pr = _pair(12, 0.5, 0.05, 1)
    N1, info1 = O.fram(pr.A, pr.B, iters=1)
    np.testing.assert_allclose(N1, 0.95 / 12, atol=1e-16)
    assert info1.deltas == [1.0] and info1.sdsn_passes == [1]
    As, Bs, _ = O.prescale(pr.A, pr.B)
    X2 = As @ N1 @ Bs
    np.testing.assert_allclose(X2, 0.95 / 12 * np.outer(As.sum(1), Bs.sum(0)), rtol=1e-13)
    assert np.linalg.matrix_rank(X2, tol=1e-10 * np.abs(X2).max()) == 1


def test_prescale_divides_by_sqrt_of_global_max():
    A = np.array([[0.0, 4.0], [4.0, 0.0]])
    B = np.array([[0.0, 9.0], [9.0, 0.0]])
    As, Bs, c = O.prescale(A, B)
    assert c == 9.0
    np.testing.assert_array_equal(As, A / 3.0)
    np.testing.assert_array_equal(Bs, B / 3.0)


@pytest.mark.parametrize("n,seed", [(20, 0), (45, 1), (80, 2)])
def test_noiseless_pair_is_solved_to_global_optimum(n, seed):
    # B = P^T A P: tr(A M B M^T) <= ||A||_F ||B||_F = ||A||_F^2 (Cauchy-Schwarz),
    # attained by M = P, so recovering perm certifies the QAP optimum at any n.
    pr = _pair(n, 0.4, 0.0, seed, weights="half_open_top")
    sigma, obj, N, info = O.solve(pr.A, pr.B, theta=2.0, iters=60)
    np.testing.assert_array_equal(sigma, pr.perm)
    assert abs(obj - (pr.A ** 2).sum()) <= 1e-12 * (pr.A ** 2).sum()


def _brute_lap(W):
    n = W.shape[0]
    return max(itertools.permutations(range(n)), key=lambda p: sum(W[i, p[i]] for i in range(n)))


@pytest.mark.parametrize("seed", range(6))
def test_discretize_equals_enumeration(seed):
    rng = np.random.default_rng(seed)
    n = 7
    W = rng.random((n, n))
    np.testing.assert_array_equal(O.discretize(W), _brute_lap(W))


def test_discretize_is_nearest_permutation():
    # eq. (2): argmin_P ||P - N||_F is the same as argmax_P <P, N>.
    rng = np.random.default_rng(9)
    n = 6
    N = rng.random((n, n))
    best = min(itertools.permutations(range(n)),
               key=lambda p: np.linalg.norm(np.eye(n)[list(p)] - N))
    np.testing.assert_array_equal(O.discretize(N), best)


def test_objective_gather_equals_trace_form():
    rng = np.random.default_rng(4)
    pr = _pair(9, 0.6, 0.1, 4)
    sigma = rng.permutation(9)
    M = np.zeros((9, 9))
    M[np.arange(9), sigma] = 1.0
    ref = np.trace(pr.A @ M @ pr.B @ M.T)
    assert abs(O.objective(pr.A, pr.B, sigma) - ref) < 1e-12 * abs(ref)


def _brute_qap(A, B):
    n = A.shape[0]
    best = -np.inf
    for p in itertools.permutations(range(n)):
        best = max(best, float(np.sum(A * B[np.ix_(p, p)])))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_qap_brute_force_small(seed):
    # FRAM is a heuristic: never above the optimum; on low-noise isomorphic
    # pairs it must reach it.
    n = 7
    pr = _pair(n, 0.6, 0.01, 50 + seed, weights="half_open_top")
    sigma, obj, _, _ = O.solve(pr.A, pr.B, iters=100)
    opt = _brute_qap(pr.A, pr.B)
    assert obj <= opt + 1e-12
    assert abs(obj - opt) <= 1e-12 * opt


def test_qap_brute_force_random_pairs_bound():
    # Unrelated graphs: FRAM is a heuristic, so only the upper bound is exact
    # (on tiny unrelated graphs it can even fall below the permutation mean).
    rng = np.random.default_rng(77)
    for t in range(6):
        n = 6
        A = synth.er_adjacency(rng, n, 0.6)
        B = synth.er_adjacency(rng, n, 0.6)
        _, obj, _, _ = O.solve(A, B, iters=100)
        vals = [float(np.sum(A * B[np.ix_(p, p)])) for p in itertools.permutations(range(n))]
        assert min(vals) - 1e-12 <= obj <= max(vals) + 1e-12


@pytest.mark.parametrize("k", [-4, 2, 6])
def test_scale_invariance_bitwise_for_powers_of_four(k):
    # Sec. 4.1: scaling A and B by c leaves the matching unchanged.  With
    # c = 2^k, k even, sqrt(c) is a power of two, every step commutes with the
    # scaling, and the N trajectory is bit-identical.
    pr = _pair(30, 0.5, 0.05, 5)
    N1, i1 = O.fram(pr.A, pr.B, iters=15)
    N2, i2 = O.fram(pr.A * 2.0 ** k, pr.B * 2.0 ** k, iters=15)
    np.testing.assert_array_equal(N1, N2)
    assert i1.sdsn_passes == i2.sdsn_passes


@pytest.mark.parametrize("c", [3.7, 1e-3, 250.0])
def test_scale_invariance_matching(c):
    pr = _pair(40, 0.5, 0.05, 6)
    s1 = O.solve(pr.A, pr.B, iters=40)[0]
    s2 = O.solve(pr.A * c, pr.B * c, iters=40)[0]
    np.testing.assert_array_equal(s1, s2)


def test_scale_invariance_of_each_graph_separately():
    # SDSN divides by max X, so A -> aA, B -> bB (a != b) also leaves the
    # trajectory unchanged up to rounding.
    pr = _pair(40, 0.5, 0.05, 8)
    s1 = O.solve(pr.A, pr.B, iters=40)[0]
    s2 = O.solve(pr.A * 5.0, pr.B * 0.01, iters=40)[0]
    np.testing.assert_array_equal(s1, s2)


def test_relabelling_equivariance():
    pr = _pair(40, 0.5, 0.05, 7)
    q = np.random.default_rng(70).permutation(40)
    A2 = np.empty_like(pr.A)
    A2[np.ix_(q, q)] = pr.A  # node k of A becomes node q[k]
    s1 = O.solve(pr.A, pr.B, iters=50)[0]
    s2 = O.solve(A2, pr.B, iters=50)[0]
    np.testing.assert_array_equal(s2[q], s1)


def test_swapping_graphs_inverts_matching():
    # SDSN commutes with transposition and (A N B)^T = B N^T A.
    pr = _pair(40, 0.5, 0.05, 8)
    s_ab = O.solve(pr.A, pr.B, iters=50)[0]
    s_ba = O.solve(pr.B, pr.A, iters=50)[0]
    inv = np.empty_like(s_ab)
    inv[s_ab] = np.arange(40)
    np.testing.assert_array_equal(s_ba, inv)


def test_do_while_and_tolerance():
    # Stops at the first t with delta^(t) <= tol (do-while), else after iters.
    pr = _pair(30, 0.5, 0.05, 9)
    _, full = O.fram(pr.A, pr.B, iters=60, tol=0.0)
    assert full.outer_iters == 60 and not full.converged
    tol = full.deltas[40] * 1.0000001
    t_stop = next(t for t, d in enumerate(full.deltas, start=1) if d <= tol)
    _, info = O.fram(pr.A, pr.B, iters=60, tol=tol)
    assert info.converged and info.outer_iters == t_stop
    assert info.deltas == full.deltas[:t_stop]


def test_accuracy_counts_inliers_only():
    perm = np.array([2, 0, 1, 3])
    sigma = np.array([2, 0, 3, 3])
    assert O.accuracy(sigma, perm) == 0.75
    assert O.accuracy(sigma, perm, np.array([True, True, False, True])) == 1.0


def test_stable_argmax_stop():
    # The optional argmax-stability stop: the loop ends at the first t whose
    # row argmax equals those of the w previous iterates (all permutations).
    pr = next(synth.config_pairs(0, [0]))  # n = 50 workload, seed 0
    _, full = O.fram(pr.A, pr.B, iters=60)
    As, Bs, _ = O.prescale(pr.A, pr.B)
    # Recompute the iterates to find the first stable run of length 3.
    N = np.zeros((50, 50))
    args = []
    for t in range(60):
        D, _ = O.sdsn(As @ N @ Bs, 2.0, 1e-6, 1000)
        N = 0.05 * N + 0.95 * D
        a = np.argmax(N, axis=1)
        args.append(a if len(np.unique(a)) == 50 else None)
    t_stop = next(t for t in range(3, 60) if all(args[t - d] is not None for d in range(4))
                  and all(np.array_equal(args[t], args[t - d]) for d in range(1, 4))) + 1
    _, info = O.fram(pr.A, pr.B, iters=60, stable_iters=3)
    assert info.outer_iters == t_stop and info.converged
    assert info.deltas == full.deltas[:t_stop]


def test_stall_step_counts_only_non_halving_deltas_below_the_threshold():
    # Early phase above stall_delta: never counted, whatever the trend.
    c, m = 0, None
    for d in [1.0, 0.7, 0.8, 0.85, 0.6, 2e-3]:
        c, m = O.stall_step(c, m, d, 1e-3)
        assert c == 0 and m is None
    # Decrease at any rate (0.41 or 0.99 per iteration): every delta is a new
    # minimum, the count stays 0.
    for k in range(10):
        c, m = O.stall_step(c, m, 9e-4 * 0.41 ** k * 0.99 ** k, 1e-3)
        assert c == 0
    # A plateau at the precision's floor: counted; a new minimum resets.
    floor = m
    counts = []
    for d in [1.5 * floor, floor, 1.1 * floor, 0.999 * floor, 2.0 * floor]:
        c, m = O.stall_step(c, m, d, 1e-3)
        counts.append(c)
    assert counts == [1, 2, 3, 0, 1]


def test_stall_rule_never_fires_while_delta_decreases():
    # In FP64 delta falls monotonically down to any tol used here (by ~0.85
    # per iteration on this pair), so the stall rule leaves the run exactly as
    # delta <= tol alone would.
    pr = next(synth.config_pairs(0, [0]))
    _, ref = O.fram(pr.A, pr.B, iters=150, tol=1e-9)
    _, info = O.fram(pr.A, pr.B, iters=150, tol=1e-9, stall_iters=3)
    assert ref.converged and info.outer_iters == ref.outer_iters
    assert info.deltas == ref.deltas


def test_stall_rule_stops_at_a_delta_floor():
    # With tol = 0 the FP64 delta decreases to its rounding floor (~1e-15,
    # after ~250 iterations on this pair) and only fluctuates there; the rule
    # stops the run at that floor instead of at the iteration cap.
    pr = next(synth.config_pairs(0, [0]))
    _, info = O.fram(pr.A, pr.B, iters=500, tol=0.0, stall_iters=3)
    assert info.converged and info.outer_iters < 500
    assert min(info.deltas) < 1e-14
    assert info.deltas[-1] >= min(info.deltas[:-1])
