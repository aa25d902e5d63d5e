"""Pins of the oracle's SDSN (Algorithm 2) and projections (Sec. 5.1, App. D).

Every expected value here comes from outside the oracle: a generic
least-squares projection (textbook KKT / pseudo-inverse), closed forms derived
from Algorithm 2 by hand, brute-force enumeration, or the paper's theorems.
"""
import itertools
import pathlib
from fractions import Fraction

import numpy as np
import pytest

from oracle import fram64 as O

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"


def affine_projection(X, rhs):
    """argmin ||Y - X||_F s.t. Y1 = rhs, Y^T 1 = rhs, by the generic formula
    y = x - C^T (C C^T)^+ (C x - b) for the stacked constraint matrix C."""
    n = X.shape[0]
    C = np.zeros((2 * n, n * n))
    for i in range(n):
        C[i, i * n:(i + 1) * n] = 1.0          # row sums
        C[n + i, i::n] = 1.0                    # column sums
    b = np.full(2 * n, rhs, dtype=float)
    x = X.ravel()
    y = x - C.T @ (np.linalg.pinv(C @ C.T) @ (C @ x - b))
    return y.reshape(n, n)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 10])
def test_p1_is_the_affine_projection_asymmetric(n):
    # Theorem 5: eq. (P1_sol) solves the projection also for asymmetric X.
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, n)) * 3.0
    Y = O.p1(X)
    np.testing.assert_allclose(Y, affine_projection(X, 1.0), atol=1e-12)
    np.testing.assert_allclose(Y.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(Y.sum(0), 1.0, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4, 7])
def test_p3_is_the_zero_sum_projection(n):
    # Truncation lemma (App. D): P3 projects onto {Y1 = 0, Y^T 1 = 0}.
    rng = np.random.default_rng(10 + n)
    X = rng.normal(size=(n, n))
    np.testing.assert_allclose(O.p3(X), affine_projection(X, 0.0), atol=1e-12)


def test_p1_of_x_plus_delta_splits_into_p1_plus_p3():
    # The decomposition used in the proof of the truncation theorem (App. D).
    rng = np.random.default_rng(3)
    X, dX = rng.random((6, 6)), 1e-3 * rng.normal(size=(6, 6))
    np.testing.assert_allclose(O.p1(X + dX), O.p1(X) + O.p3(dX), atol=1e-14)


def test_p2_is_nonnegative_part():
    X = np.array([[-1.0, 0.0, 2.5], [3.0, -0.0, -7.0], [1e-300, -1e-300, 4.0]])
    np.testing.assert_array_equal(O.p2(X), np.maximum(X, 0.0))


def test_golden_hand_worked_sdsn_identity_theta4():
    rows = [l.split() for l in (GOLDEN / "sdsn_permutation_n3_theta4.txt").read_text().splitlines()
            if l.strip() and not l.startswith("#")]
    D, info = O.sdsn(np.eye(3), theta=4.0, gamma_th=0.0, max_passes=len(rows))
    assert info.passes == len(rows)
    for (k, a_k, g_k), g in zip(rows, info.gammas):
        assert abs(g - float(Fraction(g_k))) < 1e-15
    a_last = float(Fraction(rows[-1][1]))
    np.testing.assert_allclose(D, a_last * np.eye(3), atol=1e-15)


@pytest.mark.parametrize("n,theta", [(5, 4.0), (8, 3.0), (20, 10.0)])
def test_sdsn_permutation_closed_form_large_theta(n, theta):
    # X = Pi: X^(k) = a_k Pi with 1 - a_k = (1 - theta/2)(1 - 1/n)^k, gamma_k = a_k - 1.
    rng = np.random.default_rng(n)
    Pi = np.eye(n)[rng.permutation(n)]
    gth = 1e-6
    D, info = O.sdsn(Pi, theta, gth, max_passes=100000)
    a0 = theta / 2
    k_expected = next(k for k in range(1, 10**6) if (a0 - 1) * (1 - 1 / n) ** k <= gth)
    assert info.passes == k_expected
    for k, g in enumerate(info.gammas, start=1):
        assert abs(g - (a0 - 1) * (1 - 1 / n) ** k) < 1e-12
    a = 1 - (1 - a0) * (1 - 1 / n) ** info.passes
    np.testing.assert_allclose(D, a * Pi, atol=1e-12)


@pytest.mark.parametrize("theta", [0.5, 1.0, 2.0])
def test_sdsn_permutation_closed_form_small_theta(theta):
    # theta <= 2: one pass gives (theta/2) Pi + (1 - theta/2) 11^T / n, already in D.
    n = 7
    Pi = np.eye(n)[np.random.default_rng(1).permutation(n)]
    D, info = O.sdsn(Pi, theta, 1e-6)
    assert info.passes == 1
    np.testing.assert_allclose(D, theta / 2 * Pi + (1 - theta / 2) / n, atol=1e-15)


@pytest.mark.parametrize("theta", [0.1, 2.0, 37.0])
def test_sdsn_constant_matrix_gives_uniform(theta):
    D, info = O.sdsn(np.full((6, 6), 3.25), theta, 1e-9)
    assert info.passes == 1
    np.testing.assert_allclose(D, 1 / 6, atol=1e-15)


def test_sdsn_zero_matrix_gives_uniform():
    D, info = O.sdsn(np.zeros((5, 5)), 2.0, 1e-9)
    np.testing.assert_allclose(D, 0.2, atol=1e-15)


def test_sdsn_small_theta_single_pass_is_exact_projection_and_tends_to_uniform():
    # If P1(X^(0)) >= 0 it is the projection onto D (Theorem 1) after one pass,
    # and D^theta -> 11^T/n linearly as theta -> 0 (Theorem 4).
    rng = np.random.default_rng(7)
    X = 0.5 + 0.5 * rng.random((9, 9))
    prev = None
    for theta in [1e-1, 1e-2, 1e-3]:
        D, info = O.sdsn(X, theta, 1e-12)
        X0 = theta / 2 * X / X.max()
        assert info.passes == 1
        np.testing.assert_allclose(D, affine_projection(X0, 1.0), atol=1e-14)
        err = np.abs(D - 1 / 9).max()
        if prev is not None:
            assert err < prev / 5
        prev = err


@pytest.mark.parametrize("seed", range(4))
def test_sdsn_invariants_random(seed):
    rng = np.random.default_rng(100 + seed)
    n = [10, 37, 64, 100][seed]
    X = rng.random((n, n)) ** 3
    gth = 1e-8
    D, info = O.sdsn(X, 2.0 + 4 * seed, gth, max_passes=100000)
    assert (D >= 0).all()
    assert info.gamma <= gth
    # Rows/columns: P1 output sums to 1 exactly; clipping only adds mass, and the
    # clipped mass over all rows is n * gamma (App. B.1).
    for s in (D.sum(0), D.sum(1)):
        assert (s >= 1 - 1e-12).all() and (s <= 1 + n * info.gamma + 1e-12).all()
    g = np.array(info.gammas)
    assert (np.diff(g) <= 1e-13).all(), "gamma must not increase (App. B.1)"


def test_sdsn_feasibility_to_1e12():
    rng = np.random.default_rng(5)
    n = 40
    X = rng.random((n, n))
    D, info = O.sdsn(X, 2.0, 1e-14 / n, max_passes=100000)
    assert (D >= 0).all()
    np.testing.assert_allclose(D.sum(0), 1.0, atol=1e-12)
    np.testing.assert_allclose(D.sum(1), 1.0, atol=1e-12)


def _brute_lap(W):
    n = W.shape[0]
    best, arg = -np.inf, None
    for p in itertools.permutations(range(n)):
        v = sum(W[i, p[i]] for i in range(n))
        if v > best:
            best, arg = v, p
    return np.array(arg), best


@pytest.mark.parametrize("theta", [0.5, 2.0, 10.0, 1e3])
@pytest.mark.parametrize("seed", range(3))
def test_sdsn_two_by_two_reaches_exact_projection(theta, seed):
    # n = 2: the affine set of P1 is the line Y(t) = [[t, 1-t], [1-t, t]], so the
    # projection of X^(0) onto it is t = (x11 + x22 - x12 - x21)/4 + 1/2 and the
    # projection onto D (Theorem 1's D^theta) is that t clipped to [0, 1].
    # Alternating projections reach it (for t > 1 the iterates obey
    # t' = (1 + t)/2), so SDSN must return it.
    rng = np.random.default_rng(300 + seed)
    X = rng.random((2, 2))
    X0 = theta / 2 * X / X.max()
    t = (X0[0, 0] + X0[1, 1] - X0[0, 1] - X0[1, 0]) / 4 + 0.5
    t = min(max(t, 0.0), 1.0)
    D, info = O.sdsn(X, theta, 1e-14, max_passes=1000)
    np.testing.assert_allclose(D, [[t, 1 - t], [1 - t, t]], atol=1e-12)


@pytest.mark.parametrize("theta", [0.5, 2.0, 10.0])
@pytest.mark.parametrize("seed", range(4))
def test_sdsn_normalized_assignment_error_bound(theta, seed):
    # Theorem 2: (1/n)(<D^inf, X> - <D^theta, X>) <= 1/theta, X normalised by its
    # max.  The theorem is about the exact projection D^theta; SDSN (plain
    # alternating projections) meets it at the paper's operating points
    # (theta = 2 dense, 10 sparse) but not for every X at theta >= 20, where
    # it can settle on a non-optimal vertex of D.
    rng = np.random.default_rng(11 + seed)
    n = 8
    X = rng.random((n, n))
    Xh = X / X.max()
    _, best = _brute_lap(Xh)
    D, _ = O.sdsn(X, theta, 1e-12, max_passes=200000)
    eps = (best - (D * Xh).sum()) / n
    assert -1e-12 <= eps <= 1.0 / theta + 1e-9


def test_sdsn_truncation_residual_is_not_amplified():
    # Theorem 7 (App. D): a truncation residual injected mid-iteration is
    # absorbed by the remaining passes -- the result is again feasible and
    # moves by no more than the order of the perturbation.
    rng = np.random.default_rng(17)
    n = 30
    X = rng.random((n, n))
    D_ref, _ = O.sdsn(X, 2.0, 1e-13, max_passes=100000)
    D_half, _ = O.sdsn(X, 2.0, 0.0, max_passes=5)
    dX = 1e-5 * rng.normal(size=(n, n))
    pert = D_half + dX
    # theta = 2 max(pert) makes Algorithm 2's first scaling the identity.
    D_pert, info = O.sdsn(pert, 2.0 * pert.max(), 1e-13, max_passes=100000)
    assert (D_pert >= 0).all() and info.gamma <= 1e-13
    np.testing.assert_allclose(D_pert.sum(0), 1.0, atol=1e-10)
    assert np.abs(D_pert - D_ref).max() <= 10 * np.abs(dX).max()
