"""Pins of the oracle's node term (eq. 1 and eq. 3 with K = F F~^T, weight lam;
Algorithm 1 steps 2-3 scale K by c = max(A, A~, K)).  CPU only.

* Without a node term (K = 0 or lam = 0) the run is the plain one, bitwise.
* Edgeless graphs: X = lam K / c every iteration, so D = SDSN(X) is fixed and
  N^(t) = (1 - (1 - alpha)^t) D, delta^(t) = alpha (1-alpha)^(t-1) / (1 - (1-alpha)^t).
* Node term = a scaled permutation matrix: SDSN's closed form for theta <= 2.
* Noiseless attributed pairs: by Cauchy-Schwarz the hidden permutation attains
  the largest possible objective ||A||_F^2 + 2 lam ||F||_F^2.
* The objective's node part is 2 lam <M, K>, checked against enumeration.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import fram64 as O


@pytest.mark.parametrize("seed", range(3))
def test_no_node_term_is_the_plain_run(seed):
    pr = next(synth.config_pairs(0, [seed]))
    N0, i0 = O.fram(pr.A, pr.B, iters=15)
    N1, i1 = O.fram(pr.A, pr.B, iters=15, K=np.zeros_like(pr.A), lam=1.0)
    N2, i2 = O.fram(pr.A, pr.B, iters=15, K=np.ones_like(pr.A) * 0.3, lam=0.0)
    assert np.array_equal(N0, N1) and i0.sdsn_passes == i1.sdsn_passes
    # lam = 0 with K <= max(A, B) leaves c and every step unchanged.
    assert np.array_equal(N0, N2)


def test_prescale_divides_k_by_c():
    rng = np.random.default_rng(0)
    A, B, K = rng.random((5, 5)), rng.random((5, 5)), 3.0 * rng.random((5, 5))
    As, Bs, Ks, c = O.prescale(A, B, K)
    assert c == pytest.approx(K.max())
    np.testing.assert_allclose(As * np.sqrt(c), A, rtol=1e-15)
    np.testing.assert_allclose(Bs * np.sqrt(c), B, rtol=1e-15)
    np.testing.assert_allclose(Ks * c, K, rtol=1e-15)


@pytest.mark.parametrize("theta", [2.0, 10.0])
def test_edgeless_graphs_closed_form(theta):
    rng = np.random.default_rng(int(theta))
    n, alpha, lam = 12, 0.95, 0.7
    K = rng.random((n, n))
    Z = np.zeros((n, n))
    N, info = O.fram(Z, Z, theta=theta, alpha=alpha, iters=6, K=K, lam=lam, gamma_th=1e-13,
                     sdsn_max=100000)
    D, _ = O.sdsn(lam * K / K.max(), theta, 1e-13, 100000)
    np.testing.assert_allclose(N, (1 - (1 - alpha) ** 6) * D, atol=1e-12)
    t = np.arange(1, 7)
    expect = alpha * (1 - alpha) ** (t - 1) / (1 - (1 - alpha) ** t)
    np.testing.assert_allclose(info.deltas, expect, rtol=1e-9)
    assert len(set(info.sdsn_passes)) == 1  # the same projection every iteration


@pytest.mark.parametrize("theta", [0.5, 2.0])
def test_node_term_permutation_closed_form(theta):
    # K = a permutation matrix: D = (theta/2) Pi + (1 - theta/2) 11^T / n after
    # one SDSN pass (theta <= 2), and the discretisation returns Pi.
    n, alpha = 9, 0.95
    perm = np.random.default_rng(1).permutation(n)
    K = np.zeros((n, n))
    K[np.arange(n), perm] = 1.0
    Z = np.zeros((n, n))
    N, info = O.fram(Z, Z, theta=theta, alpha=alpha, iters=1, K=K, lam=1.0)
    D = (theta / 2) * K + (1 - theta / 2) * np.ones((n, n)) / n
    np.testing.assert_allclose(N, alpha * D, atol=1e-14)
    assert info.sdsn_passes == [1]
    np.testing.assert_array_equal(O.discretize(N), perm)


@pytest.mark.parametrize("seed", range(3))
def test_noiseless_attributed_pair_reaches_the_certified_optimum(seed):
    pr = synth.make_attributed_pair(40, 0.3, 0.0, 500 + seed, feat_sigma=0.0)
    lam = 1.0
    sigma, obj, _, _ = O.solve(pr.A, pr.B, iters=60, K=pr.K, lam=lam)
    # K = F F~^T with F~[perm] = F: <M, K> <= ||F||_F^2 = trace of K along perm.
    bound = float(np.sum(pr.A ** 2)) + 2 * lam * float(np.sum(pr.K[np.arange(40), pr.perm]))
    np.testing.assert_array_equal(sigma, pr.perm)
    assert obj == pytest.approx(bound, rel=1e-12)


def test_objective_node_part_against_enumeration():
    rng = np.random.default_rng(3)
    n = 5
    A = np.triu(rng.random((n, n)), 1)
    A = A + A.T
    B = np.triu(rng.random((n, n)), 1)
    B = B + B.T
    K = rng.random((n, n))
    lam = 0.4
    for q in itertools.permutations(range(n)):
        M = np.zeros((n, n))
        M[np.arange(n), q] = 1.0
        phi = 0.5 * np.sum((M.T @ A @ M) * B) + lam * np.sum(M * K)
        assert O.objective(A, B, np.array(q), K, lam) == pytest.approx(2 * phi, rel=1e-13)


def test_scaling_edges_and_nodes_together_keeps_the_matching():
    # A, A~ -> s A, s A~ and K -> s^2 K multiply both terms of X by s^2 / c'
    # relative to c, so SDSN (which divides by max X) sees the same matrix.
    pr = synth.make_attributed_pair(30, 0.3, 0.05, 77)
    s1, _, _, _ = O.solve(pr.A, pr.B, iters=40, K=pr.K)
    s2, _, _, _ = O.solve(3.0 * pr.A, 3.0 * pr.B, iters=40, K=9.0 * pr.K)
    np.testing.assert_array_equal(s1, s2)
