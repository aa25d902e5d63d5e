"""Pins of the DSPFP oracle (Sec. 4 eq. iter.DSPFP, eq. 4, App. B.2) against
closed forms and invariants independent of its code."""
import numpy as np
import pytest

import synth
from oracle import dspfp64 as P
from oracle import fram64 as O


def test_projection_of_zero_is_the_barycentre():
    # P1(0) = 11^T/n >= 0, so every iteration returns 11^T/n.
    n = 7
    np.testing.assert_allclose(P.dsn(np.zeros((n, n))), np.full((n, n), 1.0 / n), rtol=0, atol=1e-16)


def test_doubly_stochastic_input_is_a_fixed_point():
    rng = np.random.default_rng(0)
    n = 9
    perms = [np.eye(n)[rng.permutation(n)] for _ in range(5)]
    w = rng.random(5)
    w /= w.sum()
    D = sum(wk * Pk for wk, Pk in zip(w, perms)) * 0.5 + 0.5 / n  # positive, doubly stochastic
    np.testing.assert_allclose(P.dsn(D), D, rtol=0, atol=1e-14)


@pytest.mark.parametrize("a,b,c,d", [(0.3, 0.1, 0.2, 0.4), (0.9, 0.8, 0.1, 0.05), (2.0, 0.0, 0.0, 1.0)])
def test_two_by_two_projection_closed_form(a, b, c, d):
    # D = [[p, 1-p], [1-p, p]]; minimising ||D - X||^2 over p gives
    # p = (a + d - b - c + 2)/4, clipped to [0, 1].  For n = 2 alternating
    # projections reach it (exactly when unclipped, halving the error per
    # iteration when clipped).
    X = np.array([[a, b], [c, d]])
    p = min(1.0, max(0.0, (a + d - b - c + 2.0) / 4.0))
    ref = np.array([[p, 1 - p], [1 - p, p]])
    np.testing.assert_allclose(P.dsn(X, 30), ref, rtol=0, atol=1e-8)


def test_projection_is_scale_sensitive():
    # P_D(wX) != P_D(X) (Sec. 5.1): with the 2 x 2 closed form, p moves with w.
    X = np.array([[0.3, 0.1], [0.2, 0.4]])
    p = [P.dsn(w * X, 30)[0, 0] for w in (0.5, 1.0, 4.0)]
    np.testing.assert_allclose(p, [(w * 0.4 + 2.0) / 4.0 for w in (0.5, 1.0, 4.0)], atol=1e-12)
    assert p[0] < p[1] < p[2]


def test_sdsn_is_dsn_of_the_normalised_input():
    # Algorithm 2 = the same alternating projections after X -> (theta/2) X / max X.
    rng = np.random.default_rng(3)
    X = rng.random((20, 20)) ** 2
    for theta in (1.0, 2.0, 10.0):
        D1, info = O.sdsn(X, theta, gamma_th=-2.0, max_passes=25)
        assert info.passes == 25
        np.testing.assert_allclose(D1, P.dsn((theta / 2.0) * X / X.max(), 25), rtol=0, atol=1e-15)


def test_first_outer_iteration_and_criterion():
    pr = next(synth.config_pairs(0, [0]))
    N, info = P.dspfp(pr.A, pr.B, iters=1)
    np.testing.assert_allclose(N, np.full((pr.n, pr.n), 0.95 / pr.n), rtol=0, atol=1e-15)
    assert info.criteria == [float("inf")]
    # The criterion compares max-normalised iterates: scaling N changes nothing.
    rng = np.random.default_rng(1)
    M1, M2 = rng.random((5, 5)), rng.random((5, 5))
    assert P.criterion(3.0 * M1, M2) == pytest.approx(P.criterion(M1, 0.5 * M2), abs=1e-15)
    assert P.criterion(M1, M1) == 0.0


def test_dspfp_depends_on_the_input_scale_fram_does_not():
    # The motivation of FRAM (Sec. 5.1): multiplying both graphs by w scales
    # the gradient by w^2; FRAM's max-normalisation removes it, DSPFP's plain
    # projection does not (here the projected iterates differ).
    pr = synth.make_pair(30, 0.4, 0.05, 77)
    N1, _ = P.dspfp(pr.A, pr.B, iters=5)
    N2, _ = P.dspfp(10.0 * pr.A, 10.0 * pr.B, iters=5)
    assert np.max(np.abs(N1 - N2)) > 1e-3
    F1, _ = O.fram(pr.A, pr.B, iters=5)
    F2, _ = O.fram(10.0 * pr.A, 10.0 * pr.B, iters=5)
    np.testing.assert_allclose(F1, F2, rtol=0, atol=1e-12)
