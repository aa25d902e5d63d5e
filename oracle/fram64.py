"""FP64 oracle of FRAM (Frobenius-Regularized Assignment Matching).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the library or its binding.

Every function follows the paper's algorithms in their order and notation:

* ``prescale``   -- Algorithm 1, steps 2-3 (global max c, divide A, A~ by sqrt(c)
                    and the node similarities K by c).
* ``p1``         -- the affine projection P1 onto {Y1 = 1, Y^T 1 = 1}, eq. (P1_sol)
                    in Sec. 5.1 (proved for asymmetric X in Theorem 5, App. D).
* ``p2``         -- the nonnegativity projection P2(X) = (X + |X|)/2, Sec. 5.1.
* ``p3``         -- the zero-sum projection of the truncation lemma (App. D).
* ``sdsn``       -- Algorithm 2 (SDSN) with the stopping measure gamma of Sec. 5.2
                    and App. B.1.
* ``fram``       -- Algorithm 1 (FRAM), outer fixed-point loop of eq. (3) with the
                    normalized Frobenius criterion delta of App. B.2.
* ``discretize`` -- Algorithm 1 step 10 / eq. (2): the linear assignment
                    M = argmin_P ||P - N||_F, i.e. argmax_P <P, N>, by an exact LAP
                    solver (scipy's linear_sum_assignment).
* ``objective``  -- twice Phi(M) of eq. (1): sum_{k,l} A_kl B_{s(k) s(l)}
                    = tr(A M B M^T), plus 2 lam <M, K> with node similarities,
                    on the unscaled input.

Readings of points where the paper is silent or ambiguous (each one is also
listed with its justification in the design notes):

* Initialisation: N^(0) = 0 (Alg. 1 step 1).  With no node term the first
  gradient is the zero matrix; SDSN of a matrix whose max is <= 0 starts from
  the zero matrix, and P1(0) = 11^T/n, so D^(1) = 11^T/n.
* "lambda" at the library boundary is the SDSN strength theta; the node-term
  weight is ``lam`` and multiplies K = F F~^T (optional; n = n~ only, the
  paper's own simplification in Sec. 3).
* gamma is evaluated on each pass output (Sec. 5.2 definition), at least one
  pass is made, and the loop stops when gamma <= gamma_th or at a pass cap.
* The outer loop is a do-while: stop when delta <= tol or after ``iters``
  iterations; tol = 0 runs exactly ``iters`` iterations.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.optimize import linear_sum_assignment


# ---------------------------------------------------------------- Alg. 1, steps 2-3
def prescale(A: np.ndarray, B: np.ndarray, K: np.ndarray | None = None):
    """c = max(A, A~, K), then A/sqrt(c), A~/sqrt(c), K/c -- Alg. 1 steps 2-3.

    Returns (A/sqrt(c), A~/sqrt(c), c) without K, (A/sqrt(c), A~/sqrt(c), K/c, c)
    with it.  A non-positive c leaves the inputs unscaled."""
    c = max(float(A.max()), float(B.max()))
    if K is not None:
        c = max(c, float(np.max(K)))
    if c <= 0.0:
        out = (A.astype(np.float64).copy(), B.astype(np.float64).copy())
        return (*out, c) if K is None else (*out, np.asarray(K, dtype=np.float64).copy(), c)
    s = math.sqrt(c)
    if K is None:
        return A / s, B / s, c
    return A / s, B / s, np.asarray(K, dtype=np.float64) / c, c


# ---------------------------------------------------------------- Sec. 5.1 projections
def p1(X: np.ndarray) -> np.ndarray:
    """P1(X) = X + (I/n + (1^T X 1/n^2) I - X/n) 1 1^T - 1 1^T X / n   (eq. P1_sol).

    The product (M) 1 1^T is formed as (M 1) 1^T, which is the same matrix:
    M 1 = 1/n + (1^T X 1/n^2) 1 - (X 1)/n.
    """
    n = X.shape[0]
    one = np.ones(n)
    xbar = one @ X @ one / n**2
    left = one / n + xbar * one - (X @ one) / n          # (I/n + xbar I - X/n) 1
    return X + np.outer(left, one) - np.outer(one, one @ X) / n


def p2(X: np.ndarray) -> np.ndarray:
    """P2(X) = (X + |X|)/2, the projection onto the nonnegative orthant (Sec. 5.1)."""
    return (X + np.abs(X)) / 2.0


def p3(X: np.ndarray) -> np.ndarray:
    """P3(X) = X + (1^T X 1/n^2 - X/n) 1 1^T - 1 1^T X/n, projection onto
    {Y1 = 0, Y^T 1 = 0} (truncation lemma, App. D)."""
    n = X.shape[0]
    one = np.ones(n)
    xbar = one @ X @ one / n**2
    left = xbar * one - (X @ one) / n
    return X + np.outer(left, one) - np.outer(one, one @ X) / n


# ---------------------------------------------------------------- Alg. 2: SDSN
@dataclasses.dataclass
class SdsnInfo:
    passes: int
    gamma: float
    capped: bool
    gammas: list


def sdsn(X: np.ndarray, theta: float, gamma_th: float = 1e-6, max_passes: int = 1000,
         min_passes: int = 1):
    """Scaling Doubly Stochastic Normalization, Algorithm 2.

    X^(0) = (theta/2) X / max(X); then repeat X <- P2(P1(X)) and
    gamma = 1^T X 1 / n - 1 until gamma <= gamma_th (or the pass cap).
    A matrix with max <= 0 is treated as the zero matrix (0/0 read as 0).
    Returns (D, SdsnInfo).
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    m = float(X.max())
    Y = np.zeros_like(X) if m <= 0.0 else (theta / 2.0) * X / m
    gammas = []
    k = 0
    while True:
        Y = p2(p1(Y))
        k += 1
        gamma = float(Y.sum()) / n - 1.0
        gammas.append(gamma)
        if k >= min_passes and (gamma <= gamma_th or k >= max_passes):
            break
    return Y, SdsnInfo(passes=k, gamma=gamma, capped=(gamma > gamma_th), gammas=gammas)


# ---------------------------------------------------------------- Alg. 1: FRAM
@dataclasses.dataclass
class FramInfo:
    outer_iters: int
    sdsn_passes: list
    deltas: list
    gammas: list
    converged: bool
    sdsn_capped: bool


def stall_step(count: int, dmin: float | None, delta: float, stall_delta: float):
    """One iteration of the delta-stall stop (not in the paper): once delta has
    fallen to stall_delta, count consecutive iterations whose delta is not
    below the smallest delta seen since then; a new minimum resets the count.
    Returns the new (count, dmin); the loop stops when count reaches the
    window.  While delta decreases (at any rate) nothing is counted; at the
    floor set by the arithmetic's precision delta only fluctuates, and the
    count soon runs up.  Above stall_delta nothing is counted, so the early
    phase, where delta need not decrease, never stops the loop."""
    if delta > stall_delta:
        return count, dmin
    count = count + 1 if (dmin is not None and delta >= dmin) else 0
    dmin = delta if dmin is None else min(dmin, delta)
    return count, dmin


def fram(A: np.ndarray, B: np.ndarray, theta: float = 2.0, alpha: float = 0.95,
         iters: int = 100, tol: float = 0.0, gamma_th: float = 1e-6,
         sdsn_max: int = 1000, N0: np.ndarray | None = None, stable_iters: int = 0,
         K: np.ndarray | None = None, lam: float = 1.0, stall_iters: int = 0,
         stall_delta: float = 1e-3):
    """Algorithm 1 up to (not including) the discretisation of step 10.

    Returns (N, FramInfo).  A and B are the *unscaled* inputs.  K (n x n) is
    the node-similarity matrix F F~^T of eq. (1), weighted by lam in the
    gradient of eq. (3) (step 5: X = A N A~ + lam K); None means no node term.

    stable_iters = w > 0 adds a second stop (not in the paper, whose delta_th
    is unspecified): stop once the row argmax of N (lowest column on ties)
    has been the same permutation after w consecutive iterations; the loop
    then stops at the first t where argmax(N^(t)) = argmax(N^(t-1)) = ... =
    argmax(N^(t-w)).  A row argmax that is not a permutation never counts.

    stall_iters = w > 0 adds a third stop (not in the paper): delta has reached
    the floor set by the arithmetic's precision (stall_step); meant for
    low-precision gradients whose delta levels off above tol.  In FP64 the
    floor is far below any useful tol.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if K is None:
        As, Bs, _ = prescale(A, B)
        Ks = None
    else:
        As, Bs, Ks, _ = prescale(A, B, np.asarray(K, dtype=np.float64))
    n = A.shape[0]
    N = np.zeros((n, n)) if N0 is None else np.array(N0, dtype=np.float64)
    passes, deltas, gammas = [], [], []
    converged, capped = False, False
    t = 0
    prev_arg, same = None, 0
    stall, dmin = 0, None
    while True:
        X = As @ N @ Bs                                       # step 5
        if Ks is not None:
            X = X + lam * Ks
        D, info = sdsn(X, theta, gamma_th, sdsn_max)           # step 6
        N_new = (1.0 - alpha) * N + alpha * D                  # step 7
        num = np.linalg.norm(N_new - N)                        # step 8
        den = np.linalg.norm(N_new)
        delta = num / den if den > 0 else 0.0
        N = N_new
        t += 1
        passes.append(info.passes)
        gammas.append(info.gamma)
        deltas.append(delta)
        capped = capped or info.capped
        if delta <= tol:
            converged = True
            break
        if stall_iters > 0:
            stall, dmin = stall_step(stall, dmin, delta, stall_delta)
            if stall >= stall_iters:
                converged = True
                break
        if stable_iters > 0:
            arg = np.argmax(N, axis=1)
            is_perm = len(np.unique(arg)) == n
            same = same + 1 if (is_perm and prev_arg is not None
                                and np.array_equal(arg, prev_arg)) else 0
            prev_arg = arg if is_perm else None
            if same >= stable_iters:
                converged = True
                break
        if t >= iters:
            break
    return N, FramInfo(outer_iters=t, sdsn_passes=passes, deltas=deltas, gammas=gammas,
                       converged=converged, sdsn_capped=capped)


# ---------------------------------------------------------------- step 10 and scoring
def discretize(N: np.ndarray) -> np.ndarray:
    """M = argmin_{P in Pi} ||P - N||_F = argmax_P <P, N> (eq. 2) by an exact LAP.
    Returns sigma with sigma[i] = column matched to row i."""
    rows, cols = linear_sum_assignment(np.asarray(N, dtype=np.float64), maximize=True)
    sigma = np.empty(N.shape[0], dtype=np.int64)
    sigma[rows] = cols
    return sigma


def objective(A: np.ndarray, B: np.ndarray, sigma: np.ndarray, K: np.ndarray | None = None,
              lam: float = 1.0) -> float:
    """Twice Phi(M) of eq. (1) on the unscaled inputs, M the permutation sigma:
    sum_{k,l} A_kl B_{sigma(k) sigma(l)} (= tr(A M B M^T)) plus, with node
    similarities K, 2 lam sum_k K_{k, sigma(k)} (= 2 lam <M, K>)."""
    sigma = np.asarray(sigma)
    edge = float(np.sum(np.asarray(A, dtype=np.float64) *
                        np.asarray(B, dtype=np.float64)[np.ix_(sigma, sigma)]))
    if K is None:
        return edge
    node = float(np.sum(np.asarray(K, dtype=np.float64)[np.arange(len(sigma)), sigma]))
    return edge + 2.0 * lam * node


def accuracy(sigma: np.ndarray, perm: np.ndarray, inlier: np.ndarray | None = None) -> float:
    """n_c / n over the inlier nodes (Sec. 7, Criteria)."""
    ok = np.asarray(sigma) == np.asarray(perm)
    if inlier is not None:
        ok = ok[np.asarray(inlier)]
    return float(ok.mean()) if ok.size else 1.0


def solve(A: np.ndarray, B: np.ndarray, theta: float = 2.0, alpha: float = 0.95,
          iters: int = 100, tol: float = 0.0, gamma_th: float = 1e-6, sdsn_max: int = 1000,
          stable_iters: int = 0, K: np.ndarray | None = None, lam: float = 1.0,
          stall_iters: int = 0, stall_delta: float = 1e-3):
    """Full FRAM: Algorithm 1 including step 10; returns (sigma, objective, N, FramInfo)."""
    N, info = fram(A, B, theta, alpha, iters, tol, gamma_th, sdsn_max, stable_iters=stable_iters,
                   K=K, lam=lam, stall_iters=stall_iters, stall_delta=stall_delta)
    sigma = discretize(N)
    return sigma, objective(A, B, sigma, K, lam), N, info
