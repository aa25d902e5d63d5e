"""FP64 oracle of the DSPFP baseline iteration (the method FRAM modifies).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the library or its binding.

The doubly stochastic projected fixed-point iteration of Sec. 4 (eq.
iter.DSPFP) has the same outer loop as FRAM (Algorithm 1), with two
differences the paper points out:

* ``dsn``   -- the doubly stochastic projection P_D (eq. 4) is approximated by
               plain alternating projections P2(P1(.)) on the gradient itself:
               no division by max(X) and no theta (the scale sensitivity of
               Sec. 5.1: P_D(wX) differs from P_D(X)), and a fixed number of
               iterations, 30 as in the cited fast projection (Sec. 5.2,
               convergence criterion paragraph).
* ``dspfp`` -- the outer stop uses DSPFP's own criterion (App. B.2):
               max |N^(t)/max N^(t) - N^(t-1)/max N^(t-1)| <= tol.

Readings where the paper is silent: the inputs are used as given (no
prescale: the gradient's scale is the point of the comparison), N^(0) = 0 as
in FRAM (so D^(1) = P_D(0) = 11^T/n), and the criterion is +inf while
N^(t-1) = 0 (its maximum is 0).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .fram64 import discretize, objective, p1, p2


def dsn(X: np.ndarray, iters: int = 30) -> np.ndarray:
    """``iters`` alternating projections Y <- P2(P1(Y)) from Y = X (Sec. 4,
    eq. 4 approximated as in the fast projection the paper cites)."""
    Y = np.asarray(X, dtype=np.float64)
    for _ in range(iters):
        Y = p2(p1(Y))
    return Y


@dataclasses.dataclass
class DspfpInfo:
    outer_iters: int
    criteria: list
    converged: bool


def criterion(N_new: np.ndarray, N_old: np.ndarray) -> float:
    """max |N_new/max(N_new) - N_old/max(N_old)| (App. B.2); +inf while a
    maximum is not positive."""
    m_new, m_old = float(N_new.max()), float(N_old.max())
    if m_new <= 0.0 or m_old <= 0.0:
        return float("inf")
    return float(np.max(np.abs(N_new / m_new - N_old / m_old)))


def dspfp(A: np.ndarray, B: np.ndarray, alpha: float = 0.95, iters: int = 100,
          tol: float = 0.0, dsn_iters: int = 30):
    """The DSPFP outer loop: X = A N B, D = dsn(X), N <- (1 - alpha) N + alpha D,
    until the max-abs criterion <= tol or ``iters`` iterations.  Returns
    (N, DspfpInfo)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[0]
    N = np.zeros((n, n))
    crits = []
    converged = False
    t = 0
    while True:
        D = dsn(A @ N @ B, dsn_iters)
        N_new = (1.0 - alpha) * N + alpha * D
        c = criterion(N_new, N)
        N = N_new
        t += 1
        crits.append(c)
        if c <= tol:
            converged = True
            break
        if t >= iters:
            break
    return N, DspfpInfo(outer_iters=t, criteria=crits, converged=converged)


def solve(A: np.ndarray, B: np.ndarray, alpha: float = 0.95, iters: int = 100,
          tol: float = 0.0, dsn_iters: int = 30):
    """DSPFP with the exact discretisation of eq. (2); returns
    (sigma, objective, N, DspfpInfo)."""
    N, info = dspfp(A, B, alpha, iters, tol, dsn_iters)
    sigma = discretize(N)
    return sigma, objective(A, B, sigma), N, info
