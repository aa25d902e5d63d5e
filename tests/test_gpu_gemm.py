"""GPU parity of the MFMA GEMMs of the gradient X = A N B (Algorithm 1, step 5).

Two kinds of checks through fram_gradient (C ABI):
* integer-exact inputs, where every product and partial sum is an integer far
  below 2^24, so every input type and the FP32 accumulation are exact and the
  result must equal the FP64 product bit for bit (this catches any lane,
  swizzle or tile-layout mistake);
* random inputs against the FP64 product of the same rounded inputs, within a
  bound derived from the rounding of W and FP32 accumulation.
Sizes cover a single tile, exact tile multiples and ragged tails for the
64/128/256 tile variants.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


def round_to(x, prec):
    x = np.asarray(x, dtype=np.float32)
    if prec == "fp32":
        return x.astype(np.float64)
    if prec == "fp16":
        return x.astype(np.float16).astype(np.float64)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def sym_int(rng, n, hi):
    A = np.triu(rng.integers(0, hi + 1, size=(n, n)), 1).astype(np.float64)
    return A + A.T


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("n", [1, 2, 33, 64, 65, 130, 256, 300, 1000, 1500, 4000])
def test_gradient_integer_exact(ctx, n, prec):
    rng = np.random.default_rng(n)
    A = sym_int(rng, n, 2)
    B = sym_int(rng, n, 2)
    N = np.eye(n)[rng.permutation(n)]
    if n > 2:
        N[0] = 0.0
        N[0, :3] = [0.5, 0.25, 0.25]  # dyadic fractions stay exact
    X = ctx.gradient(A, N, B, prec)
    np.testing.assert_array_equal(X.astype(np.float64), A @ N @ B)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("n", [50, 129, 257, 1000])
def test_gradient_random_within_rounding_bound(ctx, n, prec):
    rng = np.random.default_rng(1000 + n)
    A = np.triu(rng.random((n, n)), 1)
    A = A + A.T
    B = np.triu(rng.random((n, n)) * (rng.random((n, n)) < 0.4), 1)
    B = B + B.T
    N = rng.random((n, n)) ** 4
    N /= N.sum(1, keepdims=True)
    X = ctx.gradient(A, N, B, prec).astype(np.float64)
    Ar, Br, Nr = round_to(A, prec), round_to(B, prec), round_to(N, prec)
    W = Br @ Nr.T
    Wr = round_to(W, prec)
    ref = Ar @ Wr.T
    g = n * 2.0 ** -24
    e1 = g * (np.abs(Br) @ np.abs(Nr).T)
    bound = np.abs(Ar) @ (e1 + 2 * UNIT[prec] * np.abs(W)).T + g * (np.abs(Ar) @ np.abs(Wr).T)
    err = np.abs(X - ref)
    assert (err <= 2 * bound + 1e-30).all(), float((err / (bound + 1e-30)).max())
    # Against the unrounded FP64 product: input rounding (a few units of the
    # input type) plus the worst-case FP32 accumulation bound n * 2^-24.
    rel = np.abs(X - A @ N @ B).max() / np.abs(A @ N @ B).max()
    assert rel < 8 * UNIT[prec] + 2 * n * 2.0 ** -24
