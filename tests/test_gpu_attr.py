"""GPU parity of FRAM with node similarities (eq. 1, eq. 3: X = A N A~ + lam K)
through fram_solve_attr_ex / fram_solve_attr_dev against the FP64 oracle.

* FP32 GEMMs return the oracle's permutation, relative objective error <= 1e-5.
* Edgeless graphs (the node term alone) and a permutation-matrix node term
  give the oracle's / the closed-form assignment.
* Noiseless attributed pairs reach the certified optimum ||A||^2 + 2 lam ||F||^2
  with BF16 GEMMs too.
* lam = 0 is the plain solve, bitwise.
"""
import numpy as np
import pytest

import synth
from oracle import fram64 as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", range(8))
def test_small_attributed_fp32_equals_oracle(ctx, seed):
    pr = synth.make_attributed_pair(50, 0.2, 0.02, 9000 + seed, weights="half_open_top")
    s_or, obj_or, _, _ = O.solve(pr.A, pr.B, iters=100, K=pr.K, lam=1.0)
    perm, obj, st = ctx.solve(pr.A, pr.B, iters=100, tol=0.0, prec="fp32", K=pr.K,
                              node_weight=1.0)
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert st["outer_iters"] == 100


@pytest.mark.parametrize("n,lam", [(300, 1.0), (257, 0.3)])
def test_attributed_fp32_equals_oracle(ctx, n, lam):
    pr = synth.make_attributed_pair(n, 0.3, 0.05, 9100 + n)
    s_or, obj_or, _, _ = O.solve(pr.A, pr.B, iters=40, K=pr.K, lam=lam)
    perm, obj, _ = ctx.solve(pr.A, pr.B, iters=40, tol=0.0, prec="fp32", K=pr.K,
                             node_weight=lam)
    np.testing.assert_array_equal(perm, s_or)
    assert abs(obj - obj_or) <= 1e-5 * abs(obj_or)
    assert obj == pytest.approx(O.objective(pr.A, pr.B, perm, pr.K, lam), rel=1e-12)


def test_edgeless_graphs_use_the_node_term_alone(ctx):
    rng = np.random.default_rng(5)
    n = 120
    K = rng.random((n, n)) ** 3
    Z = np.zeros((n, n))
    s_or, obj_or, _, _ = O.solve(Z, Z, iters=10, K=K, lam=0.5)
    perm, obj, _ = ctx.solve(Z, Z, iters=10, tol=0.0, prec="fp32", K=K, node_weight=0.5)
    np.testing.assert_array_equal(perm, s_or)
    assert obj == pytest.approx(obj_or, rel=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_permutation_node_term_is_recovered(ctx, prec):
    n = 200
    perm_true = np.random.default_rng(2).permutation(n)
    K = np.zeros((n, n))
    K[np.arange(n), perm_true] = 1.0
    pr = next(synth.config_pairs(0, [1], n_override=n))
    # Weak random edges plus a strong exact node term.
    perm, _, _ = ctx.solve(0.01 * pr.A, 0.01 * pr.A, iters=30, tol=0.0, prec=prec, K=K,
                           node_weight=1.0)
    np.testing.assert_array_equal(perm, perm_true)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_noiseless_attributed_pair_reaches_certified_optimum(ctx, prec):
    pr = synth.make_attributed_pair(1000, 0.3, 0.0, 9200, feat_sigma=0.0)
    perm, obj, _ = ctx.solve(pr.A, pr.B, iters=60, tol=1e-6, prec=prec, K=pr.K,
                             node_weight=1.0, stable_iters=3)
    np.testing.assert_array_equal(perm, pr.perm)
    bound = float(np.sum(pr.A ** 2)) + 2.0 * float(np.sum(pr.K[np.arange(1000), pr.perm]))
    assert obj == pytest.approx(bound, rel=1e-12)


def test_zero_node_weight_is_the_plain_solve(ctx):
    pr = synth.make_attributed_pair(300, 0.3, 0.05, 9300)
    p0, o0, s0 = ctx.solve(pr.A, pr.B, iters=30, tol=0.0, prec="bf16")
    p1, o1, s1 = ctx.solve(pr.A, pr.B, iters=30, tol=0.0, prec="bf16", K=pr.K, node_weight=0.0)
    np.testing.assert_array_equal(p0, p1)
    assert o0 == o1 and s0["sdsn_passes"] == s1["sdsn_passes"]


def test_attributed_dev_entry_equals_host_entry(ctx):
    import torch
    pr = synth.make_attributed_pair(400, 0.3, 0.05, 9400)
    ph, oh, _ = ctx.solve(pr.A, pr.B, iters=25, tol=0.0, prec="bf16", K=pr.K, node_weight=1.0)
    dA, dB, dK = (torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in (pr.A, pr.B, pr.K))
    pd, od, _ = ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), 400, iters=25, tol=0.0, prec="bf16",
                              dK=dK.data_ptr(), node_weight=1.0,
                              stream=torch.cuda.current_stream().cuda_stream)
    np.testing.assert_array_equal(ph, pd)
    assert oh == od
