"""The seeded input generator keeps the conventions both sides rely on."""
import numpy as np

import synth


def test_noiseless_copy_relation_and_symmetry():
    pr = synth.make_pair(25, 0.4, 0.0, 3)
    A, B, perm = pr.A, pr.B, pr.perm
    np.testing.assert_array_equal(B[np.ix_(perm, perm)], A)
    for M in (A, B):
        assert (M == M.T).all() and (M >= 0).all() and (np.diag(M) == 0).all()


def test_noise_deletions_outliers():
    n = 200
    pr = synth.make_pair(n, 0.5, 0.05, 1001, delete_frac=0.05)
    A, B, perm = pr.A, pr.B, pr.perm
    assert (B == B.T).all() and (B >= 0).all() and (np.diag(B) == 0).all()
    Bp = B[np.ix_(perm, perm)]
    # No edge created where A had none; about 5% of A's edges deleted.
    assert ((A == 0) <= (Bp == 0)).all()
    lost = ((A > 0) & (Bp == 0)).sum() / (A > 0).sum()
    assert 0.05 < lost < 0.09  # 5% deleted plus edges the noise clipped to 0
    pr2 = synth.make_pair(n, 0.3, 0.05, 2001, outlier_frac=0.1)
    assert pr2.inlier.sum() == n - 20
    assert (pr2.B == pr2.B.T).all()


def test_seeds_are_reproducible_and_distinct():
    a = next(synth.config_pairs(0, [3]))
    b = next(synth.config_pairs(0, [3]))
    c = next(synth.config_pairs(0, [4]))
    np.testing.assert_array_equal(a.A, b.A)
    assert a.seed == 3 and not np.array_equal(a.A, c.A)


def test_batched_and_served_workloads():
    pairs = synth.batched_pairs(count=16)
    assert all(20 <= p.n <= 300 for p in pairs)
    reqs = synth.serve_requests(duration_s=2.0, warmup_s=0.5)
    ts = [r[0] for r in reqs]
    assert ts == sorted(ts) and all(30 <= r[1] <= 2000 for r in reqs)
    assert 200 < len(reqs) < 800  # ~200 req/s over 2.5 s
