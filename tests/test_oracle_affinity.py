"""Pins of the FP64 inpainting affinity (Eq. 6) against facts it must satisfy."""
import math

import numpy as np

from oracle import affinity as oaff


def _rand(seed, b, p, q, d, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, (b, p, d)), rng.normal(0, scale, (b, q, d))


def test_rows_are_distributions_over_the_source_anchors():
    xt, xs = _rand(1, 3, 5, 7, 6)
    a = oaff.affinity(xt, xs)
    assert a.shape == (3, 5, 7)
    np.testing.assert_allclose(a.sum(axis=2), 1.0, atol=1e-14)
    assert (a > 0).all()
    # columns are not normalised (the softmax runs over source anchors)
    assert not np.allclose(a.sum(axis=1), 1.0)


def test_two_source_anchors_reduce_to_a_logistic():
    # one target row t, source rows s0, s1: A[0] = sigma(t.s0 - t.s1)
    t = np.array([[0.5, -1.0, 2.0]])
    s = np.array([[1.0, 0.0, 0.5], [-0.5, 1.0, 0.25]])
    a = oaff.affinity(t[None], s[None])[0, 0]
    d = float(t[0] @ s[0] - t[0] @ s[1])
    assert math.isclose(a[0], 1.0 / (1.0 + math.exp(-d)), rel_tol=1e-14)
    assert math.isclose(a[1], 1.0 / (1.0 + math.exp(d)), rel_tol=1e-14)


def test_brute_force_on_a_tiny_case():
    xt, xs = _rand(2, 2, 3, 4, 5, scale=1.0)
    a = oaff.affinity(xt, xs)
    for b in range(2):
        for i in range(3):
            z = [sum(xt[b, i, k] * xs[b, j, k] for k in range(5)) for j in range(4)]
            e = [math.exp(v) for v in z]
            for j in range(4):
                assert math.isclose(a[b, i, j], e[j] / sum(e), rel_tol=1e-12)


def test_invariant_to_a_common_source_shift_and_equivariant_to_source_order():
    xt, xs = _rand(3, 1, 4, 6, 8)
    a = oaff.affinity(xt, xs)
    # adding c to every source row adds t.c to a whole row of logits
    c = np.random.default_rng(9).normal(0, 1, 8)
    np.testing.assert_allclose(oaff.affinity(xt, xs + c), a, atol=1e-13)
    perm = np.random.default_rng(4).permutation(6)
    np.testing.assert_allclose(oaff.affinity(xt, xs[:, perm]), a[:, :, perm], atol=1e-15)


def test_large_logits_stay_finite_and_identical_rows_give_uniform_rows():
    xt = np.full((1, 2, 4), 30.0)
    xs = np.full((1, 3, 4), 30.0)  # logits 3600 each: exp overflows without the max shift
    a = oaff.affinity(xt, xs)
    np.testing.assert_allclose(a, 1.0 / 3.0, atol=1e-15)
    assert oaff.affinity(xt, np.zeros((1, 0, 4))).shape == (1, 2, 0)
