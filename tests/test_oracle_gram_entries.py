"""Pins of oracle.gram_entries (Gram of the Hankel matrix on a region,
entry by entry): pure-Python loops over the definition
G[(k,c),(k',c')] = sum over valid u of conj(x[u+k,c]) x[u+k',c'] on tiny
inputs, and agreement with the explicit H'H on a larger one."""
import itertools

import numpy as np
import pytest

import oracle


def _brute(x, kd, lo, hi, i, j):
    nc = x.shape[3]
    taps = list(itertools.product(range(kd[0]), range(kd[1]), range(kd[2])))
    (k, c), (kp, cp) = (taps[i // nc], i % nc), (taps[j // nc], j % nc)
    tot = 0j
    for u0 in range(lo[0], hi[0] - kd[0] + 1):
        for u1 in range(lo[1], hi[1] - kd[1] + 1):
            for u2 in range(lo[2], hi[2] - kd[2] + 1):
                a = x[u0 + k[0], u1 + k[1], u2 + k[2], c]
                b = x[u0 + kp[0], u1 + kp[1], u2 + kp[2], cp]
                tot += a.conjugate() * b
    return tot


@pytest.mark.parametrize("shape,kd,lo,hi", [((1, 7, 6, 2), (1, 3, 2), (0, 1, 0), (1, 7, 6)),
                                            ((4, 5, 6, 3), (2, 3, 2), (1, 0, 1), (4, 5, 6))])
def test_entries_match_loops(shape, kd, lo, hi):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    n = kd[0] * kd[1] * kd[2] * shape[3]
    pairs = [(i, j) for i in range(n) for j in range(n)]
    got = oracle.gram_entries(x, kd, lo, hi, pairs)
    want = np.array([_brute(x, kd, lo, hi, i, j) for i, j in pairs])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_entries_match_explicit_gram():
    rng = np.random.default_rng(8)
    shape, kd, lo, hi = (6, 9, 8, 2), (3, 3, 2), (1, 0, 1), (6, 9, 8)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    G = oracle.gram(x, kd, lo, hi)
    n = G.shape[0]
    pairs = [(int(i), int(j)) for i, j in zip(rng.integers(0, n, 200), rng.integers(0, n, 200))]
    got = oracle.gram_entries(x, kd, lo, hi, pairs)
    np.testing.assert_allclose(got, [G[i, j] for i, j in pairs], rtol=1e-12, atol=1e-12)
