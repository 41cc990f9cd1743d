"""Pins for kernel masks (THEORY: the {0,1} kernel mask K gives the support
of the annihilating kernels; DISCUSSION: circular or spherical supports).
The lifting with a mask takes only the taps inside K."""
import itertools

import numpy as np
import pytest

import oracle


def _rand(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def disc(K):
    """Taps of a K x K box within the inscribed circle (centre distance <= K/2)."""
    c = (K - 1) / 2.0
    a = np.arange(K)
    return ((a[:, None] - c) ** 2 + (a[None, :] - c) ** 2 <= (K / 2.0) ** 2)[None]


def ball(K):
    c = (K - 1) / 2.0
    a = np.arange(K)
    return (a[:, None, None] - c) ** 2 + (a[None, :, None] - c) ** 2 + (a[None, None, :] - c) ** 2 <= (K / 2.0) ** 2


def _brute(x, mask, lo, hi):
    K = mask.shape
    nc = x.shape[3]
    rows = []
    for u in itertools.product(*[range(lo[a], hi[a] - K[a] + 1) for a in range(3)]):
        row = []
        for k in itertools.product(*[range(K[a]) for a in range(3)]):
            if mask[k]:
                for c in range(nc):
                    row.append(x[u[0] + k[0], u[1] + k[1], u[2] + k[2], c])
        rows.append(row)
    return np.array(rows)


@pytest.mark.parametrize("mask,shape,lo,hi", [(disc(5), (1, 9, 8, 2), (0, 0, 0), (1, 9, 8)),
                                              (ball(3), (5, 6, 5, 2), (1, 0, 0), (5, 6, 5))])
def test_masked_hankel_matches_loops(mask, shape, lo, hi):
    x = _rand(shape, np.random.default_rng(1))
    H = oracle.hankel_matrix(x, mask, lo, hi)
    np.testing.assert_array_equal(H, _brute(x, mask, lo, hi))
    assert H.shape[1] == int(mask.sum()) * shape[3]


def test_masked_gram_is_principal_submatrix_of_box_gram():
    rng = np.random.default_rng(2)
    x = _rand((1, 14, 12, 3), rng)
    mask = disc(5)
    sel = np.repeat(np.flatnonzero(mask.reshape(-1)) * 3, 3) + np.tile(np.arange(3), int(mask.sum()))
    G = oracle.gram(x, mask, (0, 0, 0), (1, 14, 12))
    Gf = oracle.gram(x, (1, 5, 5), (0, 0, 0), (1, 14, 12))
    np.testing.assert_allclose(G, Gf[np.ix_(sel, sel)], rtol=1e-12, atol=1e-12)


def test_masked_adjoint_identity_and_gradient():
    rng = np.random.default_rng(3)
    shape, mask = (5, 7, 6, 2), ball(3)
    lo, hi = (0, 0, 0), shape[:3]
    x = _rand(shape, rng)
    n = int(mask.sum()) * shape[3]
    F = _rand((n, 3), rng)
    s = oracle.hankel_matrix(x, mask, lo, hi).shape[0]
    Y = _rand((s, 3), rng)
    lhs = np.vdot(Y, oracle.forward(x, F, mask, lo, hi))
    rhs = np.vdot(oracle.adjoint(Y, F, shape, mask, lo, hi), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    J, g, _ = oracle.objective_grad(x, None, F, mask, lo, hi)
    for _ in range(8):
        d = _rand(shape, rng)
        h = 1e-3
        fd = (oracle.objective(x + h * d, F, mask, lo, hi) - oracle.objective(x - h * d, F, mask, lo, hi)) / (2 * h)
        assert abs(fd - np.vdot(g, d).real) <= 1e-8 * max(1.0, abs(fd))
