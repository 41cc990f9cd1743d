"""Pins for the explicit Hankel lifting and its adjoint (THEORY section)."""
import numpy as np
import pytest
import scipy.linalg

import oracle


def _rand(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _brute_H(x, kdims, lo, hi):
    """Element-by-element definition: row = valid output u (lexicographic),
    column = (k0, k1, k2, c) lexicographic with c fastest, entry x[u + k, c]."""
    nc = x.shape[3]
    rows = []
    for u0 in range(lo[0], hi[0] - kdims[0] + 1):
        for u1 in range(lo[1], hi[1] - kdims[1] + 1):
            for u2 in range(lo[2], hi[2] - kdims[2] + 1):
                row = []
                for k0 in range(kdims[0]):
                    for k1 in range(kdims[1]):
                        for k2 in range(kdims[2]):
                            for c in range(nc):
                                row.append(x[u0 + k0, u1 + k1, u2 + k2, c])
                rows.append(row)
    return np.array(rows)


@pytest.mark.parametrize("shape,kdims,lo,hi", [
    ((1, 7, 6, 3), (1, 3, 2), (0, 0, 0), (1, 7, 6)),
    ((4, 5, 6, 2), (2, 3, 2), (0, 0, 0), (4, 5, 6)),
    ((5, 6, 7, 2), (2, 2, 3), (1, 1, 2), (5, 5, 7)),
])
def test_hankel_matches_brute_force(shape, kdims, lo, hi):
    rng = np.random.default_rng(0)
    x = _rand(shape, rng)
    H = oracle.hankel_matrix(x, kdims, lo, hi)
    np.testing.assert_array_equal(H, _brute_H(x, kdims, lo, hi))


def test_one_dimensional_single_coil_is_scipy_hankel():
    rng = np.random.default_rng(1)
    N, K = 11, 4
    v = _rand(N, rng)
    x = v.reshape(1, 1, N, 1)
    H = oracle.hankel_matrix(x, (1, 1, K), (0, 0, 0), (1, 1, N))
    ref = scipy.linalg.hankel(v[: N - K + 1], v[N - K:])
    np.testing.assert_array_equal(H, ref)


def test_one_dimensional_multicoil_interleaves_scipy_hankel_blocks():
    rng = np.random.default_rng(2)
    N, K, nc = 9, 3, 3
    v = _rand((N, nc), rng)
    H = oracle.hankel_matrix(v.reshape(1, 1, N, nc), (1, 1, K), (0, 0, 0), (1, 1, N))
    for c in range(nc):
        ref = scipy.linalg.hankel(v[: N - K + 1, c], v[N - K:, c])
        np.testing.assert_array_equal(H[:, c::nc], ref)


def test_region_equals_crop():
    rng = np.random.default_rng(3)
    x = _rand((3, 9, 8, 2), rng)
    lo, hi, kd = (1, 2, 1), (3, 8, 7), (2, 3, 3)
    crop = x[1:3, 2:8, 1:7]
    np.testing.assert_array_equal(oracle.hankel_matrix(x, kd, lo, hi),
                                  oracle.hankel_matrix(crop, kd, (0, 0, 0), crop.shape[:3]))


def test_adjoint_brute_force_scatter():
    rng = np.random.default_rng(4)
    shape, kd, lo, hi = (2, 6, 5, 2), (1, 3, 2), (0, 1, 0), (2, 6, 5)
    m = oracle.valid_extent(lo, hi, kd)
    s, n = m[0] * m[1] * m[2], kd[0] * kd[1] * kd[2] * shape[3]
    W = _rand((s, n), rng)
    ref = np.zeros(shape, complex)
    row = 0
    for u0 in range(lo[0], hi[0] - kd[0] + 1):
        for u1 in range(lo[1], hi[1] - kd[1] + 1):
            for u2 in range(lo[2], hi[2] - kd[2] + 1):
                col = 0
                for k0 in range(kd[0]):
                    for k1 in range(kd[1]):
                        for k2 in range(kd[2]):
                            for c in range(shape[3]):
                                ref[u0 + k0, u1 + k1, u2 + k2, c] += W[row, col]
                                col += 1
                row += 1
    np.testing.assert_allclose(oracle.hankel_adjoint(W, shape, kd, lo, hi), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,kd,lo,hi,p", [
    ((1, 12, 10, 3), (1, 3, 3), (0, 0, 0), (1, 12, 10), 5),
    ((6, 7, 8, 2), (3, 2, 3), (1, 0, 2), (6, 7, 8), 4),
])
def test_adjoint_identity(shape, kd, lo, hi, p):
    """<H(x) F, Y> = <x, H'(Y F^H)> for random x, F, Y."""
    rng = np.random.default_rng(5)
    x = _rand(shape, rng)
    n = kd[0] * kd[1] * kd[2] * shape[3]
    m = oracle.valid_extent(lo, hi, kd)
    F = _rand((n, p), rng)
    Y = _rand((m[0] * m[1] * m[2], p), rng)
    lhs = np.vdot(oracle.forward(x, F, kd, lo, hi), Y)
    rhs = np.vdot(x, oracle.adjoint(Y, F, shape, kd, lo, hi))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_region_smaller_than_kernel_rejected():
    with pytest.raises(ValueError):
        oracle.valid_extent((0, 0, 0), (1, 4, 4), (1, 5, 5))


def test_pointwise_matches_explicit():
    rng = np.random.default_rng(6)
    shape, kd, lo, hi = (1, 14, 13, 3), (1, 3, 4), (0, 1, 2), (1, 14, 13)
    x = _rand(shape, rng)
    mask = (rng.random(shape[:3]) < 0.3).astype(np.uint8)
    n = kd[1] * kd[2] * 3
    F = _rand((n, 6), rng)
    _, g, _ = oracle.objective_grad(x, mask, F, kd, lo, hi)
    pts = [(0, int(a), int(b)) for a, b in zip(rng.integers(0, 14, 25), rng.integers(0, 13, 25))]
    gp = oracle.grad_at_points(x, mask, F, kd, lo, hi, pts)
    np.testing.assert_allclose(gp, np.stack([g[p] for p in pts]), rtol=0, atol=1e-12)
    upts = [(0, lo[1] + i, lo[2] + 2 * i) for i in range(4)]
    Y = oracle.forward(x, F, kd, lo, hi)
    m = oracle.valid_extent(lo, hi, kd)
    rows = [(u[1] - lo[1]) * m[2] + (u[2] - lo[2]) for u in upts]
    np.testing.assert_allclose(oracle.residual_at_points(x, F, kd, upts), Y[rows], atol=1e-12)
