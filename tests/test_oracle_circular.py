"""Pins for the circular axis of the lifting (METHODS, Study II: the
convolution along time is circular rather than valid) and for the
time-averaged initial k-space of that study."""
import numpy as np
import pytest

import oracle


def _rand(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _brute_H_circ(x, kd, wrap):
    """Loops over the definition: outputs u on every position of a circular
    axis (valid positions elsewhere), entry x[(u + k) mod N, c]."""
    D, nc = x.shape[:3], x.shape[3]
    rng_u = [range(D[a]) if wrap[a] else range(D[a] - kd[a] + 1) for a in range(3)]
    rows = []
    for u0 in rng_u[0]:
        for u1 in rng_u[1]:
            for u2 in rng_u[2]:
                row = []
                for k0 in range(kd[0]):
                    for k1 in range(kd[1]):
                        for k2 in range(kd[2]):
                            w = [(u0 + k0), (u1 + k1), (u2 + k2)]
                            w = [w[a] % D[a] if wrap[a] else w[a] for a in range(3)]
                            for c in range(nc):
                                row.append(x[w[0], w[1], w[2], c])
                rows.append(row)
    return np.array(rows)


@pytest.mark.parametrize("shape,kd,wrap", [((5, 6, 7, 2), (3, 2, 3), (True, False, False)),
                                           ((4, 5, 6, 3), (2, 3, 2), (True, False, True)),
                                           ((6, 3, 4, 1), (5, 2, 4), (True, True, True))])
def test_circular_hankel_matches_loops(shape, kd, wrap):
    x = _rand(shape, np.random.default_rng(1))
    hi = shape[:3]
    H = oracle.hankel_matrix(x, kd, (0, 0, 0), hi, wrap)
    np.testing.assert_array_equal(H, _brute_H_circ(x, kd, wrap))


def test_circular_gram_1d_is_the_autocorrelation():
    """One coil, one circular axis: G[k, k'] = sum_w conj(x[w]) x[(w + k' - k) mod N],
    the circular autocorrelation, which the FFT gives as ifft(|fft(x)|^2)."""
    N, K = 29, 7
    x = _rand((N,), np.random.default_rng(2))
    G = oracle.gram(x.reshape(1, 1, N, 1), (1, 1, K), (0, 0, 0), (1, 1, N), (False, False, True))
    R = np.fft.ifft(np.abs(np.fft.fft(x)) ** 2)
    want = np.array([[R[(kp - k) % N] for kp in range(K)] for k in range(K)])
    np.testing.assert_allclose(G, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("wrap", [(True, False, False), (False, True, True)])
def test_circular_adjoint_identity(wrap):
    rng = np.random.default_rng(3)
    shape, kd = (5, 7, 6, 2), (3, 3, 2)
    lo, hi = (0, 0, 0), shape[:3]
    x = _rand(shape, rng)
    n = kd[0] * kd[1] * kd[2] * shape[3]
    F = _rand((n, 4), rng)
    s = oracle.hankel_matrix(x, kd, lo, hi, wrap).shape[0]
    Y = _rand((s, 4), rng)
    lhs = np.vdot(Y, oracle.forward(x, F, kd, lo, hi, wrap))
    rhs = np.vdot(oracle.adjoint(Y, F, shape, kd, lo, hi, wrap), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_circular_axis_needs_the_whole_axis():
    x = _rand((6, 5, 5, 1), np.random.default_rng(4))
    with pytest.raises(ValueError):
        oracle.hankel_matrix(x, (3, 2, 2), (1, 0, 0), (6, 5, 5), (True, False, False))


def test_circular_gradient_by_finite_differences():
    rng = np.random.default_rng(5)
    shape, kd, wrap = (6, 7, 5, 2), (3, 3, 2), (True, False, False)
    lo, hi = (0, 0, 0), shape[:3]
    x = _rand(shape, rng)
    n = kd[0] * kd[1] * kd[2] * shape[3]
    F = _rand((n, 3), rng)
    J, g, _ = oracle.objective_grad(x, None, F, kd, lo, hi, wrap)
    for _ in range(10):
        d = _rand(shape, rng)
        h = 1e-3
        fd = (oracle.objective(x + h * d, F, kd, lo, hi, wrap) - oracle.objective(x - h * d, F, kd, lo, hi, wrap)) / (2 * h)
        assert abs(fd - np.vdot(g, d).real) <= 1e-8 * max(1.0, abs(fd))


def test_time_average_hand_case():
    # 3 frames x 1 x 2 locations, 1 coil: location 0 observed in frames 0 and 2,
    # location 1 in no frame
    x0 = np.zeros((3, 1, 2, 1), complex)
    mask = np.zeros((3, 1, 2), np.uint8)
    x0[0, 0, 0, 0], x0[2, 0, 0, 0] = 1 + 2j, 3 - 4j
    mask[0, 0, 0] = mask[2, 0, 0] = 1
    out = oracle.time_average_init(x0, mask, axis=0)
    assert out[0, 0, 0, 0] == 1 + 2j and out[2, 0, 0, 0] == 3 - 4j
    assert out[1, 0, 0, 0] == 2 - 1j
    assert np.all(out[:, 0, 1, 0] == 0)


def test_time_average_properties():
    rng = np.random.default_rng(6)
    x = _rand((8, 5, 6, 3), rng)
    mask = (rng.random((8, 5, 6)) < 0.3).astype(np.uint8)
    x0 = x * mask[..., None]
    for axis in (0, 1, 2):
        out = oracle.time_average_init(x0, mask, axis)
        obs = mask.astype(bool)
        np.testing.assert_array_equal(out[obs], x0[obs])
        # at unobserved samples: the mean of the location's observed frames
        idx = [slice(None)] * 3
        for loc in np.ndindex(*[s for a, s in enumerate(mask.shape) if a != axis]):
            full = list(loc)
            full.insert(axis, slice(None))
            mcol = mask[tuple(full)].astype(bool)
            xcol = x0[tuple(full)]
            ocol = out[tuple(full)]
            want = xcol[mcol].mean(axis=0) if mcol.any() else np.zeros(3)
            np.testing.assert_allclose(ocol[~mcol], np.broadcast_to(want, ocol[~mcol].shape), rtol=1e-14, atol=1e-14)
