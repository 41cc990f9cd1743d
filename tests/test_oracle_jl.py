"""Pins for the JL compression (THEORY section, second numerical technique;
Algorithm 1, JL step): P has i.i.d. N(0, 1/p) entries, so E[P P^T] = I and
the compressed filters keep the mean gradient."""
import numpy as np
import pytest
import scipy.stats

import oracle
import synth


def test_normals_are_standard_normal():
    z = oracle.philox_normals(200_000, seed=123, i=0, j=0)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # the four Box-Muller outputs of a block are uncorrelated
    b = z[: (len(z) // 4) * 4].reshape(-1, 4)
    c = np.corrcoef(b.T)
    assert np.abs(c - np.eye(4)).max() < 0.02


def test_streams_differ_and_are_reproducible():
    a = oracle.philox_normals(4096, 7, 1, 2)
    assert np.array_equal(a, oracle.philox_normals(4096, 7, 1, 2))
    for other in (oracle.philox_normals(4096, 7, 1, 3), oracle.philox_normals(4096, 7, 2, 2),
                  oracle.philox_normals(4096, 8, 1, 2), oracle.philox_normals(4096, 7, 1, 2, stream=1)):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.06


def test_philox_avalanche():
    """Flipping one counter or key bit flips about half of the 128 output bits."""
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, (512, 4), dtype=np.uint64)
    base = oracle.philox4x32_10(ctr, (0x12345678, 0x9ABCDEF0))
    flips = []
    for bit in range(0, 32, 5):
        c2 = ctr.copy()
        c2[:, 0] ^= np.uint64(1 << bit)
        out = oracle.philox4x32_10(c2, (0x12345678, 0x9ABCDEF0))
        x = (base ^ out).astype(np.uint64)
        flips.append(np.unpackbits(x.astype(">u4").view(np.uint8)).mean())
    out = oracle.philox4x32_10(ctr, (0x12345679, 0x9ABCDEF0))
    flips.append(np.unpackbits((base ^ out).astype(">u4").view(np.uint8)).mean())
    assert all(0.47 < f < 0.53 for f in flips)


def test_jl_matrix_scale():
    P = oracle.jl_matrix(3, 0, 0, 300, 16)
    assert P.shape == (300, 16)
    assert P.var() * 16 == pytest.approx(1.0, rel=0.05)


def test_jl_keeps_mean_projector_and_gradient():
    """E[Q P P^T Q'] = Q Q' and, since the gradient is linear in F F^H, the
    average JL gradient converges to the full-nullspace gradient."""
    Pb = synth.make_problem("gradcheck_48x48x4")
    lo, hi, _ = Pb["schedule"][0]
    kd, x, mask = Pb["kdims"], Pb["x0"], Pb["mask"]
    Q, _, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), Pb["rank"])
    p, T = 4, 3000
    acc = np.zeros((Q.shape[0], Q.shape[0]), complex)
    for j in range(T):
        F = Q @ oracle.jl_matrix(5, 0, j, Q.shape[1], p)
        acc += F @ F.conj().T
    acc /= T
    proj = Q @ Q.conj().T
    assert np.linalg.norm(acc - proj) / np.linalg.norm(proj) < 0.05
    _, g_full, _ = oracle.objective_grad(x, mask, Q, kd, lo, hi)
    g_mean = np.zeros_like(g_full)
    T2 = 400
    for j in range(T2):
        F = Q @ oracle.jl_matrix(6, 0, j, Q.shape[1], p)
        g_mean += oracle.objective_grad(x, mask, F, kd, lo, hi)[1]
    g_mean /= T2
    assert np.linalg.norm(g_mean - g_full) / np.linalg.norm(g_full) < 0.15
