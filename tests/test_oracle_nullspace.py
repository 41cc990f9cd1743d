"""Pins for the Gram matrix and the nullspace (THEORY section, Eq. 1, Eq. 2)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_tiny_worked_example():
    """Hand-derived 1-D case: x = [1, 2, 3], kernel 2, rank 1."""
    gold = json.load(open(os.path.join(GOLDEN, "tiny_hankel_1d.json")))
    x = np.array(gold["x"], complex).reshape(1, 1, 3, 1)
    kd, lo, hi = (1, 1, gold["kernel"]), (0, 0, 0), (1, 1, 3)
    np.testing.assert_array_equal(oracle.hankel_matrix(x, kd, lo, hi), np.array(gold["H"]))
    G = oracle.gram(x, kd, lo, hi)
    np.testing.assert_allclose(G, np.array(gold["gram"]), atol=1e-14)
    Q, ev, _ = oracle.nullspace(G, gold["rank"])
    assert ev[0] == pytest.approx(gold["lambda_min"], rel=1e-12)
    assert ev[1] == pytest.approx(gold["lambda_max"], rel=1e-12)
    q = np.array(gold["q_unnormalised"])
    q = q / np.linalg.norm(q)
    assert abs(abs(np.vdot(q, Q[:, 0])) - 1.0) < 1e-12
    assert oracle.objective(x, Q, kd, lo, hi) == pytest.approx(gold["lambda_min"], rel=1e-10)


def _problem_region():
    P = synth.make_problem("2d_64x64x4")
    lo, hi, _ = P["schedule"][0]
    return P, lo, hi


def test_tail_energy_matches_svd_of_explicit_H():
    """Eq. 1: J(x) = sum_{k>r} sigma_k^2{H(x)} computed by an SVD of H (a
    different routine) equals ||H Q||^2 with Q from the Gram eigenvectors
    and the sum of the n - r smallest Gram eigenvalues (Ky Fan)."""
    P, lo, hi = _problem_region()
    x, kd, r = P["x0"], P["kdims"], P["rank"]
    H = oracle.hankel_matrix(x, kd, lo, hi)
    sig = np.linalg.svd(H, compute_uv=False)
    tail = float((sig[r:] ** 2).sum())
    Q, ev, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), r)
    assert oracle.objective(x, Q, kd, lo, hi) == pytest.approx(tail, rel=1e-9)
    assert float(ev[: Q.shape[1]].sum()) == pytest.approx(tail, rel=1e-9)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(Q.shape[1]), atol=1e-12)


def test_nullspace_minimises_over_orthonormal_bases():
    """Any other orthonormal Q' of the same width gives ||H Q'||^2 >= J."""
    P, lo, hi = _problem_region()
    x, kd, r = P["x0"], P["kdims"], P["rank"]
    G = oracle.gram(x, kd, lo, hi)
    Q, _, _ = oracle.nullspace(G, r)
    J = oracle.objective(x, Q, kd, lo, hi)
    rng = np.random.default_rng(0)
    for _ in range(5):
        A = rng.standard_normal(Q.shape) + 1j * rng.standard_normal(Q.shape)
        Qr, _ = np.linalg.qr(Q + 0.05 * A)
        assert oracle.objective(x, Qr, kd, lo, hi) >= J * (1 - 1e-12)


def test_unit_kernel_gram_is_coil_covariance():
    """With a 1x1 kernel the Gram is X'X, X the (points x coils) data matrix."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 6, 4)) + 1j * rng.standard_normal((2, 5, 6, 4))
    X = x.reshape(-1, 4)
    G = oracle.gram(x, (1, 1, 1), (0, 0, 0), (2, 5, 6))
    np.testing.assert_allclose(G, X.conj().T @ X, atol=1e-12)


@pytest.mark.parametrize("w,K", [(3, 5), (2, 4)])
def test_bandlimited_coils_give_exact_rank_and_annihilation(w, K):
    """Coil maps with w x w k-space support make every coil's k-space an exact
    circular convolution of one image's k-space with a w x w kernel, so
    H(x) = M T with M the Hankel matrix of the image k-space for a
    (K + w - 1)^2 kernel: rank H = (K + w - 1)^2 exactly, and the nullspace
    of that rank annihilates the fully sampled data."""
    rng = np.random.default_rng(7)
    N, nc = 40, 4
    img = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    maps = synth.bandlimited_coil_maps((N, N), nc, w, rng)
    x = synth.to_kspace(img, maps)[None]
    kd, lo, hi = (1, K, K), (0, 0, 0), (1, N, N)
    H = oracle.hankel_matrix(x, kd, lo, hi)
    sig = np.linalg.svd(H, compute_uv=False)
    rank = int((sig > 1e-10 * sig[0]).sum())
    assert rank == (K + w - 1) ** 2
    Q, _, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), rank)
    J = oracle.objective(x, Q, kd, lo, hi)
    assert J / float((sig ** 2).sum()) < 1e-24
