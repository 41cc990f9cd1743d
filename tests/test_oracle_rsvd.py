"""Pins for the randomized-SVD nullspace route (THEORY, first numerical
technique; Algorithm 1, rSVD and Householder steps)."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth


def _proj(V):
    return V @ V.conj().T


def _random_x(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _bandlimited(N, nc, w, seed):
    rng = np.random.default_rng(seed)
    img = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    maps = synth.bandlimited_coil_maps((N, N), nc, w, rng)
    return synth.to_kspace(img, maps)[None]


def test_sketch_size_and_draw_layout():
    assert oracle.sketch_size(120, 400) == 180
    assert oracle.sketch_size(7, 400) == 11
    assert oracle.sketch_size(300, 400) == 400
    Om = oracle.sketch_matrix(5, 3, 40, 30)
    assert Om.shape == (40, 30)
    z = oracle.philox_normals(2 * 40 * 30, 5, 3, 0xFFFFFFFF)
    np.testing.assert_array_equal(Om[2, 7].real, z[2 * (2 * 30 + 7)])
    np.testing.assert_array_equal(Om[2, 7].imag, z[2 * (2 * 30 + 7) + 1])
    # N(0, 1) real and imaginary parts, and no overlap with the JL draws of
    # the same outer iteration
    big = oracle.sketch_matrix(1, 0, 300, 200).ravel()
    for part in (big.real, big.imag):
        assert abs(part.mean()) < 0.02 and abs(part.var() - 1.0) < 0.02
    P = oracle.jl_matrix(1, 0, 0, 300, 200) * np.sqrt(200)
    assert abs(np.corrcoef(P.ravel(), big.real)[0, 1]) < 0.02


def test_full_sketch_equals_svd_of_explicit_H():
    """With l = n the sketch spans the whole range of H, so B = U'H has the
    right singular vectors of H itself (LAPACK gesvd on the explicit H)."""
    x = _random_x((1, 12, 12, 3), 2)
    kd, lo, hi, r = (1, 3, 3), (0, 0, 0), (1, 12, 12), 10
    n = 27
    H = oracle.hankel_matrix(x, kd, lo, hi)
    _, sig, Vh = scipy.linalg.svd(H, full_matrices=False, lapack_driver="gesvd")
    V, sv = oracle.rsvd_right(x, kd, lo, hi, r, oracle.sketch_matrix(9, 0, n, n))
    np.testing.assert_allclose(sv, sig, rtol=1e-10)
    gap = (sig[r - 1] - sig[r]) / sig[0]
    assert gap > 1e-3
    err = np.linalg.norm(_proj(V) - _proj(Vh[:r].conj().T), 2)
    assert err < 1e-12 / gap


@pytest.mark.parametrize("r", [25, 20])
def test_exact_rank_recovered(r):
    """Band-limited coils give rank H = (K + w - 1)^2 = 25 exactly (see the
    nullspace pins).  A sketch with l >= 25 columns spans the range of H, so
    the rSVD is exact: for r = 25 the completed Q annihilates the data, and
    for r = 20 V spans the top 20 right singular vectors."""
    x = _bandlimited(24, 4, 2, 7)
    kd, lo, hi = (1, 4, 4), (0, 0, 0), (1, 24, 24)
    H = oracle.hankel_matrix(x, kd, lo, hi)
    _, sig, Vh = scipy.linalg.svd(H, full_matrices=False, lapack_driver="gesvd")
    assert int((sig > 1e-10 * sig[0]).sum()) == 25
    Q, sv = oracle.nullspace_rsvd(x, kd, lo, hi, r, seed=3, i=1)
    assert Q.shape == (64, 64 - r)
    assert len(sv) == oracle.sketch_size(r, 64)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(64 - r), atol=1e-12)
    P_exact = np.eye(64) - _proj(Vh[:r].conj().T)
    gap = (sig[r - 1] - sig[r]) / sig[0]
    assert np.linalg.norm(_proj(Q) - P_exact, 2) < 1e-11 / gap
    if r == 25:
        J = oracle.objective(x, Q, kd, lo, hi)
        assert J / float((sig ** 2).sum()) < 1e-24
        Qg, _, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), r)
        assert np.linalg.norm(_proj(Q) - _proj(Qg), 2) < 1e-8


def test_range_finder_within_hmt_bound():
    """||H - U U'H||_F = sqrt(||H||_F^2 - sum sv^2) for the orthonormal U of
    the sketch.  Over several draws its mean stays within the expected-error
    bound of Halko, Martinsson and Tropp, and every draw stays above the
    Eckart-Young floor of rank-l approximations."""
    P = synth.make_problem("2d_64x64x4")
    x = P["x_true"][:, 16:48, 16:48, :]
    kd, lo, hi, r, ell = (1, 5, 5), (0, 0, 0), (1, 32, 32), 12, 18
    H = oracle.hankel_matrix(x, kd, lo, hi)
    sig = np.linalg.svd(H, compute_uv=False)
    fro2 = float((sig ** 2).sum())
    errs = []
    for seed in range(8):
        _, sv = oracle.rsvd_right(x, kd, lo, hi, r, oracle.sketch_matrix(seed, 0, H.shape[1], ell))
        e = np.sqrt(max(fro2 - float((sv ** 2).sum()), 0.0))
        assert e >= np.sqrt(float((sig[ell:] ** 2).sum())) * (1 - 1e-9)
        errs.append(e)
    assert np.mean(errs) <= oracle.rsvd.hmt_bound(sig[r:], r, ell)
    # and the bound is not vacuous: the error is far below ||H||_F
    assert np.mean(errs) < 0.5 * np.sqrt(fro2)


def test_householder_real_matches_library_qr():
    """For real V the reflector is LAPACK's, so Q equals the trailing columns
    of the complete QR factor of numpy/LAPACK."""
    rng = np.random.default_rng(4)
    for n, r in [(9, 4), (20, 7), (6, 5)]:
        V, _ = np.linalg.qr(rng.standard_normal((n, r)))
        Q, _, alpha = oracle.householder_complement(V)
        Qf = np.linalg.qr(V, mode="complete")[0]
        np.testing.assert_allclose(Q.real, Qf[:, r:], atol=1e-13)
        assert np.abs(Q.imag).max() == 0.0
        np.testing.assert_allclose(np.abs(alpha), 1.0, atol=1e-13)


def test_householder_complex_properties():
    rng = np.random.default_rng(5)
    n, r = 11, 5
    V, _ = np.linalg.qr(rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r)))
    Q, W, alpha = oracle.householder_complement(V)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n - r), atol=1e-13)
    np.testing.assert_allclose(V.conj().T @ Q, 0.0, atol=1e-13)
    # the product of the reflectors, applied to V, gives R = diag(alpha) on top
    Hprod = np.eye(n, dtype=complex)
    for j in range(r):
        w = W[:, j]
        Hprod = Hprod @ (np.eye(n) - 2.0 * np.outer(w, w.conj()))
    R = Hprod.conj().T @ V
    np.testing.assert_allclose(R[:r], np.diag(alpha), atol=1e-13)
    np.testing.assert_allclose(R[r:], 0.0, atol=1e-13)
    np.testing.assert_allclose(Hprod[:, r:], Q, atol=1e-13)
    # each alpha_j points opposite to the pivot it replaces
    A = V.copy()
    for j in range(r):
        a0 = A[j, j]
        assert np.real(np.conj(alpha[j]) * a0) <= 0.0
        w = W[j:, j]
        A[j:, j:] -= 2.0 * np.outer(w, w.conj() @ A[j:, j:])
    # column phases of V do not change the reflectors, hence not Q
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, r))
    Q2, _, _ = oracle.householder_complement(V * ph[None, :])
    np.testing.assert_allclose(Q2, Q, atol=1e-13)


def test_householder_of_coordinate_vectors():
    """V = the first r columns of I: every reflector only flips e_j, so Q is
    exactly the trailing identity block."""
    n, r = 8, 3
    V = np.eye(n)[:, :r].astype(complex)
    Q, _, alpha = oracle.householder_complement(V)
    E = np.zeros((n, n - r))
    E[r:] = np.eye(n - r)
    np.testing.assert_array_equal(Q, E)
    np.testing.assert_array_equal(alpha, -np.ones(r))


def test_rank_zero_gives_identity():
    x = _random_x((1, 8, 8, 2), 3)
    Q, sv = oracle.nullspace_rsvd(x, (1, 3, 3), (0, 0, 0), (1, 8, 8), 0, seed=1, i=0)
    np.testing.assert_array_equal(Q, np.eye(18))
    assert sv.size == 0
    with pytest.raises(ValueError):
        oracle.nullspace_rsvd(x, (1, 3, 3), (0, 0, 0), (1, 8, 8), 18, seed=1, i=0)
    with pytest.raises(ValueError):
        oracle.nullspace_rsvd(x, (1, 3, 3), (0, 0, 0), (1, 8, 8), 6, seed=1, i=0, ell=5)


def test_solve_full_sketch_equals_gram_route():
    """With l = n and p = 0 the rSVD route takes the exact nullspace, and the
    iterates depend on Q only through Q Q', so the two routes agree."""
    P = synth.make_problem("2d_64x64x4")
    x0 = P["x0"][:, 20:44, 20:44, :]
    mask = P["mask"][:, 20:44, 20:44]
    kd, r = (1, 3, 3), 12
    sched = [((0, 0, 0), (1, 24, 24), 3), ((0, 0, 0), (1, 24, 24), 3)]
    xg = oracle.solve(x0, mask, kd, r, sched)
    xr = oracle.solve(x0, mask, kd, r, sched, route="rsvd", ell=36, seed=2)
    assert oracle.rel_err(xr, xg) < 1e-8


def test_solve_rsvd_route_decreases_objective():
    P = synth.make_problem("2d_64x64x4")
    x0 = P["x0"][:, 16:48, 16:48, :]
    xt = P["x_true"][:, 16:48, 16:48, :]
    mask = P["mask"][:, 16:48, 16:48]
    kd, r = (1, 5, 5), 30
    sched = [((0, 0, 0), (1, 32, 32), 4)] * 3
    trace = []
    x = oracle.solve(x0, mask, kd, r, sched, route="rsvd", seed=4, trace=trace)
    for i in range(3):
        Js = [t["J"] for t in trace if t["i"] == i]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(Js, Js[1:]))
    assert oracle.ser(x, xt) > oracle.ser(x0, xt)
    np.testing.assert_array_equal(x[mask.astype(bool)], x0[mask.astype(bool)])
