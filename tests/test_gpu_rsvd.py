"""Randomized-SVD nullspace route on the device (THEORY, first numerical
technique; Algorithm 1, rSVD and Householder steps) against the FP64
oracle, on the same sketch draw.

Tolerance.  The device sketch Y = H Omega runs with FP32 operands and
sums (relative error about sqrt(n) u, u = 2^-24); everything after it is
FP64.  That perturbs the range of Y, hence B'B = H' P_Y H, by about
sqrt(n) u of its largest eigenvalue, and by Davis-Kahan the r-dimensional
principal subspace moves by at most that over the relative eigengap
(s_r^2 - s_{r+1}^2) / s_1^2 of B'B; a factor 16 covers the constants.  The
individual singular vectors, which fix the Householder basis, move by
sqrt(n) u over the smallest relative gap between consecutive singular
values down to s_{r+1}.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2004_08962_amd as hicu
    assert torch.cuda.is_available()
    hicu.load()
    return hicu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def _proj(A):
    return A @ A.conj().T


def _bandlimited(N, nc, w, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    img = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    maps = synth.bandlimited_coil_maps((N, N), nc, w, rng)
    x = synth.to_kspace(img, maps)[None]
    if noise:
        x = x + noise * np.abs(x).max() * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    return x.astype(np.complex64)


def _cases():
    rng = np.random.default_rng(21)
    P = synth.make_problem("2d_64x64x4")
    x3 = (rng.standard_normal((6, 10, 10, 2)) + 1j * rng.standard_normal((6, 10, 10, 2))).astype(np.complex64)
    xc = (rng.standard_normal((5, 9, 11, 3)) + 1j * rng.standard_normal((5, 9, 11, 3))).astype(np.complex64)
    disc = np.zeros((1, 5, 5), bool)
    a = np.arange(5) - 2
    disc[0] = a[:, None] ** 2 + a[None, :] ** 2 <= 5
    # name: (x, kdims, lo, hi, wrap, rank, ell)
    return {
        "exact_rank_2d": (_bandlimited(24, 4, 2, 7), (1, 4, 4), (0, 0, 0), (1, 24, 24), None, 25, 0),
        "noisy_2d": (_bandlimited(24, 4, 2, 8, 1e-3), (1, 4, 4), (0, 0, 0), (1, 24, 24), None, 25, 0),
        "phantom_2d": (P["x0"].astype(np.complex64), (1, 5, 5), (0, 0, 0), (1, 64, 64), None, 30, 0),
        "phantom_centre": (P["x0"].astype(np.complex64), (1, 5, 5), (0, 18, 20), (1, 46, 44), None, 30, 50),
        "random_3d": (x3, (3, 3, 3), (0, 0, 0), (6, 10, 10), None, 10, 0),
        "circular_3d": (xc, (3, 3, 3), (0, 1, 0), (5, 9, 11), (True, False, False), 12, 0),
        "disc_mask_2d": (P["x0"].astype(np.complex64), disc, (0, 0, 0), (1, 64, 64), None, 20, 0),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_rsvd_nullspace_matches_oracle(hc, name):
    x, kd, lo, hi, wrap, r, ell = CASES[name]
    seed, outer = 5, 3
    Qd, svd, _ = hc.nullspace_rsvd(_dev(x), kd, r, ell=ell, seed=seed, outer=outer, lo=lo, hi=hi, wrap=wrap,
                                   want_sv=True)
    Q = _host(Qd).astype(np.complex128)
    sv_dev = _host(svd)
    Qo, sv = oracle.nullspace_rsvd(x.astype(np.complex128), kd, lo, hi, r, seed, outer,
                                   ell=ell if ell else None, wrap=wrap)
    n = Qo.shape[0]
    assert Q.shape == Qo.shape
    # orthonormal to FP32 rounding of the stored Q
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n - r), atol=8 * np.sqrt(n) * U32)
    # singular values of the sketched B
    np.testing.assert_allclose(sv_dev, sv, rtol=0, atol=16 * np.sqrt(n) * U32 * sv[0])
    gap = (sv[r - 1] ** 2 - sv[r] ** 2) / sv[0] ** 2 if r < len(sv) else sv[r - 1] ** 2 / sv[0] ** 2
    tol = 16 * np.sqrt(n) * U32 / gap + 8 * np.sqrt(n) * U32
    assert np.linalg.norm(_proj(Q) - _proj(Qo), 2) <= tol
    # the basis itself (Householder convention) where the singular values are apart
    top = sv[: min(r + 1, len(sv))]
    mingap = float(np.min(-np.diff(top))) / sv[0]
    np.testing.assert_allclose(Q, Qo, rtol=0, atol=16 * np.sqrt(n) * U32 / mingap + 8 * U32)


def test_exact_rank_annihilates(hc):
    """rank H = 25 <= l: the device Q annihilates the data to FP32 rounding."""
    x, kd, lo, hi, wrap, r, ell = CASES["exact_rank_2d"]
    Q = _host(hc.nullspace_rsvd(_dev(x), kd, r, seed=1, outer=0, lo=lo, hi=hi)).astype(np.complex128)
    J = oracle.objective(x.astype(np.complex128), Q, kd, lo, hi)
    H = oracle.hankel_matrix(x.astype(np.complex128), kd, lo, hi)
    assert J / float(np.sum(np.abs(H) ** 2)) < 1e-10


def test_sketch_draw_matches_oracle(hc):
    Om = _host(hc.sketch(70, 33, seed=12345, outer=4, stream_id=2))
    Oo = oracle.sketch_matrix(12345, 4, 70, 33, stream=2)
    np.testing.assert_allclose(Om.real, Oo.real, rtol=2 * U32, atol=1e-12)
    np.testing.assert_allclose(Om.imag, Oo.imag, rtol=2 * U32, atol=1e-12)


def test_rank_zero_and_argument_errors(hc):
    x, kd, lo, hi, wrap, r, ell = CASES["random_3d"]
    Q = _host(hc.nullspace_rsvd(_dev(x), kd, 0, lo=lo, hi=hi))
    np.testing.assert_array_equal(Q, np.eye(54, dtype=np.complex64))
    with pytest.raises(ValueError):
        hc.nullspace_rsvd(_dev(x), kd, 10, ell=9, lo=lo, hi=hi)
    with pytest.raises(ValueError):
        hc.nullspace_rsvd(_dev(x), kd, 54, lo=lo, hi=hi)


def test_rsvd_sketch_is_deterministic(hc):
    x, kd, lo, hi, wrap, r, ell = CASES["phantom_2d"]
    a = _host(hc.nullspace_rsvd(_dev(x), kd, r, seed=9, outer=2, lo=lo, hi=hi))
    b = _host(hc.nullspace_rsvd(_dev(x), kd, r, seed=9, outer=2, lo=lo, hi=hi))
    np.testing.assert_array_equal(a, b)
    c = _host(hc.nullspace_rsvd(_dev(x), kd, r, seed=9, outer=3, lo=lo, hi=hi))
    assert np.abs(a - c).max() > 1e-3


def _solve_problem():
    P = synth.make_problem("2d_64x64x4")
    sched = [((0, 0, 0), (1, 64, 64), 5)] * 4
    return P, sched


def test_solve_rsvd_route_matches_oracle(hc):
    """Algorithm 1 with the rSVD route: FP32 device solve against the oracle's
    rSVD solve on the same sketches (p = 0, whole nullspace).  The rank cut
    of this problem lies in a flat stretch of the spectrum, so the two
    nullspaces differ there by the FP32 sketch error over a small gap; the
    reconstructions are compared on SER and on the objective trace."""
    P, sched = _solve_problem()
    kd, r = (1, 5, 5), 30
    tro = []
    xo = oracle.solve(P["x0"], P["mask"], kd, r, sched, route="rsvd", seed=6, trace=tro)
    x, tr = hc.solve(_dev(P["x0"].astype(np.complex64)), _dev(P["mask"].astype(np.uint8)), kd, r, sched, seed=6,
                     route="rsvd")
    x = _host(x).astype(np.complex128)
    ser_o, ser_d = oracle.ser(xo, P["x_true"]), oracle.ser(x, P["x_true"])
    assert abs(ser_d - ser_o) <= 0.1
    assert ser_d > oracle.ser(P["x0"], P["x_true"]) + 1.0
    m = P["mask"].astype(bool)
    np.testing.assert_array_equal(x[m], P["x0"][m].astype(np.complex64).astype(np.complex128))
    Jd = np.array([t["J"] for t in tr])
    Jo = np.array([t["J"] for t in tro])
    np.testing.assert_allclose(Jd, Jo, rtol=0.05)


def test_solve_full_sketch_equals_gram_route(hc):
    """l = n makes the rSVD exact, so with p = 0 both device routes follow
    the same iterates up to FP32 rounding over the rank-cut gap."""
    P = synth.make_problem("2d_64x64x4")
    x0 = P["x0"][:, 16:48, 16:48, :].astype(np.complex64)
    mask = P["mask"][:, 16:48, 16:48].astype(np.uint8)
    kd, r = (1, 3, 3), 12
    sched = [((0, 0, 0), (1, 32, 32), 3)] * 2
    xg, _ = hc.solve(_dev(x0), _dev(mask), kd, r, sched)
    xr, _ = hc.solve(_dev(x0), _dev(mask), kd, r, sched, route="rsvd", ell=36)
    # projector difference at most 16 sqrt(n) u / gap = 1.2e-3 (gap 4.8e-3 of this crop)
    assert oracle.rel_err(_host(xr).astype(np.complex128), _host(xg).astype(np.complex128)) < 2e-3


def test_solve_rsvd_with_jl(hc):
    """JL on top of the rSVD route: F = Q P with the oracle's P."""
    P, sched = _solve_problem()
    kd, r, p = (1, 5, 5), 30, 8
    xo = oracle.solve(P["x0"], P["mask"], kd, r, sched, p=p, route="rsvd", seed=2)
    x, _ = hc.solve(_dev(P["x0"].astype(np.complex64)), _dev(P["mask"].astype(np.uint8)), kd, r, sched, p=p, seed=2,
                    route="rsvd")
    x = _host(x).astype(np.complex128)
    assert abs(oracle.ser(x, P["x_true"]) - oracle.ser(xo, P["x_true"])) <= 0.1
