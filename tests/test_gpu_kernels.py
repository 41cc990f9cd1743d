"""GPU parity of each C-ABI entry point against the FP64 oracle, on the same
seeded inputs (x and F rounded to complex64 once, both sides consume the
rounded values).  Tolerances are rounding-error bounds (tests/bounds.py)."""
import numpy as np
import pytest

import oracle
import synth
from bounds import forward_bound, grad_bound, sumsq_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2004_08962_amd as hicu
    assert torch.cuda.is_available(), "GPU tests need a device"
    hicu.load()
    return hicu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def _rand_problem(shape, kd, seed, mask_frac=0.3):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mask = (rng.random(shape[:3]) < mask_frac).astype(np.uint8)
    return x, mask


# (name, x, mask, kdims, lo, hi) cases: the 64x64x4 workload (full and centre
# region), the 3x3 gradient-check workload, and random 3-D / ragged / odd-coil
# / single-output / 1-D geometries.
def _cases():
    out = []
    P = synth.make_problem("2d_64x64x4")
    x = P["x0"].astype(np.complex64)
    out.append(("2d64_full", x, P["mask"], P["kdims"], (0, 0, 0), (1, 64, 64)))
    out.append(("2d64_centre", x, P["mask"], P["kdims"], (0, 24, 24), (1, 40, 40)))
    Pg = synth.make_problem("gradcheck_48x48x4")
    out.append(("gc48", Pg["x0"].astype(np.complex64), Pg["mask"], Pg["kdims"], (0, 0, 0), (1, 48, 48)))
    x3, m3 = _rand_problem((7, 21, 19, 3), (3, 3, 3), 1)
    out.append(("3d_odd", x3, m3, (3, 3, 3), (0, 0, 0), (7, 21, 19)))
    out.append(("3d_region", x3, m3, (2, 4, 3), (1, 2, 3), (7, 20, 17)))
    x5, m5 = _rand_problem((1, 37, 29, 5), (1, 5, 4), 2)
    out.append(("2d_ragged_nc5", x5, m5, (1, 5, 4), (0, 0, 0), (1, 37, 29)))
    x1, m1 = _rand_problem((1, 1, 300, 2), (1, 1, 7), 3)
    out.append(("1d", x1, m1, (1, 1, 7), (0, 0, 0), (1, 1, 300)))
    xs, ms = _rand_problem((1, 9, 9, 1), (1, 9, 9), 4)
    out.append(("single_output_nc1", xs, ms, (1, 9, 9), (0, 0, 0), (1, 9, 9)))
    return out


CASES = _cases()
IDS = [c[0] for c in CASES]


def _filters(x, kd, lo, hi, p, seed):
    n = kd[0] * kd[1] * kd[2] * x.shape[3]
    rng = np.random.default_rng(seed)
    F = (rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(n)
    return F.astype(np.complex64)


@pytest.mark.parametrize("route", [1, 0], ids=["shift_corr", "direct"])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_gram(hc, case, route):
    name, x, mask, kd, lo, hi = case
    print("gram", name, x.shape, kd, lo, hi, "route", route, flush=True)
    hc.set_gram_route(route)
    try:
        G = _host(hc.gram(_dev(x), kd, lo, hi))
    finally:
        hc.set_gram_route(1)
    xr = x.astype(np.complex128)
    Gr = oracle.gram(xr, kd, lo, hi)
    H = oracle.hankel_matrix(np.abs(xr), kd, lo, hi)
    bound = (H.shape[0] + 4) * 2.0 ** -53 * (H.T @ H).real * 2 + 1e-300
    assert np.all(np.abs(G - Gr) <= bound)
    assert np.array_equal(G, G.conj().T)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_objective_grad(hc, case, prec):
    name, x, mask, kd, lo, hi = case
    n = kd[0] * kd[1] * kd[2] * x.shape[3]
    for p in sorted({1, 7, min(n, 40)}):
        print("objective_grad", name, prec, "p", p, flush=True)
        F = _filters(x, kd, lo, hi, p, seed=p)
        xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
        J, g, gn2 = hc.objective_grad(_dev(x), _dev(mask), _dev(F), kd, lo, hi, prec=prec)
        J, g, gn2 = float(J.item()), _host(g).astype(np.complex128), float(gn2.item())
        Jr, gr, gn2r = oracle.objective_grad(xr, mask, Fr, kd, lo, hi)
        Y, eY = forward_bound(xr, Fr, kd, lo, hi, prec)
        assert abs(J - Jr) <= sumsq_bound(Y, eY), (J, Jr)
        eg = grad_bound(xr, mask, Fr, kd, lo, hi, prec)
        assert np.all(np.abs(g - gr) <= eg + 1e-30)
        assert np.all(g[mask.astype(bool)] == 0)
        inside = np.zeros(mask.shape, bool)
        inside[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
        assert np.all(g[~inside] == 0)
        assert abs(gn2 - float(np.vdot(g, g).real)) <= 1e-9 * max(gn2, 1e-30)
        assert abs(gn2 - gn2r) <= sumsq_bound(gr, eg)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("case", CASES[:4], ids=IDS[:4])
def test_line_search_and_update(hc, case, prec):
    name, x, mask, kd, lo, hi = case
    print("line_search", name, prec, flush=True)
    F = _filters(x, kd, lo, hi, 9, seed=3)
    xd, Fd = _dev(x), _dev(F)
    J, g, gn2 = hc.objective_grad(xd, _dev(mask), Fd, kd, lo, hi, prec=prec)
    eta = hc.line_search(g, gn2, Fd, kd, lo, hi, prec=prec)
    gh = _host(g).astype(np.complex128)
    Fr = F.astype(np.complex128)
    Z, eZ = forward_bound(gh, Fr, kd, lo, hi, prec)
    zz = float(np.vdot(Z, Z).real)
    gn = float(gn2.item())
    eta_r = gn / (2 * zz)
    rel = sumsq_bound(Z, eZ) / zz
    assert abs(eta.item() - eta_r) <= (rel / (1 - rel)) * eta_r + 1e-12 * eta_r
    x_before = x.copy()
    hc.update(xd, g, eta)
    xn = _host(xd)
    ref = (x_before.astype(np.complex128) - eta.item() * gh)
    assert np.all(np.abs(xn - ref) <= 2.0 ** -24 * np.abs(ref) * 1.01 + 1e-38)
    obs = mask.astype(bool)
    assert np.array_equal(xn[obs], x_before[obs])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape,kd", [((10, 40, 44, 8), (3, 3, 3)), ((1, 60, 70, 8), (1, 5, 5))], ids=["3d", "2d"])
def test_line_search_many_filters(hc, shape, kd, prec):
    """1100 filters: the line-search weights exceed 2 MB, so the launch walks
    column blocks over runs of 32 position tiles (the last run ragged)."""
    x, mask = _rand_problem(shape, kd, 21)
    F = _filters(x, kd, None, None, 1100, seed=22)
    print("line_search many filters", shape, kd, prec, flush=True)
    xd, Fd = _dev(x), _dev(F)
    J, g, gn2 = hc.objective_grad(xd, _dev(mask), Fd, kd, prec=prec)
    eta = hc.line_search(g, gn2, Fd, kd, prec=prec)
    gh = _host(g).astype(np.complex128)
    hi = shape[:3]
    Z, eZ = forward_bound(gh, F.astype(np.complex128), kd, (0, 0, 0), hi, prec)
    zz = float(np.vdot(Z, Z).real)
    eta_r = float(gn2.item()) / (2 * zz)
    rel = sumsq_bound(Z, eZ) / zz
    assert abs(eta.item() - eta_r) <= (rel / (1 - rel)) * eta_r + 1e-12 * eta_r


def test_full_mask_zero_step(hc):
    x, _ = _rand_problem((1, 30, 30, 4), (1, 5, 5), 9)
    full = np.ones((1, 30, 30), np.uint8)
    F = _filters(x, (1, 5, 5), None, None, 8, 1)
    J, g, gn2 = hc.objective_grad(_dev(x), _dev(full), _dev(F), (1, 5, 5))
    assert gn2.item() == 0.0 and np.all(_host(g) == 0)
    eta = hc.line_search(g, gn2, _dev(F), (1, 5, 5))
    assert eta.item() == 0.0


@pytest.mark.parametrize("workload", ["2d_64x64x4", "2d_256x232x16", "3d_16x28x28x8"])
def test_nullspace_matches_dense_eigh(hc, workload):
    """n = 100, 400 (the benchmarked Gram) and 1000 (5 x 5 x 5 kernel, 8 coils)."""
    import torch
    P = synth.make_problem(workload)
    x = P["x0"].astype(np.complex64).astype(np.complex128)
    lo, hi = (0, 0, 0), x.shape[:3]
    G = oracle.gram(x, P["kdims"], lo, hi)
    r = P["rank"]
    Qr, evr, Ur = oracle.nullspace(G, r)
    print("nullspace", workload, "n", G.shape[0], flush=True)
    Q, ev, V, sweeps = hc.nullspace(_dev(G), r)
    print("sweeps", sweeps, flush=True)
    ev, V, Q = _host(ev), _host(V), _host(Q)
    lmax = evr[-1]
    assert np.all(np.abs(ev - evr) <= 1e-12 * lmax)
    # projector onto the nullspace (Q rounded to complex64); FP64 subspace
    # error ~ eps lmax / gap at the rank cut
    nq = Qr.shape[1]
    gap = evr[nq] - evr[nq - 1]
    ptol = 1e-5 * np.sqrt(nq) + 1e-12 * lmax / gap
    Pg = Q.astype(np.complex128) @ Q.astype(np.complex128).conj().T
    Pr = Qr @ Qr.conj().T
    assert np.linalg.norm(Pg - Pr) <= ptol
    # individual eigenvectors where the spectrum is well separated
    gaps = np.minimum(np.r_[np.inf, np.diff(evr)], np.r_[np.diff(evr), np.inf])
    for j in np.where(gaps > 1e-6 * lmax)[0]:
        err = np.linalg.norm(V[:, j] - Ur[:, j])
        assert err <= 1e-12 * lmax / gaps[j] * 10 + 1e-10, (j, err)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(V.shape[0]), atol=1e-12)
    # warm start from the eigenvectors of a nearby Gram converges to the same split
    G2 = oracle.gram(x * (1 + 0.01 * np.random.default_rng(0).standard_normal(x.shape)), P["kdims"], lo, hi)
    Qr2, evr2, _ = oracle.nullspace(G2, r)
    Q2, ev2, _, sw2 = hc.nullspace(_dev(G2), r, V0=torch.from_numpy(V).cuda())
    print("warm sweeps", sw2, flush=True)
    assert np.all(np.abs(_host(ev2) - evr2) <= 1e-12 * evr2[-1])
    Q2 = _host(Q2).astype(np.complex128)
    gap2 = evr2[nq] - evr2[nq - 1]
    assert np.linalg.norm(Q2 @ Q2.conj().T - Qr2 @ Qr2.conj().T) <= 1e-5 * np.sqrt(nq) + 1e-12 * evr2[-1] / gap2


def test_jl_draw_matches_oracle(hc):
    rng = np.random.default_rng(5)
    n, nq, p = 100, 70, 8
    Q = (rng.standard_normal((n, nq)) + 1j * rng.standard_normal((n, nq))).astype(np.complex64)
    F, Pm = hc.jl_compress(_dev(Q), p, seed=12345678901, outer=3, inner=4, stream_id=2, return_P=True)
    Pr = oracle.jl_matrix(12345678901, 3, 4, nq, p, stream=2)
    np.testing.assert_allclose(_host(Pm), Pr, rtol=1e-13, atol=1e-13)
    Fr = Q.astype(np.complex128) @ Pr
    np.testing.assert_allclose(_host(F), Fr, rtol=0, atol=1e-5 * np.abs(Fr).max())


def test_profile_major_only(hc):
    """Major-only event timing records the contractions but not the
    per-step scalar kernels; full timing records both."""
    import torch
    x, mask = _rand_problem((1, 24, 24, 2), (1, 3, 3), seed=31)
    kd = (1, 3, 3)
    n = 18
    rng = np.random.default_rng(32)
    F = ((rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))) / np.sqrt(n)).astype(np.complex64)
    xd, md, Fd = _dev(x), _dev(mask), _dev(F)
    for minor in (False, True):
        hc.profile_begin(minor=minor)
        J, g, gn2 = hc.objective_grad(xd, md, Fd, kd, prec="fp32")
        hc.line_search(g, gn2, Fd, kd, prec="fp32")
        torch.cuda.synchronize()
        prof = hc.profile_end()
        print("minor", minor, sorted(prof), flush=True)
        assert {"conv_fwd_fp32", "conv_adj_fp32", "conv_els_fp32"} <= set(prof)
        assert ("reduce" in prof) == minor and ("eta" in prof) == minor
