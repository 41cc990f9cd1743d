"""Circular convolution along an axis (METHODS, Study II: circular along
time for the 2-D+t study) and the time-averaged initial k-space, on the
device against the FP64 oracle.

* Contractions and the Gram with a circular axis, element by element under
  the rounding bounds of tests/bounds.py, in every precision, including a
  period equal to the kernel extent and circular on all three axes.
* The time-averaged initialisation within one FP32 rounding of the oracle.
* A reconstruction of the cine workload (all 25 frames, so the time axis is
  whole; a 28 x 24 spatial crop, 12 coils, a 5 x 3 x 3 kernel over
  (t, kx, ky), rank 130) with circular time and the time-averaged start:
  FP32 within 1e-4 relative k-space error of the oracle, BF16 with FP32
  refinement within 0.1 dB SER.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import U32, forward_bound, grad_bound, sumsq_bound

pytestmark = pytest.mark.gpu


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


def _case(shape, kd, wrap, lo, hi, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mask = (rng.random(shape[:3]) < 0.3).astype(np.uint8)
    return (x, mask, kd, wrap, lo, hi)


CASES = {
    "t_circular": _case((9, 21, 19, 3), (3, 3, 3), (True, False, False), (0, 2, 1), (9, 20, 19), 1),
    "period_eq_kernel": _case((5, 12, 10, 2), (5, 3, 3), (True, False, False), (0, 0, 0), (5, 12, 10), 2),
    "all_circular": _case((6, 7, 8, 2), (3, 4, 2), (True, True, True), (0, 0, 0), (6, 7, 8), 3),
    "2d_circular_ky": _case((1, 30, 17, 4), (1, 5, 5), (False, False, True), (0, 3, 0), (1, 27, 17), 4),
}


def _filters(n, p, seed):
    rng = np.random.default_rng(seed)
    F = (rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(n)
    return F.astype(np.complex64)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp16"])
@pytest.mark.parametrize("name", list(CASES))
def test_objective_grad_line_search(hc, name, prec):
    x, mask, kd, wrap, lo, hi = CASES[name]
    n = kd[0] * kd[1] * kd[2] * x.shape[3]
    F = _filters(n, 11, 7)
    print("circular", name, prec, flush=True)
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    J, g, gn2 = hc.objective_grad(_dev(x), _dev(mask), _dev(F), kd, lo, hi, prec=prec, wrap=wrap)
    J, gh, gn2v = float(J.item()), _host(g).astype(np.complex128), float(gn2.item())
    Jr, gr, _ = oracle.objective_grad(xr, mask, Fr, kd, lo, hi, wrap)
    Y, eY = forward_bound(xr, Fr, kd, lo, hi, prec, wrap)
    assert abs(J - Jr) <= sumsq_bound(Y, eY), (J, Jr)
    eg = grad_bound(xr, mask, Fr, kd, lo, hi, prec, wrap=wrap)
    assert np.all(np.abs(gh - gr) <= eg + 1e-30)
    assert abs(gn2v - float(np.vdot(gh, gh).real)) <= 1e-9 * max(gn2v, 1e-30)
    # outside the region (non-circular axes) and at observed points g is zero
    out = np.ones(x.shape[:3], bool)
    out[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = False
    assert np.all(gh[out] == 0) and np.all(gh[mask.astype(bool)] == 0)
    eta = hc.line_search(g, gn2, _dev(F), kd, lo, hi, prec=prec, wrap=wrap)
    Z, eZ = forward_bound(gh, Fr, kd, lo, hi, prec, wrap)
    zz = float(np.vdot(Z, Z).real)
    eta_r = gn2v / (2 * zz)
    rel = sumsq_bound(Z, eZ) / zz
    assert abs(eta.item() - eta_r) <= (rel / (1 - rel)) * eta_r + 1e-12 * eta_r


@pytest.mark.parametrize("name", list(CASES))
def test_gram(hc, name):
    x, mask, kd, wrap, lo, hi = CASES[name]
    print("circular gram", name, flush=True)
    G = _host(hc.gram(_dev(x), kd, lo, hi, wrap=wrap))
    xr = x.astype(np.complex128)
    Gr = oracle.gram(xr, kd, lo, hi, wrap)
    H = oracle.hankel_matrix(np.abs(xr), kd, lo, hi, wrap)
    bound = 2.0 * (H.shape[0] + 4) * 2.0 ** -53 * (H.T @ H).real + 1e-300
    assert np.all(np.abs(G - Gr) <= bound)
    assert np.array_equal(G, G.conj().T)


def test_gram_direct_route_refuses_circular(hc):
    from paper_2004_08962_amd import HicuError
    x, mask, kd, wrap, lo, hi = CASES["t_circular"]
    hc.set_gram_route(0)
    try:
        G = hc.gram(_dev(x), kd, lo, hi, wrap=wrap)  # falls back to the shift-correlation route
        Gr = oracle.gram(x.astype(np.complex128), kd, lo, hi, wrap)
        assert np.abs(_host(G) - Gr).max() <= 1e-9 * np.abs(Gr).max()
    finally:
        hc.set_gram_route(1)
    with pytest.raises(HicuError):  # a circular axis must span the whole array
        hc.gram(_dev(x), kd, (1, 0, 0), (9, 21, 19), wrap=(True, False, False))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_time_average_init(hc, axis):
    P = synth.make_problem("cine_25x160x144x12")
    x0 = P["x0"].astype(np.complex64)
    mask = P["mask"]
    print("time average init axis", axis, flush=True)
    got = _host(hc.time_average_init(_dev(x0), _dev(mask), axis=axis))
    want = oracle.time_average_init(x0.astype(np.complex128), mask, axis)
    obs = mask.astype(bool)
    assert np.array_equal(got[obs], x0[obs])
    err = np.abs(got.astype(np.complex128) - want)
    assert np.all(err <= 2.0 * U32 * np.abs(want) + 1e-45)


@pytest.fixture(scope="module")
def cine_crop():
    P = synth.make_problem("cine_25x160x144x12")
    C = synth.crop_problem(P, (0, 66, 60), (25, 94, 84))
    C["kdims"] = (5, 3, 3)
    x0 = C["x0"].astype(np.complex64)
    xi = oracle.time_average_init(x0.astype(np.complex128), C["mask"], 0).astype(np.complex64)
    sched = [((0, 0, 0), x0.shape[:3], 3)] * 2
    return C, x0, xi, sched


def test_cine_circular_solve_matches_oracle(hc, cine_crop):
    C, x0, xi, sched = cine_crop
    wrap = (True, False, False)
    print("cine crop, circular time, time-averaged start", xi.shape, flush=True)
    # the device's time-averaged start equals the oracle's (one rounding)
    xd = hc.time_average_init(_dev(x0), _dev(C["mask"]), axis=0)
    assert np.all(np.abs(_host(xd).astype(np.complex128) - xi.astype(np.complex128)) <= 2 * U32 * np.abs(xi) + 1e-45)
    ref = oracle.solve(xi.astype(np.complex128), C["mask"], C["kdims"], C["rank"], sched, wrap=wrap)
    x, tr = hc.solve(_dev(xi), _dev(C["mask"]), C["kdims"], C["rank"], sched, prec="fp32", wrap=wrap)
    xh = _host(x)
    err = oracle.rel_err(xh, ref)
    print("circular fp32 rel err %.3e, SER %.4f (oracle %.4f)" % (err, oracle.ser(xh, C["x_true"]),
                                                                   oracle.ser(ref, C["x_true"])), flush=True)
    assert err <= 1e-4
    obs = C["mask"].astype(bool)
    assert np.array_equal(xh[obs], xi[obs])
    xb, _ = hc.solve(_dev(xi), _dev(C["mask"]), C["kdims"], C["rank"], sched, prec="bf16", refine_steps=2, wrap=wrap)
    d = oracle.ser(_host(xb), C["x_true"]) - oracle.ser(ref, C["x_true"])
    print("circular bf16+refine dSER %.4f" % d, flush=True)
    assert abs(d) <= 0.1
    # the valid-in-time reconstruction from the same start, for comparison
    xv, _ = hc.solve(_dev(xi), _dev(C["mask"]), C["kdims"], C["rank"], sched, prec="fp32")
    print("SER circular %.4f dB, valid %.4f dB, zero-filled %.4f, time-averaged start %.4f" % (
        oracle.ser(xh, C["x_true"]), oracle.ser(_host(xv), C["x_true"]), oracle.ser(x0, C["x_true"]),
        oracle.ser(xi, C["x_true"])), flush=True)
