"""Kernel masks on the device (THEORY: the {0,1} kernel mask gives the
support of the annihilating kernels; DISCUSSION: circular or spherical
supports) against the FP64 oracle: the Gram restricted to the mask's taps,
objective, gradient and line search with filters over those taps, and a
2-D reconstruction with a disc-shaped kernel."""
import numpy as np
import pytest

import oracle
import synth
from bounds import forward_bound, grad_bound, sumsq_bound

pytestmark = pytest.mark.gpu


def disc(K):
    c = (K - 1) / 2.0
    a = np.arange(K)
    return ((a[:, None] - c) ** 2 + (a[None, :] - c) ** 2 <= (K / 2.0) ** 2)[None]


def ball(K):
    c = (K - 1) / 2.0
    a = np.arange(K)
    return (a[:, None, None] - c) ** 2 + (a[None, :, None] - c) ** 2 + (a[None, None, :] - c) ** 2 <= (K / 2.0) ** 2


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


def _cases():
    rng = np.random.default_rng(11)
    P = synth.make_problem("2d_64x64x4")
    x2 = P["x0"].astype(np.complex64)
    x3 = (rng.standard_normal((8, 14, 13, 3)) + 1j * rng.standard_normal((8, 14, 13, 3))).astype(np.complex64)
    m3 = (rng.random((8, 14, 13)) < 0.3).astype(np.uint8)
    rnd = rng.random((2, 4, 3)) < 0.6
    rnd[0, 0, 0] = True
    return {
        "disc5_2d": (x2, P["mask"], disc(5), (0, 0, 0), (1, 64, 64)),
        "disc5_2d_centre": (x2, P["mask"], disc(5), (0, 20, 22), (1, 44, 42)),
        "ball5_3d": (x3, m3, ball(5), (0, 0, 0), (8, 14, 13)),
        "random_3d": (x3, m3, rnd, (1, 2, 0), (8, 13, 13)),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_masked_gram(hc, name):
    x, _, km, lo, hi = CASES[name]
    print("masked gram", name, int(km.sum()), "taps", flush=True)
    G = _host(hc.gram(_dev(x), km, lo, hi))
    xr = x.astype(np.complex128)
    Gr = oracle.gram(xr, km, lo, hi)
    assert G.shape == Gr.shape == (int(km.sum()) * x.shape[3],) * 2
    H = oracle.hankel_matrix(np.abs(xr), km, lo, hi)
    bound = 2.0 * (H.shape[0] + 4) * 2.0 ** -53 * (H.T @ H).real + 1e-300
    assert np.all(np.abs(G - Gr) <= bound)
    assert np.array_equal(G, G.conj().T)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CASES))
def test_masked_objective_grad_line_search(hc, name, prec):
    x, mask, km, lo, hi = CASES[name]
    n = int(km.sum()) * x.shape[3]
    rng = np.random.default_rng(3)
    F = ((rng.standard_normal((n, 9)) + 1j * rng.standard_normal((n, 9))) / np.sqrt(n)).astype(np.complex64)
    print("masked step", name, prec, flush=True)
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    J, g, gn2 = hc.objective_grad(_dev(x), _dev(mask), _dev(F), km, lo, hi, prec=prec)
    J, gh, gn2v = float(J.item()), _host(g).astype(np.complex128), float(gn2.item())
    Jr, gr, _ = oracle.objective_grad(xr, mask, Fr, km, lo, hi)
    Y, eY = forward_bound(xr, Fr, km, lo, hi, prec)
    assert abs(J - Jr) <= sumsq_bound(Y, eY), (J, Jr)
    eg = grad_bound(xr, mask, Fr, km, lo, hi, prec)
    assert np.all(np.abs(gh - gr) <= eg + 1e-30)
    eta = hc.line_search(g, gn2, _dev(F), km, lo, hi, prec=prec)
    Z, eZ = forward_bound(gh, Fr, km, lo, hi, prec)
    zz = float(np.vdot(Z, Z).real)
    rel = sumsq_bound(Z, eZ) / zz
    eta_r = gn2v / (2 * zz)
    assert abs(eta.item() - eta_r) <= (rel / (1 - rel)) * eta_r + 1e-12 * eta_r


def test_masked_solve_matches_oracle(hc):
    P = synth.make_problem("2d_64x64x4")
    x0 = P["x0"].astype(np.complex64)
    km = disc(5)
    sched = P["schedule"][:4]
    print("masked solve, disc kernel", int(km.sum()), "taps", flush=True)
    ref = oracle.solve(x0.astype(np.complex128), P["mask"], km, P["rank"], sched)
    x, tr = hc.solve(_dev(x0), _dev(P["mask"]), km, P["rank"], sched, prec="fp32")
    xh = _host(x)
    err = oracle.rel_err(xh, ref)
    print("rel err %.3e, SER %.4f (oracle %.4f; 5x5 box %.4f)" % (
        err, oracle.ser(xh, P["x_true"]), oracle.ser(ref, P["x_true"]),
        oracle.ser(oracle.solve(x0.astype(np.complex128), P["mask"], P["kdims"], P["rank"], sched), P["x_true"])),
        flush=True)
    assert err <= 1e-4
    obs = P["mask"].astype(bool)
    assert np.array_equal(xh[obs], x0[obs])
