"""Three-dimensional problems and filter grouping on the GPU.

* The gradient over filter groups (forced by a small budget) meets the
  oracle's rounding bounds for every precision, with and without a region
  and a mask, and agrees with the single-group gradient.  On 3-D problems
  the grouped BF16 path stores the residual as BF16 in filter blocks
  (ragged last block included).
* A 16 x 28 x 28 x 8-coil volume from the 3-D workload's generator
  (5 x 5 x 5 kernel, rank 100, 900 nullspace filters) reconstructs like the
  FP64 oracle: FP32 within 1e-4 relative k-space error, BF16 with FP32
  refinement within 0.1 dB SER.
* At the full 256 x 320 x 320 x 8 size with 900 filters (15 groups of 64
  under the default budget) the gradient matches the point-wise oracle at
  sampled locations, and J equals the forward-only J over all filters.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import forward_bound, grad_bound, grad_bound_at_points, sumsq_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2004_08962_amd as hicu
    assert torch.cuda.is_available()
    hicu.load()
    yield hicu
    hicu.set_filter_group_budget(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rand(shape, seed, mask_frac=0.3):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mask = (rng.random(shape[:3]) < mask_frac).astype(np.uint8)
    return x, mask


def _filters(n, p, seed):
    rng = np.random.default_rng(seed)
    return ((rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(n)).astype(np.complex64)


GROUP_CASES = [  # (name, shape, kdims, lo, hi, p, use mask)
    ("3d_full", (9, 14, 12, 4), (3, 3, 3), (0, 0, 0), (9, 14, 12), 100, True),
    ("3d_region", (9, 14, 12, 4), (3, 3, 3), (1, 2, 1), (8, 13, 12), 70, True),
    ("2d_nomask", (1, 40, 36, 6), (1, 5, 5), (0, 0, 0), (1, 40, 36), 97, False),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp16"])
@pytest.mark.parametrize("case", GROUP_CASES, ids=[c[0] for c in GROUP_CASES])
def test_grouped_gradient_matches_oracle(hc, case, prec):
    name, shape, kd, lo, hi, p, use_mask = case
    x, mask = _rand(shape, 11)
    mask = mask if use_mask else None
    n = kd[0] * kd[1] * kd[2] * shape[3]
    F = _filters(n, p, 12)
    s = int(np.prod([h - l - k + 1 for l, h, k in zip(lo, hi, kd)]))
    md = _dev(mask) if mask is not None else None
    hc.set_filter_group_budget(0)
    J1, g1, n1 = hc.objective_grad(_dev(x), md, _dev(F), kd, lo, hi, prec=prec)
    # groups of 64 filters and a ragged last group, for complex64 Y and for
    # the compact BF16 Y (4 bytes per value) that the 3-D BF16 path uses
    hc.set_filter_group_budget(s * 4 * 64)
    try:
        J, g, gn2 = hc.objective_grad(_dev(x), md, _dev(F), kd, lo, hi, prec=prec)
    finally:
        hc.set_filter_group_budget(0)
    ngroups = -(-p // 64)
    print(name, prec, "groups", ngroups, flush=True)
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    Jr, gr, _ = oracle.objective_grad(xr, mask, Fr, kd, lo, hi)
    Y, eY = forward_bound(xr, Fr, kd, lo, hi, prec)
    assert abs(J.item() - Jr) <= sumsq_bound(Y, eY)
    eg = grad_bound(xr, mask, Fr, kd, lo, hi, prec, groups=ngroups)
    gh = g.cpu().numpy().astype(np.complex128)
    assert np.all(np.abs(gh - gr) <= eg + 1e-30)
    # same partial sums as one group, reduced in another order
    assert abs(J.item() - J1.item()) <= 1e-12 * abs(J1.item())
    assert np.all(np.abs(gh - g1.cpu().numpy()) <= 2 * eg + 1e-30)
    assert abs(gn2.item() - float(np.vdot(gh, gh).real)) <= 1e-5 * gn2.item()
    if mask is not None:
        assert np.all(gh[mask.astype(bool)] == 0)


@pytest.fixture(scope="module")
def vol():
    P = synth.make_problem("3d_16x28x28x8")
    x0 = P["x0"].astype(np.complex64)
    xr = x0.astype(np.complex128)
    G = oracle.gram(xr, P["kdims"], (0, 0, 0), (16, 28, 28))
    lam = np.linalg.eigvalsh(G)
    nq = 1000 - P["rank"]
    print("eigengap at the rank cut / lambda_max: %.3e" % ((lam[nq] - lam[nq - 1]) / lam[-1]), flush=True)
    ref = oracle.solve(xr, P["mask"], P["kdims"], P["rank"], P["schedule"])
    return P, x0, ref


def test_volume_solve_fp32_matches_oracle(hc, vol):
    P, x0, ref = vol
    print("solve fp32 3d_16x28x28x8", flush=True)
    x, tr = hc.solve(_dev(x0), _dev(P["mask"]), P["kdims"], P["rank"], P["schedule"], prec="fp32")
    xh = x.cpu().numpy()
    err = oracle.rel_err(xh, ref)
    print("rel err", err, "ser", oracle.ser(xh, P["x_true"]), oracle.ser(ref, P["x_true"]), flush=True)
    assert err <= 1e-4
    obs = P["mask"].astype(bool)
    assert np.array_equal(xh[obs], x0[obs])
    assert len(tr) == 6


def test_volume_solve_bf16_refine_ser(hc, vol):
    P, x0, ref = vol
    x, tr = hc.solve(_dev(x0), _dev(P["mask"]), P["kdims"], P["rank"], P["schedule"], prec="bf16",
                     refine_steps=2)
    xh = x.cpu().numpy()
    d = oracle.ser(xh, P["x_true"]) - oracle.ser(ref, P["x_true"])
    print("delta SER", d, "rel err", oracle.rel_err(xh, ref), flush=True)
    assert abs(d) <= 0.1


def test_full_volume_900_filters_sampled(hc):
    """256 x 320 x 320 x 8, 5 x 5 x 5 kernel, 900 orthonormal filters, BF16:
    the launch configuration the 3-D benchmark times."""
    import torch
    P = synth.make_problem("3d_256x320x320x8", dtype=np.complex64)
    x = P["x0"]
    kd, lo, hi = P["kdims"], (0, 0, 0), (256, 320, 320)
    n, p = 1000, 900
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))
    F = np.linalg.qr(A)[0].astype(np.complex64)
    xd, md, Fd = _dev(x), _dev(P["mask"]), _dev(F)
    for prec in ("bf16",):
        print("full volume", prec, flush=True)
        J, g, gn2 = hc.objective_grad(xd, md, Fd, kd, lo, hi, prec=prec)
        J0, _, _ = hc.objective_grad(xd, md, Fd, kd, lo, hi, prec=prec, want_grad=False)
        torch.cuda.synchronize()
        assert abs(J.item() - J0.item()) <= 1e-12 * J0.item()
        pts = [(int(a), int(b), int(c)) for a, b, c in zip(rng.integers(0, 256, 6), rng.integers(0, 320, 6),
                                                           rng.integers(0, 320, 6))]
        pts += [(0, 0, 0), (255, 319, 319), (128, 160, 160), (2, 318, 1)]
        gh = np.stack([g[w].cpu().numpy() for w in pts])
        del g
        xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
        gr = oracle.grad_at_points(xr, P["mask"], Fr, kd, lo, hi, pts)
        b = grad_bound_at_points(xr, Fr, kd, lo, hi, prec, pts, groups=15)
        for i, w in enumerate(pts):
            if P["mask"][w]:
                assert np.all(gh[i] == 0)
            else:
                assert np.all(np.abs(gh[i] - gr[i]) <= b[i]), (prec, w)
