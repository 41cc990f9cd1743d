"""Differentiable objective on the GPU (48x48 x 4 coils, 3x3 kernel, 20
nullspace filters): the hand-written backward against central finite
differences (step 1e-3 relative to ||x||, 200 random directions) and
against the FP64 oracle gradient."""
import numpy as np
import pytest

import oracle
import synth
from bounds import forward_bound, grad_bound, sumsq_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2004_08962_amd as hicu
    from paper_2004_08962_amd.autograd import hicu_objective
    assert torch.cuda.is_available()
    P = synth.make_problem("gradcheck_48x48x4")
    x = P["x0"].astype(np.complex64)
    kd = P["kdims"]
    lo, hi, _ = P["schedule"][0]
    Q, _, _ = oracle.nullspace(oracle.gram(x.astype(np.complex128), kd, lo, hi), P["rank"])
    F = Q.astype(np.complex64)
    assert F.shape == (36, 20)
    return hicu, hicu_objective, torch, P, x, F, kd, lo, hi


def test_backward_is_the_adjoint_kernel(setup):
    hicu, obj, torch, P, x, F, kd, lo, hi = setup
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    Fd = torch.from_numpy(F).cuda()
    J = obj(xd, Fd, kd, lo, hi)
    (3.0 * J).backward()
    _, g, _ = hicu.objective_grad(xd.detach(), None, Fd, kd, lo, hi)
    assert torch.equal(xd.grad, 3.0 * g)
    # FP64 oracle gradient (no mask) within the rounding bound of the kernels
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    _, gr, _ = oracle.objective_grad(xr, None, Fr, kd, lo, hi)
    eg = grad_bound(xr, None, Fr, kd, lo, hi, "fp32")
    gg = g.cpu().numpy().astype(np.complex128)
    assert np.all(np.abs(gg - gr) <= eg + 1e-30)
    # with the sampling mask the gradient is projected (hard data matching)
    xm = torch.from_numpy(x).cuda().requires_grad_(True)
    md = torch.from_numpy(P["mask"]).cuda()
    obj(xm, Fd, kd, lo, hi, md).backward()
    gm = xm.grad.cpu().numpy()
    assert np.all(gm[P["mask"].astype(bool)] == 0)
    assert np.array_equal(gm[~P["mask"].astype(bool)], gg.astype(np.complex64)[~P["mask"].astype(bool)])


def test_central_differences_200_directions(setup):
    hicu, obj, torch, P, x, F, kd, lo, hi = setup
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    Fd = torch.from_numpy(F).cuda()
    obj(xd, Fd, kd, lo, hi).backward()
    g = xd.grad.cpu().numpy().astype(np.complex128)
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    eg = grad_bound(xr, None, Fr, kd, lo, hi, "fp32")
    rng = np.random.default_rng(123)
    h = 1e-3
    worst = 0.0
    for i in range(200):
        d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        d *= np.linalg.norm(xr) / np.linalg.norm(d)
        xp = (xr + h * d).astype(np.complex64)
        xm = (xr - h * d).astype(np.complex64)
        Jp = obj(torch.from_numpy(xp).cuda(), Fd, kd, lo, hi).item()
        Jm = obj(torch.from_numpy(xm).cuda(), Fd, kd, lo, hi).item()
        # the perturbed points are rounded to complex64: use the exact step taken
        dp = (xp.astype(np.complex128) - xm.astype(np.complex128)) / (2 * h)
        fd = (Jp - Jm) / (2 * h)
        an = float(np.vdot(g, dp).real)
        Yp, eYp = forward_bound(xp.astype(np.complex128), Fr, kd, lo, hi, "fp32")
        Ym, eYm = forward_bound(xm.astype(np.complex128), Fr, kd, lo, hi, "fp32")
        # J is quadratic.  With a, b the rounded points, a - b = 2 h dp and
        # a + b = 2 x + rs, the exact central difference is
        # Re<dp, g(x)> + Re<H(dp) F, H(rs) F>; the GPU values of J and g add
        # at most their rounding bounds.
        rs = xp.astype(np.complex128) + xm.astype(np.complex128) - 2 * xr
        curv = np.linalg.norm(oracle.forward(dp, Fr, kd, lo, hi)) * np.linalg.norm(oracle.forward(rs, Fr, kd, lo, hi))
        tol = (sumsq_bound(Yp, eYp) + sumsq_bound(Ym, eYm)) / (2 * h) + float(np.sum(eg * np.abs(dp))) + curv
        assert abs(fd - an) <= tol + 1e-6 * abs(an), (i, fd, an, tol)
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-30))
    print("worst relative FD mismatch over 200 directions: %.2e" % worst)
