"""2-D+t cine workload (25 frames of 160 x 144, 12 coils, 5 x 5 x 5 kernel
over (t, kx, ky), rank 130, 12 JL filters per step) on a centre crop of
10 frames x 36 x 32 (n = 1500 taps, 5376 valid outputs).

* Without JL (all 1370 nullspace filters) the reconstruction depends only
  on the projector onto the nullspace, which is unique here (relative gap
  3.3e-6 of lambda_max at the rank cut): FP32 within 1e-4 relative k-space
  error of the FP64 oracle.
* With 12 JL filters the draws F = Q P depend on the individual
  eigenvectors, and this nullspace has eigenvalues closer than 1e-17 of
  lambda_max, so its eigenvector basis is not unique and the device and
  LAPACK legitimately pick different ones.  What is compared is the
  reconstruction quality: SER within 0.05 dB of the oracle's, with the
  sampled entries unchanged.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

LO, HI = (7, 62, 56), (17, 98, 88)
SCHED = [((0, 0, 0), (10, 36, 32), 3)] * 2


@pytest.fixture(scope="module")
def crop():
    import torch
    import paper_2004_08962_amd as hicu
    assert torch.cuda.is_available()
    P = synth.make_problem("cine_25x160x144x12")
    C = synth.crop_problem(P, LO, HI)
    assert C["rank"] == 130 and C["p"] == 12
    x0 = C["x0"].astype(np.complex64)
    return hicu, torch, C, x0


def _solve(hicu, torch, C, x0, p):
    x, tr = hicu.solve(torch.from_numpy(x0).cuda(), torch.from_numpy(C["mask"]).cuda(), C["kdims"], C["rank"], SCHED,
                       p=p, seed=C["seed"], prec="fp32")
    assert len(tr) == 6
    return x.cpu().numpy()


def test_cine_crop_projector_solve_matches_oracle(crop):
    hicu, torch, C, x0 = crop
    print("cine crop, all nullspace filters", x0.shape, flush=True)
    ref = oracle.solve(x0.astype(np.complex128), C["mask"], C["kdims"], C["rank"], SCHED)
    xh = _solve(hicu, torch, C, x0, 0)
    err = oracle.rel_err(xh, ref)
    print("rel err %.3e ser %.4f / %.4f" % (err, oracle.ser(xh, C["x_true"]), oracle.ser(ref, C["x_true"])), flush=True)
    assert err <= 1e-4
    obs = C["mask"].astype(bool)
    assert np.array_equal(xh[obs], x0[obs])


def test_cine_crop_jl_solve_ser(crop):
    hicu, torch, C, x0 = crop
    print("cine crop, 12 JL filters", flush=True)
    ref = oracle.solve(x0.astype(np.complex128), C["mask"], C["kdims"], C["rank"], SCHED, p=C["p"], seed=C["seed"])
    xh = _solve(hicu, torch, C, x0, C["p"])
    d = oracle.ser(xh, C["x_true"]) - oracle.ser(ref, C["x_true"])
    print("JL dSER %.4f (rel err %.3e)" % (d, oracle.rel_err(xh, ref)), flush=True)
    assert abs(d) <= 0.05
    assert oracle.ser(xh, C["x_true"]) > oracle.ser(x0, C["x_true"]) + 0.5
    obs = C["mask"].astype(bool)
    assert np.array_equal(xh[obs], x0[obs])
