"""The benchmarked reconstruction end to end against the FP64 oracle:
256 x 232 k-space, 16 coils, 5 x 5 kernel, rank 120 (280 nullspace filters),
20 outer iterations of 5 gradient steps with exact line search, full region,
no JL (Algorithm 1).  The oracle runs the same schedule on the same
complex64-rounded input in FP64 with an explicit Hankel matrix and dense
eigh (about half a minute on the host).

Bars: FP32 within 1e-4 relative k-space error of the oracle; the BF16 paths
(BF16 with 10 refinement steps in FP32 or in split BF16, split BF16
throughout) within 0.1 dB SER of the oracle's."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2004_08962_amd as hicu
    assert torch.cuda.is_available()
    hicu.load()
    return hicu


@pytest.fixture(scope="module")
def ref():
    P = synth.make_problem("2d_256x232x16")
    x0 = P["x0"].astype(np.complex64)
    print("oracle solve 2d_256x232x16 (20 x 5 steps, 280 filters)", flush=True)
    tr = []
    xr = oracle.solve(x0.astype(np.complex128), P["mask"], P["kdims"], P["rank"], P["schedule"], trace=tr)
    ser = oracle.ser(xr, P["x_true"])
    print("oracle SER %.5f dB, final J %.6g" % (ser, tr[-1]["J"]), flush=True)
    return P, x0, xr, ser, tr


def _run(hc, P, x0, prec, refine, refine_prec="fp32"):
    import torch
    xd = torch.from_numpy(x0).cuda()
    md = torch.from_numpy(P["mask"]).cuda()
    x, tr = hc.solve(xd, md, P["kdims"], P["rank"], P["schedule"], prec=prec, refine_steps=refine,
                     refine_prec=refine_prec)
    return x.cpu().numpy(), tr


def test_fp32_matches_oracle(hc, ref):
    P, x0, xr, ser_r, tr_r = ref
    xh, tr = _run(hc, P, x0, "fp32", 0)
    err = oracle.rel_err(xh, xr)
    ser = oracle.ser(xh, P["x_true"])
    print("fp32 rel err %.3e, SER %.5f dB (oracle %.5f)" % (err, ser, ser_r), flush=True)
    assert err <= 1e-4
    obs = P["mask"].astype(bool)
    assert np.array_equal(xh[obs], x0[obs])
    assert len(tr) == len(tr_r) == 100
    # the objective follows the oracle's step by step
    for a, b in zip(tr, tr_r):
        assert abs(a["J"] - b["J"]) <= 1e-3 * b["J"], (a, b)


@pytest.mark.parametrize("prec,refine,rprec", [("bf16", 10, "fp32"), ("bf16", 10, "bf16x3"), ("bf16x3", 0, "fp32")],
                         ids=["bf16+refine", "bf16+refine_x3", "bf16x3"])
def test_bf16_paths_within_0p1_db(hc, ref, prec, refine, rprec):
    P, x0, xr, ser_r, _ = ref
    xh, tr = _run(hc, P, x0, prec, refine, rprec)
    ser = oracle.ser(xh, P["x_true"])
    print("%s: SER %.5f dB, oracle %.5f dB, dSER %.5f, rel err %.3e" % (prec, ser, ser_r, ser - ser_r,
                                                                       oracle.rel_err(xh, xr)), flush=True)
    assert abs(ser - ser_r) <= 0.1
    code = {"fp32": 0, "bf16x3": 2}[rprec]
    assert [t["prec"] for t in tr[len(tr) - refine:]] == [code] * refine
    assert all(t["prec"] == (1 if prec == "bf16" else 2) for t in tr[:len(tr) - refine])
    obs = P["mask"].astype(bool)
    assert np.array_equal(xh[obs], x0[obs])
