"""Every instantiated tile shape of the contraction kernels, pinned through
the tuning cache, against the FP64 oracle's rounding bounds: the forward
(J) for each shape without axis-2 packing, the adjoint (g, ||g||^2) for
every shape, in all three precisions, on a ragged 2-D problem and a ragged
3-D problem with a region and a mask (several tiles along every axis and
partial tiles at the ends)."""
import numpy as np
import pytest

import oracle
from bounds import forward_bound, grad_bound, sumsq_bound

pytestmark = pytest.mark.gpu

PROBLEMS = {
    # name: (shape, kdims, lo, hi, p)
    "2d": ((1, 45, 77, 6), (1, 5, 5), (0, 0, 0), (1, 45, 77), 37),
    "3d": ((11, 37, 41, 3), (3, 4, 5), (1, 2, 0), (11, 36, 41), 21),
}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2004_08962_amd as hicu
    from paper_2004_08962_amd import batch as hb
    assert torch.cuda.is_available()
    out = {}
    for name, (shape, kd, lo, hi, p) in PROBLEMS.items():
        rng = np.random.default_rng(7)
        x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
        mask = (rng.random(shape[:3]) < 0.3).astype(np.uint8)
        n = kd[0] * kd[1] * kd[2] * shape[3]
        F = ((rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(n)).astype(np.complex64)
        xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
        Jr, gr, _ = oracle.objective_grad(xr, mask, Fr, kd, lo, hi)
        bounds = {}
        for prec in ("fp32", "bf16", "bf16x3", "fp16"):
            Y, eY = forward_bound(xr, Fr, kd, lo, hi, prec)
            bounds[prec] = (sumsq_bound(Y, eY), grad_bound(xr, mask, Fr, kd, lo, hi, prec))
        out[name] = dict(x=x, mask=mask, F=F, kd=kd, lo=lo, hi=hi, p=p, Jr=Jr, gr=gr, bounds=bounds)
    yield hicu, hb, torch, out
    hb.tune_clear()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp16"])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_every_tile_shape(env, name, prec):
    hicu, hb, torch, probs = env
    P = probs[name]
    x, mask, F = _dev(torch, P["x"]), _dev(torch, P["mask"]), _dev(torch, P["F"])
    bJ, bg = P["bounds"][prec]
    checked = 0
    for tile in range(hb.tile_count()):
        T0, T2, WC, FN, D, KS = hb.tile_info(tile)
        if name == "2d" and T0 > 1:
            continue
        hb.tune_clear()
        if D == 1:
            hb.tune_put(P["x"].shape, P["kd"], P["p"], prec, 0, tile, P["x"].shape[3], P["lo"], P["hi"])
        for chunk in (16, 4):
            hb.tune_put(P["x"].shape, P["kd"], P["p"], prec, 1, tile, chunk, P["lo"], P["hi"])
            print(name, prec, "tile", tile, (T0, T2, WC, FN, D, KS), "chunk", chunk, flush=True)
            J, g, gn2 = hicu.objective_grad(x, mask, F, P["kd"], P["lo"], P["hi"], prec=prec)
            gh = g.cpu().numpy().astype(np.complex128)
            assert abs(J.item() - P["Jr"]) <= bJ, (tile, chunk)
            assert np.all(np.abs(gh - P["gr"]) <= bg + 1e-30), (tile, chunk)
            assert abs(gn2.item() - float(np.vdot(gh, gh).real)) <= 1e-5 * gn2.item()
            checked += 1
    hb.tune_clear()
    assert checked >= 20


def test_every_volume_tile_compact_residual():
    """Filter groups on a 3-D problem make the BF16 path store the residual
    as BF16 in filter blocks (ragged last block) and stage it with batched
    loads: every shape with several planes, both chunk widths, against the
    oracle's bounds."""
    import torch
    import paper_2004_08962_amd as hicu
    from paper_2004_08962_amd import batch as hb
    shape, kd, lo, hi, p = (10, 23, 26, 3), (3, 3, 3), (0, 1, 0), (10, 23, 25), 70
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mask = (rng.random(shape[:3]) < 0.3).astype(np.uint8)
    n = kd[0] * kd[1] * kd[2] * shape[3]
    F = ((rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(n)).astype(np.complex64)
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    Jr, gr, _ = oracle.objective_grad(xr, mask, Fr, kd, lo, hi)
    Y, eY = forward_bound(xr, Fr, kd, lo, hi, "bf16")
    bJ = sumsq_bound(Y, eY)
    bg = grad_bound(xr, mask, Fr, kd, lo, hi, "bf16", groups=2)
    s = int(np.prod([h - l - k + 1 for l, h, k in zip(lo, hi, kd)]))
    xd, md, Fd = (torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (x, mask, F))
    checked = 0
    hicu.set_filter_group_budget(s * 4 * 64)  # groups of 64 + 6 filters
    try:
        for tile in range(hb.tile_count()):
            T0, T2, WC, FN, D, KS = hb.tile_info(tile)
            if T0 == 1:
                continue
            for chunk in (8, 4):
                hb.tune_clear()
                hb.tune_put(shape, kd, p, "bf16", 1, tile, chunk, lo, hi)
                print("compact residual, tile", tile, (T0, T2, WC, FN, D, KS), "chunk", chunk, flush=True)
                J, g, gn2 = hicu.objective_grad(xd, md, Fd, kd, lo, hi, prec="bf16")
                gh = g.cpu().numpy().astype(np.complex128)
                assert abs(J.item() - Jr) <= bJ, (tile, chunk)
                assert np.all(np.abs(gh - gr) <= bg + 1e-30), (tile, chunk)
                assert abs(gn2.item() - float(np.vdot(gh, gh).real)) <= 1e-5 * gn2.item()
                checked += 1
    finally:
        hb.tune_clear()
        hicu.set_filter_group_budget(0)
    assert checked >= 30
