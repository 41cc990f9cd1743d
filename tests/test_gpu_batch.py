"""Batched persistent launches, HIP-graph capture and the autotuner.

* One batch of uneven 2-D problems (different sizes, coil counts, kernels,
  regions, with and without JL) stepped together equals the same steps run
  problem by problem with the single-problem entry points, bit for bit, when
  both use the same tile shapes.
* A graph of captured batch steps, replayed several times with eager work in
  between, reproduces the eager batch steps bit for bit.
* The autotuner picks a valid shape and the tuned plans still meet the
  oracle's rounding bounds; its cache round-trips through a file.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import forward_bound, grad_bound, sumsq_bound

pytestmark = pytest.mark.gpu

SHAPES = [  # (D1, D2, coils, kernel, region or None, JL filters or 0)
    (40, 52, 3, (1, 5, 5), None, 0),
    (67, 45, 5, (1, 5, 5), ((0, 10, 8), (1, 50, 40)), 4),
    (33, 33, 8, (1, 3, 3), None, 0),
    (90, 71, 4, (1, 5, 5), None, 6),
    (28, 60, 6, (1, 4, 3), None, 0),
    (55, 55, 2, (1, 5, 5), None, 3),
]
STEPS = 3


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2004_08962_amd as hicu
    from paper_2004_08962_amd import batch as hb
    assert torch.cuda.is_available()
    rng = np.random.default_rng(2024)
    probs = []
    for i, (d1, d2, nc, kd, reg, pjl) in enumerate(SHAPES):
        img = synth.ellipse_image((d1, d2), 5, rng)
        maps = synth.gaussian_coil_maps((d1, d2), nc, rng)
        x = synth.to_kspace(img, maps)[None].astype(np.complex64)
        mask = synth.line_mask((1, d1, d2), 2, synth.vd_lines(d2, d2 // 3, 4, rng))
        x0 = x * mask[..., None]
        lo, hi = reg if reg else ((0, 0, 0), (1, d1, d2))
        n = kd[0] * kd[1] * kd[2] * nc
        r = int(round(0.3 * n))
        Q, _, _ = oracle.nullspace(oracle.gram(x0.astype(np.complex128), kd, lo, hi), r)
        probs.append(dict(x0=x0, mask=mask, kd=kd, lo=lo, hi=hi, Q=Q.astype(np.complex64),
                          p=pjl if pjl else n - r, seed=100 + i))
    yield hicu, hb, torch, probs
    hb.tune_clear()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _make_batch(hb, torch, probs, prec):
    items = [dict(x=_dev(torch, p["x0"]), mask=_dev(torch, p["mask"]), Q=_dev(torch, p["Q"]), p=p["p"],
                  kdims=p["kd"], lo=p["lo"], hi=p["hi"], seed=p["seed"]) for p in probs]
    return hb.Batch(items, prec=prec), items


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_equals_single_problem_steps(env, prec):
    hicu, hb, torch, probs = env
    b, items = _make_batch(hb, torch, probs, prec)
    info = b.info()
    print("batch", info, flush=True)
    tf, ta = info["fwd_tile"], info["adj_tile"]
    # pin the single-problem plans to the batch's shared tile shapes
    for p in probs:
        hb.tune_put(p["x0"].shape, p["kd"], p["p"], prec, 0, tf, p["x0"].shape[3], p["lo"], p["hi"])
        hb.tune_put(p["x0"].shape, p["kd"], p["p"], prec, 1, ta, min(16, p["p"]), p["lo"], p["hi"])
    for _ in range(STEPS):
        b.step()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        x = _dev(torch, p["x0"])
        md = _dev(torch, p["mask"])
        Q = _dev(torch, p["Q"])
        for j in range(STEPS):
            F = Q if p["p"] == Q.shape[1] else hicu.jl_compress(Q, p["p"], p["seed"], 0, j, stream_id=i)
            J, g, gn2 = hicu.objective_grad(x, md, F, p["kd"], p["lo"], p["hi"], prec=prec)
            eta = hicu.line_search(g, gn2, F, p["kd"], p["lo"], p["hi"], prec=prec)
            hicu.update(x, g, eta)
        torch.cuda.synchronize()
        assert torch.equal(items[i]["x"], x), "problem %d" % i
        sc = b.scalars[i].cpu().numpy()
        assert sc[0] == J.item() and sc[1] == gn2.item() and sc[2] == eta.item(), (i, sc)
    hb.tune_clear()
    b.close()


def test_graph_replay_equals_eager(env):
    hicu, hb, torch, probs = env
    b, items = _make_batch(hb, torch, probs, "fp32")
    for _ in range(STEPS):
        b.step()
    torch.cuda.synchronize()
    eager = [it["x"].clone() for it in items]
    eager_sc = b.scalars.clone()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    b.capture(STEPS, side)
    for rep in range(3):
        for it, p in zip(items, probs):
            it["x"].copy_(_dev(torch, p["x0"]))   # eager work between replays
        b.set_counter(0, 0)
        b.scalars.zero_()
        torch.cuda.synchronize()
        b.replay(side)
        side.synchronize()
        for it, e in zip(items, eager):
            assert torch.equal(it["x"], e), "replay %d" % rep
        assert torch.equal(b.scalars, eager_sc)
    b.close()


def test_autotune_and_cache(env, tmp_path):
    hicu, hb, torch, probs = env
    P = synth.make_problem("2d_64x64x4")
    x = P["x0"].astype(np.complex64)
    kd, lo, hi = P["kdims"], (0, 0, 0), (1, 64, 64)
    Q, _, _ = oracle.nullspace(oracle.gram(x.astype(np.complex128), kd, lo, hi), P["rank"])
    F = Q.astype(np.complex64)
    hb.tune_clear()
    choice = hb.autotune(_dev(torch, x), _dev(torch, F), kd, lo, hi, prec="fp32")
    print("tuned", choice, [hb.tile_info(t) for t in (choice[0], choice[2])], flush=True)
    assert 0 <= choice[0] < hb.tile_count() and 0 <= choice[2] < hb.tile_count()
    assert hb.tile_info(choice[0])[0] == 1 and hb.tile_info(choice[0])[4] == 1  # 2-D: T0 = 1, no packing
    assert hb.tile_info(choice[2])[0] == 1 and choice[1] == 4 and choice[3] in (4, 8, 16)
    J, g, gn2 = hicu.objective_grad(_dev(torch, x), _dev(torch, P["mask"]), _dev(torch, F), kd, lo, hi)
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    Jr, gr, _ = oracle.objective_grad(xr, P["mask"], Fr, kd, lo, hi)
    Y, eY = forward_bound(xr, Fr, kd, lo, hi, "fp32")
    assert abs(J.item() - Jr) <= sumsq_bound(Y, eY)
    eg = grad_bound(xr, P["mask"], Fr, kd, lo, hi, "fp32")
    assert np.all(np.abs(g.cpu().numpy() - gr) <= eg + 1e-30)
    path = tmp_path / "tune.txt"
    hb.tune_save(path)
    hb.tune_clear()
    assert hb.tune_load(path) == 2
    hb.tune_clear()


def test_batched_autotune_drives_the_batch(env):
    """hicu_autotune_batched on the problem with the most work: the batch
    then runs the tuned shapes (batched kernels only) and still equals the
    single-problem steps on those shapes."""
    hicu, hb, torch, probs = env
    hb.tune_clear()
    big = max(range(len(probs)), key=lambda i: hicu.num_taps(probs[i]["x0"].shape, probs[i]["kd"]) * probs[i]["p"]
              * int(np.prod([h - l - k + 1 for l, h, k in zip(probs[i]["lo"], probs[i]["hi"], probs[i]["kd"])])))
    P = probs[big]
    F = P["Q"][:, :P["p"]]
    choice = hb.autotune(_dev(torch, P["x0"]), _dev(torch, np.ascontiguousarray(F)), P["kd"], P["lo"], P["hi"],
                         prec="bf16", batched=True)
    print("batched choice", choice, flush=True)
    batched_tiles = {0, 1, 2, 3, 4, 5, 9, 13, 14, 15}  # the tuner skips the batched k-split shapes
    assert choice[0] in batched_tiles and choice[2] in batched_tiles
    b, items = _make_batch(hb, torch, probs, "bf16")
    info = b.info()
    assert (info["fwd_tile"], info["adj_tile"]) == (choice[0], choice[2])
    b.close()
    # the single-problem cache (roles 0/1) is untouched by the batched tuning
    hb.tune_clear()
    with pytest.raises(Exception):
        hb.tune_put(P["x0"].shape, P["kd"], P["p"], "bf16", 2, 7, 16, P["lo"], P["hi"])  # no batched kernel
    hb.tune_put(P["x0"].shape, P["kd"], P["p"], "bf16", 2, 4, 16, P["lo"], P["hi"])
    hb.tune_clear()


def test_autotune_under_filter_groups(env):
    """With a tiny residual budget the gradient runs in filter groups; the
    tuner times one group (its workspace holds one group's Y) and the tuned
    plans keep the oracle's rounding bounds."""
    hicu, hb, torch, probs = env
    P = synth.make_problem("2d_64x64x4")
    x = P["x0"].astype(np.complex64)
    kd, lo, hi = P["kdims"], (0, 0, 0), (1, 64, 64)
    Q, _, _ = oracle.nullspace(oracle.gram(x.astype(np.complex128), kd, lo, hi), P["rank"])
    F = np.ascontiguousarray(Q.astype(np.complex64))
    p = F.shape[1]
    s = 60 * 60
    try:
        hicu.set_filter_group_budget(s * 64 * 8)     # groups of 64 filters
        assert hicu.filter_group(x.shape, kd, p)[0] == 64
        hb.tune_clear()
        choice = hb.autotune(_dev(torch, x), _dev(torch, F), kd, lo, hi, prec="bf16")
        J, g, gn2 = hicu.objective_grad(_dev(torch, x), _dev(torch, P["mask"]), _dev(torch, F), kd, lo, hi,
                                        prec="bf16")
    finally:
        hicu.set_filter_group_budget(0)
        hb.tune_clear()
    assert 0 <= choice[0] < hb.tile_count() and 0 <= choice[2] < hb.tile_count()
    xr, Fr = x.astype(np.complex128), F.astype(np.complex128)
    Jr, gr, _ = oracle.objective_grad(xr, P["mask"], Fr, kd, lo, hi)
    Y, eY = forward_bound(xr, Fr, kd, lo, hi, "bf16")
    assert abs(J.item() - Jr) <= sumsq_bound(Y, eY)
    eg = grad_bound(xr, P["mask"], Fr, kd, lo, hi, "bf16", groups=2)
    assert np.all(np.abs(g.cpu().numpy() - gr) <= eg + 1e-30)
