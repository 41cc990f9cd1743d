"""The shift-correlation Gram (the default route of hicu_gram) at the
benchmarked sizes: the whole 256 x 232 x 16-coil Gram against the explicit
oracle H'H, a 16 x 28 x 28 x 8-coil volume with a 5 x 5 x 5 kernel against
the oracle, and sampled entries of the full 256 x 320 x 320 x 8-coil volume
Gram (n = 1000) against entries computed one by one from the definition.
Bound: FP64 sums of exact products of FP32 values,
|G - G_ref| <= 2 (terms + 4) 2^-53 sum |products|."""
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
    hicu.set_gram_route(1)
    return hicu


def _gpu_gram(hc, x, kd, lo, hi):
    import torch
    return hc.gram(torch.from_numpy(np.ascontiguousarray(x)).cuda(), kd, lo, hi).cpu().numpy()


def _check_full(G, x, kd, lo, hi):
    xr = x.astype(np.complex128)
    Gr = oracle.gram(xr, kd, lo, hi)
    H = oracle.hankel_matrix(np.abs(xr), kd, lo, hi)
    bound = 2.0 * (H.shape[0] + 4) * 2.0 ** -53 * (H.T @ H).real + 1e-300
    err = np.abs(G - Gr)
    assert np.all(err <= bound), float((err / bound).max())
    assert np.array_equal(G, G.conj().T)
    return float((err / np.abs(Gr).max()).max())


def test_headline_2d_gram(hc):
    P = synth.make_problem("2d_256x232x16")
    x = P["x0"].astype(np.complex64)
    for lo, hi in [((0, 0, 0), (1, 256, 232)), synth.co_region((1, 256, 232), P["kdims"], (1, 2))]:
        print("gram 2d_256x232x16", lo, hi, flush=True)
        rel = _check_full(_gpu_gram(hc, x, P["kdims"], lo, hi), x, P["kdims"], lo, hi)
        print("max rel err", rel, flush=True)


def test_volume_crop_gram(hc):
    P = synth.make_problem("3d_16x28x28x8")
    x = P["x0"].astype(np.complex64)
    lo, hi = (0, 0, 0), x.shape[:3]
    print("gram 3d_16x28x28x8", flush=True)
    _check_full(_gpu_gram(hc, x, P["kdims"], lo, hi), x, P["kdims"], lo, hi)
    lo2, hi2 = (2, 3, 1), (14, 28, 20)
    _check_full(_gpu_gram(hc, x, P["kdims"], lo2, hi2), x, P["kdims"], lo2, hi2)


def test_full_volume_gram_sampled(hc):
    P = synth.make_problem("3d_256x320x320x8", dtype=np.complex64)
    x, kd = P["x0"], P["kdims"]
    lo, hi = (0, 0, 0), x.shape[:3]
    print("gram 3d_256x320x320x8 (full volume)", flush=True)
    G = _gpu_gram(hc, x, kd, lo, hi)
    n = G.shape[0]
    assert n == 1000
    rng = np.random.default_rng(5)
    pairs = [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (3, 5), (5, 3), (620, 621), (8 * 62, 8 * 62 + 7)]
    pairs += [(int(i), int(j)) for i, j in zip(rng.integers(0, n, 24), rng.integers(0, n, 24))]
    print("oracle entries", len(pairs), flush=True)
    ref = oracle.gram_entries(x, kd, lo, hi, pairs)
    mag = oracle.gram_entries(np.abs(x).astype(np.complex128), kd, lo, hi, pairs).real
    s = int(np.prod([h - l - k + 1 for l, h, k in zip(lo, hi, kd)]))
    for (i, j), r, mg in zip(pairs, ref, mag):
        assert abs(G[i, j] - r) <= 2.0 * (s + 4) * 2.0 ** -53 * mg + 1e-300, (i, j, G[i, j], r)
    assert np.array_equal(G, G.conj().T)
