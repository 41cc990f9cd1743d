"""hicu_line_search_noalloc (the line search on the library's fixed device
scratch, for callers that cannot allocate) against hicu_line_search with a
caller workspace: same eta, bit for bit, on two calls in a row with the
second on a smaller problem, and sizes beyond the scratch refused."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2004_08962_amd as hicu
    from paper_2004_08962_amd import _lib
    assert torch.cuda.is_available()
    lib = hicu.load()
    return hicu, _lib, lib, torch


def _problem(torch, hicu, shape, kd, p, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    n = kd[0] * kd[1] * kd[2] * shape[3]
    F = ((rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / np.sqrt(n)).astype(np.complex64)
    xd, Fd = torch.from_numpy(x).cuda(), torch.from_numpy(F).cuda()
    J, g, gn2 = hicu.objective_grad(xd, None, Fd, kd)
    return g, gn2, Fd


def _noalloc(lib, _lib, torch, g, gn2, F, kd, prec):
    from paper_2004_08962_amd.api import _prec, _stream, geom
    eta = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    st = lib.hicu_line_search_noalloc(ctypes.byref(geom(g.shape, kd)), ctypes.c_void_p(g.data_ptr()),
                                      ctypes.c_void_p(gn2.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                      F.shape[1], _prec(prec), ctypes.c_void_p(eta.data_ptr()), _stream())
    return st, eta


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_noalloc_line_search_matches_workspace_entry(env, prec):
    hicu, _lib, lib, torch = env
    cases = [((1, 96, 80, 8), (1, 5, 5), 120, 1), ((6, 20, 24, 4), (3, 3, 3), 40, 2)]  # second one smaller
    for shape, kd, p, seed in cases:
        print("noalloc line search", prec, shape, kd, p, flush=True)
        g, gn2, F = _problem(torch, hicu, shape, kd, p, seed)
        ref = hicu.line_search(g, gn2, F, kd, prec=prec)
        st, eta = _noalloc(lib, _lib, torch, g, gn2, F, kd, prec)
        torch.cuda.synchronize()
        assert st == 0, _lib.STATUS.get(st)
        assert eta.item() > 0
        assert eta.item() == ref.item(), (eta.item(), ref.item())


def test_noalloc_refuses_beyond_scratch(env):
    hicu, _lib, lib, torch = env
    cap = lib.hicu_line_search_noalloc_max_bytes()
    assert cap == 64 << 20
    # 8192 filters over 1000 taps: the FP32 weights alone (2n x 2p floats,
    # 131 MB) exceed the scratch
    shape, kd, p = (1, 24, 24, 40), (1, 5, 5), 8192
    assert hicu.workspace_bytes(shape, kd, p, "fp32") > cap
    g = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    gn2 = torch.ones((), dtype=torch.float64, device="cuda")
    F = torch.zeros((1000, p), dtype=torch.complex64, device="cuda")
    st, eta = _noalloc(lib, _lib, torch, g, gn2, F, kd, "fp32")
    torch.cuda.synchronize()
    assert st == -6
    assert eta.item() == -1.0  # nothing written
