"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hicu.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hicu_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2004_08962_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhicu.so not built: run __graft_entry__.build()")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    from paper_2004_08962_amd import _lib
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, "binding misses " + n


def _geom(dims=(1, 64, 64), nc=4, k=(1, 5, 5), lo=(0, 0, 0), hi=None):
    from paper_2004_08962_amd._lib import Geom
    g = Geom()
    g.ndim, g.nchan = 3, nc
    hi = dims if hi is None else hi
    for a in range(3):
        g.dims[a], g.kdims[a], g.lo[a], g.hi[a] = dims[a], k[a], lo[a], hi[a]
    return g


def test_counts_and_status_strings(lib):
    g = _geom()
    assert lib.hicu_num_taps(ctypes.byref(g)) == 100
    assert lib.hicu_num_outputs(ctypes.byref(g)) == 60 * 60
    assert lib.hicu_version() >= 100
    assert lib.hicu_status_string(-6) == b"workspace missing or too small"
    g2 = _geom(dims=(64, 64, 4), k=(5, 5, 1))   # trailing singleton axis is fine
    assert lib.hicu_num_taps(ctypes.byref(g2)) == 100
    # 2-D given with ndim = 2 is right-aligned internally
    g3 = _geom()
    g3.ndim = 2
    g3.dims[0], g3.dims[1], g3.kdims[0], g3.kdims[1] = 64, 64, 5, 5
    g3.lo[0] = g3.lo[1] = 0
    g3.hi[0], g3.hi[1] = 64, 64
    assert lib.hicu_num_outputs(ctypes.byref(g3)) == 3600


@pytest.mark.parametrize("kw", [
    dict(k=(1, 5, 70)),                          # kernel larger than region
    dict(lo=(0, 10, 10), hi=(1, 13, 40)),        # region smaller than kernel
    dict(hi=(1, 65, 64)),                        # region beyond array
    dict(lo=(0, -1, 0)),
])
def test_bad_geometry_rejected(lib, kw):
    g = _geom(**kw)
    assert lib.hicu_num_taps(ctypes.byref(g)) == -2
    assert lib.hicu_gram(ctypes.byref(g), None, None, None, 0, None) == -2


def test_bad_arguments_rejected_before_launch(lib):
    g = _geom()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.hicu_gram(ctypes.byref(g), None, fake, None, 0, None) == -1
    assert lib.hicu_gram(ctypes.byref(g), fake, fake, None, 0, None) == -6
    assert lib.hicu_objective_grad(ctypes.byref(g), fake, None, fake, 0, 0, None, None, None, None, 0, None) == -3
    assert lib.hicu_objective_grad(ctypes.byref(g), fake, None, fake, 8, 7, None, None, None, None, 0, None) == -1
    assert lib.hicu_objective_grad(ctypes.byref(g), fake, None, fake, 8, 0, None, fake, None, None, 0, None) == -6
    assert lib.hicu_nullspace(100, 100, fake, None, fake, None, None, None, None, 0, None) == -3
    assert lib.hicu_nullspace(100, -1, fake, None, fake, None, None, None, None, 0, None) == -3
    assert lib.hicu_nullspace(100, 30, fake, None, fake, None, None, None, None, 0, None) == -6
    assert lib.hicu_line_search(ctypes.byref(g), fake, None, fake, 8, 0, fake, None, 0, None) == -1
    assert lib.hicu_jl_compress(100, 70, 0, fake, 1, 0, 0, 0, fake, None, None) == -1


def test_workspace_sizes(lib):
    g = _geom(dims=(1, 256, 232), nc=16)
    s = 252 * 228
    for prec in (0, 1, 2, 3):
        b = lib.hicu_workspace_bytes(ctypes.byref(g), 280, prec)
        assert b >= s * 280 * 8            # holds the residual Y
        assert b < s * 280 * 8 + (64 << 20)
    assert lib.hicu_gram_workspace_bytes(ctypes.byref(g)) > 0
    assert lib.hicu_nullspace_workspace_bytes(400) >= 3 * 416 * 416 * 16
    assert lib.hicu_workspace_bytes(ctypes.byref(g), 280, 9) == 0


def _params(rank=30, steps=(5, 5), p=0, prec=0):
    from paper_2004_08962_amd._lib import Params
    prm = Params()
    st = (ctypes.c_int32 * len(steps))(*steps)
    prm.rank, prm.p, prm.n_outer, prm.start_outer = rank, p, len(steps), 0
    prm.steps = ctypes.cast(st, ctypes.POINTER(ctypes.c_int32))
    prm.regions = None
    prm.seed, prm.prec, prm.refine_steps, prm.warm_start = 0, prec, 0, 1
    return prm, st


def test_solve_workspace_is_the_callers(lib):
    """hicu_solve allocates nothing: it sizes its workspace up front and
    refuses a missing or short one before any launch."""
    g = _geom()
    prm, keep = _params()
    b = lib.hicu_solve_workspace_bytes(ctypes.byref(g), ctypes.byref(prm))
    n = 100
    assert b >= 3 * n * n * 16 + 64 * 64 * 4 * 8  # G, two eigenvector sets, the gradient
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.hicu_solve(ctypes.byref(g), fake, None, ctypes.byref(prm), fake, None, None, 0, None) == -6
    assert lib.hicu_solve(ctypes.byref(g), fake, None, ctypes.byref(prm), fake, None, fake, b - 1, None) == -6
    assert lib.hicu_solve(ctypes.byref(g), None, None, ctypes.byref(prm), fake, None, fake, b, None) == -1
    bad, keep2 = _params(rank=100)
    assert lib.hicu_solve_workspace_bytes(ctypes.byref(g), ctypes.byref(bad)) == 0
    assert lib.hicu_solve(ctypes.byref(g), fake, None, ctypes.byref(bad), fake, None, fake, b, None) == -3
    badp, keep3 = _params(prec=9)
    assert lib.hicu_solve_workspace_bytes(ctypes.byref(g), ctypes.byref(badp)) == 0
    # refinement in FP32 (default) or split BF16 only
    for rp, ok in ((0, True), (2, True), (1, False), (3, False)):
        q, keep4 = _params(prec=1)
        q.refine_steps, q.refine_prec = 3, rp
        assert (lib.hicu_solve_workspace_bytes(ctypes.byref(g), ctypes.byref(q)) > 0) == ok


def test_rsvd_workspace_and_validation(lib):
    """The rSVD route sizes its workspace from the sketch Y (s x l complex64)
    and refuses bad sketch sizes, ranks and tap counts before any launch."""
    g = _geom(dims=(1, 256, 232), nc=16)
    s, n = 252 * 228, 400
    b = lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), 120, 0)
    assert b >= s * 180 * 8 + 2 * n * 180 * 16     # Y (l = 180), W and B'
    assert b < s * 180 * 8 + (256 << 20)
    assert lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), 120, 200) > b
    assert lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), 120, 119) == 0   # l < r
    assert lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), 120, 401) == 0   # l > n
    assert lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), 400, 0) == 0     # r >= n
    assert lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), 0, 0) > 0
    big = _geom(dims=(1, 64, 64), nc=100, k=(1, 5, 5))                               # n = 2500
    assert lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(big), 10, 0) == 0
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.hicu_nullspace_rsvd(ctypes.byref(g), fake, 400, 0, 1, 0, 0, fake, None, None, fake, b, None) == -3
    assert lib.hicu_nullspace_rsvd(ctypes.byref(g), fake, 120, 100, 1, 0, 0, fake, None, None, fake, b, None) == -1
    assert lib.hicu_nullspace_rsvd(ctypes.byref(g), None, 120, 0, 1, 0, 0, fake, None, None, fake, b, None) == -1
    assert lib.hicu_nullspace_rsvd(ctypes.byref(big), fake, 10, 0, 1, 0, 0, fake, None, None, fake, b, None) == -7
    assert lib.hicu_sketch(0, 5, 1, 0, 0, fake, None) == -1
    # hicu_solve with the rSVD route keeps no Gram, eigenvectors or n x n eigensolver workspace
    g2 = _geom()
    prm, keep = _params(rank=30)
    gram_b = lib.hicu_solve_workspace_bytes(ctypes.byref(g2), ctypes.byref(prm))
    prm.route, prm.sketch = 1, 0
    rsvd_b = lib.hicu_solve_workspace_bytes(ctypes.byref(g2), ctypes.byref(prm))
    assert rsvd_b > 0
    assert rsvd_b >= lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g2), 30, 0)
    prm.sketch = 29
    assert lib.hicu_solve_workspace_bytes(ctypes.byref(g2), ctypes.byref(prm)) == 0
    prm.route, prm.sketch = 2, 0
    assert lib.hicu_solve_workspace_bytes(ctypes.byref(g2), ctypes.byref(prm)) == 0
    assert gram_b > 0


def test_tuner_workspace_and_batched_roles(lib):
    """The tuner times one filter group, so its workspace stays within a
    gradient step's even for the full volume; batched roles 2/3 accept only
    shapes with batched kernels."""
    g = _geom(dims=(256, 320, 320), nc=8, k=(5, 5, 5))
    tune = lib.hicu_autotune_workspace_bytes(ctypes.byref(g), 900, 1)
    step = lib.hicu_workspace_bytes(ctypes.byref(g), 900, 1)
    assert 0 < tune <= 2 * step
    assert tune < 20e9      # one 64-filter group of Y, not the 181 GB of all 900
    g2 = _geom()
    assert lib.hicu_tune_put(ctypes.byref(g2), 70, 1, 2, 7, 16) == -1    # shape 7 has no batched kernel
    assert lib.hicu_tune_put(ctypes.byref(g2), 70, 1, 2, 4, 16) == 0
    assert lib.hicu_tune_put(ctypes.byref(g2), 70, 1, 3, 10, 16) == -1   # packing shape, no batched kernel
    assert lib.hicu_tune_put(ctypes.byref(g2), 70, 1, 4, 4, 16) == -1    # no such role
    assert lib.hicu_tune_clear() == 0


def test_circular_axis_validation(lib):
    """A circular axis must span the whole array, and wrap bits must name
    given axes; both are refused before any launch."""
    g = _geom(dims=(9, 21, 19), nc=3, k=(3, 3, 3))
    g.wrap = 1
    assert lib.hicu_num_outputs(ctypes.byref(g)) == 9 * 19 * 17   # every frame is an output
    g.lo[0], g.hi[0] = 1, 9
    assert lib.hicu_num_taps(ctypes.byref(g)) == -2
    g2 = _geom(dims=(1, 40, 30), nc=2, k=(1, 5, 5))
    g2.ndim = 2
    g2.dims[0], g2.dims[1], g2.kdims[0], g2.kdims[1] = 40, 30, 5, 5
    g2.lo[0] = g2.lo[1] = 0
    g2.hi[0], g2.hi[1] = 40, 30
    g2.wrap = 4  # bit 2 names no axis of a 2-D geometry
    assert lib.hicu_num_taps(ctypes.byref(g2)) == -1
    g2.wrap = 2  # second given axis circular
    assert lib.hicu_num_outputs(ctypes.byref(g2)) == 36 * 30
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.hicu_time_average_init(ctypes.byref(g2), 2, fake, fake, fake, None) == -1
    assert lib.hicu_time_average_init(ctypes.byref(g2), 0, fake, None, fake, None) == -1


def test_kernel_mask_taps(lib):
    """A kernel mask keeps the taps with nonzero entries; an all-ones mask is
    the whole box; an empty or oversized one is refused."""
    import numpy as np
    g = _geom(dims=(1, 30, 30), nc=4, k=(1, 5, 5))
    c = 2.0
    a = np.arange(5)
    disc = (((a[:, None] - c) ** 2 + (a[None, :] - c) ** 2) <= 6.25).astype(np.uint8)
    g.kmask = disc.ctypes.data
    assert lib.hicu_num_taps(ctypes.byref(g)) == int(disc.sum()) * 4
    assert lib.hicu_num_outputs(ctypes.byref(g)) == 26 * 26
    ones = np.ones(25, np.uint8)
    g.kmask = ones.ctypes.data
    assert lib.hicu_num_taps(ctypes.byref(g)) == 100
    zeros = np.zeros(25, np.uint8)
    g.kmask = zeros.ctypes.data
    assert lib.hicu_num_taps(ctypes.byref(g)) == -2
    big = _geom(dims=(20, 30, 30), nc=2, k=(9, 9, 9))
    m9 = np.ones(729, np.uint8)
    big.kmask = m9.ctypes.data
    assert lib.hicu_num_taps(ctypes.byref(big)) == -7
