"""Thin torch-facing binding of libhicu.so: argument marshalling only.

Every array is a CUDA (HIP) torch tensor on the current device; k-space is
complex64 of shape (D0, D1, D2, Nc) (2-D data with D0 = 1), masks uint8 of
shape (D0, D1, D2).  Work is enqueued on torch's current stream.  All
arithmetic happens in the library's HIP kernels.
"""
import ctypes

import torch

from ._lib import Geom, Params, Trace, PREC, check, load


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _taps(kdims):
    """Taps of a kernel box (3 extents) or of a kernel mask (3-D array)."""
    if hasattr(kdims, "ndim") and kdims.ndim == 3:
        return int((kdims != 0).sum())
    return int(kdims[0]) * int(kdims[1]) * int(kdims[2])


def _shape_checks(x_shape=None, kdims=None, F=None, mask=None, like=None, like_name="g"):
    """Shape agreement between the arguments, checked before any device
    pointer is handed to the library (a mismatched buffer would be read or
    written out of bounds by the kernels)."""
    if x_shape is not None and len(x_shape) != 4:
        raise ValueError("k-space must have shape (D0, D1, D2, Nc), got %s" % (tuple(x_shape),))
    if F is not None:
        if F.dim() != 2:
            raise ValueError("F must be 2-D (n, p), got %s" % (tuple(F.shape),))
        if x_shape is not None and kdims is not None:
            n = _taps(kdims) * int(x_shape[3])
            if F.shape[0] != n:
                raise ValueError("F has %d rows; the kernel over %d coils has %d taps"
                                 % (F.shape[0], int(x_shape[3]), n))
    if mask is not None and x_shape is not None and tuple(mask.shape) != tuple(x_shape[:3]):
        raise ValueError("mask shape %s does not match k-space %s" % (tuple(mask.shape), tuple(x_shape[:3])))
    if like is not None and x_shape is not None and tuple(like.shape) != tuple(x_shape):
        raise ValueError("%s shape %s does not match x %s" % (like_name, tuple(like.shape), tuple(x_shape)))


def _wrap_bits(wrap):
    if wrap is None:
        return 0
    return sum(1 << a for a in range(3) if wrap[a])


def geom(shape, kdims, lo=None, hi=None, wrap=None):
    """hicu_geom for x of shape (D0, D1, D2, Nc) and a 3-axis kernel box, or a
    3-D kernel mask array (nonzero = tap, the box is its shape); ``wrap``:
    three flags, circular convolution along those axes."""
    import numpy as np
    d = [int(v) for v in shape[:3]]
    g = Geom()
    if hasattr(kdims, "ndim") and kdims.ndim == 3:
        km = np.ascontiguousarray(np.asarray(kdims) != 0, dtype=np.uint8)
        g._kmask_ref = km  # kept alive with the struct
        g.kmask = km.ctypes.data
        kdims = km.shape
    g.ndim = 3
    g.nchan = int(shape[3])
    lo = (0, 0, 0) if lo is None else lo
    hi = d if hi is None else hi
    for a in range(3):
        g.dims[a] = d[a]
        g.kdims[a] = int(kdims[a])
        g.lo[a] = int(lo[a])
        g.hi[a] = int(hi[a])
    g.wrap = _wrap_bits(wrap)
    return g


def _prec(p):
    if isinstance(p, str):
        return PREC[p]
    return int(p)


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def num_taps(shape, kdims):
    return int(load().hicu_num_taps(ctypes.byref(geom(shape, kdims))))


def gram(x, kdims, lo=None, hi=None, wrap=None):
    """G = H_S(x)' H_S(x) as complex128 (n, n)."""
    _shape_checks(x.shape)
    lib = load()
    _dev(x, torch.complex64, "x")
    g = geom(x.shape, kdims, lo, hi, wrap)
    n = int(lib.hicu_num_taps(ctypes.byref(g)))
    check(n, "hicu_num_taps")
    G = torch.empty((n, n), dtype=torch.complex128, device=x.device)
    wsb = lib.hicu_gram_workspace_bytes(ctypes.byref(g))
    ws = _workspace(wsb, x.device)
    check(lib.hicu_gram(ctypes.byref(g), _ptr(x), _ptr(G), _ptr(ws), wsb, _stream()), "hicu_gram")
    return G


def set_gram_route(route):
    """1: shift-correlation Gram (default), 0: direct products (both FP64)."""
    check(load().hicu_set_gram_route(int(route)), "hicu_set_gram_route")


def nullspace(G, rank, V0=None, want_V=True):
    """Returns (Q complex64 (n, n-r), evals float64 (n,), V complex128 or None, sweeps)."""
    if G.dim() != 2 or G.shape[0] != G.shape[1]:
        raise ValueError("G must be square, got %s" % (tuple(G.shape),))
    n = G.shape[0]
    if V0 is not None and tuple(V0.shape) != (n, n):
        raise ValueError("V0 must be %d x %d, got %s" % (n, n, tuple(V0.shape)))
    if not 0 <= int(rank) < n:
        raise ValueError("rank %d outside [0, %d)" % (int(rank), n))
    lib = load()
    _dev(G, torch.complex128, "G")
    if V0 is not None:
        _dev(V0, torch.complex128, "V0")
    Q = torch.empty((n, n - rank), dtype=torch.complex64, device=G.device)
    ev = torch.empty((n,), dtype=torch.float64, device=G.device)
    V = torch.empty((n, n), dtype=torch.complex128, device=G.device) if want_V else None
    sweeps = ctypes.c_int32(0)
    wsb = lib.hicu_nullspace_workspace_bytes(n)
    ws = _workspace(wsb, G.device)
    check(lib.hicu_nullspace(n, int(rank), _ptr(G), _ptr(V0), _ptr(Q), _ptr(ev), _ptr(V), ctypes.byref(sweeps),
                             _ptr(ws), wsb, _stream()), "hicu_nullspace")
    return Q, ev, V, int(sweeps.value)


def nullspace_rsvd(x, kdims, rank, ell=0, seed=0, outer=0, stream_id=0, lo=None, hi=None, wrap=None,
                   want_sv=False):
    """Q (complex64 (n, n - rank)) by randomized SVD of H_S(x) and Householder
    completion; with want_sv also the sketched B's singular values
    (float64 (l,), largest first) and the Jacobi sweeps.  ``ell`` = 0 takes
    ceil(3 rank / 2) sketch columns."""
    _shape_checks(x.shape)
    lib = load()
    _dev(x, torch.complex64, "x")
    g = geom(x.shape, kdims, lo, hi, wrap)
    n = int(lib.hicu_num_taps(ctypes.byref(g)))
    check(n, "hicu_num_taps")
    if not 0 <= int(rank) < n:
        raise ValueError("rank %d outside [0, %d)" % (int(rank), n))
    wsb = int(lib.hicu_nullspace_rsvd_workspace_bytes(ctypes.byref(g), int(rank), int(ell)))
    if wsb == 0:
        raise ValueError("invalid rSVD arguments (sketch size %d, rank %d, n %d)" % (int(ell), int(rank), n))
    ws = _workspace(wsb, x.device)
    l = int(ell) if ell else min(n, (3 * int(rank) + 1) // 2)
    Q = torch.empty((n, n - int(rank)), dtype=torch.complex64, device=x.device)
    sv = torch.empty((max(l, 1),), dtype=torch.float64, device=x.device) if want_sv else None
    sweeps = ctypes.c_int32(0)
    check(lib.hicu_nullspace_rsvd(ctypes.byref(g), _ptr(x), int(rank), int(ell), int(seed), int(outer),
                                  int(stream_id), _ptr(Q), _ptr(sv), ctypes.byref(sweeps), _ptr(ws), wsb,
                                  _stream()), "hicu_nullspace_rsvd")
    return (Q, sv[:l] if int(rank) > 0 else sv[:0], int(sweeps.value)) if want_sv else Q


def sketch(n, ell, seed, outer, stream_id=0, device="cuda"):
    """The rSVD test matrix Omega (complex64 (n, ell)) drawn on the device."""
    Om = torch.empty((int(n), int(ell)), dtype=torch.complex64, device=device)
    check(load().hicu_sketch(int(n), int(ell), int(seed), int(outer), int(stream_id), _ptr(Om), _stream()),
          "hicu_sketch")
    return Om


def jl_compress(Q, p, seed, outer, inner, stream_id=0, return_P=False):
    """F = Q P with P drawn on the device (Philox4x32-10 + Box-Muller)."""
    if Q.dim() != 2:
        raise ValueError("Q must be 2-D (n, nq), got %s" % (tuple(Q.shape),))
    lib = load()
    _dev(Q, torch.complex64, "Q")
    n, nq = Q.shape
    F = torch.empty((n, p), dtype=torch.complex64, device=Q.device)
    P = torch.empty((nq, p), dtype=torch.float64, device=Q.device) if return_P else None
    check(lib.hicu_jl_compress(n, nq, int(p), _ptr(Q), int(seed), int(outer), int(inner), int(stream_id),
                               _ptr(F), _ptr(P), _stream()), "hicu_jl_compress")
    return (F, P) if return_P else F


def set_filter_group_budget(nbytes):
    """Byte budget of Y = H(x)F above which the gradient runs over filter
    groups (0 restores the default)."""
    check(load().hicu_set_filter_group_budget(int(nbytes)), "hicu_set_filter_group_budget")


def filter_group(shape, kdims, p, prec="fp32", lo=None, hi=None, wrap=None):
    """(filters per group of the gradient, whether Y is the compact BF16 residual)."""
    f, c = ctypes.c_int32(0), ctypes.c_int32(0)
    check(load().hicu_filter_group(ctypes.byref(geom(shape, kdims, lo, hi, wrap)), int(p), _prec(prec), ctypes.byref(f),
                                   ctypes.byref(c)), "hicu_filter_group")
    return int(f.value), bool(c.value)


def workspace_bytes(shape, kdims, p, prec="fp32", lo=None, hi=None, wrap=None):
    return int(load().hicu_workspace_bytes(ctypes.byref(geom(shape, kdims, lo, hi, wrap)), int(p), _prec(prec)))


def objective_grad(x, mask, F, kdims, lo=None, hi=None, prec="fp32", want_grad=True, ws=None, wrap=None):
    """Returns (J, g, gnorm2): J and gnorm2 are 0-dim float64 CUDA tensors,
    g complex64 like x (None when want_grad is False)."""
    _shape_checks(x.shape, kdims, F, mask)
    lib = load()
    _dev(x, torch.complex64, "x")
    _dev(F, torch.complex64, "F")
    if mask is not None:
        _dev(mask, torch.uint8, "mask")
    g = geom(x.shape, kdims, lo, hi, wrap)
    p = F.shape[1]
    wsb = lib.hicu_workspace_bytes(ctypes.byref(g), p, _prec(prec))
    if wsb == 0:
        raise ValueError("unsupported geometry / filter count")
    ws = _workspace(wsb, x.device) if ws is None else ws
    J = torch.empty((), dtype=torch.float64, device=x.device)
    gout = torch.empty_like(x) if want_grad else None
    gn2 = torch.empty((), dtype=torch.float64, device=x.device) if want_grad else None
    check(lib.hicu_objective_grad(ctypes.byref(g), _ptr(x), _ptr(mask), _ptr(F), p, _prec(prec), _ptr(J), _ptr(gout),
                                  _ptr(gn2), _ptr(ws), ws.numel(), _stream()), "hicu_objective_grad")
    return J, gout, gn2


def line_search(gv, gnorm2, F, kdims, lo=None, hi=None, prec="fp32", ws=None, wrap=None):
    """eta = ||g||^2 / (2 ||H(g) F||^2) as a 0-dim float64 CUDA tensor."""
    _shape_checks(gv.shape, kdims, F)
    if gnorm2.numel() != 1:
        raise ValueError("gnorm2 must hold one value")
    lib = load()
    _dev(gv, torch.complex64, "g")
    _dev(F, torch.complex64, "F")
    _dev(gnorm2, torch.float64, "gnorm2")
    g = geom(gv.shape, kdims, lo, hi, wrap)
    p = F.shape[1]
    wsb = lib.hicu_workspace_bytes(ctypes.byref(g), p, _prec(prec))
    ws = _workspace(wsb, gv.device) if ws is None else ws
    eta = torch.empty((), dtype=torch.float64, device=gv.device)
    check(lib.hicu_line_search(ctypes.byref(g), _ptr(gv), _ptr(gnorm2), _ptr(F), p, _prec(prec), _ptr(eta),
                               _ptr(ws), ws.numel(), _stream()), "hicu_line_search")
    return eta


def update(x, gv, eta, kdims=(1, 1, 1)):
    """In place: x <- x - eta g (x unchanged when eta is 0 or not finite)."""
    _shape_checks(x.shape, like=gv)
    if eta.numel() != 1:
        raise ValueError("eta must hold one value")
    lib = load()
    _dev(x, torch.complex64, "x")
    _dev(gv, torch.complex64, "g")
    _dev(eta, torch.float64, "eta")
    g = geom(x.shape, kdims)
    check(lib.hicu_update(ctypes.byref(g), _ptr(x), _ptr(gv), _ptr(eta), _stream()), "hicu_update")
    return x


_ROUTES = {"gram": 0, "rsvd": 1}


def _route(route):
    if route not in _ROUTES:
        raise ValueError("route must be 'gram' or 'rsvd', got %r" % (route,))
    return _ROUTES[route]


def solve(x0, mask, kdims, rank, schedule, p=0, seed=0, prec="fp32", refine_steps=0, warm_start=True,
          start_outer=0, out=None, ws=None, raise_nonfinite=True, wrap=None, route="gram", ell=0,
          refine_prec="fp32"):
    """Algorithm 1 on the device.  ``schedule``: list of (lo, hi, steps).
    The last ``refine_steps`` steps run in ``refine_prec`` ("fp32" or "bf16x3").
    ``route``: nullspace update by the Gram eigendecomposition ("gram") or by
    randomized SVD + Householder ("rsvd", ``ell`` sketch columns, 0 =
    ceil(3 rank / 2)).
    Returns (x, trace) with trace a list of dicts (one per gradient step).
    ``ws``: optional uint8 CUDA workspace of at least solve_workspace_bytes()
    bytes (allocated here otherwise).  With raise_nonfinite=False a run that
    stops on a non-finite value returns (x, trace, status) instead of raising."""
    _shape_checks(x0.shape, mask=mask, like=out, like_name="out")
    lib = load()
    _dev(x0, torch.complex64, "x0")
    if mask is not None:
        _dev(mask, torch.uint8, "mask")
    g = geom(x0.shape, kdims, wrap=wrap)
    n_outer = len(schedule)
    steps = (ctypes.c_int32 * max(1, n_outer))(*[int(s[2]) for s in schedule])
    regs = (ctypes.c_int64 * max(1, 6 * n_outer))(
        *[int(v) for (lo, hi, _) in schedule for v in list(lo) + list(hi)])
    prm = Params()
    prm.rank = int(rank)
    prm.p = int(p)
    prm.n_outer = n_outer
    prm.start_outer = int(start_outer)
    prm.steps = ctypes.cast(steps, ctypes.POINTER(ctypes.c_int32))
    prm.regions = ctypes.cast(regs, ctypes.POINTER(ctypes.c_int64))
    prm.seed = int(seed)
    prm.prec = _prec(prec)
    prm.refine_steps = int(refine_steps)
    prm.warm_start = 1 if warm_start else 0
    prm.route = _route(route)
    prm.sketch = int(ell)
    prm.refine_prec = _prec(refine_prec)
    total = sum(int(s[2]) for s in schedule[start_outer:])
    tr = (Trace * max(1, total))()
    x = torch.empty_like(x0) if out is None else out
    wsb = int(lib.hicu_solve_workspace_bytes(ctypes.byref(g), ctypes.byref(prm)))
    if wsb == 0:
        raise ValueError("invalid solve arguments (geometry, rank, schedule or precision)")
    if ws is None or ws.numel() < wsb:
        ws = _workspace(wsb, x0.device)
    st = lib.hicu_solve(ctypes.byref(g), _ptr(x0), _ptr(mask), ctypes.byref(prm), _ptr(x), tr, _ptr(ws), ws.numel(),
                        _stream())
    trace = [dict(outer=t.outer, inner=t.inner, prec=t.prec, sweeps=t.sweeps, J=t.J, gnorm2=t.gnorm2, eta=t.eta)
             for t in tr[:total]]
    if st == -4 and not raise_nonfinite:
        return x, trace, st
    check(st, "hicu_solve")
    return x, trace


def solve_workspace_bytes(shape, kdims, rank, schedule, p=0, prec="fp32", refine_steps=0, start_outer=0, wrap=None,
                          route="gram", ell=0, refine_prec="fp32"):
    """Device bytes hicu_solve needs for this problem and schedule."""
    g = geom(shape, kdims, wrap=wrap)
    n_outer = len(schedule)
    steps = (ctypes.c_int32 * max(1, n_outer))(*[int(s[2]) for s in schedule])
    regs = (ctypes.c_int64 * max(1, 6 * n_outer))(
        *[int(v) for (lo, hi, _) in schedule for v in list(lo) + list(hi)])
    prm = Params()
    prm.rank, prm.p, prm.n_outer, prm.start_outer = int(rank), int(p), n_outer, int(start_outer)
    prm.steps = ctypes.cast(steps, ctypes.POINTER(ctypes.c_int32))
    prm.regions = ctypes.cast(regs, ctypes.POINTER(ctypes.c_int64))
    prm.prec, prm.refine_steps = _prec(prec), int(refine_steps)
    prm.route, prm.sketch, prm.refine_prec = _route(route), int(ell), _prec(refine_prec)
    return int(load().hicu_solve_workspace_bytes(ctypes.byref(g), ctypes.byref(prm)))


def time_average_init(x0, mask, axis=0, out=None):
    """Study II initialisation: unobserved samples take the mean over frames
    (axis ``axis`` of (D0, D1, D2)) of the observed samples at the same
    location and coil; locations never observed stay zero."""
    _shape_checks(x0.shape, mask=mask, like=out, like_name="out")
    if mask is None:
        raise ValueError("time_average_init needs the sampling mask")
    lib = load()
    _dev(x0, torch.complex64, "x0")
    _dev(mask, torch.uint8, "mask")
    out = torch.empty_like(x0) if out is None else _dev(out, torch.complex64, "out")
    g = geom(x0.shape, (1, 1, 1))
    check(lib.hicu_time_average_init(ctypes.byref(g), int(axis), _ptr(x0), _ptr(mask), _ptr(out), _stream()),
          "hicu_time_average_init")
    return out


def profile_begin(minor=True):
    """Start per-kernel event timing (every library launch, on its stream);
    minor=False leaves the per-step scalar and layout kernels untimed."""
    if minor:
        check(load().hicu_profile_begin(), "hicu_profile_begin")
    else:
        check(load().hicu_profile_begin_major(), "hicu_profile_begin_major")


def profile_end(max_stats=64):
    """Stop timing; returns {kernel class: dict(launches, total_ms, min_ms,
    max_ms, avg_ms, flops, bytes)} with algorithmic flops/bytes summed."""
    from ._lib import KernelStat
    buf = (KernelStat * max_stats)()
    n = ctypes.c_int32(0)
    check(load().hicu_profile_end(buf, max_stats, ctypes.byref(n)), "hicu_profile_end")
    out = {}
    for s in buf[:min(n.value, max_stats)]:
        out[s.name.decode()] = dict(launches=int(s.launches), total_ms=s.total_ms, min_ms=s.min_ms, max_ms=s.max_ms,
                                    avg_ms=s.total_ms / max(1, s.launches), flops=s.flops, bytes=s.bytes)
    return out
