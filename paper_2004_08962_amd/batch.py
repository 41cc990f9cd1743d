"""Batched gradient steps and the tile autotuner (thin binding of the
hicu_batch_* / hicu_autotune / hicu_tune_* C entry points)."""
import ctypes

import torch

from ._lib import BatchItem, PREC, check, load
from .api import _dev, _prec, _ptr, _stream, _workspace, geom


class Batch:
    """Many problems stepped together.  ``problems``: list of dicts with keys
    x (complex64 CUDA, updated in place), mask (uint8 CUDA or None), Q
    (complex64 n x nq CUDA), p (filters per step), kdims, lo, hi, seed.
    ``scalars`` (float64 (count, 3) CUDA) receives J, ||g||^2, eta of the
    latest step of every problem."""

    def __init__(self, problems, prec="fp32"):
        self.lib = load()
        self.problems = problems
        n = len(problems)
        dev = problems[0]["x"].device
        self.scalars = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        items = (BatchItem * n)()
        for i, pr in enumerate(problems):
            _dev(pr["x"], torch.complex64, "x")
            _dev(pr["Q"], torch.complex64, "Q")
            if pr.get("mask") is not None:
                _dev(pr["mask"], torch.uint8, "mask")
            items[i].geom = geom(pr["x"].shape, pr["kdims"], pr.get("lo"), pr.get("hi"))
            items[i].x = pr["x"].data_ptr()
            items[i].mask = None if pr.get("mask") is None else pr["mask"].data_ptr()
            items[i].Q = pr["Q"].data_ptr()
            items[i].nq = pr["Q"].shape[1]
            items[i].p = int(pr["p"])
            items[i].seed = int(pr.get("seed", 0))
            items[i].scalars = self.scalars[i].data_ptr()
        self._items = items
        h = ctypes.c_void_p()
        wsb = ctypes.c_size_t(0)
        check(self.lib.hicu_batch_create(items, n, _prec(prec), ctypes.byref(h), ctypes.byref(wsb)),
              "hicu_batch_create")
        self.handle = h
        self.ws = _workspace(wsb.value, dev)
        check(self.lib.hicu_batch_bind(h, _ptr(self.ws), self.ws.numel(), _stream()), "hicu_batch_bind")

    def info(self):
        buf = (ctypes.c_int64 * 6)()
        check(self.lib.hicu_batch_info(self.handle, buf), "hicu_batch_info")
        return dict(count=buf[0], fwd_items=buf[1], adj_items=buf[2], fwd_tile=buf[3], adj_tile=buf[4],
                    ws_bytes=buf[5])

    def set_counter(self, outer, inner):
        check(self.lib.hicu_batch_set_counter(self.handle, int(outer), int(inner), _stream()),
              "hicu_batch_set_counter")

    def step(self):
        check(self.lib.hicu_batch_step(self.handle, _stream()), "hicu_batch_step")

    def capture(self, steps, stream):
        """Capture `steps` steps into one graph on a non-default stream."""
        check(self.lib.hicu_batch_graph_create(self.handle, int(steps), ctypes.c_void_p(stream.cuda_stream)),
              "hicu_batch_graph_create")

    def replay(self, stream=None):
        s = _stream() if stream is None else ctypes.c_void_p(stream.cuda_stream)
        check(self.lib.hicu_batch_graph_launch(self.handle, s), "hicu_batch_graph_launch")

    def close(self):
        if self.handle:
            self.lib.hicu_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(x, F, kdims, lo=None, hi=None, prec="fp32", batched=False):
    """Time every tile shape on this problem; returns the chosen
    (forward shape id, forward chunk, adjoint shape id, adjoint chunk).
    batched=True times the shapes that have batched kernels and stores the
    choice for Batch objects whose largest problem is of this class."""
    lib = load()
    _dev(x, torch.complex64, "x")
    _dev(F, torch.complex64, "F")
    g = geom(x.shape, kdims, lo, hi)
    p = F.shape[1]
    wsb = lib.hicu_autotune_workspace_bytes(ctypes.byref(g), p, _prec(prec))
    ws = _workspace(wsb, x.device)
    choice = (ctypes.c_int32 * 4)()
    fn = lib.hicu_autotune_batched if batched else lib.hicu_autotune
    check(fn(ctypes.byref(g), _ptr(x), _ptr(F), p, _prec(prec), _ptr(ws), ws.numel(), choice, _stream()),
          "hicu_autotune_batched" if batched else "hicu_autotune")
    return tuple(choice)


def tune_put(shape, kdims, p, prec, role, tile, chunk, lo=None, hi=None):
    """Pin shape id `tile` (and adjoint channel chunk) for one contraction."""
    check(load().hicu_tune_put(ctypes.byref(geom(shape, kdims, lo, hi)), int(p), _prec(prec), int(role), int(tile),
                               int(chunk)), "hicu_tune_put")


def tile_info(tile):
    """(T0, T2, WC, FN, D, KS) of shape id `tile`."""
    cfg = (ctypes.c_int32 * 6)()
    check(load().hicu_tile_info(int(tile), cfg), "hicu_tile_info")
    return tuple(cfg)


def tile_count():
    return int(load().hicu_tile_count())


def tune_clear():
    check(load().hicu_tune_clear(), "hicu_tune_clear")


def tune_save(path):
    check(load().hicu_tune_save(str(path).encode()), "hicu_tune_save")


def tune_load(path):
    return check(load().hicu_tune_load(str(path).encode()), "hicu_tune_load")
