"""Workload table and problem assembly (inputs only).

A *problem* is a dict with the fully sampled k-space ``x_true``
(D0, D1, D2, Nc), the observation mask ``mask`` (D0, D1, D2) uint8, the
zero-filled observations ``x0 = mask * x_true``, the kernel box ``kdims``,
the rank ``rank``, the per-step filter count ``p`` (0 means "no JL, use the
whole nullspace"), the outer-iteration ``schedule`` (a list of
``(lo, hi, steps)``: region box and gradient steps) and the JL ``seed``.
"""
import numpy as np

from .phantom import (ellipse_image, ellipsoid_volume, cine_phantom, gaussian_coil_maps,
                      polynomial_coil_maps, to_kspace, add_noise)
from .masks import vd_lines, line_mask, poisson_disc_2d, volume_mask_from_plane, cine_line_masks


def full_region(dims):
    return (0, 0, 0), tuple(int(d) for d in dims)


def co_region(dims, kdims, reduce_axes):
    """Centre box: size floor(N/4) on each reduced axis (never below the
    kernel), full extent elsewhere, placed at floor((N - size) / 2)."""
    lo, hi = [], []
    for a, n in enumerate(dims):
        if a in reduce_axes:
            size = max(n // 4, kdims[a])
            l0 = (n - size) // 2
            lo.append(l0)
            hi.append(l0 + size)
        else:
            lo.append(0)
            hi.append(n)
    return tuple(lo), tuple(hi)


WORKLOADS = {
    # 64x64 x 4 coils, 5x5 kernel, rank 30 (70 filters), 50 GD steps.
    "2d_64x64x4": dict(dims=(1, 64, 64), nc=4, kdims=(1, 5, 5), rank=30, p=0,
                       outer=10, inner=5, seed=1),
    # 256x232 x 16 coils, 5x5 kernel, 280 nullspace filters, 100 GD steps.
    "2d_256x232x16": dict(dims=(1, 256, 232), nc=16, kdims=(1, 5, 5), rank=120, p=0,
                          outer=20, inner=5, seed=2),
    # gradient check: 48x48 x 4 coils, 3x3 kernel, 20 nullspace filters.
    "gradcheck_48x48x4": dict(dims=(1, 48, 48), nc=4, kdims=(1, 3, 3), rank=16, p=0,
                              outer=1, inner=1, seed=3),
    # 2-D+t cine: 25 frames of 160x144 x 12 coils, 5x5x5 kernel over (t, kx, ky).
    "cine_25x160x144x12": dict(dims=(25, 160, 144), nc=12, kdims=(5, 5, 5), rank=130, p=12,
                               outer=6, inner=5, co_outer=5, co_axes=(1, 2), seed=4),
    # the same cine data with the study's circular time axis and time-averaged start
    "cine_25x160x144x12_circ": dict(dims=(25, 160, 144), nc=12, kdims=(5, 5, 5), rank=130, p=12,
                                    outer=6, inner=5, co_outer=5, co_axes=(1, 2), seed=4,
                                    wrap=(True, False, False), init="time_average"),
    # 3-D knee-like volume 256x320x320 x 8 coils, 5x5x5 kernel, 900 nullspace filters.
    "3d_256x320x320x8": dict(dims=(256, 320, 320), nc=8, kdims=(5, 5, 5), rank=100, p=0,
                             outer=11, inner=5, last_inner=20, co_outer=10,
                             co_axes=(0, 1, 2), seed=5, centre=24),
    # the same generator on a 16x28x28 volume (oracle-sized 3-D parity case)
    "3d_16x28x28x8": dict(dims=(16, 28, 28), nc=8, kdims=(5, 5, 5), rank=100, p=0,
                          outer=2, inner=3, seed=6, centre=8),
}


def _schedule(w, dims):
    kd = w["kdims"]
    full = full_region(dims)
    co_outer = w.get("co_outer", 0)
    sched = []
    for i in range(w["outer"]):
        if i < co_outer:
            lo, hi = co_region(dims, kd, w["co_axes"])
            sched.append((lo, hi, w["inner"]))
        else:
            steps = w.get("last_inner", w["inner"]) if i == w["outer"] - 1 and co_outer else w["inner"]
            sched.append((full[0], full[1], steps))
    return sched


def _finish(name, w, x_true, mask):
    dims = tuple(int(d) for d in w["dims"])
    x0 = x_true * mask[..., None]
    return dict(name=name, x_true=x_true, mask=mask, x0=x0, kdims=tuple(w["kdims"]),
                rank=int(w["rank"]), p=int(w["p"]), schedule=_schedule(w, dims),
                seed=int(w["seed"]), wrap=w.get("wrap"), init=w.get("init", "zero"))


def make_problem(name, dtype=np.complex128):
    """Build the named workload deterministically from its seed."""
    w = WORKLOADS[name]
    rng = np.random.default_rng(w["seed"])
    dims, nc = tuple(w["dims"]), w["nc"]
    if name == "2d_64x64x4" or name == "gradcheck_48x48x4":
        shp = dims[1:]
        img = ellipse_image(shp, 6, rng)
        maps = gaussian_coil_maps(shp, nc, rng)
        x = to_kspace(img, maps)[None]
        lines = vd_lines(shp[1], int(round(shp[1] / 3)), 8, rng)
        mask = line_mask(dims, 2, lines)
    elif name == "2d_256x232x16":
        shp = dims[1:]
        img = ellipse_image(shp, 10, rng, skull=True)
        maps = polynomial_coil_maps(shp, nc, rng)
        x = add_noise(to_kspace(img, maps), 30.0, rng)[None]
        lines = vd_lines(shp[1], int(round(shp[1] / 4)), 16, rng)
        mask = line_mask(dims, 2, lines)
    elif name.startswith("cine_25x160x144x12"):
        nt, nx, ny = dims
        imgs = cine_phantom(nt, (nx, ny), 6, rng)
        maps = gaussian_coil_maps((nx, ny), nc, rng)
        x = np.stack([to_kspace(imgs[t], maps) for t in range(nt)])
        mask = cine_line_masks(nt, nx, ny, 6.0, 8, rng)
    elif name.startswith("3d_"):
        vol = ellipsoid_volume(dims, 8, rng)
        maps = gaussian_coil_maps(dims, nc, rng).astype(np.complex64)
        x = np.empty(dims + (nc,), np.complex64)
        for c in range(nc):
            x[..., c] = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(vol * maps[..., c]), norm="ortho"))
        plane = poisson_disc_2d(dims[1], dims[2], 5.0, w["centre"], rng)
        mask = volume_mask_from_plane(dims[0], plane)
    else:
        raise KeyError(name)
    return _finish(name, w, np.ascontiguousarray(x.astype(dtype)), np.ascontiguousarray(mask))


def make_batch2d(count=64, seed=44, dtype=np.complex128):
    """Independent 2-D slices of uneven size (each axis U{128..320}) and coil
    count (U{8..16}), 5x5 kernel, rank round(0.3 n), p = Nc, mask R = 4."""
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        n0, n1 = (int(v) for v in rng.integers(128, 321, 2))
        nc = int(rng.integers(8, 17))
        img = ellipse_image((n0, n1), 6, rng)
        maps = gaussian_coil_maps((n0, n1), nc, rng)
        x = to_kspace(img, maps)[None].astype(dtype)
        lines = vd_lines(n1, int(round(n1 / 4)), 8, rng)
        mask = line_mask((1, n0, n1), 2, lines)
        n = 25 * nc
        w = dict(dims=(1, n0, n1), nc=nc, kdims=(1, 5, 5), rank=int(round(0.3 * n)), p=nc,
                 outer=1, inner=5, seed=seed * 1000 + b)
        probs.append(_finish("batch2d_%d" % b, w, x, mask))
    return probs


def crop_problem(prob, lo, hi, name=None):
    """Centre (or any) crop of a problem; the schedule becomes full-region
    steps on the crop with the same step counts."""
    sl = tuple(slice(l, h) for l, h in zip(lo, hi))
    x_true = np.ascontiguousarray(prob["x_true"][sl])
    mask = np.ascontiguousarray(prob["mask"][sl])
    dims = mask.shape
    sched = [((0, 0, 0), tuple(dims), s) for (_, _, s) in prob["schedule"]]
    out = dict(prob)
    out.update(name=name or prob["name"] + "_crop", x_true=x_true, mask=mask,
               x0=x_true * mask[..., None], schedule=sched)
    return out
