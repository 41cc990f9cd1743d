"""Sampling masks (inputs only).  1 = observed k-space location."""
import numpy as np


def vd_lines(n, n_total, n_center, rng, power=2.0):
    """Variable-density choice of ``n_total`` phase-encode lines out of ``n``.

    The ``n_center`` lines around index n/2 are always taken; the rest are
    drawn without replacement with probability proportional to
    ``(1 - |k - n/2| / (n/2)) ** power``.  Returns a bool vector.
    """
    sel = np.zeros(n, bool)
    c0 = n // 2 - n_center // 2
    sel[c0:c0 + n_center] = True
    k = np.arange(n)
    w = np.clip(1.0 - np.abs(k - n / 2.0) / (n / 2.0), 1e-3, None) ** power
    w[sel] = 0.0
    extra = max(0, n_total - int(sel.sum()))
    if extra:
        pick = rng.choice(n, size=extra, replace=False, p=w / w.sum())
        sel[pick] = True
    return sel


def line_mask(dims, axis, lines):
    """Spatial mask of shape ``dims`` that is 1 wherever the index along
    ``axis`` is a selected line (every other axis fully sampled)."""
    shape = [1] * len(dims)
    shape[axis] = dims[axis]
    m = np.broadcast_to(lines.reshape(shape), dims)
    return np.ascontiguousarray(m).astype(np.uint8)


def cine_line_masks(nt, nx, ny, accel, n_center, rng):
    """Per-frame variable-density ky-line masks for 2-D+t data laid out as
    ``(nt, nx, ny)``; frame t draws its own lines."""
    m = np.zeros((nt, nx, ny), np.uint8)
    n_total = int(round(ny / accel))
    for t in range(nt):
        lines = vd_lines(ny, n_total, n_center, rng)
        m[t, :, lines] = 1
    return m


def _dart_throw(n0, n1, radius, rng):
    """Poisson-disc point set on an n0 x n1 grid by dart throwing over a random
    permutation of grid points: a point is kept if no kept point lies within
    ``radius`` (Euclidean, in grid units)."""
    taken = np.zeros((n0, n1), bool)
    rr = int(np.ceil(radius))
    offs = [(a, b) for a in range(-rr, rr + 1) for b in range(-rr, rr + 1)
            if 0 < a * a + b * b < radius * radius]
    offs = np.array(offs, dtype=np.int64).reshape(-1, 2)
    order = rng.permutation(n0 * n1)
    for idx in order:
        i, j = divmod(int(idx), n1)
        ii = i + offs[:, 0]
        jj = j + offs[:, 1]
        ok = (ii >= 0) & (ii < n0) & (jj >= 0) & (jj < n1)
        if not taken[ii[ok], jj[ok]].any():
            taken[i, j] = True
    return taken


def poisson_disc_2d(n0, n1, accel, center, rng, iters=12):
    """2-D Poisson-disc mask with a fully sampled ``center x center`` block,
    the disc radius bisected so the overall sampling rate is ~1/accel."""
    target = n0 * n1 / accel
    c0, c1 = n0 // 2 - center // 2, n1 // 2 - center // 2
    lo, hi = 1.0, 4.0
    best = None
    for _ in range(iters):
        r = 0.5 * (lo + hi)
        m = _dart_throw(n0, n1, r, rng)
        m[c0:c0 + center, c1:c1 + center] = True
        cnt = m.sum()
        if best is None or abs(cnt - target) < abs(best.sum() - target):
            best = m
        if cnt > target:
            lo = r
        else:
            hi = r
    return best.astype(np.uint8)


def volume_mask_from_plane(n_readout, plane):
    """3-D mask ``(n_readout, *plane.shape)``: the readout axis is fully sampled."""
    return np.ascontiguousarray(np.broadcast_to(plane[None], (n_readout,) + plane.shape)).astype(np.uint8)
