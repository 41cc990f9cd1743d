"""Explicit multi-level Hankel lifting and its adjoint (THEORY section).

The paper lifts the k-space array X to an m-by-n multi-level Hankel matrix
H(x) such that H(x) v is the vectorised *valid* convolution of X with the
multi-dimensional kernel whose taps are listed in v; the kernel spans all
coils, so one valid convolution also sums over coils.

Conventions (readings recorded with the project's design notes):

* x has shape (D0, D1, D2, Nc); 2-D data has D0 = 1.
* The region S = [lo, hi) per axis; valid output positions are
  u with lo <= u <= hi - K (per axis), s = prod(hi - lo - K + 1) of them.
* Row index = lexicographic (u0, u1, u2); column index = lexicographic
  (k0, k1, k2, c) with the coil c fastest.
* H[u, (k, c)] = x[u + k, c]: a correlation (no kernel flip, no conjugate).
  A flip would only permute the n columns; nothing observable changes.
* Kernel mask (THEORY: the {0,1} mask K marks the support of an
  annihilating kernel; DISCUSSION: circular or spherical supports): pass
  ``kdims`` as a 3-D boolean array instead of a box; the columns are then
  the taps k with K[k] = 1, in lexicographic order of k, coil fastest, and
  the valid extent follows the bounding box K.shape.
* Circular axes (METHODS, Study II: the convolution along time is circular
  rather than valid): on an axis flagged in ``wrap`` the region must be the
  whole axis, every position is an output (m = N) and the patch index
  wraps, H[u, (k, c)] = x[(u + k) mod N, c] along that axis.

Parity: pinned by brute-force element loops, the 1-D case against
``scipy.linalg.hankel`` and the adjoint identity (see tests).
"""
import numpy as np


def _wrap3(wrap):
    return (False, False, False) if wrap is None else tuple(bool(w) for w in wrap)


def kernel_box(kdims):
    """(box extents, tap offsets in lexicographic order) of a box or mask."""
    if isinstance(kdims, np.ndarray) and kdims.ndim == 3:
        return tuple(int(v) for v in kdims.shape), [tuple(int(v) for v in t) for t in np.argwhere(kdims)]
    K = tuple(int(v) for v in kdims)
    return K, [(a, b, c) for a in range(K[0]) for b in range(K[1]) for c in range(K[2])]


def valid_extent(lo, hi, kdims, wrap=None):
    """Number of outputs per axis: hi - lo - K + 1 (valid), hi - lo (circular)."""
    wrap = _wrap3(wrap)
    kdims = kernel_box(kdims)[0]
    m = tuple(int(h) - int(l) - (0 if w else int(k) - 1) for l, h, k, w in zip(lo, hi, kdims, wrap))
    if any(v <= 0 for v in m) or any(w and k > h - l for l, h, k, w in zip(lo, hi, kdims, wrap)):
        raise ValueError("region smaller than kernel: lo=%s hi=%s K=%s" % (lo, hi, kdims))
    return m


def _window(lo, k, m, shape, wrap):
    """Per-axis indices lo + k + [0, m), wrapped on circular axes."""
    idx = []
    for a in range(3):
        i = np.arange(lo[a] + k[a], lo[a] + k[a] + m[a])
        if wrap[a]:
            if lo[a] != 0 or m[a] != shape[a]:
                raise ValueError("a circular axis needs the whole axis as its region")
            i = i % shape[a]
        idx.append(i)
    return np.ix_(*idx)


def _offsets(kdims):
    return kernel_box(kdims)[1]


def hankel_matrix(x, kdims, lo, hi, wrap=None):
    """Explicit H(x) of shape (s, n), n = K0*K1*K2*Nc, for region [lo, hi)."""
    wrap = _wrap3(wrap)
    m = valid_extent(lo, hi, kdims, wrap)
    nc = x.shape[3]
    s = m[0] * m[1] * m[2]
    cols = []
    for k in _offsets(kdims):
        if any(wrap):
            blk = x[_window(lo, k, m, x.shape, wrap)]
        else:
            blk = x[lo[0] + k[0]: lo[0] + k[0] + m[0],
                    lo[1] + k[1]: lo[1] + k[1] + m[1],
                    lo[2] + k[2]: lo[2] + k[2] + m[2], :]
        cols.append(blk.reshape(s, nc))
    return np.concatenate(cols, axis=1)


def hankel_adjoint(W, shape, kdims, lo, hi, wrap=None):
    """H'(.) applied to a patch-space matrix W (s, n): every entry
    W[u, (k, c)] is added back onto k-space location (u + k, c) (wrapped on
    circular axes, where the window of one tap is a cyclic shift of the axis
    and holds each location once)."""
    wrap = _wrap3(wrap)
    m = valid_extent(lo, hi, kdims, wrap)
    nc = shape[3]
    out = np.zeros(shape, np.result_type(W.dtype, np.complex128))
    for j, k in enumerate(_offsets(kdims)):
        blk = W[:, j * nc:(j + 1) * nc].reshape(m + (nc,))
        if any(wrap):
            out[_window(lo, k, m, shape, wrap)] += blk
        else:
            out[lo[0] + k[0]: lo[0] + k[0] + m[0],
                lo[1] + k[1]: lo[1] + k[1] + m[1],
                lo[2] + k[2]: lo[2] + k[2] + m[2], :] += blk
    return out


def forward(x, F, kdims, lo, hi, wrap=None):
    """Y = H(x) F: the valid convolution of x with each of the filters in
    the columns of F (n, p)."""
    return hankel_matrix(x, kdims, lo, hi, wrap) @ F


def adjoint(Y, F, shape, kdims, lo, hi, wrap=None):
    """Adjoint of x -> H(x) F, applied to Y (s, p): H'(Y F^H)."""
    return hankel_adjoint(Y @ F.conj().T, shape, kdims, lo, hi, wrap)
