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

Parity: pinned by brute-force element loops, the 1-D case against
``scipy.linalg.hankel`` and the adjoint identity (see tests).
"""
import numpy as np


def valid_extent(lo, hi, kdims):
    """Number of valid outputs per axis: hi - lo - K + 1."""
    m = tuple(int(h) - int(l) - int(k) + 1 for l, h, k in zip(lo, hi, kdims))
    if any(v <= 0 for v in m):
        raise ValueError("region smaller than kernel: lo=%s hi=%s K=%s" % (lo, hi, kdims))
    return m


def _offsets(kdims):
    return [(a, b, c) for a in range(kdims[0]) for b in range(kdims[1]) for c in range(kdims[2])]


def hankel_matrix(x, kdims, lo, hi):
    """Explicit H(x) of shape (s, n), n = K0*K1*K2*Nc, for region [lo, hi)."""
    m = valid_extent(lo, hi, kdims)
    nc = x.shape[3]
    s = m[0] * m[1] * m[2]
    cols = []
    for k in _offsets(kdims):
        blk = x[lo[0] + k[0]: lo[0] + k[0] + m[0],
                lo[1] + k[1]: lo[1] + k[1] + m[1],
                lo[2] + k[2]: lo[2] + k[2] + m[2], :]
        cols.append(blk.reshape(s, nc))
    return np.concatenate(cols, axis=1)


def hankel_adjoint(W, shape, kdims, lo, hi):
    """H'(.) applied to a patch-space matrix W (s, n): every entry
    W[u, (k, c)] is added back onto k-space location (u + k, c)."""
    m = valid_extent(lo, hi, kdims)
    nc = shape[3]
    out = np.zeros(shape, np.result_type(W.dtype, np.complex128))
    for j, k in enumerate(_offsets(kdims)):
        out[lo[0] + k[0]: lo[0] + k[0] + m[0],
            lo[1] + k[1]: lo[1] + k[1] + m[1],
            lo[2] + k[2]: lo[2] + k[2] + m[2], :] += W[:, j * nc:(j + 1) * nc].reshape(m + (nc,))
    return out


def forward(x, F, kdims, lo, hi):
    """Y = H(x) F: the valid convolution of x with each of the filters in
    the columns of F (n, p)."""
    return hankel_matrix(x, kdims, lo, hi) @ F


def adjoint(Y, F, shape, kdims, lo, hi):
    """Adjoint of x -> H(x) F, applied to Y (s, p): H'(Y F^H)."""
    return hankel_adjoint(Y @ F.conj().T, shape, kdims, lo, hi)
