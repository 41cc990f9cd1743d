"""Point-by-point evaluation of the convolution and its adjoint, for checking
sampled outputs of full-size problems whose explicit H would not fit.

Same definitions as ``hankel``/``descent`` (THEORY section): the residual
row Y[u, :] = patch(u) . F with patch(u)[(k, c)] = x[u + k, c], and the
gradient entry g[w, c] = 2 sum over taps k with u = w - k a valid output of
sum_j Y[u, j] conj(F[(k, c), j]), zero at observed locations.

Parity: checked against the explicit-matrix functions on small inputs.
"""
import numpy as np


def _patch(x, u, kdims):
    return x[u[0]:u[0] + kdims[0], u[1]:u[1] + kdims[1], u[2]:u[2] + kdims[2], :].reshape(-1)


def residual_at_points(x, F, kdims, points):
    """Rows of Y = H(x) F at valid output positions ``points`` (absolute
    coordinates of the patch origin).  Returns (len(points), p)."""
    x = np.asarray(x, np.complex128)
    F = np.asarray(F, np.complex128)
    return np.stack([_patch(x, u, kdims) @ F for u in points])


def grad_at_points(x, mask, F, kdims, lo, hi, points):
    """Gradient entries g[w, :] (Nc values) at k-space locations ``points``."""
    x = np.asarray(x, np.complex128)
    F = np.asarray(F, np.complex128)
    nc = x.shape[3]
    Fc = F.conj()
    out = np.zeros((len(points), nc), np.complex128)
    for idx, w in enumerate(points):
        if mask is not None and mask[tuple(w)]:
            continue
        acc = np.zeros(nc, np.complex128)
        t = 0
        for k0 in range(kdims[0]):
            for k1 in range(kdims[1]):
                for k2 in range(kdims[2]):
                    u = (w[0] - k0, w[1] - k1, w[2] - k2)
                    ok = all(lo[a] <= u[a] <= hi[a] - kdims[a] for a in range(3))
                    if ok:
                        y = _patch(x, u, kdims) @ F
                        acc += Fc[t * nc:(t + 1) * nc, :] @ y
                    t += 1
        out[idx] = 2.0 * acc
    return out
