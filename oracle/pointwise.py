"""Point-by-point evaluation of the convolution and its adjoint, for checking
sampled outputs of full-size problems whose explicit H would not fit.

Same definitions as ``hankel``/``descent`` (THEORY section): the residual
row Y[u, :] = patch(u) . F with patch(u)[(k, c)] = x[u + k, c], and the
gradient entry g[w, c] = 2 sum over taps k with u = w - k a valid output of
sum_j Y[u, j] conj(F[(k, c), j]), zero at observed locations.

Gram entries G[(k, c), (k', c')] = sum over valid outputs u of
conj(x[u + k, c]) x[u + k', c'] (the Gram of H on the region, DISCUSSION
section) one at a time, as the inner product of two shifted windows.

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


def gram_entries(x, kdims, lo, hi, pairs):
    """Entries G[i, j] of the Gram H'H for flat tap indices i = (k, c),
    j = (k', c') (kernel offset lexicographic, coil fastest), each the inner
    product of the windows of x shifted by k and k'.  Returns complex128."""
    x = np.asarray(x, np.complex128)
    nc = x.shape[3]
    m = [hi[a] - lo[a] - kdims[a] + 1 for a in range(3)]

    def split(i):
        t, c = divmod(int(i), nc)
        k2 = t % kdims[2]
        k1 = (t // kdims[2]) % kdims[1]
        k0 = t // (kdims[2] * kdims[1])
        return (k0, k1, k2), c

    def window(k, c):
        return x[lo[0] + k[0]:lo[0] + k[0] + m[0], lo[1] + k[1]:lo[1] + k[1] + m[1],
                 lo[2] + k[2]:lo[2] + k[2] + m[2], c].reshape(-1)

    out = np.zeros(len(pairs), np.complex128)
    for idx, (i, j) in enumerate(pairs):
        k, c = split(i)
        kp, cp = split(j)
        out[idx] = np.vdot(window(k, c), window(kp, cp))
    return out
