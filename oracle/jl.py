"""Johnson-Lindenstrauss compression of the nullspace (THEORY section,
"second numerical technique"; Algorithm 1, JL step).

Before each gradient step the n - r nullspace filters are mixed down to p
filters, F = Q P, with P of i.i.d. zero-mean Gaussian entries of variance
1/p, so that E[P P^T] = I and the mean gradient direction is kept.

The paper does not say how P is drawn.  Reading used here (both the oracle
and the GPU library implement it independently, from the published
definitions):

* P is real, (n - r) x p, row-major; element e = row * p + col.
* Uniforms come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11):
  key = (seed mod 2^32, seed div 2^32), counter = (e div 4, i, j, stream)
  with i the outer and j the inner iteration.
* Each 32-bit word w maps to u = (w + 1/2) 2^-32.  The four words
  (w0, w1, w2, w3) of one block give four normals by Box-Muller:
  z0 = R cos(2 pi u1), z1 = R sin(2 pi u1) with R = sqrt(-2 ln u0), and
  likewise z2, z3 from (u2, u3).  P[e] = z[e mod 4] / sqrt(p).

Parity: the block function is pinned bit for bit against rocRAND's
independent Philox4x32-10 (ROCm's source header compiled for the host) on
structured and random counters and keys, together with the counter layout
above; the normals are pinned statistically (moments, normality,
unbiasedness of E[Q P P^T Q'] = Q Q').
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.

    ``ctr``: (..., 4) array of uint32 counters; ``key``: 2 uint32 words.
    Returns (..., 4) uint32.  Each round multiplies words 0 and 2 by the two
    Philox constants, takes the high/low halves of the 64-bit products and
    mixes them with words 1 and 3 and the round key; the key is bumped by
    the Weyl constants between rounds."""
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def philox_normals(count, seed, i, j, stream=0):
    """``count`` standard normals for counter words (block, i, j, stream)."""
    nblk = (count + 3) // 4
    ctr = np.zeros((nblk, 4), np.uint64)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64)
    ctr[:, 1] = i
    ctr[:, 2] = j
    ctr[:, 3] = stream
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = philox4x32_10(ctr, key).astype(np.float64)
    u = (w + 0.5) * 2.0 ** -32
    R01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    R23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    z = np.empty((nblk, 4))
    z[:, 0] = R01 * np.cos(2.0 * np.pi * u[:, 1])
    z[:, 1] = R01 * np.sin(2.0 * np.pi * u[:, 1])
    z[:, 2] = R23 * np.cos(2.0 * np.pi * u[:, 3])
    z[:, 3] = R23 * np.sin(2.0 * np.pi * u[:, 3])
    return z.reshape(-1)[:count]


def jl_matrix(seed, i, j, rows, p, stream=0):
    """P^(i,j): real (rows, p) with i.i.d. N(0, 1/p) entries."""
    return philox_normals(rows * p, seed, i, j, stream).reshape(rows, p) / np.sqrt(p)
