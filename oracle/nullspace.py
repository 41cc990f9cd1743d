"""Gram matrix and nullspace basis (THEORY section, Eq. 1 and Eq. 2;
Algorithm 1, nullspace update; DISCUSSION, Gram-matrix route).

The tail energy of Eq. 1, sum_{k>r} sigma_k^2{H(x)}, equals
min ||H(x) Q||_F^2 over Q with orthonormal columns (n - r of them).  The
minimiser spans the right singular vectors of H(x) belonging to its n - r
smallest singular values, i.e. the eigenvectors of the Gram H'H for its
n - r smallest eigenvalues.  The paper reaches V (the r principal right
singular vectors) by rSVD and completes Q by Householder reflections, and
notes that an SVD of the Gram matrix is the alternative route; this oracle
takes the Gram route with a dense eigendecomposition.

Parity: pinned by the Ky Fan identity ||H Q||_F^2 = sum of the n - r
smallest eigenvalues, by the tail energy recomputed from an SVD of the
explicit H (a different library routine), and by the exact annihilation of
data built from band-limited coil maps (see tests).
"""
import numpy as np

from .hankel import hankel_matrix


def gram(x, kdims, lo, hi, wrap=None):
    """G = H(x)' H(x), (n, n) Hermitian, complex128."""
    H = hankel_matrix(np.asarray(x, np.complex128), kdims, lo, hi, wrap)
    return H.conj().T @ H


def nullspace(G, rank):
    """Eigendecomposition of the Hermitian Gram G.

    Returns ``(Q, evals, U)``: eigenvalues ascending, U the full set of
    eigenvectors, and Q = U[:, :n - rank] (the n - rank smallest).

    The paper leaves the basis free (any unitary mix of Q gives the same
    objective); to make JL draws comparable across implementations each
    eigenvector is multiplied by the unit phase that makes the sum of its
    entries real and non-negative."""
    n = G.shape[0]
    if not 0 <= rank < n:
        raise ValueError("rank must satisfy 0 <= r < n")
    evals, U = np.linalg.eigh(G)
    tot = U.sum(axis=0)
    mag = np.abs(tot)
    ph = np.where(mag > 0, np.conj(tot) / np.where(mag > 0, mag, 1.0), 1.0)
    U = U * ph[None, :]
    return U[:, : n - rank], evals, U
