"""Randomized-SVD nullspace route (THEORY, first numerical technique;
Algorithm 1, rSVD and Householder steps; cost-model paragraph).

The paper takes V, the r principal right singular vectors of H(x), from a
randomized SVD (Halko, Martinsson and Tropp) that applies H and H' about
3r/2 times each, and completes the nullspace basis Q orthogonal to V with
r Householder reflections.  This module writes those steps out plainly:

1. sketch:   Y = H(x) Omega, Omega an n x l Gaussian test matrix,
             l = ceil(3 r / 2) (the paper's 3r/2 applications);
2. range:    U = an orthonormal basis of range(Y) (a QR factorisation);
3. project:  B = U' H(x), formed as (H(x)' U)', i.e. l applications of H';
4. SVD:      B = U_B S Vb'; V = the first r columns of Vb;
5. complete: the Householder QR of V, V = H_1 ... H_r [R; 0]; the last
             n - r columns of H_1 ... H_r are Q.

Readings (the paper fixes neither the draw nor the reflector convention):

* Omega^(i) for outer iteration i is complex, n x l, row-major; element
  e = row * l + col has real part z[2e] and imaginary part z[2e + 1], where
  z are the standard normals of ``philox_normals`` for counter words
  (block, i, 2^32 - 1, stream): the third word 2^32 - 1 is never an inner
  step index, so the sketch never reuses a JL draw.  No power iterations.
* Reflector j is the Hermitian H_j = I - 2 w w' / (w' w), w = a - alpha e_j,
  with a the j-th column of the partly reduced V from row j down and
  alpha = -exp(i arg a_0) ||a|| (exp(i arg 0) taken as 1), so H_j a =
  alpha e_j.  For real V this is LAPACK's reflector, so Q agrees with the
  complete Householder QR of a real library factorisation.

Parity: pinned by the exact SVD of the explicit H when l = n, by exact
recovery of an exactly low-rank H when rank(H) <= l (band-limited coils),
by the Halko-Martinsson-Tropp expected-error bound on a decaying
spectrum, by numpy's complete QR for real V, and by the unitarity of
[V Q] and the triangular R (see tests).
"""
import math

import numpy as np

from .hankel import hankel_matrix
from .jl import philox_normals

SKETCH_COUNTER = 0xFFFFFFFF


def sketch_size(rank, n):
    """l = ceil(3 r / 2), at most n."""
    return min(n, (3 * rank + 1) // 2)


def sketch_matrix(seed, i, n, ell, stream=0):
    """Omega^(i): complex (n, ell) test matrix, N(0, 1) real and imaginary parts."""
    z = philox_normals(2 * n * ell, seed, i, SKETCH_COUNTER, stream)
    return (z[0::2] + 1j * z[1::2]).reshape(n, ell)


def rsvd_right(x, kdims, lo, hi, rank, Omega, wrap=None):
    """(V, sv): the first ``rank`` right singular vectors of B = U' H(x)
    (n x rank, orthonormal columns) and all singular values of B."""
    H = hankel_matrix(np.asarray(x, np.complex128), kdims, lo, hi, wrap)
    Y = H @ Omega
    U, _ = np.linalg.qr(Y)
    B = (H.conj().T @ U).conj().T
    _, sv, Vh = np.linalg.svd(B, full_matrices=False)
    return Vh[:rank].conj().T, sv


def householder_complement(V):
    """Q (n x (n - r)) orthonormal, orthogonal to the columns of V (n x r),
    from the r Householder reflections of V's QR factorisation.
    Returns (Q, W, alpha): W[:, j] the unit reflector vectors (zero above
    row j) and alpha[j] the diagonal of R."""
    A = np.array(V, dtype=np.complex128)
    n, r = A.shape
    if r > n:
        raise ValueError("V must have at most n columns")
    W = np.zeros((n, r), np.complex128)
    alpha = np.zeros(r, np.complex128)
    for j in range(r):
        a = A[j:, j]
        norm = np.linalg.norm(a)
        phase = a[0] / abs(a[0]) if a[0] != 0 else 1.0
        alpha[j] = -phase * norm
        w = a.copy()
        w[0] -= alpha[j]
        wn = np.linalg.norm(w)
        if wn > 0:
            w = w / wn
        W[j:, j] = w
        A[j:, j:] -= 2.0 * np.outer(w, w.conj() @ A[j:, j:])
    Q = np.zeros((n, n - r), np.complex128)
    Q[r:, :] = np.eye(n - r)
    for j in reversed(range(r)):
        w = W[j:, j]
        Q[j:, :] -= 2.0 * np.outer(w, w.conj() @ Q[j:, :])
    return Q, W, alpha


def nullspace_rsvd(x, kdims, lo, hi, rank, seed, i, ell=None, stream=0, wrap=None):
    """Q (n x (n - rank)) by rSVD and Householder completion, plus the
    singular values of the sketched B (largest first)."""
    n = len(_taps(kdims)) * x.shape[3]
    if not 0 <= rank < n:
        raise ValueError("rank must satisfy 0 <= r < n")
    if rank == 0:
        return np.eye(n, dtype=np.complex128), np.zeros(0)
    ell = sketch_size(rank, n) if ell is None else int(ell)
    if not rank <= ell <= n:
        raise ValueError("sketch size must satisfy r <= l <= n")
    V, sv = rsvd_right(x, kdims, lo, hi, rank, sketch_matrix(seed, i, n, ell, stream), wrap)
    Q, _, _ = householder_complement(V)
    return Q, sv


def _taps(kdims):
    from .hankel import kernel_box
    return kernel_box(kdims)[1]


def hmt_bound(sv_tail, rank, ell):
    """Expected-error bound of the Gaussian range finder (Halko, Martinsson,
    Tropp, real test matrices, oversampling l - r >= 2):
    E ||H - U U' H||_F <= sqrt(1 + r / (l - r - 1)) (sum_{j>r} s_j^2)^(1/2)."""
    if ell - rank < 2:
        raise ValueError("the bound needs an oversampling of at least 2")
    return math.sqrt(1.0 + rank / (ell - rank - 1.0)) * math.sqrt(float(np.sum(np.square(sv_tail))))
