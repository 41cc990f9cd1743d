"""Objective, gradient, exact line search and Algorithm 1 (THEORY section,
Eq. 2, the gradient and ELS paragraphs and the hard data matching
paragraph; Algorithm 1).

* Objective: J = ||H(x) F||_F^2 for the filter bank F (the nullspace Q, or
  its JL compression Q P).
* Gradient: J is a real function of complex x; the oracle returns
  g = 2 dJ/d(conj x) = 2 H'(H(x) F F^H), i.e. the sum over the filters of
  the composition of a convolution with its adjoint.  The factor 2 is a
  convention (the step size absorbs it).  Hard data matching sets g to
  zero at observed locations (mask broadcast over coils).
* Exact line search: along -g, J(y - eta g) = J - 2 eta Re<Y, Z> + eta^2 ||Z||^2
  with Z = H(g) F, so eta = Re<Y, Z> / ||Z||^2 = ||g||^2 / (2 ||Z||^2),
  the last form because Re<Y, Z> = ||g||^2 / 2 for the masked gradient.
  When Z = 0 (equivalently g = 0) the step is eta = 0.
* Algorithm 1: for each outer iteration i pick the region S(i), build the
  Gram on S(i), take the nullspace, then run G(i) gradient steps with ELS
  on S(i), compressing the nullspace by JL before each step when p > 0.

Parity: the gradient is pinned by central finite differences (exact for a
quadratic up to rounding), ELS by the parabola through three evaluations
of J and by orthogonality of successive gradients, the loop by monotone
decrease of J and by bit-exact observed samples (see tests).
"""
import numpy as np

from .hankel import hankel_matrix, hankel_adjoint
from .nullspace import gram, nullspace
from .jl import jl_matrix
from .rsvd import nullspace_rsvd


def _as_c128(a):
    return np.asarray(a, dtype=np.complex128)


def objective(x, F, kdims, lo, hi, wrap=None):
    """J = ||H(x) F||_F^2 on region [lo, hi)."""
    Y = hankel_matrix(_as_c128(x), kdims, lo, hi, wrap) @ _as_c128(F)
    return float(np.vdot(Y, Y).real)


def objective_grad(x, mask, F, kdims, lo, hi, wrap=None):
    """Returns (J, g, ||g||^2) with g = 2 (1 - M) o H'(H(x) F F^H)."""
    x = _as_c128(x)
    F = _as_c128(F)
    Y = hankel_matrix(x, kdims, lo, hi, wrap) @ F
    J = float(np.vdot(Y, Y).real)
    g = 2.0 * hankel_adjoint(Y @ F.conj().T, x.shape, kdims, lo, hi, wrap)
    if mask is not None:
        g[np.asarray(mask).astype(bool)] = 0.0
    return J, g, float(np.vdot(g, g).real)


def line_search(g, F, gnorm2, kdims, lo, hi, wrap=None):
    """Closed-form step eta = ||g||^2 / (2 ||H(g) F||^2) (0 when H(g) F = 0)."""
    Z = hankel_matrix(_as_c128(g), kdims, lo, hi, wrap) @ _as_c128(F)
    zz = float(np.vdot(Z, Z).real)
    return 0.0 if zz == 0.0 else gnorm2 / (2.0 * zz)


def descent_step(y, mask, F, kdims, lo, hi, wrap=None):
    """One gradient step with exact line search; returns (y_new, J, gnorm2, eta)."""
    J, g, gn2 = objective_grad(y, mask, F, kdims, lo, hi, wrap)
    eta = line_search(g, F, gn2, kdims, lo, hi, wrap)
    return _as_c128(y) - eta * g, J, gn2, eta


def solve(x0, mask, kdims, rank, schedule, p=0, seed=0, start_outer=0, trace=None, wrap=None,
          route="gram", ell=None):
    """Algorithm 1.  ``route`` picks the nullspace update: "gram" (SVD of the
    Gram matrix, DISCUSSION) or "rsvd" (randomized SVD and Householder
    completion, THEORY; sketch of ``ell`` columns, default ceil(3r/2), drawn
    for outer index i as ``rsvd.sketch_matrix(seed, i, ...)``).

    ``schedule``: list of (lo, hi, steps) per outer iteration.  ``p == 0``
    uses the whole nullspace (F = Q); otherwise F = Q P^(i,j) with the JL
    matrix drawn for 0-based outer index i and inner index j.  Iterations
    before ``start_outer`` are skipped (resume from a saved x).  When
    ``trace`` is a list, one dict per gradient step is appended.  ``wrap``
    flags circular axes (each outer region must then span those axes).
    """
    x = _as_c128(x0).copy()
    for i in range(start_outer, len(schedule)):
        lo, hi, steps = schedule[i]
        if route == "gram":
            Q, evals, _ = nullspace(gram(x, kdims, lo, hi, wrap), rank)
            tail = float(evals[: Q.shape[1]].sum())
        elif route == "rsvd":
            Q, _ = nullspace_rsvd(x, kdims, lo, hi, rank, seed, i, ell=ell, wrap=wrap)
            tail = float("nan")
        else:
            raise ValueError("route must be 'gram' or 'rsvd'")
        y = x
        for j in range(steps):
            F = Q if p == 0 else Q @ jl_matrix(seed, i, j, Q.shape[1], p)
            y, J, gn2, eta = descent_step(y, mask, F, kdims, lo, hi, wrap)
            if trace is not None:
                trace.append(dict(i=i, j=j, J=J, gnorm2=gn2, eta=eta,
                                  tail=tail))
        x = y
    return x
