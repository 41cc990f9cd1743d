"""Rounding-error bounds for comparing the HIP contractions with the FP64
oracle element by element.

For a sum of products s = sum_i a_i b_i evaluated with operands rounded to
a format of unit roundoff u_op and accumulated in a format of unit
roundoff u_acc, |fl(s) - s| <= (2 u_op + u_op^2 + T u_acc) sum_i |a_i b_i|
(T = number of real terms; standard forward bound, Higham ch. 3).  The
magnitude sums are obtained by running the oracle's contractions on
absolute values.  Bounds are worst case; observed errors are much smaller.
"""
import numpy as np

import oracle

U32 = 2.0 ** -24
# Operand representation error per precision mode: FP32 inputs are exact,
# BF16 rounds to 8 significant bits, the split hi+lo BF16 pair keeps ~16 bits
# and drops the lo*lo product.
U_OP = {"fp32": 0.0, "bf16": 2.0 ** -8, "bf16x3": 3.0 * 2.0 ** -16, "fp16": 2.0 ** -11}

# FP16 operands are scaled by 2^(14 - ceil(log2 max|input|)) before
# rounding; values that land below 2^-14 are subnormal and carry an absolute
# error up to 2^-25 in scaled units.  The filters are not scaled.
F16_SUB = 2.0 ** -25


def f16_scale(maxabs, margin=1):
    """Scale the kernels pick for an input of largest magnitude maxabs, one
    binade smaller when margin=1 (covers a computed maximum slightly above
    the exact one)."""
    if maxabs <= 0:
        return 1.0
    c = int(np.ceil(np.log2(maxabs)))
    return 2.0 ** (14 - c - margin)


def _ops_factor(prec, terms):
    u = U_OP[prec]
    return 2.0 * u + u * u + terms * U32


def forward_bound(x, F, kd, lo, hi, prec, wrap=None):
    """Elementwise bound on |Y_gpu - Y| for Y = H(x) F; also returns Y."""
    n = F.shape[0]
    Y = oracle.forward(x, F, kd, lo, hi, wrap)
    Yabs = oracle.forward(np.abs(x), np.abs(F), kd, lo, hi, wrap).real
    b = _ops_factor(prec, 2 * n + 2) * Yabs
    if prec == "fp16":
        sx = f16_scale(float(np.max(np.abs(x))), margin=0)
        rows = oracle.forward(np.abs(x), np.ones((n, 1)), kd, lo, hi, wrap).real  # sum_i |H[u, i]|
        cols = np.sum(np.abs(F), axis=0)[None, :]                           # sum_i |F[i, j]|
        b = b + 2.0 * F16_SUB * (cols / sx + rows)
    return Y, b


def grad_bound(x, mask, F, kd, lo, hi, prec, groups=1, wrap=None):
    """Elementwise bound on |g_gpu - g| for g = 2 (1-M) o H'(Y F^H), with the
    propagated error of the stored Y (rounded to FP32) included.  An adjoint
    summed over `groups` filter groups adds one FP32 rounding per group."""
    p = F.shape[1]
    K = len(oracle.hankel.kernel_box(kd)[1])  # taps of the kernel box or mask
    Y, eY = forward_bound(x, F, kd, lo, hi, prec, wrap)
    eY = eY + U32 * np.abs(Y)
    Fa = np.abs(F)
    shape = x.shape
    prop = 2.0 * oracle.hankel_adjoint(eY @ Fa.T, shape, kd, lo, hi, wrap).real
    mag = 2.0 * oracle.hankel_adjoint(np.abs(Y) @ Fa.T, shape, kd, lo, hi, wrap).real
    b = prop + _ops_factor(prec, 2 * K * p + 2 + groups) * mag
    if prec == "fp16":
        n = F.shape[0]
        sy = f16_scale(float(np.max(np.abs(Y))))
        ones_s = np.ones((Y.shape[0], p))
        fsum = oracle.hankel_adjoint(ones_s @ Fa.T, shape, kd, lo, hi, wrap).real          # sum over taps, filters of |F|
        ysum = oracle.hankel_adjoint(np.abs(Y) @ np.ones((p, n)), shape, kd, lo, hi, wrap).real  # of |Y|
        b = b + 2.0 * 2.0 * F16_SUB * (fsum / sy + ysum)
    if mask is not None:
        b[np.asarray(mask).astype(bool)] = 0.0
    return b


def sumsq_bound(v, ev):
    """Bound on |sum|v_gpu|^2 - sum|v|^2| given |v_gpu - v| <= ev."""
    return float(np.sum(2.0 * np.abs(v) * ev + ev * ev)) + 1e-12 * float(np.sum(np.abs(v) ** 2))


def grad_bound_at_points(x, F, kd, lo, hi, prec, points, groups=1):
    """grad_bound evaluated only at k-space locations ``points`` (mask not
    applied), from the point-wise oracle routines on absolute values."""
    p = F.shape[1]
    K = len(oracle.hankel.kernel_box(kd)[1])  # taps of the kernel box or mask
    n = F.shape[0]
    nc = x.shape[3]
    Fa = np.abs(F)
    xa = np.abs(x)
    f1 = _ops_factor(prec, 2 * n + 2)
    f2 = _ops_factor(prec, 2 * K * p + 2 + groups)
    out = np.zeros((len(points), nc))
    for idx, w in enumerate(points):
        acc_mag = np.zeros(nc)
        acc_abs = np.zeros(nc)
        t = 0
        for k0 in range(kd[0]):
            for k1 in range(kd[1]):
                for k2 in range(kd[2]):
                    u = (w[0] - k0, w[1] - k1, w[2] - k2)
                    if all(lo[a] <= u[a] <= hi[a] - kd[a] for a in range(3)):
                        y = np.abs(oracle.residual_at_points(x, F, kd, [u])[0])
                        ya = oracle.residual_at_points(xa, Fa, kd, [u])[0].real
                        Ft = Fa[t * nc:(t + 1) * nc, :]
                        acc_mag += Ft @ y
                        acc_abs += Ft @ ya
                    t += 1
        out[idx] = 2.0 * (f1 * acc_abs + U32 * acc_mag) + f2 * 2.0 * acc_mag
    return out
