"""Reconstruction metrics (METHODS, "MR reconstruction and analysis").

SER = 20 log10(||X||_F / ||X_hat - X||_F) over the whole k-space array,
observed samples included, against the fully sampled ground truth.

Parity: pinned by hand-computed cases (see tests).
"""
import numpy as np


def ser(x_hat, x_true):
    """Signal-to-error ratio in dB."""
    x_true = np.asarray(x_true, np.complex128)
    err = np.linalg.norm(np.asarray(x_hat, np.complex128) - x_true)
    return float(20.0 * np.log10(np.linalg.norm(x_true) / err))


def rel_err(a, b):
    """||a - b||_F / ||b||_F."""
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(np.asarray(a, np.complex128) - b) / np.linalg.norm(b))
