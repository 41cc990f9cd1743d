"""Time-averaged initialisation (METHODS, Study II): the reconstruction
starts from the time-averaged k-space; a phase-encoding location that is
sampled in no frame is zero-filled.

Reading: every unobserved sample (location, frame, coil) takes the mean of
the observed samples of the same location and coil over all frames;
observed samples keep their values.

Parity: pinned by hand-worked cases and by the identities it must satisfy
(observed samples unchanged, constant along frames at unobserved entries,
equal to the per-location mean; see tests).
"""
import numpy as np


def time_average_init(x0, mask, axis=0):
    """x0: (D0, D1, D2, Nc) zero-filled observations; mask: (D0, D1, D2)
    1 = observed; ``axis``: the frame axis among the first three."""
    x0 = np.asarray(x0, np.complex128)
    m = np.asarray(mask).astype(bool)
    cnt = m.sum(axis=axis, keepdims=True)                       # observed frames per location
    tot = (x0 * m[..., None]).sum(axis=axis, keepdims=True)     # their sum per location and coil
    avg = np.where(cnt[..., None] > 0, tot / np.maximum(cnt, 1)[..., None], 0.0)
    return np.where(m[..., None], x0, np.broadcast_to(avg, x0.shape))
