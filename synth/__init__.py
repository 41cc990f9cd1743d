"""Seeded synthetic inputs for HICU workloads.

This package only *draws* inputs: phantoms, coil sensitivity maps, k-space
(centred orthonormal FFT of phantom x coil map), sampling masks and the
workload table.  It holds none of the method's arithmetic (no Hankel
lifting, no Gram, no nullspace, no gradient, no line search), so both the
CPU oracle and the HIP path can consume its outputs without sharing code.

Arrays use the canonical layout of the whole project: k-space is
``(D0, D1, D2, Nc)`` with the coil axis fastest; 2-D data has ``D0 == 1``.
Sampling masks are ``(D0, D1, D2)`` uint8 with 1 = observed.
"""
from .phantom import (ellipse_image, ellipsoid_volume, cine_phantom,
                      gaussian_coil_maps, polynomial_coil_maps,
                      bandlimited_coil_maps, to_kspace, add_noise)
from .masks import (vd_lines, line_mask, poisson_disc_2d, volume_mask_from_plane,
                    cine_line_masks)
from .configs import WORKLOADS, make_problem, make_batch2d, co_region, full_region, crop_problem

__all__ = [
    "ellipse_image", "ellipsoid_volume", "cine_phantom", "gaussian_coil_maps",
    "polynomial_coil_maps", "bandlimited_coil_maps", "to_kspace", "add_noise",
    "vd_lines", "line_mask", "poisson_disc_2d", "volume_mask_from_plane",
    "cine_line_masks", "WORKLOADS", "make_problem", "co_region", "full_region",
    "crop_problem", "make_batch2d",
]
