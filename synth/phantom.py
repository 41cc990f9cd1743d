"""Phantoms, coil maps and k-space synthesis (inputs only, no method arithmetic).

Coordinates run over [-1, 1) on every spatial axis.  Every generator takes a
``numpy.random.Generator`` so a workload is fully determined by its seed.
"""
import numpy as np


def _grid(shape):
    axes = [(np.arange(n) - n / 2.0) / (n / 2.0) for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def ellipse_image(shape, n_ellipses, rng, skull=False):
    """2-D complex image made of random ellipses.

    Each ellipse has centre U[-0.6, 0.6]^2, semi-axes U[0.1, 0.5], angle
    U[0, pi), intensity U[0.2, 1] and a constant phase U[-pi, pi).  With
    ``skull`` an outer bright ring (brain-like slice) is added first.
    """
    X, Y = _grid(shape)
    img = np.zeros(shape, np.complex128)
    if skull:
        outer = (X / 0.88) ** 2 + (Y / 0.72) ** 2 <= 1.0
        inner = (X / 0.82) ** 2 + (Y / 0.66) ** 2 <= 1.0
        img[outer] += 1.0
        img[inner] -= 0.7
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.6, 0.6, 2)
        a, b = rng.uniform(0.1, 0.5, 2)
        if skull:
            a, b = 0.6 * a, 0.6 * b
        th = rng.uniform(0.0, np.pi)
        amp = rng.uniform(0.2, 1.0) * np.exp(1j * rng.uniform(-np.pi, np.pi))
        xr = (X - cx) * np.cos(th) + (Y - cy) * np.sin(th)
        yr = -(X - cx) * np.sin(th) + (Y - cy) * np.cos(th)
        img[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] += amp
    return img


def ellipsoid_volume(shape, n_ellipsoids, rng):
    """3-D complex volume made of random axis-aligned-then-rotated ellipsoids."""
    X, Y, Z = _grid(shape)
    vol = np.zeros(shape, np.complex64)
    for _ in range(n_ellipsoids):
        c = rng.uniform(-0.5, 0.5, 3)
        ax = rng.uniform(0.15, 0.6, 3)
        th = rng.uniform(0.0, np.pi)
        amp = rng.uniform(0.2, 1.0) * np.exp(1j * rng.uniform(-np.pi, np.pi))
        xr = (X - c[0]) * np.cos(th) + (Y - c[1]) * np.sin(th)
        yr = -(X - c[0]) * np.sin(th) + (Y - c[1]) * np.cos(th)
        zr = Z - c[2]
        inside = (xr / ax[0]) ** 2 + (yr / ax[1]) ** 2 + (zr / ax[2]) ** 2 <= 1.0
        vol[inside] += np.complex64(amp)
    return vol


def cine_phantom(nt, shape, n_static, rng, period=None):
    """2-D+t phantom: static ellipses plus one ellipse whose semi-axes scale by
    ``1 - 0.2 * (1 - cos(2 pi t / period)) / 2`` (a periodically contracting
    'heart').  Returns an ``(nt, *shape)`` complex array (time slowest)."""
    period = nt if period is None else period
    static = ellipse_image(shape, n_static, rng, skull=True)
    X, Y = _grid(shape)
    cx, cy = rng.uniform(-0.2, 0.2, 2)
    a0, b0 = rng.uniform(0.15, 0.25, 2)
    amp = rng.uniform(0.6, 1.0) * np.exp(1j * rng.uniform(-np.pi, np.pi))
    out = np.empty((nt,) + tuple(shape), np.complex128)
    for t in range(nt):
        sc = 1.0 - 0.2 * 0.5 * (1.0 - np.cos(2.0 * np.pi * t / period))
        inside = ((X - cx) / (a0 * sc)) ** 2 + ((Y - cy) / (b0 * sc)) ** 2 <= 1.0
        out[t] = static
        out[t][inside] += amp
    return out


def gaussian_coil_maps(shape, nc, rng, radius=1.2, sigma=0.7):
    """Gaussian-bump sensitivities centred on a circle (2-D) or a ring in the
    first two axes (3-D) at angles 2 pi c / nc, each with a random constant
    phase.  Returns ``(*shape, nc)``."""
    G = _grid(shape)
    maps = np.empty(tuple(shape) + (nc,), np.complex128)
    for c in range(nc):
        ang = 2.0 * np.pi * c / nc
        centre = [radius * np.cos(ang), radius * np.sin(ang)] + [0.0] * (len(shape) - 2)
        d2 = sum((g - c0) ** 2 for g, c0 in zip(G, centre))
        maps[..., c] = np.exp(-d2 / (2.0 * sigma ** 2)) * np.exp(1j * rng.uniform(-np.pi, np.pi))
    return maps


def polynomial_coil_maps(shape, nc, rng, degree=3):
    """Smooth sensitivities: random complex polynomials of total degree
    <= ``degree`` in the spatial coordinates, scaled to unit peak magnitude."""
    G = _grid(shape)
    D = len(shape)
    exps = [e for e in np.ndindex(*([degree + 1] * D)) if sum(e) <= degree]
    maps = np.empty(tuple(shape) + (nc,), np.complex128)
    for c in range(nc):
        m = np.zeros(shape, np.complex128)
        for e in exps:
            coef = (rng.standard_normal() + 1j * rng.standard_normal()) / (1.0 + sum(e))
            term = np.ones(shape)
            for g, k in zip(G, e):
                term = term * g ** k
            m += coef * term
        maps[..., c] = m / np.abs(m).max()
    return maps


def bandlimited_coil_maps(shape, nc, w, rng):
    """Sensitivities whose centred DFT is supported on a ``w``-wide box in every
    axis (random complex values there, zero elsewhere).  Multiplying an
    image by such maps makes every coil's k-space an exact circular
    convolution of the image's k-space with a ``w^D`` kernel."""
    maps = np.empty(tuple(shape) + (nc,), np.complex128)
    for c in range(nc):
        k = np.zeros(shape, np.complex128)
        sl = tuple(slice(n // 2 - w // 2, n // 2 - w // 2 + w) for n in shape)
        k[sl] = rng.standard_normal((w,) * len(shape)) + 1j * rng.standard_normal((w,) * len(shape))
        axes = tuple(range(len(shape)))
        maps[..., c] = np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(k, axes=axes),
                                                    axes=axes, norm="ortho"), axes=axes)
    return maps


def to_kspace(image, maps):
    """Centred orthonormal FFT of ``image * maps[..., c]`` for every coil.
    Returns ``(*image.shape, nc)`` complex128."""
    coil_imgs = image[..., None] * maps
    axes = tuple(range(image.ndim))
    return np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(coil_imgs, axes=axes),
                                       axes=axes, norm="ortho"), axes=axes)


def add_noise(x, snr_db, rng):
    """Add circular complex Gaussian noise with ||noise|| = ||x|| 10^(-snr/20)."""
    n = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
    n *= np.linalg.norm(x) * 10.0 ** (-snr_db / 20.0) / np.linalg.norm(n)
    return x + n
