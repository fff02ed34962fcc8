"""Seeded synthetic inputs: source phantoms and raw band-limited velocity coefficients.

This module draws random numbers and builds images; it holds none of the registration
arithmetic (no band<->grid transform, no transport, no derivative).  Targets are made by
warping a phantom with the forward state map, which the caller supplies: the FP64 oracle in
tests, the GPU path in the benchmark.

Images are float64 NumPy arrays in (z, y, x) order for 3D and (y, x) order for 2D, x
fastest; callers round them once to float32 and hand the same float32 values to both
sides.  Band coefficients are complex128 arrays of shape (d, [Kz,] Ky, Kx) in centred
order: index j on an axis of size K stands for the integer frequency j - K/2.

Recipes (stand-ins for the paper's brain MRI volumes of Section 4, which are not
available):
  * 2D: a sum of Gaussian blobs on a zero background (periodic distance).
  * 3D: nested ellipsoidal shells of C tissue classes with jittered semi-axes, low-order
    angular bumps, periodic Gaussian smoothing (sigma = 1 voxel) and additive N(0, 0.01^2)
    noise.
  * velocity: complex coefficients (xi1 + i xi2) / (1 + |k|^2), xi ~ N(0, 1), over the band;
    symmetrisation and the scaling to a prescribed maximal displacement are done by the
    caller with its own band-to-grid transform.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "streams",
    "blobs_2d",
    "shells_3d",
    "raw_band_velocity",
    "random_band_direction",
    "band_shape",
]


def streams(seed: int, n: int = 4):
    """Independent PCG64 generators spawned from one seed (phantom, noise, velocity, ...)."""
    ss = np.random.SeedSequence(int(seed))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def blobs_2d(seed: int, n: int = 64, nblobs: int = 8) -> np.ndarray:
    """Sum of `nblobs` Gaussian blobs on an n x n periodic grid.

    Amplitudes U(0.3, 1), widths U(3, 8) pixels, centres uniform on [0, n)^2; distances are
    measured on the torus.  Returns float64 (y, x).
    """
    rng = streams(seed, 4)[0]
    yy, xx = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                         indexing="ij")
    img = np.zeros((n, n), dtype=np.float64)
    for _ in range(nblobs):
        amp = rng.uniform(0.3, 1.0)
        s = rng.uniform(3.0, 8.0)
        cx, cy = rng.uniform(0.0, n, size=2)
        dx = np.abs(xx - cx)
        dx = np.minimum(dx, n - dx)
        dy = np.abs(yy - cy)
        dy = np.minimum(dy, n - dy)
        img += amp * np.exp(-(dx * dx + dy * dy) / (2.0 * s * s))
    return img


def shells_3d(seed: int, shape_xyz, n_classes: int = 3, intensities=None,
              radii=None, smooth: float = 1.0, noise_std: float = 0.01) -> np.ndarray:
    """Nested ellipsoidal shells of `n_classes` tissue classes, outer to inner.

    shape_xyz = (Nx, Ny, Nz).  Class c fills the ellipsoid with semi-axes
    radii[c] * N_j / 2 * U(0.95, 1.05) around N/2 + U(-0.03, 0.03) N, modulated by a +-5%
    low-order angular bump; inner classes overwrite outer ones.  Then periodic Gaussian
    smoothing (sigma = `smooth` voxels) and additive N(0, noise_std^2) noise.
    Returns float64 (z, y, x).
    """
    nx, ny, nz = (int(v) for v in shape_xyz)
    if intensities is None:
        intensities = np.linspace(0.2, 0.8, n_classes) if n_classes != 3 else (0.2, 0.5, 0.8)
    if radii is None:
        radii = np.linspace(0.85, 0.25, n_classes)
    rng_shape, rng_noise = streams(seed, 4)[:2]
    zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    img = np.zeros((nz, ny, nx), dtype=np.float64)
    dims = np.array([nx, ny, nz], dtype=np.float64)
    for c in range(n_classes):
        semi = radii[c] * dims / 2.0 * rng_shape.uniform(0.95, 1.05, size=3)
        centre = dims / 2.0 + rng_shape.uniform(-0.03, 0.03, size=3) * dims
        ex = (xx - centre[0]) / semi[0]
        ey = (yy - centre[1]) / semi[1]
        ez = (zz - centre[2]) / semi[2]
        rho = np.sqrt(ex * ex + ey * ey + ez * ez)
        theta = np.arctan2(ey, ex)
        phi = np.arctan2(ez, np.sqrt(ex * ex + ey * ey))
        a1, a2, a3 = rng_shape.uniform(-1.0, 1.0, size=3)
        p1, p2 = rng_shape.uniform(0.0, 2.0 * np.pi, size=2)
        bump = 1.0 + 0.05 * (a1 * np.cos(2.0 * theta + p1) + a2 * np.cos(3.0 * theta + p2)
                             + a3 * np.sin(2.0 * phi)) / 3.0
        img[rho <= bump] = intensities[c]
    if smooth > 0:
        img = ndimage.gaussian_filter(img, sigma=smooth, mode="wrap")
    if noise_std > 0:
        img = img + rng_noise.normal(0.0, noise_std, size=img.shape)
    return img


def band_shape(dim: int, k_xyz) -> tuple:
    """NumPy shape of one band component: (Ky, Kx) in 2D, (Kz, Ky, Kx) in 3D."""
    return tuple(int(k_xyz[j]) for j in reversed(range(dim)))


def _centred_freqs(K: int) -> np.ndarray:
    return np.arange(K, dtype=np.float64) - K // 2


def raw_band_velocity(seed: int, dim: int, k_xyz) -> np.ndarray:
    """Raw coefficients (xi1 + i xi2) / (1 + |k|^2) with |k| the integer frequency norm.

    Returns complex128 of shape (dim,) + band_shape(dim, k_xyz).  Not symmetrised and not
    scaled: the caller projects it and scales it to the wanted maximal displacement.
    """
    rng = streams(seed, 4)[2]
    shp = band_shape(dim, k_xyz)
    grids = np.meshgrid(*[_centred_freqs(K) for K in shp], indexing="ij")
    k2 = sum(g * g for g in grids)
    out = np.empty((dim,) + shp, dtype=np.complex128)
    for c in range(dim):
        xi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
        out[c] = xi / (1.0 + k2)
    return out


def random_band_direction(seed: int, dim: int, k_xyz) -> np.ndarray:
    """A raw random band vector with N(0,1) real and imaginary parts (e.g. a PCG direction)."""
    rng = streams(seed, 4)[3]
    shp = (dim,) + band_shape(dim, k_xyz)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
