"""Inputs of the 256^3 workload (band 64^3, Nt = 20, six tissue classes, 8 voxels), built
from the seeded phantom generators and numpy.fft only (no library call), so that the GPU
tests and the script that writes the oracle's expected values see the same data.

I1 is a second phantom draw (a realistic pair of subjects, not a known warp); the point of
linearisation is half of a random band velocity scaled to 8 voxels of maximal displacement;
the direction is a random admissible band vector with max |dv~| = 1.
"""
import numpy as np

import oracle as O
from paper_1807_05117_amd import phantoms

C5_GRID, C5_BAND, C5_NT, C5_DISP = (256, 256, 256), (64, 64, 64), 20, 8.0


def fft_grid(vh, prob):
    """iota through numpy.fft (FP64): v~(k) placed at k mod N, M * ifftn, real part."""
    S = np.zeros(prob.shape, dtype=np.complex128)
    idx = np.meshgrid(*[np.mod(np.arange(K) - K // 2, N) for K, N in zip(prob.bshape, prob.shape)],
                      indexing="ij")
    S[tuple(idx)] = vh
    return (np.fft.ifftn(S) * prob.M).real


_C5 = {}


def c5():
    """dict with prob, I0, I1 (float32), vh, dv (complex64)"""
    if not _C5:
        prob = O.Problem(3, C5_GRID, C5_BAND, C5_NT)
        I0 = phantoms.shells_3d(0, C5_GRID, n_classes=6).astype(np.float32)
        I1 = phantoms.shells_3d(1, C5_GRID, n_classes=6).astype(np.float32)
        vs = O.project(phantoms.raw_band_velocity(0, 3, C5_BAND), prob)
        vmax = np.sqrt(sum(fft_grid(vs[j], prob) ** 2 for j in range(3))).max() * prob.nref
        vh = (0.5 * vs * (C5_DISP / vmax)).astype(np.complex64)
        dv = O.project(phantoms.random_band_direction(1, 3, C5_BAND), prob)
        dv = (dv / np.abs(dv).max()).astype(np.complex64)
        _C5.update(prob=prob, I0=I0, I1=I1, vh=vh, dv=dv)
    return _C5
