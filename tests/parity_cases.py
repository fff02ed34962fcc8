"""Seeded parity cases shared by the GPU tests: inputs from the phantom generators, targets
and expected values from the FP64 oracle only (nothing here comes from the HIP path)."""
from __future__ import annotations

import functools

import numpy as np

import oracle as O
from paper_1807_05117_amd import binding as B
from paper_1807_05117_amd import phantoms

# name: (dim, n, k, nt, max displacement in voxels, phantom classes)
CASES = {
    # 2D plain method: 64^2 blobs, band 16^2, Nt = 10, 4 px
    "c1_2d": (2, (64, 64), (16, 16), 10, 4.0, 0),
    # ragged 3D: x spans two 64-wide tiles with a tail, y five 4-high tiles with a tail
    "ragged_3d": (3, (72, 21, 13), (16, 10, 8), 5, 3.0, 3),
    # non-cubic brain-like shape at reduced size (l_j differ per axis)
    "brainlike_small": (3, (40, 48, 40), (10, 12, 10), 6, 3.0, 5),
    # the 128^3 workload: band 32^3, Nt = 10, 6 voxels
    "c2_full": (3, (128, 128, 128), (32, 32, 32), 10, 6.0, 3),
    # brain-shaped 160x192x160: band 40x48x40, Nt = 10, five classes, 6 voxels
    "c3_full": (3, (160, 192, 160), (40, 48, 40), 10, 6.0, 5),
    # incompressible H^1 (gamma = 1, s = 1): non-cubic 3D and 2D
    "h1_incomp_3d": (3, (40, 48, 36), (10, 12, 8), 6, 3.0, 5),
    "h1_incomp_2d": (2, (64, 64), (16, 16), 10, 4.0, 0),
    # a strongly anisotropic band (2 x 66 x 4): the deformation method's fused yx kernels then
    # give each thread two band entries (ky * 4 > 256), within their LDS limits
    "aniso_band_3d": (3, (8, 72, 12), (2, 66, 4), 4, 1.0, 3),
    # degenerate cases of the method: one time step (no incremental steps between the first
    # and the last), the full band k = n (the unpaired Nyquist planes are the only ones
    # dropped), the smallest band k = 2 (one frequency pair per axis, of which only the zero
    # frequency survives the projection), and the smallest grids the library accepts
    "nt1_3d": (3, (24, 20, 12), (8, 8, 4), 1, 1.0, 3),
    "fullband_2d": (2, (16, 16), (16, 16), 4, 1.0, 0),
    "fullband_3d": (3, (12, 10, 8), (12, 10, 8), 2, 0.5, 3),
    "minband_3d": (3, (16, 12, 10), (2, 2, 2), 3, 0.5, 3),
    "tiny_3d": (3, (8, 8, 8), (4, 4, 4), 2, 0.5, 3),
    "min_grid_2d": (2, (4, 4), (4, 4), 2, 0.5, 0),
}
# regulariser and flow model per case (default alpha = 1e-3, s = 2, gamma = 0)
MODEL = {
    "h1_incomp_3d": dict(alpha=5e-3, s=1, gamma=1),
    "h1_incomp_2d": dict(alpha=5e-3, s=1, gamma=1),
}


@functools.lru_cache(maxsize=None)
def case(name, seed=0):
    dim, n, k, nt, disp, ncls = CASES[name]
    model = dict(alpha=1e-3, s=2, gamma=0)
    model.update(MODEL.get(name, {}))
    prob = O.Problem(dim, n, k, nt, sigma=1.0, **model)
    if dim == 2:
        I0 = phantoms.blobs_2d(seed, n[0])[: n[1], : n[0]]
    else:
        I0 = phantoms.shells_3d(seed, n, n_classes=ncls)
    I0 = I0.astype(np.float32).astype(np.float64)
    vs = O.project(phantoms.raw_band_velocity(seed, dim, k), prob)
    vs *= disp / O.max_displacement_voxels(vs, prob)
    vs = vs.astype(np.complex64).astype(np.complex128)
    I1 = O.warp(I0, vs, prob).astype(np.float32).astype(np.float64)
    vh = (0.5 * vs).astype(np.complex64).astype(np.complex128)        # mid-optimisation point
    dv = O.project(phantoms.random_band_direction(seed + 1, dim, k), prob)
    dv = (dv / np.abs(dv).max()).astype(np.complex64).astype(np.complex128)
    return prob, I0, I1, vs, vh, dv


@functools.lru_cache(maxsize=None)
def oracle_state(name, seed=0):
    prob, I0, I1, vs, vh, dv = case(name, seed)
    return O.evaluate(vh, I0, I1, prob)


@functools.lru_cache(maxsize=None)
def oracle_gradient(name, seed=0):
    return O.gradient(oracle_state(name, seed))


@functools.lru_cache(maxsize=None)
def oracle_hessvec(name, seed=0):
    prob, I0, I1, vs, vh, dv = case(name, seed)
    return O.hessvec(oracle_state(name, seed), dv)


@functools.lru_cache(maxsize=None)
def oracle_hessvec_newton(name, seed=0):
    prob, I0, I1, vs, vh, dv = case(name, seed)
    return O.hessvec_newton(oracle_state(name, seed), dv)


def bl_problem(prob, precision=B.BL_FP32, **kw):
    return B.make_problem(prob.dim, prob.n, prob.k, prob.nt, alpha=prob.alpha, s=prob.s,
                          sigma=prob.sigma, gamma=prob.gamma, precision=precision, **kw)


def rel2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
                 / np.linalg.norm(np.asarray(b).ravel()))


def grad_error(g_gpu, g_ref, prob, vh):
    """|g - g_ref|_2 / (|L v|_2 + |pi(b)|_2): the regulariser and the data part are normalised
    separately so that their cancellation near an optimum does not inflate the error."""
    Lv = O.L_hat(prob)[None] * O.project(vh, prob)
    pb = g_ref - Lv
    den = np.linalg.norm(Lv.ravel()) + np.linalg.norm(pb.ravel())
    return float(np.linalg.norm((np.asarray(g_gpu) - g_ref).ravel()) / den)


def _components(a, lead):
    """view with the first `lead` axes (component, or node and component) flattened into rows"""
    a = np.asarray(a)
    rows = int(np.prod(a.shape[:lead]))
    return a.reshape(rows, -1)


def elem_error(a, ref, lead=1):
    """worst component of max_i |a_i - ref_i| / max_i |ref_i| (per velocity component, or per
    node and component for non-stationary fields)"""
    A, R = _components(a, lead), _components(ref, lead)
    return float(max(np.abs(A[c] - R[c]).max() / np.abs(R[c]).max() for c in range(R.shape[0])))


def grad_elem_error(g_gpu, g_ref, prob, vh):
    """worst component of max |g - g_ref| / (max |L v| + max |pi(b)|): the element-wise form of
    grad_error, with the regulariser and the data part normalised separately"""
    Lv = O.L_hat(prob)[None] * O.project(vh, prob)
    pb = g_ref - Lv
    G, R = np.asarray(g_gpu), np.asarray(g_ref)
    return float(max(np.abs(G[c] - R[c]).max() / (np.abs(Lv[c]).max() + np.abs(pb[c]).max())
                     for c in range(R.shape[0])))


def check_gradient(g_gpu, g_ref, prob, vh, tol, label=""):
    """gradient parity in the 2-norm and element by element (both within tol); returns both"""
    e2 = grad_error(g_gpu, g_ref, prob, vh)
    ee = grad_elem_error(g_gpu, g_ref, prob, vh)
    print(f"  {label} gradient rel err 2-norm {e2:.2e}, element-wise {ee:.2e}", flush=True)
    assert e2 < tol and ee < tol, (label, e2, ee)
    return e2, ee


def check_hessvec(h_gpu, h_ref, tol, label="", lead=1):
    """Hessian-vector parity in the 2-norm and element by element (both within tol)"""
    e2 = rel2(h_gpu, h_ref)
    ee = elem_error(h_gpu, h_ref, lead)
    print(f"  {label} hessvec rel err 2-norm {e2:.2e}, element-wise {ee:.2e}", flush=True)
    assert e2 < tol and ee < tol, (label, e2, ee)
    return e2, ee


def check_mse_rel(st_gpu, st_ref, rtol, label=""):
    """the library's per-iteration MSE_rel statistic against the oracle's (same solver
    decisions assumed: equal lengths)"""
    a = np.asarray(st_gpu["mse_rel"], dtype=np.float64)
    b = np.asarray(st_ref["mse_rel"], dtype=np.float64)
    print(f"  {label} mse_rel gpu {a[-1]:.6f} oracle {b[-1]:.6f}, max rel diff "
          f"{np.max(np.abs(a - b) / np.abs(b)):.2e}", flush=True)
    assert a.shape == b.shape, (label, a.shape, b.shape)
    assert np.all(np.abs(a - b) <= rtol * np.abs(b)), (label, a, b)
