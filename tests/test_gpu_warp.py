"""GPU: bl_lddmm_warp, the forward state alone (m(1), Section 2.2), element by element against
the FP64 oracle's m(1) on the same seeded float32 inputs at a fractional velocity, for every
model the entry point serves: stationary (plain and mixed), non-stationary and the deformation
state equation.  Bound: max |dm| <= tol * max |I0| (tol 1e-5 plain, 1e-4 mixed)."""
import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B

from parity_cases import bl_problem, case, oracle_state

pytestmark = pytest.mark.gpu

STATIONARY = ["c1_2d", "ragged_3d", "brainlike_small", "nt1_3d", "fullband_3d", "min_grid_2d"]


def _log(*a):
    print(*a, flush=True)


def _check(w, ref, I0, tol, label):
    err = np.abs(w.astype(np.float64) - ref).max() / np.abs(I0).max()
    _log(f"  {label}: max |dm| / max |I0| = {err:.2e}")
    assert w.shape == ref.shape
    assert err <= tol, (label, err)


@pytest.mark.parametrize("precision,tol", [(B.BL_FP32, 1e-5), (B.BL_MIXED, 1e-4)],
                         ids=["fp32", "mixed"])
@pytest.mark.parametrize("name", STATIONARY)
def test_warp_stationary(gpu_lib, name, precision, tol):
    prob, I0, I1, vs, vh, dv = case(name)
    _log("case", name, "warp")
    w = B.bl_lddmm_warp(bl_problem(prob, precision=precision), I0, vh.astype(np.complex64))
    _check(w, oracle_state(name).m[prob.nt], I0, tol, name)


@pytest.mark.parametrize("name", ["c1_2d", "ragged_3d"])
def test_warp_nonstationary(gpu_lib, name):
    """a velocity that varies over the time nodes"""
    prob, I0, I1, vs, vh, dv = case(name)
    V = np.stack([vh * (1.0 + 0.3 * np.sin(n)) for n in range(prob.nt + 1)])
    V = V.astype(np.complex64)
    _log("case", name, "non-stationary warp")
    ref = O.ns_evaluate(V.astype(np.complex128), I0, I1, prob).m[prob.nt]
    w = B.bl_lddmm_warp(bl_problem(prob, nonstationary=True), I0, V)
    _check(w, ref, I0, 1e-5, name + " non-stationary")


@pytest.mark.parametrize("name", ["c1_2d", "ragged_3d"])
def test_warp_deformation(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    _log("case", name, "deformation-state warp")
    ref = O.def_evaluate(vh, I0, I1, prob).m1
    w = B.bl_lddmm_warp(bl_problem(prob, deformation=True), I0, vh.astype(np.complex64))
    _check(w, ref, I0, 1e-5, name + " deformation")
