"""GPU parity of the mixed-precision form: band<->grid z contractions on BF16 matrix cores
with split hi/lo operands and FP32 accumulation, FP32 transports, FP64 reductions.

Each product hi*hi + hi*lo + lo*hi carries a relative error of about 2^-16; sums over at most
128 terms keep the transform error near 1e-5.  The asserted bound is 1e-4 (ten times that);
the measured errors are printed.
"""
import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B

from parity_cases import bl_problem, case, grad_error, oracle_gradient, oracle_hessvec, rel2

pytestmark = pytest.mark.gpu

CASES = ["c1_2d", "ragged_3d", "brainlike_small", "c2_full"]


@pytest.mark.parametrize("name", CASES[:3])
def test_mixed_transforms(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    p = bl_problem(prob, precision=B.BL_MIXED)
    grid = B.bl_band_to_grid(p, vh)
    errs = []
    for c in range(prob.dim):
        ref = O.iota(O.project(vh[c], prob), prob)
        errs.append(np.abs(grid[c] - ref).max() / np.abs(ref).max())
    f = np.stack([I0, I1]).astype(np.float32)
    band = B.bl_grid_to_band(p, f)
    perr = [rel2(band[c], O.pi_(f[c].astype(np.float64), prob)) for c in range(2)]
    print(f"mixed {name}: iota max rel err {max(errs):.2e}, pi rel err {max(perr):.2e}", flush=True)
    assert max(errs) < 1e-4 and max(perr) < 1e-4


@pytest.mark.parametrize("name", CASES)
def test_mixed_gradient_and_hessvec(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    ctx = B.Ctx(bl_problem(prob, precision=B.BL_MIXED), I0, I1)
    E, g = ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
    H = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
    ctx.close()
    eg = grad_error(g, oracle_gradient(name), prob, vh)
    eh = rel2(H, oracle_hessvec(name))
    print(f"mixed {name}: gradient rel err {eg:.2e}, hessvec rel err {eh:.2e}", flush=True)
    assert eg < 1e-4 and eh < 1e-4


def test_mixed_register_c1_matches_plain(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("c1_2d")
    v0 = np.zeros_like(vh, dtype=np.complex64)
    vp, mp, sp = B.bl_lddmm_register(bl_problem(prob), I0, I1, v0)
    vm, mm, sm = B.bl_lddmm_register(bl_problem(prob, precision=B.BL_MIXED), I0, I1, v0)
    print("plain", sp["mse_rel"][-1], sp["pcg_iters"], " mixed", sm["mse_rel"][-1], sm["pcg_iters"],
          " |dv|/|v|", rel2(vm, vp), flush=True)
    assert abs(sm["mse_rel"][-1] - sp["mse_rel"][-1]) <= 0.01 * sp["mse_rel"][-1] + 1e-3
    assert rel2(vm, vp) < 1e-2
