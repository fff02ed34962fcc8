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

from parity_cases import (bl_problem, case, check_gradient, check_hessvec, check_mse_rel,
                          oracle_gradient, oracle_hessvec, rel2)

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
    check_gradient(g, oracle_gradient(name), prob, vh, 1e-4, f"mixed {name}")
    check_hessvec(H, oracle_hessvec(name), 1e-4, f"mixed {name}")


def test_mixed_register_c1_matches_plain(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("c1_2d")
    v0 = np.zeros_like(vh, dtype=np.complex64)
    vp, mp, sp = B.bl_lddmm_register(bl_problem(prob), I0, I1, v0)
    vm, mm, sm = B.bl_lddmm_register(bl_problem(prob, precision=B.BL_MIXED), I0, I1, v0)
    print("plain", sp["mse_rel"][-1], sp["pcg_iters"], " mixed", sm["mse_rel"][-1], sm["pcg_iters"],
          " |dv|/|v|", rel2(vm, vp), flush=True)
    assert abs(sm["mse_rel"][-1] - sp["mse_rel"][-1]) <= 0.01 * sp["mse_rel"][-1] + 1e-3
    assert rel2(vm, vp) < 1e-2


@pytest.mark.parametrize("name,max_gn", [("c1_2d", 10), ("ragged_3d", 3)])
def test_mixed_register_against_oracle(gpu_lib, name, max_gn):
    """The mixed form's final velocity and warped image against the FP64 oracle's registration
    (not against the plain GPU path): same solver decisions, per-iteration energies and
    MSE_rel, and the errors of the final v~ and m(1) printed and bounded."""
    prob, I0, I1, vs, vh, dv = case(name)
    v0 = np.zeros_like(vh)
    v_ref, m_ref, st_ref = O.register(I0, I1, v0, prob, O.SolverOpts(max_gn=max_gn))
    vm, mm, sm = B.bl_lddmm_register(bl_problem(prob, precision=B.BL_MIXED), I0, I1,
                                     v0.astype(np.complex64), B.opts_struct(max_gn=max_gn))
    ev, em = rel2(vm, v_ref), float(np.abs(mm - m_ref).max() / np.abs(m_ref).max())
    print(f"mixed register {name}: final v~ rel err {ev:.2e}, m(1) max rel err {em:.2e}, "
          f"pcg {sm['pcg_iters']} vs {st_ref['pcg_iters']}", flush=True)
    assert sm["status"] == st_ref["status"]
    assert sm["pcg_iters"] == st_ref["pcg_iters"]
    assert sm["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(sm["E"], st_ref["E"], rtol=1e-4, atol=0)
    check_mse_rel(sm, st_ref, 1e-4, f"mixed {name}")
    assert ev < 1e-3 and em < 1e-3
